"""Benchmark of the El-WaveHoltz hot path on one MI355X.

A step is one Krylov iteration of the solve on the 2-D 1024 x 1024 random
log-normal medium with a traction-free top (FP64): one A_h = I - S_h
application (the half-step launch and the fused launches of K = 4 time
steps each, plus one shorter launch when 4 does not divide N_T - 1, over
every unknown node, each step with its trapezoid accumulation)
plus the FP64 M-inner-product reductions and the CG vector updates.  Inputs are resident
in HBM before timing.  value = lattice updates per second, one lattice
update = one unknown node advanced one time step (both components), with its
accumulation.

The JSON line also carries the roofline of the fused K-step kernel (HIP-event
durations of its launches on the same workload and tiling, with N_T rounded
so that every launch takes K steps), the HBM ceiling a STREAM triad reaches, the FP32-stepping and
single-step variants, the step kernels of the 3-D cube, of mapped 2-D and 3-D
grids and of the two-field operator, the time to residual 1e-8 of the
benchmark problem and of a 3-D cube, the 48-problem ragged batch, the
learned-start comparison on the 512 held-out warm-start problems, and the
CPU oracle's rate on all host cores and on one core.  The optional parts
run in order of importance inside a time budget (--budget seconds); a part
that would not fit is reported as skipped.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--budget S] [--no-cpu] [--quick]
"""

import argparse
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "elastic lattice updates/s (% HBM roofline); time-to-1e-8 residual learned+FP32 vs plain"

# Algorithmic HBM bytes per lattice update (one unknown node, one step).
# Single-step kernel (fuse = 1; the 3-D kernel):
#   FP64: read u^n (2x8), u^{n-1} (2x8), a, lambda, mu (3x8), acc (2x8);
#         write u^{n+1} (2x8), acc (2x8)                                  = 104
#   FP32 state, compensated FP64 accumulator (FP64 hi, FP32 lo): state
#         3x2x4, coefficients 3x4, acc hi+lo read and written 2x2x(8+4)    = 84
#   FP32 state, plain FP64 accumulator: 24 + 12 + 32                      = 68
#   3-D: three components; FP64 3x3x8 + 3x8 + 2x3x8 = 144; FP32
#         compensated 36 + 12 + 72 = 120; FP32 plain 36 + 12 + 48 = 96
# K-step kernel (2-D, fuse = K = 2..4), per node and launch (K lattice
# updates), independent of K:
#   FP64: read u^n, u^{n-1} (2x2x8), a, lambda, mu (3x8), acc (2x8);
#         write u^{n+K-1}, u^{n+K} (2x2x8), acc (2x8) = 120, i.e. 120/K per LUP
#   FP32 compensated: state 4x2x4 + 3x4 + acc hi+lo 2x2x(8+4) = 92
#   FP32 plain accumulator: 32 + 12 + 32 = 76
BYTES_PER_LUP = {
    (2, "f64", 1): 104, (2, "f32c", 1): 84, (2, "f32", 1): 68,
    (3, "f64", 1): 144, (3, "f32c", 1): 120, (3, "f32", 1): 96,
}
BYTES_PER_MULTI_LAUNCH = {"f64": 120, "f32c": 92, "f32": 76}
# 3-D two-step kernel, per node and launch (two lattice updates): read u^n,
# u^{n-1} (2x3x8), a, lambda, mu (3x8), acc (3x8); write u^{n+1}, u^{n+2}
# (2x3x8), acc (3x8) = 168 (FP64); FP32 state with the compensated FP64
# accumulator: 2x12 + 12 + acc hi+lo 36 read, 2x12 + 36 written = 132
BYTES_PER_LAUNCH_3D_K2 = {"f64": 168, "f32c": 132}
# Mapped (curvilinear) 2-D grids, single-step kernel: the three coefficient
# arrays become seven (a = c dt^2/(rho J), lambda/J, mu/J and the metric
# vectors J grad q, J grad r):
#   FP64: state 3x2x8 + 7x8 + acc 2x2x8 = 136; FP32 compensated:
#   24 + 28 + 48 = 100; FP32 plain accumulator: 24 + 28 + 32 = 84
BYTES_PER_LUP_MAPPED = {"f64": 136, "f32c": 100, "f32": 84}
# Two-field step with impedance faces (FP64, one step per launch): state u^n,
# u^{n-1} read and u^{n+1} written (3 x 2 x 8), a, lambda, mu (3 x 8), the
# displacement and velocity accumulators read and written (2 x 2 x 2 x 8)
BYTES_PER_LUP_TWOFIELD = 136
TWOFIELD_WORKLOAD = ("the 1024^2 random-medium benchmark workload (medium, source, omega) with every face "
                     "absorbing (impedance Z = rho c_p normal, rho c_s tangential): an open box")
MAPPED_WORKLOAD = ("quarter annulus of the iterations-vs-frequency experiment at omega = 200 + sqrt(2)/10 "
                   "(801 x 4003 cells, 20 points per shear wavelength at c_s = 1), random log-normal medium "
                   "(seed 14), Dirichlet sides")


def step_launches(nt, fuse):
    """Steps per launch of the N_T - 1 steps after the half step."""
    out, rem = [], nt - 1
    while fuse >= 2 and rem >= 2:
        k = min(fuse, rem)
        out.append(k)
        rem -= k
    return out + [1] * rem


def phase_bytes(dim, tag, fuse, nt, nodes):
    """Algorithmic bytes of the N_T - 1 steps after the half step, and the
    number of launches that move them."""
    ks = step_launches(nt, fuse)
    b = sum((BYTES_PER_MULTI_LAUNCH[tag] if k >= 2 else BYTES_PER_LUP[(dim, tag, 1)]) * nodes for k in ks)
    return b, len(ks)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def unknown_nodes(case):
    cnt = 1
    for a in range(case.dim):
        n = case.n[a]
        lo_d = case.bc[2 * a] == 0
        hi_d = case.bc[2 * a + 1] == 0
        cnt *= (n + 1) - int(lo_d) - int(hi_d)
    return cnt


def read_traffic(kernel_tag, tile, family="2d"):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    one exists for this kernel, workload and tiling and the kernel's sources
    have not changed since (else None)."""
    path = os.path.join(ROOT, "profiles", f"{kernel_tag}_counters.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        # "traffic_bytes_per_launch[V,TY]: bytes" per tiling, "kernel_source_hash: h"
        m = re.match(r"\s*(traffic_bytes_per_launch\[\d+,\d+\]|kernel_source_hash)\s*[:=]\s*(\S+)", line)
        if m:
            vals[m.group(1)] = m.group(2)
    key = f"traffic_bytes_per_launch[{tile[0]},{tile[1]}]"
    if key not in vals:
        return None
    src_hash = vals.get("kernel_source_hash")
    if src_hash != kernel_source_hash(family):
        return None          # the kernel changed since the counters were taken
    return float(vals[key])


# the sources each step-kernel family is built from (a counters summary holds
# the hash of its family's sources at the time of collection)
KERNEL_SOURCES = {
    "2d": ("kernels2d.hip", "kernels2d_multi.hip", "step2d_common.h", "xcd.h", "lanes.h"),
    "3d": ("kernels3d.hip", "kernels3d_k2.hip", "step3d_common.h", "xcd.h", "lanes.h"),
}


def kernel_source_hash(family="2d"):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[family]:
        h.update(open(os.path.join(ROOT, "paper_2205_12344_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def time_cg(ctx, steps, warmup):
    import torch
    ctx.cg_iterate(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.cg_iterate(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # profiled repeat of the same steps: per-launch HIP events on the
    # context's stream around every fused step kernel
    ctx.profile_enable(True)
    ctx.cg_iterate(steps)
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    return t1 - t0, prof


def kernel_rate(ctx, napply):
    """Profile napply A_h applications of a context (any precision)."""
    import torch
    x = torch.zeros(ctx.field_shape, dtype=torch.float64, device="cuda")
    ctx.apply_A(x)
    ctx.profile_enable(True)
    for _ in range(napply):
        ctx.apply_A(x)
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    return prof


def mapped_rates(elwh, inputs, napply=3):
    """Step-kernel rate on the mapped workload (FP64 and FP32 compensated)."""
    x, y, rho, lam, mu, om, _ = inputs.sector_case(200, 1, seed=14)
    nodes = (x.shape[0] - 2) * (x.shape[1] - 2)
    out = {}
    for tag, kw in (("f64", {}), ("f32c", {"prec": elwh.FP32_STEP, "compensated": 1})):
        ctx = elwh.MappedContext(x, y, rho, lam, mu, om, **kw)
        p = kernel_rate(ctx, napply)
        avg_s = p["step_ms"] * 1e-3 / max(p["nstep"], 1)
        bb = BYTES_PER_LUP_MAPPED[tag]
        t = ctx.get_tile(elwh.FP64 if tag == "f64" else elwh.FP32_STEP)
        out[tag] = {"workload": MAPPED_WORKLOAD, "cells": [x.shape[1] - 1, x.shape[0] - 1], "omega": om,
                    "nt": ctx.info()["nt"], "tile": list(t), "kernel": "curv2d_kernel",
                    "step_kernel_us": round(1e6 * avg_s, 3), "glup_s_kernel": round(nodes / avg_s / 1e9, 3),
                    "bytes_per_lup": bb, "achieved_GBs": round(bb * nodes / avg_s / 1e9, 1),
                    "frac": round(bb * nodes / avg_s / 1e9 / HBM_PEAK_GBS, 4)}
        log(f"mapped {tag}: {out[tag]}")
        ctx.close()
    return out


def twofield_rates(elwh, inputs, napply=3, solve=True):
    """Two-field (impedance) step-kernel rate on the 1024^2 absorbing workload,
    and optionally the GMRES solve of its fixed point to 1e-8."""
    import torch
    case = inputs.absorbing_square()
    nodes = unknown_nodes(case)
    ctx = elwh.context_from_case(case)
    x = torch.zeros(ctx.field_shape, dtype=torch.float64, device="cuda")
    ctx.apply_A2(x, x)
    ctx.profile_enable(True)
    for _ in range(napply):
        ctx.apply_A2(x, x)
    p = ctx.profile_read()
    ctx.profile_enable(False)
    avg_s = p["step_ms"] * 1e-3 / max(p["nstep"], 1)
    bb = BYTES_PER_LUP_TWOFIELD
    out = {"workload": TWOFIELD_WORKLOAD, "nt": ctx.info()["nt"], "tile": list(ctx.get_tile(elwh.FP64)),
           "kernel": "damped2d_kernel", "step_kernel_us": round(1e6 * avg_s, 3),
           "glup_s_kernel": round(nodes / avg_s / 1e9, 3), "bytes_per_lup": bb,
           "achieved_GBs": round(bb * nodes / avg_s / 1e9, 1),
           "frac": round(bb * nodes / avg_s / 1e9 / HBM_PEAK_GBS, 4)}
    if solve:
        # GMRES(30) to 1e-8 on the same workload, from zero
        f = torch.tensor(case.f, device="cuda")
        ctx.solve2(f, tol=1e-2, maxit=3, raise_on_fail=False)      # allocate the basis
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, info = ctx.solve2(f, tol=1e-8, maxit=4000, raise_on_fail=False)
        el = time.perf_counter() - t0
        out["gmres_to_1e-8"] = {"seconds": round(el, 3), "iters": info["iters"], "napply": info["napply"],
                                "status": info["status"], "relres_fp64": info["relres_fp64"], "gmres_m": 30,
                                "step_share": round(info["napply"] * (info["nt"] + 1) * avg_s / el, 3)}
        # the same solve with two periods per application (eq. many_periods_filter)
        c2 = elwh.context_from_case(case, periods=2)
        c2.solve2(f, tol=1e-2, maxit=3, raise_on_fail=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, i2 = c2.solve2(f, tol=1e-8, maxit=4000, raise_on_fail=False)
        el2 = time.perf_counter() - t0
        out["gmres_to_1e-8_two_periods"] = {"seconds": round(el2, 3), "iters": i2["iters"], "status": i2["status"],
                                            "relres_fp64": i2["relres_fp64"], "gmres_m": 30}
        c2.close()
    ctx.close()
    log(f"two-field: {out}")
    return out


def cpu_worker(seconds):
    """One CPU process of the oracle baseline: A_h applications of the oracle
    (sparse matrix-vector products and NumPy vector updates, one thread) on
    the benchmark workload for about `seconds`; prints one JSON line."""
    import numpy as np
    from oracle.operator import Operator
    from oracle.problem import Problem
    from oracle.stepping import WaveHoltz
    from paper_2205_12344_amd import inputs
    case = inputs.random_square()
    prob = Problem(case.dim, case.n, length=case.length, bc=case.bc)
    op = Operator(prob, case.rho, case.lam, case.mu)
    wh = WaveHoltz(op, case.omega)
    x = np.random.default_rng(0).standard_normal(op.ndof)
    napply = 0
    t0 = time.perf_counter()
    while True:
        x = wh.apply_A(x)
        x /= np.linalg.norm(x)
        napply += 1
        if time.perf_counter() - t0 >= seconds:
            break
    el = time.perf_counter() - t0
    print(json.dumps({"napply": napply, "seconds": el, "nt": wh.nt, "nodes": unknown_nodes(case)}))


def cpu_extras_worker():
    """The oracle's other reference timings, one process and one thread:
    config 1 (64^2 constant medium, omega = 10) solved by CG to 1e-10 and by a
    sparse LU of the discrete Helmholtz system, and one A_h application in
    FP64 on a 64^3 sample of the 3-D layered cube (the same construction as the
    256^3 workload; the 256^3 operator would need tens of GB as a sparse
    matrix).  Operator assembly is timed apart.  Prints one JSON line."""
    import numpy as np
    from oracle import direct, krylov
    from oracle.operator import Operator
    from oracle.problem import Problem
    from oracle.stepping import WaveHoltz
    from paper_2205_12344_amd import inputs
    out = {}
    c1 = inputs.constant_square64()
    t0 = time.perf_counter()
    prob = Problem(c1.dim, c1.n, length=c1.length, bc=c1.bc)
    op = Operator(prob, c1.rho, c1.lam, c1.mu)
    wh = WaveHoltz(op, c1.omega)
    t1 = time.perf_counter()
    fv = prob.gather(c1.f)
    res = krylov.cg(wh.apply_A, wh.rhs(fv), op.m, tol=1e-10, maxit=1000)
    t2 = time.perf_counter()
    xs = direct.solve(op, c1.omega, fv)
    t3 = time.perf_counter()
    out["config1"] = {"assembly_s": round(t1 - t0, 4), "cg_s": round(t2 - t1, 4), "cg_iters": res.iters,
                      "splu_s": round(t3 - t2, 4), "nt": wh.nt, "dof": int(op.ndof),
                      "cg_vs_direct_rel": float(np.linalg.norm(res.x - xs) / np.linalg.norm(xs))}
    c3 = inputs.layered_cube(n=64)
    t0 = time.perf_counter()
    prob3 = Problem(c3.dim, c3.n, length=c3.length, bc=c3.bc)
    op3 = Operator(prob3, c3.rho, c3.lam, c3.mu)
    wh3 = WaveHoltz(op3, c3.omega)
    t1 = time.perf_counter()
    x = np.random.default_rng(0).standard_normal(op3.ndof)
    wh3.apply_A(x)
    t2 = time.perf_counter()
    nodes = op3.ndof // 3
    out["config3_sample64"] = {"assembly_s": round(t1 - t0, 3), "apply_s": round(t2 - t1, 3), "nt": wh3.nt,
                               "nodes": int(nodes), "lup_s": wh3.nt * nodes / (t2 - t1)}
    print(json.dumps(out))


def cpu_extras():
    """Run cpu_extras_worker in a child process with one thread."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    p = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-extras-worker"], stdout=subprocess.PIPE,
                       stderr=subprocess.DEVNULL, env=env, timeout=600)
    if p.returncode != 0:
        raise RuntimeError(f"cpu extras worker failed ({p.returncode})")
    return json.loads(p.stdout.decode().strip().splitlines()[-1])


def cpu_baseline(seconds=10.0):
    """The oracle timed on the host: one worker process alone (one core), then
    one worker per core on every core the box gives this job (os.cpu_count(),
    at most 16), each doing A_h applications on the same 1024^2 workload;
    the all-core figure is the aggregate rate.  Worker processes are plain
    child processes with one thread each (no GPU use)."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-worker", str(seconds)]

    def run(n):
        procs = [subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.DEVNULL, env=env) for _ in range(n)]
        outs = []
        for p in procs:
            out, _ = p.communicate(timeout=seconds + 300)
            if p.returncode != 0:
                raise RuntimeError(f"cpu worker failed ({p.returncode})")
            outs.append(json.loads(out.decode().strip().splitlines()[-1]))
        return outs

    one = run(1)[0]
    ncores = max(1, min(os.cpu_count() or 1, 16))
    many = run(ncores) if ncores > 1 else [one]
    lup1 = one["napply"] * one["nt"] * one["nodes"] / one["seconds"]
    lupn = sum(o["napply"] * o["nt"] * o["nodes"] / o["seconds"] for o in many)
    sample = (f"A_h applications ({one['nt']} steps each) of the oracle on the same 1024^2 workload for "
              f"about {seconds:.0f} s per process (operator assembly excluded): one process alone "
              f"({one['napply']} applications), then {ncores} processes at once "
              f"({sum(o['napply'] for o in many)} applications in all)")
    return {"value": lupn, "unit": "LUP/s", "cores": ncores, "kind": "oracle", "sample": sample,
            "os_cpu_count": os.cpu_count(), "one_core": {"value": lup1, "unit": "LUP/s", "cores": 1}}


def triad_ceiling(elwh, n=2 ** 28, reps=10):
    """The HBM bandwidth a STREAM triad (the library's elwh_stream_triad)
    reaches over three 2 GiB arrays, and a device copy for comparison."""
    import torch
    a = torch.empty(n, dtype=torch.float64, device="cuda")
    b = torch.ones(n, dtype=torch.float64, device="cuda")
    c = torch.ones(n, dtype=torch.float64, device="cuda")
    for _ in range(3):
        elwh.stream_triad(a, b, c)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        elwh.stream_triad(a, b, c)
    e1.record()
    torch.cuda.synchronize()
    triad = 24 * n * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    e0.record()
    for _ in range(reps):
        a.copy_(b)
    e1.record()
    torch.cuda.synchronize()
    copy = 16 * n * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b, c
    torch.cuda.empty_cache()
    return {"triad_GBs": round(triad, 1), "copy_GBs": round(copy, 1), "frac_of_peak": round(triad / HBM_PEAK_GBS, 4),
            "arrays": "3 x 2 GiB FP64 (triad a = b + s c, 24 B per element); copy 2 x 2 GiB"}


def time_to_tol(elwh, case, tol=1e-8, maxit=20000, **kw):
    """Wall time of one solve to tol (context creation excluded)."""
    import torch
    ctx = elwh.context_from_case(case, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, info = ctx.solve(case.f, tol=tol, maxit=maxit, raise_on_fail=False)
    el = time.perf_counter() - t0
    ctx.close()
    return {"seconds": round(el, 3), "iters": info["iters"], "status": info["status"],
            "relres_fp64": info["relres_fp64"], "outer": info["outer"], "fp64_iters": info["fp64_iters"],
            "nt": info["nt"]}


def sequential_plain(elwh, first_seed=4096, n=48, tol=1e-8, maxit=4000):
    """The first n held-out warm-start problems solved one after the other,
    each in its own context (plain FP64 from zero; creation excluded): the
    unbatched context for the batched time to tol."""
    import torch
    from paper_2205_12344_amd import inputs
    secs, iters, ok = 0.0, [], True
    for s in range(first_seed, first_seed + n):
        c = inputs.warmstart_problem(s, n=256)
        ctx = elwh.context_from_case(c)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = ctx.solve(c.f, tol=tol, maxit=maxit, raise_on_fail=False)
        secs += time.perf_counter() - t0
        iters.append(info["iters"] + info["cr_iters"])
        ok &= info["status"] == "OK" and info["relres_fp64"] <= tol
        ctx.close()
    return {"problems": n, "seconds": round(secs, 3), "mean_iters": float(sum(iters) / n), "all_ok": bool(ok)}


def solves_2d_and_3d(elwh, inputs):
    """Time to 1e-8 of the layered cube at 64^3, FP64 stepping against FP32
    stepping with the compensated FP64 accumulator; and five CG iterations of
    the 256^3 cube per precision (the 64^3 cube needs about 1e4 iterations
    and the count grows like omega^3 in 3-D, Sec. 5.6, so the full 256^3
    solve would need some 5e5: hours of GPU time).  (The
    1024^2 benchmark problem is not solved here: its A_h is near-singular,
    a condition estimate of 1.6e11 from the CG Lanczos coefficients, and no
    Krylov method reaches 1e-8 on it within 3e4 iterations.)"""
    import torch
    out = {}
    # config 1 (64^2 constant medium, CG to 1e-10): launch-latency bound on
    # the GPU; the oracle's CG and sparse LU of the same problem are timed in
    # the CPU leg
    c1 = inputs.constant_square64()
    time_to_tol(elwh, c1, tol=1e-10)                                       # warm-up
    out["config1_cg_1e-10"] = time_to_tol(elwh, c1, tol=1e-10)
    log(f"config 1 to 1e-10: {out['config1_cg_1e-10']}")
    c64 = inputs.layered_cube(n=64)
    out["cube64"] = {"fp64": time_to_tol(elwh, c64), "fp32c": time_to_tol(elwh, c64, prec=elwh.FP32_STEP),
                     "omega": c64.omega}
    log(f"64^3 to 1e-8: {out['cube64']}")
    c256 = inputs.layered_cube()
    per = {}
    for tag, kw in (("fp64", {}), ("fp32c", {"prec": elwh.FP32_STEP})):
        ctx = elwh.context_from_case(c256, **kw)
        ctx.solve(c256.f, tol=0.0, maxit=1, raise_on_fail=False)          # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = ctx.solve(c256.f, tol=0.0, maxit=5, raise_on_fail=False)
        el = time.perf_counter() - t0
        per[tag] = {"seconds_for_5_iterations": round(el, 3), "napply": info["napply"],
                    "relres_after_5": info["relres_fp64"]}
        ctx.close()
        torch.cuda.empty_cache()
    out["cube256_iterations"] = per
    log(f"256^3 five CG iterations: {per}")
    return out


def ragged_batch_solve(elwh, inputs, nprob=48, precisions=("fp64", "fp32")):
    """The ragged batch: 48 problems (256^2..1024^2 cells, omega in [10, 80], 1-4
    sources) solved to 1e-8 as one batch (one launch per tick for all
    problems, CG phase replayed as a hipGraph), FP32 stepping and FP64; nprob
    takes the first problems of the same draw."""
    import torch
    cases = inputs.ragged_batch()[:nprob]
    out = {"workload": f"ragged batch: {nprob} problems, n ~ U{{256..1024}}, omega ~ U[10, 80], 1-4 Gaussian "
                       "sources, random log-normal media, free top", "tol": 1e-8}
    for tag, kw in (("fp64", {}), ("fp32", {"prec": elwh.FP32_STEP})):
        if tag not in precisions:
            continue
        log(f"ragged batch {tag}: solving")
        bt = elwh.Batch(cases, **kw)
        fs = [c.f for c in cases]
        torch.cuda.synchronize()
        _, infos, st = bt.solve(fs, tol=1e-8, maxit=4000)
        s = bt.stats()
        lup = sum(i["iters"] * i["nt"] * unknown_nodes(c) for i, c in zip(infos, cases))
        out[tag] = {"seconds": round(s["seconds"], 3), "status": st, "ticks": s["ticks"],
                    "tiles": {"fp64": s["tile64"], "fp32": s["tile32"]},
                    "iters_mean": round(sum(i["iters"] for i in infos) / len(infos), 1),
                    "max_relres_fp64": max(i["relres_fp64"] for i in infos),
                    "aggregate_glup_s": round(lup / s["seconds"] / 1e9, 2)}
        log(f"ragged batch {tag}: {out[tag]}")
        bt.close()
    return out


def learned_start_comparison(elwh, nprob=512, first_seed=4096, batch=48, learned_fp64_batches=2):
    """The time-to-1e-8 half of the metric on the warm-start workload: nprob
    held-out problems (seeds first_seed..) in batches of `batch`, plain FP64
    from zero against the learned start with FP32 stepping (every batch), and
    the learned start with FP64 stepping on the first batches (the start's own
    iteration reduction, apart from the precision's effect).  Both stop at an
    FP64-recomputed relative residual of 1e-8."""
    from paper_2205_12344_amd import warmstart
    net = elwh.WarmStartNet(max_batch=batch, H=warmstart.N_CELLS, seed=0)
    meta = warmstart.load_weights(net)
    r = warmstart.evaluate(net, list(range(first_seed, first_seed + nprob)), batch=batch, tol=1e-8,
                           zero_fp32=False, learned_fp64_batches=learned_fp64_batches)
    net.close()
    r["workload"] = (f"warm-start workload: {nprob} held-out problems (seeds {first_seed}..{first_seed + nprob - 1}) "
                     f"in batches of {batch}, 256^2 cells, omega ~ U[20, 60], 1-4 Gaussian sources of width U[2h, 6h]")
    r["weights"] = {k: meta.get(k) for k in ("n_train", "epochs", "val_loss_after", "label_tol")}
    return r


# Mapped 3-D grids, one step per launch: state u^n, u^{n-1} read, u^{n+1}
# written (3 x 3 x 8), twelve coefficient arrays (a = c dt^2/(rho J),
# lambda/J, mu/J and the nine metric values, 12 x 8), accumulator read and
# written (2 x 3 x 8): 216 B; FP32 state and coefficients with the
# compensated FP64 accumulator: 36 + 48 + 72 = 156 B
BYTES_PER_LUP_MAPPED3 = {"f64": 216, "f32c": 156}
MAPPED3_WORKLOAD = ("the partial toroidal shell of the 3-D curvilinear experiment (R = 4, 1 <= r <= 2, 0 <= theta, "
                    "phi <= pi, free radial faces) on its smaller grid, 400 x 120 x 40 points, omega = 5.1234, "
                    "constant lambda = 2, mu = rho = 1")


def mapped3_rates(elwh, napply=2):
    """Step-kernel rate of the mapped 3-D kernel on the toroidal shell."""
    import numpy as np
    from paper_2205_12344_amd.inputs import torus_section
    x, y, z = torus_section(399, 119, 39)
    one = np.ones(x.shape)
    nodes = 398 * 118 * 40
    out = {}
    for tag, kw in (("f64", {}), ("f32c", {"prec": elwh.FP32_STEP, "compensated": 1})):
        ctx = elwh.MappedContext3(x, y, z, one, 2 * one, one, 5.1234, bc=(0, 0, 0, 0, 1, 1), **kw)
        p = kernel_rate(ctx, napply)
        avg_s = p["step_ms"] * 1e-3 / max(p["nstep"], 1)
        bb = BYTES_PER_LUP_MAPPED3[tag]
        out[tag] = {"workload": MAPPED3_WORKLOAD, "nt": ctx.info()["nt"], "kernel": "curv3d_kernel",
                    "step_kernel_us": round(1e6 * avg_s, 3), "glup_s_kernel": round(nodes / avg_s / 1e9, 3),
                    "bytes_per_lup": bb, "achieved_GBs": round(bb * nodes / avg_s / 1e9, 1),
                    "frac": round(bb * nodes / avg_s / 1e9 / HBM_PEAK_GBS, 4)}
        log(f"mapped 3-D {tag}: {out[tag]}")
        ctx.close()
    return out


def omega_sweep(elwh, inputs, ks=range(3, 41), tol=1e-8):
    """The iterations-against-frequency experiment of Sec. 5.5 on the GPU: the
    5 x 1 rectangle and the quarter and half annuli (outer arc 5), lambda = 2,
    mu = rho = 1, Dirichlet sides, the standard explicit scheme, about 20
    points per wavelength (n = 4 L omega + 1 cells along a side of length L),
    a discrete point source of amplitude omega^2, omega = k + sqrt(2)/10,
    conjugate residual to 1e-8.  The paper shows the counts only as a figure
    and states that they grow like omega^2 in 2-D; the log-log slope of each
    geometry's counts is reported beside them."""
    import numpy as np
    import torch
    out = {"tol": tol, "scheme": "standard", "krylov": "CR", "rows": []}
    for k in ks:
        w = k + math.sqrt(2) / 10
        row = {"k": k, "omega": round(w, 4)}
        # rectangle, x along the long side
        n = (int(20 * w + 1), int(4 * w + 1))
        shape = (n[1] + 1, n[0] + 1)
        one = np.ones(shape)
        f = np.zeros((2,) + shape)
        f[0, n[1] // 2, n[0] // 10] = w * w / ((5.0 / n[0]) * (1.0 / n[1]))
        runs = [("rectangle", lambda: elwh.Context(2, n, one, 2 * one, one, w, (0, 0, 0, 0), length=(5.0, 1.0),
                                                   scheme=elwh.SCHEME_STANDARD, krylov=elwh.KRYLOV_CR), f)]
        for n_an, key in ((1, "quarter"), (2, "half")):
            x, y, rho, lam, mu, wa, fa = inputs.sector_case(k, n_an)
            runs.append((key, lambda x=x, y=y, rho=rho, lam=lam, mu=mu, wa=wa: elwh.MappedContext(
                x, y, rho, lam, mu, wa, scheme=elwh.SCHEME_STANDARD, krylov=elwh.KRYLOV_CR), fa))
        for key, make, fk in runs:
            ctx = make()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, info = ctx.solve(fk, tol=tol, maxit=20000, raise_on_fail=False)
            el = time.perf_counter() - t0
            ctx.close()
            row[key] = {"iters": info["iters"], "seconds": round(el, 3), "status": info["status"], "nt": info["nt"]}
        out["rows"].append(row)
        log(f"omega sweep k = {k}: " + ", ".join(f"{g} {row[g]['iters']}" for g in ("rectangle", "quarter", "half")))
    for g in ("rectangle", "quarter", "half"):
        ws = [r["omega"] for r in out["rows"] if r[g]["status"] == "OK"]
        its = [r[g]["iters"] for r in out["rows"] if r[g]["status"] == "OK"]
        out[f"slope_{g}"] = round(float(np.polyfit(np.log(ws), np.log(its), 1)[0]), 3) if len(ws) > 1 else None
    return out


def cube_bc_sweep(elwh, inputs, omegas=(4, 6, 8, 10, 12, 16, 20, 24, 32, 40), tol=1e-9):
    """The boundary-condition experiment of Sec. 5.6 on the GPU: the unit cube
    with all faces Dirichlet, or traction-free z = 0, 1 and Dirichlet
    elsewhere; h omega = 0.4, lambda = 2, mu = rho = 1, three Gaussian
    component sources (inputs.cube_bc_case), the standard explicit scheme,
    conjugate residual to 1e-9 from zero.  The paper shows the counts only as
    a figure and states that they grow like omega^3; the log-log slope of
    each boundary set's counts (omega >= 8) is reported beside them."""
    import numpy as np
    import torch
    out = {"tol": tol, "scheme": "standard", "krylov": "CR", "h_omega": 0.4, "rows": []}
    for w in omegas:
        row = {"omega": w}
        for key, fz in (("dirichlet", False), ("free_z", True)):
            c = inputs.cube_bc_case(float(w), free_z=fz)
            ctx = elwh.context_from_case(c, scheme=elwh.SCHEME_STANDARD, krylov=elwh.KRYLOV_CR)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, info = ctx.solve(c.f, tol=tol, maxit=40000, raise_on_fail=False)
            el = time.perf_counter() - t0
            ctx.close()
            row["cells"] = c.n[0]
            row[key] = {"iters": info["iters"], "seconds": round(el, 3), "status": info["status"], "nt": info["nt"],
                        "relres_fp64": info["relres_fp64"]}
        out["rows"].append(row)
        log(f"cube sweep omega = {w} ({row['cells']}^3 cells): dirichlet {row['dirichlet']['iters']}, "
            f"free z {row['free_z']['iters']}")
        torch.cuda.empty_cache()
    for g in ("dirichlet", "free_z"):
        pts = [(r["omega"], r[g]["iters"]) for r in out["rows"] if r[g]["status"] == "OK" and r["omega"] >= 8]
        out[f"slope_{g}"] = (round(float(np.polyfit(np.log([p[0] for p in pts]), np.log([p[1] for p in pts]), 1)[0]), 3)
                             if len(pts) > 1 else None)
    return out


TORUS_CASES = {1: (5.1234, (399, 119, 39), 1490), 2: (10.2468, (399, 119, 39), 2875),
               3: (20.276, (1599, 479, 159), 3713)}


def torus_shell_solve(elwh, case, tol=1e-5, maxit=20000):
    """The toroidal-shell experiment of Sec. 5.11: the partial shell R = 4,
    1 <= r <= 2, 0 <= theta, phi <= pi with free radial faces, lambda = 2,
    mu = rho = 1, forced by sqrt(sigma^3)/20 (1, 1, 1) exp(-zeta^2),
    sigma = 100 omega, zeta^2 = sigma |x - (4, 0.5, 1)|^2 / 2; the conjugate
    residual method to a relative residual of 1e-5, as in the paper.  The
    paper's iteration count (another discretisation) is context only."""
    import numpy as np
    import torch
    from paper_2205_12344_amd.inputs import torus_section
    om, cells, paper_iters = TORUS_CASES[case]
    x, y, z = torus_section(*cells)
    one = np.ones(x.shape)
    sig = 100.0 * om
    g = math.sqrt(sig ** 3) / 20.0 * np.exp(-0.5 * sig * ((x - 4.0) ** 2 + (y - 0.5) ** 2 + (z - 1.0) ** 2))
    f = np.stack([g, g, g])
    ctx = elwh.MappedContext3(x, y, z, one, 2.0 * one, one, om, bc=(0, 0, 0, 0, 1, 1), krylov=elwh.KRYLOV_CR)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, info = ctx.solve(f, tol=tol, maxit=maxit, raise_on_fail=False)
    el = time.perf_counter() - t0
    ctx.close()
    out = {"case": case, "omega": om, "points": [c + 1 for c in cells], "tol": tol, "seconds": round(el, 2),
           "iters": info["iters"], "status": info["status"], "relres_fp64": info["relres_fp64"], "nt": info["nt"],
           "paper_iters_context": paper_iters}
    log(f"toroidal shell case {case}: {out}")
    return out


def counters_pass_3d(rb, tz, prec):
    """Dispatches for the HBM-traffic counters of the 3-D step kernels: the
    256 MiB calibration copy, then two A_h applications of the 256^3
    layered-cube workload with the fixed tiling (RB, TZ) (RB 2, 4, 6: two
    steps per launch; RB 1: single steps), FP64 or FP32 compensated."""
    import torch
    from paper_2205_12344_amd import elwh, inputs
    x = torch.ones(2 ** 25, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    kw = {} if prec == "f64" else {"prec": elwh.FP32_STEP, "compensated": 1}
    ctx = elwh.context_from_case(inputs.layered_cube(), autotune=0, **kw)
    ctx.set_tile(elwh.FP64 if prec == "f64" else elwh.FP32_STEP, int(rb), int(tz))
    z = torch.zeros(ctx.field_shape, dtype=torch.float64, device="cuda")
    for _ in range(2):
        ctx.apply_A(z)
    torch.cuda.synchronize()
    log(f"3-D counters pass done (RB={rb}, TZ={tz}, {prec})")


def counters_pass_twofield(tile):
    """The counter pass of the two-field step kernel: the 256 MiB calibration
    copy, then three A_h applications of the 1024^2 absorbing workload with a
    fixed tiling."""
    import torch
    from paper_2205_12344_amd import elwh, inputs
    parts = [int(t) for t in tile.split(",")]
    v, ty = parts[0], parts[1]
    kw = {"fuse": parts[2]} if len(parts) > 2 else {}     # steps per launch (default: the library's)
    x = torch.ones(2 ** 25, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    ctx = elwh.context_from_case(inputs.absorbing_square(), autotune=0)
    ctx.set_tile(elwh.FP64, v, ty)
    z = torch.zeros(ctx.field_shape, dtype=torch.float64, device="cuda")
    for _ in range(3):
        ctx.apply_A2(z, z)
    torch.cuda.synchronize()
    log(f"two-field counters pass done (tile V={v} TY={ty})")


def counters_pass(tile, mapped=False):
    """Dispatches for the HBM-traffic counters: a plain copy of 256 MiB (the
    scale reference: 262144 KiB read, 262144 KiB written) and three A_h
    applications of the benchmark workload (or of the mapped workload) with
    a fixed FP64 tiling."""
    import torch
    from paper_2205_12344_amd import elwh, inputs
    parts = [int(t) for t in tile.split(",")]
    v, ty = parts[0], parts[1]
    kw = {"fuse": parts[2]} if len(parts) > 2 else {}     # steps per launch (default: the library's)
    x = torch.ones(2 ** 25, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    if mapped:
        xs, ys, rho, lam, mu, om, _ = inputs.sector_case(200, 1, seed=14)
        ctx = elwh.MappedContext(xs, ys, rho, lam, mu, om, autotune=0)
    else:
        ctx = elwh.context_from_case(inputs.random_square(), autotune=0, **kw)
    ctx.set_tile(elwh.FP64, v, ty)
    z = torch.zeros(ctx.field_shape, dtype=torch.float64, device="cuda")
    for _ in range(3):
        ctx.apply_A(z)
    torch.cuda.synchronize()
    log(f"counters pass done (tile V={v} TY={ty})")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--budget", type=float, default=540.0,
                    help="seconds the whole run may take; optional parts that would not fit are skipped")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--quick", action="store_true", help="headline, roofline and kernel rates only")
    ap.add_argument("--cpu-worker", type=float, default=None, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-extras-worker", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--batch-only", action="store_true",
                    help="only the ragged-batch FP64 solve (for kernel traces)")
    ap.add_argument("--batch-problems", type=int, default=48,
                    help="with --batch-only: the first N problems of the ragged batch")
    ap.add_argument("--counters", default=None, metavar="V,TY[,K]",
                    help="only the dispatches for the HBM-traffic counters (benchmark workload, FP64 tiling)")
    ap.add_argument("--counters-mapped", default=None, metavar="V,TY",
                    help="the same for the mapped-grid workload")
    ap.add_argument("--counters-3d", default=None, metavar="RB,TZ,PREC",
                    help="the same for the 256^3 layered cube (PREC f64 or f32c; RB 1 = single steps)")
    ap.add_argument("--counters-twofield", default=None, metavar="V,TY",
                    help="the same for the two-field (impedance) workload")
    ap.add_argument("--twofield-only", action="store_true",
                    help="only the two-field step-kernel measurement and its GMRES solve")
    ap.add_argument("--omega-sweep", action="store_true",
                    help="only the iterations-against-frequency experiment of Sec. 5.5 (k = 3..40, three geometries)")
    ap.add_argument("--torus-shell", default=None, metavar="CASES",
                    help="only the toroidal-shell CR solves of Sec. 5.11 (cases 1, 2, 3, comma-separated)")
    ap.add_argument("--cube-sweep", action="store_true",
                    help="only the boundary-condition experiment of Sec. 5.6 (unit cube, Dirichlet or free z faces)")
    ap.add_argument("--mapped-only", action="store_true",
                    help="only the mapped-grid step-kernel measurement (for kernel traces and counters)")
    args = ap.parse_args()
    if args.cpu_worker is not None:
        cpu_worker(args.cpu_worker)
        return
    if args.cpu_extras_worker:
        cpu_extras_worker()
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the hot path runs on a single MI355X "
              "(sharding across GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)
    t_start = time.perf_counter()

    import torch
    from paper_2205_12344_amd import elwh, inputs

    torch.cuda.set_device(0)
    if args.counters:
        counters_pass(args.counters)
        return
    if args.counters_mapped:
        counters_pass(args.counters_mapped, mapped=True)
        return
    if args.counters_twofield:
        counters_pass_twofield(args.counters_twofield)
        return
    if args.counters_3d:
        rb, tz, prec = args.counters_3d.split(",")
        counters_pass_3d(rb, tz, prec)
        return
    if args.omega_sweep:
        print(json.dumps(omega_sweep(elwh, inputs)))
        return
    if args.cube_sweep:
        print(json.dumps(cube_bc_sweep(elwh, inputs)))
        return
    if args.torus_shell:
        print(json.dumps([torus_shell_solve(elwh, int(k)) for k in args.torus_shell.split(",")]))
        return
    if args.mapped_only:
        print(json.dumps(mapped_rates(elwh, inputs)))
        return
    if args.batch_only:
        print(json.dumps(ragged_batch_solve(elwh, inputs, nprob=args.batch_problems, precisions=("fp64",))))
        return
    if args.twofield_only:
        print(json.dumps(twofield_rates(elwh, inputs, solve=True)))
        return
    t0 = time.perf_counter()
    case = inputs.random_square()
    log(f"workload {case.name}: omega {case.omega:.3f}, inputs {time.perf_counter() - t0:.1f} s")
    nodes = unknown_nodes(case)

    ctx = elwh.context_from_case(case)
    info = ctx.info()
    nt = info["nt"]
    tv, tr = ctx.get_tile(elwh.FP64)
    ctx.cg_begin(case.f)
    el, prof = time_cg(ctx, args.steps, args.warmup)
    lup_per_step = nt * nodes
    value = lup_per_step * args.steps / el
    ms_per_step = 1e3 * el / args.steps
    # every application runs N_T - 1 steps after the half step: K-step
    # launches and, when K does not divide N_T - 1, one shorter launch
    napp = prof["nstep"] // max(nt - 1, 1)
    fuse = elwh.default_opts().fuse
    bytes_app, launches_app = phase_bytes(2, "f64", fuse, nt, nodes)
    phase_gbs = bytes_app * napp / (prof["step_ms"] * 1e-3) / 1e9
    # the dominant kernel alone: the same workload and tiling with N_T
    # rounded up so that K divides N_T - 1 (the weights change, the kernel's
    # work per launch does not); HIP events on the context's stream
    nt_k = fuse * ((nt - 1 + fuse - 1) // fuse) + 1
    ck = elwh.context_from_case(case, nt=nt_k, autotune=0)
    ck.set_tile(elwh.FP64, tv, tr)
    pk = kernel_rate(ck, 10)
    ck.close()
    step_avg_ms = pk["step_ms"] / max(pk["nstep"] // fuse, 1)
    achieved = BYTES_PER_MULTI_LAUNCH["f64"] * nodes / (step_avg_ms * 1e-3) / 1e9
    traffic = read_traffic(f"multi2d_k{fuse}_f64_square1024", (tv, tr))
    log(f"tile V={tv} TY={tr}")
    log(f"fp64: {ms_per_step:.3f} ms/step, {value / 1e9:.2f} GLUP/s, {fuse}-step kernel {1e3 * step_avg_ms:.2f} us "
        f"({pk['nstep'] // fuse} launches at N_T = {nt_k}), {achieved:.0f} GB/s; step phase of the CG "
        f"iteration {phase_gbs:.0f} GB/s")
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic,
                "kernel": f"multi2d_kernel<double,V={tv},TY={tr},K={fuse},FORCE=0,COMP=0>",
                "bytes_per_lup": BYTES_PER_MULTI_LAUNCH["f64"] / fuse, "lup_per_launch": fuse * nodes,
                "bytes_per_launch": BYTES_PER_MULTI_LAUNCH["f64"] * nodes,
                "avg_launch_us": round(1e3 * step_avg_ms, 3),
                "launch_timing": f"{pk['nstep'] // fuse} launches, same workload and tiling at N_T = {nt_k}",
                # bytes the counters saw moved per launch over the same duration
                "traffic_GBs": round(traffic / (step_avg_ms * 1e-3) / 1e9, 1) if traffic else None,
                "step_phase_GBs": round(phase_gbs, 1),
                # effective fraction: lattice updates per second times the
                # single-step algorithmic bytes (104 B/LUP), the measure under
                # which temporal blocking can exceed 1 (the K-step kernel
                # needs 120/K B/LUP, frac above)
                "effective_frac_kernel": round(fuse * nodes / (step_avg_ms * 1e-3) * BYTES_PER_LUP[(2, "f64", 1)]
                                               / (HBM_PEAK_GBS * 1e9), 4),
                "effective_frac_end_to_end": round(value * BYTES_PER_LUP[(2, "f64", 1)] / (HBM_PEAK_GBS * 1e9), 4),
                "note": (f"temporal blocking: {fuse} time steps per launch at 120 B per node and launch "
                         f"({BYTES_PER_MULTI_LAUNCH['f64'] / fuse:g} B per lattice update); frac prices the kernel "
                         "at its own bytes, effective_frac_* price lattice updates at the single step's 104 B; "
                         "the launch is latency- and issue-bound at two waves per SIMD, not bandwidth-bound")}
    ctx.close()

    variants = {}
    vlist = [("f32c", "f32c", {"prec": elwh.FP32_STEP, "compensated": 1}),
             ("f32", "f32", {"prec": elwh.FP32_STEP, "compensated": 0})]
    for k in (1, 2, 3, 4):
        if k != fuse:
            vlist.append((f"f64_fuse{k}", "f64", {"fuse": k}))
    for k in (1, 3, 4):
        vlist.append((f"f32c_fuse{k}", "f32c", {"prec": elwh.FP32_STEP, "compensated": 1, "fuse": k}))
    for tag, prec, kw in vlist:
        fuse_v = kw.setdefault("fuse", fuse)
        c2 = elwh.context_from_case(case, **kw)
        p = kernel_rate(c2, 10)
        t2 = c2.get_tile(elwh.FP64 if prec == "f64" else elwh.FP32_STEP)
        napp = p["nstep"] // max(nt - 1, 1)
        bapp, lapp = phase_bytes(2, prec, fuse_v, nt, nodes)
        gbs = bapp * napp / (p["step_ms"] * 1e-3) / 1e9
        variants[tag] = {"tile": list(t2), "steps_per_launch": fuse_v,
                         "launch_us": round(1e3 * p["step_ms"] / max(napp * lapp, 1), 3),
                         "glup_s_kernel": round(napp * (nt - 1) * nodes / (p["step_ms"] * 1e-3) / 1e9, 3),
                         "bytes_per_lup": round(bapp / ((nt - 1) * nodes), 2), "achieved_GBs": round(gbs, 1),
                         "frac": round(gbs / HBM_PEAK_GBS, 4)}
        log(f"{tag}: {variants[tag]}")
        c2.close()

    ceiling = triad_ceiling(elwh)
    log(f"HBM ceiling: {ceiling}")

    # the same kernel where the working set (~2 GB) is far beyond the 256 MB
    # Infinity Cache: the benchmark workload's construction at 4096^2
    c4k = inputs.random_square(n=4096)
    n4k = unknown_nodes(c4k)
    ctx4k = elwh.context_from_case(c4k)
    nt4k = ctx4k.info()["nt"]
    p = kernel_rate(ctx4k, 3)
    t4k = ctx4k.get_tile(elwh.FP64)
    napp = p["nstep"] // max(nt4k - 1, 1)
    bapp, lapp = phase_bytes(2, "f64", fuse, nt4k, n4k)
    gbs = bapp * napp / (p["step_ms"] * 1e-3) / 1e9
    variants["f64_square4096"] = {
        "workload": "the benchmark workload's construction at 4096^2 cells (random medium, free top, omega for 10 "
                    "points per shear wavelength)", "nt": nt4k, "unknown_nodes": n4k, "tile": list(t4k),
        "steps_per_launch": fuse, "launch_us": round(1e3 * p["step_ms"] / max(napp * lapp, 1), 2),
        "glup_s_kernel": round(napp * (nt4k - 1) * n4k / (p["step_ms"] * 1e-3) / 1e9, 3),
        "achieved_GBs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
        "frac_of_triad": round(gbs / ceiling["triad_GBs"], 4)}
    log(f"4096^2: {variants['f64_square4096']}")
    ctx4k.close()
    del c4k
    torch.cuda.empty_cache()

    # 3-D step kernels on the 256^3 layered cube: the tiling the autotuner
    # picks (two steps per launch where that is faster), and single steps
    c3 = inputs.layered_cube()
    n3 = unknown_nodes(c3)
    for tag, kw in (("f64", {}), ("f32c", {"prec": elwh.FP32_STEP, "compensated": 1})):
        for fuse3 in (2, 1):
            ctx3 = elwh.context_from_case(c3, fuse=fuse3, **kw)
            nt3 = ctx3.info()["nt"]
            p = kernel_rate(ctx3, 2)
            step_us = 1e3 * p["step_ms"] / max(p["nstep"], 1)      # per time step
            rb, tz = ctx3.get_tile(elwh.FP32_STEP if tag != "f64" else elwh.FP64)
            two = fuse3 >= 2 and rb >= 2
            # the N_T - 1 steps after the half step: pair launches, and one
            # single step when N_T - 1 is odd
            pairs = (nt3 - 1) // 2 if two else 0
            single = (nt3 - 1) - 2 * pairs
            bytes_app = (pairs * BYTES_PER_LAUNCH_3D_K2[tag] + single * BYTES_PER_LUP[(3, tag, 1)]) * n3
            bytes_per_lup = bytes_app / ((nt3 - 1) * n3)
            gbs = bytes_per_lup * n3 / step_us / 1e3
            key = "3d_" + tag + ("" if fuse3 >= 2 else "_single")
            variants[key] = {"workload": c3.name, "nt": nt3, "tile_rows_planes": [rb, tz],
                             "steps_per_launch": 2 if two else 1, "step_us": round(step_us, 2),
                             "launches_per_application": pairs + single,
                             "glup_s_kernel": round(n3 / step_us / 1e3, 3),
                             "bytes_per_lup": round(bytes_per_lup, 2), "achieved_GBs": round(gbs, 1),
                             "frac": round(gbs / HBM_PEAK_GBS, 4),
                             "frac_of_triad": round(gbs / ceiling["triad_GBs"], 4),
                             # lattice updates per second times the FP64
                             # single-step algorithmic bytes (144 B/LUP) in
                             # both precisions, so that FP64 and FP32 compare
                             "effective_frac": round(BYTES_PER_LUP[(3, "f64", 1)] * n3 / step_us / 1e3
                                                     / HBM_PEAK_GBS, 4),
                             "traffic": read_traffic(f"step3d_{tag}_cube256", (rb, tz), "3d")}
            log(f"3d {tag} fuse {fuse3}: tile {rb},{tz}, {step_us:.1f} us per step, {gbs:.0f} GB/s")
            ctx3.close()
    del c3
    torch.cuda.empty_cache()

    for tag, v in mapped_rates(elwh, inputs).items():
        variants["mapped_" + tag] = v
    for tag, v in mapped3_rates(elwh).items():
        variants["mapped3d_" + tag] = v
    variants["twofield_f64"] = twofield_rates(elwh, inputs, solve=False)
    torch.cuda.empty_cache()

    # optional parts, in order of importance, inside the time budget
    extra = {}
    deadline = t_start + args.budget
    cpu_s = 0.0 if args.no_cpu else 60.0       # what the CPU leg at the end needs

    def fits(name, est_s):
        left = deadline - time.perf_counter() - cpu_s
        if args.quick or left < est_s:
            why = "--quick" if args.quick else f"time budget (needs about {est_s:.0f} s, {max(left, 0):.0f} s left)"
            extra[name] = {"skipped": why}
            log(f"{name}: skipped")
            return False
        return True

    if fits("time_to_1e-8", 210):
        extra["time_to_1e-8"] = learned_start_comparison(elwh)
        log(f"time to 1e-8: {json.dumps(extra['time_to_1e-8'])}")
        if fits("time_to_1e-8_sequential", 40):
            seq = sequential_plain(elwh)
            per = extra["time_to_1e-8"].get("plain_fp64_seconds_per_batch") or [None]
            seq["batched_seconds_same_problems"] = per[0]
            extra["time_to_1e-8"]["plain_fp64_unbatched_first48"] = seq
            log(f"unbatched plain FP64, first 48: {seq}")
    if fits("ragged_batch48", 165):
        extra["ragged_batch48"] = ragged_batch_solve(elwh, inputs, precisions=("fp32",))
    if fits("solves_to_1e-8", 60):
        extra["solves_to_1e-8"] = solves_2d_and_3d(elwh, inputs)
    if fits("ragged_batch48_fp64", 130):
        extra.setdefault("ragged_batch48", {}).update(ragged_batch_solve(elwh, inputs, precisions=("fp64",)))
    torch.cuda.synchronize()

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline()
        log(f"cpu oracle: {cpu['value'] / 1e6:.2f} MLUP/s on {cpu['cores']} cores, "
            f"{cpu['one_core']['value'] / 1e6:.2f} MLUP/s on one ({cpu['sample']})")
        cpu["other_timings_one_core"] = cpu_extras()
        log(f"cpu oracle, config 1 and a 64^3 sample of config 3: {cpu['other_timings_one_core']}")

    out = {
        "metric": METRIC, "value": value, "unit": "LUP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "2-D 1024x1024 cells, random log-normal medium (corr. length 0.1, sigma 0.2, "
                               "lambda/mu in [1,3]), Dirichlet sides and bottom, traction-free top, one "
                               "Gaussian source, omega for 10 points per shear wavelength; one CG iteration "
                               "per step",
                   "grid": list(case.n), "omega": case.omega, "nt": nt, "unknown_nodes": nodes,
                   "lup_per_step": lup_per_step},
        "roofline": roofline, "cpu_baseline": cpu, "hbm_ceiling": ceiling, "variants": variants, **extra,
        "bench_seconds": round(time.perf_counter() - t_start, 1),
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
