"""Build libelwh.so (HIP for gfx950) in-tree with hipcc.

``python -m paper_2205_12344_amd.build`` compiles every source under csrc/
into paper_2205_12344_amd/libelwh.so.  It runs on a machine without a GPU
(hipcc cross-compiles the device code).
"""

import os
import shutil
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libelwh.so")
SOURCES = ["api.hip", "batch.hip", "batch_kernels.hip", "kernels2d.hip", "kernels2d_multi.hip", "kernels2d_curv.hip", "kernels2d_damped.hip", "kernels3d.hip", "kernels3d_k2.hip", "kernels3d_curv.hip", "blas.hip", "nn.hip", "nn_kernels.hip",
           "noalloc.hip", "plan.cpp"]
ARCH = "gfx950"


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def flags():
    return [
        f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result",
        # keep the compiler from forming packed FP32 instructions
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", os.path.join(HERE, "..", "include"),
    ]


def build(verbose=True, jobs=None):
    """Compile every source to an object, then link libelwh.so; always rebuilds."""
    t0 = time.time()
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    cc = hipcc()
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src + ".o")
        objs.append(obj)
        cmd = [cc] + flags() + ["-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((src, cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = False
    for src, cmd, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            failed = True
            sys.stderr.write(f"[build] {src} failed:\n{' '.join(cmd)}\n{out.decode(errors='replace')}\n")
        elif verbose and out.strip():
            sys.stderr.write(out.decode(errors="replace"))
    if failed:
        raise RuntimeError("libelwh build failed")
    tmp = LIB + ".tmp"
    link = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs + ["-pthread"]
    r = subprocess.run(link, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout.decode(errors="replace"))
    os.replace(tmp, LIB)
    if verbose:
        print(f"[build] {LIB} ({time.time() - t0:.1f} s)")
    return LIB


if __name__ == "__main__":
    build()
