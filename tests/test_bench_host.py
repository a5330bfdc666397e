"""Host-side checks of the benchmark's bookkeeping (no GPU): how the N_T - 1
steps after the half step split into launches, the algorithmic bytes priced
on them, the remainder-free N_T used to time the K-step kernel alone, and
the refusal of more than one GPU."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.mark.parametrize("nt,fuse,expect", [
    (63, 4, [4] * 15 + [2]),        # the 1024^2 benchmark workload
    (63, 2, [2] * 31),
    (64, 4, [4] * 15 + [3]),
    (66, 4, [4] * 16 + [1]),
    (5, 3, [3, 1]),
    (3, 4, [2]),
    (6, 1, [1] * 5),
])
def test_step_launches_split_like_the_library(nt, fuse, expect):
    """K-step launches while K or more steps are left, then one shorter
    multi-step launch for two or three steps, or one single step."""
    got = bench.step_launches(nt, fuse)
    assert got == expect
    assert sum(got) == nt - 1


@pytest.mark.parametrize("nt", [4, 9, 63, 64, 65, 66, 121])
@pytest.mark.parametrize("fuse", [2, 3, 4])
def test_remainder_free_nt_gives_only_k_step_launches(nt, fuse):
    nt_k = fuse * ((nt - 1 + fuse - 1) // fuse) + 1
    assert nt_k >= nt and nt_k - nt < fuse
    assert set(bench.step_launches(nt_k, fuse)) == {fuse}


def test_phase_bytes_price_each_launch():
    nodes = 1047552
    b, n = bench.phase_bytes(2, "f64", 4, 63, nodes)
    assert n == 16
    assert b == 16 * bench.BYTES_PER_MULTI_LAUNCH["f64"] * nodes
    b1, n1 = bench.phase_bytes(2, "f64", 1, 63, nodes)
    assert n1 == 62 and b1 == 62 * bench.BYTES_PER_LUP[(2, "f64", 1)] * nodes
    # a single-step remainder is priced at the single step's bytes
    b2, n2 = bench.phase_bytes(2, "f32c", 4, 66, nodes)
    assert n2 == 17
    assert b2 == (16 * bench.BYTES_PER_MULTI_LAUNCH["f32c"] + bench.BYTES_PER_LUP[(2, "f32c", 1)]) * nodes


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
