"""CPU checks of the benchmark's contract that need no GPU: more than one GPU
is refused with a message, and the algorithmic byte counts it reports follow
their stated per-pass sums."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_byte_counts():
    import bench
    # 2-D: each forward and adjoint iterate moves 160 B per point in the 12 passes
    fwd = [bench.PASS_BYTES[i] for i in range(6)]
    adj = [bench.PASS_BYTES[i] for i in range(6, 12)]
    assert sum(fwd) == 160 and sum(adj) == 160
    # 3-D: per pass (field bytes, half-spectrum bytes in units of h = (nx/2 + 1)/nx)
    fwd3 = [(0, 36), (36, 48), (0, 52), (28, 40), (0, 40), (24, 24)]
    adj3 = [(16, 40), (0, 40), (32, 40), (0, 52), (36, 48), (0, 52)]
    for nx in (49, 64):
        h = (nx // 2 + 1) / nx
        assert bench.bytes_3d_pair(nx) == pytest.approx(sum(a + b * h for a, b in fwd3 + adj3))
    assert bench.bytes_3d_pair(49) == pytest.approx(433.22, abs=0.01)
    # optical CG iteration: A p 48, update 48, r.z 16, direction 24; V-cycle 108 per
    # level node (restriction 50, correction + post-sweep 58) over 4/3 of the fine nodes
    assert bench.OPT_BYTES_PER_NODE_ITER == pytest.approx(48 + 48 + 16 + 24 + (50 + 58) * 4 / 3)
