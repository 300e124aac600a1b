"""qpat_dot_noalloc (the inner product whose partial sums sit in a static
device array, for callers that cannot allocate) against qpat_dot, through the
C ABI: same kernels, so the same bits, on two calls in a row with the second
on a smaller input (the array keeps the first call's partials), and against
an FP64 host dot product."""
import ctypes

import numpy as np
import pytest

import qpat_inputs as qi

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1810_11685_amd as q
    return q


def test_dot_noalloc_matches_dot(q):
    import torch
    L = q.lib()
    s = torch.cuda.current_stream().cuda_stream
    for n, seed in ((1_000_003, 1), (70_001, 5)):
        a = qi.gaussian_field(n, seed)
        b = qi.gaussian_field(n, seed + 1)
        ta = torch.as_tensor(a, dtype=torch.float32, device="cuda")
        tb = torch.as_tensor(b, dtype=torch.float32, device="cuda")
        o1 = torch.full((), np.nan, dtype=torch.float64, device="cuda")
        o2 = torch.full((), np.nan, dtype=torch.float64, device="cuda")
        assert L.qpat_dot_noalloc(ta.data_ptr(), tb.data_ptr(), n, o1.data_ptr(), s) == 0
        assert L.qpat_dot(ta.data_ptr(), tb.data_ptr(), n, o2.data_ptr(), s) == 0
        torch.cuda.synchronize()
        got, ref = float(o1.cpu()), float(o2.cpu())
        assert got == ref
        exact = float(np.dot(a.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)))
        assert abs(got - exact) <= 1e-12 * np.sqrt(np.dot(a, a) * np.dot(b, b))


def test_dot_noalloc_checks(q):
    import torch
    L = q.lib()
    o = torch.zeros((), dtype=torch.float64, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    assert L.qpat_dot_noalloc(None, None, 0, o.data_ptr(), s) == 0
    torch.cuda.synchronize()
    assert float(o.cpu()) == 0.0
    assert L.qpat_dot_noalloc(None, None, -1, o.data_ptr(), s) == 1
    assert L.qpat_dot_noalloc(None, None, (1 << 40) + 1, o.data_ptr(), s) == 1
    assert L.qpat_dot_noalloc(None, None, 5, o.data_ptr(), s) == 1
    assert L.qpat_dot_noalloc(None, None, 5, None, s) == 1
