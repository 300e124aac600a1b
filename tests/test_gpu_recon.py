"""GPU parity of the reconstruction driver's pieces and of the driver itself
against the oracle (oracle/recon.py): TV weights, M_gamma, the M_gamma solve,
the TV value, axpby, and Algorithms 4 / 5 on batched J^T J v."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import qpat_inputs as qi
from oracle import kspace as K
from oracle import recon as R

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1810_11685_amd as q
    return q


def T(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float32, device="cuda")


def N(t):
    return t.detach().double().cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, float) - b) / np.linalg.norm(b))


@pytest.mark.parametrize("ny,nx", [(48, 64), (37, 50), (3, 2), (512, 512)])
def test_tv_apply_solve_value_match_oracle(q, ny, nx):
    """Odd sizes give multigrid aggregates of one column or row; 3 x 2 has
    three levels.  At 512^2 the V-cycle keeps the CG iterations few."""
    rng = np.random.default_rng(ny + nx)
    B, beta, gamma = 2, 2e-3, 1e-2
    xs = np.stack([qi.blobs(ny, nx, 7 + b, count=4, radius_cells=min(ny, nx) / 8) for b in range(B)])
    xs = xs.astype(np.float32).astype(float)        # the library sees the float32 fields
    us = rng.standard_normal((B, ny, nx)).astype(np.float32).astype(float)
    tv = q.TV(nx, ny, B)
    tv.set_weights(T(xs), beta)
    D = R.tv_difference(ny, nx)
    got = N(tv.apply(T(us), gamma))
    z, it = tv.solve(T(us), gamma, tol=1e-7, max_iter=50000)
    vals = tv.value(T(xs), beta)
    for b in range(B):
        M = R.tv_matrix(D, xs[b], beta, gamma)
        assert rel(got[b].ravel(), M @ us[b].ravel()) <= 1e-6
        ref = spla.spsolve(M.tocsc(), us[b].ravel())
        assert rel(N(z)[b].ravel(), ref) <= 1e-5
        assert abs(vals[b] - R.tv_value(D, xs[b], beta)) <= 1e-9 * R.tv_value(D, xs[b], beta)
    assert 0 < it < 50000
    if nx == 512:
        assert it <= 200, it      # the diagonal preconditioner needed thousands
    tv.close()


def test_axpby(q):
    rng = np.random.default_rng(3)
    x = rng.standard_normal(1000).astype(np.float32)
    y = rng.standard_normal(1000).astype(np.float32)
    yt = T(y)
    q.axpby(0.5, T(x), -2.0, yt)
    assert np.allclose(N(yt), 0.5 * x.astype(float) - 2.0 * y, rtol=1e-6, atol=1e-6)


def small_problem(n=64, nt=120, ns=24, seed=51):
    c0, rho0 = qi.medium(n, n, seed, seed + 1, sigma_cells=4.0)
    dx = 1e-4
    prm = qi.make_params(n, n, dx, 0.3 * dx / c0.max(), nt, c0.max(), qi.ring_sensors(ns, 0.38 * n, dx),
                         pml_size=8, alpha0_db=0.75)
    return prm, c0, rho0


def test_ld_reconstruct_matches_oracle(q):
    """Two data sets, fixed iteration counts (tol_in = tol_out = -inf) so both
    sides run the same steps: images and misfit histories agree.  beta and
    gamma keep M_gamma moderately conditioned: with gamma near the paper's
    1e-6 the priorconditioned PCG amplifies rounding so much that the FP64
    oracle itself, fed operator outputs rounded to FP32, moves by several %."""
    prm, c0, rho0 = small_problem()
    n = prm["nx"]
    ops = K.Operators(prm, c0, rho0)
    p0s = [qi.blobs(n, n, 61 + b, count=3, radius_cells=6.0) for b in range(2)]
    datas = [K.forward(prm, c0, rho0, p, ops=ops) for p in p0s]
    kw = dict(beta=1e-2, gamma=1e-1, i_max=4, i_m=2, tol_in=-np.inf, tol_out=-np.inf, outer_max=2)
    plan = q.Plan(prm, c0, rho0)
    x, hist, iters, solves = q.ld_reconstruct(plan, T(np.stack(datas)), T(np.zeros((2, n, n))),
                                              solve_tol=1e-7, **kw)
    fwd = lambda v: K.forward(prm, c0, rho0, v, ops=ops)
    adj = lambda r: K.adjoint(prm, c0, rho0, r, ops=ops)
    for b in range(2):
        xr, hr, ir = R.ld_newton(fwd, adj, datas[b], np.zeros((n, n)), **kw)
        assert iters[b] == ir == [4, 4]
        assert rel(N(x)[b], xr) <= 1e-3
        # the misfit falls ~2000x in two outer steps; FP32 rounding of the
        # operators moves the last value by ~1e-3 of itself (with the inner
        # solve converged to 1e-11), ~6e-7 of the first misfit
        assert np.allclose(hist[b], hr, rtol=1e-3, atol=1e-6 * hr[0])
        assert hist[b][-1] < hist[b][0]
    assert solves > 0


def test_ld_reconstruct_stops_like_the_paper(q):
    """With the paper's rule (tol_in = 0) every data set stops its PCG loop by
    itself, the outer loop ends at tol_out, and the misfit decreases."""
    prm, c0, rho0 = small_problem(seed=71)
    n = prm["nx"]
    ops = K.Operators(prm, c0, rho0)
    p0 = qi.blobs(n, n, 81, count=3, radius_cells=6.0)
    data = K.forward(prm, c0, rho0, p0, ops=ops)
    plan = q.Plan(prm, c0, rho0)
    x, hist, iters, _ = q.ld_reconstruct(plan, T(data[None]), T(np.zeros((1, n, n))), beta=1e-3, gamma=1e-4,
                                         i_max=30, i_m=5, tol_in=0.0, tol_out=1e-2, outer_max=6)
    h = hist[0]
    assert all(b < a for a, b in zip(h, h[1:]))
    assert len(h) <= 7 and all(1 <= it <= 30 for it in iters[0])
    assert rel(N(x)[0], p0) < 0.1
