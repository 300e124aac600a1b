"""Pins of the reconstruction-driver oracle (oracle/recon.py) against what the
paper and linear algebra fix: the TV difference operator and its Laplacian,
the gradient of the smoothed TV functional (eq jm), positivity of M_gamma,
the Krylov optimality of Algorithm 4, its stopping rule, and the outer loop of
Algorithm 5 on problems with a known answer."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import qpat_inputs as qi
from oracle import kspace as K
from oracle import recon as R


def laplacian_brute(ny, nx):
    """5-point graph Laplacian of the ny x nx grid with Neumann ends, by loops."""
    n = ny * nx
    L = np.zeros((n, n))
    for j in range(ny):
        for i in range(nx):
            a = j * nx + i
            for dj, di in ((0, 1), (1, 0), (0, -1), (-1, 0)):
                jj, ii = j + dj, i + di
                if 0 <= jj < ny and 0 <= ii < nx:
                    L[a, a] += 1.0
                    L[a, jj * nx + ii] -= 1.0
    return L


def test_difference_operator_is_the_grid_graph():
    ny, nx = 5, 7
    D = R.tv_difference(ny, nx)
    assert D.shape == (ny * (nx - 1) + (ny - 1) * nx, ny * nx)
    assert np.allclose(D @ np.ones(ny * nx), 0.0)
    assert np.array_equal((D.T @ D).toarray(), laplacian_brute(ny, nx))


def test_tv_gradient_is_m_times_x():
    rng = np.random.default_rng(5)
    ny, nx, beta = 6, 8, 2e-3
    D = R.tv_difference(ny, nx)
    x = rng.standard_normal(ny * nx)
    g = R.tv_matrix(D, x, beta, 0.0) @ x
    h = 1e-6
    fd = np.array([(R.tv_value(D, x + h * e, beta) - R.tv_value(D, x - h * e, beta)) / (2 * h)
                   for e in np.eye(ny * nx)])
    assert np.linalg.norm(fd - g) / np.linalg.norm(g) < 1e-7


def test_m_gamma_is_symmetric_positive_definite():
    rng = np.random.default_rng(6)
    D = R.tv_difference(5, 6)
    gamma = 1e-6
    M = R.tv_matrix(D, rng.standard_normal(30), 2e-5, gamma).toarray()
    assert np.allclose(M, M.T, atol=0)
    ev = np.linalg.eigvalsh(M)
    assert ev.min() > 0.5 * gamma
    # the constant vector is in the kernel of D^T C D: its eigenvalue is gamma
    assert np.allclose(M @ np.ones(30), gamma)


def spd(n, seed, cond=50.0):
    rng = np.random.default_rng(seed)
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return (q * np.geomspace(1.0, cond, n)) @ q.T


def test_pcg_iterates_are_krylov_optimal():
    """After k steps, Algorithm 4 minimises the H-norm of the error over
    x in span{(M^-1 H)^i M^-1 r0, i < k} (brute-force least squares)."""
    n = 24
    H, M = spd(n, 1), spd(n, 2, cond=8.0)
    g = np.random.default_rng(3).standard_normal(n)
    xs = -np.linalg.solve(H, g)
    Minv = np.linalg.inv(M)
    for k in (1, 3, 6):
        x, _, it = R.pcg(lambda v: H @ v, g, lambda r: Minv @ r, k, 10 ** 9, 0.0)
        assert it == k
        basis = [Minv @ (-g)]
        for _ in range(k - 1):
            basis.append(Minv @ (H @ basis[-1]))
        V = np.linalg.qr(np.array(basis).T)[0]
        # minimise (x - xs)^T H (x - xs) over x = V c
        c = np.linalg.solve(V.T @ H @ V, V.T @ H @ xs)
        assert np.linalg.norm(x - V @ c) / np.linalg.norm(xs) < 1e-10


def test_pcg_without_preconditioner_is_cg_and_converges():
    n = 20
    H = spd(n, 4)
    g = np.random.default_rng(7).standard_normal(n)
    seen = []
    spla.cg(H, -g, rtol=1e-14, maxiter=3, callback=lambda xk: seen.append(xk.copy()))
    x, _, _ = R.pcg(lambda v: H @ v, g, lambda r: r.copy(), 3, 10 ** 9, 0.0)
    assert np.linalg.norm(x - seen[-1]) / np.linalg.norm(x) < 1e-10
    x, _, _ = R.pcg(lambda v: H @ v, g, lambda r: r.copy(), 4 * n, 10 ** 9, -np.inf)
    assert np.linalg.norm(H @ x + g) / np.linalg.norm(g) < 1e-10


def test_pcg_stopping_rule():
    n = 20
    H = spd(n, 8)
    g = np.random.default_rng(9).standard_normal(n)
    # 1 - ratio > 1 never holds for positive r.z: the loop stops at i = i_m
    _, rz, it = R.pcg(lambda v: H @ v, g, lambda r: r.copy(), 30, 4, 1.0)
    assert it == 4 and len(rz) == 5
    _, _, it = R.pcg(lambda v: H @ v, g, lambda r: r.copy(), 7, 2, -np.inf)
    assert it == 7


def test_ld_identity_operator_recovers_the_data_in_one_step():
    """With H = I (forward = identity) the normal equation of the first outer
    step has the solution d = data - x0; a full PCG solve lands on it."""
    rng = np.random.default_rng(10)
    ny, nx = 6, 5
    data = rng.standard_normal((ny, nx))
    x0 = rng.standard_normal((ny, nx))
    x, hist, iters = R.ld_newton(lambda v: v, lambda r: r, data, x0, beta=0.1, gamma=0.1,
                                 i_max=4 * ny * nx, i_m=10 ** 6, tol_in=-np.inf, tol_out=0.5, outer_max=1)
    assert np.abs(x - data).max() < 1e-9
    assert hist[-1] < 1e-18 * max(hist[0], 1.0)


def test_ld_reduces_the_misfit_on_an_acoustic_problem():
    """Noise-free data of a small lossy solve: every outer step lowers eps
    (the paper's observation for alpha = 1) and the image approaches p0."""
    n, nt = 24, 40
    c0, rho0 = qi.medium(n, n, 41, 42, sigma_cells=3.0)
    dx = 1e-4
    prm = qi.make_params(n, n, dx, 0.3 * dx / c0.max(), nt, c0.max(), qi.ring_sensors(16, 9, dx),
                         pml_size=4, alpha0_db=0.75)
    ops = K.Operators(prm, c0, rho0)
    p0 = qi.blobs(n, n, 43, count=3, radius_cells=4.0)
    data = K.forward(prm, c0, rho0, p0, ops=ops)
    fwd = lambda v: K.forward(prm, c0, rho0, v, ops=ops)
    adj = lambda r: K.adjoint(prm, c0, rho0, r, ops=ops)
    x, hist, iters = R.ld_newton(fwd, adj, data, np.zeros((n, n)), beta=1e-4, gamma=1e-6,
                                 i_max=6, i_m=3, tol_in=0.0, tol_out=1e-6, outer_max=3)
    assert all(b < a for a, b in zip(hist, hist[1:]))
    assert hist[-1] < 0.2 * hist[0]
    assert np.linalg.norm(x - p0) < np.linalg.norm(p0)
