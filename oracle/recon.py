"""Oracle of the inexact-Newton reconstruction driver: lagged-diffusivity TV
priorconditioning (Section 5.2 of the paper: eqs tvm, dd, jm, m, m1, pre),
the PCG loop of Algorithm 4 and the outer loop of Algorithm 5, for the
acoustic-only problem of recovering p0 from sensor data.

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this module; the library never imports it.

Readings (the paper states the method for log-scaled optical coefficients on
an FEM mesh; here the unknown is p0 itself on the acoustic grid):
  * X-bar = p0 (identity scaling, so dX/dX-bar = I in eqs gr and apj); with
    several data sets (illuminations q) the problems are independent and are
    solved side by side.
  * The TV "elements" are the grid nodes and its "internal edges" the pairs of
    horizontally or vertically adjacent nodes; every edge has the same length,
    taken as a_l = 1 (a common edge length only rescales beta and gamma).
  * Algorithm 4 is followed as printed: the loop runs while i < i_max and
    (i < i_m or 1 - r_i.z_i / r_{i-i_m}.z_{i-i_m} > Tol_in); M_gamma z = r is
    solved exactly (sparse direct solve).
  * Algorithm 5: step alpha = 1; the loop runs while k = 0 or
    1 - eps^k / eps^{k-1} > Tol_out, with an added cap on outer iterations.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def tv_difference(ny: int, nx: int) -> sp.csr_matrix:
    """D of eq dd for one field on an ny x nx grid (nodes numbered row-major):
    one row per internal edge, +1 at the first node and -1 at the second;
    horizontal edges (j, i)-(j, i+1) first, then vertical (j, i)-(j+1, i)."""
    idx = np.arange(ny * nx).reshape(ny, nx)
    a = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()])
    b = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()])
    nl = a.size
    rows = np.concatenate([np.arange(nl), np.arange(nl)])
    cols = np.concatenate([a, b])
    vals = np.concatenate([np.ones(nl), -np.ones(nl)])
    return sp.csr_matrix((vals, (rows, cols)), shape=(nl, ny * nx))


def tv_weights(D: sp.csr_matrix, x: np.ndarray, beta: float) -> np.ndarray:
    """Diagonal of C[X] (eq m1): (|D x|^2 + beta)^(-1/2), one entry per edge."""
    g = D @ np.asarray(x, float).ravel()
    return 1.0 / np.sqrt(g * g + beta)


def tv_matrix(D: sp.csr_matrix, x: np.ndarray, beta: float, gamma: float) -> sp.csr_matrix:
    """M_gamma = D^T C[x] D + gamma I (eq m, with the shift of the LD method)."""
    C = sp.diags(tv_weights(D, x, beta))
    n = D.shape[1]
    return (D.T @ C @ D + gamma * sp.identity(n)).tocsr()


def tv_value(D: sp.csr_matrix, x: np.ndarray, beta: float) -> float:
    """Smoothed TV functional sum_l sqrt((D x)_l^2 + beta); its gradient is
    M[x] x (eq jm)."""
    g = D @ np.asarray(x, float).ravel()
    return float(np.sum(np.sqrt(g * g + beta)))


def pcg(apply_h, grad: np.ndarray, solve_m, i_max: int, i_m: int, tol_in: float):
    """Algorithm 4: PCG for H d = -grad with preconditioner M (solve_m(r)
    returns M^-1 r).  Returns (d, list of r_i.z_i, iterations)."""
    g = np.asarray(grad, float).ravel()
    x = np.zeros_like(g)
    r = -g
    z = solve_m(r)
    d = z.copy()
    rz = [float(r @ z)]
    i = 0
    while i < i_max and (i < i_m or 1.0 - rz[i] / rz[i - i_m] > tol_in):
        hd = apply_h(d)
        alpha = rz[i] / float(d @ hd)
        x = x + alpha * d
        r = r - alpha * hd
        z = solve_m(r)
        rz.append(float(r @ z))
        beta = rz[i + 1] / rz[i]
        d = z + beta * d
        i += 1
    return x, rz, i


def ld_newton(forward, adjoint, data: np.ndarray, x0: np.ndarray, *, beta: float, gamma: float,
              i_max: int = 30, i_m: int = 5, tol_in: float = 0.0, tol_out: float = 1e-3,
              outer_max: int = 30):
    """Algorithm 5 (inexact Newton with lagged diffusivity) for one data set
    of the linear acoustic problem: eps(x) = 0.5 ||forward(x) - data||^2,
    grad = adjoint(forward(x) - data) (eq gr), H = adjoint(forward(.)) (eq apj),
    each outer step solving eq pre with Algorithm 4 and M_gamma built at the
    current iterate.  Returns (x, list of eps^k, list of PCG iteration counts)."""
    shape = np.shape(x0)
    ny, nx = shape
    D = tv_difference(ny, nx)
    x = np.asarray(x0, float).ravel().copy()

    def eps_grad(v):
        res = forward(v.reshape(shape)) - data
        return 0.5 * float(np.sum(res * res)), np.asarray(adjoint(res), float).ravel()

    def apply_h(v):
        return np.asarray(adjoint(forward(v.reshape(shape))), float).ravel()

    eps, grad = eps_grad(x)
    hist, iters = [eps], []
    k = 0
    while k < outer_max and (k == 0 or 1.0 - hist[k] / hist[k - 1] > tol_out):
        lu = spla.splu(tv_matrix(D, x, beta, gamma).tocsc())
        d, _, it = pcg(apply_h, grad, lu.solve, i_max, i_m, tol_in)
        x = x + d
        iters.append(it)
        eps, grad = eps_grad(x)
        hist.append(eps)
        k += 1
    return x.reshape(shape), hist, iters
