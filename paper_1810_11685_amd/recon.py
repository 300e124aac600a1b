"""Inexact-Newton reconstruction of p0 with lagged-diffusivity TV
priorconditioning (Section 5.2 of the paper: PCG of Algorithm 4 inside the
outer loop of Algorithm 5), on the library's batched J^T J v.

The unknown is p0 itself (acoustic-only problem, identity scaling), so the
Gauss-Newton Hessian of eq apj is H = H_a^* H_a and the gradient of eq gr is
H_a^*(H_a p0 - data).  Several data sets (one per illumination) are solved
side by side: every H d of the PCG loop is one batched qpat_jtjv call, every
M_gamma z = r one batched qpat_tv_solve, and the scalars of each data set are
its own.  All field arithmetic runs in the library (qpat_jtjv, qpat_forward,
qpat_adjoint, qpat_tv_*, qpat_axpby, qpat_dot); this module only sequences
the steps and keeps the scalars.
"""
from __future__ import annotations

import ctypes
import math

import torch

from ._lib import check, lib, on_stream
from .ops import Plan, _ptr, _stream, dot


class TV:
    """Edge weights of C[x] (eq m1) and the solver of M_gamma z = r for up to
    `batch` fields of an ny x nx grid (qpat_tv_*)."""

    def __init__(self, nx: int, ny: int, batch: int):
        h = ctypes.c_void_p()
        check(lib().qpat_tv_create(nx, ny, batch, ctypes.byref(h)), "qpat_tv_create")
        self._h, self.nx, self.ny, self.batch = h, nx, ny, batch

    def close(self) -> None:
        if self._h:
            lib().qpat_tv_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _fields(self, x: torch.Tensor) -> tuple[torch.Tensor, int]:
        x = x.contiguous()
        if x.dtype != torch.float32 or x.shape[-2:] != (self.ny, self.nx):
            raise ValueError("TV: fields must be float32 [..., ny, nx]")
        b = 1 if x.dim() == 2 else x.shape[0]
        return x, b

    @on_stream
    def set_weights(self, x: torch.Tensor, beta: float, stream=None) -> None:
        x, b = self._fields(x)
        check(lib().qpat_tv_set_weights(self._h, _ptr(x), float(beta), b, _stream(stream)), "qpat_tv_set_weights")

    @on_stream
    def apply(self, x: torch.Tensor, gamma: float, stream=None) -> torch.Tensor:
        x, b = self._fields(x)
        y = torch.empty_like(x)
        check(lib().qpat_tv_apply(self._h, float(gamma), _ptr(x), _ptr(y), b, _stream(stream)), "qpat_tv_apply")
        return y

    @on_stream
    def solve(self, r: torch.Tensor, gamma: float, tol: float = 1e-6, max_iter: int = 20000,
              stream=None) -> tuple[torch.Tensor, int]:
        r, b = self._fields(r)
        z = torch.empty_like(r)
        it = ctypes.c_int32()
        check(lib().qpat_tv_solve(self._h, float(gamma), _ptr(r), _ptr(z), b, float(tol), int(max_iter),
                                  ctypes.byref(it), _stream(stream)), "qpat_tv_solve")
        return z, int(it.value)

    @on_stream
    def value(self, x: torch.Tensor, beta: float, stream=None) -> list[float]:
        x, b = self._fields(x)
        out = (ctypes.c_double * b)()
        check(lib().qpat_tv_value(self._h, _ptr(x), float(beta), b, out, _stream(stream)), "qpat_tv_value")
        return list(out)


@on_stream
def axpby(a: float, x: torch.Tensor, b: float, y: torch.Tensor, stream=None) -> torch.Tensor:
    """y <- a x + b y in place (qpat_axpby); x and y contiguous float32 of one size."""
    if not (x.is_contiguous() and y.is_contiguous()) or x.numel() != y.numel():
        raise ValueError("axpby: contiguous tensors of one size required")
    check(lib().qpat_axpby(y.numel(), float(a), _ptr(x), float(b), _ptr(y), _stream(stream)), "qpat_axpby")
    return y


@on_stream
def _dot(a: torch.Tensor, b: torch.Tensor, stream=None) -> float:
    return float(dot(a, b, stream).item())


@on_stream
def ld_reconstruct(plan: Plan, data: torch.Tensor, x0: torch.Tensor, *, beta: float, gamma: float,
                   i_max: int = 30, i_m: int = 5, tol_in: float = 0.0, tol_out: float = 1e-3,
                   outer_max: int = 30, solve_tol: float = 1e-6, solve_max_iter: int = 20000, stream=None):
    """Algorithm 5 with Algorithm 4 for B data sets [B][nt][ns] from initial
    images x0 [B][ny][nx].  Per data set the outer loop runs while k = 0 or
    1 - eps^k / eps^{k-1} > tol_out (at most outer_max steps, step length 1);
    each step builds M_gamma at the current image and runs PCG while
    i < i_max and (i < i_m or 1 - r_i.z_i / r_{i-i_m}.z_{i-i_m} > tol_in).
    Returns (images [B][ny][nx], eps history per data set, PCG iterations per
    outer step per data set, M_gamma solver iterations in total)."""
    if data.dim() != 3 or x0.dim() != 3 or data.shape[0] != x0.shape[0]:
        raise ValueError("ld_reconstruct: data [B][nt][ns] and x0 [B][ny][nx] required")
    B = data.shape[0]
    data = data.contiguous()
    x = x0.contiguous().clone()
    tv = TV(x.shape[2], x.shape[1], B)
    solves = 0

    def eps_grad(img):
        res = plan.forward(img, stream=stream)
        axpby(-1.0, data, 1.0, res, stream)                       # H_a x - data
        eps = [0.5 * _dot(res[b], res[b], stream) for b in range(B)]
        return eps, plan.adjoint(res, stream=stream)               # eq gr

    eps, grad = eps_grad(x)
    hist = [[e] for e in eps]
    iters = [[] for _ in range(B)]
    active = [True] * B
    k = 0
    try:
        while k < outer_max:
            if k > 0:
                active = [active[b] and (1.0 - hist[b][k] / hist[b][k - 1] > tol_out) for b in range(B)]
            if not any(active):
                break
            # ---- Algorithm 4 on H d = -grad with preconditioner M_gamma[x^k]
            tv.set_weights(x, beta, stream)
            r = grad.clone()
            axpby(0.0, grad, -1.0, r, stream)                       # r0 = -grad
            z, n_it = tv.solve(r, gamma, solve_tol, solve_max_iter, stream)
            solves += n_it
            d = z.clone()
            sol = torch.zeros_like(x)
            rz = [[_dot(r[b], z[b], stream)] for b in range(B)]
            i = 0
            done = [not a for a in active]
            while True:
                live = [not done[b] and i < i_max and
                        (i < i_m or 1.0 - rz[b][i] / rz[b][i - i_m] > tol_in) for b in range(B)]
                if not any(live):
                    break
                hd = plan.jtjv(d, stream=stream)                   # H d, one batched call
                for b in range(B):
                    if not live[b]:
                        continue
                    alpha = rz[b][i] / _dot(d[b], hd[b], stream)
                    axpby(alpha, d[b], 1.0, sol[b], stream)
                    axpby(-alpha, hd[b], 1.0, r[b], stream)
                z, n_it = tv.solve(r, gamma, solve_tol, solve_max_iter, stream)
                solves += n_it
                for b in range(B):
                    if not live[b]:
                        done[b] = True
                        continue
                    rz[b].append(_dot(r[b], z[b], stream))
                    axpby(1.0, z[b], rz[b][i + 1] / rz[b][i], d[b], stream)   # d = z + beta d
                i += 1
            for b in range(B):
                if active[b]:
                    axpby(1.0, sol[b], 1.0, x[b], stream)           # X^{k+1} = X^k + d^k
                    iters[b].append(len(rz[b]) - 1)
            eps, grad = eps_grad(x)
            for b in range(B):
                hist[b].append(eps[b] if active[b] else hist[b][-1])
            k += 1
    finally:
        tv.close()
    return x, hist, iters, solves


__all__ = ["TV", "axpby", "ld_reconstruct"]
