"""Inexact-Newton reconstruction of p0 with lagged-diffusivity TV
priorconditioning (Section 5.2 of the paper: PCG of Algorithm 4 inside the
outer loop of Algorithm 5), on the library's batched J^T J v.

The unknown is p0 itself (acoustic-only problem, identity scaling), so the
Gauss-Newton Hessian of eq apj is H = H_a^* H_a and the gradient of eq gr is
H_a^*(H_a p0 - data).  Several data sets (one per illumination) are solved
side by side: every H d of the PCG loop is one batched qpat_jtjv call, every
M_gamma z = r one batched qpat_tv_solve, and the scalars of each data set are
its own.  The loop itself runs in the library (qpat_ld_run), with the PCG
scalars on the device; this module marshals arguments.
"""
from __future__ import annotations

import ctypes
import math

import torch

from ._lib import QpatLdParams, check, lib, on_stream
from .ops import Plan, _ptr, _stream


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
def ld_reconstruct(plan: Plan, data: torch.Tensor, x0: torch.Tensor, *, beta: float, gamma: float,
                   i_max: int = 30, i_m: int = 5, tol_in: float = 0.0, tol_out: float = 1e-3,
                   outer_max: int = 30, solve_tol: float = 1e-6, solve_max_iter: int = 20000, stream=None):
    """Algorithm 5 with Algorithm 4 for B data sets [B][nt][ns] from initial
    images x0 [B][ny][nx] (qpat_ld_run: the whole loop runs in the library).
    Per data set the outer loop runs while k = 0 or 1 - eps^k / eps^{k-1} >
    tol_out (at most outer_max steps, step length 1); each step builds
    M_gamma at the current image and runs PCG while i < i_max and (i < i_m or
    1 - r_i.z_i / r_{i-i_m}.z_{i-i_m} > tol_in).  Returns (images [B][ny][nx],
    eps history per data set, PCG iterations per outer step per data set,
    M_gamma solver iterations in total)."""
    if data.dim() != 3 or x0.dim() != 3 or data.shape[0] != x0.shape[0]:
        raise ValueError("ld_reconstruct: data [B][nt][ns] and x0 [B][ny][nx] required")
    B = data.shape[0]
    if tuple(data.shape[1:]) != (plan.nt, plan.ns) or tuple(x0.shape[1:]) != (plan.ny, plan.nx):
        raise ValueError("ld_reconstruct: shapes do not match the plan")
    data = data.contiguous()
    x = x0.contiguous().clone()
    h = ctypes.c_void_p()
    check(lib().qpat_ld_create(plan.handle, B, ctypes.byref(h)), "qpat_ld_create")
    try:
        prm = QpatLdParams(beta=float(beta), gamma=float(gamma), i_max=int(i_max), i_m=int(i_m),
                           tol_in=float(tol_in), outer_max=int(outer_max), tol_out=float(tol_out),
                           solve_tol=float(solve_tol), solve_max_iter=int(solve_max_iter))
        K = int(outer_max)
        eps = (ctypes.c_double * (B * (K + 1)))()
        its = (ctypes.c_int32 * max(1, B * K))()
        steps, solves = ctypes.c_int32(), ctypes.c_int32()
        check(lib().qpat_ld_run(h, _ptr(data), _ptr(x), ctypes.byref(prm), eps, its, ctypes.byref(steps),
                                ctypes.byref(solves), _stream(stream)), "qpat_ld_run")
    finally:
        lib().qpat_ld_destroy(h)
    k = steps.value
    hist = [[eps[b * (K + 1) + j] for j in range(k + 1)] for b in range(B)]
    iters = [[its[b * K + j] for j in range(k) if its[b * K + j] >= 0] for b in range(B)]
    return x, hist, iters, solves.value
