"""Torch binding of the optical operators (qpat_optical_* in include/qpat.h)
and the composite QPAT Jacobian J = H_a o P o J_o of Definition 3 (eqs
com_des, J_des), P the map from elemental heating to the initial pressure on
the acoustic grid.  Argument marshalling and sequencing only: every step runs
in the library."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from ._lib import check, lib, on_stream
from .ops import Plan, _ptr, _stream


class Optical:
    """Diffusion-approximation operators for `batch` illuminations on the mesh
    matched to an nx x ny acoustic grid of spacing dx (2 nx ny elements)."""

    def __init__(self, nx: int, ny: int, dx: float, batch: int, tol: float = 1e-10, max_iter: int = 200000):
        h = ctypes.c_void_p()
        check(lib().qpat_optical_create(nx, ny, float(dx), batch, ctypes.byref(h)), "qpat_optical_create")
        self._h, self.nx, self.ny, self.batch = h, nx, ny, batch
        self.ne = 2 * nx * ny
        self.tol, self.max_iter = tol, max_iter
        self.iters = 0

    def close(self) -> None:
        if self._h:
            lib().qpat_optical_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _el(self, t: torch.Tensor, name: str) -> tuple[torch.Tensor, int]:
        t = t.contiguous()
        if t.dtype != torch.float32 or t.shape[-1] != self.ne:
            raise ValueError(f"{name} must be float32 [..., {self.ne}]")
        return t, (1 if t.dim() == 1 else t.shape[0])

    @on_stream
    def forward(self, kappa: torch.Tensor, mu: torch.Tensor, currents, stream=None) -> torch.Tensor:
        """H = mu o I Phi with A_o Phi = G; currents [batch][4] (bottom, top, left, right)."""
        kappa, b = self._el(kappa, "kappa")
        mu, _ = self._el(mu, "mu")
        cur = np.ascontiguousarray(np.asarray(currents, dtype=np.float64).reshape(b, 4))
        H = torch.empty_like(kappa)
        it = ctypes.c_int32()
        check(lib().qpat_optical_forward(self._h, _ptr(kappa), _ptr(mu),
                                         cur.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _ptr(H), b, self.tol,
                                         self.max_iter, ctypes.byref(it), _stream(stream)), "qpat_optical_forward")
        self.iters = int(it.value)
        return H

    @on_stream
    def jv(self, dkappa: torch.Tensor, dmu: torch.Tensor, stream=None) -> torch.Tensor:
        dkappa, b = self._el(dkappa, "dkappa")
        dmu, _ = self._el(dmu, "dmu")
        out = torch.empty_like(dkappa)
        it = ctypes.c_int32()
        check(lib().qpat_optical_jv(self._h, _ptr(dkappa), _ptr(dmu), _ptr(out), b, self.tol, self.max_iter,
                                    ctypes.byref(it), _stream(stream)), "qpat_optical_jv")
        self.iters = int(it.value)
        return out

    @on_stream
    def jtv(self, H: torch.Tensor, stream=None) -> tuple[torch.Tensor, torch.Tensor]:
        H, b = self._el(H, "H")
        gk, gm = torch.empty_like(H), torch.empty_like(H)
        it = ctypes.c_int32()
        check(lib().qpat_optical_jtv(self._h, _ptr(H), _ptr(gk), _ptr(gm), b, self.tol, self.max_iter,
                                     ctypes.byref(it), _stream(stream)), "qpat_optical_jtv")
        self.iters = int(it.value)
        return gk, gm

    @on_stream
    def pixels(self, H: torch.Tensor, stream=None) -> torch.Tensor:
        """Initial pressure [.., ny, nx]: the mean of each pixel's two elements."""
        H, b = self._el(H, "H")
        p = torch.empty(*H.shape[:-1], self.ny, self.nx, device=H.device, dtype=torch.float32)
        check(lib().qpat_optical_pixels(self._h, _ptr(H), _ptr(p), 0, b, _stream(stream)), "qpat_optical_pixels")
        return p

    @on_stream
    def pixels_T(self, p: torch.Tensor, stream=None) -> torch.Tensor:
        p = p.contiguous()
        if p.dtype != torch.float32 or p.shape[-2:] != (self.ny, self.nx):
            raise ValueError("p must be float32 [..., ny, nx]")
        b = 1 if p.dim() == 2 else p.shape[0]
        H = torch.empty(*p.shape[:-2], self.ne, device=p.device, dtype=torch.float32)
        check(lib().qpat_optical_pixels(self._h, _ptr(p), _ptr(H), 1, b, _stream(stream)), "qpat_optical_pixels")
        return H


class QPATJacobian:
    """The composite operator of Definition 3 for N_q illuminations side by
    side: H(X) = H_a P H_o(X), J dX = H_a P J_o dX, J^* r = J_o^* P^T H_a^* r,
    with X = (kappa, mu) elemental, one acoustic vector per illumination."""

    def __init__(self, plan: Plan, optical: Optical):
        if (plan.nx, plan.ny) != (optical.nx, optical.ny):
            raise ValueError("the acoustic grid and the optical mesh must match")
        self.plan, self.optical = plan, optical

    @on_stream
    def forward(self, kappa, mu, currents, stream=None) -> torch.Tensor:
        H = self.optical.forward(kappa, mu, currents, stream)
        return self.plan.forward(self.optical.pixels(H, stream), stream=stream)

    @on_stream
    def jv(self, dkappa, dmu, stream=None) -> torch.Tensor:
        dH = self.optical.jv(dkappa, dmu, stream)
        return self.plan.jv(self.optical.pixels(dH, stream), stream=stream)

    @on_stream
    def jtv(self, r, stream=None) -> tuple[torch.Tensor, torch.Tensor]:
        g = self.plan.adjoint(r, stream=stream)
        return self.optical.jtv(self.optical.pixels_T(g, stream), stream)


__all__ = ["Optical", "QPATJacobian"]
