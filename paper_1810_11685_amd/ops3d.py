"""Torch binding of the 3-D solver (qpat3d_* in include/qpat.h): argument
marshalling only, every step runs in the library's kernels."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from ._lib import QpatParams3d, check, lib, on_stream
from .ops import _need, _ptr, _stream

OPS3 = {"dx+": 0, "dx-": 1, "dy+": 2, "dy-": 3, "dz+": 4, "dz-": 5, "ydis": 6, "yabs": 7}


def make_params3d(prm: dict) -> tuple[QpatParams3d, np.ndarray]:
    xyz = np.ascontiguousarray(prm["sensor_xyz"], dtype=np.float64).reshape(-1, 3)
    p = QpatParams3d(nx=prm["nx"], ny=prm["ny"], nz=prm["nz"], dx=prm["dx"], dy=prm["dy"], dz=prm["dz"],
                     dt=prm["dt"], nt=prm["nt"], c_ref=prm["c_ref"], pml_size=prm["pml_size"],
                     pml_alpha=prm["pml_alpha"], alpha0_db=prm["alpha0_db"], y=prm["y"], ns=len(xyz),
                     sensor_xyz=xyz.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return p, xyz


def validate3d(prm: dict) -> int:
    """Host-only parameter check; returns the qpat status code (0 = ok)."""
    p, _keep = make_params3d(prm)
    return int(lib().qpat3d_validate(ctypes.byref(p)))


class Plan3D:
    """A 3-D k-space acoustic problem on the current HIP device (qpat3d_plan_create)."""

    def __init__(self, prm: dict, c0, rho0):
        L = lib()
        p, self._xyz = make_params3d(prm)
        c0 = np.ascontiguousarray(c0, dtype=np.float64)
        rho0 = np.ascontiguousarray(rho0, dtype=np.float64)
        shape = (prm["nz"], prm["ny"], prm["nx"])
        if c0.shape != shape or rho0.shape != shape:
            raise ValueError("c0 / rho0 must have shape [nz, ny, nx]")
        h = ctypes.c_void_p()
        check(L.qpat3d_plan_create(ctypes.byref(p), c0.ctypes.data, rho0.ctypes.data, ctypes.byref(h)),
              "qpat3d_plan_create")
        self._h = h
        self.params = dict(prm)
        self.nx, self.ny, self.nz, self.nt = prm["nx"], prm["ny"], prm["nz"], prm["nt"]
        self.ns = len(self._xyz)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().qpat3d_plan_destroy(h)
            except Exception:
                pass
            self._h = None

    def _fields(self, t, name):
        t = _need(t, (self.nz, self.ny, self.nx), name)
        return t, t.numel() // (self.nx * self.ny * self.nz), t.shape[:-3]

    def _data(self, t, name):
        t = _need(t, (self.nt, self.ns), name)
        return t, t.numel() // (self.nt * self.ns), t.shape[:-2]

    @on_stream
    def forward(self, p0: torch.Tensor, stream=None) -> torch.Tensor:
        """H_a p0: [..., nz, ny, nx] -> [..., nt, ns]."""
        p0, b, lead = self._fields(p0, "p0")
        out = torch.empty(*lead, self.nt, self.ns, device=p0.device, dtype=torch.float32)
        check(lib().qpat3d_forward(self._h, _ptr(p0), _ptr(out), b, _stream(stream)), "qpat3d_forward")
        return out

    jv = forward

    @on_stream
    def adjoint(self, res: torch.Tensor, stream=None) -> torch.Tensor:
        """H_a^* r: [..., nt, ns] -> [..., nz, ny, nx]."""
        res, b, lead = self._data(res, "res")
        out = torch.empty(*lead, self.nz, self.ny, self.nx, device=res.device, dtype=torch.float32)
        check(lib().qpat3d_adjoint(self._h, _ptr(res), _ptr(out), b, _stream(stream)), "qpat3d_adjoint")
        return out

    @on_stream
    def jtjv(self, v: torch.Tensor, stream=None) -> torch.Tensor:
        v, b, _ = self._fields(v, "v")
        out = torch.empty_like(v)
        check(lib().qpat3d_jtjv(self._h, _ptr(v), _ptr(out), b, _stream(stream)), "qpat3d_jtjv")
        return out

    @on_stream
    def apply(self, op: str, x: torch.Tensor, stream=None) -> torch.Tensor:
        """One spectral operator ('dx+', 'dx-', 'dy+', 'dy-', 'dz+', 'dz-', 'ydis', 'yabs')."""
        x, b, _ = self._fields(x, "x")
        out = torch.empty_like(x)
        check(lib().qpat3d_apply(self._h, OPS3[op], _ptr(x), _ptr(out), b, _stream(stream)), "qpat3d_apply")
        return out

    def set_tiles(self, rows: int, cols: int, row_threads: int | None = None,
                  plane_threads: int | None = None) -> None:
        _, _, rth, pth = self.tiles()
        rth = rth if row_threads is None else row_threads
        pth = pth if plane_threads is None else plane_threads
        check(lib().qpat3d_set_tiles(self._h, rows, cols, rth, pth), "qpat3d_set_tiles")

    def tiles(self) -> tuple[int, int, int, int]:
        """(lines per row block, columns per plane block, row threads, plane threads)."""
        v = [ctypes.c_int32() for _ in range(4)]
        check(lib().qpat3d_get_tiles(self._h, *[ctypes.byref(x) for x in v]), "qpat3d_get_tiles")
        return tuple(int(x.value) for x in v)

    def set_graph(self, enable: bool = True) -> None:
        check(lib().qpat3d_set_graph(self._h, int(bool(enable))), "qpat3d_set_graph")


__all__ = ["Plan3D", "validate3d", "make_params3d", "OPS3"]
