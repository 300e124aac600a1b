"""Python front end of libqpat: plans, batches and operators on torch tensors.

Torch supplies device memory and the current stream; every step of the solve
runs in the HIP kernels of libqpat.so.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np
import torch

from ._lib import QpatParams, check, lib, on_stream

OPS = {"dx+": 0, "dx-": 1, "dy+": 2, "dy-": 3, "ydis": 4, "yabs": 5}

# pass ids of qpat_time_pass: (name, kernel kind)
PASSES = [("fwd_col_grad_p", "col"), ("fwd_row_velocity", "row"), ("fwd_col_div_v", "col"),
          ("fwd_row_density", "row"), ("fwd_col_fraclap", "col"), ("fwd_row_pressure", "row"),
          ("adj_row_pressure", "row"), ("adj_col_fraclap", "col"), ("adj_row_density", "row"),
          ("adj_col_grad", "col"), ("adj_row_velocity", "row"), ("adj_col_div", "col")]


def _stream(stream=None) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def _ptr(t: torch.Tensor) -> int:
    return t.data_ptr()


def _need(t: torch.Tensor, shape, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    if tuple(t.shape[-len(shape):]) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected [..., {', '.join(map(str, shape))}]")
    return t.contiguous()


def make_params(prm: dict) -> tuple[QpatParams, np.ndarray]:
    xy = np.ascontiguousarray(prm["sensor_xy"], dtype=np.float64).reshape(-1, 2)
    p = QpatParams(nx=prm["nx"], ny=prm["ny"], dx=prm["dx"], dy=prm["dy"], dt=prm["dt"], nt=prm["nt"],
                   c_ref=prm["c_ref"], pml_size=prm["pml_size"], pml_alpha=prm["pml_alpha"],
                   alpha0_db=prm["alpha0_db"], y=prm["y"], ns=len(xy),
                   sensor_xy=xy.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return p, xy


def validate(prm: dict) -> int:
    """Host-only parameter check; returns the qpat status code (0 = ok)."""
    p, _keep = make_params(prm)
    return int(lib().qpat_validate(ctypes.byref(p)))


class Plan:
    """A k-space acoustic problem on the current HIP device (see qpat_plan_create)."""

    def __init__(self, prm: dict, c0, rho0):
        L = lib()
        p, self._xy = make_params(prm)
        c0 = np.ascontiguousarray(c0, dtype=np.float64)
        rho0 = np.ascontiguousarray(rho0, dtype=np.float64)
        if c0.shape != (prm["ny"], prm["nx"]) or rho0.shape != c0.shape:
            raise ValueError("c0 / rho0 must have shape [ny, nx]")
        h = ctypes.c_void_p()
        check(L.qpat_plan_create(ctypes.byref(p), c0.ctypes.data, rho0.ctypes.data, ctypes.byref(h)),
              "qpat_plan_create")
        self._h = h
        self._c0 = c0.copy()
        self.params = dict(prm)
        self.nx, self.ny, self.nt = prm["nx"], prm["ny"], prm["nt"]
        self.ns = len(self._xy)
        self.device = torch.device("cuda", torch.cuda.current_device())

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().qpat_plan_destroy(h)
            except Exception:
                pass
            self._h = None

    @property
    def handle(self):
        return self._h

    def sound_speed(self) -> np.ndarray:
        """The FP64 sound speed [ny, nx] the plan was built from."""
        return self._c0

    # ---- shapes
    def _fields(self, t, name):
        t = _need(t, (self.ny, self.nx), name)
        return t, (t.numel() // (self.nx * self.ny)), t.shape[:-2]

    def _data(self, t, name):
        t = _need(t, (self.nt, self.ns), name)
        return t, (t.numel() // (self.nt * self.ns)), t.shape[:-2]

    # ---- operators
    @on_stream
    def forward(self, p0: torch.Tensor, stream=None) -> torch.Tensor:
        """H_a p0: [..., ny, nx] -> [..., nt, ns]."""
        p0, b, lead = self._fields(p0, "p0")
        out = torch.empty(*lead, self.nt, self.ns, device=p0.device, dtype=torch.float32)
        check(lib().qpat_forward(self._h, _ptr(p0), _ptr(out), b, _stream(stream)), "qpat_forward")
        return out

    jv = forward

    @on_stream
    def adjoint(self, res: torch.Tensor, stream=None) -> torch.Tensor:
        """H_a^* r: [..., nt, ns] -> [..., ny, nx]."""
        res, b, lead = self._data(res, "res")
        out = torch.empty(*lead, self.ny, self.nx, device=res.device, dtype=torch.float32)
        check(lib().qpat_adjoint(self._h, _ptr(res), _ptr(out), b, _stream(stream)), "qpat_adjoint")
        return out

    @on_stream
    def jtjv(self, v: torch.Tensor, stream=None) -> torch.Tensor:
        """H_a^* H_a v: [..., ny, nx] -> [..., ny, nx]."""
        v, b, lead = self._fields(v, "v")
        out = torch.empty_like(v)
        check(lib().qpat_jtjv(self._h, _ptr(v), _ptr(out), b, _stream(stream)), "qpat_jtjv")
        return out

    @on_stream
    def jtjv_data(self, v: torch.Tensor, stream=None) -> tuple[torch.Tensor, torch.Tensor]:
        """(H_a v, H_a^* H_a v) from one call (qpat_jtjv_data)."""
        v, b, lead = self._fields(v, "v")
        jv = torch.empty(*lead, self.nt, self.ns, device=v.device, dtype=torch.float32)
        out = torch.empty_like(v)
        check(lib().qpat_jtjv_data(self._h, _ptr(v), _ptr(jv), _ptr(out), b, _stream(stream)), "qpat_jtjv_data")
        return jv, out

    @on_stream
    def apply(self, op: str, x: torch.Tensor, stream=None) -> torch.Tensor:
        """One spectral operator ('dx+', 'dx-', 'dy+', 'dy-', 'ydis', 'yabs')."""
        x, b, lead = self._fields(x, "x")
        out = torch.empty_like(x)
        check(lib().qpat_apply(self._h, OPS[op], _ptr(x), _ptr(out), b, _stream(stream)), "qpat_apply")
        return out

    # ---- checkpoints
    def ckpt_bytes(self, interval: int, batch: int = 1) -> int:
        n = ctypes.c_size_t()
        check(lib().qpat_ckpt_bytes(self._h, interval, batch, ctypes.byref(n)), "qpat_ckpt_bytes")
        return int(n.value)

    @on_stream
    def forward_ckpt(self, p0: torch.Tensor, interval: int, stream=None):
        """(data, checkpoints): checkpoints [B, ceil(nt/K), 5, ny, nx]."""
        p0, b, lead = self._fields(p0, "p0")
        nck = math.ceil(self.nt / interval)
        ck = torch.empty(b, nck, 5, self.ny, self.nx, device=p0.device, dtype=torch.float32)
        out = torch.empty(*lead, self.nt, self.ns, device=p0.device, dtype=torch.float32)
        check(lib().qpat_forward_ckpt(self._h, _ptr(p0), _ptr(out), interval, _ptr(ck), b, _stream(stream)),
              "qpat_forward_ckpt")
        return out, ck

    @on_stream
    def replay(self, p0: torch.Tensor, ckpt: torch.Tensor, interval: int, seg: int, stream=None):
        """States z_m [B, cnt, 5, ny, nx] of segment `seg` recomputed from its checkpoint."""
        p0, b, _ = self._fields(p0, "p0")
        ckpt = ckpt.contiguous()
        cnt = min(interval, self.nt - seg * interval)
        out = torch.empty(b, max(cnt, 0), 5, self.ny, self.nx, device=p0.device, dtype=torch.float32)
        check(lib().qpat_replay(self._h, _ptr(p0), _ptr(ckpt), interval, seg, _ptr(out), b, _stream(stream)),
              "qpat_replay")
        return out

    # ---- sound-speed gradient
    def medium_grad_bytes(self, interval: int, batch: int = 1) -> int:
        n = ctypes.c_size_t()
        check(lib().qpat_medium_grad_bytes(self._h, interval, batch, ctypes.byref(n)), "qpat_medium_grad_bytes")
        return int(n.value)

    @on_stream
    def medium_grad(self, p0: torch.Tensor, res: torch.Tensor, interval: int | None = None, work=None,
                    stream=None) -> tuple[torch.Tensor, torch.Tensor]:
        """(d<res, H_a[c0] p0>/dc0, H_a^* res) for p0 [..., ny, nx] and res
        [..., nt, ns] (c_ref fixed), recomputing the forward wavefield from
        checkpoints every `interval` iterates (None: keep every sensitivity).
        `work` may pass a reusable uint8 device buffer of medium_grad_bytes."""
        p0, b, lead = self._fields(p0, "p0")
        res, b2, _ = self._data(res, "res")
        if b2 != b:
            raise ValueError("medium_grad: p0 and res must hold the same number of vectors")
        k = max(self.nt - 1, 1) if interval is None else int(interval)
        need = self.medium_grad_bytes(k, b)
        if work is None:
            work = torch.empty(need, device=p0.device, dtype=torch.uint8)
        elif work.numel() * work.element_size() < need or not work.is_contiguous():
            raise ValueError(f"medium_grad: work buffer needs {need} contiguous bytes")
        gp = torch.empty(*lead, self.ny, self.nx, device=p0.device, dtype=torch.float32)
        gc = torch.empty_like(gp)
        check(lib().qpat_medium_grad(self._h, _ptr(p0), _ptr(res), k, _ptr(work), _ptr(gp), _ptr(gc), b,
                                     _stream(stream)), "qpat_medium_grad")
        return gc, gp

    # ---- launch shape
    def set_tiles(self, rows: int, cols: int, row_threads: int = 256, col_threads: int = 256) -> None:
        check(lib().qpat_set_tiles(self._h, rows, cols, row_threads, col_threads), "qpat_set_tiles")

    def tiles(self) -> tuple[int, int, int, int]:
        """(rows per row block, columns per column block, row threads, column threads)."""
        r, c, rh, ch = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        check(lib().qpat_get_tiles(self._h, ctypes.byref(r), ctypes.byref(c), ctypes.byref(rh),
                                   ctypes.byref(ch)), "qpat_get_tiles")
        return int(r.value), int(c.value), int(rh.value), int(ch.value)

    @on_stream
    def tune(self, batch: int = 1, stream=None) -> tuple[int, int, int, int]:
        check(lib().qpat_tune(self._h, batch, _stream(stream)), "qpat_tune")
        return self.tiles()

    def set_graph(self, enable: bool = True) -> None:
        check(lib().qpat_set_graph(self._h, int(bool(enable))), "qpat_set_graph")

    @on_stream
    def time_pass(self, pass_id: int, batch: int = 1, reps: int = 20, stream=None) -> float:
        """Mean duration in ms of one launch of a pass kind (qpat_time_pass)."""
        ms = ctypes.c_float()
        check(lib().qpat_time_pass(self._h, pass_id, batch, reps, _stream(stream), ctypes.byref(ms)),
              "qpat_time_pass")
        return float(ms.value)

    def set_check(self, enable: bool = True) -> None:
        """Scan every solve's output for NaN / Inf (qpat_set_check)."""
        check(lib().qpat_set_check(self._h, int(bool(enable))), "qpat_set_check")

    @on_stream
    def outputs_finite(self, stream=None) -> bool:
        """Synchronise the stream; False if a checked output since the last
        call held NaN or Inf (qpat_check returned QPAT_E_NONFINITE)."""
        st = lib().qpat_check(self._h, _stream(stream))
        if st == 6:
            return False
        check(st, "qpat_check")
        return True

    def device_bytes(self) -> int:
        n = ctypes.c_size_t()
        check(lib().qpat_plan_info(self._h, None, None, None, None, ctypes.byref(n)), "qpat_plan_info")
        return int(n.value)


class Batch:
    """Plans of different sizes advanced together (qpat_batch_*)."""

    def __init__(self, plans: list[Plan]):
        self.plans = list(plans)
        arr = (ctypes.c_void_p * len(plans))(*[p.handle.value for p in plans])
        h = ctypes.c_void_p()
        check(lib().qpat_batch_create(arr, len(plans), ctypes.byref(h)), "qpat_batch_create")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().qpat_batch_destroy(h)
            except Exception:
                pass
            self._h = None

    @staticmethod
    def _arr(ts):
        return (ctypes.c_void_p * len(ts))(*[t.data_ptr() for t in ts])

    @on_stream
    def forward(self, p0s, stream=None):
        ins = [_need(x, (p.ny, p.nx), "p0") for x, p in zip(p0s, self.plans)]
        outs = [torch.empty(p.nt, p.ns, device=x.device, dtype=torch.float32) for x, p in zip(ins, self.plans)]
        check(lib().qpat_batch_forward(self._h, self._arr(ins), self._arr(outs), _stream(stream)),
              "qpat_batch_forward")
        return outs

    @on_stream
    def adjoint(self, ress, stream=None):
        ins = [_need(x, (p.nt, p.ns), "res") for x, p in zip(ress, self.plans)]
        outs = [torch.empty(p.ny, p.nx, device=x.device, dtype=torch.float32) for x, p in zip(ins, self.plans)]
        check(lib().qpat_batch_adjoint(self._h, self._arr(ins), self._arr(outs), _stream(stream)),
              "qpat_batch_adjoint")
        return outs

    @on_stream
    def jtjv(self, vs, stream=None, out=None):
        ins = [_need(x, (p.ny, p.nx), "v") for x, p in zip(vs, self.plans)]
        outs = out if out is not None else [torch.empty_like(x) for x in ins]
        check(lib().qpat_batch_jtjv(self._h, self._arr(ins), self._arr(outs), _stream(stream)),
              "qpat_batch_jtjv")
        return outs

    def set_graph(self, enable: bool = True) -> None:
        check(lib().qpat_batch_set_graph(self._h, int(bool(enable))), "qpat_batch_set_graph")

    def set_schedule(self, schedule: int) -> None:
        """0: one launch per pass for every problem; 1: one launch sequence per
        grid size, side by side on forked streams (qpat_batch_set_schedule)."""
        check(lib().qpat_batch_set_schedule(self._h, int(schedule)), "qpat_batch_set_schedule")

    def schedule(self) -> int:
        v = ctypes.c_int32()
        check(lib().qpat_batch_get_schedule(self._h, ctypes.byref(v)), "qpat_batch_get_schedule")
        return int(v.value)

    @on_stream
    def tune(self, stream=None) -> int:
        """Launch shapes per grid size and the schedule (qpat_batch_tune); returns the schedule."""
        check(lib().qpat_batch_tune(self._h, _stream(stream)), "qpat_batch_tune")
        return self.schedule()


@on_stream
def probe_barrier(design: int, nblocks: int, threads: int = 256, iters: int = 400, words: int = 0,
                  stream=None) -> tuple[float, bool]:
    """Mean microseconds of one exchange step under a grid barrier (design 0:
    one counter, 1: hierarchical, cooperative launches) or kernel boundaries
    in a graph (design 2), and whether a bounded wait gave up
    (qpat_probe_barrier)."""
    us = ctypes.c_float()
    to = ctypes.c_int32()
    check(lib().qpat_probe_barrier(design, nblocks, threads, iters, words, _stream(stream), ctypes.byref(us),
                                   ctypes.byref(to)), "qpat_probe_barrier")
    return float(us.value), bool(to.value)


@on_stream
def dot(a: torch.Tensor, b: torch.Tensor, stream=None) -> torch.Tensor:
    """<a, b> with FP64 accumulation (qpat_dot); returns a 0-d float64 CUDA tensor."""
    a = a.contiguous()
    b = b.contiguous()
    if a.numel() != b.numel():
        raise ValueError("dot: size mismatch")
    out = torch.empty((), device=a.device, dtype=torch.float64)
    check(lib().qpat_dot(_ptr(a), _ptr(b), a.numel(), _ptr(out), _stream(stream)), "qpat_dot")
    return out
