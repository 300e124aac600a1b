"""ctypes declarations of the C ABI in include/qpat.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import functools
import inspect
import os
import threading

import torch  # noqa: F401  (loads torch's HIP runtime first so libqpat binds to the same one)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqpat.so")

c_int32 = ctypes.c_int32
c_double = ctypes.c_double
c_void_p = ctypes.c_void_p
c_size_t = ctypes.c_size_t
c_int64 = ctypes.c_int64


class QpatParams(ctypes.Structure):
    _fields_ = [
        ("nx", c_int32), ("ny", c_int32),
        ("dx", c_double), ("dy", c_double), ("dt", c_double),
        ("nt", c_int32),
        ("c_ref", c_double),
        ("pml_size", c_int32),
        ("pml_alpha", c_double),
        ("alpha0_db", c_double),
        ("y", c_double),
        ("ns", c_int32),
        ("sensor_xy", ctypes.POINTER(c_double)),
    ]


class QpatParams3d(ctypes.Structure):
    _fields_ = [
        ("nx", c_int32), ("ny", c_int32), ("nz", c_int32),
        ("dx", c_double), ("dy", c_double), ("dz", c_double), ("dt", c_double),
        ("nt", c_int32),
        ("c_ref", c_double),
        ("pml_size", c_int32),
        ("pml_alpha", c_double),
        ("alpha0_db", c_double),
        ("y", c_double),
        ("ns", c_int32),
        ("sensor_xyz", ctypes.POINTER(c_double)),
    ]


class QpatLdParams(ctypes.Structure):
    _fields_ = [
        ("beta", c_double), ("gamma", c_double),
        ("i_max", c_int32), ("i_m", c_int32),
        ("tol_in", c_double),
        ("outer_max", c_int32),
        ("tol_out", c_double),
        ("solve_tol", c_double),
        ("solve_max_iter", c_int32),
    ]


STATUS = {0: "QPAT_OK", 1: "QPAT_E_INVALID", 2: "QPAT_E_UNSUPPORTED", 3: "QPAT_E_UNSTABLE",
          4: "QPAT_E_HIP", 5: "QPAT_E_OOM", 6: "QPAT_E_NONFINITE"}

# name -> (restype, argtypes)
_SIGS = {
    "qpat_validate": (c_int32, [ctypes.POINTER(QpatParams)]),
    "qpat_plan_create": (c_int32, [ctypes.POINTER(QpatParams), c_void_p, c_void_p, ctypes.POINTER(c_void_p)]),
    "qpat_plan_destroy": (None, [c_void_p]),
    "qpat_forward": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_void_p]),
    "qpat_adjoint": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_void_p]),
    "qpat_jv": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_void_p]),
    "qpat_jtjv": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_void_p]),
    "qpat_jtjv_data": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_void_p]),
    "qpat_apply": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_int32, c_void_p]),
    "qpat_ckpt_bytes": (c_int32, [c_void_p, c_int32, c_int32, ctypes.POINTER(c_size_t)]),
    "qpat_forward_ckpt": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_void_p, c_int32, c_void_p]),
    "qpat_replay": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_int32, c_void_p, c_int32, c_void_p]),
    "qpat_medium_grad_bytes": (c_int32, [c_void_p, c_int32, c_int32, ctypes.POINTER(c_size_t)]),
    "qpat_medium_grad": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_int32,
                                   c_void_p]),
    "qpat_set_tiles": (c_int32, [c_void_p, c_int32, c_int32, c_int32, c_int32]),
    "qpat_get_tiles": (c_int32, [c_void_p, ctypes.POINTER(c_int32), ctypes.POINTER(c_int32),
                                 ctypes.POINTER(c_int32), ctypes.POINTER(c_int32)]),
    "qpat_tune": (c_int32, [c_void_p, c_int32, c_void_p]),
    "qpat_set_graph": (c_int32, [c_void_p, c_int32]),
    "qpat_probe_barrier": (c_int32, [c_int32, c_int32, c_int32, c_int32, c_int32, c_void_p,
                                     ctypes.POINTER(ctypes.c_float), ctypes.POINTER(c_int32)]),
    "qpat_time_pass": (c_int32, [c_void_p, c_int32, c_int32, c_int32, c_void_p, ctypes.POINTER(ctypes.c_float)]),
    "qpat_batch_create": (c_int32, [ctypes.POINTER(c_void_p), c_int32, ctypes.POINTER(c_void_p)]),
    "qpat_batch_destroy": (None, [c_void_p]),
    "qpat_batch_forward": (c_int32, [c_void_p, ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p), c_void_p]),
    "qpat_batch_adjoint": (c_int32, [c_void_p, ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p), c_void_p]),
    "qpat_batch_jtjv": (c_int32, [c_void_p, ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p), c_void_p]),
    "qpat_batch_set_graph": (c_int32, [c_void_p, c_int32]),
    "qpat_batch_set_schedule": (c_int32, [c_void_p, c_int32]),
    "qpat_batch_get_schedule": (c_int32, [c_void_p, ctypes.POINTER(c_int32)]),
    "qpat_batch_tune": (c_int32, [c_void_p, c_void_p]),
    "qpat_dot": (c_int32, [c_void_p, c_void_p, c_int64, c_void_p, c_void_p]),
    "qpat_dot_noalloc": (c_int32, [c_void_p, c_void_p, c_int64, c_void_p, c_void_p]),
    "qpat_tv_create": (c_int32, [c_int32, c_int32, c_int32, ctypes.POINTER(c_void_p)]),
    "qpat_tv_destroy": (None, [c_void_p]),
    "qpat_tv_set_weights": (c_int32, [c_void_p, c_void_p, ctypes.c_double, c_int32, c_void_p]),
    "qpat_tv_apply": (c_int32, [c_void_p, ctypes.c_double, c_void_p, c_void_p, c_int32, c_void_p]),
    "qpat_tv_solve": (c_int32, [c_void_p, ctypes.c_double, c_void_p, c_void_p, c_int32, ctypes.c_double, c_int32,
                                ctypes.POINTER(c_int32), c_void_p]),
    "qpat_tv_value": (c_int32, [c_void_p, c_void_p, ctypes.c_double, c_int32, ctypes.POINTER(ctypes.c_double),
                                c_void_p]),
    "qpat_axpby": (c_int32, [c_int64, ctypes.c_float, c_void_p, ctypes.c_float, c_void_p, c_void_p]),
    "qpat_ld_create": (c_int32, [c_void_p, c_int32, ctypes.POINTER(c_void_p)]),
    "qpat_ld_destroy": (None, [c_void_p]),
    "qpat_ld_run": (c_int32, [c_void_p, c_void_p, c_void_p, ctypes.POINTER(QpatLdParams),
                              ctypes.POINTER(c_double), ctypes.POINTER(c_int32), ctypes.POINTER(c_int32),
                              ctypes.POINTER(c_int32), c_void_p]),
    "qpat3d_validate": (c_int32, [ctypes.POINTER(QpatParams3d)]),
    "qpat3d_plan_create": (c_int32, [ctypes.POINTER(QpatParams3d), c_void_p, c_void_p, ctypes.POINTER(c_void_p)]),
    "qpat3d_plan_destroy": (None, [c_void_p]),
    "qpat3d_forward": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_void_p]),
    "qpat3d_adjoint": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_void_p]),
    "qpat3d_jtjv": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_void_p]),
    "qpat3d_apply": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_int32, c_void_p]),
    "qpat3d_set_tiles": (c_int32, [c_void_p, c_int32, c_int32, c_int32, c_int32]),
    "qpat3d_get_tiles": (c_int32, [c_void_p, ctypes.POINTER(c_int32), ctypes.POINTER(c_int32),
                                   ctypes.POINTER(c_int32), ctypes.POINTER(c_int32)]),
    "qpat3d_set_graph": (c_int32, [c_void_p, c_int32]),
    "qpat_optical_create": (c_int32, [c_int32, c_int32, c_double, c_int32, ctypes.POINTER(c_void_p)]),
    "qpat_optical_destroy": (None, [c_void_p]),
    "qpat_optical_forward": (c_int32, [c_void_p, c_void_p, c_void_p, ctypes.POINTER(c_double), c_void_p, c_int32,
                                       c_double, c_int32, ctypes.POINTER(c_int32), c_void_p]),
    "qpat_optical_jv": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_double, c_int32,
                                  ctypes.POINTER(c_int32), c_void_p]),
    "qpat_optical_jtv": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_double, c_int32,
                                   ctypes.POINTER(c_int32), c_void_p]),
    "qpat_optical_pixels": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_int32, c_void_p]),
    "qpat_set_check": (c_int32, [c_void_p, c_int32]),
    "qpat_check": (c_int32, [c_void_p, c_void_p]),
    "qpat_plan_info": (c_int32, [c_void_p, ctypes.POINTER(c_int32), ctypes.POINTER(c_int32),
                                 ctypes.POINTER(c_int32), ctypes.POINTER(c_int32), ctypes.POINTER(c_size_t)]),
    "qpat_status_string": (ctypes.c_char_p, [c_int32]),
    "qpat_last_error": (ctypes.c_char_p, []),
}

EXPORTED = tuple(_SIGS)

_lock = threading.Lock()
_lib = None


class QpatError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS.get(status, status)}: {msg}")
        self.status = status


def lib() -> ctypes.CDLL:
    """The loaded libqpat.so.  Raises if it has not been built: there is no
    fallback implementation."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                                   "`python -m paper_1810_11685_amd.build` (hipcc, gfx950)")
            L = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in _SIGS.items():
                f = getattr(L, name)
                f.restype = res
                f.argtypes = args
            _lib = L
        return _lib


def check(status: int, where: str) -> None:
    if status != 0:
        msg = lib().qpat_last_error()
        raise QpatError(status, where, msg.decode() if msg else "")


def _cuda_tensors(objs):
    for o in objs:
        if isinstance(o, torch.Tensor):
            if o.is_cuda:
                yield o
        elif isinstance(o, (list, tuple)):
            yield from _cuda_tensors(o)


def on_stream(fn):
    """Run a binding on the stream given as its `stream` argument.

    The library enqueues its work on that stream; for a stream other than the
    current one the wrapper first makes it wait for the work already queued
    on the current stream (the inputs' producers), runs the binding with it
    as the current stream (so outputs and temporaries are allocated on it)
    and marks the tensor arguments as used by it (so the caching allocator
    does not reuse their memory while it still reads them).  The results
    then belong to that stream; a caller using them elsewhere synchronises
    with it first."""
    sig = inspect.signature(fn)

    @functools.wraps(fn)
    def wrapper(*args, **kw):
        bound = sig.bind(*args, **kw)
        stream = bound.arguments.get("stream")
        cur = torch.cuda.current_stream()
        if stream is None or stream == cur:
            return fn(*args, **kw)
        bound.arguments["stream"] = None
        stream.wait_stream(cur)
        for t in _cuda_tensors(list(bound.arguments.values())):
            t.record_stream(stream)
        with torch.cuda.stream(stream):
            return fn(*bound.args, **bound.kwargs)

    return wrapper
