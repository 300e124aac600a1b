"""CPU-only checks of the C ABI: the library loads, exports every entry point
declared in include/qpat.h, and rejects bad arguments on the host before any
device work."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import qpat_inputs as qi
from oracle import kspace as K
from oracle import kspace3d as K3

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qpat.h")


@pytest.fixture(scope="module")
def q():
    import paper_1810_11685_amd as q
    if not os.path.exists(q.LIB_PATH):
        pytest.fail("libqpat.so is not built (run __graft_entry__.build())")
    return q


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qpat(?:3d)?_[a-z_0-9]+)\s*\(", src)))


def test_exports_every_declared_symbol(q):
    names = declared()
    assert len(names) >= 20
    L = q.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(q.EXPORTED)


def good(**kw):
    prm = qi.make_params(64, 48, 1e-4, 2e-8, 50, 1600.0, qi.ring_sensors(8, 15, 1e-4), pml_size=6)
    prm.update(kw)
    return prm


@pytest.mark.parametrize("kw,status", [
    ({}, 0),
    ({"nx": 100}, 2), ({"ny": 4}, 2), ({"nx": 4096}, 2), ({"nx": 63}, 2), ({"nx": 384, "ny": 768}, 0), ({"nx": 2048}, 2),
    ({"dx": 0.0}, 1), ({"dt": -1.0}, 1), ({"dy": float("nan")}, 1),
    ({"nt": 0}, 1), ({"c_ref": 0.0}, 1),
    ({"pml_size": 24}, 1), ({"pml_size": -1}, 1), ({"pml_alpha": -2.0}, 1),
    ({"alpha0_db": -0.1}, 1), ({"y": 1.0}, 2), ({"y": 3.0}, 2), ({"y": 1.0, "alpha0_db": 0.0}, 0),
    ({"sensor_xy": np.array([[0.0, 3e-3]])}, 1), ({"sensor_xy": np.array([[-3.3e-3, 0.0]])}, 1),
    ({"sensor_xy": np.array([[-3.2e-3, -2.4e-3]])}, 0),
])
def test_validate(q, kw, status):
    assert q.validate(good(**kw)) == status


def test_null_and_status_strings(q):
    L = q.lib()
    assert L.qpat_validate(None) == 1
    assert b"NULL" in L.qpat_last_error()
    for s in range(7):
        assert L.qpat_status_string(s)
    assert L.qpat_status_string(6) == b"non-finite output"
    f, t = ctypes.c_float(), ctypes.c_int32()
    assert L.qpat_probe_barrier(3, 256, 256, 10, 0, None, ctypes.byref(f), ctypes.byref(t)) == 1
    assert L.qpat_probe_barrier(0, 256, 100, 10, 0, None, ctypes.byref(f), ctypes.byref(t)) == 1
    assert L.qpat_probe_barrier(0, 256, 256, 1, 0, None, ctypes.byref(f), ctypes.byref(t)) == 1
    assert L.qpat_probe_barrier(2, 256, 256, 10, 6, None, ctypes.byref(f), ctypes.byref(t)) == 1
    assert L.qpat_jtjv_data(None, None, None, None, 1, None) == 1
    hh = ctypes.c_void_p()
    assert L.qpat_ld_create(None, 1, ctypes.byref(hh)) == 1 and hh.value is None
    assert L.qpat_ld_run(None, None, None, None, None, None, None, None, None) == 1
    assert L.qpat_batch_set_schedule(None, 1) == 1
    assert L.qpat_batch_tune(None, None) == 1
    assert L.qpat_set_check(None, 1) == 1
    assert L.qpat_check(None, None) == 1
    h = ctypes.c_void_p()
    p, _keep = q.make_params(good())
    assert L.qpat_plan_create(ctypes.byref(p), None, None, ctypes.byref(h)) == 1
    assert h.value is None
    assert L.qpat_forward(None, None, None, 1, None) == 1
    assert L.qpat_batch_create(None, 0, ctypes.byref(h)) == 1
    assert L.qpat_dot(None, None, 4, None, None) == 1


def test_medium_checks_happen_on_host(q):
    prm = good()
    c0, rho0 = qi.medium(48, 64, 1, 2)
    bad = c0.copy()
    bad[3, 5] = -1.0
    with pytest.raises(q.QpatError) as e:
        q.Plan(prm, bad, rho0)
    assert e.value.status == 1
    bad = rho0.copy()
    bad[0, 0] = float("inf")
    with pytest.raises(q.QpatError) as e:
        q.Plan(prm, c0, bad)
    assert e.value.status == 1


def test_stability_bound_agrees_with_oracle(q):
    c0, rho0 = qi.medium(48, 64, 1, 2)
    cref = 0.6 * c0.max()
    lim = K.stability_limit(c0.max(), cref, 1e-4, 1e-4)
    assert math.isfinite(lim)
    with pytest.raises(q.QpatError) as e:
        q.Plan(good(dt=1.001 * lim, c_ref=cref), c0, rho0)
    assert e.value.status == 3
    try:   # below the bound the host checks pass; without a GPU the upload then fails
        q.Plan(good(dt=0.999 * lim, c_ref=cref), c0, rho0)
    except q.QpatError as e2:
        assert e2.status in (4, 5)


# ---------------------------------------------------------------- 3-D
def good3(**kw):
    sens = np.array([[0.0, 0.0, 0.0], [1e-4, -2e-4, 3e-4]])
    prm = qi.make_params3d(49, 33, 20, 1e-4, 2e-8, 30, 1600.0, sens, pml_size=6)
    prm.update(kw)
    return prm


@pytest.mark.parametrize("kw,status", [
    ({}, 0), ({"nx": 37, "ny": 53, "nz": 13}, 0), ({"nz": 12}, 1), ({"nx": 128, "ny": 64, "nz": 64}, 0),
    ({"nx": 3}, 2), ({"nx": 129}, 2), ({"ny": 128, "nz": 64}, 2), ({"nz": 256}, 2),
    ({"dz": 0.0}, 1), ({"nt": 0}, 1), ({"pml_size": 10}, 1), ({"alpha0_db": -1.0}, 1), ({"y": 1.0}, 1),
    ({"sensor_xyz": np.array([[0.0, 0.0, 1.1e-3]])}, 1), ({"sensor_xyz": np.array([[0.0, 0.0, 0.9e-3]])}, 0),
    ({"sensor_xyz": np.zeros((0, 3))}, 0),
])
def test_validate3d(q, kw, status):
    assert q.validate3d(good3(**kw)) == status


def test_plan3d_host_checks(q):
    c0, rho0 = qi.medium3d(20, 33, 49, 1, 2)
    bad = c0.copy()
    bad[1, 2, 3] = 0.0
    with pytest.raises(q.QpatError) as e:
        q.Plan3D(good3(), bad, rho0)
    assert e.value.status == 1
    cref = 0.6 * c0.max()
    lim = K3.stability_limit(c0.max(), cref, 1e-4, 1e-4, 1e-4)
    with pytest.raises(q.QpatError) as e:
        q.Plan3D(good3(dt=1.001 * lim, c_ref=cref), c0, rho0)
    assert e.value.status == 3
    L = q.lib()
    assert L.qpat3d_validate(None) == 1
    assert L.qpat3d_forward(None, None, None, 1, None) == 1
    assert L.qpat3d_set_tiles(None, 2, 1, 256, 256) == 1


def test_optical_create_checks(q):
    L = q.lib()
    h = ctypes.c_void_p()
    assert L.qpat_optical_create(0, 4, 1e-4, 1, ctypes.byref(h)) == 1
    assert L.qpat_optical_create(4, 4, 0.0, 1, ctypes.byref(h)) == 1
    assert L.qpat_optical_create(4, 4, 1e-4, 65, ctypes.byref(h)) == 1
    assert L.qpat_optical_create(4, 4, 1e-4, 1, None) == 1
    assert L.qpat_optical_forward(None, None, None, None, None, 1, 1e-8, 10, None, None) == 1


def test_build_lists_every_source_once():
    """Every translation unit under csrc/ is compiled, each to its own object
    (optical.hip and optical.cpp share a stem, so object names keep the
    extension)."""
    import os
    from paper_1810_11685_amd import build as B
    units = sorted(f for f in os.listdir(B.CSRC) if f.endswith((".hip", ".cpp")))
    assert sorted(B.SOURCES) == units
    assert len({s + ".o" for s in B.SOURCES}) == len(B.SOURCES)
