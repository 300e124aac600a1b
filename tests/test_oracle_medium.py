"""Pins of the sound-speed gradient oracle (oracle/medium.py): central finite
differences of <r, H_a[c0] p0> along smooth directions (c_ref held fixed),
lossy and lossless, heterogeneous medium with PML and off-node sensors; and
the split into the equation-of-state and source parts."""
import numpy as np
import pytest

import qpat_inputs as qi
from oracle import kspace as K
from oracle import medium as Mg


def problem(alpha0_db, n=32, nt=40, ns=12, seed=21):
    c0, rho0 = qi.medium(n, n, seed, seed + 1, sigma_cells=3.0)
    dx = 1e-4
    prm = qi.make_params(n, n, dx, 0.3 * dx / c0.max(), nt, c0.max(), qi.ring_sensors(ns, 11, dx, phase=0.1),
                         pml_size=5, alpha0_db=alpha0_db, y=1.5)
    p0 = qi.blobs(n, n, seed + 2, count=3, radius_cells=4.0)
    r = qi.gaussian_field((nt, ns), seed + 3)
    return prm, c0, rho0, p0, r


@pytest.mark.parametrize("alpha0_db", [0.75, 0.0])
def test_sound_speed_gradient_matches_finite_differences(alpha0_db):
    prm, c0, rho0, p0, r = problem(alpha0_db)
    g, g0 = Mg.sound_speed_gradient(prm, c0, rho0, p0, r)
    assert np.array_equal(g0, K.adjoint(prm, c0, rho0, r))
    f = lambda c: float(np.sum(r * K.forward(prm, c, rho0, p0)))
    h = 1e-2                                     # m/s, against c ~ 1500 m/s
    for seed in (31, 32):
        d = qi.smooth_noise(prm["ny"], prm["nx"], 3.0, seed)
        d = d / np.abs(d).max()
        fd = (f(c0 + h * d) - f(c0 - h * d)) / (2 * h)
        assert abs(fd - float(np.sum(g * d))) <= 1e-6 * abs(fd)


def test_source_part_is_minus_two_over_c_times_p0_gradient():
    """With r = 0 except the first sample only the n = -1 iterate reaches the
    data: the state part is pb * dp^0/dc and the source part -2 p0 g0 / c."""
    prm, c0, rho0, p0, r = problem(0.75)
    r0 = np.zeros_like(r)
    r0[0] = r[0]
    g, g0 = Mg.sound_speed_gradient(prm, c0, rho0, p0, r0)
    op = K.Operators(prm, c0, rho0)
    # p^0 = c^2 (S - eta Y_dis S + tau Y_abs u) with S = 2 b, u = 0, b = p0 / (4 c^2):
    # p^0 = p0/2 - eta Y_dis(p0 / (2 c^2)) c^2; its c-derivative is taken by the oracle
    state = {}
    K.forward(prm, c0, rho0, p0, ops=op, record=lambda n, st: state.setdefault(n, st), nsteps=1)
    pb = op.measure_T(r0[0])
    expect = pb * Mg.pressure_sensitivity(op, prm, state[-1]) - 2.0 * p0 * g0 / np.sqrt(op.c2)
    assert np.allclose(g, expect, rtol=1e-12, atol=1e-12 * np.abs(expect).max())
