"""Oracle of the sound-speed gradient of the acoustic data: the derivative of
<r, H_a[c0] p0> with respect to c0 at every node, by reverse mode through the
recursion of Section 3.2.3, with the reference speed c_ref (which sets kappa
and the PML) held fixed.

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this module; the library never imports it.

c0 enters the discrete forward operator in two places:
  * the equation of state (eq num-p) through c^2, c^2 eta and c^2 tau, where
    eta and tau follow eq Twelve (c^2 eta ~ c^(y+2), c^2 tau ~ c^(y+1)): with
    S = rho_x + rho_y, Ys = Y_dis S and Yu = Y_abs u of iterate n,
      dp^{n+1}/dc = (2 c^2 S - (y + 2) c^2 eta Ys + (y + 1) c^2 tau Yu) / c;
  * the additive source of eq s1, dt s = p0 / (2 d c^2), whose derivative is
    -2 / c times itself.
The gradient is therefore sum_n pb_n * dp^{n+1}/dc - (2 / c) p0 * H_a^T r,
with pb_n the adjoint of p^{n+1} (reverse mode) and H_a^T r the p0-gradient.
"""
from __future__ import annotations

import numpy as np

from . import kspace as K


def pressure_sensitivity(op: K.Operators, prm: dict, state: dict) -> np.ndarray:
    """dp^{n+1}/dc at every node from the state of iterate n (v^{n+1/2},
    rho^{n+1}), recomputing S, u, Y_dis S and Y_abs u as eq num-p does."""
    S = state["rx"] + state["ry"]
    c = np.sqrt(op.c2)
    if not op.lossy:
        return 2.0 * op.c2 * S / c
    ex = op.spectral(op.mxm, state["vx"])
    ey = op.spectral(op.mym, state["vy"])
    u = op.rho0 * (op.arx * ex + op.ary * ey)
    y = prm["y"]
    ys = op.spectral(op.ldis, S)
    yu = op.spectral(op.labs, u)
    return (2.0 * op.c2 * S - (y + 2.0) * op.c2 * op.eta * ys + (y + 1.0) * op.c2 * op.tau * yu) / c


def sound_speed_gradient(prm: dict, c0, rho0, p0, r, *, ops: K.Operators | None = None):
    """(d/dc0 <r, H_a[c0] p0>, H_a^T r) for p0 [ny][nx] and r [nt][ns]."""
    op = K.Operators(prm, c0, rho0) if ops is None else ops
    sens = {}
    K.forward(prm, c0, rho0, p0, ops=op, record=lambda n, st: sens.__setitem__(n, pressure_sensitivity(op, prm, st)))
    acc = np.zeros((prm["ny"], prm["nx"]))

    def take(n, pb):
        nonlocal acc
        acc = acc + pb * sens[n]

    g0 = K.adjoint(prm, c0, rho0, r, ops=op, record=take)
    c = np.sqrt(op.c2)
    return acc - 2.0 * np.asarray(p0, float) * g0 / c, g0
