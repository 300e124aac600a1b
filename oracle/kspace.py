"""Plain FP64 k-space PSTD forward operator H_a and its adjoints (2-D).

TEST INFRASTRUCTURE (see the package docstring): slow, literal, FP64.

Conventions (readings of points the paper leaves open; each one is also
listed in the design notes):

* Fields are [ny, nx] arrays, x along the last axis.  Node (j, i) sits at
  x = (i - nx/2) dx, y = (j - ny/2) dy, so the centre node is the origin
  (Section 6.1: the 2-D domain [-5, 4.92] mm with 128 nodes).
* F is numpy's unnormalised forward DFT, F^-1 carries 1/N.  Wavenumbers are
  2 pi fftfreq; the Nyquist bin of an even grid is -pi/dx.  There the
  staggered-gradient symbol i k e^{+-i k dx/2} is real, so the operators are
  real matrices and (grad_i^+)^T = -grad_i^- holds exactly.
* sinc(x) = sin(x)/x in the k-space correction of eq grr, with a caller-given
  reference speed c_ref.
* The fractional-Laplacian symbols |k|^(y-2) and |k|^(y-1) are set to 0 at k = 0.
* eta Y_dis and tau Y_abs apply the spectral filter first, then the diagonal.
* alpha0 is given in dB MHz^-y cm^-1 (Section 6.1.4) and converted to
  Np (rad/s)^-y m^-1 before eq Twelve.
* The PML (eq dis-pml) lies inside the grid, pml_size cells on each side,
  with a 4th-power profile sigma = pml_alpha * (c_ref/dx) * (xi/L)^4 [1/s]
  (pml_alpha in Np per cell), xi the depth into the layer in cells.  Velocity
  components use the profile at their staggered half-node positions,
  density components at the nodes.
* The staggered density rho0_i is the mean of the two neighbouring nodes
  (periodic wrap).
* The smoothing operator S of eq s1 is the identity.
* The measurement operator M of eq num-m is bilinear interpolation from the
  four surrounding nodes.
* Data are time-major [nt, ns]: row n+1 holds P_{n+1} = M p_{n+1} for the loop
  n = -1 .. nt-2 (Definition 4).
"""
from __future__ import annotations

import math
import os

import numpy as np
from scipy import fft as sfft

D = 2  # spatial dimension d of the paper (this oracle is 2-D)
_WORKERS = int(os.environ.get("QPAT_ORACLE_WORKERS", "0")) or (os.cpu_count() or 1)


def set_workers(n: int) -> None:
    """Number of threads scipy.fft may use inside the oracle."""
    global _WORKERS
    _WORKERS = max(1, int(n))


def workers() -> int:
    return _WORKERS


def alpha0_np(alpha0_db: float, y: float) -> float:
    """dB MHz^-y cm^-1  ->  Np (rad/s)^-y m^-1.

    alpha(f) [dB/cm] = alpha0_db * f_MHz^y; 1 Np = 20 log10(e) dB; 1/cm = 100/m;
    f_MHz = omega / (2 pi 1e6)."""
    return alpha0_db * 100.0 / (20.0 * math.log10(math.e)) * (1e-6 / (2.0 * math.pi)) ** y


def tau_eta(c0: np.ndarray, alpha0_db: float, y: float):
    """Absorption and dispersion proportionality coefficients, eq Twelve."""
    a0 = alpha0_np(alpha0_db, y)
    tau = -2.0 * a0 * c0 ** (y - 1.0)
    eta = 2.0 * a0 * c0 ** y * math.tan(math.pi * y / 2.0)
    return tau, eta


def stability_limit(c_max: float, c_ref: float, dx: float, dy: float) -> float:
    """Largest stable dt of the k-space scheme.

    In a homogeneous medium of speed c each Fourier mode obeys
    p^{n+1} + p^{n-1} = (2 - dt^2 c^2 |k|^2 sinc^2(c_ref |k| dt/2)) p^n, which is
    bounded iff |sin(c_ref |k| dt/2)| <= c_ref/c.  With c_ref >= c_max this holds
    for every dt; otherwise dt <= 2 asin(c_ref/c_max) / (c_ref k_max)."""
    if c_ref >= c_max:
        return math.inf
    kmax = math.hypot(math.pi / dx, math.pi / dy)
    return 2.0 * math.asin(c_ref / c_max) / (c_ref * kmax)


def sensor_taps(prm: dict):
    """Bilinear interpolation taps of the measurement operator M (eq num-m).

    Returns (flat_index[ns, 4], weight[ns, 4]).  A sensor must lie inside the
    node grid; a tap that would fall off the last node has weight 0 and is
    clamped onto the grid."""
    nx, ny, dx, dy = prm["nx"], prm["ny"], prm["dx"], prm["dy"]
    xy = np.asarray(prm["sensor_xy"], dtype=np.float64).reshape(-1, 2)
    idx = np.zeros((len(xy), 4), dtype=np.int64)
    w = np.zeros((len(xy), 4))
    for s, (x, y) in enumerate(xy):
        u = x / dx + nx / 2
        v = y / dy + ny / 2
        if not (0.0 <= u <= nx - 1 and 0.0 <= v <= ny - 1):
            raise ValueError(f"sensor {s} at ({x}, {y}) m lies outside the grid")
        ix, iy = int(math.floor(u)), int(math.floor(v))
        fx, fy = u - ix, v - iy
        ix1, iy1 = min(ix + 1, nx - 1), min(iy + 1, ny - 1)
        for t, (jj, ii, ww) in enumerate(((iy, ix, (1 - fx) * (1 - fy)), (iy, ix1, fx * (1 - fy)),
                                          (iy1, ix, (1 - fx) * fy), (iy1, ix1, fx * fy))):
            idx[s, t] = jj * nx + ii
            w[s, t] = ww
    return idx, w


class Operators:
    """All discretised operators and medium diagonals of Section 3.2.2."""

    def __init__(self, prm: dict, c0: np.ndarray, rho0: np.ndarray):
        nx, ny = prm["nx"], prm["ny"]
        dx, dy, dt = prm["dx"], prm["dy"], prm["dt"]
        c0 = np.asarray(c0, dtype=np.float64)
        rho0 = np.asarray(rho0, dtype=np.float64)
        assert c0.shape == (ny, nx) and rho0.shape == (ny, nx)
        self.prm, self.nx, self.ny, self.dt = prm, nx, ny, dt

        # wavenumbers (rad/m), Nyquist at -pi/dx
        kx = 2.0 * math.pi * np.fft.fftfreq(nx, dx)
        ky = 2.0 * math.pi * np.fft.fftfreq(ny, dy)
        KX, KY = np.meshgrid(kx, ky)
        K = np.sqrt(KX ** 2 + KY ** 2)
        self.K = K
        # k-space correction sinc(c_ref k dt / 2), eq grr
        arg = prm["c_ref"] * K * dt / 2.0
        safe = np.where(arg == 0.0, 1.0, arg)
        kappa = np.where(arg == 0.0, 1.0, np.sin(safe) / safe)
        self.kappa = kappa
        # staggered k-space gradients d/dr_i^{+-}, eq grr
        self.mxp = 1j * KX * np.exp(1j * KX * dx / 2.0) * kappa
        self.mxm = 1j * KX * np.exp(-1j * KX * dx / 2.0) * kappa
        self.myp = 1j * KY * np.exp(1j * KY * dy / 2.0) * kappa
        self.mym = 1j * KY * np.exp(-1j * KY * dy / 2.0) * kappa
        # fractional Laplacian symbols of Y_abs and Y_dis (zero at k = 0)
        y = prm["y"]
        Ks = np.where(K == 0.0, 1.0, K)
        self.labs = np.where(K == 0.0, 0.0, Ks ** (y - 2.0))
        self.ldis = np.where(K == 0.0, 0.0, Ks ** (y - 1.0))

        # medium diagonals
        self.c2 = c0 ** 2
        self.rho0 = rho0
        self.rhox = 0.5 * (rho0 + np.roll(rho0, -1, axis=1))   # at x + dx/2
        self.rhoy = 0.5 * (rho0 + np.roll(rho0, -1, axis=0))   # at y + dy/2
        self.lossy = prm["alpha0_db"] != 0.0
        if self.lossy:
            self.tau, self.eta = tau_eta(c0, prm["alpha0_db"], y)
        else:
            self.tau = np.zeros_like(c0)
            self.eta = np.zeros_like(c0)

        # PML diagonals A_i = exp(-alpha_i dt / 2), eq dis-pml
        L = prm["pml_size"]

        def sigma(pos, n, d):
            if L <= 0:
                return np.zeros_like(pos)
            xi = np.maximum(0.0, np.maximum(L - pos, pos - (n - 1 - L)))
            return prm["pml_alpha"] * (prm["c_ref"] / d) * (xi / L) ** 4

        ix = np.arange(nx, dtype=np.float64)
        iy = np.arange(ny, dtype=np.float64)
        self.arx = np.exp(-sigma(ix, nx, dx) * dt / 2.0)[None, :]
        self.avx = np.exp(-sigma(ix + 0.5, nx, dx) * dt / 2.0)[None, :]
        self.ary = np.exp(-sigma(iy, ny, dy) * dt / 2.0)[:, None]
        self.avy = np.exp(-sigma(iy + 0.5, ny, dy) * dt / 2.0)[:, None]

        self.tap_idx, self.tap_w = sensor_taps(prm)

    # F^-1 { m F{f} } for a real field f (the result is real by symmetry of m)
    def spectral(self, m: np.ndarray, f: np.ndarray) -> np.ndarray:
        return np.real(sfft.ifft2(m * sfft.fft2(f, workers=_WORKERS), workers=_WORKERS))

    def measure(self, p: np.ndarray) -> np.ndarray:
        """M p: bilinear samples at the sensors."""
        return (p.reshape(-1)[self.tap_idx] * self.tap_w).sum(axis=1)

    def measure_T(self, r: np.ndarray) -> np.ndarray:
        """M^T r: scatter of sensor values back onto the nodes."""
        out = np.zeros(self.nx * self.ny)
        np.add.at(out, self.tap_idx.reshape(-1), (self.tap_w * r[:, None]).reshape(-1))
        return out.reshape(self.ny, self.nx)


def forward(prm: dict, c0, rho0, p0, *, ops: Operators | None = None, record=None,
            inject=(-1, 0), nsteps: int | None = None) -> np.ndarray:
    """H_a p0: sensor data [nt, ns] (Section 3.2.3, steps 1-4).

    The initial pressure enters as the additive mass source of eq s1,
    dt * s = p0 / (2 d c0^2), at iterates n = -1 and 0 (`inject` can change the
    set for bookkeeping tests).  `record(n, state)` receives v^{n+1/2},
    rho^{n+1} and p^{n+1} after every iterate.  `nsteps` stops early (the
    returned array then holds only the first `nsteps` samples)."""
    op = Operators(prm, c0, rho0) if ops is None else ops
    nt = prm["nt"] if nsteps is None else nsteps
    dt = prm["dt"]
    shape = (prm["ny"], prm["nx"])
    vx = np.zeros(shape); vy = np.zeros(shape)
    rx = np.zeros(shape); ry = np.zeros(shape)
    p = np.zeros(shape)
    b = np.asarray(p0, dtype=np.float64) / (2.0 * D * op.c2)
    data = np.zeros((nt, len(op.tap_w)))
    for n in range(-1, nt - 1):
        # 1. momentum, eq num-vel
        gx = op.spectral(op.mxp, p)
        gy = op.spectral(op.myp, p)
        vx = op.avx * (op.avx * vx - dt * gx / op.rhox)
        vy = op.avy * (op.avy * vy - dt * gy / op.rhoy)
        # 2. mass with the additive source, eq num-rho
        ex = op.spectral(op.mxm, vx)
        ey = op.spectral(op.mym, vy)
        rx = op.arx * (op.arx * rx - dt * op.rho0 * ex)
        ry = op.ary * (op.ary * ry - dt * op.rho0 * ey)
        if n in inject:
            rx = rx + b
            ry = ry + b
        # 3. equation of state with absorption and dispersion, eq num-p
        S = rx + ry
        u = op.rho0 * (op.arx * ex + op.ary * ey)
        if op.lossy:
            p = op.c2 * (S - op.eta * op.spectral(op.ldis, S) + op.tau * op.spectral(op.labs, u))
        else:
            p = op.c2 * S
        # 4. measurement, eq num-m
        data[n + 1] = op.measure(p)
        if record is not None:
            record(n, dict(vx=vx, vy=vy, rx=rx, ry=ry, p=p))
    return data


def adjoint(prm: dict, c0, rho0, r, *, ops: Operators | None = None, record=None) -> np.ndarray:
    """H_a^T r by reverse-mode transposition of `forward`, one linear
    operation at a time, under the unweighted Euclidean inner products of
    R^N and R^{Ns Nt} (discretise-then-adjoint, Section 3.2.4).

    Transposes used: the medium, PML and source maps are diagonal;
    (F^-1 diag(m) F)^T = F^-1 diag(conj m) F for a real operator, hence
    (grad_i^+)^T = -grad_i^- and Y_abs, Y_dis are symmetric.  `record(n, pb)`
    receives the complete adjoint of p^{n+1} at every iterate n."""
    op = Operators(prm, c0, rho0) if ops is None else ops
    nt, dt = prm["nt"], prm["dt"]
    r = np.asarray(r, dtype=np.float64).reshape(nt, -1)
    shape = (prm["ny"], prm["nx"])
    vbx = np.zeros(shape); vby = np.zeros(shape)
    rbx = np.zeros(shape); rby = np.zeros(shape)
    pb = np.zeros(shape)
    gsrc = np.zeros(shape)
    for n in range(nt - 2, -2, -1):
        # 4^T: measurement
        pb = pb + op.measure_T(r[n + 1])
        if record is not None:
            record(n, pb)
        # 3^T: equation of state (p^{n+1} does not depend on p^n directly)
        q = op.c2 * pb
        if op.lossy:
            Sb = q - op.spectral(op.ldis, op.eta * q)
            ub = op.spectral(op.labs, op.tau * q)
        else:
            Sb = q
            ub = np.zeros(shape)
        rbx = rbx + Sb
        rby = rby + Sb
        # 2^T: source and mass update
        if n in (-1, 0):
            gsrc = gsrc + rbx + rby
        ebx = op.rho0 * op.arx * (ub - dt * rbx)
        eby = op.rho0 * op.ary * (ub - dt * rby)
        rbx = op.arx ** 2 * rbx
        rby = op.ary ** 2 * rby
        vbx = vbx - op.spectral(op.mxp, ebx)    # (grad_x^-)^T = -grad_x^+
        vby = vby - op.spectral(op.myp, eby)
        # 1^T: momentum update
        gbx = -dt * op.avx * vbx / op.rhox
        gby = -dt * op.avy * vby / op.rhoy
        vbx = op.avx ** 2 * vbx
        vby = op.avy ** 2 * vby
        pb = -op.spectral(op.mxm, gbx) - op.spectral(op.mym, gby)   # (grad^+)^T = -grad^-
    return gsrc / (2.0 * D * op.c2)


def adjoint_paper(prm: dict, c0, rho0, r, *, ops: Operators | None = None) -> np.ndarray:
    """H_a^* r by the paper's adjoint recursion (Lemma 2, eqs adj_data, col1,
    t41), in the rescaled variables rho_hat = Q A^-1 rho, v_hat = (A Q_s)^-1 v.

    The recursion applies T^* nt-1 times to z^*, driven by the pairwise-summed
    data s^adj = M^T (P_{m} + P_{m-1}); the result is
    theta( sum_i (I - Y_dis eta) C p + A Q^-1 rho_hat ), theta = S / (2 d C).
    With the split PML diagonals, A_rho multiplies the density lines and A_v
    the velocity line."""
    op = Operators(prm, c0, rho0) if ops is None else ops
    nt, dt = prm["nt"], prm["dt"]
    r = np.asarray(r, dtype=np.float64).reshape(nt, -1)
    shape = (prm["ny"], prm["nx"])
    rhx = np.zeros(shape); rhy = np.zeros(shape)
    vhx = np.zeros(shape); vhy = np.zeros(shape)

    def X_of(p):   # (I - Y_dis eta) C p
        cp = op.c2 * p
        return cp - op.spectral(op.ldis, op.eta * cp) if op.lossy else cp

    def W_of(p):   # (Y_abs / dt) tau C p
        return op.spectral(op.labs, op.tau * op.c2 * p) / dt if op.lossy else np.zeros(shape)

    p = op.measure_T(r[nt - 1])                 # z*_0 (source at n = -1)
    for k in range(0, nt - 1):                  # z*_{k+1} = T* z*_k + S^adj
        X = X_of(p)
        W = W_of(p)
        rhx = op.arx * (op.arx * rhx + op.rho0 * X)
        rhy = op.ary * (op.ary * rhy + op.rho0 * X)
        vhx = op.avx * (op.avx * vhx + (dt / op.rhox) * op.spectral(op.mxp, rhx - op.rho0 * op.arx * W))
        vhy = op.avy * (op.avy * vhy + (dt / op.rhoy) * op.spectral(op.myp, rhy - op.rho0 * op.ary * W))
        sadj = op.measure_T(r[nt - 1 - k] + r[nt - 2 - k])
        p = dt * (op.spectral(op.mxm, vhx) + op.spectral(op.mym, vhy)) + sadj
    tot = D * X_of(p) + op.arx * rhx / op.rho0 + op.ary * rhy / op.rho0
    return tot / (2.0 * D * op.c2)


def gradient(prm: dict, c0, rho0, p0, d, *, ops: Operators | None = None) -> np.ndarray:
    """Gradient of 0.5 ||H_a p0 - d||^2 with respect to p0: H_a^T (H_a p0 - d)."""
    op = Operators(prm, c0, rho0) if ops is None else ops
    res = forward(prm, c0, rho0, p0, ops=op) - np.asarray(d).reshape(prm["nt"], -1)
    return adjoint(prm, c0, rho0, res, ops=op)
