"""Plain FP64 k-space PSTD forward operator H_a and its adjoint in 3-D.

TEST INFRASTRUCTURE (see the package docstring): slow, literal, FP64.

The scheme is the one of Section 3.2.3 with d = 3: three velocity and three
density components, so the stacked state z_n of the paper holds 7N values
(Section 3.2.4), and the additive source of eq s1 puts p0 / (2 d c^2) with
d = 3 into each density component at iterates n = -1 and 0.

The conventions of the 2-D oracle carry over axis by axis: fields are
[nz, ny, nx] arrays, x along the last axis; node (k, j, i) sits at
((i - nx/2) dx, (j - ny/2) dy, (k - nz/2) dz); numpy DFT convention with the
Nyquist bin at -pi/d; sinc(x) = sin x / x with a caller-given c_ref in eq grr,
now with the 3-D |k|; |k|^(y-2), |k|^(y-1) set to 0 at k = 0; the PML inside
the grid with the 4th-power profile on every axis, velocities at half nodes;
the staggered density is the mean of the two neighbours along its axis;
the smoothing operator S is the identity; the measurement M is trilinear
interpolation from the eight surrounding nodes.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import fft as sfft

from .kspace import tau_eta, workers

D = 3  # spatial dimension d of the paper


def stability_limit(c_max: float, c_ref: float, dx: float, dy: float, dz: float) -> float:
    """Largest stable dt: the per-mode recursion of the homogeneous scheme is
    bounded iff |sin(c_ref |k| dt / 2)| <= c_ref / c for every mode."""
    if c_ref >= c_max:
        return math.inf
    kmax = math.sqrt((math.pi / dx) ** 2 + (math.pi / dy) ** 2 + (math.pi / dz) ** 2)
    return 2.0 * math.asin(c_ref / c_max) / (c_ref * kmax)


def sensor_taps(prm: dict):
    """Trilinear interpolation taps of M: (flat_index[ns, 8], weight[ns, 8]).
    A sensor must lie inside the node grid; a tap past the last node has
    weight 0 and is clamped onto the grid."""
    nx, ny, nz = prm["nx"], prm["ny"], prm["nz"]
    dx, dy, dz = prm["dx"], prm["dy"], prm["dz"]
    xyz = np.asarray(prm["sensor_xyz"], dtype=np.float64).reshape(-1, 3)
    idx = np.zeros((len(xyz), 8), dtype=np.int64)
    w = np.zeros((len(xyz), 8))
    for s, (x, y, z) in enumerate(xyz):
        u, v, t = x / dx + nx / 2, y / dy + ny / 2, z / dz + nz / 2
        if not (0.0 <= u <= nx - 1 and 0.0 <= v <= ny - 1 and 0.0 <= t <= nz - 1):
            raise ValueError(f"sensor {s} at ({x}, {y}, {z}) m lies outside the grid")
        i0, j0, k0 = int(math.floor(u)), int(math.floor(v)), int(math.floor(t))
        fx, fy, fz = u - i0, v - j0, t - k0
        i1, j1, k1 = min(i0 + 1, nx - 1), min(j0 + 1, ny - 1), min(k0 + 1, nz - 1)
        e = 0
        for kk, wz in ((k0, 1 - fz), (k1, fz)):
            for jj, wy in ((j0, 1 - fy), (j1, fy)):
                for ii, wx in ((i0, 1 - fx), (i1, fx)):
                    idx[s, e] = (kk * ny + jj) * nx + ii
                    w[s, e] = wz * wy * wx
                    e += 1
    return idx, w


class Operators:
    """Discretised operators and medium diagonals of Section 3.2.2 in 3-D."""

    def __init__(self, prm: dict, c0: np.ndarray, rho0: np.ndarray):
        nx, ny, nz = prm["nx"], prm["ny"], prm["nz"]
        dx, dy, dz, dt = prm["dx"], prm["dy"], prm["dz"], prm["dt"]
        c0 = np.asarray(c0, dtype=np.float64)
        rho0 = np.asarray(rho0, dtype=np.float64)
        assert c0.shape == (nz, ny, nx) and rho0.shape == (nz, ny, nx)
        self.prm, self.nx, self.ny, self.nz, self.dt = prm, nx, ny, nz, dt

        kx = 2.0 * math.pi * np.fft.fftfreq(nx, dx)
        ky = 2.0 * math.pi * np.fft.fftfreq(ny, dy)
        kz = 2.0 * math.pi * np.fft.fftfreq(nz, dz)
        KZ, KY, KX = np.meshgrid(kz, ky, kx, indexing="ij")
        K = np.sqrt(KX ** 2 + KY ** 2 + KZ ** 2)
        self.K = K
        arg = prm["c_ref"] * K * dt / 2.0
        safe = np.where(arg == 0.0, 1.0, arg)
        kappa = np.where(arg == 0.0, 1.0, np.sin(safe) / safe)
        self.kappa = kappa
        # staggered k-space gradients, eq grr, one per axis
        self.mp = [1j * KK * np.exp(1j * KK * d / 2.0) * kappa for KK, d in ((KX, dx), (KY, dy), (KZ, dz))]
        self.mm = [1j * KK * np.exp(-1j * KK * d / 2.0) * kappa for KK, d in ((KX, dx), (KY, dy), (KZ, dz))]
        y = prm["y"]
        Ks = np.where(K == 0.0, 1.0, K)
        self.labs = np.where(K == 0.0, 0.0, Ks ** (y - 2.0))
        self.ldis = np.where(K == 0.0, 0.0, Ks ** (y - 1.0))

        self.c2 = c0 ** 2
        self.rho0 = rho0
        # rho0 at the staggered positions r_i + d_i / 2 (axis 2 = x, 1 = y, 0 = z)
        self.rhos = [0.5 * (rho0 + np.roll(rho0, -1, axis=a)) for a in (2, 1, 0)]
        self.lossy = prm["alpha0_db"] != 0.0
        if self.lossy:
            self.tau, self.eta = tau_eta(c0, prm["alpha0_db"], y)
        else:
            self.tau = np.zeros_like(c0)
            self.eta = np.zeros_like(c0)

        L = prm["pml_size"]

        def sigma(pos, n, d):
            if L <= 0:
                return np.zeros_like(pos)
            xi = np.maximum(0.0, np.maximum(L - pos, pos - (n - 1 - L)))
            return prm["pml_alpha"] * (prm["c_ref"] / d) * (xi / L) ** 4

        shapes = ((1, 1, nx), (1, ny, 1), (nz, 1, 1))
        self.ar, self.av = [], []
        for n, d, shp in ((nx, dx, shapes[0]), (ny, dy, shapes[1]), (nz, dz, shapes[2])):
            pos = np.arange(n, dtype=np.float64)
            self.ar.append(np.exp(-sigma(pos, n, d) * dt / 2.0).reshape(shp))
            self.av.append(np.exp(-sigma(pos + 0.5, n, d) * dt / 2.0).reshape(shp))

        self.tap_idx, self.tap_w = sensor_taps(prm)

    def spectral(self, m: np.ndarray, f: np.ndarray) -> np.ndarray:
        """F^-1 { m F{f} } for a real field f."""
        w = workers()
        return np.real(sfft.ifftn(m * sfft.fftn(f, workers=w), workers=w))

    def measure(self, p: np.ndarray) -> np.ndarray:
        return (p.reshape(-1)[self.tap_idx] * self.tap_w).sum(axis=1)

    def measure_T(self, r: np.ndarray) -> np.ndarray:
        out = np.zeros(self.nx * self.ny * self.nz)
        np.add.at(out, self.tap_idx.reshape(-1), (self.tap_w * r[:, None]).reshape(-1))
        return out.reshape(self.nz, self.ny, self.nx)


def forward(prm: dict, c0, rho0, p0, *, ops: Operators | None = None, record=None,
            nsteps: int | None = None) -> np.ndarray:
    """H_a p0 in 3-D: sensor data [nt, ns] (Section 3.2.3, steps 1-4, d = 3).
    `record(n, state)` receives v^{n+1/2} (list of 3), rho^{n+1} (list of 3)
    and p^{n+1} after every iterate."""
    op = Operators(prm, c0, rho0) if ops is None else ops
    nt = prm["nt"] if nsteps is None else nsteps
    dt = prm["dt"]
    shape = (prm["nz"], prm["ny"], prm["nx"])
    v = [np.zeros(shape) for _ in range(3)]
    rho = [np.zeros(shape) for _ in range(3)]
    p = np.zeros(shape)
    b = np.asarray(p0, dtype=np.float64) / (2.0 * D * op.c2)
    data = np.zeros((nt, len(op.tap_w)))
    for n in range(-1, nt - 1):
        # 1. momentum, eq num-vel
        for i in range(3):
            g = op.spectral(op.mp[i], p)
            v[i] = op.av[i] * (op.av[i] * v[i] - dt * g / op.rhos[i])
        # 2. mass with the additive source, eq num-rho
        e = [op.spectral(op.mm[i], v[i]) for i in range(3)]
        for i in range(3):
            rho[i] = op.ar[i] * (op.ar[i] * rho[i] - dt * op.rho0 * e[i])
            if n in (-1, 0):
                rho[i] = rho[i] + b
        # 3. equation of state, eq num-p
        S = rho[0] + rho[1] + rho[2]
        if op.lossy:
            u = op.rho0 * (op.ar[0] * e[0] + op.ar[1] * e[1] + op.ar[2] * e[2])
            p = op.c2 * (S - op.eta * op.spectral(op.ldis, S) + op.tau * op.spectral(op.labs, u))
        else:
            p = op.c2 * S
        # 4. measurement, eq num-m
        data[n + 1] = op.measure(p)
        if record is not None:
            record(n, dict(v=list(v), rho=list(rho), p=p))
    return data


def adjoint(prm: dict, c0, rho0, r, *, ops: Operators | None = None) -> np.ndarray:
    """H_a^T r in 3-D by reverse-mode transposition of `forward`, one linear
    operation at a time (discretise-then-adjoint, Section 3.2.4), under the
    unweighted inner products of R^N and R^{Ns Nt}."""
    op = Operators(prm, c0, rho0) if ops is None else ops
    nt, dt = prm["nt"], prm["dt"]
    r = np.asarray(r, dtype=np.float64).reshape(nt, -1)
    shape = (prm["nz"], prm["ny"], prm["nx"])
    vb = [np.zeros(shape) for _ in range(3)]
    rb = [np.zeros(shape) for _ in range(3)]
    pb = np.zeros(shape)
    gsrc = np.zeros(shape)
    for n in range(nt - 2, -2, -1):
        # 4^T: measurement
        pb = pb + op.measure_T(r[n + 1])
        # 3^T: equation of state
        q = op.c2 * pb
        if op.lossy:
            Sb = q - op.spectral(op.ldis, op.eta * q)
            ub = op.spectral(op.labs, op.tau * q)
        else:
            Sb = q
            ub = np.zeros(shape)
        for i in range(3):
            rb[i] = rb[i] + Sb
        # 2^T: source and mass update
        if n in (-1, 0):
            gsrc = gsrc + rb[0] + rb[1] + rb[2]
        for i in range(3):
            eb = op.rho0 * op.ar[i] * (ub - dt * rb[i])
            rb[i] = op.ar[i] ** 2 * rb[i]
            vb[i] = vb[i] - op.spectral(op.mp[i], eb)     # (grad_i^-)^T = -grad_i^+
        # 1^T: momentum update
        pb = np.zeros(shape)
        for i in range(3):
            gb = -dt * op.av[i] * vb[i] / op.rhos[i]
            vb[i] = op.av[i] ** 2 * vb[i]
            pb = pb - op.spectral(op.mm[i], gb)           # (grad_i^+)^T = -grad_i^-
    return gsrc / (2.0 * D * op.c2)
