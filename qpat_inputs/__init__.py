"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module only *draws* inputs: tissue-like media, initial-pressure phantoms,
ring sensor layouts, residuals and noise.  It contains none of the k-space
method's arithmetic (no wavenumbers, no operators, no time stepping), so both
the FP64 oracle and the GPU library can be fed from it without sharing code.

The paper's own phantoms exist only as figures that are not available, so
these generators stand in for them with the shapes the paper uses: 2-D square
grids, a smooth heterogeneous sound speed and density, power-law absorption
with the paper's alpha0 = 0.75 dB MHz^-y cm^-1 and y = 1.5 (Section 6.1,
"Acoustic properties"), a PML of 20 cells with a maximum attenuation of
2 Np per cell, and point detectors around the object.

Every generator takes an explicit seed and uses numpy's PCG64.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "smooth_noise", "medium", "blobs", "ring_sensors", "gaussian_field",
    "make_params", "config", "block_mean", "CONFIGS",
    "smooth_noise3d", "medium3d", "blobs3d", "face_sensors", "make_params3d", "config3d",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def smooth_noise(n_y: int, n_x: int, sigma_cells: float, seed: int) -> np.ndarray:
    """White N(0,1) noise, periodically Gaussian-filtered (sigma in cells),
    mean removed and scaled to a maximum absolute value of 1."""
    w = _rng(seed).standard_normal((n_y, n_x))
    fy = np.fft.fftfreq(n_y)[:, None]
    fx = np.fft.fftfreq(n_x)[None, :]
    g = np.exp(-2.0 * (math.pi * sigma_cells) ** 2 * (fx ** 2 + fy ** 2))
    s = np.real(np.fft.ifft2(np.fft.fft2(w) * g))
    s -= s.mean()
    m = np.abs(s).max()
    return s / m if m > 0 else s


def medium(n_y: int, n_x: int, seed_c: int, seed_rho: int, *, c_mean=1500.0,
           c_amp=100.0, rho_mean=1000.0, rho_amp=80.0, sigma_cells=8.0):
    """Tissue-like heterogeneous medium: c0 = 1500 +- 100 m/s and
    rho0 = 1000 +- 80 kg/m^3, each a smooth random field (independent seeds)."""
    c0 = c_mean + c_amp * smooth_noise(n_y, n_x, sigma_cells, seed_c)
    rho0 = rho_mean + rho_amp * smooth_noise(n_y, n_x, sigma_cells, seed_rho)
    return c0, rho0


def blobs(n_y: int, n_x: int, seed: int, *, count=5, radius_cells=None,
          sigma_range=(2.0, 6.0), amp_range=(0.0, 1.0)) -> np.ndarray:
    """Initial pressure: a sum of `count` Gaussian blobs.  Centres are drawn
    uniformly in a disc about the centre node (n_x/2, n_y/2)."""
    rng = _rng(seed)
    if radius_cells is None:
        radius_cells = 0.2 * min(n_x, n_y)
    yy, xx = np.mgrid[0:n_y, 0:n_x].astype(np.float64)
    out = np.zeros((n_y, n_x))
    for _ in range(count):
        r = radius_cells * math.sqrt(rng.uniform())
        t = rng.uniform(0.0, 2.0 * math.pi)
        cx = n_x / 2 + r * math.cos(t)
        cy = n_y / 2 + r * math.sin(t)
        sg = rng.uniform(*sigma_range)
        a = rng.uniform(*amp_range)
        out += a * np.exp(-((xx - cx) ** 2 + (yy - cy) ** 2) / (2.0 * sg * sg))
    return out


def ring_sensors(ns: int, radius_cells: float, dx: float, dy: float | None = None,
                 phase: float = 0.0) -> np.ndarray:
    """`ns` point detectors equally spaced on a circle about the centre node.
    Returns [ns, 2] positions (x, y) in metres relative to the centre node."""
    dy = dx if dy is None else dy
    th = phase + 2.0 * math.pi * np.arange(ns) / ns
    return np.stack([radius_cells * dx * np.cos(th), radius_cells * dy * np.sin(th)], axis=1)


def gaussian_field(shape, seed: int, scale: float = 1.0) -> np.ndarray:
    """i.i.d. N(0, scale^2) array (random test vectors and residuals)."""
    return scale * _rng(seed).standard_normal(shape)


def block_mean(a: np.ndarray, f: int) -> np.ndarray:
    """f x f block mean (used to make a coarse copy of a fine-grid input)."""
    ny, nx = a.shape
    return a.reshape(ny // f, f, nx // f, f).mean(axis=(1, 3))


def make_params(nx, ny, dx, dt, nt, c_ref, sensor_xy, *, dy=None, pml_size=20,
                pml_alpha=2.0, alpha0_db=0.75, y=1.5) -> dict:
    """Problem parameters in the form both the oracle and the library take."""
    return dict(nx=int(nx), ny=int(ny), dx=float(dx), dy=float(dx if dy is None else dy),
                dt=float(dt), nt=int(nt), c_ref=float(c_ref), pml_size=int(pml_size),
                pml_alpha=float(pml_alpha), alpha0_db=float(alpha0_db), y=float(y),
                sensor_xy=np.ascontiguousarray(sensor_xy, dtype=np.float64))


# Workload table.  "small" is the 128^2 parity case; "fwdadj512" the headline
# 512^2 forward+adjoint; "autograd512" the differentiation case; "uneven" the
# mixed-grid batch; "gn1024" the Gauss-Newton batch (with its 256^2 coarse copy).
CONFIGS = {
    "small": dict(n=128, nt=600, ns=64, ring=55, seeds=(1810, 1811, 1812), alpha0_db=0.75, y=1.5),
    "fwdadj512": dict(n=512, nt=2000, ns=256, ring=220, seeds=(1820, 1821, 1822), alpha0_db=0.75, y=1.5),
    "autograd512": dict(n=512, nt=2000, ns=256, ring=220, seeds=(1820, 1821, 1822), alpha0_db=0.75, y=1.5),
    "gn1024": dict(n=1024, nt=4000, ns=512, ring=440, seeds=(3000, 3001, 3002), alpha0_db=0.5, y=1.3),
}


def config(name: str, *, n=None, nt=None, ns=None, ring=None, cfl=0.3, dx=1e-4,
           seeds=None, alpha0_db=None, y=None, pml_size=20, pml_alpha=2.0) -> dict:
    """Build a full problem (params + c0, rho0, p0) for a named workload,
    optionally overriding its sizes.  dt = cfl * dx / max(c0); c_ref = max(c0)."""
    base = dict(CONFIGS[name])
    n = base["n"] if n is None else n
    nt = base["nt"] if nt is None else nt
    ns = base["ns"] if ns is None else ns
    ring = round(base["ring"] * n / base["n"]) if ring is None else ring
    sc, sr, sp = base["seeds"] if seeds is None else seeds
    a0 = base["alpha0_db"] if alpha0_db is None else alpha0_db
    yy = base["y"] if y is None else y
    c0, rho0 = medium(n, n, sc, sr)
    p0 = blobs(n, n, sp, radius_cells=0.5 * ring)
    cmax = float(c0.max())
    dt = cfl * dx / cmax
    prm = make_params(n, n, dx, dt, nt, cmax, ring_sensors(ns, ring, dx),
                      pml_size=pml_size, pml_alpha=pml_alpha, alpha0_db=a0, y=yy)
    return dict(params=prm, c0=c0, rho0=rho0, p0=p0)


def uneven_batch(seed0: int = 2000, dx: float = 1e-4, dt: float = 1.875e-8,
                 counts=((256, 12), (384, 10), (512, 10)), c_min=1400.0, c_nom=1600.0,
                 cfl=0.3, nt_scale: float = 1.0):
    """Mixed-grid batch: per grid size N, Nt is the time for a wave at c_min to
    cross the grid diagonal (times nt_scale), Ns = N/2 ring sensors at radius
    round(55 N / 128) cells.  Each instance has its own medium and p0."""
    probs = []
    i = 0
    for n, cnt in counts:
        nt = int(math.ceil(nt_scale * math.sqrt(2.0) * n * c_nom / (cfl * c_min)))
        ring = round(55 * n / 128)
        for _ in range(cnt):
            s = seed0 + 10 * i
            c0, rho0 = medium(n, n, s, s + 1)
            p0 = blobs(n, n, s + 2, radius_cells=0.5 * ring)
            prm = make_params(n, n, dx, dt, nt, float(max(c0.max(), c_nom)),
                              ring_sensors(n // 2, ring, dx))
            probs.append(dict(params=prm, c0=c0, rho0=rho0, p0=p0))
            i += 1
    return probs


# ---------------------------------------------------------------- 3-D inputs
def smooth_noise3d(n_z: int, n_y: int, n_x: int, sigma_cells: float, seed: int) -> np.ndarray:
    """3-D white N(0,1) noise, periodically Gaussian-filtered, mean removed and
    scaled to a maximum absolute value of 1."""
    w = _rng(seed).standard_normal((n_z, n_y, n_x))
    fz = np.fft.fftfreq(n_z)[:, None, None]
    fy = np.fft.fftfreq(n_y)[None, :, None]
    fx = np.fft.fftfreq(n_x)[None, None, :]
    g = np.exp(-2.0 * (math.pi * sigma_cells) ** 2 * (fx ** 2 + fy ** 2 + fz ** 2))
    s = np.real(np.fft.ifftn(np.fft.fftn(w) * g))
    s -= s.mean()
    m = np.abs(s).max()
    return s / m if m > 0 else s


def medium3d(n_z: int, n_y: int, n_x: int, seed_c: int, seed_rho: int, *, c_range=(1390.0, 1897.0),
             rho_range=(956.0, 1252.0), sigma_cells=3.0):
    """Smooth heterogeneous 3-D medium spanning the given ranges (defaults: the
    reconstruction-grid ranges of the paper's 3-D phantom, Table 3)."""
    cm, ca = 0.5 * (c_range[0] + c_range[1]), 0.5 * (c_range[1] - c_range[0])
    rm, ra = 0.5 * (rho_range[0] + rho_range[1]), 0.5 * (rho_range[1] - rho_range[0])
    c0 = cm + ca * smooth_noise3d(n_z, n_y, n_x, sigma_cells, seed_c)
    rho0 = rm + ra * smooth_noise3d(n_z, n_y, n_x, sigma_cells, seed_rho)
    return c0, rho0


def blobs3d(n_z: int, n_y: int, n_x: int, seed: int, *, count=5, radius_cells=None,
            sigma_range=(1.5, 3.0), amp_range=(0.0, 1.0)) -> np.ndarray:
    """Initial pressure: `count` Gaussian blobs with centres drawn uniformly in a
    ball about the centre node."""
    rng = _rng(seed)
    if radius_cells is None:
        radius_cells = 0.2 * min(n_x, n_y, n_z)
    zz, yy, xx = np.mgrid[0:n_z, 0:n_y, 0:n_x].astype(np.float64)
    out = np.zeros((n_z, n_y, n_x))
    for _ in range(count):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        r = radius_cells * rng.uniform() ** (1.0 / 3.0)
        cx, cy, cz = n_x / 2 + r * d[0], n_y / 2 + r * d[1], n_z / 2 + r * d[2]
        sg = rng.uniform(*sigma_range)
        a = rng.uniform(*amp_range)
        out += a * np.exp(-((xx - cx) ** 2 + (yy - cy) ** 2 + (zz - cz) ** 2) / (2.0 * sg * sg))
    return out


def face_sensors(n: int, lo: int, d: float, n_grid: int) -> np.ndarray:
    """Detectors at the nodes of two adjacent faces (x = lo and y = lo) of the
    n x n x n block of nodes lo .. lo+n-1 of an n_grid^3 grid, the shared edge
    once: 2 n^2 - n detectors (2145 for n = 33, as in the paper's 3-D
    reconstruction).  Returns [ns, 3] positions (x, y, z) in metres, node i at
    (i - n_grid/2) d."""
    idx = np.arange(lo, lo + n)
    pos = lambda i: (i - n_grid / 2) * d
    pts = [(pos(lo), pos(j), pos(k)) for k in idx for j in idx]
    pts += [(pos(i), pos(lo), pos(k)) for k in idx for i in idx if i != lo]
    return np.asarray(pts, dtype=np.float64)


def make_params3d(nx, ny, nz, dx, dt, nt, c_ref, sensor_xyz, *, dy=None, dz=None, pml_size=8,
                  pml_alpha=2.0, alpha0_db=0.75, y=1.5) -> dict:
    return dict(nx=int(nx), ny=int(ny), nz=int(nz), dx=float(dx), dy=float(dx if dy is None else dy),
                dz=float(dx if dz is None else dz), dt=float(dt), nt=int(nt), c_ref=float(c_ref),
                pml_size=int(pml_size), pml_alpha=float(pml_alpha), alpha0_db=float(alpha0_db), y=float(y),
                sensor_xyz=np.ascontiguousarray(sensor_xyz, dtype=np.float64))


def config3d(name: str = "vol33", *, seeds=(3300, 3301, 3302), cfl=0.3) -> dict:
    """The 3-D reconstruction workload of the paper (Section 6.2): a 33^3 node
    domain of spacing 0.3125 mm with an 8-cell PML added on every side (a 49^3
    grid), Nt = 292, detectors at the 2145 nodes of two adjacent domain faces,
    tissue absorption alpha0 = 0.75 dB MHz^-1.5 cm^-1, y = 1.5, a smooth
    medium spanning Table 3's reconstruction ranges and Gaussian blobs for p0.
    "vol37" is the data-generation grid: 37^3 nodes of 0.278 mm (53^3 with the
    PML) with the same physical detector positions, off its nodes."""
    if name == "vol33":
        n, d = 33, 3.125e-4
    elif name == "vol37":
        n, d = 37, 2.78e-4
    else:
        raise KeyError(name)
    pml = 8
    ng = n + 2 * pml
    sc, sr, sp = seeds
    c0, rho0 = medium3d(ng, ng, ng, sc, sr, sigma_cells=3.0 * ng / 49)
    p0 = blobs3d(ng, ng, ng, sp, radius_cells=0.25 * n, sigma_range=(1.5 * ng / 49, 3.0 * ng / 49))
    cmax = float(c0.max())
    sens = face_sensors(33, 8, 3.125e-4, 49)
    prm = make_params3d(ng, ng, ng, d, cfl * d / cmax, 292, cmax, sens, pml_size=pml)
    return dict(params=prm, c0=c0, rho0=rho0, p0=p0)
