"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test pins the oracle to something other than itself: a closed form, a
textbook solution, an exact invariant, a dense brute force assembled from the
paper's block matrices, or the paper's own numbers.  A plausible slip in the
oracle (a dropped term, a wrong sign or shift, a transposed axis, a wrong
source split or unit conversion) fails at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate, special

import qpat_inputs as qi
from oracle import kspace as K
from oracle.dense import DenseModel

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def homogeneous(n, c=1500.0, rho=1000.0, ny=None):
    ny = n if ny is None else ny
    return np.full((ny, n), c), np.full((ny, n), rho)


def node_sensors(nodes, n, dx, ny=None):
    """Sensors exactly on nodes (i, j) -> metres (x_i = (i - n/2) dx)."""
    ny = n if ny is None else ny
    return np.array([[(i - n / 2) * dx, (j - ny / 2) * dx] for i, j in nodes], dtype=float)


def kgrid(nx, ny, dx, dy):
    kx = 2 * np.pi * np.fft.fftfreq(nx, dx)
    ky = 2 * np.pi * np.fft.fftfreq(ny, dy)
    KX, KY = np.meshgrid(kx, ky)
    return KX, KY


# ----------------------------------------------------------------------------
# P1: exact periodic closed form (homogeneous, lossless, no PML, c_ref = c).
# With sinc(c k dt/2) the k-space step gives p^{n+1} + p^{n-1} = 2 cos(c|k|dt) p^n
# per mode; the two half-injections of eq s1 give p^0 = P0/2, p^1 = cos P0.
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("nx,ny,cfl", [(32, 32, 0.3), (48, 40, 0.9), (24, 36, 2.5)])
def test_p1_closed_form_cosine(nx, ny, cfl):
    c, dx = 1500.0, 1e-4
    dt = cfl * dx / c
    c0, rho0 = homogeneous(nx, c, ny=ny)
    nodes = [(3, 5), (nx // 2, ny // 2), (nx - 1, ny - 2), (7, 0)]
    prm = qi.make_params(nx, ny, dx, dt, 40, c, node_sensors(nodes, nx, dx, ny), pml_size=0,
                         alpha0_db=0.0)
    p0 = qi.gaussian_field((ny, nx), 11)
    rec = {}
    data = K.forward(prm, c0, rho0, p0, record=lambda n, s: rec.__setitem__(n + 1, s["p"].copy()))
    KX, KY = kgrid(nx, ny, dx, dx)
    th = c * np.sqrt(KX ** 2 + KY ** 2) * dt
    P0 = np.fft.fft2(p0)
    scale = np.abs(p0).max()
    for n in range(40):
        exact = 0.5 * p0 if n == 0 else np.real(np.fft.ifft2(np.cos(n * th) * P0))
        assert np.abs(rec[n] - exact).max() <= 1e-12 * scale * max(1, n)
        samp = np.array([exact[j, i] for i, j in nodes])
        assert np.abs(data[n] - samp).max() <= 1e-12 * scale * max(1, n)


# ----------------------------------------------------------------------------
# P2: 2-D free-space Green's solution for a Gaussian initial pressure.
# p(r,t) = A s^2 int_0^inf exp(-k^2 s^2/2) cos(c k t) J0(k r) k dk   (t > 0).
# Valid on the periodic grid until the first image arrives.
# ----------------------------------------------------------------------------
def test_p2_green_gaussian():
    n, c, dx = 128, 1500.0, 1e-4
    dt = 0.3 * dx / c
    sig = 4.0 * dx
    c0, rho0 = homogeneous(n, c)
    radii = [0, 10, 20, 30]
    nodes = [(n // 2 + r, n // 2) for r in radii]
    nt = 180   # c t <= 54 cells: the nearest image front (r=30) arrives after ~ (128-30-4*4) cells
    prm = qi.make_params(n, n, dx, dt, nt, c, node_sensors(nodes, n, dx), pml_size=0, alpha0_db=0.0)
    yy, xx = np.mgrid[0:n, 0:n]
    rr2 = ((xx - n // 2) ** 2 + (yy - n // 2) ** 2) * dx * dx
    p0 = np.exp(-rr2 / (2 * sig * sig))
    data = K.forward(prm, c0, rho0, p0)

    def green(r, t):
        f = lambda k: sig * sig * np.exp(-0.5 * (k * sig) ** 2) * np.cos(c * k * t) * special.j0(k * r) * k
        val, _ = integrate.quad(f, 0.0, 12.0 / sig, limit=400, epsabs=1e-14, epsrel=1e-12)
        return val

    err = 0.0
    for ni in list(range(1, nt, 7)) + [nt - 1]:
        for s, r in enumerate(radii):
            err = max(err, abs(data[ni, s] - green(r * dx, ni * dt)))
    assert err <= 1e-8
    assert abs(data[0, 0] - 0.5) <= 1e-14   # p^0 = P0 / 2 at the centre


# ----------------------------------------------------------------------------
# P3: discrete energy invariant, heterogeneous lossless medium, no PML.
# E_n = 1/2 sum p_n^2/(rho0 c^2) + 1/2 sum_i rho_i v_i^{n+1/2} v_i^{n-1/2}
# is constant for n >= 1 when (grad^+)^T = -grad^- and the medium is diagonal.
# ----------------------------------------------------------------------------
def test_p3_energy_invariant():
    nx, ny, dx = 40, 32, 1e-4
    c0, rho0 = qi.medium(ny, nx, 5, 6, sigma_cells=3.0, c_amp=300.0, rho_amp=400.0)
    dt = 0.3 * dx / c0.max()
    prm = qi.make_params(nx, ny, dx, dt, 150, c0.min(), qi.ring_sensors(4, 5.5, dx), pml_size=0,
                         alpha0_db=0.0)
    p0 = qi.blobs(ny, nx, 7, count=3, radius_cells=6, sigma_range=(1.5, 3.0), amp_range=(0.5, 1.0))
    rhox = 0.5 * (rho0 + np.roll(rho0, -1, axis=1))
    rhoy = 0.5 * (rho0 + np.roll(rho0, -1, axis=0))
    hist = []
    K.forward(prm, c0, rho0, p0, record=lambda n, s: hist.append({k: v.copy() for k, v in s.items()}))
    E = []
    for m in range(2, len(hist)):   # hist[m] holds p^{m}, v^{m-1/2}; hist[m-1] holds v^{m-3/2}
        # energy at iterate n = m-1: p^{n}, v^{n+1/2} (hist[m]), v^{n-1/2} (hist[m-1])
        p = hist[m - 1]["p"]
        e = 0.5 * np.sum(p * p / (rho0 * c0 ** 2))
        e += 0.5 * np.sum(rhox * hist[m]["vx"] * hist[m - 1]["vx"])
        e += 0.5 * np.sum(rhoy * hist[m]["vy"] * hist[m - 1]["vy"])
        E.append(e)
    E = np.array(E)
    assert E[0] > 0
    assert np.abs(E - E[0]).max() <= 1e-12 * E[0]


# ----------------------------------------------------------------------------
# P4: plane-wave evolution and power-law decay (homogeneous, lossy, no PML).
# Per Fourier mode the state (R = rho_x + rho_y, W = div v) follows a 2x2
# recursion derived from eqs num-vel, num-rho, num-p; its determinant is
# 1 + dt c^2 kappa^2 tau |k|^y, so the amplitude decays like
# exp(-alpha0 (c|k|)^y kappa^2 c t): the paper's alpha0 omega^y law (eq Twelve).
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("mode", [(3, 0), (2, 5), (7, 7)])
def test_p4_plane_wave_decay(mode):
    n, c, rho, dx = 32, 1500.0, 1000.0, 1e-4
    a0db, y = 5.0, 1.5     # stronger than tissue so the decay is large over the run
    dt = 0.3 * dx / c
    c0, rho0 = homogeneous(n, c, rho)
    nt = 120
    prm = qi.make_params(n, n, dx, dt, nt, c, qi.ring_sensors(3, 4.2, dx), pml_size=0,
                         alpha0_db=a0db, y=y)
    mx, my = mode
    yy, xx = np.mgrid[0:n, 0:n]
    p0 = np.cos(2 * np.pi * (mx * xx + my * yy) / n)
    ps = []
    K.forward(prm, c0, rho0, p0, record=lambda i, s: ps.append(np.fft.fft2(s["p"])[my, mx]))
    kv = 2 * np.pi * math.hypot(mx, my) / (n * dx)
    kap = math.sin(c * kv * dt / 2) / (c * kv * dt / 2)
    # independent unit conversion: 1 Np = 20 log10(e) dB, 1 cm^-1 = 100 m^-1
    a0 = a0db * 100 / (20 * math.log10(math.e)) / (2 * math.pi * 1e6) ** y
    tau = -2 * a0 * c ** (y - 1)
    eta = 2 * a0 * c ** y * math.tan(math.pi * y / 2)
    beta = dt * kv * kv * kap * kap / rho
    a = c * c * (1 - eta * kv ** (y - 1))
    b = c * c * tau * kv ** (y - 2) * rho
    P0 = np.fft.fft2(p0)[my, mx]
    src = P0 / (4 * c * c)
    R, W = 0.0, 0.0
    pred = []
    for i in range(-1, nt - 1):
        Pn = a * R + b * W
        W = W + beta * Pn
        R = R - dt * rho * W + (2 * src if i in (-1, 0) else 0)
        pred.append(a * R + b * W)
    pred = np.array(pred)
    ps = np.array(ps)
    assert np.abs(ps - pred).max() <= 1e-11 * abs(P0)
    # determinant identity and the alpha0 omega^y law
    M = np.array([[1 - dt * rho * beta * a, -dt * rho * (1 + beta * b)], [beta * a, 1 + beta * b]])
    lam = np.linalg.eigvals(M)
    assert abs(abs(lam[0]) ** 2 - (1 + dt * c * c * kap * kap * tau * kv ** y)) <= 1e-13
    alpha_eff = -math.log(abs(lam[0])) / (c * dt)          # Np/m
    alpha_law = a0 * (c * kv) ** y
    # first order in the per-step decay: alpha_eff = alpha_law * kappa^2 (1 + O(dt alpha c))
    assert 0.97 * alpha_law <= alpha_eff <= 1.005 * alpha_law
    assert abs(alpha_eff / (alpha_law * kap * kap) - 1) <= 2 * alpha_law * c * dt


def test_alpha0_unit_conversion():
    # 0.75 dB MHz^-1.5 cm^-1 at 1 MHz is 0.75 dB/cm = 75 dB/m = 75/8.685889638 Np/m
    a0 = K.alpha0_np(0.75, 1.5)
    assert abs(a0 * (2 * math.pi * 1e6) ** 1.5 - 75.0 / 8.685889638065035) <= 1e-12
    tau, eta = K.tau_eta(np.array([1500.0]), 0.75, 1.5)
    assert tau[0] < 0                                   # absorption, not gain
    assert abs(eta[0] / tau[0] + 1500 * math.tan(math.pi * 0.75)) <= 1e-9 * 1500


# ----------------------------------------------------------------------------
# P5: adjoint identity for both adjoints (heterogeneous, lossy, PML, off-node
# sensors, non-square grid), and agreement of the two adjoint formulations.
# ----------------------------------------------------------------------------
def _small_problem(nx=40, ny=24, nt=50, pml=5, seed=20, alpha0_db=2.0, y=1.5):
    c0, rho0 = qi.medium(ny, nx, seed, seed + 1, sigma_cells=3.0)
    dx = 1e-4
    prm = qi.make_params(nx, ny, dx, 0.3 * dx / c0.max(), nt, c0.max(),
                         qi.ring_sensors(9, 8.3, dx, phase=0.1), pml_size=pml,
                         alpha0_db=alpha0_db, y=y)
    return prm, c0, rho0


@pytest.mark.parametrize("nx,ny,a0,y", [(40, 24, 2.0, 1.5), (24, 36, 0.5, 1.3), (32, 32, 0.0, 1.5)])
def test_p5_adjoint_identity(nx, ny, a0, y):
    prm, c0, rho0 = _small_problem(nx, ny, alpha0_db=a0, y=y)
    x = qi.gaussian_field((ny, nx), 31)
    ydat = qi.gaussian_field((prm["nt"], 9), 32)
    op = K.Operators(prm, c0, rho0)
    Hx = K.forward(prm, c0, rho0, x, ops=op)
    gA = K.adjoint(prm, c0, rho0, ydat, ops=op)
    gB = K.adjoint_paper(prm, c0, rho0, ydat, ops=op)
    lhs = np.sum(Hx * ydat)
    den = np.linalg.norm(Hx) * np.linalg.norm(ydat)
    assert abs(lhs - np.sum(x * gA)) <= 1e-12 * den
    assert abs(lhs - np.sum(x * gB)) <= 1e-12 * den
    assert np.linalg.norm(gA - gB) <= 1e-13 * np.linalg.norm(gA)


# ----------------------------------------------------------------------------
# P6: central differences of the quadratic 0.5||H p0 - d||^2 are exact.
# ----------------------------------------------------------------------------
def test_p6_quadratic_fd():
    prm, c0, rho0 = _small_problem(32, 28, nt=40)
    op = K.Operators(prm, c0, rho0)
    p0 = qi.blobs(28, 32, 3, count=3, radius_cells=5)
    d = K.forward(prm, c0, rho0, qi.blobs(28, 32, 4, count=3, radius_cells=5), ops=op)
    g = K.gradient(prm, c0, rho0, p0, d, ops=op)
    f = lambda q: 0.5 * np.sum((K.forward(prm, c0, rho0, q, ops=op) - d) ** 2)
    h = 1e-3
    for j in range(3):
        u = qi.gaussian_field(p0.shape, 100 + j)
        fd = (f(p0 + h * u) - f(p0 - h * u)) / (2 * h)
        assert abs(fd - np.sum(g * u)) <= 1e-8 * max(abs(fd), 1e-30) + 1e-14


# ----------------------------------------------------------------------------
# P7: source bookkeeping. Injecting at n=-1 only gives a response h; the
# paper's two-step split equals h plus h delayed by one step (the fact behind
# the pairwise-summed adjoint data of eq adj_data).
# ----------------------------------------------------------------------------
def test_p7_two_step_source_is_shifted_sum():
    prm, c0, rho0 = _small_problem(32, 32, nt=30)
    op = K.Operators(prm, c0, rho0)
    p0 = qi.gaussian_field((32, 32), 8)
    full = K.forward(prm, c0, rho0, p0, ops=op)
    h = K.forward(prm, c0, rho0, p0, ops=op, inject=(-1,))
    shifted = np.vstack([np.zeros((1, h.shape[1])), h[:-1]])
    assert np.abs(full - (h + shifted)).max() <= 1e-13 * np.abs(full).max()


# ----------------------------------------------------------------------------
# P8: the paper's grid (Section 6.1): x_i = (i - N/2) dx puts node 0 at -5 mm
# and node 127 at +4.92 mm; f_max = c_min / (2 dx) reproduces the quoted
# maximal frequencies (weak pin: rounding in the paper).
# ----------------------------------------------------------------------------
def test_p8_paper_grid_fixture():
    g = json.load(open(os.path.join(GOLD, "paper_grid_2d.json")))
    n = g["n_gen"]
    dx = (g["domain_max_mm"] - g["domain_min_mm"]) / (n - 1)   # 9.92/127 mm
    dx_pow = 10.0 / n                                           # 10/128 mm
    assert abs(dx - dx_pow) / dx_pow < 2e-3
    dxm = dx_pow * 1e-3
    prm = qi.make_params(n, n, dxm, 1e-8, 2, 1500.0,
                         np.array([[g["domain_min_mm"] * 1e-3, g["domain_min_mm"] * 1e-3],
                                   [(n - 1 - n / 2) * dxm, (n - 1 - n / 2) * dxm]]), pml_size=0)
    idx, w = K.sensor_taps(prm)
    assert idx[0, 0] == 0 and abs(w[0, 0] - 1.0) < 1e-12
    assert idx[1, 0] == n * n - 1 and abs(w[1, 0] - 1.0) < 1e-12
    assert abs((n - 1 - n / 2) * dx_pow - g["domain_max_mm"]) < 0.005
    f_gen = g["c_min_gen"] / (2 * dxm) / 1e6
    f_rec = g["c_min_recon"] / (2 * g["dx_recon_mm"] * 1e-3) / 1e6
    assert abs(f_gen - g["fmax_gen_MHz"]) / g["fmax_gen_MHz"] < 1e-3
    assert abs(f_rec - g["fmax_recon_MHz"]) / g["fmax_recon_MHz"] < 1e-3


# ----------------------------------------------------------------------------
# P9: D4 symmetry of the homogeneous response (radial p0 at the centre node,
# no PML, sensors at symmetric nodes, lossy).
# ----------------------------------------------------------------------------
def test_p9_symmetry():
    n, c, dx = 32, 1500.0, 1e-4
    c0, rho0 = homogeneous(n, c)
    a, b = 5, 2
    pts = [(a, b), (-a, b), (a, -b), (-a, -b), (b, a), (-b, a), (b, -a), (-b, -a)]
    nodes = [(n // 2 + u, n // 2 + v) for u, v in pts]
    prm = qi.make_params(n, n, dx, 0.3 * dx / c, 60, c, node_sensors(nodes, n, dx), pml_size=0,
                         alpha0_db=3.0, y=1.4)
    yy, xx = np.mgrid[0:n, 0:n]
    p0 = np.exp(-((xx - n // 2) ** 2 + (yy - n // 2) ** 2) / 6.0)
    d = K.forward(prm, c0, rho0, p0)
    assert np.abs(d - d[:, :1]).max() <= 1e-13 * np.abs(d).max()


# ----------------------------------------------------------------------------
# P10: continuity of the loss switch.
# ----------------------------------------------------------------------------
def test_p10_lossless_limit():
    prm, c0, rho0 = _small_problem(24, 24, nt=30, alpha0_db=0.0)
    p0 = qi.gaussian_field((24, 24), 9)
    d0 = K.forward(prm, c0, rho0, p0)
    prm2 = dict(prm, alpha0_db=1e-13)
    d1 = K.forward(prm2, c0, rho0, p0)
    assert np.abs(d1 - d0).max() <= 1e-10 * np.abs(d0).max()


# ----------------------------------------------------------------------------
# P11: dense brute force.  The FFT oracle equals the recursion built from the
# paper's block matrix T (eq Tprod), and both adjoints equal the dense
# transpose of H_a (Lemma 2).
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("nx,ny,pml,a0", [(8, 8, 2, 1.0), (10, 6, 2, 3.0), (6, 12, 0, 0.0)])
def test_p11_dense_bruteforce(nx, ny, pml, a0):
    c0, rho0 = qi.medium(ny, nx, 41, 42, sigma_cells=1.2, c_amp=200, rho_amp=300)
    dx = 1e-4
    prm = qi.make_params(nx, ny, dx, 0.3 * dx / c0.max(), 6, c0.max(),
                         qi.ring_sensors(5, min(nx, ny) / 2 - 1.3, dx, phase=0.3), pml_size=pml,
                         alpha0_db=a0, y=1.6)
    dm = DenseModel(prm, c0, rho0)
    H = dm.H()
    p0 = qi.gaussian_field((ny, nx), 43)
    r = qi.gaussian_field((6, 5), 44)
    d = K.forward(prm, c0, rho0, p0)
    Hp = (H @ p0.reshape(-1)).reshape(d.shape)
    assert np.abs(d - Hp).max() <= 1e-13 * np.abs(Hp).max()
    HT = (H.T @ r.reshape(-1)).reshape(ny, nx)
    for g in (K.adjoint(prm, c0, rho0, r), K.adjoint_paper(prm, c0, rho0, r)):
        assert np.abs(g - HT).max() <= 1e-13 * np.abs(HT).max()
    # (grad^+)^T = -grad^- (the paper's Phi^* = -Psi) as explicit matrices
    assert np.abs(dm.Gxp.T + dm.Gxm).max() <= 1e-12 * np.abs(dm.Gxm).max()
    assert np.abs(dm.Gyp.T + dm.Gym).max() <= 1e-12 * np.abs(dm.Gym).max()


# ----------------------------------------------------------------------------
# Stability bound of the k-space scheme with c_ref < c (used by validation).
# ----------------------------------------------------------------------------
def test_stability_limit_matches_oracle():
    n, c, dx = 32, 1500.0, 1e-4
    c_ref = 600.0
    lim = K.stability_limit(c, c_ref, dx, dx)
    c0, rho0 = homogeneous(n, c)
    p0 = qi.gaussian_field((n, n), 5)
    grow = {}
    for f in (0.9, 1.2):
        prm = qi.make_params(n, n, dx, f * lim, 400, c_ref, qi.ring_sensors(4, 5, dx), pml_size=0,
                             alpha0_db=0.0)
        rec = []
        K.forward(prm, c0, rho0, p0, record=lambda i, s: rec.append(np.abs(s["p"]).max()))
        grow[f] = rec[-1] / max(rec[:5])
    assert grow[0.9] < 2.0
    assert grow[1.2] > 1e3
    assert math.isinf(K.stability_limit(c, c, dx, dx))


# ----------------------------------------------------------------------------
# P12: where the velocity lives on the staggered grid (Section 3.2.1, eq grr).
# After the first two iterates the velocity is -dt A_v grad^+ (P0/2) / rho_i.
# For P0 = sin(k1 x) + sin(k2 y) the staggered gradient of eq grr is exactly
# k kappa(k) cos(k (r + d/2)): the derivative half a cell ahead.  The density
# that divides it must be the one at that half node (the mean of the two
# neighbouring nodes) and the PML factor the one at i + 1/2.  Everything
# expected below is computed here from those statements, not from the
# oracle's tables, so a consistent swap of the +/- shifts on both axes, a
# density averaged towards the wrong neighbour or a velocity PML taken at the
# nodes each fails.
# ----------------------------------------------------------------------------
def _pml_factor(pos, n, L, alpha, c_ref, d, dt):
    xi = np.maximum(0.0, np.maximum(L - pos, pos - (n - 1 - L)))
    return np.exp(-alpha * (c_ref / d) * (xi / L) ** 4 * dt / 2.0)


def test_p12_velocity_staggering():
    nx, ny, dx, dy, c = 40, 30, 1e-4, 1.3e-4, 1500.0
    dt = 0.3 * dx / c
    yy, xx = np.mgrid[0:ny, 0:nx].astype(float)
    rho0 = 1000.0 + 150.0 * np.sin(2 * np.pi * xx / nx + 0.4) + 90.0 * np.cos(2 * np.pi * 2 * yy / ny)
    c0 = np.full((ny, nx), c)
    L, alpha = 5, 2.0
    prm = qi.make_params(nx, ny, dx, dt, 4, c, qi.ring_sensors(3, 4.5, dx, dy=dy), dy=dy,
                         pml_size=L, pml_alpha=alpha, alpha0_db=0.0)
    k1 = 2 * np.pi * 3 / (nx * dx)
    k2 = 2 * np.pi * 2 / (ny * dy)
    x = (xx - nx / 2) * dx
    y = (yy - ny / 2) * dy
    p0 = np.sin(k1 * x) + np.sin(k2 * y)
    rec = {}
    K.forward(prm, c0, rho0, p0, record=lambda n, s: rec.__setitem__(n, {k: v.copy() for k, v in s.items()}))
    # iterate n = -1 starts from p = 0, so v stays 0 and p becomes P0/2
    assert np.abs(rec[-1]["vx"]).max() == 0.0 and np.abs(rec[-1]["vy"]).max() == 0.0
    assert np.abs(rec[-1]["p"] - 0.5 * p0).max() <= 1e-13
    kap = lambda k: math.sin(c * k * dt / 2) / (c * k * dt / 2)
    gx = 0.5 * k1 * kap(k1) * np.cos(k1 * (x + dx / 2))
    gy = 0.5 * k2 * kap(k2) * np.cos(k2 * (y + dy / 2))
    rho_half_x = 0.5 * (rho0 + np.roll(rho0, -1, axis=1))
    rho_half_y = 0.5 * (rho0 + np.roll(rho0, -1, axis=0))
    avx = _pml_factor(np.arange(nx) + 0.5, nx, L, alpha, c, dx, dt)[None, :]
    avy = _pml_factor(np.arange(ny) + 0.5, ny, L, alpha, c, dy, dt)[:, None]
    vx = -dt * avx * gx / rho_half_x
    vy = -dt * avy * gy / rho_half_y
    assert np.abs(rec[0]["vx"] - vx).max() <= 1e-12 * np.abs(vx).max()
    assert np.abs(rec[0]["vy"] - vy).max() <= 1e-12 * np.abs(vy).max()


# ----------------------------------------------------------------------------
# P13: the measurement operator at sensors between nodes (eq num-m, read as
# bilinear interpolation from the four surrounding nodes).  Bilinear
# interpolation reproduces every field a + b x + c y + e x y exactly, so M
# applied to its node values must return the field at the sensor.  The
# fractions 0.3 / 0.7 / 0.25 / 0.85 are far from any node, and the grid is
# non-square with dx != dy, so swapped x / y weights, weights taken from the
# wrong side or a wrong coordinate origin fail.
# ----------------------------------------------------------------------------
def test_p13_offnode_bilinear_measurement():
    nx, ny, dx, dy = 24, 18, 1e-4, 1.7e-4
    frac = [(3.3, 2.7), (10.25, 14.85), (0.7, 0.3), (22.85, 16.25), (12.5, 9.1), (5.0, 7.6)]
    pos = np.array([[(u - nx / 2) * dx, (v - ny / 2) * dy] for u, v in frac])
    prm = qi.make_params(nx, ny, dx, 1e-8, 2, 1500.0, pos, dy=dy, pml_size=0)
    op = K.Operators(prm, np.full((ny, nx), 1500.0), np.full((ny, nx), 1000.0))
    yy, xx = np.mgrid[0:ny, 0:nx].astype(float)
    X, Y = (xx - nx / 2) * dx, (yy - ny / 2) * dy
    f = lambda x, y: 0.7 - 3e3 * x + 5e3 * y + 4e7 * x * y
    got = op.measure(f(X, Y))
    want = f(pos[:, 0], pos[:, 1])
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    # M^T is the scatter with the same weights: <M g, r> = <g, M^T r>
    g = qi.gaussian_field((ny, nx), 5)
    r = np.linspace(-1.0, 2.0, len(frac))
    assert abs(np.sum(op.measure(g) * r) - np.sum(g * op.measure_T(r))) <= 1e-12 * np.abs(g).sum()
    # and the forward samples its pressure through that operator
    rec = {}
    prm2 = dict(prm, nt=3)
    d = K.forward(prm2, np.full((ny, nx), 1500.0), np.full((ny, nx), 1000.0), g,
                  record=lambda n, s: rec.__setitem__(n + 1, s["p"].copy()))
    for m in range(3):
        p = rec[m]
        i0 = np.floor(np.array(frac)[:, 0]).astype(int)
        j0 = np.floor(np.array(frac)[:, 1]).astype(int)
        fx = np.array(frac)[:, 0] - i0
        fy = np.array(frac)[:, 1] - j0
        i1 = np.minimum(i0 + 1, nx - 1)
        j1 = np.minimum(j0 + 1, ny - 1)
        want = ((1 - fy) * ((1 - fx) * p[j0, i0] + fx * p[j0, i1])
                + fy * ((1 - fx) * p[j1, i0] + fx * p[j1, i1]))
        assert np.abs(d[m] - want).max() <= 1e-12 * np.abs(p).max()
