"""Pins of the 3-D oracle (oracle/kspace3d.py) against what the paper and the
mathematics fix: the exact homogeneous solution of the k-space scheme (d = 3
source split), the free-space Green's function of a Gaussian, the adjoint
identity, reduction to the (separately pinned) 2-D oracle for a z-invariant
problem, invariance under a permutation of the axes, the discrete energy of
the lossless scheme, and the 3-D stability bound."""
import math

import numpy as np
import pytest
from scipy import fft as sfft

import qpat_inputs as qi
from oracle import kspace as K2
from oracle import kspace3d as K3


def homog(nz, ny, nx, c=1500.0, rho=1000.0):
    return np.full((nz, ny, nx), c), np.full((nz, ny, nx), rho)


def off_node_sensors(nz, ny, nx, d, count, seed):
    rng = np.random.default_rng(seed)
    lo = np.array([1.0, 1.0, 1.0])
    hi = np.array([nx - 2.0, ny - 2.0, nz - 2.0])
    u = lo + (hi - lo) * rng.uniform(size=(count, 3))
    return (u - np.array([nx, ny, nz]) / 2) * np.asarray(d)


def test_closed_form_homogeneous_lossless():
    """c_ref = c, no PML, no absorption: p^0 = P0/2 (each of the d = 3 density
    components gets P0 / (6 c^2) at n = -1) and p^n = F^-1[cos(c|k| n dt) F P0]."""
    nz, ny, nx = 10, 12, 16
    dx, dy, dz = 1e-4, 1.2e-4, 0.9e-4
    c = 1500.0
    c0, rho0 = homog(nz, ny, nx, c)
    rho0 = rho0 * (1.0 + 0.0)
    dt = 0.4 * dx / c
    prm = qi.make_params3d(nx, ny, nz, dx, dt, 12, c, off_node_sensors(nz, ny, nx, (dx, dy, dz), 3, 1),
                           dy=dy, dz=dz, pml_size=0, alpha0_db=0.0)
    p0 = qi.gaussian_field((nz, ny, nx), 2)
    ps = {}
    K3.forward(prm, c0, rho0, p0, record=lambda n, s: ps.__setitem__(n + 1, s["p"].copy()))
    op = K3.Operators(prm, c0, rho0)
    assert np.abs(ps[0] - p0 / 2).max() <= 1e-13
    P0 = sfft.fftn(p0)
    for m in range(1, 12):
        ref = np.real(sfft.ifftn(np.cos(c * op.K * m * dt) * P0))
        assert np.abs(ps[m] - ref).max() <= 1e-12 * np.abs(p0).max(), m


def test_green_function_of_a_gaussian():
    """Free space, homogeneous: a radial Gaussian g(r) spreads as
    p(r, t) = [(r - ct) g(r - ct) + (r + ct) g(r + ct)] / (2 r); the grid is
    large enough that nothing wraps within the run."""
    n, dx, c = 48, 1e-4, 1500.0
    sg = 2.5 * dx
    c0, rho0 = homog(n, n, n, c)
    dt = 0.3 * dx / c
    nt = 21
    sens = np.array([[4 * dx, 0.0, 0.0], [3 * dx, 4 * dx, 0.0], [2 * dx, -2 * dx, 5 * dx], [0.5 * dx, 7 * dx, 1 * dx]])
    prm = qi.make_params3d(n, n, n, dx, dt, nt, c, sens, pml_size=0, alpha0_db=0.0)
    g = lambda s: np.exp(-s * s / (2 * sg * sg))
    zz, yy, xx = (np.mgrid[0:n, 0:n, 0:n] - n / 2) * dx
    p0 = g(np.sqrt(xx ** 2 + yy ** 2 + zz ** 2))
    ps = {}
    K3.forward(prm, c0, rho0, p0, record=lambda k, s: ps.__setitem__(k + 1, s["p"].copy()))
    for m in (5, 12, 20):
        t = m * dt
        for (x, y, z) in sens[:3]:     # on-node sensors: compare the node value
            i, j, k = [int(round(v / dx + n / 2)) for v in (x, y, z)]
            r = math.sqrt(x * x + y * y + z * z)
            ref = ((r - c * t) * g(r - c * t) + (r + c * t) * g(r + c * t)) / (2 * r)
            assert abs(ps[m][k, j, i] - ref) <= 1e-8, (m, x, y, z)


@pytest.mark.parametrize("alpha0_db", [0.75, 0.0])
def test_adjoint_identity(alpha0_db):
    nz, ny, nx = 8, 10, 12
    dx = 1e-4
    c0, rho0 = qi.medium3d(nz, ny, nx, 11, 12, sigma_cells=2.0)
    prm = qi.make_params3d(nx, ny, nz, dx, 0.3 * dx / c0.max(), 15, c0.max(),
                           off_node_sensors(nz, ny, nx, (dx, dx, 1.3 * dx), 7, 3), dz=1.3 * dx, pml_size=2,
                           alpha0_db=alpha0_db)
    op = K3.Operators(prm, c0, rho0)
    x = qi.gaussian_field((nz, ny, nx), 4)
    yv = qi.gaussian_field((15, 7), 5)
    hx = K3.forward(prm, c0, rho0, x, ops=op)
    hty = K3.adjoint(prm, c0, rho0, yv, ops=op)
    lhs, rhs = float(np.sum(hx * yv)), float(np.sum(x * hty))
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(hx) * np.linalg.norm(yv)


def test_z_invariant_problem_reduces_to_2d():
    """Without a PML, a problem constant along z evolves like the 2-D one: the
    density total S gets p0 / (2 c^2) per injection in both, and every z
    derivative vanishes."""
    nz, ny, nx, dx = 4, 20, 24, 1e-4
    c2d, r2d = qi.medium(ny, nx, 21, 22, sigma_cells=3.0)
    p2d = qi.blobs(ny, nx, 23, count=3, radius_cells=4.0)
    dt = 0.3 * dx / c2d.max()
    s2 = qi.ring_sensors(6, 7.3, dx, phase=0.2)
    prm2 = qi.make_params(nx, ny, dx, dt, 30, c2d.max(), s2, pml_size=0, alpha0_db=0.75)
    s3 = np.concatenate([s2, np.full((len(s2), 1), (1 - nz / 2) * 1.7 * dx)], axis=1)
    prm3 = qi.make_params3d(nx, ny, nz, dx, dt, 30, c2d.max(), s3, dz=1.7 * dx, pml_size=0, alpha0_db=0.75)
    rep = lambda a: np.repeat(a[None], nz, axis=0)
    d2 = K2.forward(prm2, c2d, r2d, p2d)
    d3 = K3.forward(prm3, rep(c2d), rep(r2d), rep(p2d))
    assert np.abs(d3 - d2).max() <= 1e-12 * np.abs(d2).max()
    r = qi.gaussian_field(d2.shape, 24)
    g2 = K2.adjoint(prm2, c2d, r2d, r)
    g3 = K3.adjoint(prm3, rep(c2d), rep(r2d), r)
    # the 3-D adjoint spreads the 2-D gradient over the nz layers of a z-invariant
    # field: sum over z of g3 equals g2 (the sensors sample one node layer)
    assert np.abs(g3.sum(axis=0) - g2).max() <= 1e-11 * np.abs(g2).max()


def test_axis_permutation():
    """Relabelling the axes (x, y, z) -> (y, z, x) of every input permutes
    nothing in the data: lossy, PML, anisotropic spacing, off-node sensors."""
    nz, ny, nx = 8, 10, 12
    d = (1e-4, 1.1e-4, 1.3e-4)
    c0, rho0 = qi.medium3d(nz, ny, nx, 31, 32, sigma_cells=2.0)
    p0 = qi.blobs3d(nz, ny, nx, 33, count=2, radius_cells=2.0)
    dt = 0.3 * d[0] / c0.max()
    sens = off_node_sensors(nz, ny, nx, d, 5, 34)
    prm = qi.make_params3d(nx, ny, nz, d[0], dt, 14, c0.max(), sens, dy=d[1], dz=d[2], pml_size=2)
    # new axes: x' = y, y' = z, z' = x; arrays [z', y', x'] = [x, z, y]
    tr = lambda a: np.transpose(a, (2, 0, 1))
    prm_p = qi.make_params3d(ny, nz, nx, d[1], dt, 14, c0.max(), sens[:, [1, 2, 0]], dy=d[2], dz=d[0],
                             pml_size=2)
    da = K3.forward(prm, c0, rho0, p0)
    db = K3.forward(prm_p, tr(c0), tr(rho0), tr(p0))
    assert np.abs(da - db).max() <= 1e-12 * np.abs(da).max()


def test_energy_invariant_lossless():
    nz, ny, nx, dx = 12, 14, 16, 1e-4
    c0, rho0 = qi.medium3d(nz, ny, nx, 41, 42, sigma_cells=2.0, c_range=(1300, 1800), rho_range=(700, 1400))
    dt = 0.3 * dx / c0.max()
    prm = qi.make_params3d(nx, ny, nz, dx, dt, 60, c0.min(), off_node_sensors(nz, ny, nx, (dx,) * 3, 2, 5),
                           pml_size=0, alpha0_db=0.0)
    p0 = qi.blobs3d(nz, ny, nx, 43, count=2, radius_cells=2.0, amp_range=(0.5, 1.0))
    op = K3.Operators(prm, c0, rho0)
    hist = []
    K3.forward(prm, c0, rho0, p0, ops=op, record=lambda n, s: hist.append(dict(
        v=[a.copy() for a in s["v"]], p=s["p"].copy())))
    E = []
    for m in range(2, len(hist)):
        e = 0.5 * np.sum(hist[m - 1]["p"] ** 2 / (rho0 * c0 ** 2))
        for i in range(3):
            e += 0.5 * np.sum(op.rhos[i] * hist[m]["v"][i] * hist[m - 1]["v"][i])
        E.append(e)
    E = np.array(E)
    assert E[0] > 0
    assert np.abs(E - E[0]).max() <= 1e-12 * E[0]


def test_stability_bound_3d():
    """Homogeneous lossless: just inside the bound of stability_limit the run
    stays bounded, 5% outside it the highest mode grows."""
    n, dx, c = 8, 1e-4, 1500.0
    c0, rho0 = homog(n, n, n, c)
    c_ref = 0.8 * c
    lim = K3.stability_limit(c, c_ref, dx, dx, dx)
    p0 = qi.gaussian_field((n, n, n), 6)
    out = {}
    for f in (0.98, 1.05):
        prm = qi.make_params3d(n, n, n, dx, f * lim, 400, c_ref, off_node_sensors(n, n, n, (dx,) * 3, 2, 7),
                               pml_size=0, alpha0_db=0.0)
        out[f] = np.abs(K3.forward(prm, c0, rho0, p0)).max()
    assert out[0.98] < 10 * np.abs(p0).max()
    assert out[1.05] > 1e6 * np.abs(p0).max()


def test_face_sensor_count():
    assert qi.face_sensors(33, 8, 3.125e-4, 49).shape == (2145, 3)


def _pml_factor(pos, n, L, alpha, c_ref, d, dt):
    xi = np.maximum(0.0, np.maximum(L - pos, pos - (n - 1 - L)))
    return np.exp(-alpha * (c_ref / d) * (xi / L) ** 4 * dt / 2.0)


def test_velocity_staggering_3d():
    """Where each velocity component lives (Section 3.2.1, eq grr): after the
    first two iterates v_i = -dt A_v,i grad_i^+ (P0/2) / rho_i.  For
    P0 = sin(k1 x) + sin(k2 y) + sin(k3 z) the staggered gradient is exactly
    k kappa(k) cos(k (r + d/2)), the density is the mean of the node and its
    neighbour ahead along the axis, and the PML factor is taken at i + 1/2.
    The expected fields are computed here from those statements, so a swap of
    the +/- shifts, a wrong staggering axis or node-placed velocity PML fails."""
    nz, ny, nx = 14, 18, 20
    dx, dy, dz, c = 1e-4, 1.3e-4, 0.8e-4, 1500.0
    dt = 0.3 * dz / c
    zz, yy, xx = np.mgrid[0:nz, 0:ny, 0:nx].astype(float)
    rho0 = (1000.0 + 120.0 * np.sin(2 * np.pi * xx / nx + 0.3) + 80.0 * np.cos(2 * np.pi * yy / ny)
            + 60.0 * np.sin(2 * np.pi * 2 * zz / nz + 1.0))
    c0 = np.full((nz, ny, nx), c)
    L, alpha = 3, 2.0
    prm = qi.make_params3d(nx, ny, nz, dx, dt, 3, c, off_node_sensors(nz, ny, nx, (dx, dy, dz), 2, 7),
                           dy=dy, dz=dz, pml_size=L, pml_alpha=alpha, alpha0_db=0.0)
    x, y, z = (xx - nx / 2) * dx, (yy - ny / 2) * dy, (zz - nz / 2) * dz
    ks = (2 * np.pi * 3 / (nx * dx), 2 * np.pi * 2 / (ny * dy), 2 * np.pi * 1 / (nz * dz))
    p0 = np.sin(ks[0] * x) + np.sin(ks[1] * y) + np.sin(ks[2] * z)
    rec = {}
    K3.forward(prm, c0, rho0, p0, record=lambda n, s: rec.__setitem__(n, [v.copy() for v in s["v"]]))
    kap = lambda k: math.sin(c * k * dt / 2) / (c * k * dt / 2)
    for i, (r, d, n, axis, shape) in enumerate(((x, dx, nx, 2, (1, 1, nx)), (y, dy, ny, 1, (1, ny, 1)),
                                                (z, dz, nz, 0, (nz, 1, 1)))):
        k = ks[i]
        g = 0.5 * k * kap(k) * np.cos(k * (r + d / 2))
        rho_half = 0.5 * (rho0 + np.roll(rho0, -1, axis=axis))
        av = _pml_factor(np.arange(n) + 0.5, n, L, alpha, c, d, dt).reshape(shape)
        want = -dt * av * g / rho_half
        assert np.abs(rec[-1][i]).max() == 0.0
        assert np.abs(rec[0][i] - want).max() <= 1e-12 * np.abs(want).max(), i


def test_offnode_trilinear_measurement():
    """M at sensors between nodes (eq num-m read as trilinear interpolation):
    trilinear interpolation reproduces every field spanned by 1, x, y, z, xy,
    yz, xz, xyz, so M applied to node values returns the field at the sensor.
    Fractions far from any node and three different spacings make swapped
    axis weights fail."""
    nz, ny, nx = 9, 11, 13
    dx, dy, dz = 1e-4, 1.4e-4, 0.7e-4
    frac = [(3.3, 2.7, 1.25), (10.25, 8.85, 6.6), (0.7, 0.3, 0.15), (11.85, 9.25, 7.9), (6.5, 5.1, 4.35)]
    pos = np.array([[(u - nx / 2) * dx, (v - ny / 2) * dy, (w - nz / 2) * dz] for u, v, w in frac])
    prm = qi.make_params3d(nx, ny, nz, dx, 1e-8, 2, 1500.0, pos, dy=dy, dz=dz, pml_size=0)
    c0, rho0 = homog(nz, ny, nx)
    op = K3.Operators(prm, c0, rho0)
    zz, yy, xx = np.mgrid[0:nz, 0:ny, 0:nx].astype(float)
    X, Y, Z = (xx - nx / 2) * dx, (yy - ny / 2) * dy, (zz - nz / 2) * dz
    f = lambda x, y, z: (0.4 - 2e3 * x + 3e3 * y + 5e3 * z + 2e7 * x * y - 3e7 * y * z + 4e7 * x * z
                         + 6e10 * x * y * z)
    got = op.measure(f(X, Y, Z))
    want = f(pos[:, 0], pos[:, 1], pos[:, 2])
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
