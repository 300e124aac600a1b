"""GPU (FP32 HIP) vs FP64 3-D oracle (oracle/kspace3d.py), through the C ABI.

Bar: relative L2 <= 1e-4 on sensor data and adjoint gradients; bitwise
equality where the same arithmetic is replayed (batching, launch shape,
graph replay).  Grids cover the radices 2, 3, 4, 5, 7, 8, the direct-DFT
stage of larger primes (11, 13, 37, 53), odd and even axes, ragged row and
column tiles, lossy and lossless media, and the paper's 3-D workload at full
size (49^3 = 33^3 plus an 8-cell PML, Nt = 292, 2145 face detectors)."""
import numpy as np
import pytest

import qpat_inputs as qi
from oracle import kspace3d as K3

pytestmark = pytest.mark.gpu

TOL = 1e-4


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1810_11685_amd as q
    return q


def T(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float32, device="cuda")


def N(t):
    return t.detach().double().cpu().numpy()


def problem(nx, ny, nz, nt, *, seed=1, alpha0_db=0.75, y=1.5, pml=2, ns=9, dz_f=1.2):
    c0, rho0 = qi.medium3d(nz, ny, nx, seed, seed + 1, sigma_cells=2.0)
    dx = 1e-4
    rng = np.random.default_rng(seed + 5)
    dims = np.array([nx, ny, nz], float)
    sens = (1.0 + (dims - 3.0) * rng.uniform(size=(ns, 3)) - dims / 2) * np.array([dx, dx, dz_f * dx])
    prm = qi.make_params3d(nx, ny, nz, dx, 0.3 * dx / c0.max(), nt, c0.max(), sens, dz=dz_f * dx,
                           pml_size=pml, alpha0_db=alpha0_db, y=y)
    p0 = qi.blobs3d(nz, ny, nx, seed + 2, count=3, radius_cells=0.2 * min(nx, ny, nz))
    return prm, c0, rho0, p0


@pytest.mark.parametrize("shape", [(16, 12, 10), (11, 14, 9), (49, 20, 15), (37, 13, 8)])
@pytest.mark.parametrize("op", ["dx+", "dx-", "dy+", "dy-", "dz+", "dz-", "ydis", "yabs"])
def test_apply_spectral_operator_3d(q, shape, op):
    nx, ny, nz = shape
    prm, c0, rho0, _ = problem(nx, ny, nz, 4)
    plan = q.Plan3D(prm, c0, rho0)
    f = qi.gaussian_field((2, nz, ny, nx), 7)
    got = N(plan.apply(op, T(f)))
    o = K3.Operators(prm, c0, rho0)
    m = {"dx+": o.mp[0], "dx-": o.mm[0], "dy+": o.mp[1], "dy-": o.mm[1], "dz+": o.mp[2], "dz-": o.mm[2],
         "ydis": o.ldis, "yabs": o.labs}[op]
    for b in range(2):
        assert rel(got[b], o.spectral(m, f[b])) <= 2e-6


CASES = [
    # nx, ny, nz, nt, alpha0_db, y, pml, tiles
    (16, 12, 10, 40, 0.75, 1.5, 3, None),
    (11, 14, 9, 30, 0.5, 1.3, 2, (4, 2, 64, 128)),     # prime 11 (direct DFT stage), odd axes, ragged tiles
    (13, 7, 10, 30, 0.0, 1.5, 2, (6, 3)),     # lossless, prime 13 and 7
    (24, 20, 18, 40, 0.75, 1.5, 4, (16, 5)),
    (10, 15, 6, 25, 2.0, 1.5, 2, (2, 4)),      # radix 5
    (10, 49, 49, 8, 0.75, 1.5, 4, None),       # compile-time 49-point plane passes, runtime-plan rows
    (9, 53, 53, 6, 0.75, 1.5, 4, None),        # compile-time 53-point plane passes, runtime-plan rows
    (49, 12, 10, 8, 0.75, 1.5, 3, None),       # compile-time 49-point rows, runtime-plan planes
    (53, 10, 9, 8, 0.75, 1.5, 3, None),        # compile-time 53-point rows, runtime-plan planes
]


@pytest.mark.parametrize("nx,ny,nz,nt,a0,y,pml,tiles", CASES)
def test_forward_adjoint_parity_3d(q, nx, ny, nz, nt, a0, y, pml, tiles):
    prm, c0, rho0, p0 = problem(nx, ny, nz, nt, alpha0_db=a0, y=y, pml=pml)
    plan = q.Plan3D(prm, c0, rho0)
    if tiles:
        plan.set_tiles(*tiles)
    ops = K3.Operators(prm, c0, rho0)
    x = np.stack([p0, qi.gaussian_field(p0.shape, 11)])
    d = N(plan.forward(T(x)))
    r = qi.gaussian_field((2, nt, prm["sensor_xyz"].shape[0]), 12)
    g = N(plan.adjoint(T(r)))
    for b in range(2):
        assert rel(d[b], K3.forward(prm, c0, rho0, x[b], ops=ops)) <= TOL
        assert rel(g[b], K3.adjoint(prm, c0, rho0, r[b], ops=ops)) <= TOL


@pytest.mark.parametrize("kind", ["data", "adjoint"])
def test_full_size_vol33_prefix(q, kind):
    """The paper's 3-D reconstruction workload (49^3 with the PML, Nt = 292,
    2145 detectors) in the launch shape the benchmark uses: the first K + 1
    samples of the data of a random p0, and the gradient of a residual
    supported on the first K + 1 samples, against the oracle's K + 1 sample
    run."""
    cfg = qi.config3d("vol33")
    prm, c0, rho0 = cfg["params"], cfg["c0"], cfg["rho0"]
    plan = q.Plan3D(prm, c0, rho0)
    Kp = 30
    short = dict(prm, nt=Kp + 1)
    ops = K3.Operators(short, c0, rho0)
    ns = prm["sensor_xyz"].shape[0]
    if kind == "data":
        x = qi.gaussian_field((49, 49, 49), 3301)
        d = N(plan.forward(T(x)))
        assert d.shape == (292, ns)
        assert rel(d[:Kp + 1], K3.forward(short, c0, rho0, x, ops=ops)) <= TOL
    else:
        r = np.zeros((292, ns))
        r[:Kp + 1] = qi.gaussian_field((Kp + 1, ns), 3302)
        assert rel(N(plan.adjoint(T(r))), K3.adjoint(short, c0, rho0, r[:Kp + 1], ops=ops)) <= TOL


def test_full_length_vol33(q):
    """The paper's 3-D reconstruction workload in full (49^3, Nt = 292, 2145
    detectors; Definition 4, Lemma 2) in the benchmark's launch (automatic
    shape, hipGraph replay on a non-default stream): data of the workload's
    blobs over all 292 samples, once the wave has crossed to the detector
    faces, and the gradient of 0.5 ||H_a p0 - d||^2 for data d of other
    blobs, against the oracle."""
    import torch
    cfg = qi.config3d("vol33")
    prm, c0, rho0, p0 = cfg["params"], cfg["c0"], cfg["rho0"], cfg["p0"]
    ops = K3.Operators(prm, c0, rho0)
    d_ref = K3.forward(prm, c0, rho0, p0, ops=ops)
    p1 = qi.blobs3d(49, 49, 49, 3310, radius_cells=0.25 * 33, sigma_range=(1.5, 3.0))
    dobs = K3.forward(prm, c0, rho0, p1, ops=ops)
    g_ref = K3.adjoint(prm, c0, rho0, d_ref - dobs, ops=ops)
    plan = q.Plan3D(prm, c0, rho0)
    plan.set_graph(True)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for rep in range(2):
            d = plan.forward(T(p0))
            g = plan.adjoint(d - T(dobs))
            s.synchronize()
            assert rel(N(d), d_ref) <= TOL
            assert rel(N(g), g_ref) <= TOL
    plan.set_graph(False)


def test_vol37_generation_grid_prime_axes(q):
    """53^3 (37^3 plus the PML; 53 is prime, a direct DFT stage): a short
    prefix of the data against the oracle."""
    cfg = qi.config3d("vol37")
    prm, c0, rho0 = cfg["params"], cfg["c0"], cfg["rho0"]
    short = dict(prm, nt=12)
    plan = q.Plan3D(short, c0, rho0)
    x = qi.gaussian_field((53, 53, 53), 3701)
    assert rel(N(plan.forward(T(x))), K3.forward(short, c0, rho0, x)) <= TOL


def test_batch_tiles_graph_bitwise_3d(q):
    """Batched and single calls, the automatic shape (chosen per batch size)
    and fixed shapes, and graph replays all give the same bits."""
    prm, c0, rho0, p0 = problem(18, 14, 12, 20)
    plan = q.Plan3D(prm, c0, rho0)
    # automatic shape for one vector: 168 lines in 11 blocks of 16 leave CUs
    # idle (8 lines), 3 x 10 plane blocks fit one per CU (1024 threads)
    assert plan.tiles() == (8, 1, 256, 1024)
    xs = np.stack([p0, qi.gaussian_field(p0.shape, 21), qi.gaussian_field(p0.shape, 22)])
    base = N(plan.forward(T(xs)))
    for b in range(3):
        assert np.array_equal(N(plan.forward(T(xs[b]))), base[b])
    r = qi.gaussian_field((3, 20, 9), 23)
    gbase = N(plan.adjoint(T(r)))
    for tiles in [(2, 1, 64, 64), (8, 3, 512, 1024), (14, 10, 256, 512), (64, 2, 128, 256)]:
        plan.set_tiles(*tiles)
        assert plan.tiles() == tiles
        assert np.array_equal(N(plan.forward(T(xs))), base), tiles
        assert np.array_equal(N(plan.adjoint(T(r))), gbase), tiles
    import torch
    plan.set_graph(True)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for _ in range(3):
            d = plan.forward(T(xs), stream=s)
            g = plan.adjoint(T(r), stream=s)
            s.synchronize()
            assert np.array_equal(N(d), base)
            assert np.array_equal(N(g), gbase)


def test_jtjv_and_adjoint_identity_3d(q):
    prm, c0, rho0, _ = problem(12, 10, 14, 25, seed=31)
    plan = q.Plan3D(prm, c0, rho0)
    x = qi.gaussian_field((2, 14, 10, 12), 32)
    hx = N(plan.forward(T(x)))
    yv = qi.gaussian_field(hx.shape, 33)
    hty = N(plan.adjoint(T(yv)))
    for b in range(2):
        lhs, rhs = np.sum(hx[b] * yv[b]), np.sum(x[b] * hty[b])
        assert abs(lhs - rhs) <= 1e-5 * np.linalg.norm(hx[b]) * np.linalg.norm(yv[b])
    assert np.array_equal(N(plan.jtjv(T(x))), N(plan.adjoint(plan.forward(T(x)))))


@pytest.mark.parametrize("nt", [1, 2])
def test_nt_one_and_two_3d(q, nt):
    prm, c0, rho0, p0 = problem(8, 8, 8, nt, pml=1, ns=4)
    plan = q.Plan3D(prm, c0, rho0)
    assert rel(N(plan.forward(T(p0))), K3.forward(prm, c0, rho0, p0)) <= TOL
    r = qi.gaussian_field((nt, 4), 41)
    assert rel(N(plan.adjoint(T(r))), K3.adjoint(prm, c0, rho0, r)) <= TOL


def test_plane_column_tile_width_does_not_change_bits(q):
    """Plane blocks of one spectrum column and of six: same arithmetic per
    line, so the same bits (24 x 24 planes; also a different row tile and
    thread counts)."""
    prm, c0, rho0, p0 = problem(16, 24, 24, 12, ns=6)
    plan = q.Plan3D(prm, c0, rho0)
    x = T(np.stack([p0, qi.gaussian_field(p0.shape, 51)]))
    r = T(qi.gaussian_field((2, 12, 6), 52))
    plan.set_tiles(8, 1, 256, 1024)
    d1, g1 = N(plan.forward(x)), N(plan.adjoint(r))
    plan.set_tiles(8, 6, 256, 512)
    assert np.array_equal(N(plan.forward(x)), d1)
    assert np.array_equal(N(plan.adjoint(r)), g1)
    assert rel(d1[0], K3.forward(prm, c0, rho0, p0)) <= TOL


def test_batched_and_single_launches_agree_bitwise(q):
    """Four vectors in one launch and four one-vector launches give the same
    bits per vector (65 column tiles, so the launches differ in block count
    and in which XCD a tile lands on)."""
    prm, c0, rho0, p0 = problem(128, 8, 8, 10, ns=5, pml=1)
    plan = q.Plan3D(prm, c0, rho0)
    xs = np.stack([p0] + [qi.gaussian_field(p0.shape, 60 + b) for b in range(3)])
    r = qi.gaussian_field((4, 10, 5), 64)
    d4, g4 = N(plan.forward(T(xs))), N(plan.adjoint(T(r)))
    for b in range(4):
        assert np.array_equal(N(plan.forward(T(xs[b]))), d4[b])
        assert np.array_equal(N(plan.adjoint(T(r[b]))), g4[b])
    assert rel(d4[0], K3.forward(prm, c0, rho0, p0)) <= TOL
