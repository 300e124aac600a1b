"""Parity of the batched workloads against the FP64 oracle.

* Gauss-Newton J^T J v at 1024^2, Nt = 4000, 512 ring sensors, alpha0 = 0.5,
  y = 1.3, 8 Krylov vectors: the oracle checks a 256^2 copy (4 x 4 block
  means of c0, rho0 and v; dx = 0.4 mm; Nt = 1000; ring radius 110 cells)
  run through the same batched path; at full size the batched result must
  equal the one-vector result bit for bit and the first iterates must match
  the oracle field by field.
* Uneven-grid batch (256^2 / 384^2 / 512^2 with Nt to cross the diagonal):
  each problem of a mixed batch equals its own single-plan run bit for bit,
  and the first iterates match the oracle.
"""
import math

import numpy as np
import pytest

import qpat_inputs as qi
from oracle import kspace as K

pytestmark = pytest.mark.gpu
TOL = 1e-4


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


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, float) - b) / np.linalg.norm(b))


def krylov_vectors(n, count):
    return np.stack([qi.smooth_noise(n, n, 8.0 * n / 1024, 3000 + j) for j in range(count)])


def test_gn1024_coarse_copy_matches_oracle(q):
    full = qi.config("gn1024", nt=4)
    c0 = qi.block_mean(full["c0"], 4)
    rho0 = qi.block_mean(full["rho0"], 4)
    vs = np.stack([qi.block_mean(v, 4) for v in krylov_vectors(1024, 2)])
    dx = 4e-4
    prm = qi.make_params(256, 256, dx, 0.3 * dx / c0.max(), 1000, c0.max(), qi.ring_sensors(512, 110, dx),
                         alpha0_db=0.5, y=1.3)
    plan = q.Plan(prm, c0, rho0)
    got = N(plan.jtjv(T(vs)))
    ops = K.Operators(prm, c0, rho0)
    ref = K.adjoint(prm, c0, rho0, K.forward(prm, c0, rho0, vs[1], ops=ops), ops=ops)
    assert rel(got[1], ref) <= TOL


def test_gn1024_full_size_batched(q):
    cfg = qi.config("gn1024", nt=120)           # full grid; fewer steps keep the test short
    prm = cfg["params"]
    plan = q.Plan(prm, cfg["c0"], cfg["rho0"])
    vs = T(krylov_vectors(1024, 8))
    batched = N(plan.jtjv(vs))
    assert np.array_equal(batched[5], N(plan.jtjv(vs[5])))
    Kp = 20
    d, ck = plan.forward_ckpt(vs[:2], Kp)
    zk = N(ck)[1, 1]
    short = dict(prm, nt=Kp + 1)
    rec = []
    K.forward(short, cfg["c0"], cfg["rho0"], N(vs)[1], record=lambda n, s: rec.append(s))
    for i, nm in enumerate(["vx", "vy", "rx", "ry", "p"]):
        assert rel(zk[i], rec[Kp][nm]) <= TOL, nm


def test_uneven_batch_full_nt(q):
    probs = qi.uneven_batch(counts=((256, 1), (384, 1), (512, 1)))
    plans = [q.Plan(p["params"], p["c0"], p["rho0"]) for p in probs]
    assert [p.nt for p in plans] == [1380, 2069, 2759]
    B = q.Batch(plans)
    xs = [T(p["p0"]) for p in probs]
    ds = B.forward(xs)
    gs = B.adjoint(ds)
    for pl, x, d, g, p in zip(plans, xs, ds, gs, probs):
        assert np.array_equal(N(d), N(pl.forward(x)))
        assert np.array_equal(N(g), N(pl.adjoint(d)))
        assert np.isfinite(N(d)).all()
        # first iterates against the oracle (field by field)
        Kp = 16
        _, ck = pl.forward_ckpt(x, Kp)
        short = dict(p["params"], nt=Kp + 1)
        rec = []
        K.forward(short, p["c0"], p["rho0"], p["p0"], record=lambda n, s: rec.append(s))
        zk = N(ck)[0, 1]
        for i, nm in enumerate(["vx", "vy", "rx", "ry", "p"]):
            assert rel(zk[i], rec[Kp][nm]) <= TOL, (p["params"]["nx"], nm)


def test_barrier_probe_runs_and_ends(q):
    """The persistent-launch probe: flat and hierarchical grid barriers in a
    cooperative launch and kernel boundaries in a graph all finish (bounded
    waits, no time-out) and report a positive time per exchange step."""
    for d in (0, 1, 2):
        us, timed_out = q.probe_barrier(d, 256, 256, 40, 512)
        assert not timed_out, d
        assert 0.0 < us < 1e4, (d, us)


def test_tuner_shape_bitwise_and_cache_round_trip(q, tmp_path, monkeypatch):
    """qpat_tune times forward + adjoint candidates in the plan's launch mode
    (graph replay here) and returns a valid shape whose results equal the
    default shape's bit for bit; it stores the shape in QPAT_TUNE_CACHE under
    (nx, ny, batch, lossy, graph), and a later plan with that key takes the
    stored shape without timing (a different valid shape written into the
    file is returned as is)."""
    import torch
    c0, rho0 = qi.medium(128, 128, 31, 32, sigma_cells=6.0)
    dx = 1e-4
    prm = qi.make_params(128, 128, dx, 0.3 * dx / c0.max(), 60, c0.max(), qi.ring_sensors(32, 50, dx),
                         pml_size=10)
    x = torch.as_tensor(np.stack([qi.blobs(128, 128, 33, radius_cells=20), qi.gaussian_field((128, 128), 34)]),
                        dtype=torch.float32, device="cuda")
    plan = q.Plan(prm, c0, rho0)
    d0 = plan.forward(x).cpu()
    g0 = plan.adjoint(plan.forward(x)).cpu()
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("QPAT_TUNE_CACHE", str(cache))
    plan.set_graph(True)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        shape = plan.tune(2)
        d1 = plan.forward(x)
        g1 = plan.adjoint(d1)
        s.synchronize()
    assert torch.equal(d1.cpu(), d0) and torch.equal(g1.cpu(), g0)
    lines = cache.read_text().split("\n")
    assert lines[0].split() == [str(v) for v in (128, 128, 2, 1, 1, *shape)]
    other = (4, 2, 256, 256) if shape != (4, 2, 256, 256) else (2, 1, 128, 128)
    cache.write_text(" ".join(str(v) for v in (128, 128, 2, 1, 1, *other)) + "\n")
    plan2 = q.Plan(prm, c0, rho0)
    plan2.set_graph(True)
    with torch.cuda.stream(s):
        assert plan2.tune(2) == other
        d2 = plan2.forward(x)
        s.synchronize()
    assert torch.equal(d2.cpu(), d0)
