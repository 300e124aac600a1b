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
