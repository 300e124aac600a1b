"""autograd.Functions over the acoustic operator with hand-written backward
passes: p0 -> data with the adjoint solve (Lemma 2) as backward, and
(p0, c0) -> data whose sound-speed gradient recomputes the forward from
checkpoints.  Checked against the FP64 oracle's gradient and against central
differences."""
import os

import numpy as np
import pytest

import qpat_inputs as qi
from oracle import kspace as K
from oracle import medium as Mg

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


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


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, float) - b) / np.linalg.norm(b))


def test_autograd_gradient_matches_oracle(q):
    cfg = qi.config("small")
    prm, c0, rho0, p0 = cfg["params"], cfg["c0"], cfg["rho0"], cfg["p0"]
    plan = q.Plan(prm, c0, rho0)
    ops = K.Operators(prm, c0, rho0)
    d = K.forward(prm, c0, rho0, qi.blobs(128, 128, 1823, radius_cells=27.5), ops=ops)
    d = d + 0.01 * np.sqrt(np.mean(d ** 2)) * qi.gaussian_field(d.shape, 1824)
    x = T(p0).requires_grad_(True)
    data = q.acoustic(x, plan)
    loss = 0.5 * ((data.double() - T(d).double()) ** 2).sum()
    loss.backward()
    g_ref = K.gradient(prm, c0, rho0, p0, d, ops=ops)
    assert rel(x.grad.double().cpu().numpy(), g_ref) <= 1e-4


def test_autograd_512_oracle_gradient_and_fd(q):
    """512^2, Nt = 2000: the gradient of 0.5 ||A p0 - d||^2, d from other
    blobs plus 1% noise, against the FP64 oracle's gradient over the full
    run (stored by tests/golden/make_fwdadj512.py), and against central
    differences along 16 seeded smooth directions.  The loss is quadratic in
    p0, so its central difference is exact for any step h; h = 0.5 keeps the
    difference of the two losses far above their FP32 rounding.  Each
    direction is held to its own scale: |fd - <g, u>| <= 1e-3 |<g, u>|."""
    gold = np.load(os.path.join(GOLD, "fwdadj512_oracle.npz"))
    cfg = qi.config("autograd512")
    prm, c0, rho0, p0 = cfg["params"], cfg["c0"], cfg["rho0"], cfg["p0"]
    plan = q.Plan(prm, c0, rho0)
    d = T(gold["dobs"]).double()
    x = T(p0).requires_grad_(True)
    loss = 0.5 * ((q.acoustic(x, plan).double() - d) ** 2).sum()
    loss.backward()
    g = x.grad.double().cpu().numpy()
    assert rel(g, gold["grad"]) <= 1e-4

    def f(v):
        r = plan.forward(v).double() - d
        return 0.5 * float((r * r).sum())

    pn = np.linalg.norm(p0)
    h = 0.5
    for j in range(16):
        u = qi.smooth_noise(512, 512, 8.0, 1900 + j)
        u *= pn / np.linalg.norm(u)
        fd = (f(T(p0 + h * u)) - f(T(p0 - h * u))) / (2 * h)
        an = float(np.sum(g * u))
        assert abs(fd - an) <= 1e-3 * abs(an), (j, fd, an)


def test_acoustic_medium_checkpointed_gradient(q):
    """(p0, c0) -> data: the backward gives H_a^* r in p0 and d<r, H_a[c0] p0>/dc0
    through qpat_medium_grad, which recomputes the forward from checkpoints
    every K iterates.  Against the oracle's sound-speed gradient; the result
    does not depend on K (bitwise) and a batch sums the per-vector c0
    gradients."""
    import torch
    nx = ny = 64
    nt = 90
    c0, rho0 = qi.medium(ny, nx, 5, 6, sigma_cells=4.0)
    dx = 1e-4
    prm = qi.make_params(nx, ny, dx, 0.3 * dx / c0.max(), nt, c0.max(), qi.ring_sensors(16, 22.0, dx),
                         pml_size=6)
    p0 = qi.blobs(ny, nx, 7, count=3, radius_cells=10)
    r = qi.gaussian_field((nt, 16), 8)
    plan = q.Plan(prm, c0, rho0)
    ct = torch.as_tensor(c0, dtype=torch.float64, device="cuda")
    grads = []
    for k in (10, None):
        x = T(p0).requires_grad_(True)
        c = ct.clone().requires_grad_(True)
        out = q.acoustic_medium(x, c, plan, ckpt_interval=k)
        (out.double() * T(r).double()).sum().backward()
        grads.append((x.grad.double().cpu().numpy(), c.grad.cpu().numpy()))
    assert np.array_equal(grads[0][0], grads[1][0]) and np.array_equal(grads[0][1], grads[1][1])
    gc_ref, gp_ref = Mg.sound_speed_gradient(prm, c0, rho0, p0, r)
    assert rel(grads[0][0], gp_ref) <= 1e-4
    assert rel(grads[0][1], gc_ref) <= 1e-4
    # a batch of two: the c0 gradient is the sum of the two vectors' gradients
    xb = T(np.stack([p0, 0.5 * p0])).requires_grad_(True)
    c = ct.clone().requires_grad_(True)
    out = q.acoustic_medium(xb, c, plan, ckpt_interval=10)
    (out.double() * T(np.stack([r, r])).double()).sum().backward()
    assert rel(c.grad.cpu().numpy(), 1.5 * gc_ref) <= 1e-4
    with pytest.raises(ValueError):
        q.acoustic_medium(T(p0), ct + 1.0, plan)
