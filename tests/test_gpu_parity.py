"""GPU (FP32 HIP) vs FP64 oracle parity, through the C ABI.

Bar: relative L2 <= 1e-4 on sensor data and on adjoint gradients (FP32
fields against the FP64 oracle on identical seeded inputs); bitwise equality
where the same arithmetic is replayed (batching, checkpoint replay, graphs).
"""
import math
import os

import numpy as np
import pytest

import qpat_inputs as qi
from oracle import kspace as K

pytestmark = pytest.mark.gpu

TOL = 1e-4
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


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


def problem(nx, ny, nt, *, seed=1, alpha0_db=0.75, y=1.5, pml=8, ns=23, ring=None, cfl=0.3):
    c0, rho0 = qi.medium(ny, nx, seed, seed + 1, sigma_cells=max(2.0, min(nx, ny) / 16))
    dx = 1e-4
    ring = 0.38 * min(nx, ny) if ring is None else ring
    prm = qi.make_params(nx, ny, dx, cfl * dx / c0.max(), nt, c0.max(),
                         qi.ring_sensors(ns, ring, dx, phase=0.05), pml_size=pml, alpha0_db=alpha0_db, y=y)
    p0 = qi.blobs(ny, nx, seed + 2, count=4, radius_cells=0.2 * min(nx, ny))
    return prm, c0, rho0, p0


# ---------------------------------------------------------------- spectral operators
@pytest.mark.parametrize("nx,ny", [(64, 48), (96, 64), (32, 192), (128, 128)])
@pytest.mark.parametrize("op", ["dx+", "dx-", "dy+", "dy-", "ydis", "yabs"])
def test_apply_spectral_operator(q, nx, ny, op):
    prm, c0, rho0, _ = problem(nx, ny, 4)
    plan = q.Plan(prm, c0, rho0)
    f = qi.gaussian_field((3, ny, nx), 7)
    got = N(plan.apply(op, T(f)))
    o = K.Operators(prm, c0, rho0)
    m = {"dx+": o.mxp, "dx-": o.mxm, "dy+": o.myp, "dy-": o.mym, "ydis": o.ldis, "yabs": o.labs}[op]
    for b in range(3):
        assert rel(got[b], o.spectral(m, f[b])) <= 2e-6


# ---------------------------------------------------------------- forward / adjoint parity
CASES = [
    # nx, ny, nt, alpha0_db, y, pml
    (64, 64, 120, 0.75, 1.5, 8),
    (96, 64, 90, 0.5, 1.3, 6),      # radix-3 rows, non-square
    (48, 96, 100, 2.0, 1.5, 5),     # radix-3 rows and columns
    (64, 32, 80, 0.0, 1.5, 6),      # lossless
    (128, 128, 150, 0.75, 1.5, 20),
    (128, 48, 80, 0.75, 1.5, 6),    # 128-point row instance, all-length column kernel
    (48, 256, 60, 0.75, 1.5, 8),    # all-length row kernel, 256-point column instance
    (384, 256, 340, 0.75, 1.5, 10), # 384-point rows, 256-point columns (the wave reaches the ring)
]


@pytest.mark.parametrize("nx,ny,nt,a0,y,pml", CASES)
def test_forward_adjoint_parity(q, nx, ny, nt, a0, y, pml):
    prm, c0, rho0, p0 = problem(nx, ny, nt, alpha0_db=a0, y=y, pml=pml)
    plan = q.Plan(prm, c0, rho0)
    ops = K.Operators(prm, c0, rho0)
    d_ref = K.forward(prm, c0, rho0, p0, ops=ops)
    d_gpu = N(plan.forward(T(p0)))
    assert rel(d_gpu, d_ref) <= TOL
    r = qi.gaussian_field(d_ref.shape, 99)
    g_ref = K.adjoint(prm, c0, rho0, r, ops=ops)
    g_gpu = N(plan.adjoint(T(r)))
    assert rel(g_gpu, g_ref) <= TOL


def test_small_config_full(q):
    """The 128^2, Nt = 600 workload (5 blobs, 64 ring sensors) in full: data and
    the end-to-end gradient H^T (H p0 - d)."""
    cfg = qi.config("small")
    prm, c0, rho0, p0 = cfg["params"], cfg["c0"], cfg["rho0"], cfg["p0"]
    plan = q.Plan(prm, c0, rho0)
    ops = K.Operators(prm, c0, rho0)
    d_ref = K.forward(prm, c0, rho0, p0, ops=ops)
    d_gpu = N(plan.forward(T(p0)))
    assert rel(d_gpu, d_ref) <= TOL
    p1 = qi.blobs(128, 128, 1813, radius_cells=27.5)
    dobs = K.forward(prm, c0, rho0, p1, ops=ops)
    dobs = dobs + 0.01 * np.sqrt(np.mean(dobs ** 2)) * qi.gaussian_field(dobs.shape, 1814)
    g_ref = K.adjoint(prm, c0, rho0, d_ref - dobs, ops=ops)
    g_gpu = N(plan.adjoint(T(d_gpu - dobs)))
    assert rel(g_gpu, g_ref) <= TOL
    # FP32 adjoint identity
    x = qi.gaussian_field((128, 128), 5)
    yv = qi.gaussian_field(d_ref.shape, 6)
    hx = N(plan.forward(T(x)))
    hty = N(plan.adjoint(T(yv)))
    lhs, rhs = np.sum(hx * yv), np.sum(x * hty)
    assert abs(lhs - rhs) <= 1e-5 * np.linalg.norm(hx) * np.linalg.norm(yv)


def test_headline_full_length_in_bench_launch(q):
    """The headline workload in full (512^2, Nt = 2000, 256 ring sensors, lossy,
    20-cell PML; Definition 4, Lemma 2) in the launch the benchmark times: the
    launch shape picked by the tuner, hipGraph capture and replay, on a
    non-default stream.  Against the FP64 oracle's stored results
    (tests/golden/make_fwdadj512.py):
      data       H_a p0 for the workload's blobs, every sample;
      gradient   H_a^* r for the oracle's residual r = H_a p0 - dobs;
      end to end H_a^* (d_gpu - dobs), the gradient of 0.5 ||H_a p0 - dobs||^2.
    Also the default launch shape, the fixed shape (2, 1, 512, 128) and eager
    launches give the same bits."""
    import torch
    gold = np.load(os.path.join(GOLD, "fwdadj512_oracle.npz"))
    cfg = qi.config("fwdadj512")
    prm, c0, rho0, p0 = cfg["params"], cfg["c0"], cfg["rho0"], cfg["p0"]
    plan = q.Plan(prm, c0, rho0)
    default = plan.tiles()
    s = torch.cuda.Stream()
    x = T(p0)
    dobs = T(gold["dobs"])
    r_or = T(gold["data"].astype(np.float64) - gold["dobs"].astype(np.float64))
    with torch.cuda.stream(s):
        plan.set_graph(True)
        plan.tune(1)
        tuned = plan.tiles()
        outs = []
        for rep in range(2):              # the capture run, then a replay
            d = plan.forward(x)
            g1 = plan.adjoint(r_or)
            g2 = plan.adjoint(d - dobs)
            s.synchronize()
            outs.append((N(d), N(g1), N(g2)))
        plan.set_graph(False)
    print(f"headline parity: tuned shape {tuned}, default {default}")
    for d, g1, g2 in outs:
        assert d.shape == (2000, 256)
        assert rel(d, gold["data"]) <= TOL
        assert rel(g1, gold["grad"]) <= TOL
        assert rel(g2, gold["grad"]) <= TOL
    assert all(np.array_equal(a, b) for a, b in zip(outs[0], outs[1]))
    for shape in {default, (2, 1, 512, 128)}:
        plan.set_tiles(*shape)
        assert np.array_equal(N(plan.forward(x)), outs[0][0]), shape
        assert np.array_equal(N(plan.adjoint(r_or)), outs[0][1]), shape


@pytest.mark.parametrize("kind", ["fields", "data", "adjoint"])
def test_full_size_512_prefix(q, kind):
    """512^2, Nt = 2000, 256 ring sensors (the headline workload) with the
    default launch shape and eager launches.  The first K samples (and states) depend
    only on the first K iterates, and a residual supported on the first K
    samples has an adjoint equal to the K-step adjoint, so the oracle can
    check the full-size run in seconds:
      fields  - every field of the state z_K after K iterates of the blob p0;
      data    - the first K samples for a random p0 (the blob wave has not yet
                reached the ring after K steps, so its samples are roundoff);
      adjoint - the gradient for a residual on the first K samples."""
    cfg = qi.config("fwdadj512")
    prm, c0, rho0, p0 = cfg["params"], cfg["c0"], cfg["rho0"], cfg["p0"]
    plan = q.Plan(prm, c0, rho0)
    Kp = 40
    short = dict(prm, nt=Kp + 1)
    ops = K.Operators(short, c0, rho0)
    if kind == "fields":
        d_gpu, ck = plan.forward_ckpt(T(p0), Kp)
        assert np.isfinite(N(d_gpu)).all()
        zk = N(ck)[0, 1]
        rec = []
        K.forward(short, c0, rho0, p0, ops=ops, record=lambda n, s: rec.append(s))
        for i, nm in enumerate(["vx", "vy", "rx", "ry", "p"]):
            assert rel(zk[i], rec[Kp][nm]) <= TOL, nm
    elif kind == "data":
        x = qi.gaussian_field((512, 512), 77)
        d_gpu = N(plan.forward(T(x)))
        d_ref = K.forward(short, c0, rho0, x, ops=ops)
        assert rel(d_gpu[:Kp + 1], d_ref) <= TOL
    else:
        r = np.zeros((prm["nt"], 256))
        r[:Kp + 1] = qi.gaussian_field((Kp + 1, 256), 1823)
        g_gpu = N(plan.adjoint(T(r)))
        g_ref = K.adjoint(short, c0, rho0, r[:Kp + 1], ops=ops)
        assert rel(g_gpu, g_ref) <= TOL


def test_jtjv_is_adjoint_of_forward(q):
    prm, c0, rho0, p0 = problem(64, 48, 70)
    plan = q.Plan(prm, c0, rho0)
    v = T(qi.gaussian_field((2, 48, 64), 3))
    a = N(plan.jtjv(v))
    b = N(plan.adjoint(plan.forward(v)))
    assert np.array_equal(a, b)
    ops = K.Operators(prm, c0, rho0)
    ref = K.adjoint(prm, c0, rho0, K.forward(prm, c0, rho0, N(v)[1], ops=ops), ops=ops)
    assert rel(a[1], ref) <= TOL
    # qpat_jtjv_data hands back the intermediate H_a v as well: bitwise qpat_jv's and qpat_jtjv's
    jv, c = plan.jtjv_data(v)
    assert np.array_equal(N(jv), N(plan.forward(v))) and np.array_equal(N(c), a)


def test_batch_equals_single_bitwise(q):
    prm, c0, rho0, _ = problem(64, 64, 60)
    plan = q.Plan(prm, c0, rho0)
    x = T(qi.gaussian_field((5, 64, 64), 4))
    db = N(plan.forward(x))
    rb = T(qi.gaussian_field((5, 60, 23), 8))
    gb = N(plan.adjoint(rb))
    for i in range(5):
        assert np.array_equal(db[i], N(plan.forward(x[i])))
        assert np.array_equal(gb[i], N(plan.adjoint(rb[i])))


@pytest.mark.parametrize("n,a0", [(512, 0.75), (512, 0.0), (256, 0.75), (384, 0.75), (1024, 0.75)])
def test_launch_variants_bitwise_at_compiled_lengths(q, n, a0):
    """Lengths with compile-time kernel instances run different code by block
    count: about one block per CU takes global twiddles and ping-pong stages
    (at 512 the velocity passes share their FFTs' boundary stage in
    registers), several blocks per CU take LDS twiddles and in-place row
    stages.  One vector and a batch of eight (which crosses that line) must
    agree bit for bit, forward and adjoint, lossy and lossless."""
    nt = 24 if n >= 1024 else 40
    prm, c0, rho0, _ = problem(n, n, nt, alpha0_db=a0, ns=32)
    plan = q.Plan(prm, c0, rho0)
    plan.set_tiles(2, 1, 512 if n <= 512 else 256, 128 if n <= 512 else 256)
    x = T(np.stack([qi.smooth_noise(n, n, 3.0, 70 + b) for b in range(8)]))
    r = T(qi.gaussian_field((8, nt, 32), 71))
    db, gb = N(plan.forward(x)), N(plan.adjoint(r))
    for i in (0, 5):
        assert np.array_equal(db[i], N(plan.forward(x[i])))
        assert np.array_equal(gb[i], N(plan.adjoint(r[i])))


def test_tiles_do_not_change_results(q):
    prm, c0, rho0, p0 = problem(64, 64, 50)
    plan = q.Plan(prm, c0, rho0)
    base = N(plan.forward(T(p0)))
    # the per-line arithmetic does not depend on the launch shape
    for shape in [(2, 1, 64, 64), (4, 4, 128, 256), (16, 8, 256, 128), (2, 2, 256, 64), (2, 1, 512, 512),
                  (4, 4, 512, 256)]:
        plan.set_tiles(*shape)
        assert plan.tiles() == shape
        assert np.array_equal(N(plan.forward(T(p0))), base)


def test_large_lds_tiles_do_not_change_results(q):
    """1024-point lines: tiles whose LDS exceeds 64 KB (up to the 160 KB of a
    gfx950 work-group) and 512-thread blocks give the same bits."""
    prm, c0, rho0, p0 = problem(1024, 1024, 12, ns=64)
    plan = q.Plan(prm, c0, rho0)
    plan.set_tiles(2, 1, 256, 256)
    x = T(p0)
    d0 = N(plan.forward(x))
    r = T(qi.gaussian_field((12, 64), 7))
    g0 = N(plan.adjoint(r))
    for shape in [(4, 2, 512, 512), (2, 2, 256, 512), (4, 1, 512, 256)]:
        plan.set_tiles(*shape)
        assert plan.tiles() == shape
        assert np.array_equal(N(plan.forward(x)), d0)
        assert np.array_equal(N(plan.adjoint(r)), g0)


@pytest.mark.parametrize("n", [256, 512])
def test_storage_tile_heights_bitwise(q, n):
    """Spectra are stored in tiles of max(rows per row tile, 4) rows: row
    blocks of two rows write and read half of every tile, blocks of four or
    eight rows whole tiles, and the column passes read runs of four or eight
    rows.  Forward and adjoint results do not depend on it, for a batch of
    four and for one vector (about one block per CU)."""
    nt = 30
    prm, c0, rho0, _ = problem(n, n, nt, ns=32)
    plan = q.Plan(prm, c0, rho0)
    x = T(np.stack([qi.smooth_noise(n, n, 3.0, 90 + b) for b in range(4)]))
    r = T(qi.gaussian_field((4, nt, 32), 91))
    ref = None
    for shape in [(2, 1, 512, 512), (4, 1, 512, 256), (8, 2, 512, 256), (2, 2, 256, 512), (8, 1, 512, 128)]:
        plan.set_tiles(*shape)
        assert plan.tiles() == shape
        out = (N(plan.forward(x)), N(plan.adjoint(r)), N(plan.forward(x[1])), N(plan.adjoint(r[2])))
        if ref is None:
            ref = out
            assert np.array_equal(out[2], out[0][1]) and np.array_equal(out[3], out[1][2])
        else:
            assert all(np.array_equal(a, b) for a, b in zip(out, ref)), shape


def test_graph_mode_replays_match(q):
    """Captured hipGraph replays equal direct launches bit for bit, on every
    replay, with eager work and synchronisation in between."""
    import torch
    prm, c0, rho0, p0 = problem(64, 48, 40)
    plan = q.Plan(prm, c0, rho0)
    xs = [T(p0 * (k + 1)) for k in range(3)]
    refs = [(N(plan.forward(x)), N(plan.adjoint(plan.forward(x)))) for x in xs]
    plan.set_graph(True)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for rep in range(2):
            for x, (dref, gref) in zip(xs, refs):
                d = plan.forward(x)
                g = plan.adjoint(d)
                s.synchronize()
                assert np.array_equal(N(d), dref)
                assert np.array_equal(N(g), gref)
                _ = (x * 2).sum().item()     # eager work between replays
    plan.set_graph(False)


def test_checkpoint_replay_bitwise(q):
    prm, c0, rho0, p0 = problem(64, 64, 37)
    plan = q.Plan(prm, c0, rho0)
    x = T(p0)
    d0 = N(plan.forward(x))
    d1, ck1 = plan.forward_ckpt(x, 1)
    assert np.array_equal(N(d1), d0)
    Kc = 10
    d2, ck = plan.forward_ckpt(x, Kc)
    assert np.array_equal(N(d2), d0)
    assert ck.shape[1] == math.ceil(37 / Kc)
    assert plan.ckpt_bytes(Kc) == ck.numel() * 4
    allstates = N(ck1)[0]          # every state z_m, m = 0..nt-1
    for seg in range(ck.shape[1]):
        st = N(plan.replay(x, ck, Kc, seg))[0]
        assert np.array_equal(st, allstates[seg * Kc: seg * Kc + st.shape[0]])
    # the pressure of state m is the sampled field of the oracle
    hist = []
    K.forward(prm, c0, rho0, p0, record=lambda n, s: hist.append(s["p"].copy()), nsteps=37)
    assert rel(allstates[36, 4], hist[36]) <= TOL


def test_uneven_batch_matches_single(q):
    probs = []
    for (nx, nt, seed) in [(64, 50, 3), (96, 70, 5), (128, 40, 9), (64, 30, 11)]:
        prm, c0, rho0, p0 = problem(nx, nx, nt, seed=seed, ns=nx // 4)
        probs.append((q.Plan(prm, c0, rho0), p0))
    B = q.Batch([p for p, _ in probs])
    xs = [T(p0) for _, p0 in probs]
    refs = [(N(plan.forward(x)), N(plan.jtjv(x))) for (plan, _), x in zip(probs, xs)]
    # one launch set for all problems, then one launch sequence per grid size
    # on forked streams (eager and graph-replayed): the same bits
    for schedule, graph in ((0, False), (1, False), (1, True), (1, True)):
        B.set_schedule(schedule)
        B.set_graph(graph)
        assert B.schedule() == schedule
        ds = B.forward(xs)
        gs = B.jtjv(xs)
        for (dref, gref), d, g in zip(refs, ds, gs):
            assert np.array_equal(N(d), dref)
            assert np.array_equal(N(g), gref)


def test_mixed_batch_matches_fused_single_plans(q):
    """A batch mixing 256^2 and 512^2 grids launches the all-length kernels
    (runtime plans, density updates between two separate FFTs); single plans
    of those sizes launch the compile-time instances whose density passes fuse
    the FFTs' boundary stage (one row per work item, lane pairs exchanging
    their packed-line halves). The same bits."""
    probs = []
    for (nx, nt, seed) in [(256, 14, 21), (512, 10, 23)]:
        prm, c0, rho0, p0 = problem(nx, nx, nt, seed=seed, ns=nx // 8)
        probs.append((q.Plan(prm, c0, rho0), p0))
    B = q.Batch([p for p, _ in probs])
    B.set_schedule(0)
    xs = [T(p0) for _, p0 in probs]
    refs = [(N(plan.forward(x)), N(plan.jtjv(x))) for (plan, _), x in zip(probs, xs)]
    ds = B.forward(xs)
    gs = B.jtjv(xs)
    for (dref, gref), d, g in zip(refs, ds, gs):
        assert np.array_equal(N(d), dref)
        assert np.array_equal(N(g), gref)


def test_batch_of_16_at_128_matches_single_calls(q):
    """128^2 with 16 vectors per launch is a many-block launch: its density
    passes fuse the FFTs' boundary stage with two rows per work item (the
    radix-4 boundary form); one vector per launch takes the unfused passes.
    Each vector of the batch equals its single call bit for bit."""
    import torch
    prm, c0, rho0, p0 = problem(128, 128, 24, seed=31, ns=32)
    plan = q.Plan(prm, c0, rho0)
    plan.set_tiles(2, 1, 64, 64)  # 64 row blocks per vector: 16 vectors are 1024 blocks, one vector 64
    vs = torch.stack([T(p0)] + [T(qi.gaussian_field((128, 128), 40 + j)) for j in range(15)])
    d16, g16 = N(plan.forward(vs)), N(plan.jtjv(vs))
    for j in (0, 7, 15):
        assert np.array_equal(N(plan.forward(vs[j])), d16[j])
        assert np.array_equal(N(plan.jtjv(vs[j])), g16[j])


def test_uneven_batch_tuner(q):
    """qpat_batch_tune picks launch shapes per grid size and a schedule; the
    results stay those of the single plans."""
    import torch
    probs = []
    for (nx, nt, seed) in [(64, 50, 3), (128, 40, 9), (64, 30, 11), (128, 60, 13)]:
        prm, c0, rho0, p0 = problem(nx, nx, nt, seed=seed, ns=nx // 4)
        probs.append((q.Plan(prm, c0, rho0), p0))
    xs = [T(p0) for _, p0 in probs]
    refs = [N(plan.jtjv(x)) for (plan, _), x in zip(probs, xs)]
    B = q.Batch([p for p, _ in probs])
    B.set_graph(True)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        sched = B.tune()
        gs = B.jtjv(xs)
        s.synchronize()
    assert sched in (0, 1)
    for ref, g in zip(refs, gs):
        assert np.array_equal(N(g), ref)


def test_dot_fp64_accumulation(q):
    import torch
    a = qi.gaussian_field(1_000_003, 1)
    b = qi.gaussian_field(1_000_003, 2)
    got = float(q.dot(T(a), T(b)).cpu())
    ref = float(np.dot(a.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)))
    assert abs(got - ref) <= 1e-12 * np.sqrt(np.dot(a, a) * np.dot(b, b))
    z = torch.zeros(0, device="cuda")
    assert float(q.dot(z, z).cpu()) == 0.0


def test_nt_one_and_two(q):
    for nt in (1, 2):
        prm, c0, rho0, p0 = problem(32, 32, nt, pml=4, ns=5)
        plan = q.Plan(prm, c0, rho0)
        ops = K.Operators(prm, c0, rho0)
        assert rel(N(plan.forward(T(p0))), K.forward(prm, c0, rho0, p0, ops=ops)) <= TOL
        r = qi.gaussian_field((nt, 5), 3)
        assert rel(N(plan.adjoint(T(r))), K.adjoint(prm, c0, rho0, r, ops=ops)) <= TOL


def test_output_check_flags_nonfinite(q):
    """Opt-in failure detection: with the check on, a solve whose output holds
    NaN / Inf (here from a NaN in p0, or in the residual) is reported by the
    next check, which then clears the flag; clean solves report nothing."""
    prm, c0, rho0, p0 = problem(64, 48, 40)
    plan = q.Plan(prm, c0, rho0)
    plan.set_check(True)
    x = T(p0)
    d = plan.forward(x)
    plan.adjoint(d)
    assert plan.outputs_finite()
    bad = p0.copy()
    bad[20, 30] = np.nan
    plan.forward(T(bad))
    assert not plan.outputs_finite()
    assert plan.outputs_finite()          # cleared by the read
    r = N(d)
    r[5, 3] = np.inf
    plan.adjoint(T(r))
    assert not plan.outputs_finite()
    plan.set_check(False)
    plan.forward(T(bad))
    assert plan.outputs_finite()          # not checked
