#!/usr/bin/env python3
"""Benchmark of the FP32 k-space acoustic forward + adjoint on one MI355X.

Headline: grid-point-steps/s of one forward solve H_a p0 plus one adjoint
solve H_a^* r on the 512 x 512, Nt = 2000, 256-ring-sensor workload (lossy,
alpha0 = 0.75 dB MHz^-1.5 cm^-1, y = 1.5, 20-cell PML).  One benchmark step is
that forward + adjoint pair; value = 2 * 512^2 * 2000 / step time, with inputs
resident in HBM.

Also reported on the same JSON line:
  roofline      - the kernel with the largest share of the step: algorithmic
                  bytes per launch (the scope table's per-point figure times
                  the grid points of one launch) / its mean launch time (HIP
                  events, live, on the stream it runs on), against 8 TB/s HBM;
  cpu_baseline  - the FP64 oracle on the host cores, on a bounded sample;
  batched       - Gauss-Newton J^T J v on 8 Krylov vectors at 1024^2, Nt = 4000
                  (alpha0 = 0.5, y = 1.3): one batched call vs 8 plain calls;
  uneven        - 32 J^T J v products over 256^2 / 384^2 / 512^2 grids in one
                  batched call vs one call per problem.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "grid-point-steps/s fwd+adjoint (512², FP32) and batched J^TJv/s vs plain"
HBM_PEAK_GBS = 8000.0
REPEATS = 5          # timed runs of each batched / uneven measurement (median reported)

# Algorithmic HBM bytes per grid point moved by one launch of each pass kind
# (FP32 fields 4 B/pt; a half spectrum [ny][nx/2] of complex64 is 4 B/pt; the
# [ny][nx/2+1] multiplier tables ~2 B/pt each).  Sum: 160 B/pt per forward
# iterate and 160 B/pt per adjoint iterate.
PASS_BYTES = {
    0: 4 + 8 + 2,            # col grad p: spec p in, 2 spectra out, kappa
    1: 8 + 8 + 8 + 8 + 8,    # row velocity: 2 spectra in, v in, dt/rho_i, v out, 2 spectra out
    2: 8 + 8 + 2,            # col div v
    3: 8 + 8 + 4 + 8 + 8,    # row density: 2 spectra, rho in, rho0, rho out, 2 spectra out
    4: 8 + 8 + 4,            # col Y_dis, Y_abs: 2 in, 2 out, two tables
    5: 8 + 8 + 12 + 4,       # row pressure: 2 spectra, rho in, c^2, c^2 eta, c^2 tau, spec p out
    6: 4 + 12 + 4 + 8,       # adj row: spec p* in, c^2 c^2eta c^2tau, q out, 2 spectra out
    7: 8 + 8 + 4,            # adj col Y
    8: 8 + 4 + 8 + 4 + 8 + 8,  # adj row density: 2 spectra, q, rho* in, rho0, rho* out, 2 spectra out
    9: 8 + 8 + 2,            # adj col grad
    10: 8 + 8 + 8 + 8 + 8,   # adj row velocity
    11: 8 + 4 + 2,           # adj col div: 2 in, 1 out, kappa
}


# The same per grid point as the scope table of the hot path counts them
# (fields and half spectra only, no multiplier tables): 152 B per forward
# iterate.  Each adjoint pass is the transpose of one forward pass and is
# given that pass's count (152 B per adjoint iterate).  These are the bytes
# the roofline line uses.
SCOPE_BYTES = {0: 12, 1: 40, 2: 16, 3: 36, 4: 16, 5: 32,
               6: 32, 7: 16, 8: 36, 9: 16, 10: 40, 11: 12}
# Passes served by one kernel (the fractional-Laplacian column pass is the
# same kernel forward and adjoint); every other pass has a kernel of its own.
KERNEL_OF_PASS = {4: "col_fraclap", 7: "col_fraclap"}


# Algorithmic HBM bytes per FEM node of one conjugate-gradient iteration of
# the optical solve (FP64).  CG: A p reads p and the two elemental
# coefficients of the pixel it owns (8 + 32) and writes q (8); the update
# reads x, p, r, q (32) and writes x, r (16); r.z reads r, z (16); the new
# direction reads z, p (16) and writes p (8).  V-cycle, per node of a level
# (the first sweep's x = om dinv b is recomputed, not stored): the
# restriction reads b, the inverse diagonal and the 4-array stencil (48) and
# writes a quarter of a coarse value (2); correction and post-sweep read the
# same (48) and a quarter of a coarse value (2) and write t (8).  The levels
# add up to 4/3 of the fine grid's nodes.
OPT_CG_BYTES = 48.0 + 48.0 + 16.0 + 24.0
OPT_VCYCLE_BYTES = (50.0 + 58.0) * 4.0 / 3.0
OPT_BYTES_PER_NODE_ITER = OPT_CG_BYTES + OPT_VCYCLE_BYTES


def bytes_3d_pair(nx: int) -> float:
    """Algorithmic HBM bytes per grid point of one lossy 3-D forward + adjoint
    iterate pair.  A half spectrum holds h = (nx/2 + 1)/nx complex values per
    point (8h bytes).  Forward: plane d_i^+ p 36h, row velocity 36 + 48h,
    plane d_i^- v 52h, row density 28 + 40h, plane Y terms 40h, row pressure
    24 + 24h; adjoint: row p* (reads the three divergence terms) 16 + 40h,
    plane Y terms 40h, row density 32 + 40h, plane d_i^+ 52h, row velocity
    36 + 48h, plane divergence terms d_i^- (3 -> 3) 52h (fields 4 B, spectra
    8h B, k-space tables 4h B per point)."""
    h = (nx // 2 + 1) / nx
    return 172.0 + 512.0 * h


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in ("kernels.hip", "qpat_internal.hpp", "plan.cpp"):   # plan.cpp fixes the spectrum layout
        with open(os.path.join(ROOT, "paper_1810_11685_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def pmc_traffic(pass_name: str, record: str = "fwdadj512_pmc_traffic.json", tiles=None):
    """HBM traffic per launch from a committed rocprofv3 counter summary, if it
    was taken with the current kernel source (and, where the record names its
    launch shape, with the same rows and columns per tile); else None."""
    path = os.path.join(ROOT, "profiles", record)
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_hash") != kernel_hash():
        return None
    if tiles is not None and rec.get("tiles") is not None and list(rec["tiles"])[:2] != list(tiles)[:2]:
        return None
    if pass_name in ("fwd_col_fraclap", "adj_col_fraclap"):
        pass_name = "col_fraclap"      # one kernel serves both
    k = rec.get("per_pass", {}).get(pass_name)
    return None if k is None else k.get("bytes_per_launch")


def dominant_kernel(passes: dict, npts: int, batch: int = 1) -> dict:
    """Roofline entry of the kernel with the largest share of an iterate pair:
    its launches per pair times their mean duration.  achieved = algorithmic
    bytes per launch (scope-table bytes per point times the points of one
    launch) / mean launch duration."""
    names = [n for n, _ in PASSES_ORDER()]
    kern = {}
    for pid, name in enumerate(names):
        k = KERNEL_OF_PASS.get(pid, name)
        kern.setdefault(k, []).append(pid)
    total = sum(v["ms"] for v in passes.values())
    best = max(kern, key=lambda k: sum(passes[names[p]]["ms"] for p in kern[k]))
    pids = kern[best]
    ms = sum(passes[names[p]]["ms"] for p in pids) / len(pids)
    byts = sum(SCOPE_BYTES[p] for p in pids) / len(pids) * npts * batch
    gbs = byts / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None, "kernel": best,
            "passes": [names[p] for p in pids], "bytes_per_launch": int(byts), "launch_ms": round(ms, 5),
            "share_of_step": round(ms * len(pids) / total, 4)}


def PASSES_ORDER():
    from paper_1810_11685_amd.ops import PASSES
    return PASSES


def sync():
    import torch
    torch.cuda.synchronize()


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, budget_s: float):
    """FP64 oracle forward + adjoint on a bounded number of iterates of the same
    512^2 workload, with every host thread for scipy.fft and with one; returns
    grid-point-steps/s and what was sampled."""
    import qpat_inputs as qi
    from oracle import kspace as K
    prm, c0, rho0, p0 = cfg["params"], cfg["c0"], cfg["rho0"], cfg["p0"]
    ops = K.Operators(prm, c0, rho0)
    n_pts = prm["nx"] * prm["ny"]
    ncpu = os.cpu_count() or 1
    res = {}
    for workers, share in ((ncpu, 0.6), (1, 0.4)):
        K.set_workers(workers)
        t = time.perf_counter()
        K.forward(prm, c0, rho0, p0, ops=ops, nsteps=3)
        per = (time.perf_counter() - t) / 3
        steps = int(max(5, min(prm["nt"], share * budget_s / (2.2 * per))))
        short = dict(prm, nt=steps)
        t0 = time.perf_counter()
        d = K.forward(short, c0, rho0, p0, ops=ops)
        t1 = time.perf_counter()
        K.adjoint(short, c0, rho0, qi.gaussian_field(d.shape, 5), ops=ops)
        t2 = time.perf_counter()
        res[workers] = (2 * n_pts * steps / (t2 - t0), steps, t1 - t0, t2 - t1)
    K.set_workers(ncpu)
    v, steps, tf, ta = res[ncpu]
    v1, steps1, tf1, ta1 = res[1]
    return {"value": v, "unit": "grid-point-steps/s", "cores": ncpu, "kind": "oracle",
            "cpu_model": cpu_model(), "host_cpus": ncpu, "value_1_thread": v1,
            "sample": f"FP64 numpy/scipy.fft oracle, 512x512 workload, forward + adjoint over the first "
                      f"{steps} of 2000 iterates with {ncpu} scipy.fft threads ({tf:.1f} s + {ta:.1f} s), "
                      f"and over the first {steps1} with 1 thread ({tf1:.1f} s + {ta1:.1f} s)"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched J^T J v comparisons")
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch tiles")
    ap.add_argument("--graph", choices=["on", "off"], default="on")
    ap.add_argument("--no-recon", action="store_true", help="skip the reconstruction-driver measurement")
    ap.add_argument("--no-medium", action="store_true", help="skip the sound-speed gradient measurement")
    ap.add_argument("--no-3d", action="store_true", help="skip the 3-D solver measurement")
    ap.add_argument("--no-optical", action="store_true", help="skip the optical operator measurement")
    ap.add_argument("--no-probe", action="store_true", help="skip the grid-barrier probe")
    ap.add_argument("--batches3d", default="1,3,8,16", help="batch sizes of the 3-D measurement")
    ap.add_argument("--tiles", default=None,
                    help="launch shape rows,cols,row_threads,col_threads of the headline plan (skips tuning)")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the library runs on one GPU (the operator shards over independent "
              "solves, not within one); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1810_11685_amd as q
    import qpat_inputs as qi
    from paper_1810_11685_amd.ops import PASSES

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    T = lambda x: torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float32, device=dev)

    # ------------------------------------------------------------ headline
    cfg = qi.config("fwdadj512")
    prm = cfg["params"]
    nx, ny, nt, ns = prm["nx"], prm["ny"], prm["nt"], len(prm["sensor_xy"])
    plan = q.Plan(prm, cfg["c0"], cfg["rho0"])
    tiles_default = plan.tiles()
    plan.set_graph(args.graph == "on")
    stream = torch.cuda.Stream(device=dev)
    if args.tiles:
        plan.set_tiles(*[int(v) for v in args.tiles.split(",")])
        log(f"tiles {plan.tiles()} (given)")
    elif not args.no_tune:
        t = time.perf_counter()
        plan.tune(1, stream=stream)           # forward + adjoint candidates, in the launch mode timed below
        log(f"tuned tiles {plan.tiles()} (default {tiles_default}) in {time.perf_counter() - t:.1f} s")
    p0 = T(cfg["p0"])
    res = T(qi.gaussian_field((nt, ns), 1823))

    def step():
        plan.forward(p0)
        plan.adjoint(res)

    with torch.cuda.stream(stream):
        for i in range(args.warmup):
            step()
            sync()
            log(f"warmup step {i + 1}/{args.warmup} done")
        sync()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        sync()
        t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    value = 2.0 * nx * ny * nt / (ms * 1e-3)
    log(f"forward+adjoint {ms:.2f} ms/step -> {value:.3e} grid-point-steps/s")

    # ------------------------------------------------------------ roofline (live, HIP events)
    passes = {}
    with torch.cuda.stream(stream):
        for pid, (name, kind) in enumerate(PASSES):
            t_ms = plan.time_pass(pid, batch=1, reps=50, stream=stream)
            gbs = SCOPE_BYTES[pid] * nx * ny / (t_ms * 1e-3) / 1e9
            passes[name] = {"kernel": kind, "ms": round(t_ms, 5), "bytes_per_pt": SCOPE_BYTES[pid],
                            "bytes_per_pt_with_tables": PASS_BYTES[pid], "GB_s": round(gbs, 1)}
    roofline = dominant_kernel(passes, nx * ny)
    roofline["traffic"] = pmc_traffic(roofline["kernel"])
    whole = value * 152.0 / 1e9
    log(f"dominant kernel {roofline['kernel']}: {roofline['launch_ms'] * 1e3:.1f} us per launch, "
        f"{roofline['achieved']:.0f} GB/s, {roofline['share_of_step']:.1%} of the step; "
        f"whole solve {whole:.0f} GB/s algorithmic")

    out = {"metric": METRIC, "value": round(value, 1), "unit": "grid-point-steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "fwdadj512: one forward + one adjoint k-space solve, 512x512 grid, "
                                  "Nt=2000, 256 ring sensors, lossy (alpha0=0.75 dB/MHz^1.5/cm, y=1.5), "
                                  "20-cell PML, heterogeneous c0/rho0",
                      "grid": [ny, nx], "nt": nt, "ns": ns, "batch": 1,
                      "launch": "hipGraph" if args.graph == "on" else "stream",
                      "tiles": list(plan.tiles()), "whole_solve_GB_s": round(whole, 1)},
           "roofline": roofline, "passes": passes}

    # ------------------------------------------------------------ batched vs plain J^T J v
    if not args.no_batch:
        g = qi.config("gn1024")
        gp = g["params"]
        B = 8
        gplan = q.Plan(gp, g["c0"], g["rho0"])
        tiles_1 = tiles_b = gplan.tiles()
        if not args.no_tune:                      # each path gets the launch shape tuned for its batch
            gplan.tune(1, stream=stream)          # plain calls launch eagerly
            tiles_1 = gplan.tiles()
            gplan.set_graph(args.graph == "on")
            gplan.tune(B, stream=stream)          # the batched call in its launch mode
            tiles_b = gplan.tiles()
            gplan.set_graph(False)
        vs = T(np.stack([qi.smooth_noise(1024, 1024, 8.0, 3000 + j) for j in range(B)]))
        with torch.cuda.stream(stream):
            gplan.set_tiles(*tiles_1)
            gplan.set_graph(False)
            gplan.jtjv(vs[0])                     # warm-up (plain)
            sync()
            t_single = []                         # each plain call timed on its own
            for j in range(B):
                t = time.perf_counter()
                gplan.jtjv(vs[j])
                sync()
                t_single.append(time.perf_counter() - t)
            t_plain = B * statistics.median(t_single)
            log(f"plain J^T J v x{B} (1024^2, Nt=4000): {t_plain:.2f} s (8 x median of {B} single calls)")
            gplan.set_tiles(*tiles_b)
            gplan.set_graph(args.graph == "on")
            gplan.jtjv(vs)                        # warm-up (batched; captures the graph)
            sync()
            t_runs = []
            for _ in range(REPEATS):
                t = time.perf_counter()
                gplan.jtjv(vs)
                sync()
                t_runs.append(time.perf_counter() - t)
            t_batch = statistics.median(t_runs)
            log(f"batched J^T J v x{B}: {t_batch:.2f} s (median of {REPEATS})")
            # per-pass bandwidth of the batched launches (in-sequence HIP-event timing)
            bpass = {}
            for pid, (name, kind) in enumerate(PASSES):
                t_ms = gplan.time_pass(pid, batch=B, reps=5, stream=stream)
                bpass[name] = {"kernel": kind, "ms": round(t_ms, 4), "bytes_per_pt": SCOPE_BYTES[pid],
                               "GB_s": round(SCOPE_BYTES[pid] * 1024 * 1024 * B / (t_ms * 1e-3) / 1e9, 1)}
            broof = dominant_kernel(bpass, 1024 * 1024, B)
            bsum = sum(v["ms"] for v in bpass.values())
            bavg = sum(SCOPE_BYTES.values()) * 1024 * 1024 * B / (bsum * 1e-3) / 1e9
            log(f"batched passes: dominant {broof['kernel']} {broof['achieved']:.0f} GB/s; "
                f"iterate pair {bsum * 1e3:.0f} us = {bavg:.0f} GB/s algorithmic")
        pts = 2.0 * 1024 * 1024 * gp["nt"] * B
        out["batched"] = {"workload": "gn1024: J^T J v, 1024x1024, Nt=4000, 512 ring sensors, "
                                      "alpha0=0.5, y=1.3, 8 Krylov vectors",
                          "jtjv_per_s_plain": round(B / t_plain, 4), "jtjv_per_s_batched": round(B / t_batch, 4),
                          "speedup": round(t_plain / t_batch, 3),
                          "timing": f"plain: {B} x the median of {B} single calls; batched: median of {REPEATS}",
                          "batched_runs_s": [round(v, 4) for v in t_runs],
                          "plain_single_s": [round(v, 4) for v in t_single],
                          "grid_point_steps_per_s_batched": round(pts / t_batch, 1),
                          "tiles_plain": list(tiles_1), "tiles_batched": list(tiles_b),
                          "passes": bpass,
                          "roofline": dict(broof, traffic=pmc_traffic(broof["kernel"], "gn1024x8_pmc_traffic.json",
                                                                      tiles_b),
                                           iterate_pair_GB_s=round(bavg, 1),
                                           iterate_pair_frac=round(bavg / HBM_PEAK_GBS, 4))}
        del gplan, vs
        torch.cuda.empty_cache()

        probs = qi.uneven_batch()
        plans = [q.Plan(p["params"], p["c0"], p["rho0"]) for p in probs]
        xs = [T(p["p0"]) for p in probs]
        pts = sum(2.0 * p["params"]["nx"] * p["params"]["ny"] * p["params"]["nt"] for p in probs)
        # plain path: every problem alone, with the launch shape tuned for one
        # vector of its grid size
        sizes = sorted({p["params"]["nx"] for p in probs})
        shape_1 = {}
        for n in sizes:
            group = [pl for pl, p in zip(plans, probs) if p["params"]["nx"] == n]
            if not args.no_tune:
                group[0].tune(1, stream=stream)
            shape_1[n] = group[0].tiles()
        for pl, p in zip(plans, probs):
            pl.set_tiles(*shape_1[p["params"]["nx"]])
        def timed(fn, reps):
            out_t = []
            for _ in range(reps):
                t = time.perf_counter()
                fn()
                sync()
                out_t.append(time.perf_counter() - t)
            return statistics.median(out_t), out_t

        def plain_jtjv():
            for pl, x in zip(plans, xs):
                pl.jtjv(x)

        def plain_jv():                           # J v = H_a v: one forward solve per problem
            for pl, x in zip(plans, xs):
                pl.forward(x)

        with torch.cuda.stream(stream):
            plain_jtjv()                          # warm-up
            plain_jv()
            sync()
            t_plain, runs_plain = timed(plain_jtjv, REPEATS)
            t_plain_jv, runs_plain_jv = timed(plain_jv, REPEATS)
            # batched path: launch shapes per grid size and the schedule (one
            # launch set for all, or one per grid size on forked streams) from
            # the batch tuner
            bat = q.Batch(plans)
            bat.set_graph(args.graph == "on")
            sched = bat.tune(stream=stream) if not args.no_tune else bat.schedule()
            shape_b = {n: next(pl for pl, p in zip(plans, probs) if p["params"]["nx"] == n).tiles() for n in sizes}
            bat.jtjv(xs)                          # warm-up (captures the graphs)
            bat.forward(xs)
            sync()
            t_batch, runs_batch = timed(lambda: bat.jtjv(xs), REPEATS)
            t_batch_jv, runs_batch_jv = timed(lambda: bat.forward(xs), REPEATS)
        log(f"uneven batch of {len(probs)}: J^T J v plain {t_plain:.2f} s, batched {t_batch:.2f} s; "
            f"J v plain {t_plain_jv:.2f} s, batched {t_batch_jv:.2f} s")
        out["uneven"] = {"workload": "32 problems over 12x256^2 (Nt=1380), 10x384^2 (Nt=2069), "
                                     "10x512^2 (Nt=2759), N/2 ring sensors each, dt=1.875e-8 s: "
                                     "J v (one forward solve each) and J^T J v",
                         "jv_per_s_plain": round(len(probs) / t_plain_jv, 3),
                         "jv_per_s_batched": round(len(probs) / t_batch_jv, 3),
                         "jv_speedup": round(t_plain_jv / t_batch_jv, 3),
                         "jtjv_per_s_plain": round(len(probs) / t_plain, 3),
                         "jtjv_per_s_batched": round(len(probs) / t_batch, 3),
                         "speedup": round(t_plain / t_batch, 3),
                         "timing": f"median of {REPEATS} runs each",
                         "runs_s": {"jtjv_plain": [round(v, 4) for v in runs_plain],
                                    "jtjv_batched": [round(v, 4) for v in runs_batch],
                                    "jv_plain": [round(v, 4) for v in runs_plain_jv],
                                    "jv_batched": [round(v, 4) for v in runs_batch_jv]},
                         "grid_point_steps_per_s_batched": round(pts / t_batch, 1),
                         "schedule": ["one launch set for all problems",
                                      "one launch sequence per grid size on forked streams"][sched],
                         "tiles_plain": {str(n): list(shape_1[n]) for n in sizes},
                         "tiles_batched": {str(n): list(shape_b[n]) for n in sizes}}
        del bat, plans, xs
        torch.cuda.empty_cache()

    # ------------------------------------------------------------ reconstruction driver
    # One outer step of the inexact-Newton method (PCG of Algorithm 4 with the
    # TV priorconditioner, fixed 10 iterations) for 4 data sets of the
    # headline workload, solved side by side on batched J^T J v.
    if not args.no_recon:
        nq, its = 4, 10
        p0s = T(np.stack([qi.blobs(ny, nx, 1900 + j, count=5, radius_cells=0.2 * 220) for j in range(nq)]))
        tiles_step = plan.tiles()
        with torch.cuda.stream(stream):
            if not args.no_tune:
                plan.tune(nq, stream=stream)      # the driver's calls carry nq vectors each
            tiles_recon = plan.tiles()
            datas = plan.forward(p0s)
            v = torch.zeros_like(p0s)
            plan.jtjv(v)                          # warm-up of the batched graph
            sync()
            t = time.perf_counter()
            plan.jtjv(v)
            sync()
            t_h = time.perf_counter() - t
            t = time.perf_counter()
            x, hist, iters, solves = q.ld_reconstruct(plan, datas, torch.zeros_like(p0s), beta=1e-3, gamma=1e-4,
                                                      i_max=its, i_m=its, tol_in=-np.inf, tol_out=-np.inf,
                                                      outer_max=1, solve_tol=1e-6, stream=stream)
            sync()
            t_r = time.perf_counter() - t
        rel_err = [float(torch.linalg.norm(x[j] - p0s[j]) / torch.linalg.norm(p0s[j])) for j in range(nq)]
        log(f"reconstruction step: {its} PCG iterations x {nq} data sets in {t_r:.2f} s "
            f"(batched J^T J v {t_h:.3f} s each; {solves} M_gamma solver iterations)")
        out["recon"] = {"workload": f"one inexact-Newton step (Algorithm 5) with {its} PCG iterations "
                                    f"(Algorithm 4, TV priorconditioner beta=1e-3, gamma=1e-4) for {nq} "
                                    "data sets of the 512x512 Nt=2000 workload, side by side",
                        "seconds": round(t_r, 3), "seconds_per_pcg_iteration": round(t_r / its, 4),
                        "jtjv_batched_seconds": round(t_h, 4),
                        "jtjv_fraction": round(its * t_h / t_r, 3), "mgamma_solver_iterations": solves,
                        "misfit_reduction": [round(h[-1] / h[0], 6) for h in hist],
                        "rel_error_vs_p0": [round(e, 4) for e in rel_err], "tiles": list(tiles_recon)}
        del p0s, datas, v, x
        plan.set_tiles(*tiles_step)
        torch.cuda.empty_cache()

    # ------------------------------------------------------------ sound-speed gradient
    # d<r, H_a[c0] p0>/dc0 for the headline workload: checkpoints every 100
    # iterates with the reverse sweep recomputing one segment at a time, and
    # every sensitivity kept (no recomputation); compared with one forward +
    # adjoint pair.
    if not args.no_medium:
        mg = {}
        with torch.cuda.stream(stream):
            for label, k in (("K100", 100), ("all", nt - 1)):
                for b in (1, 4):
                    pb = p0.expand(b, ny, nx).contiguous()
                    rb = res.expand(b, nt, ns).contiguous()
                    work = torch.empty(plan.medium_grad_bytes(k, b), dtype=torch.uint8, device=dev)
                    plan.medium_grad(pb, rb, interval=k, work=work)       # warm-up
                    sync()
                    t = time.perf_counter()
                    plan.medium_grad(pb, rb, interval=k, work=work)
                    sync()
                    dt_g = time.perf_counter() - t
                    mg[f"{label}_B{b}"] = {"interval": k, "batch": b, "seconds": round(dt_g, 4),
                                           "workspace_MB": round(work.numel() / 2 ** 20, 1),
                                           "vs_fwd_adj": round(dt_g / (b * ms * 1e-3), 3)}
                    log(f"medium gradient K={k} B={b}: {dt_g * 1e3:.1f} ms "
                        f"({dt_g / (b * ms * 1e-3):.2f} x forward+adjoint per vector), "
                        f"workspace {work.numel() / 2 ** 20:.0f} MB")
                    del work, pb, rb
                    torch.cuda.empty_cache()
        out["medium_grad"] = {"workload": "sound-speed gradient d<r, H_a[c0] p0>/dc0 of the 512x512 Nt=2000 "
                                          "workload (grad_p0 as a by-product)", "runs": mg}

    # ------------------------------------------------------------ 3-D solver
    # The paper's 3-D reconstruction grid: 33^3 nodes plus an 8-cell PML
    # (49^3), Nt = 292, 2145 detectors on two faces; forward + adjoint for one
    # vector, for the three illuminations of the paper side by side, and for
    # 16 Krylov vectors.
    if not args.no_3d:
        c3 = qi.config3d("vol33")
        p3 = c3["params"]
        n3, nt3, ns3 = p3["nx"] * p3["ny"] * p3["nz"], p3["nt"], p3["sensor_xyz"].shape[0]
        BYTES_3D_PAIR = bytes_3d_pair(p3["nx"])
        plan3 = q.Plan3D(p3, c3["c0"], c3["rho0"])
        plan3.set_graph(args.graph == "on")
        runs = {}
        with torch.cuda.stream(stream):
            for b in [int(v) for v in args.batches3d.split(",")]:
                x3 = T(np.stack([c3["p0"]] * b))
                r3 = T(qi.gaussian_field((b, nt3, ns3), 3303))
                plan3.forward(x3, stream=stream)
                plan3.adjoint(r3, stream=stream)
                sync()
                t = time.perf_counter()
                for _ in range(2):
                    plan3.forward(x3, stream=stream)
                    plan3.adjoint(r3, stream=stream)
                sync()
                dt3 = (time.perf_counter() - t) / 2
                gps3 = 2.0 * n3 * nt3 * b / dt3
                runs[f"B{b}"] = {"batch": b, "ms": round(dt3 * 1e3, 2), "grid_point_steps_per_s": round(gps3, 1),
                                 "algorithmic_GB_s": round(gps3 / 2 * BYTES_3D_PAIR / 1e9, 1)}
                log(f"3-D 49^3 Nt=292 forward+adjoint B={b}: {dt3 * 1e3:.1f} ms -> {gps3:.3e} grid-point-steps/s")
                del x3, r3
        out["vol33"] = {"workload": "3-D: 33^3 nodes of 0.3125 mm plus an 8-cell PML (49^3 grid), Nt=292, "
                                    "2145 detectors on two faces, lossy (alpha0=0.75, y=1.5), forward + adjoint",
                        "shape": "automatic per batch size", "tiles_one_vector": list(plan3.tiles()),
                        "bytes_per_point_per_iterate_pair": BYTES_3D_PAIR,
                        "runs": runs}
        del plan3
        torch.cuda.empty_cache()
        # the paper's other 3-D grid: 37^3 nodes plus the PML (53^3, a prime
        # axis length), for one vector and the three illuminations
        c37 = qi.config3d("vol37")
        p37 = c37["params"]
        n37, nt37, ns37 = p37["nx"] * p37["ny"] * p37["nz"], p37["nt"], p37["sensor_xyz"].shape[0]
        plan37 = q.Plan3D(p37, c37["c0"], c37["rho0"])
        plan37.set_graph(args.graph == "on")
        runs37 = {}
        with torch.cuda.stream(stream):
            for b in (1, 3):
                x3 = T(np.stack([c37["p0"]] * b))
                r3 = T(qi.gaussian_field((b, nt37, ns37), 3707))
                plan37.forward(x3, stream=stream)
                plan37.adjoint(r3, stream=stream)
                sync()
                t = time.perf_counter()
                for _ in range(2):
                    plan37.forward(x3, stream=stream)
                    plan37.adjoint(r3, stream=stream)
                sync()
                dt3 = (time.perf_counter() - t) / 2
                gps3 = 2.0 * n37 * nt37 * b / dt3
                runs37[f"B{b}"] = {"batch": b, "ms": round(dt3 * 1e3, 2), "grid_point_steps_per_s": round(gps3, 1),
                                   "algorithmic_GB_s": round(gps3 / 2 * bytes_3d_pair(p37["nx"]) / 1e9, 1)}
                log(f"3-D 53^3 Nt={nt37} forward+adjoint B={b}: {dt3 * 1e3:.1f} ms -> {gps3:.3e} grid-point-steps/s")
                del x3, r3
        out["vol37"] = {"workload": "3-D: 37^3 nodes plus an 8-cell PML (53^3 grid, prime axis length), Nt=292, "
                                    "2145 detectors on two faces, lossy, forward + adjoint",
                        "bytes_per_point_per_iterate_pair": bytes_3d_pair(p37["nx"]), "runs": runs37}
        del plan37
        torch.cuda.empty_cache()

    # ------------------------------------------------------------ optical operators
    # The diffusion-approximation solve (FP64 Jacobi-CG on the grid-matched P1
    # mesh) for N_q = 4 illuminations (one per side), on the paper's 2-D
    # data-generation grid (128^2 pixels of 78.1 um) and on the headline
    # 512^2 grid; then one composite J dX and J^* r on the headline workload.
    if not args.no_optical:
        runs = {}
        for n_o, dx_o in ((128, 7.81e-5), (512, 1e-4)):
            opt = q.Optical(n_o, n_o, dx_o, 4, tol=1e-8)
            g1 = qi.smooth_noise(n_o, n_o, 8.0, 4100)
            g2 = qi.smooth_noise(n_o, n_o, 8.0, 4101)
            mu_e = np.repeat((10.0 * (1.0 + 0.5 * g1)).ravel(), 2)
            kap_e = np.repeat((1.0 / (3.0 * (10.0 * (1.0 + 0.5 * g1) + 1000.0 * (1.0 + 0.3 * g2)))).ravel(), 2)
            kt, mt = T(np.stack([kap_e] * 4)), T(np.stack([mu_e] * 4))
            with torch.cuda.stream(stream):
                opt.forward(kt, mt, np.eye(4), stream=stream)
                sync()
                t = time.perf_counter()
                opt.forward(kt, mt, np.eye(4), stream=stream)
                sync()
                t_f = time.perf_counter() - t
                its = opt.iters
                t = time.perf_counter()
                opt.jv(kt, mt, stream=stream)
                sync()
                t_j = time.perf_counter() - t
            nn_o = (n_o + 1) ** 2
            gbs = OPT_BYTES_PER_NODE_ITER * nn_o * 4 * its / t_f / 1e9
            runs[f"{n_o}"] = {"grid": [n_o, n_o], "illuminations": 4, "forward_s": round(t_f, 4), "cg_iterations": its,
                              "us_per_iteration": round(t_f / its * 1e6, 2), "jv_s": round(t_j, 4),
                              "algorithmic_GB_s": round(gbs, 1)}
            log(f"optical {n_o}^2 x4: forward {t_f * 1e3:.1f} ms ({its} CG iterations, "
                f"{t_f / its * 1e6:.1f} us each, {gbs:.0f} GB/s), J_o v {t_j * 1e3:.1f} ms")
            del opt
        out["optical"] = {"workload": "P1-FEM diffusion approximation (Robin boundary) on the grid-matched mesh, "
                                      "4 illuminations, FP64 CG preconditioned by a multigrid V-cycle, to 1e-8",
                          "bytes_per_node_per_iteration": OPT_BYTES_PER_NODE_ITER, "runs": runs}

    # ------------------------------------------------------------ persistent launch vs kernel boundaries
    # One exchange step of a single-vector solve (every block writes its share
    # of 2 MiB, the two spectra a 512^2 pass hands on, then reads another
    # block's share) synchronised by a grid barrier inside one cooperative
    # kernel (flat and hierarchical) or by a kernel boundary in a graph.
    if not args.no_probe:
        designs = {0: "barrier_flat", 1: "barrier_hierarchical", 2: "kernel_boundary_graph"}
        probe = {}
        with torch.cuda.stream(stream):
            for nb in (256, 512):
                for words_total in (0, 1 << 19):
                    for d, name in designs.items():
                        us, to = q.probe_barrier(d, nb, 256, 400, words_total // nb, stream=stream)
                        probe[f"{name}_{nb}blocks_{'2MiB' if words_total else 'nodata'}"] = \
                            {"us_per_step": round(us, 2), "timed_out": to}
        log("grid barrier probe (us per exchange step): " +
            ", ".join(f"{k} {v['us_per_step']}" for k, v in probe.items()))
        out["persistent_probe"] = {"what": "one exchange step (write own slot, synchronise, read another block's "
                                           "slot), 256 threads per block", "runs": probe}

    # ------------------------------------------------------------ CPU baseline (oracle)
    if not args.no_cpu:
        t = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_budget)
        log(f"cpu baseline {out['cpu_baseline']['value']:.3e} grid-point-steps/s "
            f"({time.perf_counter() - t:.1f} s)")
    else:
        out["cpu_baseline"] = None

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
