"""Measurement helpers of the benchmark (not part of the library): a calibration copy kernel for rocprofv3 byte counters and
summaries of rocprofv3 CSV output.

    python bench_profile.py copy --mib 256
        runs a plain device-to-device copy of the given size (the reference
        for scaling FETCH_SIZE / WRITE_SIZE to bytes).
    python bench_profile.py stats <kernel_stats.csv>
        prints a short per-kernel table from a --stats CSV.
    python bench_profile.py pmc <dir_fetch> <dir_write> <dir_cfetch> <dir_cwrite> \
            --copy-mib 256 --out profiles/pmc_traffic.json
        combines two counter runs of the benchmark with two of the copy kernel
        into per-pass HBM traffic per launch.
    python bench_profile.py passes --cfg gn1024 --batch 8 --tiles 2,1,256,256
        times every pass kind of one plan on its own (qpat_time_pass), for
        counter runs that should see one pass kind per kernel name.
    python bench_profile.py table <pmc_dir> [<pmc_dir> ...]
        per-pass averages of every counter found in rocprofv3 --pmc CSV
        directories.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1810_11685_amd")

# kernel-name fragments of the pass kinds (row kernels by mode without its modifier bits, template arg U)
ROW_MODES = {0: "fwd_row_velocity", 1: "fwd_row_density", 2: "fwd_row_density", 3: "fwd_row_pressure",
             4: "adj_row_pressure", 5: "adj_row_pressure", 6: "adj_row_density", 7: "adj_row_velocity"}


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in ("kernels.hip", "qpat_internal.hpp", "plan.cpp"):   # plan.cpp fixes the spectrum layout
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def copy_kernel(mib: int, reps: int = 5) -> None:
    import torch
    n = mib * 1024 * 1024 // 4
    a = torch.ones(n, device="cuda", dtype=torch.float32)
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"copied {mib} MiB x {reps}", flush=True)


COL_MODES = {0: "fwd_col_grad_p", 1: "fwd_col_div_v", 2: "col_fraclap", 3: "adj_col_grad", 4: "adj_col_div",
             5: "col_apply"}


def pass_of(name: str):
    """Pass-kind name of a row / column kernel dispatch (the Y_dis/Y_abs column
    kernel serves the forward and the adjoint pass alike: 'col_fraclap')."""
    if "col_kernel<" in name:
        mode = int(name.split("col_kernel<")[1].split(",")[1].split(">")[0])
        return COL_MODES.get(mode, f"col_mode_{mode}")
    if "row_kernel<" in name:
        mode = int(name.split("row_kernel<")[1].split(",")[0].split(">")[0])
        mode &= ~(16 | 32)  # modifiers: sensitivity store (16), fused-only density instance (32)
        return ROW_MODES.get(mode, f"row_mode_{mode}")
    return None


def read_counters(d: str, counter: str):
    """{kernel name: [values per dispatch]} from a rocprofv3 --pmc CSV directory."""
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    out = {}
    for f in files:
        for r in csv.DictReader(open(f)):
            if r.get("Counter_Name") != counter:
                continue
            out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return out


def stats_table(path: str) -> str:
    rows = list(csv.DictReader(open(path)))
    lines = [f"{'calls':>7} {'avg_us':>9} {'min_us':>9} {'max_us':>9} {'total_ms':>9} {'pct':>6}  kernel"]
    for r in rows:
        lines.append(f"{int(r['Calls']):7d} {float(r['AverageNs']) / 1e3:9.2f} {float(r['MinNs']) / 1e3:9.2f} "
                     f"{float(r['MaxNs']) / 1e3:9.2f} {float(r['TotalDurationNs']) / 1e6:9.2f} "
                     f"{float(r['Percentage']):6.1f}  {r['Name'][:110]}")
    return "\n".join(lines)


def pmc_summary(dfetch, dwrite, dcf, dcw, copy_mib, out, tiles=""):
    fetch, write = read_counters(dfetch, "FETCH_SIZE"), read_counters(dwrite, "WRITE_SIZE")
    cf, cw = read_counters(dcf, "FETCH_SIZE"), read_counters(dcw, "WRITE_SIZE")

    def copy_val(d):
        best = None
        for k, v in d.items():
            if "copy" in k.lower() or "elementwise" in k.lower() or "Copy" in k:
                m = max(v)
                best = m if best is None else max(best, m)
        return best

    expected_kib = copy_mib * 1024.0
    sf = expected_kib / copy_val(cf) if copy_val(cf) else None
    sw = expected_kib / copy_val(cw) if copy_val(cw) else None
    per = {}
    vals = {}
    for name in sorted(set(fetch) | set(write)):
        p = pass_of(name)
        if p is None:
            continue
        v = vals.setdefault(p, {"f": [], "w": []})
        v["f"] += fetch.get(name, [])
        v["w"] += write.get(name, [])
        per.setdefault(p, {"kernels": []})["kernels"].append(name[:80])
    for p, v in vals.items():
        # a pass kind may run as several instances (first iterates apart):
        # averages over all its dispatches
        fk = sum(v["f"]) / len(v["f"]) if v["f"] else None
        wk = sum(v["w"]) / len(v["w"]) if v["w"] else None
        e = per[p]
        e["fetch_KiB_per_launch"] = fk
        e["write_KiB_per_launch"] = wk
        if fk is not None and wk is not None and sf and sw:
            e["bytes_per_launch"] = (fk * sf + wk * sw) * 1024.0
    rec = {"kernel_hash": kernel_hash(), "copy_MiB": copy_mib, "scale_fetch": sf, "scale_write": sw,
           "note": "HBM-side bytes per launch = FETCH_SIZE*scale_fetch + WRITE_SIZE*scale_write (KiB -> B); "
                   "scales make a plain copy of known size read and write exactly its size",
           "per_pass": per}
    if tiles:
        rec["tiles"] = [int(v) for v in tiles.split(",")]
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec, indent=1))


def time_passes(cfg: str, batch: int, tiles: str, reps: int, nt: int) -> None:
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    import paper_1810_11685_amd as q
    import qpat_inputs as qi
    from paper_1810_11685_amd.ops import PASSES
    from bench import SCOPE_BYTES
    g = qi.config(cfg, nt=nt)
    plan = q.Plan(g["params"], g["c0"], g["rho0"])
    if tiles:
        plan.set_tiles(*[int(v) for v in tiles.split(",")])
    n = g["params"]["nx"] * g["params"]["ny"]
    for pid in range(len(PASSES)):
        t = plan.time_pass(pid, batch=batch, reps=reps)
        print(f"{PASSES[pid][0]:18s} {t * 1e3:8.1f} us  {SCOPE_BYTES[pid] * n * batch / (t * 1e-3) / 1e9:7.0f} GB/s",
              flush=True)


def counter_table(dirs) -> str:
    """Per-pass mean of every counter in the given --pmc directories."""
    vals = {}
    names = set()
    for d in dirs:
        files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        for f in files:
            for r in csv.DictReader(open(f)):
                p = pass_of(r["Kernel_Name"])
                if p is None:
                    continue
                names.add(r["Counter_Name"])
                vals.setdefault(p, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    cols = sorted(names)
    lines = [f"{'pass':18s} " + " ".join(f"{c[:22]:>22s}" for c in cols)]
    for p in sorted(vals):
        row = [sum(vals[p][c]) / len(vals[p][c]) if c in vals[p] else float("nan") for c in cols]
        lines.append(f"{p:18s} " + " ".join(f"{v:22.1f}" for v in row))
    return "\n".join(lines)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("copy")
    c.add_argument("--mib", type=int, default=256)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    p = sub.add_parser("pmc")
    p.add_argument("fetch")
    p.add_argument("write")
    p.add_argument("copy_fetch")
    p.add_argument("copy_write")
    p.add_argument("--copy-mib", type=int, default=256)
    p.add_argument("--out", required=True)
    p.add_argument("--tiles", default="", help="launch shape the counters were taken with (recorded)")
    t = sub.add_parser("passes")
    t.add_argument("--cfg", default="gn1024")
    t.add_argument("--batch", type=int, default=8)
    t.add_argument("--tiles", default="")
    t.add_argument("--reps", type=int, default=5)
    t.add_argument("--nt", type=int, default=64)
    tb = sub.add_parser("table")
    tb.add_argument("dirs", nargs="+")
    a = ap.parse_args(argv)
    if a.cmd == "copy":
        copy_kernel(a.mib)
    elif a.cmd == "stats":
        print(stats_table(a.csv))
    elif a.cmd == "passes":
        time_passes(a.cfg, a.batch, a.tiles, a.reps, a.nt)
    elif a.cmd == "table":
        print(counter_table(a.dirs))
    else:
        pmc_summary(a.fetch, a.write, a.copy_fetch, a.copy_write, a.copy_mib, a.out, a.tiles)


if __name__ == "__main__":
    sys.exit(main())
