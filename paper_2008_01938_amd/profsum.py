"""Summaries of rocprofv3 output for the profiles kept with the library.

    python -m paper_2008_01938_amd.profsum stats DIR
    python -m paper_2008_01938_amd.profsum counters --evals EVALS_JSON DIR...
    python -m paper_2008_01938_amd.profsum traffic FETCH_DIR WRITE_DIR
    python -m paper_2008_01938_amd.profsum trafficfile FETCH_DIR WRITE_DIR KERNEL EVALS TILE SOURCE
    python -m paper_2008_01938_amd.profsum clock CLK_DIR
    python -m paper_2008_01938_amd.profsum sq [--clock GHZ] [--evals EVALS_JSON] DIR...

DIR is a rocprofv3 ``-d`` directory written with ``--output-format csv``;
the CSV files are found under it at any depth.  Kernel names are shortened
to the kernel's own name with its template arguments (``k_bulk<64>``).
Every figure printed is a sum or ratio of what rocprofv3 wrote; nothing is
estimated here.
"""
from __future__ import annotations

import csv
import glob
import json
import os
import re
import sys
from collections import defaultdict

COPY_KERNEL = "copyBuffer"


def short_name(name: str) -> str:
    """`void mcm::(anonymous namespace)::k_bulk<64>(...)` -> `k_bulk<64>`."""
    m = re.search(r"(k_\w+)(<[^()]*?>)?\s*\(", name)
    if m:
        return m.group(1) + (m.group(2) or "").replace(" ", "")
    if "copyBuffer" in name:
        return COPY_KERNEL
    return name.split("(")[0].strip()[:60]


def _rows(d: str, suffix: str):
    files = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not files:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    for f in files:
        with open(f, newline="") as fh:
            yield from csv.DictReader(fh)


def _col(row: dict, *names):
    low = {k.lower(): v for k, v in row.items()}
    for n in names:
        if n.lower() in low:
            return low[n.lower()]
    raise KeyError(f"none of {names} in {list(row)}")


def kernel_stats(d: str):
    """[(kernel, calls, total_ns, avg_ns, min_ns, max_ns, percent)] from the
    kernel-stats CSV, merged by short name."""
    agg = {}
    for r in _rows(d, "kernel_stats.csv"):
        k = short_name(_col(r, "Name", "KERNEL_NAME"))
        calls = int(_col(r, "Calls"))
        tot = float(_col(r, "TotalDurationNs"))
        mn = float(_col(r, "MinNs"))
        mx = float(_col(r, "MaxNs"))
        a = agg.setdefault(k, [0, 0.0, float("inf"), 0.0])
        a[0] += calls
        a[1] += tot
        a[2] = min(a[2], mn)
        a[3] = max(a[3], mx)
    total = sum(v[1] for v in agg.values()) or 1.0
    out = [(k, v[0], v[1], v[1] / max(v[0], 1), v[2], v[3], 100.0 * v[1] / total)
           for k, v in agg.items()]
    return sorted(out, key=lambda x: -x[2])


def dispatches(d: str):
    """Per-dispatch records of a kernel-trace CSV: (dispatch id, kernel,
    start ns, end ns), in start order."""
    out = []
    for r in _rows(d, "kernel_trace.csv"):
        out.append((int(_col(r, "Dispatch_Id")), short_name(_col(r, "Kernel_Name")),
                    int(_col(r, "Start_Timestamp")), int(_col(r, "End_Timestamp"))))
    return sorted(out, key=lambda x: x[2])


def counters(d: str):
    """{dispatch id: {"kernel": name, counter: value}} from a counter-collection
    CSV (values summed over the rows rocprofv3 wrote for the dispatch)."""
    per = defaultdict(dict)
    for r in _rows(d, "counter_collection.csv"):
        did = int(_col(r, "Dispatch_Id"))
        rec = per[did]
        rec["kernel"] = short_name(_col(r, "Kernel_Name"))
        cname = _col(r, "Counter_Name")
        rec[cname] = rec.get(cname, 0.0) + float(_col(r, "Counter_Value"))
    return per


def durations(d: str):
    """{dispatch id: duration ns} from the kernel trace of a counter run."""
    try:
        return {did: e - s for did, _, s, e in dispatches(d)}
    except FileNotFoundError:
        return {}


def per_kernel(recs: dict, names):
    """Sums of the named counters and the dispatch count, per kernel."""
    agg = defaultdict(lambda: defaultdict(float))
    for rec in recs.values():
        a = agg[rec["kernel"]]
        a["dispatches"] += 1
        for n in names:
            a[n] += rec.get(n, 0.0)
    return agg


def cmd_stats(d: str) -> None:
    print("| kernel | calls | total ms | average us | min us | max us | % |")
    print("|---|---|---|---|---|---|---|")
    for k, calls, tot, avg, mn, mx, pct in kernel_stats(d):
        print(f"| {k} | {calls} | {tot / 1e6:.3f} | {avg / 1e3:.2f} | {mn / 1e3:.2f} | "
              f"{mx / 1e3:.2f} | {pct:.1f} |")


def cmd_traffic(fetch_dir: str, write_dir: str) -> None:
    """HBM bytes per dispatch of every kernel, each counter scaled by what it
    reads for the probe's plain 1 GiB device copy."""
    fetch, write = counters(fetch_dir), counters(write_dir)
    f_agg = per_kernel(fetch, ["FETCH_SIZE"])
    w_agg = per_kernel(write, ["WRITE_SIZE"])
    copy_kib = float(1 << 20)
    f_scale = copy_kib / (f_agg[COPY_KERNEL]["FETCH_SIZE"] / max(f_agg[COPY_KERNEL]["dispatches"], 1))
    w_scale = copy_kib / (w_agg[COPY_KERNEL]["WRITE_SIZE"] / max(w_agg[COPY_KERNEL]["dispatches"], 1))
    print(f"fetch_scale: {f_scale:.6f}")
    print(f"write_scale: {w_scale:.6f}")
    print("| kernel | dispatches | fetch MB per dispatch | write MB per dispatch |")
    print("|---|---|---|---|")
    for k in sorted(f_agg, key=lambda x: -f_agg[x]["FETCH_SIZE"]):
        if k == COPY_KERNEL:
            continue
        nd = f_agg[k]["dispatches"]
        fb = f_agg[k]["FETCH_SIZE"] * 1024 * f_scale / nd
        wb = w_agg[k]["WRITE_SIZE"] * 1024 * w_scale / max(w_agg[k]["dispatches"], 1)
        print(f"| {k} | {int(nd)} | {fb / 1e6:.2f} | {wb / 1e6:.2f} |")


def cmd_trafficfile(fetch_dir: str, write_dir: str, kernel: str, evals: float,
                    tile: int, source: str) -> None:
    """The key: value summary bench.py reads for `roofline.traffic`: HBM bytes
    per dispatch of `kernel` (FETCH_SIZE and WRITE_SIZE scaled as in
    `traffic`), and the algorithmic operand bytes per dispatch (two 8-byte
    panel elements per staged split, reused by the tile's `tile` cells of a
    row or column: 16 / tile bytes per split evaluation) for `evals` split
    evaluations over all its dispatches.  `source` is the kernel's source
    file, whose sha256 marks which build the counters belong to."""
    import hashlib
    fetch, write = counters(fetch_dir), counters(write_dir)
    f_agg = per_kernel(fetch, ["FETCH_SIZE"])
    w_agg = per_kernel(write, ["WRITE_SIZE"])
    copy_kib = float(1 << 20)
    f_scale = copy_kib / (f_agg[COPY_KERNEL]["FETCH_SIZE"] / max(f_agg[COPY_KERNEL]["dispatches"], 1))
    w_scale = copy_kib / (w_agg[COPY_KERNEL]["WRITE_SIZE"] / max(w_agg[COPY_KERNEL]["dispatches"], 1))
    nd = f_agg[kernel]["dispatches"]
    fb = f_agg[kernel]["FETCH_SIZE"] * 1024 * f_scale / nd
    wb = w_agg[kernel]["WRITE_SIZE"] * 1024 * w_scale / max(w_agg[kernel]["dispatches"], 1)
    with open(source, "rb") as fh:
        sha = hashlib.sha256(fh.read()).hexdigest()
    print(f"kernel_source_sha256: {sha}")
    print(f"fetch_scale: {f_scale:.6f}")
    print(f"write_scale: {w_scale:.6f}")
    print(f"bulk_launches: {int(nd)}")
    print(f"bulk_fetch_bytes_per_launch: {fb:.0f}")
    print(f"bulk_write_bytes_per_launch: {wb:.0f}")
    print(f"bulk_hbm_bytes_per_launch: {fb + wb:.0f}")
    print(f"bulk_algorithmic_operand_bytes_per_launch: {evals * 16.0 / tile / nd:.0f}")


def cmd_counters(dirs, evals_json: str | None) -> None:
    """SQ counters per kernel: instruction counts per dispatch, VALU issue
    rate against one wave instruction per CU per cycle, LDS bank-conflict
    cycles against LDS-active cycles, and fp64 FMA instructions per split
    evaluation (when the split evaluations per kernel are given)."""
    evals = {}
    if evals_json:
        with open(evals_json) as f:
            evals = json.load(f)
    recs, durs = {}, {}
    for d in dirs:
        c = counters(d)
        du = durations(d)
        for did, rec in c.items():
            key = (d, did)
            recs[key] = rec
            durs[key] = du.get(did)
    names = sorted({n for r in recs.values() for n in r if n != "kernel"})
    agg = defaultdict(lambda: defaultdict(float))
    for key, rec in recs.items():
        a = agg[(rec["kernel"])]
        for n in names:
            if n in rec:
                a[n] += rec[n]
                a["n_" + n] += 1
        if durs.get(key):
            a["dur_ns"] += durs[key]
            a["n_dur"] += 1
    print("| kernel | " + " | ".join(names) + " |")
    print("|---|" + "---|" * len(names))
    for k in sorted(agg):
        a = agg[k]
        cells = []
        for n in names:
            cnt = a.get("n_" + n, 0)
            cells.append(f"{a[n] / cnt:.4g}" if cnt else "-")
        print(f"| {k} | " + " | ".join(cells) + " |")
    print()
    print(json.dumps({k: {n: v for n, v in a.items()} for k, a in agg.items()}, indent=None))


def cmd_sq(dirs, clock_ghz: float, evals_json: str | None) -> None:
    """Utilisation figures per kernel from SQ counter runs of one workload
    (each DIR one rocprofv3 --pmc pass with its kernel trace; a counter's
    value is taken from the pass that collected it, durations are averaged
    over the passes):
      VALU busy (device)  wave VALU instructions x 4 cycles (a wave64
                          instruction occupies a 16-lane SIMD for four
                          cycles) over 1024 SIMDs x summed duration x clock;
      VALU busy (own CUs) the same over 4 SIMDs x SQ_BUSY_CU_CYCLES, i.e.
                          on the compute units the kernel occupied;
      LDS bank-conflict cycles over LDS-active cycles;
      fp64 FMA / ADD wave instructions per 64 split evaluations (when the
      evaluations per kernel are given)."""
    evals = {}
    if evals_json:
        with open(evals_json) as f:
            evals = json.load(f)
    vals = defaultdict(lambda: defaultdict(list))   # kernel -> counter -> per-pass sums
    for d in dirs:
        c = counters(d)
        du = durations(d)
        per = defaultdict(lambda: defaultdict(float))
        for did, rec in c.items():
            a = per[rec["kernel"]]
            for k, v in rec.items():
                if k != "kernel":
                    a[k] += v
            a["dur_ns"] += du.get(did, 0)
            a["dispatches"] += 1
        for kern, a in per.items():
            for k, v in a.items():
                vals[kern][k].append(v)
    tot = {kern: {k: sum(v) / len(v) for k, v in a.items()} for kern, a in vals.items()}
    print(f"clock used for SIMD-cycles: {clock_ghz:.3f} GHz")
    print("| kernel | dispatches | VALU wave-instr per dispatch | VALU busy (device) "
          "| VALU busy (own CUs) | fp64 FMA per 64 evals | fp64 ADD per 64 evals "
          "| LDS instr per VALU instr | LDS bank-conflict / LDS-active |")
    print("|---|---|---|---|---|---|---|---|---|")
    for k in sorted(tot, key=lambda x: -tot[x].get("SQ_INSTS_VALU", 0)):
        a = tot[k]
        nd = a["dispatches"]
        valu = a.get("SQ_INSTS_VALU", 0.0)
        simd_cycles = 1024 * a["dur_ns"] * 1e-9 * clock_ghz * 1e9
        busy = 4 * valu / simd_cycles if simd_cycles else float("nan")
        cu = a.get("SQ_BUSY_CU_CYCLES", 0.0)
        busy_cu = f"{valu / cu:.3f}" if cu else "-"
        ev = evals.get(k)
        fma = f"{a.get('SQ_INSTS_VALU_FMA_F64', 0) * 64 / ev:.3f}" if ev else "-"
        add = f"{a.get('SQ_INSTS_VALU_ADD_F64', 0) * 64 / ev:.3f}" if ev else "-"
        lds = a.get("SQ_INSTS_LDS", 0.0)
        act = a.get("SQ_ACTIVE_INST_LDS", 0.0)
        conf = a.get("SQ_LDS_BANK_CONFLICT", 0.0)
        print(f"| {k} | {int(nd)} | {valu / max(nd, 1):.4g} | {busy:.3f} | {busy_cu} | {fma} | "
              f"{add} | {lds / valu if valu else float('nan'):.3f} | "
              f"{conf / act if act else float('nan'):.3f} |")


def cmd_clock(d: str) -> None:
    """Shader clock while each kernel runs: a least-squares line of
    GRBM_COUNT (summed over the XCDs) against the dispatch's duration."""
    recs = counters(d)
    du = durations(d)
    xs = defaultdict(list)
    for did, rec in recs.items():
        if "GRBM_COUNT" in rec and du.get(did):
            xs[rec["kernel"]].append((du[did], rec["GRBM_COUNT"]))
    print("| kernel | dispatches | duration range us | slope / 8 (GHz) | intercept / 8 (cycles) | r^2 |")
    print("|---|---|---|---|---|---|")
    for k, pts in sorted(xs.items(), key=lambda kv: -len(kv[1])):
        if len(pts) < 3:
            continue
        n = len(pts)
        mx = sum(p[0] for p in pts) / n
        my = sum(p[1] for p in pts) / n
        sxx = sum((p[0] - mx) ** 2 for p in pts)
        sxy = sum((p[0] - mx) * (p[1] - my) for p in pts)
        syy = sum((p[1] - my) ** 2 for p in pts)
        if sxx <= 0 or syy <= 0:
            continue
        b = sxy / sxx
        a = my - b * mx
        r2 = sxy * sxy / (sxx * syy)
        lo = min(p[0] for p in pts) / 1e3
        hi = max(p[0] for p in pts) / 1e3
        print(f"| {k} | {n} | {lo:.1f} - {hi:.1f} | {b / 8:.3f} | {a / 8:.0f} | {r2:.4f} |")


def main(argv) -> int:
    if len(argv) < 2:
        print(__doc__)
        return 2
    cmd = argv[1]
    if cmd == "stats":
        cmd_stats(argv[2])
    elif cmd == "trafficfile":
        cmd_trafficfile(argv[2], argv[3], argv[4], float(argv[5]), int(argv[6]), argv[7])
    elif cmd == "traffic":
        cmd_traffic(argv[2], argv[3])
    elif cmd == "clock":
        cmd_clock(argv[2])
    elif cmd == "sq":
        args = argv[2:]
        clock, ev = 2.4, None
        while args and args[0].startswith("--"):
            if args[0] == "--clock":
                clock, args = float(args[1]), args[2:]
            elif args[0] == "--evals":
                ev, args = args[1], args[2:]
            else:
                break
        cmd_sq(args, clock, ev)
    elif cmd == "counters":
        args = argv[2:]
        ev = None
        if args and args[0] == "--evals":
            ev, args = args[1], args[2:]
        cmd_counters(args, ev)
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv))
