#!/usr/bin/env python3
"""Benchmark of the matrix-chain-multiplication table fill on one MI355X.

One step = one complete solve (m and s tables, every kernel of the path)
of the synthetic n = 8192 chain (dims uniform in [1, 1024], seed 2), with
the chain already resident in device memory and the output tables
preallocated.  Prints one JSON line:

  value      split evaluations per second, (n^3 - n)/6 per step
  roofline   the bulk kernel (the dominant one) against the fp64 VALU issue
             rate: each split evaluation is an fp64 fma, add and min, i.e.
             3 VALU lane-ops; peak = 256 CUs x 64 lanes x 2.4 GHz.  Its
             duration is measured with HIP events on the launch streams
             around every launch of the last timed step.  `traffic` comes from the committed
             rocprofv3 FETCH_SIZE/WRITE_SIZE summary, and is null when the
             kernel source changed since it was taken.
  cpu_baseline  the CPU oracle on a bounded window of the same chain.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MCM split evals/s at n=8192; batched instances/s + p99 latency vs plain"
UNIT = "split evals/s"
PEAK_OPS = 256 * 64 * 2.4e9      # fp64 VALU lane-ops per second
OPS_PER_EVAL = 3                 # fma + add + min
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_bulk_n8192_hbm_traffic.txt")
TILED_SRC = os.path.join(ROOT, "paper_2008_01938_amd", "csrc", "k_tiled.hip")

WORKLOADS = {
    "mcm_single_n8192": ("single_n8192", "n=8192, dims uniform int32 [1,1024], seed 2"),
    "mcm_single_n2048": ("single_n2048", "n=2048, dims uniform int32 [1,1024], seed 1"),
    "mcm_single_n128": ("single_n128", "n=128, dims uniform int32 [1,64], seed 0"),
}


def source_sha() -> str:
    with open(TILED_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def read_traffic():
    """HBM bytes per bulk launch from the committed counter summary, or None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256") != source_sha():
        return None
    try:
        return float(kv["bulk_hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


SCLK_FILE = os.path.join(ROOT, "profiles", "k_bulk_n8192_sclk.md")


def read_sclk():
    """Shader clock (GHz) while k_bulk runs, from the committed counter fit."""
    if not os.path.exists(SCLK_FILE):
        return None
    with open(SCLK_FILE) as f:
        for line in f:
            cells = [c.strip() for c in line.strip().strip("|").split("|")]
            if len(cells) >= 4 and cells[0] == "k_bulk":
                try:
                    return float(cells[3])
                except ValueError:
                    return None
    return None


def host_threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        n = min(n, int(env))
    return max(1, n)


def host_cpu() -> dict:
    """Model name and logical CPU count of the host (from /proc/cpuinfo)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count(), "threads_allowed": host_threads()}


def cpu_baseline(p, target_s: float):
    """Time the oracle on a window p[0:L+1] of the chain, L sized so the
    run takes about target_s seconds of wall time on all host threads."""
    import oracle
    threads = host_threads()
    n = len(p) - 1
    L = min(1024, n)
    t0 = time.perf_counter()
    oracle.fill(p[:L + 1], threads=threads)
    dt = time.perf_counter() - t0
    rate = (L ** 3 - L) / 6 / max(dt, 1e-9)
    want = int((6 * rate * target_s) ** (1 / 3))
    L = max(L, min(n, want))
    t0 = time.perf_counter()
    oracle.fill(p[:L + 1], threads=threads)
    dt = time.perf_counter() - t0
    evals = (L ** 3 - L) / 6
    return {"value": evals / dt, "unit": UNIT, "cores": threads, "kind": "oracle",
            "host": host_cpu(),
            "sample": f"oracle on the window of the first {L} matrices of the benchmark "
                      f"chain ({evals:.3g} split evals, {dt:.1f} s wall, OpenMP over the "
                      f"cells of each diagonal)"}


def bench_batched(binding, workloads, torch, reps: int = 3):
    """4096 chains (n in [16, 512], dims in [1, 256], seed 3): one batched
    solve (a reusable plan, and the one-shot mcm_solve_batched) against 4096
    plain per-chain solves on one stream (chains already resident on the
    device for the plain solves)."""
    b = workloads.batched_4096()
    off = binding.table_offsets(b.ns)
    total = int(off[-1] + int(b.ns[-1]) ** 2)
    m_all = torch.empty(total, dtype=torch.int64, device="cuda")
    s_all = torch.empty(total, dtype=torch.int32, device="cuda")
    binding.solve_batched_into(b.ns, b.p_off, b.p_all, off, m_all, s_all)
    torch.cuda.synchronize()
    oneshot = None
    for _ in range(reps):
        t0 = time.perf_counter()
        binding.solve_batched_into(b.ns, b.p_off, b.p_all, off, m_all, s_all)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        oneshot = dt if oneshot is None else min(oneshot, dt)
    # The same batch through a plan built (and autotuned) once for its shape.
    t0 = time.perf_counter()
    plan = binding.Plan(b.ns, b.p_off, off, int(b.p_all.max()))
    plan_build = time.perf_counter() - t0
    choice = plan.autotune(b.p_all, m_all, s_all)
    best = None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.solve_into(b.p_all, m_all, s_all)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        best = dt if best is None else min(best, dt)
    plan.close()
    # Read back all 4096 trees (with their costs) in one launch.
    node_off = binding.node_offsets(b.ns)
    g = int(node_off[-1] + b.ns[-1] - 1)
    lo = torch.empty(g, dtype=torch.int32, device="cuda")
    hi = torch.empty(g, dtype=torch.int32, device="cuda")
    cost = torch.empty(b.ns.size, dtype=torch.int64, device="cuda")
    rb = None
    for _ in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        binding.parenthesize_batched_into(b.ns, off, s_all, node_off, lo, hi, p_off=b.p_off,
                                          p_all=b.p_all, cost_all=cost)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        rb = dt if rb is None else min(rb, dt)
    roots = m_all[torch.as_tensor(off + b.ns.astype(np.int64) - 1, device="cuda")]
    rb_ok = bool(torch.equal(roots, cost))
    chains = [binding.Chain(b.dims(i)) for i in range(b.ns.size)]
    views = [(m_all[int(off[i]):int(off[i]) + int(n) ** 2],
              s_all[int(off[i]):int(off[i]) + int(n) ** 2]) for i, n in enumerate(b.ns)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for ch, (mv, sv) in zip(chains, views):
        ch.solve_into(mv, sv)
    torch.cuda.synchronize()
    plain = time.perf_counter() - t0
    for ch in chains:
        ch.close()
    evals = float(np.sum((b.ns.astype(np.float64) ** 3 - b.ns) / 6))
    count = int(b.ns.size)
    return {"workload": "mcm_batched_4096 (n in [16,512], dims [1,256], seed 3)",
            "instances_per_s": count / best, "ms": 1e3 * best,
            "split_evals_per_s": evals / best,
            "plain_instances_per_s": count / plain, "plain_ms": 1e3 * plain,
            "speedup_vs_plain": plain / best,
            "oneshot_ms": 1e3 * oneshot, "plan_build_ms": 1e3 * plan_build,
            "plan_pair_min_blocks": choice,
            "readback_ms": 1e3 * rb, "readback_costs_equal_m0n": rb_ok,
            "note": "ms: mcm_plan_solve of a plan built and autotuned once for the batch "
                    "(host dims upload included); oneshot_ms: mcm_solve_batched, which also "
                    "plans and uploads its launch tables; readback is "
                    "mcm_parenthesize_batched (trees and costs of all chains)"}


def bench_reconstruction(binding, torch, p, m, s, reps: int = 5):
    """Optimal order read back from the solved n = 8192 table on the device
    (mcm_parenthesize: node intervals, tree cost and parenthesized text),
    best of `reps` calls, wall time including the host side of the call."""
    n = len(p) - 1
    lo = torch.empty(n - 1, dtype=torch.int32, device="cuda")
    hi = torch.empty(n - 1, dtype=torch.int32, device="cuda")
    cost = torch.empty(1, dtype=torch.int64, device="cuda")
    text = torch.empty(binding.parens_length(n) + 1, dtype=torch.uint8, device="cuda")
    out = {}
    for what, kw in (("tree_ms", dict(lo=lo, hi=hi)),
                     ("tree_cost_text_ms", dict(lo=lo, hi=hi, cost=cost, p=p, text=text))):
        best = None
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            binding.parenthesize_into(s, n, **kw)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        out[what] = 1e3 * best
    out["cost_equals_m0n"] = int(cost.item()) == int(m.view(-1)[n - 1].item())
    out["solve_fraction"] = None
    return out


# Table I of the paper (PIPELINE column, ms, GTX TITAN Black, averages over
# n and k in each range): context for the S-DP timings, not a target.
SDP_PAPER_PIPELINE_MS = {"sdp_small": 78, "sdp_medium": 386, "sdp_large": 2408}


def bench_sdp(binding, workloads, torch, reps: int = 3):
    """The simplified DP problem (Section II-A) at the top of each n / k
    range of Table I, minimum operator, random offsets (seed 12)."""
    out = {}
    for name, (n, k) in workloads.SDP_CONFIGS.items():
        a, init = workloads.sdp_instance(n, k, 12)
        st = torch.zeros(n, dtype=torch.int32, device="cuda")
        st[:int(a[0])] = torch.from_numpy(init).cuda()
        binding.sdp_solve_into(a, st, "min")
        torch.cuda.synchronize()
        best = None
        for _ in range(reps):
            t0 = time.perf_counter()
            binding.sdp_solve_into(a, st, "min")
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        pairs = float(n - int(a[0])) * k
        out[name] = {"n": n, "k": k, "a1": int(a[0]), "ms": 1e3 * best,
                     "terms_per_s": pairs / best,
                     "paper_pipeline_ms_gtx_titan_black": SDP_PAPER_PIPELINE_MS[name]}
    return {"workload": "S-DP, min, k offsets drawn from [1, 2k], n and k at the top of "
                        "each Table I range (seed 12)", "configs": out}


def bench_obst(binding, torch, n: int = 8192, reps: int = 3):
    """Optimal binary search tree over n keys (key and gap weights iid in
    [0, 2^16), seed 5), the interval DP of the same split shape: the tiled
    kernels in their weight-interval mode (what AUTO picks here), and the
    int64 diagonal launches for comparison."""
    rng = np.random.default_rng(5)
    p = rng.integers(0, 1 << 16, size=n).astype(np.int32)
    q = rng.integers(0, 1 << 16, size=n + 1).astype(np.int32)
    out = {"workload": f"optimal BST, n={n} keys, weights uniform [0, 2^16), seed 5"}
    for algo, tries in (("tiled", reps), ("wavefront", 1)):
        e, r = binding.obst_solve(p, q, algo=algo)
        torch.cuda.synchronize()
        best = None
        for _ in range(tries):
            t0 = time.perf_counter()
            e, r = binding.obst_solve(p, q, algo=algo)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        out[f"{algo}_ms"] = 1e3 * best
    L = n + 1
    out["split_evals_per_s"] = (L ** 3 - L) / 6 / (out["tiled_ms"] / 1e3)
    return out


def bench_pipeline(binding, workloads, torch, sizes=(512, 1024)):
    """Ablation: the paper's pipeline (Fig. 8, with stalls; one workgroup, a
    barrier per step) against the wavefront and tiled paths, same chains
    (dims uniform [1, 1024], seed 7)."""
    out = {}
    for n in sizes:
        p = workloads.uniform_dims(n, 1, 1024, 7)
        row = {}
        for algo in ("pipeline", "wavefront", "tiled"):
            m, s = binding.solve(p, algo=algo)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            m, s = binding.solve(p, algo=algo)
            torch.cuda.synchronize()
            row[f"{algo}_ms"] = 1e3 * (time.perf_counter() - t0)
        out[f"n{n}"] = row
    return {"workload": "MCM chains, dims uniform [1, 1024], seed 7", "sizes": out}


def bench_serving(binding, workloads, torch, count: int, rate: float):
    """Open-loop Poisson stream (seed 4, n log-uniform in [8, 4096], dims in
    [1, 1024]): continuous-batching server against plain FIFO solves."""
    from paper_2008_01938_amd import serve
    st = workloads.serving_stream(count=count, rate=rate, seed=4)
    served = serve.run_served(st, mem_budget=24 << 30, max_slots=256).summary()
    plain = serve.run_plain(st).summary()
    # Saturation: the same requests all arriving at once; throughput is
    # requests over the time to finish them all.
    sat = workloads.serving_stream(count=count, rate=1e12, seed=4)
    sat_served = serve.run_served(sat, mem_budget=24 << 30, max_slots=256).summary()
    sat_plain = serve.run_plain(sat).summary()
    # Overload: arrivals at twice the plain saturated capacity, where plain
    # solving cannot keep up (its queue grows for the whole stream).
    over_rate = 2.0 * sat_plain["requests_per_s"]
    over = workloads.serving_stream(count=count, rate=over_rate, seed=4)
    over_served = serve.run_served(over, mem_budget=24 << 30, max_slots=256).summary()
    over_plain = serve.run_plain(over).summary()
    return {"workload": f"mcm_serving ({count} requests of the seed-4 stream recipe, "
                        f"Poisson {rate:g}/s, n log-uniform [8,4096], dims [1,1024])",
            "served": served, "plain": plain,
            "p99_speedup_vs_plain": plain["p99_ms"] / served["p99_ms"],
            "p50_speedup_vs_plain": plain["p50_ms"] / served["p50_ms"],
            "saturation": {"served_requests_per_s": sat_served["requests_per_s"],
                           "plain_requests_per_s": sat_plain["requests_per_s"],
                           "speedup_vs_plain": sat_served["requests_per_s"] /
                           sat_plain["requests_per_s"]},
            "overload": {"rate_per_s": over_rate, "served": over_served, "plain": over_plain,
                         "p99_speedup_vs_plain": over_plain["p99_ms"] / over_served["p99_ms"]}}


def traffic_probe(binding, torch, chain, m, s):
    """One solve, then a plain device copy of a known size, for counter
    collection under rocprofv3 --pmc (FETCH_SIZE / WRITE_SIZE)."""
    chain.solve_into(m, s)
    torch.cuda.synchronize()
    nbytes = 1 << 30
    src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"traffic_probe": True, "copy_bytes": nbytes,
                      "kernel_source_sha256": source_sha()}), flush=True)


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="mcm_single_n8192", choices=sorted(WORKLOADS))
    ap.add_argument("--algo", default="auto", choices=["auto", "tiled", "wavefront"])
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="wall time target of the CPU-baseline sample (0 = skip)")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="one solve plus a 1 GiB copy, for rocprofv3 --pmc runs")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched section")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving section")
    ap.add_argument("--no-sdp", action="store_true", help="skip the S-DP section")
    ap.add_argument("--no-obst", action="store_true", help="skip the optimal-BST section")
    ap.add_argument("--no-pipeline", action="store_true",
                    help="skip the pipeline (Fig. 8) ablation section")
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--serve-rate", type=float, default=600.0, help="Poisson arrivals per second")
    args = ap.parse_args()

    if args.steps < 1 or args.warmup < 0:
        print("bench.py needs --steps >= 1 and --warmup >= 0", file=sys.stderr)
        return 2
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the solver is a "
              "single-device library and multi-GPU runs are not part of this build.",
              file=sys.stderr)
        return 2

    import torch

    from paper_2008_01938_amd import binding, workloads

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    torch.cuda.set_device(0)
    binding.load()

    maker, desc = WORKLOADS[args.workload]
    p = getattr(workloads, maker)()
    n = len(p) - 1
    algo = args.algo
    chosen = {binding.ALGO_TILED: "tiled", binding.ALGO_WAVEFRONT: "wavefront"}[
        binding.select_algo(p) if algo == "auto" else binding.ALGOS[algo]]

    chain = binding.Chain(p)
    m = torch.empty((n, n), dtype=torch.int64, device="cuda")
    s = torch.empty((n, n), dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()

    if args.traffic_probe:
        traffic_probe(binding, torch, chain, m, s)
        return 0

    for _ in range(args.warmup):
        chain.solve_into(m, s, algo=algo)
    torch.cuda.synchronize()

    # The last timed step marks the dominant kernel's launches with events
    # (every marked launch adds two event records to its stream, so marking
    # every step would tax the throughput being measured).
    dom = "bulk" if chosen == "tiled" else "wavefront"
    dom_class = binding.PROF_BULK if dom == "bulk" else binding.PROF_WAVE
    binding.profile_enable(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for step in range(args.steps):
        if step == args.steps - 1:
            binding.profile_enable(True, classes=[dom_class])
        chain.solve_into(m, s, algo=algo)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    d = binding.profile_read(dom_class)
    binding.profile_enable(False)

    # Per-class kernel time from one more solve with every class marked.
    binding.profile_enable(True)
    chain.solve_into(m, s, algo=algo)
    torch.cuda.synchronize()
    prof = {name: binding.profile_read(c) for c, name in
            enumerate(["setup", "bulk", "close", "wavefront", "batched"])}
    binding.profile_enable(False)

    elapsed = t1 - t0
    evals = (n ** 3 - n) / 6
    value = evals * args.steps / elapsed
    ms_per_step = 1e3 * elapsed / args.steps
    avg_s = d["ms"] / 1e3 / max(1, d["launches"])
    evals_per_launch = d["split_evals"] / max(1, d["launches"])
    achieved = evals_per_launch * OPS_PER_EVAL / avg_s if avg_s > 0 else 0.0
    traffic = read_traffic() if chosen == "tiled" and args.workload == "mcm_single_n8192" else None
    roofline = {
        "bound": "alu",
        "achieved": round(achieved / 1e12, 4),
        "peak": round(PEAK_OPS / 1e12, 4),
        "unit": "TOP/s",
        "frac": round(achieved / PEAK_OPS, 4),
        "traffic": traffic,
        "kernel": "k_bulk" if dom == "bulk" else "k_wave_diag",
        "ops_per_split_eval": OPS_PER_EVAL,
        "avg_launch_ms": round(avg_s * 1e3, 5),
        "launches_per_step": d["launches"],
    }
    sclk = read_sclk() if dom == "bulk" else None
    if sclk:
        # The same fraction against the clock measured while k_bulk runs.
        roofline["sclk_ghz_measured"] = sclk
        roofline["frac_at_measured_sclk"] = round(achieved / (256 * 64 * sclk * 1e9), 4)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "dims": desc, "algo": chosen,
                   "exact_integer": True, "parallelism": "single GPU"},
        "roofline": roofline,
        "kernels_ms_per_step": {k: round(v["ms"], 4) for k, v in prof.items()},
    }
    rec = bench_reconstruction(binding, torch, p, m, s)
    rec["solve_fraction"] = round(rec["tree_cost_text_ms"] / ms_per_step, 4)
    out["reconstruction"] = rec
    chain.close()
    del m, s
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    if not args.no_batched:
        out["batched"] = bench_batched(binding, workloads, torch)
    if not args.no_serving:
        out["serving"] = bench_serving(binding, workloads, torch, args.serve_requests,
                                       args.serve_rate)
    if not args.no_sdp:
        out["sdp"] = bench_sdp(binding, workloads, torch)
    if not args.no_obst:
        out["obst"] = bench_obst(binding, torch)
    if not args.no_pipeline:
        out["pipeline_ablation"] = bench_pipeline(binding, workloads, torch)
    if args.cpu_seconds > 0:
        out["cpu_baseline"] = cpu_baseline(p, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
