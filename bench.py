#!/usr/bin/env python3
"""Benchmark of the matrix-chain-multiplication table fill on one MI355X.

One step = one complete solve (m and s tables, every kernel of the path)
of the synthetic n = 8192 chain (dims uniform in [1, 1024], seed 2), with
the chain already resident in device memory and the output tables
preallocated.  Prints one JSON line:

  value      split evaluations per second, (n^3 - n)/6 per step
  roofline   the bulk kernel (the dominant one) against the integer-VALU
             roofline fixed before any tuning: 7 VALU lane-ops per split
             evaluation (a 24-bit multiply, two 64-bit adds, a 64-bit
             compare, three selects), peak 256 CUs x 64 lanes x 2.4 GHz =
             39.3 TOP/s, i.e. 5.62e12 split evaluations/s.  The kernel's own
             instruction basis (fp64 keys: fma + add + min, 3 lane-ops per
             evaluation) is reported beside it.  The kernel's duration comes
             from one solve on the serial schedule (every launch alone on the
             device, HIP events on the launch stream), so launches that
             overlap in the timed steps are not counted twice; the whole-step
             rate on both bases is reported as well.  `traffic` comes from the
             committed rocprofv3 FETCH_SIZE/WRITE_SIZE summary, and is null
             when the kernel source changed since it was taken.
  c1, c2     the n = 128 and n = 2048 chains: median latency over 100 solves
             (HIP events on the stream), and split evaluations/s.
  batched    4096 chains (n in [16, 512]) in one plan solve vs plain solves
             (and the plan replayed from a HIP graph).
  wide       n = 8192 with dims in [1, 4096]: the int64 tiled kernels and the
             int64 wavefront.
  serving    the 20000-request Poisson stream at 0.8 x the measured plain
             capacity (and at 2 x, and all at once), served vs plain.
  cpu_baseline  the CPU oracle on a bounded window of the n = 8192 chain on
             all host threads, and single-threaded on the n = 128 and n = 2048
             chains.

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
PEAK_OPS = 256 * 64 * 2.4e9      # VALU lane-ops per second (int32 and fp64 alike)
OPS_PER_EVAL = 7                 # integer accounting of a split evaluation, fixed before tuning
FP64_OPS_PER_EVAL = 3            # the kernels' own fp64-key evaluation: fma + add + min
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_bulk_n8192_hbm_traffic.txt")
TILED_SRC = os.path.join(ROOT, "paper_2008_01938_amd", "csrc", "k_tiled.hip")

WORKLOADS = {
    "mcm_single_n8192": ("single_n8192", "n=8192, dims uniform int32 [1,1024], seed 2"),
    "mcm_single_n2048": ("single_n2048", "n=2048, dims uniform int32 [1,1024], seed 1"),
    "mcm_single_n128": ("single_n128", "n=128, dims uniform int32 [1,64], seed 0"),
}


def progress(msg: str) -> None:
    """A progress line on stderr (stdout carries only the JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


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
            if len(cells) >= 4 and cells[0] in ("k_bulk", "k_bulk<64>"):
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


def cpu_baseline(p, target_s: float, workloads=None):
    """Time the oracle on a window p[0:L+1] of the chain, L sized so the
    run takes about target_s seconds of wall time on all host threads; then
    single-threaded on the n = 128 chain (median of 1000 fills) and the
    n = 2048 chain (median of 3 fills)."""
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
    out = {"value": evals / dt, "unit": UNIT, "cores": threads, "kind": "oracle",
           "host": host_cpu(),
           "sample": f"oracle on the window of the first {L} matrices of the benchmark "
                     f"chain ({evals:.3g} split evals, {dt:.1f} s wall, OpenMP over the "
                     f"cells of each diagonal)"}
    if workloads is not None:
        single = {}
        for name, maker, reps in (("mcm_single_n128", workloads.single_n128, 1000),
                                  ("mcm_single_n2048", workloads.single_n2048, 3)):
            q = maker()
            k = len(q) - 1
            ts = []
            for _ in range(reps):
                t0 = time.perf_counter()
                oracle.fill(q, threads=1)
                ts.append(time.perf_counter() - t0)
            med = float(np.median(ts))
            single[name] = {"n": k, "fills": reps, "median_ms": 1e3 * med,
                            "split_evals_per_s": (k ** 3 - k) / 6 / med}
        out["single_thread"] = single
    return out


def bench_small(binding, workloads, torch, name: str, runs: int = 100, warmup: int = 3):
    """Latency of one chain (device-resident dims, preallocated tables):
    HIP events on the caller's stream around each solve (the library joins
    its second stream back into it before returning), median over `runs`;
    for the path AUTO picks and for the int64 wavefront."""
    maker, desc = WORKLOADS[name]
    p = getattr(workloads, maker)()
    n = len(p) - 1
    chain = binding.Chain(p)
    m = torch.empty((n, n), dtype=torch.int64, device="cuda")
    s = torch.empty((n, n), dtype=torch.int32, device="cuda")
    evals = (n ** 3 - n) / 6
    out = {"workload": name, "dims": desc, "n": n,
           "algo_auto": {binding.ALGO_TILED: "tiled", binding.ALGO_WAVEFRONT: "wavefront"}[
               binding.select_algo(p)]}
    for algo in ("auto", "wavefront"):
        for _ in range(warmup):
            chain.solve_into(m, s, algo=algo)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(runs)]
        wall = []
        for e0, e1 in ev:
            t0 = time.perf_counter()
            e0.record()
            chain.solve_into(m, s, algo=algo)
            e1.record()
            e1.synchronize()
            wall.append(time.perf_counter() - t0)
        ms = np.array([e0.elapsed_time(e1) for e0, e1 in ev])
        key = "" if algo == "auto" else "wavefront_"
        out[key + "median_ms"] = float(np.median(ms))
        out[key + "p10_ms"] = float(np.percentile(ms, 10))
        out[key + "p90_ms"] = float(np.percentile(ms, 90))
        out[key + "wall_median_ms"] = 1e3 * float(np.median(wall))
        out[key + "split_evals_per_s"] = evals / (float(np.median(ms)) / 1e3)
    out["runs"] = runs
    chain.close()
    return out


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
    t0 = time.perf_counter()
    choice = plan.autotune(b.p_all, m_all, s_all)
    tune_s = time.perf_counter() - t0
    autotune = {"candidates": plan.candidates(), "chosen": choice, "config": plan.config(),
                "wall_s": tune_s}
    best = None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.solve_into(b.p_all, m_all, s_all)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        best = dt if best is None else min(best, dt)
    # The same plan replayed from a HIP graph recorded once for these outputs.
    gstream = torch.cuda.Stream()
    graph_ms = None
    with torch.cuda.stream(gstream):
        plan.graph_create(m_all, s_all, stream=gstream)
        plan.graph_solve(b.p_all, stream=gstream)
        gstream.synchronize()
        for _ in range(reps):
            t0 = time.perf_counter()
            plan.graph_solve(b.p_all, stream=gstream)
            gstream.synchronize()
            dt = time.perf_counter() - t0
            graph_ms = 1e3 * dt if graph_ms is None else min(graph_ms, 1e3 * dt)
    torch.cuda.synchronize()
    plan.close()
    # The one-shot call again: it now starts from the tuning cache's entry
    # for this batch's bucket.
    oneshot_cached = None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        binding.solve_batched_into(b.ns, b.p_off, b.p_all, off, m_all, s_all)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        oneshot_cached = dt if oneshot_cached is None else min(oneshot_cached, dt)
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
            "oneshot_ms": 1e3 * oneshot, "oneshot_after_autotune_ms": 1e3 * oneshot_cached,
            "graph_replay_ms": graph_ms,
            "plan_build_ms": 1e3 * plan_build,
            "autotune": autotune,
            "readback_ms": 1e3 * rb, "readback_costs_equal_m0n": rb_ok,
            "note": "ms: mcm_plan_solve of a plan built and autotuned once for the batch "
                    "(autotune: every configuration once untimed and three times timed, the "
                    "fastest run each; ms of the candidates are those runs) "
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


def bench_wide(binding, workloads, torch, reps: int = 3):
    """n = 8192 with dims uniform in [1, 4096] (seed 4096): (n-1) max(p)^3 is
    about 2^49, past the fp64 keys' exact range, so AUTO runs the tiled
    schedule on the int64 kernels; the int64 wavefront beside it."""
    p = workloads.uniform_dims(8192, 1, 4096, 4096)
    n = len(p) - 1
    chain = binding.Chain(p)
    m = torch.empty((n, n), dtype=torch.int64, device="cuda")
    s = torch.empty((n, n), dtype=torch.int32, device="cuda")
    out = {"workload": "n=8192, dims uniform int32 [1,4096], seed 4096 (beyond the fp64 keys)"}
    for algo, tries in (("auto", reps), ("wavefront", 1)):
        chain.solve_into(m, s, algo=algo)
        torch.cuda.synchronize()
        best = None
        for _ in range(tries):
            t0 = time.perf_counter()
            chain.solve_into(m, s, algo=algo)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        key = "tiled_int64" if algo == "auto" else "wavefront"
        out[f"{key}_ms"] = 1e3 * best
        out[f"{key}_split_evals_per_s"] = (n ** 3 - n) / 6 / best
    chain.close()
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


def bench_serving(binding, workloads, torch, count: int, load: float):
    """Open-loop Poisson stream (seed 4, n log-uniform in [8, 4096], dims in
    [1, 1024]): continuous-batching server against plain FIFO solves.  The
    plain saturated capacity C is measured first (every request arriving at
    once, solved one at a time); the headline runs the stream at load * C,
    the overload run at 2 C.  The stream's n and dims do not depend on the
    rate (the gaps are drawn first and scaled by it)."""
    from paper_2008_01938_amd import serve
    budget, slots = 24 << 30, 256
    sat = workloads.serving_stream(count=count, rate=1e12, seed=4)
    sat_plain = serve.run_plain(sat).summary()
    progress(f"serving: plain capacity {sat_plain['requests_per_s']:.1f}/s")
    sat_served = serve.run_served(sat, mem_budget=budget, max_slots=slots).summary()
    progress(f"serving: served saturated {sat_served['requests_per_s']:.1f}/s")
    cap = sat_plain["requests_per_s"]
    rate = load * cap
    st = workloads.serving_stream(count=count, rate=rate, seed=4)
    served = serve.run_served(st, mem_budget=budget, max_slots=slots).summary()
    progress(f"serving at {rate:.1f}/s: served p99 {served['p99_ms']:.2f} ms")
    plain = serve.run_plain(st).summary()
    progress(f"serving at {rate:.1f}/s: plain p99 {plain['p99_ms']:.2f} ms")
    over_rate = 2.0 * cap
    over = workloads.serving_stream(count=count, rate=over_rate, seed=4)
    over_served = serve.run_served(over, mem_budget=budget, max_slots=slots).summary()
    progress(f"serving at {over_rate:.1f}/s: served p99 {over_served['p99_ms']:.2f} ms")
    over_plain = serve.run_plain(over).summary()
    progress(f"serving at {over_rate:.1f}/s: plain p99 {over_plain['p99_ms']:.2f} ms")
    return {"workload": f"mcm_serving ({count} requests of the seed-4 stream, n log-uniform "
                        f"[8,4096], dims [1,1024]; Poisson at {load:g} x the plain capacity = "
                        f"{rate:.1f}/s)",
            "requests": count, "plain_capacity_per_s": cap, "load_vs_plain_capacity": load,
            "rate_per_s": rate, "served": served, "plain": plain,
            "p99_speedup_vs_plain": plain["p99_ms"] / served["p99_ms"],
            "p50_speedup_vs_plain": plain["p50_ms"] / served["p50_ms"],
            "saturation": {"served_requests_per_s": sat_served["requests_per_s"],
                           "plain_requests_per_s": sat_plain["requests_per_s"],
                           "speedup_vs_plain": sat_served["requests_per_s"] /
                           sat_plain["requests_per_s"],
                           "served": sat_served, "plain": sat_plain},
            "overload": {"rate_per_s": over_rate, "load_vs_plain_capacity": 2.0,
                         "served": over_served, "plain": over_plain,
                         "p99_speedup_vs_plain": over_plain["p99_ms"] / over_served["p99_ms"]}}


def counter_probe(binding, workloads, torch, chain, m, s, which: str):
    """For rocprofv3 counter runs, one workload per process so that every
    kernel's dispatches belong to it: `single`, one n = 8192 solve on the
    serial schedule (every launch alone on the device); `batched`, one plan
    solve of the 4096-chain batch on 64-edge tiles, then one on 32-edge
    tiles.  Then a plain device copy of a known size (the counters' scale)."""
    if which == "single":
        binding.profile_enable(True, classes=[], serial=True)
        chain.solve_into(m, s)
        torch.cuda.synchronize()
        binding.profile_enable(False)
    else:
        b = workloads.batched_4096()
        off = binding.table_offsets(b.ns)
        total = int(off[-1] + int(b.ns[-1]) ** 2)
        m_all = torch.empty(total, dtype=torch.int64, device="cuda")
        s_all = torch.empty(total, dtype=torch.int32, device="cuda")
        plan = binding.Plan(b.ns, b.p_off, off, int(b.p_all.max()))
        for edge in (64, 32):
            plan.set_config(edge)
            plan.solve_into(b.p_all, m_all, s_all)
            torch.cuda.synchronize()
        plan.close()
        del m_all, s_all
    nbytes = 1 << 30
    src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"counter_probe": which, "copy_bytes": nbytes,
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
    ap.add_argument("--counter-probe", choices=["single", "batched"],
                    help="for rocprofv3 counter runs: one n=8192 solve on the serial "
                         "schedule (single) or the 4096-chain batch on 64- and 32-edge tiles "
                         "(batched), then a 1 GiB copy")
    ap.add_argument("--no-small", action="store_true", help="skip the n=128 / n=2048 section")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched section")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving section")
    ap.add_argument("--no-sdp", action="store_true", help="skip the S-DP section")
    ap.add_argument("--no-obst", action="store_true", help="skip the optimal-BST section")
    ap.add_argument("--no-wide", action="store_true",
                    help="skip the n=8192 dims [1,4096] section (int64 tiled kernels)")
    ap.add_argument("--no-pipeline", action="store_true",
                    help="skip the pipeline (Fig. 8) ablation section")
    ap.add_argument("--serve-requests", type=int, default=20000)
    ap.add_argument("--serve-load", type=float, default=0.8,
                    help="arrival rate as a multiple of the measured plain capacity")
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

    if args.counter_probe:
        counter_probe(binding, workloads, torch, chain, m, s, args.counter_probe)
        return 0

    for _ in range(args.warmup):
        chain.solve_into(m, s, algo=algo)
    torch.cuda.synchronize()

    # The timed steps carry no profiling events.
    binding.profile_enable(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        chain.solve_into(m, s, algo=algo)
    torch.cuda.synchronize()
    t1 = time.perf_counter()

    # Per-class kernel time from one more solve with every class marked, on
    # the benchmark's own (overlapped) schedule: launches of different
    # classes run at once, so the classes' sums exceed the step.
    names = ["setup", "bulk", "close", "wavefront", "batched"]
    binding.profile_enable(True)
    chain.solve_into(m, s, algo=algo)
    torch.cuda.synchronize()
    prof = {name: binding.profile_read(c) for c, name in enumerate(names)}
    binding.profile_enable(False)
    # The same solve on the serial schedule: every launch alone on the
    # device, so each class's event-timed duration is the kernel's own.
    binding.profile_enable(True, serial=True)
    ts0 = time.perf_counter()
    chain.solve_into(m, s, algo=algo)
    torch.cuda.synchronize()
    serial_wall = time.perf_counter() - ts0
    prof_serial = {name: binding.profile_read(c) for c, name in enumerate(names)}
    binding.profile_enable(False)

    elapsed = t1 - t0
    evals = (n ** 3 - n) / 6
    value = evals * args.steps / elapsed
    ms_per_step = 1e3 * elapsed / args.steps
    dom = "bulk" if chosen == "tiled" else "wavefront"
    d = prof_serial[dom]
    avg_s = d["ms"] / 1e3 / max(1, d["launches"])
    rate = d["split_evals"] / (d["ms"] / 1e3) if d["ms"] > 0 else 0.0
    traffic = read_traffic() if chosen == "tiled" and args.workload == "mcm_single_n8192" else None
    roofline = {
        "bound": "alu",
        "achieved": round(rate * OPS_PER_EVAL / 1e12, 4),
        "peak": round(PEAK_OPS / 1e12, 4),
        "unit": "TOP/s",
        "frac": round(rate * OPS_PER_EVAL / PEAK_OPS, 4),
        "traffic": traffic,
        "kernel": "k_bulk" if dom == "bulk" else "k_wave_diag",
        "basis": "7 int32-VALU lane-ops per split evaluation (fixed before tuning); "
                 "peak 256 CUs x 64 lanes x 2.4 GHz",
        "ops_per_split_eval": OPS_PER_EVAL,
        "kernel_split_evals_per_s": rate,
        "avg_launch_ms": round(avg_s * 1e3, 5),
        "launches_per_solve": d["launches"],
        "split_evals_per_launch": d["split_evals"] / max(1, d["launches"]),
        "duration_source": "HIP events around each launch of one solve on the serial schedule",
        "frac_fp64_issue": round(rate * FP64_OPS_PER_EVAL / PEAK_OPS, 4),
        "step_frac": round(value * OPS_PER_EVAL / PEAK_OPS, 4),
        "step_frac_fp64_issue": round(value * FP64_OPS_PER_EVAL / PEAK_OPS, 4),
    }
    sclk = read_sclk() if dom == "bulk" else None
    if sclk:
        # The fp64-issue fraction against the clock measured while k_bulk runs.
        roofline["sclk_ghz_measured"] = sclk
        roofline["frac_fp64_issue_at_measured_sclk"] = round(
            rate * FP64_OPS_PER_EVAL / (256 * 64 * sclk * 1e9), 4)

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
        "kernels_ms_serial": {k: round(v["ms"], 4) for k, v in prof_serial.items()},
        "kernels_split_evals_serial": {k: v["split_evals"] for k, v in prof_serial.items()},
        "kernels_launches_serial": {k: v["launches"] for k, v in prof_serial.items()},
        "serial_solve_ms": round(1e3 * serial_wall, 3),
    }
    progress(f"n={n}: {ms_per_step:.3f} ms per step; serial solve {1e3 * serial_wall:.2f} ms")
    rec = bench_reconstruction(binding, torch, p, m, s)
    rec["solve_fraction"] = round(rec["tree_cost_text_ms"] / ms_per_step, 4)
    out["reconstruction"] = rec
    chain.close()
    del m, s
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    if not args.no_small:
        out["c1"] = bench_small(binding, workloads, torch, "mcm_single_n128")
        out["c2"] = bench_small(binding, workloads, torch, "mcm_single_n2048")
        progress(f"n=128 {out['c1']['median_ms']:.3f} ms, n=2048 {out['c2']['median_ms']:.3f} ms")
    if not args.no_batched:
        out["batched"] = bench_batched(binding, workloads, torch)
        progress(f"batched {out['batched']['ms']:.2f} ms")
    if not args.no_serving:
        out["serving"] = bench_serving(binding, workloads, torch, args.serve_requests,
                                       args.serve_load)
    if not args.no_sdp:
        out["sdp"] = bench_sdp(binding, workloads, torch)
        progress("sdp done")
    if not args.no_obst:
        out["obst"] = bench_obst(binding, torch)
        progress("obst done")
    if not args.no_wide:
        out["wide"] = bench_wide(binding, workloads, torch)
        progress(f"wide: tiled int64 {out['wide']['tiled_int64_ms']:.2f} ms, "
                 f"wavefront {out['wide']['wavefront_ms']:.1f} ms")
    if not args.no_pipeline:
        out["pipeline_ablation"] = bench_pipeline(binding, workloads, torch)
        progress("pipeline ablation done")
    if args.cpu_seconds > 0:
        out["cpu_baseline"] = cpu_baseline(p, args.cpu_seconds, workloads)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
