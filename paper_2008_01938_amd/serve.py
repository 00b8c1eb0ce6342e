"""Open-loop request driver for the continuous-batching server.

`run_served` replays a :class:`workloads.RequestStream` against an
``mcm_server``: each request is submitted at its scheduled arrival time,
completions are polled, and each request's latency is its completion time
minus its scheduled arrival (both on the server's steady clock).
`run_plain` replays the same stream as plain per-request solves: one
``mcm_solve`` at a time on one stream, in arrival order, each started when
its request has arrived and the previous one has finished.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import binding
from .workloads import RequestStream


@dataclass
class ServeResult:
    latencies: np.ndarray          # seconds, per request, in request order
    makespan: float                # first arrival -> last completion, seconds
    count: int
    outputs: dict = field(default_factory=dict)   # request index -> (m, s) when kept

    @property
    def throughput(self) -> float:
        return self.count / self.makespan if self.makespan > 0 else 0.0

    def summary(self) -> dict:
        lat = self.latencies
        return {"requests": self.count, "requests_per_s": self.throughput,
                "p50_ms": 1e3 * float(np.percentile(lat, 50)),
                "p99_ms": 1e3 * float(np.percentile(lat, 99)),
                "mean_ms": 1e3 * float(lat.mean()), "makespan_s": self.makespan}


def run_served(stream: RequestStream, mem_budget: int = 16 << 30, max_slots: int = 256,
               keep=None, idle_sleep: float = 50e-6) -> ServeResult:
    """Replay `stream` against a fresh server.  `keep`: request indices
    whose tables are copied to the host before release."""
    keep = set(keep or ())
    batch = stream.batch
    count = int(batch.ns.size)
    lat = np.zeros(count)
    outputs = {}
    with binding.Server(mem_budget, max_slots) as srv:
        t0 = binding.clock_now()
        arrive = t0 + stream.arrivals
        nxt = 0
        finished = 0
        last_done = t0
        while finished < count:
            now = binding.clock_now()
            while nxt < count and arrive[nxt] <= now:
                srv.submit(batch.dims(nxt), nxt)
                nxt += 1
            infos = srv.poll()
            for info in infos:
                i = int(info.tag)
                if info.status != binding.OK:
                    raise binding.MCMError(info.status, f"served request {i}")
                lat[i] = info.t_done - arrive[i]
                last_done = max(last_done, info.t_done)
                if i in keep:
                    outputs[i] = srv.fetch(info)
                srv.release(i)
                finished += 1
            if not infos and (nxt >= count or arrive[nxt] > now + idle_sleep):
                time.sleep(idle_sleep)
    return ServeResult(latencies=lat, makespan=last_done - t0, count=count, outputs=outputs)


def run_plain(stream: RequestStream, keep=None) -> ServeResult:
    """Replay `stream` as one mcm_solve at a time (FIFO, one stream)."""
    import torch
    keep = set(keep or ())
    batch = stream.batch
    count = int(batch.ns.size)
    lat = np.zeros(count)
    outputs = {}
    nmax = int(batch.ns.max()) if count else 1
    m = torch.empty(nmax * nmax, dtype=torch.int64, device="cuda")
    s = torch.empty(nmax * nmax, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    t0 = binding.clock_now()
    arrive = t0 + stream.arrivals
    last_done = t0
    for i in range(count):
        while binding.clock_now() < arrive[i]:
            pass
        n = int(batch.ns[i])
        binding.solve_into(batch.dims(i), m[:n * n], s[:n * n])
        torch.cuda.synchronize()
        done = binding.clock_now()
        lat[i] = done - arrive[i]
        last_done = done
        if i in keep:
            outputs[i] = (m[:n * n].view(n, n).cpu().numpy(), s[:n * n].view(n, n).cpu().numpy())
    return ServeResult(latencies=lat, makespan=last_done - t0, count=count, outputs=outputs)
