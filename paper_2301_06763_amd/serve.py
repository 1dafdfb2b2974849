"""Driver for the continuous-batching serving loop of libnmc.

The scheduling itself (admission by HBM footprint, grouping by N and
precision, launching on the library's serving streams, retiring finished
batches) is native (nmc_serve_* in include/nmc.h); this module only feeds
requests at their arrival times and records completion times on the host.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class ServeResult:
    arrivals: np.ndarray          # s, relative to the start
    completions: np.ndarray       # s, relative to the start
    wall_s: float
    stats: dict = field(default_factory=dict)

    @property
    def latencies_ms(self) -> np.ndarray:
        return (self.completions - self.arrivals) * 1e3

    def summary(self) -> dict:
        lat = np.sort(self.latencies_ms)
        n = len(lat)
        q = lambda p: float(lat[min(n - 1, max(0, int(math.ceil(p / 100 * n)) - 1))])
        return {"requests": n, "solves_per_s": n / self.wall_s, "wall_s": self.wall_s,
                "p50_ms": q(50), "p99_ms": q(99), "mean_ms": float(lat.mean()), "max_ms": float(lat[-1])}


def poisson_arrivals(n: int, rate: float, seed: int = 5) -> np.ndarray:
    """Arrival times (s) of a Poisson process of the given rate (rate <= 0 or
    inf: everything at t = 0)."""
    if not rate or rate == float("inf") or rate <= 0:
        return np.zeros(n)
    gaps = np.random.default_rng(seed).exponential(1.0 / rate, size=n)
    return np.cumsum(gaps) - gaps[0]


def run_stream(ctx, requests, arrivals, outs=None) -> ServeResult:
    """Submit requests[i] = (rho, h0, G, flags) at arrivals[i] (seconds after
    start), tick the native scheduler continuously, and record when each one
    completes.  Returns arrival and completion times."""
    import torch
    n = len(requests)
    order = np.argsort(arrivals, kind="stable")
    comp = np.full(n, np.nan)
    ticket_of = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nxt = 0
    done = 0
    while done < n:
        now = time.perf_counter() - t0
        while nxt < n and arrivals[order[nxt]] <= now:
            i = int(order[nxt])
            rho, h0, G, flags = requests[i]
            out = outs[i] if outs is not None else None
            tk = ctx.submit(rho, h0, G, flags, out=out)
            ticket_of[tk.id] = i
            nxt += 1
        for t in ctx.take_completed():
            comp[ticket_of.pop(t)] = time.perf_counter() - t0
            done += 1
    wall = time.perf_counter() - t0
    return ServeResult(np.asarray(arrivals, dtype=float), comp, wall, ctx.stats())


def one_at_a_time(ctx, requests, outs=None, sync_each: bool = True):
    """Solve requests one after another (each synchronised), returning the
    per-request service times in seconds."""
    import torch
    svc = np.zeros(len(requests))
    torch.cuda.synchronize()
    for i, (rho, h0, G, flags) in enumerate(requests):
        t = time.perf_counter()
        ctx.solve(rho, h0, G, flags, out=None if outs is None else outs[i])
        if sync_each:
            torch.cuda.synchronize()
        svc[i] = time.perf_counter() - t
    return svc


def fifo_latencies(arrivals: np.ndarray, service: np.ndarray) -> np.ndarray:
    """Completion times of a single FIFO server with the given service times
    (one request at a time, in arrival order)."""
    order = np.argsort(arrivals, kind="stable")
    comp = np.zeros_like(arrivals, dtype=float)
    t = 0.0
    for i in order:
        t = max(t, arrivals[i]) + service[i]
        comp[i] = t
    return comp
