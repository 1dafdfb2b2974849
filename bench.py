#!/usr/bin/env python3
"""Benchmark of the nested-mesh convolution solver on one MI355X.

One step = one complete nested solve (restriction, the five FFT passes over
all 2L-1 grids, carry cascade and assembly) of a synthetic density already
resident in HBM.  Prints ONE JSON line (see --help for the workloads).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s

WORKLOADS = {
    # name: (description, N, L)
    "plummer32": ("Plummer sphere M=1 a=0.05, 3 levels of 32^3", 32, 3),
    "ellipsoid64": ("homogeneous ellipsoid 0.08/0.05/0.03 + 1% noise, 5 levels of 64^3", 64, 5),
    "binary128": ("Plummer pair 1 + 0.5 at +-3 finest cells, 8 levels of 128^3", 128, 8),
    "clumps256": ("64 Plummer clumps, 6 levels of 256^3", 256, 6),
}


# default timed solves per precision (about 50-100 ms of work each)
WORKLOAD_STEPS = {"plummer32": 500, "ellipsoid64": 400, "binary128": 50, "clumps256": 10}


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed solves (default: about 50 ms of work per precision for the workload)")
    ap.add_argument("--flags", type=int, default=0, help="nmc flag bits passed to every solve")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="clumps256", choices=sorted(WORKLOADS) + ["serving", "copyref"])
    ap.add_argument("--requests", type=int, default=1000, help="serving: number of requests")
    ap.add_argument("--budget-gb", type=float, default=24.0, help="serving: HBM admission budget")
    ap.add_argument("--dtype", default="f64", choices=["f32", "f64"],
                    help="precision of the primary line (the other is reported beside it)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="wall-clock budget of the CPU oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--side", default="binary128",
                    help="workload reported in a sub-object beside the primary one ('none' to skip)")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the serving sub-object of a solve workload's line")
    ap.add_argument("--no-oracle-check", action="store_true")
    a = ap.parse_args()
    if a.steps is None:
        a.steps = WORKLOAD_STEPS.get(a.workload, 20)
        if a.workload in ("serving",):
            a.steps = a.requests
        if a.workload == "copyref":
            a.steps = 10
    return a


def time_solves(ctx, rho, h0, steps, warmup, torch, flags=0):
    """Timed region: `steps` solves back to back (repeated calls replay the
    captured graph).  Then the same `steps` solves again with per-pass HIP
    events recorded by the library on its launch stream (direct launches)."""
    out = torch.empty_like(rho)
    for _ in range(warmup):
        ctx.solve(rho, h0, flags=flags, out=out)
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        starts[k].record()
        ctx.solve(rho, h0, flags=flags, out=out)
        ends[k].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lat = sorted(s.elapsed_time(e) for s, e in zip(starts, ends))
    ctx.profile(True)
    torch.cuda.synchronize()
    for k in range(steps):
        ctx.solve(rho, h0, flags=flags, out=out)
    torch.cuda.synchronize()
    prof = ctx.profile_read()
    ctx.profile(False)
    return out, (t1 - t0), prof, lat


def time_acceleration(ctx, phi, h0, steps, torch):
    """nmc_acceleration on a solved potential (a separate entry point, not part
    of the solve step): kernel time per call from the library's per-pass
    events, and its algorithmic bytes (potential read, three components
    written)."""
    g = ctx.acceleration(phi, h0)
    torch.cuda.synchronize()
    ctx.profile(True)
    for _ in range(steps):
        ctx.acceleration(phi, h0, out=g)
    torch.cuda.synchronize()
    st = ctx.profile_read()["acceleration"]
    ctx.profile(False)
    ms = st["total_ms"] / st["launches"]
    gbs = st["bytes"] / st["launches"] / (ms * 1e-3) / 1e9
    return {"avg_launch_ms": round(ms, 5), "GB_s": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
            "algo_bytes_per_launch": int(st["bytes"] / st["launches"])}


def pct(v, q):
    if not v:
        return None
    i = min(len(v) - 1, max(0, int(math.ceil(q / 100.0 * len(v))) - 1))
    return v[i]


def pass_table(prof):
    tab = {}
    for name, st in prof.items():
        if st["launches"] == 0:
            continue
        ms = st["total_ms"] / st["launches"]
        by = st["bytes"] / st["launches"]
        gbs = by / (ms * 1e-3) / 1e9 if ms > 0 else None
        tab[name] = {"launches": st["launches"], "avg_ms": round(ms, 5), "algo_MB_per_launch": round(by / 1e6, 3),
                     "GB_s": round(gbs, 1) if gbs else None,
                     "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 4) if gbs else None}
    return tab


ROOT = os.path.dirname(os.path.abspath(__file__))
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "z_pass_traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2301_06763_amd", "csrc", f) for f in ("kernels.hip", "fft_core.hpp", "kernels.h")]


def kernel_source_hash() -> str:
    """SHA-256 of the kernel sources with comments and blank space removed
    (an edit of a comment leaves the counters valid; any code change does
    not)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, encoding="utf-8") as fh:
            code = fh.read()
        code = re.sub(r"/\*.*?\*/", " ", code, flags=re.S)
        code = re.sub(r"//[^\n]*", " ", code)
        h.update(" ".join(code.split()).encode())
    return h.hexdigest()


def measured_traffic(workload: str, dtype: str):
    """HBM bytes per z-pass launch from the committed rocprofv3 counter runs
    (FETCH_SIZE and WRITE_SIZE, each scaled by the same counter's reading of
    a copy of known size); None when the kernel sources changed since."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256") != kernel_source_hash():
        return None
    e = t.get("entries", {}).get(f"{workload}/{dtype}")
    return None if e is None else int(e["traffic_bytes_per_launch"])


def cpu_oracle_baseline(rho_np, h0, budget_s):
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    import oracle  # test infrastructure: the CPU baseline leg only
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    n = 0
    t0 = time.perf_counter()
    while True:
        oracle.solve(rho_np, h0)
        n += 1
        el = time.perf_counter() - t0
        if el >= budget_s or n >= 50:
            break
    return {"value": round(n / el, 4), "unit": "solves/s", "cores": cores, "kind": "oracle",
            "sample": f"{n} full FP64 solves of the same workload (NumPy/SciPy pocketfft, "
                      f"workers={cores}) in {el:.1f} s"}


def serving_run(args, torch):
    """Continuous-batching serving of a seeded stream of mixed nested solves
    (N in {32, 64, 128}, L in 2..8, 1-4 Plummer/ellipsoid components, FP32),
    against the same requests solved one at a time in FP64.  Returns the
    serving record (saturated rate, p50/p99 under Poisson arrivals, baseline)."""
    import numpy as np
    from paper_2301_06763_amd import inputs, nmc, serve

    n = args.requests
    print(f"serving: generating {n} requests", file=sys.stderr, flush=True)
    ws = [inputs.serving_request(i, device="cuda") for i in range(n)]
    reqs32 = [(w.rho.float().contiguous(), w.h0, 1.0, 0) for w in ws]
    outs = [torch.empty_like(r[0]) for r in reqs32]
    budget = int(args.budget_gb * (1 << 30))
    ctx = nmc.Context(budget_bytes=budget)
    # warm-up: Green spectra of every N, and the workspace pool filled by one
    # untimed pass over the stream (the first pool allocations after the
    # solve workloads' large frees are slow and not part of serving)
    warm = {}
    for i, w in enumerate(ws):
        warm.setdefault(w.N, i)
    for i in warm.values():
        ctx.solve(*reqs32[i][:2])
    torch.cuda.synchronize()
    serve.run_stream(ctx, reqs32, np.zeros(n), outs)
    torch.cuda.synchronize()
    burst = serve.run_stream(ctx, reqs32, np.zeros(n), outs)
    X = burst.summary()["solves_per_s"]
    print(f"serving: saturated {X:.1f} solves/s", file=sys.stderr, flush=True)
    runs = {"burst": burst.summary()}
    for frac in (0.5, 0.9):
        arr = serve.poisson_arrivals(n, frac * X, seed=5)
        r = serve.run_stream(ctx, reqs32, arr, outs)
        runs[f"poisson_{frac}X"] = dict(r.summary(), rate_per_s=frac * X)
        print(f"serving: poisson {frac}X done", file=sys.stderr, flush=True)
    st = ctx.stats()
    # spot check: results in the mix equal the same request solved alone
    same = 0
    picks = list(range(0, n, max(1, n // 16)))
    for i in picks:
        alone = ctx.solve(reqs32[i][0], reqs32[i][1], flags=nmc.NMC_NO_GRAPH)
        torch.cuda.synchronize()
        same += int(torch.equal(alone, outs[i]))
    # baseline: the same requests one at a time in FP64 (each synchronised)
    ctx64 = nmc.Context()
    for i in warm.values():
        ctx64.solve(ws[i].rho, ws[i].h0)
    torch.cuda.synchronize()
    svc = serve.one_at_a_time(ctx64, [(w.rho, w.h0, 1.0, nmc.NMC_NO_GRAPH) for w in ws])
    base = {"solves_per_s": n / svc.sum(), "mean_service_ms": float(svc.mean() * 1e3),
            "latency_model": "p50/p99 under the same Poisson arrivals are computed from the measured "
                             "per-request service times as a single FIFO server (not replayed live)"}
    for frac in (0.5, 0.9):
        arr = serve.poisson_arrivals(n, frac * X, seed=5)
        comp = serve.fifo_latencies(arr, svc)
        lat = np.sort((comp - arr) * 1e3)
        base[f"poisson_{frac}X"] = {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99))}
    ctx.close()
    ctx64.close()
    return {
        "what": "continuous batching of mixed nested solves, FP32 (native scheduler: footprint admission, "
                "grouping by N / precision / method, four serving streams)",
        "workload": {"requests": n, "N": [32, 64, 128], "L": [2, 8], "admission_budget_GB": args.budget_gb,
                     "serving_streams": 4},
        "solves_per_s": round(X, 3), "runs": runs,
        "scheduler": {k: st[k] for k in ("batches", "peak_inflight_bytes", "budget_bytes", "completed")},
        "mix_equals_alone": f"{same}/{len(picks)} bitwise",
        "baseline_one_at_a_time_f64": base,
    }


def bench_serving(args):
    """The serving record as the primary line (--workload serving)."""
    import torch
    rec = serving_run(args, torch)
    X = rec["solves_per_s"]
    line = {
        "metric": "serving: nested-mesh solves/s with p50/p99 latency (continuous batching, FP32)",
        "value": X, "unit": "solves/s", "n_gpus": 1, "steps": args.requests, "warmup": 3,
        "ms_per_step": round(1e3 / X, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic (seeded Plummer/ellipsoid superpositions, inputs resident in HBM)",
        "config": {"workload": "serving", **rec["workload"]},
    }
    line.update({k: v for k, v in rec.items() if k not in ("workload", "solves_per_s")})
    print(json.dumps(line), flush=True)


def copy_bandwidth(torch, reps=20):
    """Attainable HBM rate on this GPU for context beside the 8 TB/s peak:
    a 1 GiB device-to-device copy (1 GiB read + 1 GiB written) timed with
    events on the current stream, median over the repetitions."""
    n = (1 << 30) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    del a, b
    torch.cuda.empty_cache()
    return 2 * (1 << 30) / (pct(sorted(times), 50) * 1e-3) / 1e9


def bench_copyref(args):
    """A plain device copy of known size (1 GiB read + 1 GiB written per
    launch), used to scale the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    n = (1 << 30) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(args.warmup):
        b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.copy_(a)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    gbs = 2 * (1 << 30) * args.steps / el / 1e9
    print(json.dumps({"metric": "device copy GB/s (counter reference)", "value": round(gbs, 1), "unit": "GB/s",
                      "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "bytes_per_launch": 2 << 30,
                      "config": {"workload": "copyref"}}), flush=True)


def z_roofline(prof):
    """The z pass (forward z, Green multiply, inverse z: the dominant kernel)
    of a profiled run: algorithmic bytes per launch over its average launch
    duration (HIP events recorded by the kernel launch itself)."""
    z = prof["z"]
    z_ms = z["total_ms"] / z["launches"]
    z_bytes = z["bytes"] / z["launches"]
    achieved = z_bytes / (z_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "kernel": "k_z (fused forward-z, Green multiply, inverse-z)",
            "avg_launch_ms": round(z_ms, 5), "algo_bytes_per_launch": int(z_bytes), "launches": z["launches"]}


def run_workload(ctx, name, steps, warmup, flags, torch, with_modified=True, with_accel=True):
    """Both precisions of one workload: timed solves, pass table, FP32 error
    against FP64, and (where the scaled grids fit) the modified methods."""
    from paper_2301_06763_amd import inputs, nmc
    desc, N, L = WORKLOADS[name]
    print(f"bench: {name} (N={N}, L={L}): generating input", file=sys.stderr, flush=True)
    w = inputs.WORKLOADS[name](device="cuda")
    res, outs, accel = {}, {}, {}
    modified, mouts, modified3 = {}, {}, {}
    mod_steps = max(10, steps // 4)
    mod3_steps = max(10, steps // 16)
    for tag, dt in (("f64", torch.float64), ("f32", torch.float32)):
        rho = w.rho.to(dt).contiguous()
        out, el, prof, lat = time_solves(ctx, rho, w.h0, steps, warmup, torch, flags)
        print(f"bench: {name} {tag}: {steps / el:.2f} solves/s", file=sys.stderr, flush=True)
        if with_accel:
            accel[tag] = time_acceleration(ctx, out, w.h0, min(steps, 50), torch)
        outs[tag] = out.double()
        res[tag] = {"solves_per_s": steps / el, "ms_per_step": el / steps * 1e3,
                    "passes": pass_table(prof), "lat": lat, "prof": prof}
        if with_modified and 2 * nmc.period(N) <= 1024:  # the modified method's doubled grids fit
            mo, mel, mprof, mlat = time_solves(ctx, rho, w.h0, mod_steps, warmup, torch, flags | nmc.NMC_MODIFIED)
            mouts[tag] = mo.double()
            modified[tag] = {"solves_per_s": round(mod_steps / mel, 3), "ms_per_step": round(mel / mod_steps * 1e3, 4),
                             "latency_ms": {"p50": round(pct(mlat, 50), 4), "p99": round(pct(mlat, 99), 4)},
                             "steps": mod_steps, "passes": pass_table(mprof)}
        if with_modified and L >= 3 and 4 * nmc.period(N) <= 1024:  # quadrupled grids fit
            _, m3el, m3prof, m3lat = time_solves(ctx, rho, w.h0, mod3_steps, warmup, torch,
                                                 flags | nmc.NMC_MODIFIED3)
            modified3[tag] = {"solves_per_s": round(mod3_steps / m3el, 3),
                              "ms_per_step": round(m3el / mod3_steps * 1e3, 4),
                              "latency_ms": {"p50": round(pct(m3lat, 50), 4), "p99": round(pct(m3lat, 99), 4)},
                              "steps": mod3_steps, "passes": pass_table(m3prof)}
        del rho
    # FP32 against the FP64 GPU result (the FP64 path is checked against the oracle in tests)
    e = ((outs["f32"] - outs["f64"]).abs() / outs["f64"].abs())
    err32 = {"max_rel_err": float(e.max()), "rms_rel_err": float(e.pow(2).mean().sqrt()),
             "per_level_max": [float(e[l].max()) for l in range(L)],
             "per_level_rms": [float(e[l].pow(2).mean().sqrt()) for l in range(L)], "tolerance": 1e-5}
    del e
    rec = {"w": w, "desc": desc, "N": N, "L": L, "res": res, "err32": err32, "accel": accel}
    if modified:
        em = ((mouts["f32"] - mouts["f64"]).abs() / mouts["f64"].abs())
        rec["modified"] = {
            "what": "the dipole-preserving method of Sect. 7 / Appendix B (NMC_MODIFIED): per level pair a "
                    "doubled grid of period 2P (2N cells of the finer spacing) in addition to the hole grids; "
                    "z and x..inv_y pass rows mix both periods",
            "doubled_period": 2 * nmc.period(N),
            "f32": modified["f32"], "f64": modified["f64"],
            "fp32_vs_fp64": {"max_rel_err": float(em.max()), "rms_rel_err": float(em.pow(2).mean().sqrt())}}
    if modified3:
        rec["modified3"] = {
            "what": "the three-level dipole scheme of Appendix B (NMC_MODIFIED3): in addition, a quadrupled grid "
                    "of period 4P per level with two finer levels",
            "quadrupled_period": 4 * nmc.period(N), "f32": modified3["f32"], "f64": modified3["f64"]}
    return rec


def precision_summary(r):
    z = z_roofline(r["prof"])
    return {"solves_per_s": round(r["solves_per_s"], 3), "ms_per_step": round(r["ms_per_step"], 4),
            "latency_ms": {"p50": round(pct(r["lat"], 50), 4), "p99": round(pct(r["lat"], 99), 4)},
            "z_pass": {k: z[k] for k in ("achieved", "frac", "avg_launch_ms", "algo_bytes_per_launch")},
            "passes": r["passes"]}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding is a design note, not built.", file=sys.stderr)
        sys.exit(2)
    import torch
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from paper_2301_06763_amd import nmc
    torch.cuda.set_device(0)
    if args.workload == "serving":
        return bench_serving(args)
    if args.workload == "copyref":
        return bench_copyref(args)

    ctx = nmc.Context()
    rec = run_workload(ctx, args.workload, args.steps, args.warmup, args.flags, torch)
    N, L, w = rec["N"], rec["L"], rec["w"]
    res = rec["res"]
    prim = res[args.dtype]
    roofline = z_roofline(prim["prof"])
    roofline["traffic"] = measured_traffic(args.workload, args.dtype)
    roofline["bytes_convention"] = ("per grid (n_in + n_out) P (P/2) complex values moved, the spectrum octant "
                                    "(P/2+1)^3 reals once per launch")
    copy_gbs = copy_bandwidth(torch)
    roofline["copy_GB_s"] = round(copy_gbs, 1)        # measured 1 GiB device copy, same GPU
    roofline["frac_of_copy"] = round(roofline["achieved"] / copy_gbs, 4)
    total_bytes = sum(st["bytes"] for st in prim["prof"].values()) / args.steps
    line = {
        "metric": "nested-mesh solves/s + FFT HBM GB/s, FP32 vs FP64 at \u22641e-5 rel err; p50/p99",
        "value": round(prim["solves_per_s"], 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(prim["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic (seeded analytic densities sampled at cell centres, inputs resident in HBM)",
        "config": {"workload": args.workload, "description": rec["desc"], "N": N, "L": L,
                   "grids_per_solve": 2 * L - 1, "padded_period": nmc.period(N), "batch": 1,
                   "parallelism": "none (1 GPU)"},
        "roofline": roofline,
        "latency_ms": {"p50": round(pct(prim["lat"], 50), 4), "p99": round(pct(prim["lat"], 99), 4)},
        "effective_GB_s": round(total_bytes / (prim["ms_per_step"] * 1e-3) / 1e9, 1),
        "passes": prim["passes"],
        "fp32_vs_fp64": rec["err32"],
        "acceleration": {"what": "nmc_acceleration on the solved potential (six-point stencil with the "
                                 "interface rules of Appendix A); a separate call, not in the solve step",
                         **rec["accel"]},
    }
    other = "f64" if args.dtype == "f32" else "f32"
    line[other] = precision_summary(res[other])
    for k in ("modified", "modified3"):
        if k in rec:
            line[k] = rec[k]
    del rec, res, prim
    if args.side and args.side != "none" and args.side != args.workload:
        side = run_workload(ctx, args.side, max(10, WORKLOAD_STEPS.get(args.side, 20) // 2), args.warmup,
                            args.flags, torch, with_modified=True, with_accel=False)
        line["side"] = {"workload": args.side, "description": side["desc"], "N": side["N"], "L": side["L"],
                        "f64": precision_summary(side["res"]["f64"]), "f32": precision_summary(side["res"]["f32"]),
                        "fp32_vs_fp64": side["err32"]}
        for k in ("modified", "modified3"):
            if k in side:
                line["side"][k] = side[k]
        if "modified3" in side:  # cost of each method against the original (Appendix B quotes x8.5 at N = 128)
            line["side"]["method_cost_ratio"] = {
                tag: {"modified": round(side["res"][tag]["solves_per_s"] / side["modified"][tag]["solves_per_s"], 2),
                      "modified3": round(side["res"][tag]["solves_per_s"] / side["modified3"][tag]["solves_per_s"], 2)}
                for tag in ("f64", "f32")}
        del side
    ctx.close()
    torch.cuda.empty_cache()
    if not args.no_serving:
        line["serving"] = serving_run(args, torch)
    if not args.no_cpu_baseline:
        print("bench: CPU oracle baseline", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_oracle_baseline(w.rho.cpu().numpy(), w.h0, args.cpu_seconds)
        f64_rate = line["value"] if args.dtype == "f64" else line["f64"]["solves_per_s"]
        line["cpu_baseline"]["gpu_speedup_f64"] = round(f64_rate / line["cpu_baseline"]["value"], 1)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
