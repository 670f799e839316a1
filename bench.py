#!/usr/bin/env python3
"""Throughput of the split-operator step on one MI355X.

Workload: the 3D soft-core atom in a pulse, 512^3 points on [-40, 40)^3,
V = -1/sqrt(r^2 + 1) + E(t) z, E(t) = 0.05 exp(-((t-10)/4)^2) cos(1.5 t),
Gaussian start (sigma 1 at the origin), dt = 0.01, FP32 state with FP64 phase
arguments.  One bench step = one full time step of that grid (four line
passes in the steady state).  The state is resident in HBM when timing starts.

Prints one JSON line: site-steps/s of the FP32 path, the FP64 path beside it,
the roofline of the dominant kernel (device time from HIP events attached to
each of its launches inside real steps), the FP32-vs-FP64 error of the run, and the CPU oracle timed on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import re

import numpy as np
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
METRIC = "site-steps/s at 3D 512³ FP32 vs FP64; p50/p99 latency of served solves"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SOURCES = ("paper_1306_3247_amd/csrc/wp_kernels.hip", "paper_1306_3247_amd/csrc/wp_device.hpp",
                  "paper_1306_3247_amd/csrc/wp_internal.hpp", "paper_1306_3247_amd/csrc/wp_pass.hpp",
                  "paper_1306_3247_amd/csrc/wp_pass_c64.hip", "paper_1306_3247_amd/csrc/wp_pass_c64_t1.hip",
                  "paper_1306_3247_amd/csrc/wp_pass_c64_t2.hip", "paper_1306_3247_amd/csrc/wp_pass_c64_t3.hip",
                  "paper_1306_3247_amd/csrc/wp_pass_c128.hip", "paper_1306_3247_amd/csrc/wp_pass_c128_t2.hip")
BYTES_PER_POINT = {"c64": 8, "c128": 16}


def code_only(text: str) -> str:
    """C++ source without its comments, whitespace runs collapsed: what a
    change to the kernels' code changes and a change to their comments does
    not.  (String literals in the kernel sources hold no comment markers.)"""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), encoding="utf-8") as f:
            h.update(code_only(f.read()).encode())
    return h.hexdigest()[:16]


def traffic_for(kind: str, workload: str, precision: str, tune: int = 0):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel sources; else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash():
        return None
    e = t.get("entries", {}).get(f"{workload}:{precision}:{kind}:t{tune}")
    return None if e is None else e.get("bytes_per_launch")


def roofline_of(S, s, precision: str, prob, workload: str, warmup: int, profile_steps: int, pass_reps: int):
    """Roofline of the dominant kernel of a handle's step, timed live inside
    real steps: every launch of `profile_steps` steps carries an event pair
    attached to its own dispatch (wp_profile_propagate), so the pair spans
    exactly that kernel and nothing is enqueued between kernels.  A
    first-axis pass covers the whole grid; a middle pass covers one x slab
    of it.  Each pass reads and writes its part of the state once: the
    algorithmic bytes of a launch are 2 x the bytes it covers.  With more
    than one slab the slabs alternate between two streams, so middle-pass
    launches overlap and their in-step durations are not device time per
    step; the dominant kernel is then the potential pass of the first axis,
    the largest kernel of a step and the one that runs alone.  With one
    slab it is the class with the most device time per step.  Each class is
    also launched back to back over the whole grid (wp_time_pass, best of
    three rounds, each from a fresh copy of the solution: repeated
    unnormalised transforms grow the values until they overflow, and passes
    over such data run faster than over a real state).  Leaves the handle's
    state advanced by warmup + profile_steps steps, then overwritten by the
    pass timing (not a solution afterwards)."""
    state_bytes = prob.grid.points() * BYTES_PER_POINT[precision]
    alg_bytes = 2 * state_bytes
    nslab = s.slabs()
    # Warm-up steps queued right before the profiled ones, as before the
    # timed region: after a pause (a host copy) the first-axis launches of a
    # short profiled run measured 0.65-0.67 ms against 0.57-0.59 ms without
    # it (same box; the timed steps and repeats unaffected).
    s.propagate(warmup)
    prof = s.profile_propagate(max(2, profile_steps))  # a steady first-axis pass needs 2 steps
    share = {"axis0": 1, "edge": 1, "mid_fwd": nslab, "last": nslab, "mid_inv": nslab}
    steady = {k: v for k, v in prof.items() if k in (("axis0",) if nslab > 1 else ("axis0", "mid_fwd", "last", "mid_inv"))}
    kind = max(steady, key=lambda k: steady[k][1])
    count, total_ms = steady[kind]
    avg_ms = total_ms / count
    launch_bytes = alg_bytes // share[kind]
    achieved = launch_bytes / (avg_ms / 1e3) / 1e9
    fresh = s.buffer.clone()

    def time_fresh(k):
        s.buffer.copy_(fresh)
        return s.time_pass(k, pass_reps)

    timed = {k: min(time_fresh(k) for _ in range(3)) for k in ("axis0", "mid_fwd", "last", "mid_inv")}
    del fresh
    lg = int(np.log2(prob.grid.n[0]))
    tp = "c128" if precision == "c128" else "c64"
    variant = {"axis0": S.tune_get(False, tp, lg, True, "potential"),
               "mid_fwd": S.tune_get(False, tp, lg, True, "fft"),
               "mid_inv": S.tune_get(False, tp, lg, True, "fft"),
               "last": S.tune_get(False, tp, lg, False, "kinetic")}
    traffic = traffic_for(kind, workload, precision, variant[kind]) if share[kind] == 1 else None
    return {"bound": "hbm", "kernel": f"pass:{kind}", "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic, "variant": variant[kind], "avg_launch_ms": round(avg_ms, 4),
            "launches": count, "alg_bytes_per_launch": launch_bytes, "slabs": nslab,
            "timing": "in-step, dispatch-attached events",
            "passes_in_step": {k: {"launches": c, "avg_ms": round(m / c, 4),
                                   "GB/s": round(alg_bytes / share.get(k, 1) / (m / c / 1e3) / 1e9, 1)
                                   if k in share else None}
                               for k, (c, m) in prof.items()},
            "passes_back_to_back": {k: {"avg_ms": round(m, 4), "GB/s": round(alg_bytes / (m / 1e3) / 1e9, 1)}
                                    for k, m in timed.items()},
            "back_to_back_reps": pass_reps}


def copy_bandwidth(gib: int = 1, reps: int = 10) -> dict:
    """A plain device-to-device copy of `gib` GiB (torch's copy kernel): the
    read-and-write bandwidth a streaming kernel can reach on this machine."""
    import torch

    src = torch.ones(gib << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    moved = 2 * src.numel() * 4
    del src, dst
    return {"bytes_per_copy": moved, "ms": round(ms, 4), "GB/s": round(moved / (ms / 1e3) / 1e9, 1),
            "frac_of_peak": round(moved / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}


def full_length_accuracy(S, W, n: int, steps: int) -> dict:
    """The stated run of the 3D workload from the Gaussian start: `steps`
    steps in FP32 and in FP64 (the FP64 state is pinned to the oracle), the
    FP32 error against it over every point, and both norm drifts."""
    import torch

    prob = W.softcore_3d(n=n, steps=steps)
    a = S.from_problem(prob, precision="c64")
    b = S.from_problem(prob, precision="c128")
    t = time.perf_counter()
    for x in (a, b):
        x.propagate(steps)
        x.synchronize()
    el = time.perf_counter() - t
    d = torch.view_as_real(a.state_tensor()).double() - torch.view_as_real(b.state_tensor())
    rel = float(torch.linalg.vector_norm(d) / torch.linalg.vector_norm(torch.view_as_real(b.state_tensor())))
    del d
    n32, n64 = a.observables(1)["norm"], b.observables(1)["norm"]
    a.close()
    b.close()
    torch.cuda.synchronize()
    return {"steps": steps, "t_end": prob.t0 + steps * prob.grid.dt, "rel_l2_f32_vs_f64": rel,
            "norm_drift_f32": abs(n32 - 1.0), "norm_drift_f64": abs(n64 - 1.0),
            "bound_rel_l2_f32": 1e-4, "bound_norm_drift_f32": 1e-5, "wall_s": round(el, 2)}


def time_gpu(sim_mod, prob, precision, steps, warmup, tune_reps=0):
    """Time `steps` steps after `warmup`; with tune_reps > 0 the kernel
    variants are tuned first (before the warm-up, outside the timed region).
    Returns (handle, ms, wall seconds, tuning timings)."""
    import torch

    stream = torch.cuda.current_stream()
    s = sim_mod.from_problem(prob, precision=precision, stream=stream)
    tuned = s.autotune(tune_reps) if tune_reps > 0 else None
    s.propagate(warmup)
    s.synchronize()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    start.record(stream)
    s.propagate(steps)
    end.record(stream)
    end.synchronize()
    wall = time.perf_counter() - w0
    torch.cuda.synchronize()
    return s, start.elapsed_time(end), wall, tuned


def batch_bench(S, W, count: int, steps: int, graph_steps: int, ref_solves: int, ref_steps: int,
                tune_reps: int = 0):
    """The batched workload: `count` independent 2D driven traps of sizes
    {128, 256, 512}^2 (seeded), FP32 state, advanced together; against the
    same solves advanced one by one with FP64 launches (timed on a sample)."""
    import torch

    probs = W.batch_2d(count=count, seed=1306, steps=steps, precision="c64")
    sites = sum(p.grid.points() for p in probs)
    stream = torch.cuda.current_stream()
    sims = [S.from_problem(p, stream=stream) for p in probs]
    b = S.Batch(sims, stream=stream, graph_steps=graph_steps)
    if tune_reps:
        b.autotune(tune_reps)  # states are restored
    b.propagate(graph_steps + 1)  # warm-up: graph capture, first replay
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    b.propagate(steps)
    end.record(stream)
    end.synchronize()
    ms = start.elapsed_time(end)
    b.close()
    # per-solve FP64 launches, one solve after another, on a sample
    sample = probs[:ref_solves]
    ref_sites = sum(p.grid.points() for p in sample)
    refs = [S.from_problem(p, precision="c128", stream=stream) for p in sample]
    refs[0].propagate(2)
    torch.cuda.synchronize()
    start.record(stream)
    for r in refs:
        r.propagate(ref_steps)
    end.record(stream)
    end.synchronize()
    ms_ref = start.elapsed_time(end)
    # accuracy of the batched FP32 results: same solves, same steps, FP64 alone
    errs = []
    for p, s in list(zip(probs, sims))[:4]:
        r = S.from_problem(p, precision="c128", stream=stream)
        r.propagate(graph_steps + 1 + steps)
        a, bb = s.get_state("c128"), r.get_state("c128")
        errs.append(float(np.linalg.norm(a - bb) / np.linalg.norm(bb)))
        r.close()
    for x in sims + refs:
        x.close()
    sizes = {}
    for p in probs:
        sizes[p.grid.n[0]] = sizes.get(p.grid.n[0], 0) + 1
    return {"workload": f"batch_2d_{count}", "solves": count, "sizes": sizes, "sites": sites, "steps": steps,
            "graph_steps": graph_steps, "autotuned": bool(tune_reps), "ms": round(ms, 3),
            "value": sites * steps / (ms / 1e3),
            "unit": "site-steps/s", "dtype": "f32",
            "per_solve_fp64": {"value": ref_sites * ref_steps / (ms_ref / 1e3), "unit": "site-steps/s",
                               "sample": f"{ref_solves} solves x {ref_steps} steps, one after another"},
            "speedup_vs_per_solve_fp64": (sites * steps / (ms / 1e3)) / (ref_sites * ref_steps / (ms_ref / 1e3)),
            "max_rel_l2_vs_fp64": max(errs)}


def sweep_counts(count: int, warm: int, rates, capacity: float, limit_s: float):
    """Requests per arrival rate for a sweep: a stream at rate f * capacity
    takes about (warm + count) / (f * capacity) seconds; if the whole sweep
    would take longer than limit_s (> 0), count and warm shrink by the same
    factor (at least 100 measured and 10 warm-up requests).  Returns (count,
    warm, projected seconds of the asked counts)."""
    projected = sum((warm + count) / (f * capacity) for f in rates)
    if limit_s > 0 and projected > limit_s:
        scale = limit_s / projected
        count, warm = max(100, int(count * scale)), max(10, int(warm * scale))
    return count, warm, projected


def serve_bench(S, W, V, count: int, warm: int, rates, cap_count: int, tick: int, graph_steps: int,
                budget_gib: float, ref_count: int, sweep_seconds: float = 0.0):
    """The serving workload: Poisson request streams (60% 1D 2^10..2^16, 30%
    2D 128..1024^2, 10% 3D 64..256^3, 500..5000 steps, FP32 state) served with
    admission by HBM budget and continuous batching.  Rates are fractions of
    the closed-loop capacity (every request present at time zero).  A stream
    at rate f*C takes about (warm + count)/(f*C) seconds; if the sweep would
    take longer than sweep_seconds, warm and count are scaled down by the
    same factor for every rate (the counts used are reported)."""
    import torch

    kw = dict(budget_bytes=int(budget_gib * (1 << 30)), tick_steps=tick, graph_steps=graph_steps)

    def progress(label):
        def show(done, total, t):
            if done % 100 == 0 or done == total:
                print(f"serving {label}: {done}/{total} results, {t:.1f} s", file=sys.stderr, flush=True)
        return show
    cap_reqs = W.serving_stream(cap_count, float("inf"), seed=1306)
    cap_rep = V.Server(**kw).run(cap_reqs, progress("closed loop"))
    cap = cap_rep.summary()
    # Capacity in requests/s: the saturated throughput in site-steps/s over
    # the mean work of a request of this mix (the mean over a long sample is
    # steadier than the request count of a short closed-loop run).
    mix = W.serving_stream(5000, float("inf"), seed=7)
    mean_work = float(np.mean([r.problem.grid.points() * r.problem.steps for r in mix]))
    C = cap["site_steps_per_s"] / mean_work
    asked = (count, warm)
    count, warm, projected = sweep_counts(count, warm, rates, C, sweep_seconds)
    runs = []
    for i, f in enumerate(rates):
        reqs = W.serving_stream(warm + count, f * C, seed=1306 + 1 + i)
        keep = {r.rid for r in reqs[warm:warm + 3]} if i == 0 else False
        rep = V.Server(keep_results=keep, **kw).run(reqs, progress(f"rate {f:g} C"))
        s = rep.summary(first_rid=warm)
        s.update({"rate_frac": f, "rate_hz": f * C})
        runs.append(s)
        if i == 0:
            kept = [(r, x) for r, x in zip(reqs, rep.served) if x.result is not None]
    # per-solve FP64 launches, one solve after another, on the first requests
    ref = W.serving_stream(ref_count, float("inf"), seed=1306)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t = time.perf_counter()
    ref_sites = 0
    for r in ref:
        s = S.from_problem(r.problem, precision="c128", stream=stream)
        s.propagate(r.problem.steps)
        s.synchronize()
        s.close()
        ref_sites += r.problem.grid.points() * r.problem.steps
    ref_rate = ref_sites / (time.perf_counter() - t)
    # accuracy of served FP32 results against the same solves in FP64
    errs = []
    for r, x in kept:
        s = S.from_problem(r.problem, precision="c128", stream=stream)
        s.propagate(r.problem.steps)
        y = s.get_state("c128")
        s.close()
        errs.append(float(np.linalg.norm(x.result.astype(np.complex128) - y) / np.linalg.norm(y)))
    best = max(runs, key=lambda z: z["site_steps_per_s"])
    return {"workload": "serving_poisson_mixed", "capacity_req_per_s": C, "mean_site_steps_per_request": mean_work,
            "capacity": cap, "requests_per_rate": count, "warmup_per_rate": warm,
            "requests_per_rate_asked": asked[0], "warmup_per_rate_asked": asked[1],
            "sweep_projected_s": round(projected, 1), "sweep_limit_s": sweep_seconds,
            "runs": runs, "tick_steps": tick, "graph_steps": graph_steps, "budget_gib": budget_gib,
            "per_solve_fp64": {"value": ref_rate, "unit": "site-steps/s",
                               "sample": f"first {ref_count} requests of the closed-loop stream, one after another"},
            "speedup_vs_per_solve_fp64": best["site_steps_per_s"] / ref_rate,
            "max_rel_l2_vs_fp64": max(errs) if errs else None,
            "accuracy_sample": [r.problem.name for r, _ in kept]}


def cpu_baseline(S, prob, budget_s: float):
    """The oracle on the host cores over a bounded sample of whole steps of
    the workload; the GPU FP32 and FP64 states after the same steps from the
    same start are compared with the oracle's (the run's error against the
    FP64 oracle at full size)."""
    import oracle

    g = prob.grid
    psi = oracle.gaussian(g, prob.init.center, prob.init.sigma, prob.init.k)
    steps, elapsed = 0, 0.0
    while steps == 0 or elapsed < budget_s * 0.5:
        t0 = time.perf_counter()
        psi = oracle.propagate(g, prob.pot, psi, 1, t0=prob.t0, n0=steps)
        elapsed += time.perf_counter() - t0
        steps += 1
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), model)
    except OSError:
        pass
    base = {"value": g.points() * steps / elapsed, "unit": "site-steps/s", "cores": oracle.num_threads(),
            "kind": "oracle", "cpu": model, "host_cpus": os.cpu_count(),
            "sample": f"{steps} step(s) of the same {'x'.join(map(str, g.shape()))} workload in FP64 "
                      f"from the Gaussian start, {elapsed:.1f} s wall"}
    parity = {"steps": steps, "grid": list(g.shape())}
    ref_norm = float(np.linalg.norm(psi))
    for prec, key in (("c64", "rel_l2_fp32_vs_oracle"), ("c128", "rel_l2_fp64_vs_oracle")):
        s = S.from_problem(prob, precision=prec)
        s.propagate(steps)
        got = s.get_state("c128")
        s.close()
        got -= psi
        parity[key] = float(np.linalg.norm(got)) / ref_norm
        del got
    return base, parity


def small_workloads(S, W, with_oracle: bool):
    """The cache-resident workloads: the driven 1D oscillator (1024 points,
    1000 steps, one workgroup holds the line for every step: latency of one
    solve) and the modulated 2D trap (1024^2, 2000 steps; 8-16 MiB, so the
    memory-side cache, not HBM, serves it), in FP64 and FP32, against the
    oracle (W1 at full length, W2 on a sample of steps)."""
    import torch

    stream = torch.cuda.current_stream()
    out = {}
    for name, make in (("driven_ho_1d_1024", W.driven_ho_1d), ("modulated_trap_2d_1024", W.modulated_trap_2d)):
        row = {}
        for prec in ("c128", "c64"):
            prob = make(precision=prec)
            s = S.from_problem(prob, stream=stream)
            tuned = s.autotune(10) if prob.grid.ndim > 1 else None
            s.propagate(min(100, prob.steps))  # warm-up (the state is reset below)
            s.close()
            times = []
            for _ in range(3):
                s = S.from_problem(prob, stream=stream)
                s.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                s.propagate(prob.steps)
                e1.record(stream)
                e1.synchronize()
                times.append(e0.elapsed_time(e1))
                s.close()
            ms = float(np.median(times))
            sites = prob.grid.points()
            row[prec] = {"steps": prob.steps, "ms_total": round(ms, 3), "us_per_step": round(1e3 * ms / prob.steps, 3),
                         "site_steps_per_s": sites * prob.steps / (ms / 1e3)}
            if tuned:
                row[prec]["autotune_chosen"] = {c: min(r, key=r.get) for c, r in tuned.items()}
            if prob.grid.ndim > 1:
                bps = 32 if prec == "c64" else 64  # two passes x (read + write) per 2D step
                row[prec]["bytes_frac_of_hbm_peak"] = round(bps * sites * prob.steps / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
        if with_oracle:
            import oracle

            prob = make(precision="c128")
            g = prob.grid
            psi = oracle.gaussian(g, prob.init.center, prob.init.sigma, prob.init.k)
            n = prob.steps if g.ndim == 1 else 20
            t = time.perf_counter()
            oracle.propagate(g, prob.pot, psi, n, t0=prob.t0)
            el = time.perf_counter() - t
            row["cpu_oracle"] = {"site_steps_per_s": g.points() * n / el, "steps": n, "cores": oracle.num_threads(),
                                 "wall_s": round(el, 3)}
        out[name] = row
    return out


def mixed_radix(S, W, sizes, steps: int = 20, warmup: int = 5):
    """The 3D soft-core workload at the same spacing (0.15625) on grids whose
    lengths are 7-smooth but not powers of two (the sizes the paper advises
    for the transforms): site-steps/s in FP32 and FP64 state, one step being
    the same four-pass schedule run by the mixed-radix kernels (FP64
    arithmetic in both)."""
    return cube_rates(S, W, sizes, steps, warmup)


def large_grid(S, W, sizes, steps: int = 5, warmup: int = 2):
    """The 3D soft-core workload at the same spacing (0.15625) on cubes far
    beyond 512^3 that one device's memory still holds (2048^3: a 64 GiB FP32
    or 128 GiB FP64 state, one at a time): site-steps/s in FP32 and FP64."""
    import torch

    torch.cuda.empty_cache()
    return cube_rates(S, W, sizes, steps, warmup)


def cube_rates(S, W, sizes, steps: int, warmup: int):
    import torch

    stream = torch.cuda.current_stream()
    out = {}
    for n in sizes:
        row = {}
        for prec in ("c64", "c128"):
            prob = W.softcore_3d(n=n, precision=prec, half_width=n * 0.078125)
            torch.cuda.empty_cache()
            need, (free, _) = S.state_bytes(prob.grid, prec), torch.cuda.mem_get_info()
            if need + (4 << 30) > free:
                # a leg beside the headline: its absence must not cost the line
                row[prec] = {"skipped": f"state {need / 2**30:.0f} GiB, {free / 2**30:.0f} GiB free"}
                continue
            s = S.from_problem(prob, stream=stream)
            s.propagate(warmup)
            s.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            s.propagate(steps)
            e1.record(stream)
            e1.synchronize()
            ms = e0.elapsed_time(e1) / steps
            s.close()
            del s
            torch.cuda.empty_cache()
            row[prec] = {"ms_per_step": round(ms, 4), "site_steps_per_s": n ** 3 / (ms / 1e3),
                         "bytes_frac_of_hbm_peak_4pass": round(4 * 2 * BYTES_PER_POINT[prec] * n ** 3 /
                                                               (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
        out[f"{n}^3"] = row
    return out


def rocprof_summary(base: str, n: int, precision: str = "all") -> int:
    """Summarise the four rocprofv3 runs of this benchmark (kernel trace,
    SQ counters, FETCH_SIZE, WRITE_SIZE, written with -d base/<name> -o
    <name> for name in trace, sq, fetch, write) as markdown on stdout, and
    write base/traffic.json: HBM bytes per full-grid launch of every line-pass
    kernel, each counter scaled by what it reads for the run's 1 GiB device
    copy (--copy-calibration).  With the trace alone, prints per-kernel
    launch counts and times only.  precision "c64" or "c128" keeps the
    tables to the line passes of that state type (traffic.json keeps all)."""
    keep_type = {"c64": "<float,", "c128": "<double,"}.get(precision)

    def shown(k):
        return keep_type is None or keep_type in k or not k.startswith(("pass<", "edge<", "batch<"))
    import collections
    import re
    import sqlite3

    kinds = {"0": "F", "1": "V", "2": "K", "3": "VS", "4": "KS"}
    heads = {"pass_kernel": "pass", "edge_pass_kernel": "edge", "batch_pass_kernel": "batch"}

    def short(name):
        m = re.match(r"void wp::(\w*pass_kernel)<(\w+), (\w+), (\d+), (\w+), (\d), (\d)>", name)
        if m and m.group(1) in heads:
            lay = "strided" if m.group(5) == "true" else "contig"
            return f"{heads[m.group(1)]}<{m.group(2)},{m.group(3)},{m.group(4)},{lay},{kinds[m.group(6)]},t{m.group(7)}>"
        return name.split("(")[0].replace("void ", "")[:60]

    def db(name):
        return sqlite3.connect(os.path.join(base, name, f"{name}_results.db"))

    # Launch order of the trace: runs of three or more consecutive launches
    # of one kernel on one stream are back-to-back timing (variant tuning,
    # isolated pass timing); shorter runs are launches inside steps (two in
    # a row where the inverse middle pass of one x slab meets the forward
    # pass of the next).  Runs are counted per stream (the two slab streams
    # interleave).  Rows are per kernel and launch size (grid), so that slab
    # launches and full-grid launches are not averaged together.
    def cols(name, view):
        return [r[1] for r in db(name).execute(f"pragma table_info({view})")]

    tcols = cols("trace", "kernels")
    skey = next((c for c in ("stream_id", "queue_id") if c in tcols), "0")
    gkey = next((c for c in ("grid_x", "grid_size") if c in tcols), "0")
    per_stream = collections.defaultdict(list)
    full = {}
    for nm, d, sid, g in db("trace").execute(f"select name, duration, {skey}, {gkey} from kernels order by start"):
        per_stream[sid].append(((short(nm), g), d))
        full[short(nm)] = nm
    dur = collections.defaultdict(list)
    ctx = collections.defaultdict(lambda: {"step": [], "b2b": []})
    for seq in per_stream.values():
        i = 0
        while i < len(seq):
            j = i
            while j < len(seq) and seq[j][0][0] == seq[i][0][0]:
                j += 1
            for key, d in seq[i:j]:
                dur[key].append(d)
                ctx[key]["step" if j - i < 3 else "b2b"].append(d)
            i = j

    mean = lambda xs: sum(xs) / len(xs) if xs else float("nan")
    if not os.path.exists(os.path.join(base, "sq")):
        print("| kernel | grid (threads) | launches | avg µs | total ms | in-step launches | in-step avg µs "
              "| back-to-back avg µs |")
        print("|---|---|---|---|---|---|---|---|")
        # every launch size of the single-grid line passes, then the other
        # kernels (batched passes, solves, reductions) with the most time
        passes = sorted((kv for kv in dur.items() if kv[0][0].startswith(("pass<", "edge<"))),
                        key=lambda kv: (kv[0][0], -kv[0][1]))
        others = sorted((kv for kv in dur.items() if not kv[0][0].startswith(("pass<", "edge<"))),
                        key=lambda kv: -sum(kv[1]))[:20]
        for (k, g), ds in passes + others:
            if not shown(k):
                continue
            c = ctx[(k, g)]
            print(f"| `{k}` | {g} | {len(ds)} | {mean(ds) / 1e3:.1f} | {sum(ds) / 1e6:.2f} | "
                  f"{len(c['step'])} | {mean(c['step']) / 1e3:.1f} | {mean(c['b2b']) / 1e3:.1f} |")
        return 0

    def counters(name):
        cc = cols(name, "counters_collection")
        g = next((c for c in ("grid_size", "grid_x", "grid_size_x") if c in cc), "0")
        per = collections.defaultdict(lambda: collections.defaultdict(list))
        q = (f"select dispatch_id, kernel_name, counter_name, sum(value), max({g}) from counters_collection "
             "group by dispatch_id, counter_name")
        for _, k, c, v, gs in db(name).execute(q).fetchall():
            per[(short(k), gs)][c].append(v)
        return per

    sq, fe, wr = counters("sq"), counters("fetch"), counters("write")
    # Every 1 GiB device copy of the run (the --copy-calibration ones and the
    # copy-bandwidth timing); the median reading, since a dispatch now and
    # then reports the counts of two.
    copy = next(k for k in fe if k[0] == "__amd_rocclr_copyBuffer")
    kib = (1 << 30) / 1024
    med = lambda xs: float(np.median(xs))
    sf = kib / med(fe[copy]["FETCH_SIZE"])
    sw = kib / med(wr[copy]["WRITE_SIZE"])
    print(f"Counter calibration (1 GiB device copies: 1 GiB read, 1 GiB written each): FETCH_SIZE reads "
          f"{med(fe[copy]['FETCH_SIZE']):.0f} KiB (median of {len(fe[copy]['FETCH_SIZE'])} copies; "
          f"{min(fe[copy]['FETCH_SIZE']):.0f}..{max(fe[copy]['FETCH_SIZE']):.0f}) -> scale {sf:.4f}; WRITE_SIZE reads "
          f"{med(wr[copy]['WRITE_SIZE']):.0f} KiB ({min(wr[copy]['WRITE_SIZE']):.0f}..{max(wr[copy]['WRITE_SIZE']):.0f}) "
          f"-> scale {sw:.4f}.")
    print()
    print("| kernel | part of grid | launches | avg µs | in-step launches | in-step avg µs | back-to-back avg µs "
          "| HBM read GB/launch | HBM write GB/launch | GB/s | LDS conflict cycles / LDS instr | VALU instr / wave |")
    print("|---|---|---|---|---|---|---|---|---|---|---|---|")
    workload = f"softcore_3d_{n}"
    classes = {"passV": ("axis0",), "edgeV": ("edge",), "passF": ("mid_fwd", "mid_inv"), "passK": ("last",)}
    # storage type of a pass kernel -> precision of the handle and bytes of its state
    prec_of = {"float": ("c64", 8 * n ** 3), "double": ("c128", 16 * n ** 3)}
    gmax = collections.defaultdict(int)
    for k, g in dur:
        gmax[k] = max(gmax[k], g)
    entries = {}
    for (k, g), ds in sorted(dur.items(), key=lambda kv: (kv[0][0], -kv[0][1])):
        if "wp::" not in k and "pass<" not in k and "edge<" not in k:
            continue
        rd = [v * 1024 * sf for v in fe[(k, g)]["FETCH_SIZE"]]
        wt = [v * 1024 * sw for v in wr[(k, g)]["WRITE_SIZE"]]
        r, w = mean(rd) / 1e9, mean(wt) / 1e9
        q = sq[(k, g)]
        conf = mean(q["SQ_LDS_BANK_CONFLICT"]) / max(1.0, mean(q["SQ_INSTS_LDS"])) if q["SQ_INSTS_LDS"] else float("nan")
        vpw = mean(q["SQ_INSTS_VALU"]) / max(1.0, mean(q["SQ_WAVES"])) if q["SQ_WAVES"] else float("nan")
        c = ctx[(k, g)]
        part = "1" if g == gmax[k] else f"1/{gmax[k] // max(1, g)}"
        if shown(k):
            print(f"| `{k}` | {part} | {len(ds)} | {mean(ds) / 1e3:.1f} | {len(c['step'])} | "
                  f"{mean(c['step']) / 1e3:.1f} | {mean(c['b2b']) / 1e3:.1f} | {r:.3f} | {w:.3f} | "
                  f"{(r + w) / (mean(ds) * 1e-9):.0f} | {conf:.3f} | {vpw:.0f} |")
        m = re.match(r"(pass|edge)<(float|double),(float|double),\d+,\w+,(\w+),t(\d)>", k)
        cls = m and classes.get(m.group(1) + m.group(4))
        prec, state = prec_of[m.group(2)] if m else (None, 0)
        if m and m.group(2) == "float" and m.group(3) == "double":
            prec = "c64x"
        if cls and rd and wt and g == gmax[k] and mean(rd) >= 0.75 * state:
            e = {"kernel": full[k], "read_bytes": int(mean(rd)), "write_bytes": int(mean(wt)),
                 "launches": len(rd), "avg_us": round(mean(ds) / 1e3, 1)}
            e["bytes_per_launch"] = e["read_bytes"] + e["write_bytes"]
            for cl in cls:
                entries[f"{workload}:{prec}:{cl}:t{m.group(5)}"] = e
    print()
    print("Raw SQ counters (mean per dispatch, per kernel and grid):")
    print()
    print("```")
    for (k, g), q in sorted(sq.items()):
        if ("pass<" in k or "edge<" in k or "wp::" in k) and shown(k):
            print(f"{k} grid {g}: " + ", ".join(f"{c}={mean(v):.4g}" for c, v in sorted(q.items())))
    print("```")
    with open(os.path.join(base, "traffic.json"), "w") as f:
        json.dump({"kernel_hash": kernel_hash(), "source": "profiles/pass_kernels_softcore_3d_512_*.md",
                   "scale": {"FETCH_SIZE": round(sf, 4), "WRITE_SIZE": round(sw, 4)}, "entries": entries},
                  f, indent=1)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=512, help="points per axis")
    ap.add_argument("--profile-steps", type=int, default=10, help="steps of the per-launch event breakdown")
    ap.add_argument("--pass-reps", type=int, default=20, help="back-to-back launches per timed pass class")
    ap.add_argument("--no-autotune", action="store_true", help="run the default kernel variants")
    ap.add_argument("--tune-reps", type=int, default=10)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--also-c64x", action="store_true", help="also time the FP32-state / FP64-arithmetic mode")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-solves", type=int, default=256)
    ap.add_argument("--batch-steps", type=int, default=1000)
    ap.add_argument("--batch-graph-steps", type=int, default=16)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=1000, help="measured requests per arrival rate")
    ap.add_argument("--serve-warmup", type=int, default=100, help="requests served before the measured ones")
    ap.add_argument("--serve-rates", type=str, default="0.25,0.5,0.75,0.9,1.1",
                    help="fractions of the closed-loop capacity")
    ap.add_argument("--serve-seconds", type=float, default=180.0,
                    help="projected wall time of the arrival-rate sweep: if the asked request counts would take "
                         "longer at the measured capacity, they are scaled down alike for every rate (0: no limit)")
    ap.add_argument("--accuracy-steps", type=int, default=2000,
                    help="steps of the full-length FP32-vs-FP64 run of the 3D workload (0: skip)")
    ap.add_argument("--serve-capacity-requests", type=int, default=200)
    ap.add_argument("--serve-tick", type=int, default=250)
    ap.add_argument("--serve-graph-steps", type=int, default=16)
    ap.add_argument("--serve-budget-gib", type=float, default=192.0)
    ap.add_argument("--small-workloads", action=argparse.BooleanOptionalAction, default=True,
                    help="also time the 1D (1024 points) and 2D (1024^2) workloads and their oracle")
    ap.add_argument("--mixed-radix", type=str, default="480",
                    help="comma-separated 7-smooth axis lengths: also time the 3D workload on those cubes "
                         "('' to skip)")
    ap.add_argument("--large-grid", type=str, default="2048",
                    help="comma-separated power-of-two axis lengths: also time the 3D workload on those cubes, "
                         "one state at a time ('' to skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (for scaling HBM byte counters)")
    ap.add_argument("--summary-precision", choices=("all", "c64", "c128"), default="all",
                    help="with --rocprof-summary: tables of the line passes of this state type only")
    ap.add_argument("--rocprof-summary", metavar="DIR",
                    help="summarise the rocprofv3 runs under DIR (no GPU work) and exit")
    args = ap.parse_args()
    if args.rocprof_summary:
        return rocprof_summary(args.rocprof_summary, args.n, args.summary_precision)

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU: this build has no multi-GPU path "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE {world}).", file=sys.stderr)
        return 2

    import torch

    from paper_1306_3247_amd import sim as S
    from paper_1306_3247_amd import workloads as W

    if args.copy_calibration:
        # A plain copy of known size: its FETCH_SIZE / WRITE_SIZE counters
        # (1 GiB each) calibrate the counter readings of the pass kernels.
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    prob = W.softcore_3d(n=args.n, precision="c64")
    workload = f"softcore_3d_{args.n}"
    sites = prob.grid.points()

    tune_reps = 0 if args.no_autotune else args.tune_reps
    s32, ms32, wall32, tuned32 = time_gpu(S, prob, "c64", args.steps, args.warmup, tune_reps)
    value = sites * args.steps / (ms32 / 1e3)
    out = {"metric": METRIC, "value": value, "unit": "site-steps/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms32 / args.steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": workload, "grid": list(prob.grid.shape()), "box": [-40.0, 40.0],
                      "dt": prob.grid.dt, "state": "complex64", "phase_args": "f64"},
           "wall_s_timed": round(wall32, 4)}
    if tuned32:
        out["autotune"] = {"reps": tune_reps,
                           "ms": {c: {str(v): round(m, 4) for v, m in row.items()} for c, row in tuned32.items()},
                           "chosen": {c: min(row, key=row.get) for c, row in tuned32.items()}}

    # The state after the timed steps, kept (in host memory) for the
    # FP32-vs-FP64 comparison of the timed run below: the roofline run
    # advances the handle's state.
    state32 = s32.get_state("c64") if not args.no_fp64 else None
    drift32 = abs(s32.observables(1)["norm"] - 1.0)
    # The timed region again, five more times, continuing the same solution
    # (after warm-up steps queued without a pause, as before the timed
    # region): the spread of the headline figure.
    s32.propagate(args.warmup)
    reps = []
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(5):
        ev0.record(stream)
        s32.propagate(args.steps)
        ev1.record(stream)
        ev1.synchronize()
        reps.append(ev0.elapsed_time(ev1) / args.steps)
    out["repeats"] = {"ms_per_step": [round(x, 4) for x in reps], "median_ms_per_step": round(float(np.median(reps)), 4),
                      "steps_each": args.steps}
    out["roofline"] = roofline_of(S, s32, "c64", prob, workload, args.warmup, args.profile_steps, args.pass_reps)
    # Whole-step view against the 4-pass byte model (64 B per site-step), and
    # against the compulsory floor of one read and one write per step (16 B):
    # the slabs keep part of the middle passes' traffic in the memory-side
    # cache, so the passes move less than 4 x 16 B through HBM.
    alg_bytes = 2 * sites * BYTES_PER_POINT["c64"]
    step_gbs = 4 * alg_bytes * args.steps / (ms32 / 1e3) / 1e9
    out["step_roofline"] = {"model": "4 passes x (read+write) per step", "achieved": round(step_gbs, 1),
                            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(step_gbs / HBM_PEAK_GBS, 4),
                            "floor_16B_frac": round(step_gbs / 4 / HBM_PEAK_GBS, 4)}
    s32.close()
    torch.cuda.synchronize()
    # What a plain streaming copy reaches on this machine, beside the 8 TB/s peak.
    out["hbm_copy"] = copy_bandwidth()
    out["roofline"]["frac_of_copy"] = round(out["roofline"]["achieved"] / out["hbm_copy"]["GB/s"], 4)
    if not args.no_fp64:
        # Same start, same number of steps, FP64 state: the FP32 error of the
        # timed run; then the FP64 dominant kernel's roofline.
        s64, ms64, _, tuned64 = time_gpu(S, prob, "c128", args.steps, args.warmup, tune_reps)
        b = s64.get_state("c128")

        def err(psi32):
            return float(np.linalg.norm(psi32.astype(np.complex128) - b) / np.linalg.norm(b))

        out["fp64"] = {"value": sites * args.steps / (ms64 / 1e3), "ms_per_step": ms64 / args.steps,
                       "dtype": "f64"}
        if tuned64:
            out["fp64"]["autotune_chosen"] = {c: min(row, key=row.get) for c, row in tuned64.items()}
        out["accuracy_timed_run"] = {"steps": args.warmup + args.steps, "rel_l2_f32_vs_f64": err(state32),
                                     "norm_drift_f32": drift32,
                                     "norm_drift_f64": abs(s64.observables(1)["norm"] - 1.0)}
        if args.also_c64x:
            sx, msx, _, _ = time_gpu(S, prob, "c64x", args.steps, args.warmup)
            relx, driftx = err(sx.get_state("c64")), abs(sx.observables(1)["norm"] - 1.0)
            out["c64x"] = {"value": sites * args.steps / (msx / 1e3), "ms_per_step": msx / args.steps,
                           "dtype": "f64 arithmetic, f32 state", "rel_l2_vs_f64": relx, "norm_drift": driftx,
                           "passes": {k: round(m / c, 4) for k, (c, m) in sx.profile_propagate(4).items()}}
            sx.close()
        del state32, b
        out["fp64"]["roofline"] = roofline_of(S, s64, "c128", prob, workload, args.warmup, args.profile_steps,
                                              args.pass_reps)
        out["fp64"]["roofline"]["frac_of_copy"] = round(out["fp64"]["roofline"]["achieved"] / out["hbm_copy"]["GB/s"], 4)
        s64.close()
        torch.cuda.synchronize()
        if args.accuracy_steps > 0:
            out["accuracy"] = full_length_accuracy(S, W, args.n, args.accuracy_steps)

    def leg(name, fn):
        """A leg beside the headline: a Python-level failure in it (say, an
        allocation the device cannot serve) is reported in its field and on
        stderr instead of costing the whole line."""
        try:
            out[name] = fn()
        except Exception as e:  # noqa: BLE001 - reported, not hidden
            import traceback

            traceback.print_exc()
            out[name] = {"error": f"{type(e).__name__}: {e}"}

    if not args.no_batch:
        leg("batch", lambda: batch_bench(S, W, args.batch_solves, args.batch_steps, args.batch_graph_steps, 32, 200,
                                         tune_reps))
    if not args.no_serve:
        from paper_1306_3247_amd import serve as V

        rates = [float(x) for x in args.serve_rates.split(",") if x]
        leg("serving", lambda: serve_bench(S, W, V, args.serve_requests, args.serve_warmup, rates,
                                           args.serve_capacity_requests, args.serve_tick, args.serve_graph_steps,
                                           args.serve_budget_gib, 20, args.serve_seconds))
    if args.small_workloads:
        leg("small_workloads", lambda: small_workloads(S, W, not args.no_cpu_baseline))
    if args.mixed_radix:
        leg("mixed_radix", lambda: mixed_radix(S, W, [int(x) for x in args.mixed_radix.split(",") if x]))
    if args.large_grid:
        leg("large_grid", lambda: large_grid(S, W, [int(x) for x in args.large_grid.split(",") if x]))
    if not args.no_cpu_baseline:
        def cpu():
            base, parity = cpu_baseline(S, W.softcore_3d(n=args.n, precision="c128"), args.cpu_seconds)
            out["oracle_parity"] = parity
            return base

        leg("cpu_baseline", cpu)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
