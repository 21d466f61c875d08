"""Benchmark of the timestep-splitting EM particle step on one MI355X.

Workload (the metric's configuration): the 64-edge Langevin star
(quadratic potentials, sigma = sqrt(2), b = 1/64), 1e7 particles uniform by
length, 1e4 steps at dt = 1e-2 and at dt = 1e-3, 256 bins per edge.  One
benchmark step is one pass of the whole hot path for both dt: particle
initialisation, the fused multi-step kernel, exit counts and the histogram.
The FP32 path is the headline value; the FP64 path is timed beside it and
the FP32 histograms and exit probabilities are compared with FP64's under
common random numbers.

Prints one JSON line.  Only one GPU: --gpus above 1 exits with a message.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particle-substeps/s at 1 GPU, FP32 vs FP64, + % VALU peak at TV≤2e-3"
# VALU lane-operation ceiling of one MI355X: 256 CUs x 4 SIMDs x 32 lane-ops
# per cycle (the 16-lane SIMD issuing packed/dual operations, the width
# behind the 157.3 TFLOP/s FP32 vector figure with FMA = 2 flops) x 2.4 GHz.
PEAK_LANE_OPS = 256 * 4 * 32 * 2.4e9

# Algorithmic VALU operations of the method per unit of work: the minimal
# gfx950 instruction sequence, counted once per instruction whatever its rate.
# FP32 particle-step: 1/4 Philox4x32-10 (10 rounds x 2 multiplies + 2
# three-input xors) = 10; 1/2 Box-Muller pair (2 converts, 2 fma, log, mul,
# sqrt, cos, sin, 2 mul) = 5.5; the first sub-step from per-frame constants
# (2 fma, 2 adds and 2 subtractions of the compensated sum, 2 compares,
# 2 selects) = 10; 1/4 re-anchor (compare, subtraction, 3 selects, xor,
# multiply, select) = 2.
ALG_FP32_STEP = 27.5
ALG_FP32_HIT = 80.0      # per vertex hit: Philox, one normal, root, time, slot, edge
# FP64 particle-step: 1/4 Philox = 10; 1/2 Box-Muller pair (2 converts and
# 2 scalings of the uniforms; the logarithm by an integer range reduction
# and a degree-6 polynomial for the atanh series, 29; the factor -2, 1; the
# square root, 9; the angle, 1; sine and cosine by quarter-turn reduction
# and two degree-5 polynomials, 23; 2 multiplies) = 34.5; the first sub-step
# (2 fma, 2 compares, 2 selects of 64-bit values) = 8.5.
ALG_FP64_STEP = 53.0
ALG_FP64_HIT = 130.0
# cubic drift and diffusion: two Horner steps more for mu and three for
# sigma at every sub-step start (a step, or a restart from a vertex)
ALG_FP64_CUBIC = 5.0
# FP32 with cubic coefficients: the frame position (select, subtraction),
# both cubics (6 fma), the frame sign (2 selects), sigma sqrt(dt) and the
# drift times dt (2 multiplies), against the per-frame constants' 2 fma
ALG_FP32_CUBIC = 10.0


# HBM bytes per k_pool32 launch on this workload from the FETCH_SIZE and
# WRITE_SIZE counter passes (scaled by a 1 GiB copy), valid for the kernel
# source whose sha256 prefix is given; reported as null for any other build.
TRAFFIC = {"kernel_sha256": "ef2cc7cec6d26aa1", "bytes_per_launch": 270.6e6}


def kernel_traffic():
    import hashlib
    src = os.path.join(ROOT, "paper_2512_02175_amd", "csrc", "mg_kernels.hip")
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    return TRAFFIC["bytes_per_launch"] if h == TRAFFIC["kernel_sha256"] else None


def alg_work(prec: int, steps: int, hits: int) -> float:
    if prec == 1:
        return ALG_FP32_STEP * steps + ALG_FP32_HIT * hits
    return ALG_FP64_STEP * steps + ALG_FP64_HIT * hits


def exit_probs(ex, offsets):
    import numpy as np
    p = np.zeros(ex.size)
    for v in range(offsets.size - 1):
        s0, s1 = offsets[v], offsets[v + 1]
        t = ex[s0:s1].sum()
        if t:
            p[s0:s1] = ex[s0:s1] / t
    return p


MIN_EXITS = 10_000


def exit_err(ex_a, ex_b, offsets, min_exits=MIN_EXITS):
    """Exit-probability error of one run against another: the largest
    |p_a - p_b| over the slots of vertices that record at least min_exits
    exits in run b (below that a single differing path moves a probability
    by more than 1e-4), and the exit-weighted mean over all vertices."""
    import numpy as np
    pa, pb = exit_probs(ex_a, offsets), exit_probs(ex_b, offsets)
    worst, num, den = 0.0, 0.0, 0.0
    for v in range(offsets.size - 1):
        s0, s1 = offsets[v], offsets[v + 1]
        tot = float(ex_b[s0:s1].sum())
        if tot == 0.0:
            continue
        d = float(np.abs(pa[s0:s1] - pb[s0:s1]).max())
        num += tot * d
        den += tot
        if tot >= min_exits:
            worst = max(worst, d)
    return worst, (num / den if den else 0.0)


def run_pass(B, G, g, run, prec, dt, torch, kernel_times, schedules=None, schedule=0):
    """One pass of the path at one dt: init, schedule tuning (FP32), simulate,
    exit counts, histogram.  kernel_times gets the HIP-event time of the
    step launches alone."""
    p = B.mg_particles_init(G, run["n_particles"], B.MG_INIT_UNIFORM_LENGTH, init_seed=0,
                            precision=prec, max_splits=run["max_splits"], schedule=schedule)
    launches = 1
    if prec == B.MG_FP32:
        t = B.mg_autotune(p, dt, run["seed"])
        spl = t["steps_per_launch"]
        if spl:
            launches = -(-run["n_steps"] // spl)
        if schedules is not None:
            schedules.append((f"k_pool32 ({t['pool_size']} per wave, {t['window']}-step windows, "
                              f"idle {t['idle_trigger']})"
                              if t["schedule"] != B.MG_SCHED_LANES else "k_step<fp32>")
                             + (f" x{launches} launches of {spl} steps" if spl else ""))
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    B.mg_simulate(p, run["n_steps"], dt, run["seed"])
    e1.record()
    ex, ab, tot = B.mg_exit_counts(p)
    hist = B.mg_histogram(p, run["bins"])
    kernel_times.append(e0.elapsed_time(e1) * 1e-3)
    return dict(substeps=int(tot[1]), hits=int(tot[2]), steps=int(tot[3]),
                trunc=int(tot[0]), exit=ex, hist=hist, launches=launches)


def environment(torch) -> dict:
    """The machine and software a line was measured on."""
    props = torch.cuda.get_device_properties(0)
    return {"gpu": torch.cuda.get_device_name(0),
            "arch": getattr(props, "gcnArchName", None),
            "compute_units": props.multi_processor_count,
            "hbm_gib": round(props.total_memory / 2**30, 1),
            "hip": torch.version.hip, "torch": torch.__version__,
            "host_cpu": _cpu_model(), "host_nproc": os.cpu_count()}


def emit(line: dict, torch) -> None:
    line["env"] = environment(torch)
    print(json.dumps(line), flush=True)


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(g, run, n_sample: int, dt: float = 1e-3, repeats: int = 3,
                 n_single: int | None = None):
    """The oracle timed on the host cores: the median of `repeats` runs of
    particle ids 0..n_sample-1 with all threads (OMP_NUM_THREADS, else every
    core this process may use), and the median of `repeats` single-thread
    runs of the first n_single ids; the particle loop only (the initial
    states are drawn before the clock starts)."""
    import numpy as np
    import oracle
    affinity = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None
    threads = int(os.environ.get("OMP_NUM_THREADS", affinity or os.cpu_count() or 1))
    n_single = n_single or max(1, n_sample // 10)

    def timed(n, th):
        rates, subs, els = [], [], []
        for _ in range(repeats):
            st = oracle.init(g, run["n_particles"], oracle.INIT_UNIFORM_LENGTH, seed=0,
                             pids=np.arange(n))
            t0 = time.perf_counter()
            c = oracle.simulate(g, st, 0, run["n_steps"], dt, run["seed"], threads=th,
                                max_splits=run["max_splits"])
            el = time.perf_counter() - t0
            rates.append(c.substeps / el)
            subs.append(c.substeps)
            els.append(el)
        k = int(np.argsort(rates)[len(rates) // 2])
        return rates[k], subs[k], els[k], rates

    v, sub, el, all_r = timed(n_sample, threads)
    v1, sub1, el1, all_r1 = timed(n_single, 1)
    return {"value": v, "unit": "particle-substeps/s", "cores": threads, "kind": "oracle",
            "sample": f"particle ids 0..{n_sample - 1} of the same workload at dt={dt:.3g}, "
                      f"{run['n_steps']} steps, FP64, median of {repeats} runs "
                      f"({sub} sub-steps in {el:.2f} s)",
            "runs": all_r,
            "single_thread": {"value": v1, "unit": "particle-substeps/s",
                              "sample": f"particle ids 0..{n_single - 1}, median of {repeats} "
                                        f"runs ({sub1} sub-steps in {el1:.2f} s)",
                              "runs": all_r1},
            "nproc": os.cpu_count(), "affinity_cpus": affinity, "cpu_model": _cpu_model()}


def batch_leg(B, torch):
    """The batched form on the default line: 512 independent uneven graphs
    (stars and random recursive trees, 3..4096 edges, 1e4..1e6 particles
    each, half with quadratic potentials), 1000 steps of dt 1e-3 in FP32,
    one batched call (a launch per LDS group) against one launch per graph;
    the batched call's roofline fraction from its HIP-event time."""
    import numpy as np
    import workloads
    graphs, counts, run = workloads.config4()
    Gs = [B.mg_graph_create(g) for g in graphs]

    def make():
        return [B.mg_particles_init(G, c, B.MG_INIT_UNIFORM_LENGTH, init_seed=i, graph_tag=i,
                                    precision=B.MG_FP32, max_splits=run["max_splits"])
                for i, (G, c) in enumerate(zip(Gs, counts))]

    def totals(sets):
        t = np.zeros(4, np.uint64)
        for q in sets:
            t += B.mg_exit_counts(q)[2]
        return t
    sets = make()
    batch = B.mg_batch_create(sets)
    B.mg_batch_simulate(batch, 8, run["dt"], run["seed"])  # builds the launch graph
    torch.cuda.synchronize()
    t_before = totals(sets)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    B.mg_batch_simulate(batch, run["n_steps"], run["dt"], run["seed"])
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    k = e0.elapsed_time(e1) * 1e-3
    tot = totals(sets) - t_before
    solo = make()
    for q in solo:
        B.mg_simulate(q, 8, run["dt"], run["seed"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for q in solo:
        B.mg_simulate(q, run["n_steps"], run["dt"], run["seed"])
    torch.cuda.synchronize()
    wall_solo = time.perf_counter() - t1
    return {"workload": "batch512: 512 stars/random trees, 3..4096 edges, 1e4..1e6 particles "
                        "each, zero drift or quadratic potentials, dt=1e-3, 1000 steps, FP32, "
                        "one batched call (a launch per LDS group)",
            "n_particles": int(sum(counts)), "value": float(tot[1]) / wall,
            "kernel_substeps_per_s": float(tot[1]) / k,
            "unbatched_value": float(tot[1]) / wall_solo, "batch_speedup": wall_solo / wall,
            "roofline_frac": alg_work(1, int(tot[3]), int(tot[2])) / k / PEAK_LANE_OPS,
            "hits_per_step": float(tot[2]) / float(tot[3])}


def at_scale(B, torch):
    """The accuracy targets at 1e8 particles: the synthetic vascular network
    (20k vertices, 26k edges, 1e8 particles uniform by length, 1e4 steps,
    64 bins per edge), FP32 and FP64 from the same initial states and random
    integers; histogram TV, exit-probability error, throughput of both
    precisions and the FP32 kernel's roofline fraction."""
    import numpy as np
    import workloads
    g, run = workloads.config3()
    G = B.mg_graph_create(g)
    n = run["n_particles"]
    res = {}
    for prec in (B.MG_FP32, B.MG_FP64):
        p = B.mg_particles_init(G, n, B.MG_INIT_UNIFORM_LENGTH, init_seed=0, precision=prec,
                                max_splits=run["max_splits"])
        if prec == B.MG_FP32:
            B.mg_autotune(p, run["dt"], run["seed"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        B.mg_simulate(p, run["n_steps"], run["dt"], run["seed"])
        e1.record()
        ex, ab, tot = B.mg_exit_counts(p)
        wall = time.perf_counter() - t0
        res[prec] = dict(k=e0.elapsed_time(e1) * 1e-3, wall=wall, ex=ex, ab=int(ab.sum()),
                         sub=int(tot[1]), hits=int(tot[2]), steps=int(tot[3]),
                         hist=B.mg_histogram(p, run["bins"]))
        del p
    r32, r64 = res[B.MG_FP32], res[B.MG_FP64]
    w, m = exit_err(r32["ex"], r64["ex"], g.vtx_offsets)
    frac = alg_work(1, r32["steps"], r32["hits"]) / r32["k"] / PEAK_LANE_OPS
    return {"workload": "vascular20k: 20k vertices, 26k edges, Poiseuille drift, absorbing "
                        "outlets, 1e8 particles uniform by length, 1e4 steps at 10x the FVM "
                        "CFL dt, 64 bins/edge, M=8",
            "n_particles": n, "n_steps": run["n_steps"], "dt": run["dt"],
            "fp32_substeps_per_s": r32["sub"] / r32["wall"],
            "fp32_kernel_substeps_per_s": r32["sub"] / r32["k"],
            "fp64_substeps_per_s": r64["sub"] / r64["wall"],
            "fp64_kernel_substeps_per_s": r64["sub"] / r64["k"],
            "tv_fp32_vs_fp64": _tv(r32["hist"], r64["hist"]),
            "exit_prob_err_fp32_vs_fp64": w, "exit_prob_err_weighted_mean": m,
            "absorbed_fraction": [r32["ab"] / n, r64["ab"] / n],
            "roofline_frac": frac, "hits_per_step": r32["hits"] / r32["steps"]}


def _tv(a, b):
    import numpy as np
    return 0.5 * float(np.abs(a.astype(float) - b.astype(float)).sum()) / max(float(b.sum()), 1.0)


def run_vascular(args, B, torch):
    """Synthetic vascular network (20k vertices, 26k edges, advective drift,
    absorbing outlets): 1e8 FP32 particles uniform by length, 1e4 steps at
    ten times the upwind finite-volume CFL limit, 64 bins per edge; FP64
    beside it under common random numbers."""
    import numpy as np
    import workloads
    g, run = workloads.config3()
    G = B.mg_graph_create(g)
    n = run["n_particles"]

    scheds = []

    def one(prec, ktimes):
        p = B.mg_particles_init(G, n, B.MG_INIT_UNIFORM_LENGTH, init_seed=0, precision=prec,
                                max_splits=run["max_splits"])
        if prec == B.MG_FP32:
            t = B.mg_autotune(p, run["dt"], run["seed"])
            scheds.append("k_pool32" if t["schedule"] != B.MG_SCHED_LANES else "k_step<fp32>")
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        B.mg_simulate(p, run["n_steps"], run["dt"], run["seed"])
        e1.record()
        ex, ab, tot = B.mg_exit_counts(p)
        h = B.mg_histogram(p, run["bins"])
        ktimes.append(e0.elapsed_time(e1) * 1e-3)
        out = dict(substeps=int(tot[1]), hits=int(tot[2]), steps=int(tot[3]), exit=ex,
                   absorbed=int(ab.sum()), hist=h)
        del p
        return out

    for _ in range(args.warmup):
        one(1, [])
    torch.cuda.synchronize()
    kt = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r32 = one(1, kt)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    value = r32["substeps"] * args.steps / wall
    line = {"metric": METRIC, "value": value, "unit": "particle-substeps/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": "vascular20k: synthetic microvascular network, 20k vertices, "
                                   "26k edges, Poiseuille drift, absorbing outlets, 1e8 particles, "
                                   "1e4 steps of 10x the FVM CFL dt, 64 bins/edge",
                       "dt": run["dt"], "n_particles": n, "n_steps": run["n_steps"]},
            "hits_per_step": r32["hits"] / r32["steps"], "absorbed_fraction": r32["absorbed"] / n,
            "kernel_substeps_per_s": r32["substeps"] / float(np.mean(kt))}
    if not args.no_fp64:
        k64 = []
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        r64 = one(0, k64)
        torch.cuda.synchronize()
        w64 = time.perf_counter() - t1
        line["fp64"] = {"value": r64["substeps"] / w64, "unit": "particle-substeps/s",
                        "fp32_speedup": value / (r64["substeps"] / w64)}
        line["tv_fp32_vs_fp64"] = _tv(r32["hist"], r64["hist"])
        w, m = exit_err(r32["exit"], r64["exit"], g.vtx_offsets)
        line["exit_prob_err_fp32_vs_fp64"] = w
        line["exit_prob_err_weighted_mean"] = m
    achieved = alg_work(1, r32["steps"], r32["hits"]) / float(np.mean(kt))
    line["roofline"] = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                        "unit": "T VALU lane-ops/s", "frac": achieved / PEAK_LANE_OPS,
                        "traffic": None, "kernel": "/".join(sorted(set(scheds)))}
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(g, run, args.cpu_sample, dt=run["dt"])
    return line


def run_batch(args, B, torch):
    """512 independent uneven graphs (stars and random trees, edges
    loguniform 3..4096, particles loguniform 1e4..1e6, half with quadratic
    potentials): one batched call (a launch per LDS group) against one launch
    per graph."""
    import numpy as np
    import workloads
    graphs, counts, run = workloads.config4()
    Gs = [B.mg_graph_create(g) for g in graphs]

    def make(prec=B.MG_FP32):
        return [B.mg_particles_init(G, c, B.MG_INIT_UNIFORM_LENGTH, init_seed=i, graph_tag=i,
                                    precision=prec, max_splits=run["max_splits"])
                for i, (G, c) in enumerate(zip(Gs, counts))]

    def totals(sets):
        t = np.zeros(4, np.uint64)
        for s in sets:
            t += B.mg_exit_counts(s)[2]
        return t

    sets = make()
    batch = B.mg_batch_create(sets)
    B.mg_batch_simulate(batch, 8, run["dt"], run["seed"])      # warm-up
    torch.cuda.synchronize()
    t_before = totals(sets)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        B.mg_batch_simulate(batch, run["n_steps"], run["dt"], run["seed"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tot = totals(sets) - t_before
    value = float(tot[1]) / wall
    acc = {}
    if not args.no_fp64:
        # FP64 batch from the same initial states and counters (common random
        # numbers): histogram TV and exit-probability error, worst member
        s64 = make(B.MG_FP64)
        b64 = B.mg_batch_create(s64)
        B.mg_batch_simulate(b64, 8, run["dt"], run["seed"])
        torch.cuda.synchronize()
        t64_before = totals(s64)
        t64 = time.perf_counter()
        for _ in range(args.steps):
            B.mg_batch_simulate(b64, run["n_steps"], run["dt"], run["seed"])
        torch.cuda.synchronize()
        wall64 = time.perf_counter() - t64
        sub64 = float((totals(s64) - t64_before)[1])
        tv = ee = em = 0.0
        for g, a, c in zip(graphs, sets, s64):
            tv = max(tv, _tv(B.mg_histogram(a, run["bins"]), B.mg_histogram(c, run["bins"])))
            w, m = exit_err(B.mg_exit_counts(a)[0], B.mg_exit_counts(c)[0], g.vtx_offsets)
            ee, em = max(ee, w), max(em, m)
        acc = {"fp64_value": sub64 / wall64, "fp32_speedup_over_fp64": value / (sub64 / wall64),
               "tv_fp32_vs_fp64_max": tv, "exit_prob_err_fp32_vs_fp64_max": ee,
               "exit_prob_err_weighted_mean_max": em,
               "exit_err_min_exits_per_vertex": MIN_EXITS}
        del b64, s64
    # the same work launched graph by graph
    solo = make()
    for s in solo:
        B.mg_simulate(s, 8, run["dt"], run["seed"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for s in solo:
        B.mg_simulate(s, run["n_steps"], run["dt"], run["seed"])
    torch.cuda.synchronize()
    wall_solo = time.perf_counter() - t1
    line = {"metric": METRIC, "value": value, "unit": "particle-substeps/s", "n_gpus": 1,
            "steps": args.steps, "warmup": 1, "ms_per_step": wall / args.steps * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": "batch512: 512 stars/random trees, 3..4096 edges, 1e4..1e6 "
                                   "particles each, zero drift or quadratic potentials, dt=1e-3, "
                                   "1000 steps per call, one batched call (a launch per "
                                   "LDS group)",
                       "n_graphs": len(graphs), "n_particles": int(sum(counts)),
                       "n_edges": int(sum(g.n_edges for g in graphs))},
            "unbatched_value": float(tot[1]) / args.steps / wall_solo,
            "batch_speedup": wall_solo * args.steps / wall,
            "hits_per_step": float(tot[2]) / float(tot[3])}
    line.update(acc)
    return line


def run_sweep(args, B, torch):
    """Batched FP32 vs FP64 over dt: the vascular network and 128 Langevin
    stars in one batch per precision and dt, over fixed horizons.  Reports
    per dt the throughput of both precisions, the largest histogram TV
    between them (same random integers), and how far the exit probabilities
    are from the jump probabilities b (Corollary 1: they converge as dt -> 0),
    weighted by the exits each vertex records."""
    import numpy as np
    import workloads
    graphs, counts, run = workloads.config5()
    Gs = [B.mg_graph_create(g) for g in graphs]
    rows = []
    sub32_total = wall32_total = 0.0
    for dt in run["dts"]:
        res = {}
        for prec in (B.MG_FP32, B.MG_FP64):
            sets = [B.mg_particles_init(G, c, B.MG_INIT_UNIFORM_LENGTH, init_seed=i,
                                        graph_tag=i, precision=prec,
                                        max_splits=run["max_splits"])
                    for i, (G, c) in enumerate(zip(Gs, counts))]
            steps = [max(1, int(round(T / dt))) for T in run["horizons"]]
            batch_net = B.mg_batch_create(sets[:1])
            batch_st = B.mg_batch_create(sets[1:])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            B.mg_batch_simulate(batch_net, steps[0], dt, run["seed"])
            B.mg_batch_simulate(batch_st, steps[1], dt, run["seed"])
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            sub = 0
            hists, exits = [], []
            for s_, nb in zip(sets, run["bins"]):
                ex, ab, tot = B.mg_exit_counts(s_)
                sub += int(tot[1])
                exits.append(ex)
                hists.append(B.mg_histogram(s_, nb))
            res[prec] = dict(wall=wall, sub=sub, hists=hists, exits=exits)
            del batch_net, batch_st, sets
        tv = max(_tv(a, b) for a, b in zip(res[B.MG_FP32]["hists"], res[B.MG_FP64]["hists"]))
        ee = max(exit_err(a, b, g.vtx_offsets)[0]
                 for a, b, g in zip(res[B.MG_FP32]["exits"], res[B.MG_FP64]["exits"], graphs))
        # distance of the FP64 exit law from b, per vertex weighted by exits
        dev = {}
        for name, idx in (("network", [0]), ("stars", list(range(1, len(graphs))))):
            num = den = 0.0
            for i in idx:
                g, ex = graphs[i], res[B.MG_FP64]["exits"][i]
                pr = exit_probs(ex, g.vtx_offsets)
                for v in range(g.n_vertices):
                    s0, s1 = g.vtx_offsets[v], g.vtx_offsets[v + 1]
                    tot_v = float(ex[s0:s1].sum())
                    if s1 - s0 < 2 or tot_v == 0:
                        continue
                    num += tot_v * 0.5 * float(np.abs(pr[s0:s1] - g.slot_jump_prob[s0:s1]).sum())
                    den += tot_v
            dev[name] = num / den if den else None
        r32, r64 = res[B.MG_FP32], res[B.MG_FP64]
        sub32_total += r32["sub"]
        wall32_total += r32["wall"]
        rows.append({"dt": dt, "fp32_substeps_per_s": r32["sub"] / r32["wall"],
                     "fp64_substeps_per_s": r64["sub"] / r64["wall"],
                     "tv_fp32_vs_fp64_max": tv, "exit_prob_err_fp32_vs_fp64_max": ee,
                     "exit_law_tv_from_b_network": dev["network"],
                     "exit_law_tv_from_b_stars": dev["stars"]})
    return {"metric": METRIC, "value": sub32_total / wall32_total, "unit": "particle-substeps/s",
            "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": wall32_total * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": "accuracy_sweep: vascular20k + 128 Langevin stars, one batch "
                                   "per precision and dt, dt in {1e-2,3e-3,1e-3,3e-4}, horizons "
                                   "0.05 (network) and 2 (stars), 1e8 + 1e8 particles per dt"},
            "per_dt": rows}


def run_density(args, B, torch):
    """The paper's accuracy experiment (Sec. 4.1, Fig. "error"): the 5-edge
    star metric graph with the linear (mu_i = -10 i) and quadratic
    (mu_i = -10 i x) potentials, b = 1/5, sigma = 1, semi-infinite edges as
    in the paper (Def. 3), binned over [0, 2] of each edge (100 bins; the
    mass beyond is below 1e-8).  Particles start on the vertex, burn in for
    0.5 time units, then the streamed histogram takes a snapshot every 0.01
    time units for 2 time units (inside the step kernels).  Reported per
    potential, dt and particle count: the empirical L2 error of the
    time-averaged density against the closed-form stationary density and the
    FP32 throughput of the whole run."""
    import numpy as np
    import workloads
    from workloads import stationary
    bins, burn_t, obs_t, gap_t = 100, 0.5, 2.0, 0.01
    rows = []
    sub_total = wall_total = 0.0
    for pot in ("linear", "quadratic"):
        g = workloads.paper_star5(pot, length=np.inf, bin_span=2.0)
        G = B.mg_graph_create(g)
        ref = stationary.star_bin_means(g, bins)
        for dt in (1e-2, 1e-3, 1e-4):
            for n in (10_000, 100_000, 1_000_000, 10_000_000):
                p = B.mg_particles_init(G, n, B.MG_INIT_AT_VERTEX, vertex=0, init_seed=1,
                                        precision=B.MG_FP32)
                burn = int(round(burn_t / dt))
                every = max(1, int(round(gap_t / dt)))
                steps = int(round(obs_t / dt))
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                B.mg_simulate(p, burn, dt, 11)
                B.mg_observe_histogram(p, bins, every)
                B.mg_simulate(p, steps, dt, 12)
                h, snaps = B.mg_observed_histogram(p)
                wall = time.perf_counter() - t0
                tot = B.mg_exit_counts(p)[2]
                l2 = B.mg_density_l2(G, bins, h, ref)
                sub_total += float(tot[1])
                wall_total += wall
                rows.append({"potential": pot, "dt": dt, "particles": n, "snapshots": snaps,
                             "l2_error": l2, "substeps_per_s": float(tot[1]) / wall,
                             "hits_per_step": float(tot[2]) / float(tot[3])})
                print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
                del p
    return {"metric": METRIC, "value": sub_total / wall_total, "unit": "particle-substeps/s",
            "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": wall_total * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": "paper_star5 density error: semi-infinite edges, linear "
                                   "and quadratic potentials, dt in {1e-2,1e-3,1e-4}, 1e4..1e7 "
                                   "particles, burn-in 0.5, snapshots every 0.01 for 2.0, "
                                   "100 bins/edge over [0, 2]"},
            "runs": rows}


def run_nohit(args, B, torch):
    """The step kernel's no-hit ceiling: 1e7 FP32 particles in the middle of
    one edge of length 1e9 (sigma = sqrt(2)), 2000 steps at dt = 1e-3, so no
    move reaches a vertex; the same launch path as the metric's workload."""
    import numpy as np
    import workloads
    g = workloads.segment(1e9, 0.0, 0.0, np.sqrt(2.0))
    G = B.mg_graph_create(g)
    n, steps, dt = 10_000_000, 2000, 1e-3
    ktimes, walls, res = [], [], None
    for it in range(args.warmup + args.steps):
        p = B.mg_particles_init(G, n, B.MG_INIT_EXPLICIT, edge=np.zeros(n, np.int32),
                                pos=np.full(n, 5e8), precision=B.MG_FP32)
        t = B.mg_autotune(p, dt, 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        B.mg_simulate(p, steps, dt, 0)
        e1.record()
        tot = B.mg_exit_counts(p)[2]
        wall = time.perf_counter() - t0
        if it >= args.warmup:
            ktimes.append(e0.elapsed_time(e1) * 1e-3)
            walls.append(wall)
            res = tot
        del p
    k = float(np.mean(ktimes))
    achieved = ALG_FP32_STEP * float(res[3]) / k
    kern = "k_pool32" if t["schedule"] != B.MG_SCHED_LANES else "k_step<fp32>"
    launches = -(-steps // t["steps_per_launch"]) if t["steps_per_launch"] else 1
    return {"metric": METRIC, "value": float(res[1]) / float(np.mean(walls)),
            "unit": "particle-substeps/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": float(np.mean(walls)) * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": "nohit_segment: 1e7 particles mid-edge of a 1e9-long "
                                   "segment, 2000 steps at dt=1e-3, no vertex hits"},
            "hits": int(res[2]),
            "roofline": {"bound": "alu", "achieved": achieved / 1e12,
                         "peak": PEAK_LANE_OPS / 1e12, "unit": "T VALU lane-ops/s",
                         "frac": achieved / PEAK_LANE_OPS, "traffic": None, "kernel": kern,
                         "kernel_ms_per_launch": k / launches * 1e3,
                         "launches_per_call": launches}}


def run_double_well(args, B, torch):
    """General coefficients: the 64-edge double-well star (cubic drift,
    graded diffusion), 1e7 particles uniform by length, 1e4 steps at
    dt = 1e-3.  FP32 (wave pools) is the value; FP64 is timed beside it
    and compared under common random numbers."""
    import numpy as np
    import workloads
    g = workloads.double_well_star(64)
    G = B.mg_graph_create(g)
    n, steps, dt, bins = 10_000_000, 10_000, 1e-3, 64

    def one(prec):
        p = B.mg_particles_init(G, n, B.MG_INIT_UNIFORM_LENGTH, init_seed=0, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        B.mg_simulate(p, steps, dt, 0)
        e1.record()
        ex, _, tot = B.mg_exit_counts(p)
        hist = B.mg_histogram(p, bins)
        wall = time.perf_counter() - t0
        return e0.elapsed_time(e1) * 1e-3, wall, tot, ex, hist

    ktimes, walls, res = [], [], None
    for it in range(args.warmup + args.steps):
        k, w, tot, ex, hist = one(B.MG_FP32)
        if it >= args.warmup:
            ktimes.append(k)
            walls.append(w)
            res = (tot, ex, hist)
    k64, w64, tot64, ex64, hist64 = one(B.MG_FP64)
    tot, ex, hist = res
    k = float(np.mean(ktimes))
    per_step = ALG_FP32_STEP + ALG_FP32_CUBIC
    work = per_step * float(tot[3]) + (ALG_FP32_HIT + ALG_FP32_CUBIC) * float(tot[2])
    achieved = work / k
    value = float(tot[1]) / float(np.mean(walls))
    tv = 0.5 * float(np.abs(hist.astype(float) - hist64.astype(float)).sum()) / float(hist64.sum())
    return {"metric": METRIC, "value": value,
            "unit": "particle-substeps/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": float(np.mean(walls)) * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": "double_well_star64: 64-edge star, cubic drift -V' of a "
                                   "double-well potential per edge, graded sigma(x), 1e7 "
                                   "particles uniform by length, 1e4 steps at dt=1e-3"},
            "hits_per_step": float(tot[2]) / float(tot[3]),
            "fp64": {"value": float(tot64[1]) / w64, "unit": "particle-substeps/s",
                     "fp32_speedup": value / (float(tot64[1]) / w64),
                     "kernel_ms_per_call": k64 * 1e3},
            "tv_fp32_vs_fp64": tv,
            "exit_prob_err_fp32_vs_fp64": exit_err(ex, ex64, g.vtx_offsets)[0],
            "roofline": {"bound": "alu", "achieved": achieved / 1e12,
                         "peak": PEAK_LANE_OPS / 1e12, "unit": "T VALU lane-ops/s",
                         "frac": achieved / PEAK_LANE_OPS, "traffic": None,
                         "kernel": "k_pool32 (128 per wave, 8-step windows, cubic "
                                   "coefficients)",
                         "kernel_ms_per_call": k * 1e3,
                         "alg_lane_ops_per_particle_step": per_step}}


def run_tracer(args, B, torch):
    """Tracer transport on the vascular network (Sec. 4.2): a pulse of 1e8
    FP32 particles injected at the inlets in proportion to their inflow,
    advanced 1e4 steps at config 3's dt with the streamed histogram taking a
    snapshot every 100 steps (64 bins per edge; 1.66e6 bins, in global
    memory).  By linearity the time-summed
    histogram of a pulse is the steady state of a constant injection, the
    tracer density the paper visualises.  Reported: substeps/s of the whole
    run (init, stepping with snapshots, readout), the absorbed fraction and
    the mean residence time the occupation gives."""
    import numpy as np
    import workloads
    g, run = workloads.config3()
    G = B.mg_graph_create(g)
    n, steps, dt, bins = run["n_particles"], run["n_steps"], run["dt"], run["bins"]
    every = 100  # 3e-4 T0 between snapshots; the mean residence is ~7000 steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p = B.mg_particles_init_sources(G, n, g.meta["inlets"], g.meta["inflow"], init_seed=0,
                                    precision=B.MG_FP32)
    B.mg_autotune(p, dt, run["seed"])
    B.mg_observe_histogram(p, bins, every)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    B.mg_simulate(p, steps, dt, run["seed"])
    e1.record()
    h, snaps = B.mg_observed_histogram(p)
    ex, ab, tot = B.mg_exit_counts(p)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    k = e0.elapsed_time(e1) * 1e-3
    return {"metric": METRIC, "value": float(tot[1]) / wall, "unit": "particle-substeps/s",
            "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": wall * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": "vascular20k tracer pulse: 1e8 particles injected at the "
                                   "inlets by inflow, 1e4 steps at 10x CFL dt, snapshot "
                                   "every 100 steps, 64 bins/edge"},
            "kernel_substeps_per_s": float(tot[1]) / k,
            "absorbed_fraction": float(ab.sum()) / n,
            "mean_residence_time_T0": float(h.sum()) * every * dt / n,
            "snapshots": snaps, "hits_per_step": float(tot[2]) / float(tot[3])}


def calibrate_copy(torch):
    """A 1 GiB device-to-device copy: the kernel of known size that HBM
    counter readings (FETCH_SIZE, WRITE_SIZE) are scaled by."""
    a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison")
    ap.add_argument("--no-1e8", action="store_true",
                    help="skip the 1e8-particle accuracy leg of the default workload")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 512-graph batch leg of the default workload")
    ap.add_argument("--cpu-sample", type=int, default=40_000)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first copy 1 GiB on the device (scale for HBM counters)")
    ap.add_argument("--workload", default="langevin_star64",
                    choices=["langevin_star64", "langevin_star64_mirror", "vascular20k",
                             "batch512", "accuracy_sweep", "density_error", "nohit_segment",
                             "vascular_tracer", "double_well_star64"],
                    help="the metric's configuration (default) or another workload")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus > 1 or world > 1:
        print(f"bench.py runs on one GPU only (asked for {max(args.gpus, world)}); the "
              "particle step shards by particle range with no communication but no "
              "multi-GPU path is built.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads
    from paper_2512_02175_amd import binding as B

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        calibrate_copy(torch)
    if args.workload == "vascular_tracer":
        emit(run_tracer(args, B, torch), torch)
        return
    if args.workload == "nohit_segment":
        emit(run_nohit(args, B, torch), torch)
        return
    if args.workload == "double_well_star64":
        emit(run_double_well(args, B, torch), torch)
        return
    if args.workload == "vascular20k":
        emit(run_vascular(args, B, torch), torch)
        return
    if args.workload == "batch512":
        emit(run_batch(args, B, torch), torch)
        return
    if args.workload == "accuracy_sweep":
        emit(run_sweep(args, B, torch), torch)
        return
    if args.workload == "density_error":
        emit(run_density(args, B, torch), torch)
        return
    g, run = workloads.config2()
    mirror = args.workload == "langevin_star64_mirror"
    if mirror:
        # the same star with mirror leaves (reflection by the mirror image)
        g = workloads.star_graph(g.n_edges, g.length, g.drift_a, g.drift_c, g.sigma,
                                 b_center=np.ones(g.n_edges), meta=g.meta, leaf_kind=2)
    G = B.mg_graph_create(g)
    dts = run["dts"]

    scheds = []

    def step(prec, ktimes, schedule=0):
        return [run_pass(B, G, g, run, prec, dt, torch, ktimes, scheds, schedule) for dt in dts]

    # FP32: the headline path
    for _ in range(args.warmup):
        step(1, [])
    torch.cuda.synchronize()
    ktimes32 = []
    t0 = time.perf_counter()
    res32 = None
    for _ in range(args.steps):
        res32 = step(1, ktimes32)
    torch.cuda.synchronize()
    wall32 = time.perf_counter() - t0
    sub32 = sum(r["substeps"] for r in res32) * args.steps
    value = sub32 / wall32

    out_fp64 = None
    tv = exit_e = None
    if not args.no_fp64:
        ktimes64 = []
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        res64 = step(0, ktimes64)
        torch.cuda.synchronize()
        wall64 = time.perf_counter() - t1
        sub64 = sum(r["substeps"] for r in res64)
        tv = [0.5 * float(np.abs(a["hist"].astype(float) - b["hist"].astype(float)).sum())
              / float(b["hist"].sum()) for a, b in zip(res32, res64)]
        exit_e = [exit_err(a["exit"], b["exit"], g.vtx_offsets)[0]
                  for a, b in zip(res32, res64)]
        k64 = sum(ktimes64)
        w64 = sum(alg_work(0, r["steps"], r["hits"]) for r in res64)
        # the plain FP64 kernel (one particle per lane, unbatched) beside it
        kt_plain = []
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        res_plain = step(0, kt_plain, B.MG_SCHED_LANES)
        torch.cuda.synchronize()
        wall_plain = time.perf_counter() - t2
        sub_plain = sum(r["substeps"] for r in res_plain)
        out_fp64 = {"value": sub64 / wall64, "unit": "particle-substeps/s",
                    "kernel": "k_pool64 (128 per wave, 8-step windows)",
                    "kernel_substeps_per_s": sub64 / k64,
                    "alg_frac_of_alu_peak": w64 / k64 / PEAK_LANE_OPS,
                    "fp32_speedup": value / (sub64 / wall64),
                    "plain_lane_kernel": {
                        "kernel": "k_step<fp64> (one particle per lane)",
                        "value": sub_plain / wall_plain,
                        "kernel_substeps_per_s": sub_plain / sum(kt_plain),
                        "fp32_speedup": value / (sub_plain / wall_plain),
                        "fp64_pools_speedup": (sub64 / wall64) / (sub_plain / wall_plain)}}

    # roofline of the dominant kernel (the fused step kernel), per launch
    # measured VALU issue rates beside the published peak
    rates = {name: B.mg_valu_rate(op)[0] / 1e12 for name, op in (
        ("v_fma_f32", B.MG_VALU_FMA_F32), ("v_fma_f64", B.MG_VALU_FMA_F64),
        ("v_mad_u64_u32", B.MG_VALU_MAD_U64_U32), ("v_bitop3_b32", B.MG_VALU_BITOP3),
        ("v_add_u32", B.MG_VALU_ADD_U32), ("v_log_f32", B.MG_VALU_LOG_F32))}
    # (a call is one launch unless the tuner split it; the rate is per call)
    k32 = float(np.mean(ktimes32))
    per_call = [alg_work(1, r["steps"], r["hits"]) for r in res32]
    achieved = float(np.mean(per_call)) / k32
    n_launch = float(np.mean([r["launches"] for r in res32]))
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12,
            "unit": "T VALU lane-ops/s", "frac": achieved / PEAK_LANE_OPS,
            "traffic": None if mirror else kernel_traffic(),
            "kernel": "/".join(sorted(set(scheds))), "kernel_ms_per_launch": k32 / n_launch * 1e3,
            "alg_lane_ops_per_particle_step": ALG_FP32_STEP,
            "alg_lane_ops_per_hit": ALG_FP32_HIT,
            "measured_issue_rates": rates,
            "frac_of_measured_v_fma_f32": achieved / 1e12 / rates["v_fma_f32"]}
    if out_fp64 is not None:
        # the FP64 path's algorithmic rate against the measured FP64 FMA rate
        out_fp64["frac_of_measured_v_fma_f64"] = (
            out_fp64["alg_frac_of_alu_peak"] * PEAK_LANE_OPS / 1e12 / rates["v_fma_f64"])

    line = {
        "metric": METRIC, "value": value, "unit": "particle-substeps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall32 / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": ("langevin_star64_mirror" if mirror else "langevin_star64")
                               + ": 64-edge star, V_e=k(x-m)^2, sigma=sqrt(2), "
                               "b=1/64, 1e7 particles uniform by length, 1e4 steps at "
                               "dt=1e-2 and dt=1e-3, M=8, 256 bins/edge"
                               + (", mirror leaves" if mirror else ""),
                   "n_particles": run["n_particles"], "n_steps": run["n_steps"],
                   "dts": list(dts), "bins_per_edge": run["bins"]},
        "particle_steps_per_s": sum(r["steps"] for r in res32) * args.steps / wall32,
        "kernel_substeps_per_s": sum(r["substeps"] for r in res32) / sum(ktimes32) * args.steps,
        "hits_per_step": [r["hits"] / r["steps"] for r in res32],
        "truncations": [r["trunc"] for r in res32],
        "fp64": out_fp64,
        "tv_fp32_vs_fp64": tv,
        "exit_prob_err_fp32_vs_fp64": exit_e,
        "roofline": roof,
    }
    if not args.no_1e8:
        line["at_1e8"] = at_scale(B, torch)
    if not args.no_batch:
        line["batch512"] = batch_leg(B, torch)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(g, run, args.cpu_sample)
    emit(line, torch)


if __name__ == "__main__":
    main()
