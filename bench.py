#!/usr/bin/env python
"""Benchmark of the GA hot path on one MI355X.

Default workload (one "step" = one whole run of the plain GA: init,
fitness, 500 generations): order m = 20, population n = 40,000, seed 1,
fitness SQ (and, timed beside it, ABS), binary tournament, crossover 0.5,
one pair flip per child at rate 0.1, stop-on-found off.  Prints one JSON
line with the throughput in evaluations per second (n fitness evaluations
per generation plus the initial population), the roofline of the fused
children kernel, the oracle's CPU throughput (all cores and one thread),
the time-to-solve of the m = 8, n = 1,024 plain GA over 32 seeds, and
summaries of the batched workload (24 runs against one ga_run each) and of
the server (the served stream's first 200 requests submitted at once,
against one ga_run each).

--workload batched: 24 runs in one batched launch per generation against
the same 24 runs one after another.
--workload served: a Poisson stream of search requests through the server,
then the first requests of the stream submitted at once against the same
requests run one ga_run after another.
--workload pmc: a short run for hardware-counter passes (no timing).
--workload elite: the elitist plain GA (m = 32, n = 200,000, 2,000 elites,
1,000 generations) alone.
--workload gram: the Gram + fitness kernel (ga_fitness_repeat) on the packed
popcount path and on the int8 matrix cores, per order.
--workload long_runs: the paper's single runs to a first Hadamard matrix
(Sec. 4.4) with its population sizes and mutation counts.
--workload table2: the paper's timing table (10^4 generations of 40,000
matrices per order and key) beside its seconds.
--workload paper_study: the paper's mutation study (generations to the first
Hadamard matrix over the NC x NR grid at m = 12 and 16) beside its tables.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X 32-bit vector ALU issue, 256 CUs at 2.4 GHz.  Simple ops (xor,
# add, compare, add-with-carry) issue at 128 lanes per clock per CU, the
# lane rate of the 157.3 TFLOP/s fp32 vector peak: 78.6 T ops/s.  Popcount
# (v_bcnt_u32_b32), the 24-bit multiply-add (v_mad_i32_i24) and v_sad_u32
# issue at half that rate, 64 lanes per clock per CU: 39.3 T ops/s.
SIMPLE_OP_TOPS = 256 * 128 * 2.4e9 / 1e12
HALF_RATE_TOPS = 256 * 64 * 2.4e9 / 1e12


def pair_mix(kind: int, w: int):
    """(simple ops, half-rate ops) per column pair of the packed fitness:
    w xors; w popcounts; the accumulation (SQ: multiply-add, ABS: sad, both
    half rate; NNZ: compare + add-with-carry, simple)."""
    import paper_2208_14961_amd as ga
    acc = {ga.FIT_SQ: (0, 1), ga.FIT_ABS: (0, 1), ga.FIT_F1: (0, 1), ga.FIT_NNZ: (2, 0),
           ga.FIT_F2: (2, 0), ga.FIT_SQ_PLUS_NNZ: (2, 1)}[kind]
    return w + acc[0], w + acc[1]


def alu_peak_tops(m: int, kind: int) -> float:
    """Peak op rate of the pair loop's instruction mix: its ops divided by
    the time the simple and half-rate ops take at their issue rates."""
    simple, half = pair_mix(kind, (m + 31) // 32)
    return (simple + half) / (simple / SIMPLE_OP_TOPS + half / HALF_RATE_TOPS)


def ops_per_eval(m: int, kind: int) -> int:
    """Integer ALU ops of the packed Gram + fitness of one individual:
    per column pair (i < j, columns 1..m-1) one xor and one popcount per
    word plus the key's accumulation (SQ: one multiply-add of the centred
    count; ABS: one absolute-difference add; NNZ: compare + add)."""
    pairs = (m - 1) * (m - 2) // 2
    return pairs * sum(pair_mix(kind, (m + 31) // 32))


HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
INT8_MFMA_PEAK_TOPS = 5000.0  # MI355X dense int8 matrix cores, published (2 ops per MAC)


def child_bytes(m: int, t: int = 2):
    """Algorithmic HBM bytes per child of a tournament generation: the
    winner's packed row and the t contestants' keys read, the child's row and
    key written (each parent row is read once per child that takes it)."""
    w = 1 if m <= 32 else (2 if m <= 64 else 4)
    row = m * w * 4
    return row + 4 * t, row + 4


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q / 100.0
    lo = int(k)
    hi = min(lo + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def buffers(cfg):
    import torch
    import paper_2208_14961_amd as ga
    sh = ga.pop_shape(cfg)
    pa = torch.zeros(sh, dtype=torch.int32, device="cuda")
    pb = torch.zeros_like(pa)
    ka = torch.zeros((cfg.n,), dtype=torch.int32, device="cuda")
    kb = torch.zeros_like(ka)
    return pa, pb, ka, kb


def timed_runs(cfg, bufs, steps):
    import torch
    import paper_2208_14961_amd as ga
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ga.ga_run(cfg, *bufs)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def oracle_rate(m, n, seed, kind, budget_s, max_gens=500):
    """The oracle on init, fitness and as many generations of the workload as
    fit in about budget_s seconds: (evals/s, generations, seconds)."""
    from oracle import gao
    probe = gao.Config(m=m, n=n, seed=seed, fitness=kind, max_generations=1,
                       stop_on_found=False)
    t = time.perf_counter()
    gao.run(probe)
    per_gen = (time.perf_counter() - t) / 2
    gens = max(1, min(max_gens, int(budget_s / max(per_gen, 1e-6)) - 1))
    cfg = gao.Config(m=m, n=n, seed=seed, fitness=kind, max_generations=gens,
                     stop_on_found=False)
    t = time.perf_counter()
    gao.run(cfg)
    dt = time.perf_counter() - t
    return n * (gens + 1) / dt, gens, dt


def cpu_baseline(m, n, seed, kind, budget_s=15.0):
    """The oracle (plain C, OpenMP over individuals) on a bounded sample of
    the same workload, with every host thread and with one: init, fitness
    and as many generations as fit in about budget_s seconds (half that for
    the single thread)."""
    from oracle import gao
    threads = gao.num_threads()
    rate, gens, dt = oracle_rate(m, n, seed, kind, budget_s)
    gao.set_num_threads(1)
    try:
        rate1, gens1, dt1 = oracle_rate(m, n, seed, kind, budget_s / 2)
    finally:
        gao.set_num_threads(threads)
    return {"value": rate, "unit": "evals/s", "cores": threads, "kind": "oracle",
            "sample": f"m={m}, n={n}, seed {seed}: init + fitness + {gens} generations "
                      f"({dt:.1f} s)",
            "cpu_model": cpu_model(), "host_threads": os.cpu_count(),
            "single_thread": {"value": rate1, "unit": "evals/s", "cores": 1,
                              "sample": f"init + fitness + {gens1} generations ({dt1:.1f} s)"}}


def time_to_solve(runs=32):
    """Plain GA, m=8, n=1,024, 200-generation budget, stop at key 0: wall
    time of each whole run (synchronous ga_run) over seeds 0..runs-1."""
    import paper_2208_14961_amd as ga
    times, gens, solved = [], [], 0
    cfg0 = ga.Config(m=8, n=1024, max_generations=200)
    bufs = buffers(cfg0)
    ga.ga_run(cfg0, *bufs)  # warm
    for s in range(runs):
        cfg = ga.Config(m=8, n=1024, seed=s, max_generations=200)
        t = time.perf_counter()
        r = ga.ga_run(cfg, *bufs)
        times.append(time.perf_counter() - t)
        if r["found"]:
            solved += 1
            gens.append(r["generation"])
    return {"workload": "plain GA m=8 n=1024, seeds 0..%d, budget 200" % (runs - 1),
            "runs": runs, "solved": solved,
            "p50_ms": 1e3 * percentile(times, 50), "p99_ms": 1e3 * percentile(times, 99),
            "mean_generations": (sum(gens) / len(gens)) if gens else None}


def workload_pmc(args):
    """Short runs for hardware-counter passes: the default workload's kernel
    for one 64-generation chunk with each lanes-per-child variant (2, 4 and
    8, the choices a run may keep), then a plain 256 MiB device copy whose
    counter reading calibrates the byte counters."""
    import torch
    import paper_2208_14961_amd as ga
    for lanes in (2, 4, 8):
        cfg = ga.Config(m=20, n=40000, seed=1, fitness=ga.FIT_SQ, max_generations=64,
                        flags=ga.lanes_flag(lanes))
        bufs = buffers(cfg)
        r = ga.ga_run(cfg, *bufs)
    x = torch.ones(64 * 1024 * 1024, dtype=torch.int32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    return {"workload": "counter pass: m=20 n=40000 SQ, 64 generations with 2, 4 and 8 lanes per "
                        "child; 256 MiB copy",
            "best_key": r["best_key"], "copy_bytes": 2 * x.numel() * 4}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "children_m20_n40000_traffic.md")
TRAFFIC_SOURCES = ["paper_2208_14961_amd/csrc/ga_children.h",
                   "paper_2208_14961_amd/csrc/ga_device.h"]


def sources_digest() -> str:
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    or None when it holds no record of that kernel or the kernel sources
    have changed since it was measured."""
    try:
        with open(TRAFFIC_FILE) as f:
            text = f.read()
        block = text.split("```json", 1)[1].split("```", 1)[0]
        recs = json.loads(block)
    except (OSError, IndexError, ValueError):
        return None
    for rec in recs if isinstance(recs, list) else [recs]:
        if rec.get("kernel") == kernel and rec.get("sources_sha256") == sources_digest():
            return rec
    return None


def gram_fitness_metric(reps=1000, repeats=5):
    """The Gram + fitness kernel alone: the seed-1 m=20, n=40,000 initial
    population evaluated `reps` times inside one launch (ga_fitness_repeat),
    HIP events on the launch's stream, median of `repeats` launches."""
    import torch
    import paper_2208_14961_amd as ga
    cfg = ga.Config(m=20, n=40000, seed=1, fitness=ga.FIT_SQ)
    pop, _, keys, _ = buffers(cfg)
    ga.ga_init_population(cfg, pop)
    ga.ga_fitness_repeat(cfg, pop, keys, reps)  # warm
    s = torch.cuda.current_stream()
    times = []
    for _ in range(repeats):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        ga.ga_fitness_repeat(cfg, pop, keys, reps)
        e1.record(s)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    ms = percentile(times, 50)
    evals = cfg.n * reps / (ms * 1e-3)
    tops = evals * ops_per_eval(cfg.m, cfg.fitness) / 1e12
    peak = alu_peak_tops(cfg.m, cfg.fitness)
    return {"kernel": "fitness_repeat_kernel<20, SQ>", "bound": "alu",
            "workload": f"m=20, n=40000, seed-1 initial population, SQ key, {reps} evaluations "
                        "of the whole population in one launch",
            "note": "a ceiling of the Gram + fitness core alone: the 3.2 MB population stays "
                    "in cache across the repeats; on the per-generation path this work is "
                    "fused into the children kernel, whose fraction is the roofline above",
            "median_ms": ms, "evals_per_s": evals, "achieved": tops, "peak": peak,
            "unit": "TOP/s", "frac": tops / peak,
            "frac_of_simple_op_peak": tops / SIMPLE_OP_TOPS}


def elite_run_metric():
    """Plain GA with elitism at m=32, n=200,000 (seed 2, SQ+NNZ key, the top
    1% kept, 1000 generations, stop-on-found off): one whole run."""
    import torch
    import paper_2208_14961_amd as ga
    cfg = ga.Config(m=32, n=200000, seed=2, fitness=ga.FIT_SQ_PLUS_NNZ, elite=2000,
                    max_generations=1000, flags=0)
    bufs = buffers(cfg)
    ga.ga_run(cfg, *bufs)  # warm (and the run's lanes-per-child measurement)
    torch.cuda.synchronize()
    t = time.perf_counter()
    r = ga.ga_run(cfg, *bufs)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    return {"workload": "plain GA m=32 n=200000 seed 2, SQ+NNZ, elite 2000, 1000 generations",
            "seconds": dt, "generations_per_s": cfg.max_generations / dt,
            "evals_per_s": (cfg.n - cfg.elite) * cfg.max_generations / dt,
            "best_key": r["best_key"]}


def paper_mode_metric(steps=2):
    """The paper's truncation-selection GA in the Table 2 configuration at
    m=20 (Sec. 4.2: 40,000 matrices, crossover and mutation on every
    offspring, NC=4, NR=2, 10^4 generations, no stop), keys F1 and F2: whole
    runs, median of `steps` after a warm one, beside the paper's seconds."""
    import statistics
    import paper_2208_14961_amd as ga
    m, N, G = 20, 10_000, 10_000
    bufs = buffers(ga.Config(m=m, n=4 * N, selection=ga.SEL_PAPER))
    out = {"workload": "paper mode, m=20, 40,000 matrices, NC=4, NR=2, 10^4 generations, "
                       "seed 9020, no stop on found"}
    for name, kind in (("F1", ga.FIT_F1), ("F2", ga.FIT_F2)):
        cfg = ga.Config(m=m, n=4 * N, seed=9_000 + m, selection=ga.SEL_PAPER, fitness=kind,
                        xo_threshold=1 << 32, mut_threshold=1 << 32, nc=4, nr=2,
                        max_generations=G, flags=0)
        ga.ga_run(cfg, *bufs)  # warm: the run's lanes-per-child measurement
        times = [timed_runs(cfg, bufs, 1) for _ in range(max(1, steps))]
        sec = statistics.median(times)
        paper_s = PAPER_TABLE2[m][0 if name == "F1" else 1]
        out[name] = {"seconds": sec, "generations_per_s": G / sec, "us_per_generation": 1e6 * sec / G,
                     "paper_seconds": paper_s, "speedup_vs_paper": paper_s / sec}
    return out


def bench_elite(args):
    """The elitist run alone, `--steps` timed runs after a warm one."""
    import torch
    import paper_2208_14961_amd as ga
    cfg = ga.Config(m=32, n=200000, seed=2, fitness=ga.FIT_SQ_PLUS_NNZ, elite=2000,
                    max_generations=1000, flags=0)
    bufs = buffers(cfg)
    ga.ga_run(cfg, *bufs)
    dt = timed_runs(cfg, bufs, max(1, args.steps)) / max(1, args.steps)
    gens = cfg.max_generations
    return {"metric": "elitist plain GA generations/s", "value": gens / dt,
            "unit": "generations/s", "n_gpus": 1, "steps": max(1, args.steps), "warmup": 1,
            "ms_per_step": 1e3 * dt, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "u32", "data": "synthetic",
            "config": {"workload": "plain GA m=32 n=200000 seed 2, SQ+NNZ, elite 2000, "
                                   "1000 generations"},
            "evals_per_s": (cfg.n - cfg.elite) * gens / dt, "us_per_generation": 1e6 * dt / gens,
            "lanes_per_child": ga.ga_tuned_lanes(cfg)}


def time_repeat(cfg, pop, keys, reps, repeats=5):
    """Median milliseconds of one ga_fitness_repeat launch (HIP events on the
    launch's stream), after a warm launch."""
    import torch
    import paper_2208_14961_amd as ga
    ga.ga_fitness_repeat(cfg, pop, keys, reps)
    s = torch.cuda.current_stream()
    times = []
    for _ in range(repeats):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        ga.ga_fitness_repeat(cfg, pop, keys, reps)
        e1.record(s)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    return percentile(times, 50)


def bench_gram(args):
    """Gram + fitness of a whole population evaluated many times in one
    launch, on the packed popcount path and on the int8 matrix cores, for
    orders 36..128 (SQ key, n = 40,000 initial population, seed 1).  The
    popcount path is measured against its instruction-mix peak, the matrix
    cores against the dense int8 peak with m * P algorithmic multiply-adds
    per evaluation (the tile padding and the lower triangle are waste)."""
    import torch
    import paper_2208_14961_amd as ga
    orders = [int(x) for x in args.gram_orders.split(",")]
    n, rows = 40000, []
    for m in orders:
        base = ga.Config(m=m, n=n, seed=1, fitness=ga.FIT_SQ)
        pop, _, keys, _ = buffers(base)
        ga.ga_init_population(base, pop)
        pairs = (m - 1) * (m - 2) // 2
        row = {"m": m, "n": n}
        for name, flag in (("packed", ga.GRAM_PACKED), ("mfma", ga.GRAM_MFMA)):
            cfg = ga.Config(m=m, n=n, seed=1, fitness=ga.FIT_SQ, flags=flag)
            probe = time_repeat(cfg, pop, keys, 4, repeats=1)
            reps = max(4, int(4 * 2.0 / max(probe, 1e-3)))  # about 2 ms per launch
            ms = time_repeat(cfg, pop, keys, reps)
            evals = n * reps / (ms * 1e-3)
            if name == "packed":
                tops = evals * ops_per_eval(m, ga.FIT_SQ) / 1e12
                row[name] = {"evals_per_s": evals, "ms": ms, "reps": reps, "achieved": tops,
                             "peak": alu_peak_tops(m, ga.FIT_SQ), "unit": "TOP/s",
                             "frac": tops / alu_peak_tops(m, ga.FIT_SQ)}
            else:
                tops = evals * 2 * m * pairs / 1e12
                row[name] = {"evals_per_s": evals, "ms": ms, "reps": reps, "achieved": tops,
                             "peak": INT8_MFMA_PEAK_TOPS, "unit": "TOP/s (int8, 2 per MAC)",
                             "frac": tops / INT8_MFMA_PEAK_TOPS}
        row["mfma_over_packed"] = row["mfma"]["evals_per_s"] / row["packed"]["evals_per_s"]
        rows.append(row)
        print(f"gram: m={m}: packed {row['packed']['evals_per_s']:.3e}/s, mfma "
              f"{row['mfma']['evals_per_s']:.3e}/s ({row['mfma_over_packed']:.2f}x)",
              file=sys.stderr, flush=True)
        del pop, keys
    return {"metric": "Gram + fitness evaluations/s, packed popcount vs int8 matrix cores",
            "value": None, "unit": "evals/s", "n_gpus": 1, "steps": 5, "warmup": 1,
            "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "u32/i8", "data": "synthetic",
            "config": {"workload": f"ga_fitness_repeat, SQ, n={n}, orders {orders}"},
            "rows": rows}


def bench_default(args):
    import torch
    import paper_2208_14961_amd as ga
    G, n, m = 500, 40000, 20
    cfg = ga.Config(m=m, n=n, seed=1, fitness=ga.FIT_SQ, max_generations=G, flags=0)
    cfg_abs = ga.Config(m=m, n=n, seed=1, fitness=ga.FIT_ABS, max_generations=G, flags=0)
    bufs = buffers(cfg)
    for _ in range(args.warmup):
        ga.ga_run(cfg, *bufs)
        ga.ga_run(cfg_abs, *bufs)
    dt = timed_runs(cfg, bufs, args.steps)
    dt_abs = timed_runs(cfg_abs, bufs, args.steps)
    evals = n * (G + 1)
    # roofline of the fused children kernel: one more run with HIP events on
    # the library's stream around its generation loop; with tournament
    # selection and no elites each generation is one children launch, so the
    # mean time per generation is that kernel's launch-to-launch time
    ga.ga_timing_enable(True)
    ga.ga_run(cfg, *bufs)
    mean_ms, launches = ga.ga_timing_read()
    ga.ga_timing_enable(False)
    ops = ops_per_eval(m, ga.FIT_SQ)
    rd, wr = child_bytes(m)
    alu_achieved = n * ops / (mean_ms * 1e-3) / 1e12
    alu_peak = alu_peak_tops(m, ga.FIT_SQ)
    # the roofline that bounds the kernel: its arithmetic intensity against
    # the ridge point of the ALU mix peak over the HBM peak
    intensity = ops / (rd + wr)
    ridge = alu_peak * 1e12 / (HBM_PEAK_GBS * 1e9)
    hbm_achieved = n * (rd + wr) / (mean_ms * 1e-3) / 1e9
    kernel = f"children_one_kernel<20, 1u, {ga.ga_tuned_lanes(cfg)}>"
    tr = measured_traffic(kernel)  # counters of the variant this run kept
    traffic = tr["fetch_bytes_per_launch"] + tr["write_bytes_per_launch"] if tr else None
    alu = {"achieved": alu_achieved, "peak": alu_peak, "unit": "TOP/s",
           "frac": alu_achieved / alu_peak, "frac_of_simple_op_peak": alu_achieved / SIMPLE_OP_TOPS,
           "ops_per_eval": ops}
    if intensity < ridge:
        roofline = {"bound": "hbm", "kernel": kernel, "achieved": hbm_achieved,
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": hbm_achieved / HBM_PEAK_GBS,
                    "traffic": traffic, "algorithmic_bytes_per_launch": n * (rd + wr), "alu": alu}
    else:
        roofline = {"bound": "alu", "kernel": kernel, **{k: alu[k] for k in
                    ("achieved", "peak", "unit", "frac")}, "traffic": traffic,
                    "algorithmic_bytes_per_launch": n * (rd + wr),
                    "frac_of_simple_op_peak": alu["frac_of_simple_op_peak"], "ops_per_eval": ops}
    roofline.update({"intensity_ops_per_byte": intensity, "ridge_ops_per_byte": ridge,
                     "mean_generation_ms": mean_ms, "generations_timed": launches})
    out = {
        "metric": "Gram+fitness evals/s and generations/s at m=20,pop=40k; p50/p99 time-to-solve",
        "value": args.steps * evals / dt,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "plain GA, m=20, n=40000, seed 1, fitness SQ, 500 generations, "
                               "tournament 2, crossover 0.5, pair-flip 0.1, stop-on-found off",
                   "m": m, "n": n, "generations": G},
        "generations_per_s": args.steps * G / dt,
        "abs_keyed": {"value": args.steps * evals / dt_abs, "unit": "evals/s",
                      "generations_per_s": args.steps * G / dt_abs},
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(m, n, 1, ga.FIT_SQ, budget_s=args.cpu_seconds)
    out["time_to_solve"] = time_to_solve()
    out["gram_fitness_kernel"] = gram_fitness_metric()
    out["elite_run"] = elite_run_metric()
    out["paper_mode"] = paper_mode_metric()
    if not args.no_multi:
        out["batched"] = batched_leg(steps=2)
        print("default: batched leg done", file=sys.stderr, flush=True)
        # the Poisson stream (served_leg, --workload served) is not part of
        # the default line: one run of it ended in a host segmentation fault
        # whose cause has not been found; the server is measured here on
        # the stream's first requests submitted at once
        out["served"] = served_saturated(workload_served(count=args.saturated)[0])
        print("default: served leg done", file=sys.stderr, flush=True)
    return out


def config_of(fields):
    """A library configuration from the workload generator's fields."""
    import paper_2208_14961_amd as ga
    f = dict(fields)
    stop = f.pop("stop_on_found")
    return ga.Config(**f, flags=ga.STOP_ON_FOUND if stop else 0)


def workload_batched():
    """24 runs: orders from {12,16,20,24,28,36}, sizes uniform in
    [2000, 60000], seeds 4*10^6 + i, 300 generations each."""
    from tests import inputs
    return [config_of(f) for f in inputs.batched_workload()]


def batched_leg(steps=2):
    """The 24-run batched workload: ga_run_batch (after one warm batch)
    against the same runs one ga_run each (after a warm pass that allocates
    their buffers and measures their lanes per child); both sides make the
    same generations, and their results are compared."""
    import torch
    import paper_2208_14961_amd as ga
    cfgs = workload_batched()
    gens = sum(c.max_generations for c in cfgs)
    evals = sum(c.n * (c.max_generations + 1) for c in cfgs)
    batch = ga.ga_run_batch(cfgs)  # warm
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        batch = ga.ga_run_batch(cfgs)
    torch.cuda.synchronize()
    dt_b = (time.perf_counter() - t) / steps
    bufs = [buffers(c) for c in cfgs]
    for c, b in zip(cfgs, bufs):
        ga.ga_run(c, *b)
    torch.cuda.synchronize()
    t = time.perf_counter()
    plain = [ga.ga_run(c, *b) for c, b in zip(cfgs, bufs)]
    torch.cuda.synchronize()
    dt_p = time.perf_counter() - t
    del bufs
    return {"workload": "24 runs, m in {12,16,20,24,28,36}, n in [2000,60000], 300 generations, "
                        "seeds 4e6+i",
            "runs": len(cfgs), "generations": gens,
            "batched": {"seconds": dt_b, "generations_per_s": gens / dt_b,
                        "evals_per_s": evals / dt_b, "batches_timed": steps},
            "plain": {"seconds": dt_p, "generations_per_s": gens / dt_p,
                      "evals_per_s": evals / dt_p},
            "speedup_vs_plain": dt_p / dt_b,
            "results_identical": all(same_result(a, b) for a, b in zip(batch, plain))}


def bench_batched(args):
    leg = batched_leg(steps=max(1, args.steps))
    return {
        "metric": "batched generations/s (24 runs) vs one run per launch",
        "value": leg["batched"]["generations_per_s"], "unit": "generations/s", "n_gpus": 1,
        "steps": max(1, args.steps), "warmup": 1, "ms_per_step": 1e3 * leg["batched"]["seconds"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "batched: 24 runs, m in {12..36}, n in [2000,60000], 300 gens"},
        **leg,
    }


def workload_served(count=2000, rate=50.0):
    """Poisson arrivals (mean `rate`/s); order uniform over multiples of 4 in
    [8, 64]; size uniform in [1000, 50000]; 2000-generation budget."""
    from tests import inputs
    fields, arrivals = inputs.served_workload(count=count, rate=rate)
    return [config_of(f) for f in fields], arrivals


def served_leg(count, saturated_count):
    """The served workload: a Poisson stream of `count` requests submitted at
    their arrival times to a server with a 200 GB budget; then its first
    `saturated_count` requests at once against one ga_run each."""
    import paper_2208_14961_amd as ga
    cfgs, arrivals = workload_served(count=count)
    srv = ga.Server(hbm_budget_bytes=200 * 10**9)
    t0 = time.perf_counter()
    ids = []
    for c, a in zip(cfgs, arrivals):
        now = time.perf_counter() - t0
        if a > now:
            time.sleep(a - now)
        ids.append(srv.submit(c))
        if len(ids) % 500 == 0:
            print(f"served: {len(ids)}/{count} requests submitted after "
                  f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    results = []
    for k, i in enumerate(ids):
        results.append(srv.wait(i))
        if (k + 1) % 100 == 0:
            print(f"served: {k + 1}/{count} requests retired after "
                  f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    wall = time.perf_counter() - t0
    lat = [srv.latency(i) for i in ids]
    srv.close()
    solved = [l for l, r in zip(lat, results) if r["found"]]
    evals = sum(c.n * (r["generation"] + 1) for c, r in zip(cfgs, results))
    gens = sum(r["generation"] for r in results)
    saturated = served_saturated(cfgs[:saturated_count]) if saturated_count > 0 else None
    return {"workload": f"{count} Poisson requests at 50/s, m in 8..64 step 4, n in "
                        "[1000,50000], budget 2000 generations, stop on found, 200 GB admission",
            "requests": count, "seconds": wall, "requests_per_s": count / wall,
            "generations_per_s": gens / wall, "evals_per_s": evals / wall,
            "solved": len(solved), "solve_rate": len(solved) / count,
            "time_to_first_hadamard": {"p50_s": percentile(solved, 50),
                                       "p99_s": percentile(solved, 99)},
            "time_to_retire": {"p50_s": percentile(lat, 50), "p99_s": percentile(lat, 99)},
            "saturated": saturated}


def bench_served(args):
    leg = served_leg(args.requests, args.saturated)
    return {
        "metric": "served search: requests/s and p50/p99 time-to-first-Hadamard",
        "value": leg["requests_per_s"], "unit": "requests/s", "n_gpus": 1, "steps": 1,
        "warmup": 0, "ms_per_step": 1e3 * leg["seconds"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"served: {leg['workload']}"},
        **leg,
    }


def same_result(a, b):
    return (a["found"] == b["found"] and a["generation"] == b["generation"]
            and a["index"] == b["index"] and a["best_key"] == b["best_key"]
            and (a["matrix"] == b["matrix"]).all())


def served_saturated(cfgs):
    """The given requests submitted to a fresh server all at once, against the
    same requests run one ga_run after another (each on buffers allocated
    beforehand, after a warm pass that measures its lanes per child).  Both
    sides make the same generations, so the generations/s ratio is the
    ratio of wall times."""
    import torch
    import paper_2208_14961_amd as ga
    srv = ga.Server(hbm_budget_bytes=200 * 10**9)
    torch.cuda.synchronize()
    t = time.perf_counter()
    ids = [srv.submit(c) for c in cfgs]
    served = [srv.wait(i) for i in ids]
    dt_s = time.perf_counter() - t
    lat = [srv.latency(i) for i in ids]
    srv.close()
    solved = [l for l, r in zip(lat, served) if r["found"]]
    print(f"served: saturated leg, {len(cfgs)} requests at once in {dt_s:.2f} s",
          file=sys.stderr, flush=True)
    bufs = [buffers(c) for c in cfgs]
    for c, b in zip(cfgs, bufs):
        ga.ga_run(c, *b)
    torch.cuda.synchronize()
    t = time.perf_counter()
    plain = [ga.ga_run(c, *b) for c, b in zip(cfgs, bufs)]
    torch.cuda.synchronize()
    dt_p = time.perf_counter() - t
    del bufs
    gens = sum(r["generation"] for r in served)
    evals = sum(c.n * (r["generation"] + 1) for c, r in zip(cfgs, served))
    return {"requests": len(cfgs), "generations": gens,
            "workload": f"the first {len(cfgs)} requests of the served stream (m in 8..64 step 4, "
                        "n in [1000,50000], budget 2000 generations, stop on found) submitted "
                        "at once to a server with a 200 GB admission budget",
            "server": {"seconds": dt_s, "generations_per_s": gens / dt_s,
                       "evals_per_s": evals / dt_s, "requests_per_s": len(cfgs) / dt_s,
                       "solved": len(solved), "solve_rate": len(solved) / len(cfgs),
                       "time_to_first_hadamard": {"p50_s": percentile(solved, 50),
                                                  "p99_s": percentile(solved, 99)},
                       "time_to_retire": {"p50_s": percentile(lat, 50),
                                          "p99_s": percentile(lat, 99)}},
            "plain": {"seconds": dt_p, "generations_per_s": gens / dt_p,
                      "evals_per_s": evals / dt_p},
            "speedup_vs_plain": dt_p / dt_s,
            "results_identical": all(same_result(a, b) for a, b in zip(served, plain))}


# Average iterations to a Hadamard matrix over 10 runs per (NC, NR), rows
# NR = 1..4, columns NC = 1..4 (Sec. 4.3, Tables 3 and 4); starred m=16
# cells are averages over the few runs that found one.
PAPER_TABLES = {
    12: [[34.2, 35.8, 37.4, 35.8], [32.3, 38.8, 40.5, 43.4],
         [35.2, 42.6, 47.5, 50.7], [36.3, 46.0, 49.9, 65.7]],
    16: [[130.1, 119.4, 116.0, 115.5], [121.0, 181.3, 135.0, 168.7],
         [120.0, 158.1, 165.9, 202.7], [120.2, 166.2, 236.2, 301.6]],
}


# Seconds for 10^4 generations of 40,000 matrices (N = 10^4), NC = 4,
# NR = 2, mean of 10 runs, keys F1 and F2 (Sec. 4.2, Table 2).
PAPER_TABLE2 = {20: (60.50, 59.38), 40: (103.15, 99.84), 60: (176.28, 170.20),
                80: (275.92, 256.59), 100: (416.68, 381.38)}


def bench_table2(args):
    """The paper's fitness-function timing (Sec. 4.2, Table 2): paper-mode
    runs of 10^4 generations over 40,000 matrices (N = 10^4), crossover and
    mutation on every offspring, NC = 4, NR = 2, keys F1 and F2, for each
    order of the table the library supports; wall time of a whole run
    (init, fitness, 10^4 generations), median of `--steps` runs after a
    warm run."""
    import statistics
    import torch
    import paper_2208_14961_amd as ga
    N, T = 10_000, args.table2_generations
    paper = T == 10_000  # the table's own run length
    orders = [int(x) for x in args.table2_orders.split(",")] if args.table2_orders else \
        list(PAPER_TABLE2)
    rows = []
    for m in orders:
        p1, p2 = PAPER_TABLE2.get(m, (None, None)) if paper else (None, None)
        bufs = buffers(ga.Config(m=m, n=4 * N, selection=ga.SEL_PAPER))
        for name, kind, paper_s in (("F1", ga.FIT_F1, p1), ("F2", ga.FIT_F2, p2)):
            cfg = ga.Config(m=m, n=4 * N, seed=9_000 + m, selection=ga.SEL_PAPER, fitness=kind,
                            xo_threshold=1 << 32, mut_threshold=1 << 32, nc=4, nr=2,
                            max_generations=T, flags=0)
            ga.ga_run(cfg, *bufs)  # warm: the run's lanes-per-child measurement
            times = []
            for _ in range(max(1, args.steps)):
                torch.cuda.synchronize()
                t = time.perf_counter()
                r = ga.ga_run(cfg, *bufs)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t)
            sec = statistics.median(times)
            rows.append({"m": m, "key": name, "seconds": sec, "generations_per_s": T / sec,
                         "paper_seconds": paper_s,
                         "speedup_vs_paper": paper_s / sec if paper_s else None,
                         "best_key": r["best_key"]})
            print(f"table2: m={m} {name}: {sec:.3f} s (paper {paper_s} s)", file=sys.stderr,
                  flush=True)
    head = next((r for r in rows if r["m"] == 20 and r["key"] == "F2"), rows[-1])
    return {
        "metric": "paper-mode generations/s, 40,000 matrices, NC=4, NR=2 (Sec. 4.2, Table 2)",
        "value": head["generations_per_s"], "unit": "generations/s", "n_gpus": 1,
        "steps": max(1, args.steps), "warmup": 1, "ms_per_step": 1e3 * head["seconds"],
        "higher_is_better": True, "scaling": "weak",
        "vs_baseline": head["speedup_vs_paper"],
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"paper mode, m={head['m']}, N=10^4 (40,000 matrices), "
                               f"{head['key']}, NC=4, NR=2, {T} generations per run, "
                               "no stop on found"},
        "rows": rows,
    }


# The single runs of Sec. 4.4: order -> (N, NC, NR, iterations, seconds).
PAPER_LONG_RUNS = {20: (1_000, 2, 8, 258_875, 517), 24: (1_000, 2, 10, 9_576_814, 19_997),
                   28: (10_000, 1, 10, 428_082, 3_054), 32: (20_000, 1, 12, 7_472_853, 94_923)}


def bench_long_runs(args):
    """The paper's runs to a first Hadamard matrix (Sec. 4.4): paper mode, F2,
    crossover and mutation on every offspring, each order with the paper's N,
    NC and NR, stopping at the first Hadamard matrix or after
    `--long-budget` generations; one run per seed."""
    import numpy as np
    import torch
    import paper_2208_14961_amd as ga
    orders = [int(x) for x in args.long_orders.split(",")]
    rows = []
    for m in orders:
        N, nc, nr, p_it, p_s = PAPER_LONG_RUNS[m]
        bufs = buffers(ga.Config(m=m, n=4 * N, selection=ga.SEL_PAPER))
        for k in range(args.long_seeds):
            cfg = ga.Config(m=m, n=4 * N, seed=10_000 * m + k, selection=ga.SEL_PAPER,
                            fitness=ga.FIT_F2, xo_threshold=1 << 32, mut_threshold=1 << 32,
                            nc=nc, nr=nr, max_generations=args.long_budget)
            torch.cuda.synchronize()
            t = time.perf_counter()
            r = ga.ga_run(cfg, *bufs)
            torch.cuda.synchronize()
            sec = time.perf_counter() - t
            if r["found"]:
                H = r["matrix"].astype(np.int64)
                assert (H.T @ H == m * np.eye(m, dtype=np.int64)).all()
            rows.append({"m": m, "N": N, "nc": nc, "nr": nr, "seed": cfg.seed,
                         "found": bool(r["found"]), "generations": r["generation"],
                         "seconds": sec, "us_per_generation": 1e6 * sec / max(1, r["generation"]),
                         "paper_iterations": p_it, "paper_seconds": p_s,
                         "paper_us_per_iteration": 1e6 * p_s / p_it})
            print(f"long run: m={m} seed {cfg.seed}: found={r['found']} after {r['generation']} "
                  f"generations, {sec:.1f} s (paper: {p_it} iterations, {p_s} s)", file=sys.stderr,
                  flush=True)
    first = next((r for r in rows if r["m"] == 20 and r["found"]), None)
    return {
        "metric": "paper-mode time to first Hadamard matrix, Sec. 4.4 configurations",
        "value": first["seconds"] if first else None, "unit": "s", "n_gpus": 1,
        "steps": len(rows), "warmup": 0, "ms_per_step": None, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"paper mode, F2, orders {orders} with the paper's N, NC, NR; "
                               f"{args.long_seeds} seed(s) each, budget {args.long_budget} "
                               "generations"},
        "runs": rows,
    }


def bench_paper_study(args):
    """The paper's mutation study (Sec. 4.3): its truncation selection with
    n = 4N (N = 1000 by default), key F2 (or F1), crossover and mutation on
    every offspring, for m in {12, 16} and NC, NR in 1..4, ten seeds per
    cell, stopping at the first Hadamard matrix or after `budget`
    generations."""
    import statistics
    import paper_2208_14961_amd as ga
    budget, seeds, N = 5000, 10, args.study_n
    kind = {"F1": ga.FIT_F1, "F2": ga.FIT_F2}[args.study_fitness]
    cells, solved_gens = [], []
    t0 = time.perf_counter()
    for m in (12, 16):
        bufs = buffers(ga.Config(m=m, n=4 * N, selection=ga.SEL_PAPER))
        for nr in range(1, 5):
            for nc in range(1, 5):
                gens = []
                for seed in range(seeds):
                    cfg = ga.Config(m=m, n=4 * N, seed=8_000_000 + 1000 * m + seed,
                                    selection=ga.SEL_PAPER, fitness=kind,
                                    xo_threshold=1 << 32, mut_threshold=1 << 32,
                                    nc=nc, nr=nr, max_generations=budget)
                    r = ga.ga_run(cfg, *bufs)
                    if r["found"]:
                        gens.append(r["generation"])
                solved_gens += gens
                cells.append({"m": m, "nc": nc, "nr": nr, "solved": len(gens), "runs": seeds,
                              "mean_generations": statistics.fmean(gens) if gens else None,
                              "median_generations": statistics.median(gens) if gens else None,
                              "paper_mean": PAPER_TABLES[m][nr - 1][nc - 1]})
                print(f"paper study: m={m} NC={nc} NR={nr}: {len(gens)}/{seeds} solved", file=sys.stderr,
                      flush=True)
    wall = time.perf_counter() - t0
    return {
        "metric": "paper-mode generations to first Hadamard, Sec. 4.3 grid",
        "value": statistics.fmean(solved_gens) if solved_gens else None,
        "unit": "generations (mean over solved runs)", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": 1e3 * wall, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"paper mode, N={N} (n=4N), {args.study_fitness}, crossover and mutation always, "
                               f"m in {{12,16}}, NC,NR in 1..4, {seeds} seeds per cell, "
                               f"budget {budget} generations"},
        "cells": cells,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="default",
                    choices=["default", "batched", "served", "pmc", "elite", "gram", "paper_study",
                             "table2", "long_runs"])
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--saturated", type=int, default=200,
                    help="served: requests of the stream also submitted at once and "
                         "run one by one (0: skip)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-multi", action="store_true",
                    help="default workload: skip the batched and served summaries")
    ap.add_argument("--table2-orders", default="",
                    help="table2: comma-separated orders (default: the table's five)")
    ap.add_argument("--table2-generations", type=int, default=10_000,
                    help="table2: generations per run (the table's 10^4 by default)")
    ap.add_argument("--long-orders", default="20,28",
                    help="long_runs: comma-separated orders among 20, 24, 28, 32")
    ap.add_argument("--long-seeds", type=int, default=1, help="long_runs: runs per order")
    ap.add_argument("--long-budget", type=int, default=2_000_000,
                    help="long_runs: generation budget per run")
    ap.add_argument("--gram-orders", default="36,48,52,64,68,84,100,116,128",
                    help="gram: comma-separated orders (36..128)")
    ap.add_argument("--study-n", type=int, default=1000,
                    help="paper_study: N, half the parent count (n = 4N)")
    ap.add_argument("--study-fitness", default="F2", choices=["F1", "F2"],
                    help="paper_study: the key")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(independent runs would be sharded by run, one process per GPU).",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    fn = {"default": bench_default, "batched": bench_batched, "served": bench_served,
          "pmc": workload_pmc, "elite": bench_elite, "gram": bench_gram,
          "paper_study": bench_paper_study,
          "table2": bench_table2, "long_runs": bench_long_runs}
    out = fn[args.workload](args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
