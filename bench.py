"""Benchmark: batched simplex-in-cell steps on one MI355X.

Default workload: the mixed batch of 4096 independent 1D1V instances (seeded
draw: Landau or two-stream, k in [0.2, 0.6], alpha log-uniform in
[1e-3, 0.5], 32-512 sheets x 64-2048 tracers, 64-1024 cells), all resident in
HBM, advanced together.  One step = one pass of the whole hot path (move,
deposit, field solve) over every instance.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp64]

Besides the batched throughput (``value``) the line carries the same
instances run one simulation per launch sequence (``plain``), the roofline of
the tracer kernel (HIP-event timing of the kernel itself) and the FP64 CPU
oracle timed on a bounded sample (``cpu_baseline``).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "tracer-updates/s batched vs plain at <=1e-6 rel field-energy err; p50/p99 latency"
HBM_PEAK_GBPS = 8000.0
BYTES_PER_TRACER = 32  # read + write of x and v (8 B each) per fused step
BYTES_PER_CELL = 32    # per instance per step: E read, charge accumulators read and cleared, E written


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def profiled_traffic(precision, instances, tuning):
    """HBM bytes per tracer-kernel launch from the committed rocprofv3 counter
    summary, valid only for the profiled workload, launch shape and window,
    and only while the kernel source is the one that was profiled (None
    otherwise)."""
    import hashlib

    if precision != "fp64" or instances != 4096:
        return None
    summ = os.path.join(ROOT, "profiles", "k_tracers_fp64_mixed4096_traffic.md")
    src = os.path.join(ROOT, "paper_1506_07207_amd", "csrc", "sic_kernels.hip")
    try:
        kv = dict(line.strip().split("=", 1) for line in open(summ) if "=" in line and " " not in line.strip())
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    if kv.get("kernel_source_sha256_16") != digest:
        return None
    shape = f"{tuning['tile_chunks']},{tuning['block_threads']},{tuning['grid_blocks']}"
    if kv.get("launch_shape") != shape:
        return None
    return float(kv["traffic_bytes_per_launch"])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=500,
                    help="untimed steps first: by default the timed window starts past the two-stream "
                         "instances' saturation, where the sheets have folded")
    ap.add_argument("--early-steps", type=int, default=20,
                    help="also time this many steps right after 5 warm-up steps (0: skip)")
    ap.add_argument("--instances", type=int, default=4096)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "split_f32", "split_u32"])
    ap.add_argument("--deposit-order", type=int, default=0, choices=[0, 1, 2],
                    help="0 constant segments, 1 piecewise-linear segments, 2 first-order weighting")
    ap.add_argument("--segment-charges", action="store_true",
                    help="store a charge per segment (the form vertical sheets and refinement use)")
    ap.add_argument("--plain-instances", type=int, default=256)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-single", action="store_true", help="skip the single-simulation set-ups")
    ap.add_argument("--no-refine", action="store_true", help="skip the refinement run")
    ap.add_argument("--cpu-seconds", type=float, default=24.0, help="CPU work of the oracle baseline (core-seconds)")
    ap.add_argument("--cpu-cores", type=int, default=0, help="worker processes for the oracle (0: the host share)")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="time the default launch shape instead of the autotuner's pick")
    ap.add_argument("--serve-seconds", type=float, default=20.0,
                    help="seconds of Poisson arrivals for the serving run (0: skip)")
    ap.add_argument("--serve-load", type=float, default=0.8, help="arrival rate as a fraction of saturation")
    ap.add_argument("--serve-requests", type=int, default=0,
                    help="length of the served stream in requests (0: --serve-seconds of arrivals)")
    ap.add_argument("--plain-serve-requests", type=int, default=100)
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--grid", type=int, default=0)
    return ap.parse_args()


def device_inputs(problem, torch):
    line = torch.from_numpy(problem.line).cuda()
    x0 = line.repeat(problem.n_sheets)
    v0 = torch.from_numpy(problem.sheet_v).cuda().repeat_interleave(int(problem.n_tracers[0]))
    return x0, v0


def build_batch(B, specs, precision, torch, history_rows=256, deposit_order=0, seg=False):
    total = sum(s.tracers for s in specs)
    max_cells = max(s.n_cells for s in specs)
    b = B.sic_batch_create(total, len(specs), max_cells, precision=precision, history_rows=history_rows,
                           deposit_order=deposit_order, flags=B.SIC_BATCH_SEGMENT_CHARGES if seg else 0)
    t0 = time.time()
    cells = 0
    for i, s in enumerate(specs):
        p = s.build()
        x0, v0 = device_inputs(p, torch)
        c0 = torch.from_numpy(p.seg_charges).cuda() if seg else None
        B.sic_batch_admit(b, p.L, p.n_cells, p.dt, p.n_tracers, p.q, p.closed, x0, v0, p.n_steps,
                          precision=precision, deposit_order=deposit_order, seg_charges=c0)
        cells += p.n_cells
        if (i + 1) % 512 == 0:
            log(f"admitted {i + 1}/{len(specs)} instances ({time.time() - t0:.1f}s)")
    return b, total, cells


def time_batched(B, b, steps, torch):
    """Wall time of ``steps`` batch steps, bracketed by device syncs."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.sic_batch_step(b, steps)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def updates_in_window(specs, first, last):
    """Tracer-updates of batch steps first+1 .. last: an instance advances
    until its own step count is reached and is then masked."""
    return sum(s.tracers * max(0, min(s.n_steps, last) - min(s.n_steps, first)) for s in specs)


def kernel_timing(B, b, steps=5):
    B.sic_batch_set_timing(b, True)
    B.sic_batch_step(b, steps)
    tr, so = B.sic_batch_last_timing(b)
    B.sic_batch_set_timing(b, False)
    return tr, so


def time_plain(B, specs, precision, steps, torch):
    """The same instances, one simulation per launch sequence (no batching)."""
    sims = []
    n_tr = 0
    for s in specs:
        p = s.build()
        x0, v0 = device_inputs(p, torch)
        sims.append(B.Simulation(p, precision=precision, history_rows=64, x0=x0, v0=v0))
        n_tr += p.total_tracers
    for sim in sims:
        sim.step(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for sim in sims:
        sim.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    for sim in sims:
        sim.close()
    return n_tr * steps / dt, n_tr, dt


def time_single_configs(B, I, torch):
    """The single-simulation set-ups of the parity tests, each run alone for
    its full step count: a first run captures the step graphs it needs (HIP
    graphs of up to 32 steps), then the initial state is loaded again and
    the same run is timed (events on the launch stream; the cost of a step
    grows as the sheets stretch, so the timed run covers the set-up's own
    steps).  Reports the time per step, the resulting tracer-updates/s, the
    launch path of the steps and the kernel launches per step: one tracer
    launch per step plus a solve and a clearing launch per graph of up to 32
    steps on the solve-first path, 2 (tracer kernel and solve) on the fused
    launch pairs, 1 / steps for a small simulation, whose steps run in one
    resident launch."""
    cases = [
        ("cold oscillation, FP64 (1 x 1024 tracers, 128 cells)", I.cold_oscillation(), B.SIC_FP64),
        ("Landau damping, FP64 (256 x 512 tracers, 256 cells)", I.landau(), B.SIC_FP64),
        ("two-stream, split int cell + f32 offset (512 x 4096 tracers, 1024 cells)", I.two_stream(),
         B.SIC_SPLIT_F32),
        ("two-stream, split int cell + u32 fraction (512 x 4096 tracers, 1024 cells)", I.two_stream(),
         B.SIC_SPLIT_U32),
        ("large served job, FP64 (2048 x 16384 tracers, 4096 cells, 64 steps)",
         I.landau(n_sheets=2048, n_tracers=16384, n_cells=4096, n_steps=64), B.SIC_FP64),
    ]
    # the oracle's field-energy history of the full two-stream run, stored by
    # tests/golden/make_two_stream_ensemble.py: the timed split-form runs
    # report their error against it
    ref_path = os.path.join(ROOT, "tests", "golden", "two_stream_full_ensemble.txt")
    ref_w = np.loadtxt(ref_path)[:, 1] if os.path.exists(ref_path) else None
    out = []
    for name, p, prec in cases:
        x0, v0 = device_inputs(p, torch)
        with_ref = ref_w is not None and name.startswith("two-stream") and len(ref_w) == p.n_steps + 1
        sim = B.Simulation(p, precision=prec, history_rows=(p.n_steps + 1) if with_ref else 64, x0=x0, v0=v0)
        del x0, v0
        try:
            x_init, v_init, _ = sim.state()
            sim.step(p.n_steps)
            sim.set_state(0, x_init, v_init)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            sim.step(p.n_steps)
            e1.record()
            e1.synchronize()
            ms = e0.elapsed_time(e1)
            err = None
            if with_ref:
                W = sim.diagnostics()["history"]["W_E"]
                P = int(math.ceil(2 * math.pi / p.dt))
                env = np.array([ref_w[max(0, i - P): i + P + 1].max() for i in range(len(ref_w))])
                e = np.abs(W - ref_w) / env
                over = np.nonzero(e > 1e-6)[0]
                err = {"max_envelope_rel": float(e.max()), "first_step_over_1e-6": int(over[0]) if len(over) else None,
                       "against": "stored oracle history (tests/golden/two_stream_full_ensemble.txt)"}
            path = B.sic_last_step_path(sim.h)
        finally:
            sim.close()
        n = p.total_tracers
        graphs = math.ceil(p.n_steps / 32)
        if path == B.SIC_PATH_RESIDENT:
            launches = math.ceil(p.n_steps / 8192) / p.n_steps
        elif path == B.SIC_PATH_SOLVE_FIRST:
            launches = (p.n_steps + 2 * graphs) / p.n_steps
        else:
            launches = 2
        names = {B.SIC_PATH_FUSED: "fused launch pairs", B.SIC_PATH_RESIDENT: "resident",
                 B.SIC_PATH_REFINING: "refining", B.SIC_PATH_SOLVE_FIRST: "solve-first"}
        out.append({"workload": name, "tracers": n, "cells": p.n_cells, "steps": p.n_steps, "ms": ms,
                    "us_per_step": 1e3 * ms / p.n_steps, "tracer_updates_per_s": n * p.n_steps / (ms * 1e-3),
                    "path": names.get(path, str(path)), "kernel_launches_per_step": launches,
                    "field_energy_error": err})
        log(f"single: {name}: {1e3 * ms / p.n_steps:.1f} us/step, {n * p.n_steps / (ms * 1e-3):.3e} tracer-updates/s")
    torch.cuda.empty_cache()
    return out


def time_refinement(B, I, torch, steps=700, tail=50):
    """The refinement experiment of section 2.6 (two cold beams, 10 tracers
    per cell per stream, 100 cells, dt 0.1) with refinement at one cell after
    every move, all ``steps`` in one sic_step call (the passes run on the
    device); then the same final state stepped without refinement, for the
    cost of a refining step against a plain one at the same tracer count."""
    p = I.refinement_two_stream(n_steps=steps)
    dx = p.L / p.n_cells
    cap = 4_000_000
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    with B.Simulation(p, l_max=dx, max_tracers=cap, history_rows=steps + 8) as s:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(steps - tail)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        s.step(tail)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        nt, total = s.layout()
        x, v, step = s.state()
        c = s.charges()
    with B.Simulation(p, seg_charges=p.seg_charges, max_tracers=total, history_rows=64) as s2:
        s2.load_state(step, nt, x, v, c)
        s2.step(1)
        e0, e1 = ev(), ev()
        e0.record()
        s2.step(tail)
        e1.record()
        e1.synchronize()
        plain_ms = e0.elapsed_time(e1)
    torch.cuda.empty_cache()
    refining_us = 1e6 * (t2 - t1) / tail
    plain_us = 1e3 * plain_ms / tail
    return {"workload": f"section 2.6 two-stream refinement run, l_max = 1 cell, {steps} steps in one call",
            "steps": steps, "tracers_start": p.total_tracers, "tracers_end": int(total),
            "seconds": t2 - t0, "us_per_step_last_refining": refining_us,
            "us_per_step_plain_same_state": plain_us, "refining_over_plain": refining_us / plain_us}


DEPOSIT_BYTES_PER_TRACER = 8   # the position word, read once
DEPOSIT_BYTES_PER_CELL = 16    # P and D accumulators written


def time_deposit(B, I, precision, torch, sheets=8192, tracers=16384, cells=1024, reps=100, warmup=150):
    """The standalone deposit (sic_deposit) of one large simulation: 8192
    Landau sheets x 16384 tracers (134M tracers, 1.07 GB of positions, far
    beyond the caches) on 1024 cells, timed with events on the stream the
    kernel runs on (the current torch stream).  The deposit is paced by
    instruction issue, and the engine clock takes about 100 launches (30 ms)
    to ramp up after the GPU was idle or only streaming memory (windows of 20
    launches: 0.31, 0.29, 0.28, 0.27, 0.26 ms, then flat), so ``warmup``
    untimed launches come first."""
    p = I.landau(n_sheets=sheets, n_tracers=tracers, n_cells=cells, n_steps=1)
    x0, v0 = device_inputs(p, torch)
    sim = B.Simulation(p, precision=precision, history_rows=8, x0=x0, v0=v0)
    del x0, v0
    try:
        for _ in range(warmup):
            sim.deposit()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            sim.deposit()
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
    finally:
        sim.close()
        torch.cuda.empty_cache()
    n = p.total_tracers
    algo = DEPOSIT_BYTES_PER_TRACER * n + DEPOSIT_BYTES_PER_CELL * cells
    gbps = algo / (ms * 1e-3) / 1e9
    return {"tracers": n, "cells": cells, "ms": ms, "segments_per_s": n / (ms * 1e-3), "achieved": gbps,
            "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": gbps / HBM_PEAK_GBPS, "algorithmic_bytes": algo,
            "workload": f"one Landau simulation, {sheets} sheets x {tracers} tracers, {cells} cells, "
                        "sic_deposit (zeroing of the mesh included)"}


def _oracle_worker(job):
    """One host core: the FP64 oracle (one thread) on whole instances of the
    mix (every ``stride``-th one from ``first``), 2 steps each, for about
    ``seconds`` of its own time.  Returns (tracer-updates, instances, seconds)."""
    specs, seconds = job
    from oracle import oracle as O

    done, n, t_total = 0, 0, 0.0
    for s in specs:
        p = s.build()
        t0 = time.perf_counter()
        O.run_problem(p, 2)
        t_total += time.perf_counter() - t0
        done += 2 * p.total_tracers
        n += 1
        if t_total >= seconds:
            break
    return done, n, t_total


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.lower().startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_cores():
    """Host cores this process may use (the OMP_NUM_THREADS share when set)."""
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    omp = os.environ.get("OMP_NUM_THREADS", "")
    return max(1, min(avail, int(omp))) if omp.isdigit() and int(omp) > 0 else avail


def cpu_baseline(specs, cpu_seconds, cores):
    """The FP64 oracle on the host cores: instances of the same mix dealt out
    to one worker process per core (each runs the single-threaded oracle),
    about ``cpu_seconds`` of CPU work in total.  Aggregate tracer-updates per
    second of wall time over the workers' timed loops."""
    import multiprocessing as mp

    per = max(1.0, cpu_seconds / cores)
    jobs = [([specs[i] for i in range(w, len(specs), cores)], per) for w in range(cores)]
    # fresh interpreters: the workers never touch the GPU this process uses
    with mp.get_context("spawn").Pool(cores) as pool:
        res = pool.map(_oracle_worker, jobs)
    updates = sum(r[0] for r in res)
    n_inst = sum(r[1] for r in res)
    wall = max(r[2] for r in res)
    return updates / wall, n_inst, sum(r[2] for r in res)


def serving(B, S, I, value, args, torch):
    """Continuous-batching run: Poisson arrivals drawn like the mixed batch
    plus rare large jobs (2048 x 16384 tracers on 4096 cells), at a fraction
    of the measured saturation rate; then the plain one-request-at-a-time
    server on a prefix of the same stream."""
    sample = list(I.request_stream(4000, 1.0, seed=20251204))
    mean_work = float(np.mean([r.spec.tracers * r.spec.n_steps for r in sample]))
    rate = args.serve_load * value / mean_work
    n = args.serve_requests if args.serve_requests > 0 else max(20, int(rate * args.serve_seconds))
    reqs = S.poisson_stream(n, rate)
    log(f"serving {n} requests at {rate:.1f}/s (mean {mean_work:.3e} tracer-updates per request)")
    ex = S.GpuExecutor()
    try:
        # the first 10 % of the stream, while the batch fills, is not counted
        rep = S.Server(ex, chunk_steps=32).run(reqs, warmup_fraction=0.1, prepare=S.serve_prepare(ex),
                                               progress=lambda d, t: log(f"served {d}/{t}"))
    finally:
        ex.close()
    torch.cuda.empty_cache()
    summ = rep.summary()
    log(f"served: p50 {summ['p50_s']:.3f}s p99 {summ['p99_s']:.3f}s, {summ['tracer_updates_per_s']:.3e} tracer-updates/s")
    out = {"rate_rps": rate, "load": args.serve_load, "mean_updates_per_request": mean_work, **summ}
    m = min(args.plain_serve_requests, n)
    if m > 0:
        prefix = reqs[:m]
        ex = S.GpuExecutor()
        try:
            brep = S.Server(ex, chunk_steps=32).run(prefix, warmup_fraction=0.0, prepare=S.serve_prepare(ex))
        finally:
            ex.close()
        prep = S.serve_plain(prefix)
        prep.warmup_fraction = 0.0
        ps, bs = prep.summary(), brep.summary()
        out["prefix_requests"] = m
        out["prefix_batched"] = {k: bs[k] for k in ("p50_s", "p99_s", "tracer_updates_per_s", "wall_s")}
        out["prefix_plain"] = {k: ps[k] for k in ("p50_s", "p99_s", "tracer_updates_per_s", "wall_s")}
        log(f"prefix of {m}: batched p50 {bs['p50_s']:.3f}s p99 {bs['p99_s']:.3f}s; "
            f"plain p50 {ps['p50_s']:.3f}s p99 {ps['p99_s']:.3f}s")
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the batched path shards by "
              "instance across GPUs with no exchange, so multi-GPU figures are not produced here.",
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1506_07207_amd import binding as B
    from paper_1506_07207_amd import inputs as I

    if not os.path.exists(B.LIB_PATH):
        from paper_1506_07207_amd import build as hb
        hb.build()
    torch.cuda.set_device(0)
    precision = B.PRECISIONS[args.precision]
    specs = I.batch_mix(args.instances)
    log(f"building batch of {len(specs)} instances ({args.precision})")
    t_setup = time.time()
    b, total, cells = build_batch(B, specs, precision, torch, deposit_order=args.deposit_order,
                                  seg=args.segment_charges)
    tuned = None
    if args.tile or args.block or args.grid:
        B.sic_batch_set_tuning(b, args.tile, args.block, args.grid)
    elif args.autotune:
        t0 = time.time()
        best, best_ms = B.sic_batch_autotune(b, 3)
        tuned = {"best": best, "ms_per_step": best_ms, "seconds": time.time() - t0}
        log(f"autotune: {best} {best_ms:.3f} ms/step ({time.time() - t0:.1f}s)")
    tuning = B.sic_batch_get_tuning(b)
    log(f"resident tracers {total:.3e}, setup {time.time() - t_setup:.1f}s, tuning {tuning}")

    done = 0
    early = None
    if args.early_steps > 0:
        B.sic_batch_step(b, 5)
        done = 5
        el = time_batched(B, b, args.early_steps, torch)
        upd = updates_in_window(specs, done, done + args.early_steps)
        early = {"steps": f"{done + 1}-{done + args.early_steps}", "ms_per_step": 1e3 * el / args.early_steps,
                 "value": upd / el}
        done += args.early_steps
        log(f"batched, early window (steps {early['steps']}): {early['ms_per_step']:.3f} ms/step, "
            f"{early['value']:.4e} tracer-updates/s")
        e_tr, e_so = kernel_timing(B, b)
        done += 5
        early["kernel_ms"], early["solve_ms"] = e_tr, e_so
    if args.warmup > done:
        B.sic_batch_step(b, args.warmup - done)
        done = args.warmup
    elapsed = time_batched(B, b, args.steps, torch)
    ms_per_step = 1e3 * elapsed / args.steps
    updates = updates_in_window(specs, done, done + args.steps)
    value = updates / elapsed
    window = f"{done + 1}-{done + args.steps}"
    log(f"batched, steps {window}: {ms_per_step:.3f} ms/step, {value:.4e} tracer-updates/s")
    done += args.steps

    tr_ms, so_ms = kernel_timing(B, b)
    # a charge word per tracer is read with per-segment charges; linear
    # segments also read and clear a ramp array per cell
    bytes_tracer = BYTES_PER_TRACER + (8 if args.segment_charges else 0)
    bytes_cell = BYTES_PER_CELL + (8 if args.deposit_order == 1 else 0)
    # per launch, averaged over the five timed launches: the instances still
    # advancing (finished ones are masked)
    act_tracers = updates_in_window(specs, done, done + 5) / 5
    act_cells = sum(s.n_cells * max(0, min(s.n_steps, done + 5) - min(s.n_steps, done)) for s in specs) / 5
    bytes_launch = bytes_tracer * act_tracers + bytes_cell * act_cells
    done += 5
    achieved = bytes_launch / (tr_ms * 1e-3) / 1e9
    copy_gbps = B.sic_copy_bandwidth(4 << 30, 5)
    log(f"tracer kernel {tr_ms:.3f} ms ({achieved:.0f} GB/s), solve kernel {so_ms:.3f} ms, copy {copy_gbps:.0f} GB/s")
    B.sic_batch_destroy(b)
    torch.cuda.empty_cache()

    deposit = time_deposit(B, I, precision, torch)
    log(f"standalone deposit: {deposit['ms']:.3f} ms for {deposit['tracers']:.3e} tracers "
        f"({deposit['achieved']:.0f} GB/s, {deposit['segments_per_s']:.3e} segments/s)")

    single = None if args.no_single else time_single_configs(B, I, torch)

    refine = None
    if not args.no_refine:
        refine = time_refinement(B, I, torch)
        log(f"refinement: {refine['seconds']:.3f} s for {refine['steps']} steps ({refine['tracers_start']} -> "
            f"{refine['tracers_end']} tracers); last steps {refine['us_per_step_last_refining']:.1f} us refining vs "
            f"{refine['us_per_step_plain_same_state']:.1f} us plain")

    plain = None
    if not args.no_plain:
        rng = np.random.default_rng(7)
        idx = rng.choice(len(specs), size=min(args.plain_instances, len(specs)), replace=False)
        sub = [specs[i] for i in sorted(idx)]
        rate, n_tr, dt = time_plain(B, sub, precision, 5, torch)
        plain = {"value": rate, "unit": "tracer-updates/s", "instances": len(sub), "tracers": n_tr,
                 "steps": 5, "batched_over_plain": value / rate}
        log(f"plain: {rate:.4e} tracer-updates/s over {len(sub)} instances")

    serve = None
    if args.serve_seconds > 0 or args.serve_requests > 0:
        from paper_1506_07207_amd import serve as S
        serve = serving(B, S, I, value, args, torch)

    cpu = None
    if not args.no_cpu_baseline:
        cores = args.cpu_cores or host_cores()
        rate, n_inst, secs = cpu_baseline(specs, args.cpu_seconds, cores)
        cpu = {"value": rate, "unit": "tracer-updates/s", "cores": cores, "kind": "oracle", "cpu_model": cpu_model(),
               "sample": f"{n_inst} instances of the same mix dealt to {cores} worker processes (one per core, "
                         f"each the single-threaded FP64 oracle), 2 steps each, {secs:.1f} s of CPU work"}
        log(f"cpu oracle: {rate:.4e} tracer-updates/s")

    traffic = None
    if args.deposit_order == 0 and not args.segment_charges:
        traffic = profiled_traffic(args.precision, args.instances, tuning)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "tracer-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "split_f32": "i32+f32/i64/f64", "split_u32": "i32+u32/i64/f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"batched mix of {len(specs)} SIC 1D1V instances (Landau/two-stream, "
                               "32-512 sheets x 64-2048 tracers, 64-1024 cells), one shared step",
                   "timed_steps": window, "early": early,
                   "instances": len(specs), "tracers": total, "cells": cells, "precision": args.precision,
                   "deposit_order": args.deposit_order, "segment_charges": bool(args.segment_charges),
                   "tuning": tuning, "autotune": tuned},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic,
                     "kernel": "k_tracers (move + deposit)", "kernel_ms": tr_ms, "solve_ms": so_ms,
                     "algorithmic_bytes": bytes_launch, "copy_gbps": copy_gbps},
        "deposit": deposit,
        "single": single,
        "refinement": refine,
        "plain": plain,
        "serving": serve,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
