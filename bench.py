#!/usr/bin/env python
"""Throughput of the A3 photoionisation source-term step on one MI355X.

Workload: the 256^3 clumpy medium -- lognormal density (sigma_ln = 1, power
spectrum k^-11/3, seed 1201), mean n_H = 5 cm^-3, central 1e5 K blackbody
source of 5e48 photons/s with rates tabulated against optical depth, evolving
temperature, timestep criterion dt02 -- advanced from a neutral start to
0.1 t_rec before timing.  One "step" is one full second-order step
(algorithm 3): timestep reduction, predictor micro-physics, raytrace of the
half-step state, corrector micro-physics, raytrace of the new state.

Prints ONE JSON line: cell-updates/s (whole job), ms per step, the roofline
object of the dominant kernel (measured live with HIP events on the stream the
kernels run on; its HBM fraction and the whole step's beside the ALU figure),
the FP64 oracle's rate on a bounded CPU sample (one thread and OpenMP, with the
host's CPU model), the error of the same kernels against the oracle on that
sample, and p50/p99 latency of a served stream of config-5-sized requests
(n 48..256, each to 2 t_rec) at a stated arrival rate the GPU sustains.

Other workloads (--workload): batch (64 uneven grids advanced together, and
the FP64 single-grid path on a sample of them), serve (Poisson requests to the
library's server; p50/p99 latency), hardening (the 37 500 K blackbody runs of
Sect. 4 as one batch, with A3-dt02 against smaller steps), a1 (algorithm 1
steps on the same 256^3 medium), sources (the same medium lit by four point
sources).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# MI355X vector peaks [TFLOP/s]: 256 CUs x 2.4 GHz x 2 flops per FMA x FMA
# lanes per CU per clock.  FP64: 64 lanes, 78.6.  FP32: 128 lanes with packed
# FP32 instructions (the published 157.3), 64 lanes without them -- and this
# build turns packed FP32 off, so 78.6 is the FP32 issue rate it can reach.
VALU_PEAK = {"fp32": 78.6, "fp64": 78.6, "mixed": 78.6, "mixed_front": 78.6}
VALU_PEAK_NOTE = ("FMA issue rate without packed FP32: 256 CU x 64 lanes x 2 flops x 2.4 GHz "
                  "(the published FP32 vector peak, 157.3, needs packed FP32, which the build "
                  "disables)")
# Algorithmic HBM bytes per cell-update of the whole step (two raytraces, two
# micro-physics updates and the timestep, with the columns carried between
# steps): read n_H, x, E, tau, write x, E, tau -- seven words.
STEP_WORDS = 7
# Algorithmic flops of the micro-physics, counted from the source (add, mul,
# each half of a fused multiply-add, reciprocal, square root and
# transcendental = 1 flop each): one Newton iteration of the coupled (x, E)
# stage solve with the tabulated spectrum, evolving temperature, power-law
# recombination, collisional ionisation and cooling, optically thick branch;
# and the per-cell set-up of one micro-integration (geometry, entering-column
# table lookup, initial rate).  A table lookup of P and H (log of tau, the two
# interval cubics and their derivatives in Horner form, two exponentials) is 33
# of them: one in a Newton iteration, two in the set-up.
FLOP_NEWTON = 222
FLOP_CELL_SETUP = 250
# The raytrace's arithmetic per cell, counted the same way: the geometry of
# the short characteristic (offsets, two quotients, the path length), the
# four upstream depths, the Mellema-weighted average and the cell's own
# depth -- small beside the micro-physics it is fused with.
FLOP_SWEEP_CELL = 60


KERNEL_SOURCES = ("paper_1201_5651_amd/csrc/physics.h", "paper_1201_5651_amd/csrc/kernels.h",
                  "paper_1201_5651_amd/csrc/kernels.hip")
TRAFFIC_PROFILE = "profiles/cfg3_256_mixed_k_chem_sweep_traffic.md"


def kernel_code_digest() -> str:
    """sha256 of the kernel sources with their comments and blank lines taken
    out: an edit of comments alone leaves a hardware-counter summary valid."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        text = open(os.path.join(ROOT, f)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        h.update("\n".join(l.rstrip() for l in text.splitlines() if l.strip()).encode())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the fused micro-physics and raytrace from the
    committed hardware-counter summary, or None when the kernel code has
    changed since it was taken."""
    import re
    try:
        text = open(os.path.join(ROOT, TRAFFIC_PROFILE)).read()
    except OSError:
        return None
    m = re.search(r"kernel_code_sha256: ([0-9a-f]+)", text)
    t = re.search(r"k_chem_sweep_traffic_bytes_per_launch: ([0-9.eE+-]+)", text)
    if not m or not t or m.group(1) != kernel_code_digest():
        return None
    return float(t.group(1))


def word_bytes(precision: str) -> int:
    return 8 if precision == "fp64" else 4


def dtype_name(precision: str) -> str:
    # mixed: float cells; the double reductions and the (reported) double
    # re-solves of precision-sensitive cells do not change the cells' type
    return {"fp64": "f64", "fp32": "f32", "mixed": "f32", "mixed_front": "f32+f64"}[precision]


PRECISION_DETAIL = {
    "fp64": "double cells and reductions",
    "fp32": "float cells, double timestep and diagnostic reductions",
    "mixed": "float cells, double timestep and diagnostic reductions, double re-solve of the "
             "cells whose float integration took a precision-sensitive decision "
             "(fp64_resolved_frac)",
    "mixed_front": "float cells, double reductions, double integration of the ionisation-front "
                   "cells (starting x in [1e-3, 0.5]) and of precision-sensitive cells",
}


def host_cpu():
    """Model name and logical CPU count of the host."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count()


def _cpu_case(n: int):
    """The headline recipe on an n^3 grid of the same box (2.4 R_S), from the
    synthetic partly ionised start (an ionised sphere of 0.375 n cells'
    radius, the radius the 256^3 benchmark state has); inputs as the float
    grid holds them."""
    import numpy as np

    from paper_1201_5651_amd import synth
    spec = synth.cfg3(n=n, box_cells=n)
    f32 = lambda a: np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)
    nH = f32(synth.density(spec))
    x, T = synth.ionised_sphere(spec, 0.375 * n)
    x = f32(x)
    E = f32(1.5 * 1.380649e-16 * nH * (2.0 - x) * T)
    return spec, nH, x, E


def cpu_oracle_steps(n: int, budget_s: float, max_steps: int):
    """The FP64 oracle on _cpu_case(n): whole A3 steps for at least budget_s
    seconds (at most max_steps).  Returns the rate, the steps and the final
    state (for the error of the GPU against it)."""
    import oracle
    spec, nH, x, E = _cpu_case(n)
    pb = oracle.Problem.from_spec(spec)
    st = {"nH": nH, "x": x.copy(), "E": E.copy(), "t": 0.0}
    st["tau"] = pb.raytrace(nH, st["x"])
    steps = 0
    t0 = time.perf_counter()
    while True:
        pb.step(st, 1e30)
        steps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or steps >= max_steps:
            break
    return spec.ncells * steps / el, steps, el, pb, st


def cpu_baseline(n: int, budget_s: float, n_omp: int, omp_steps: int):
    """The FP64 oracle on the host: one thread on the headline recipe at n^3
    (whole box, synthetic front start), timed over at least budget_s of whole
    A3 steps; and its OpenMP build (bitwise the same results) on all host
    cores at n_omp^3, timed over omp_steps steps, in a child process."""
    import subprocess
    rate, steps, el, pb, st = cpu_oracle_steps(n, budget_s, 200)
    model, ncpu = host_cpu()
    out = {
        "value": rate,
        "unit": "cell-updates/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"FP64 oracle, 1 thread, {steps} A3 steps of the benchmark recipe at {n}^3 "
                  f"(same 2.4 R_S box, lognormal seed 1201, from an ionised sphere of "
                  f"{0.375 * n:.0f} cells' radius); {el:.1f} s",
        "cpu_model": model,
        "nproc": ncpu,
    }
    env = dict(os.environ, ORACLE_OPENMP="1")
    cmd = [sys.executable, os.path.abspath(__file__), "--omp-leg", str(n_omp), str(omp_steps)]
    try:
        r = subprocess.run(cmd, env=env, capture_output=True, text=True, timeout=600)
        leg = json.loads(r.stdout.strip().splitlines()[-1])
        out["openmp"] = leg
    except Exception as e:   # reported, not fatal: the single-thread leg stands
        out["openmp"] = {"error": str(e)[:200]}
    return out, (steps, pb, st)


def omp_leg(n: int, steps: int) -> int:
    """Child process of cpu_baseline: the OpenMP oracle's rate at n^3."""
    rate, k, el, _, _ = cpu_oracle_steps(n, 1e30, steps)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count()))
    print(json.dumps({"value": rate, "unit": "cell-updates/s", "cores": threads,
                      "sample": f"FP64 oracle built with OpenMP, {threads} threads, {k} A3 steps "
                                f"of the benchmark recipe at {n}^3 from the same start; {el:.1f} s"}))
    return 0


def error_vs_oracle(torch, binding, n: int, steps: int, pb, st, precision: str):
    """The GPU path of the headline (same precision, same kernels) on the
    same small case as the CPU baseline, stepped as many times: relative
    error of x (floor 1e-12) and T on every cell against the oracle's state."""
    import numpy as np
    spec, nH, x, E = _cpu_case(n)
    g = binding.Grid(spec, precision=precision)
    g.nH.copy_(torch.as_tensor(nH, dtype=g.dtype))
    g.x.copy_(torch.as_tensor(x, dtype=g.dtype))
    g.E.copy_(torch.as_tensor(E, dtype=g.dtype))
    g.raytrace()
    g.set_time(0.0, 0)
    for _ in range(steps):
        g.step_o2(1e30)
    torch.cuda.synchronize()
    xg = g.x.double().cpu().numpy()
    Eg = g.E.double().cpu().numpy()
    g.close()
    T = lambda xx, EE: 2.0 * EE / (3.0 * 1.380649e-16 * st["nH"] * (2.0 - xx))
    ex = np.abs(xg - st["x"]) / np.maximum(np.abs(st["x"]), 1e-12)
    eT = np.abs(T(xg, Eg) / T(st["x"], st["E"]) - 1.0)
    return {"case": f"benchmark recipe at {n}^3, {steps} A3 steps from the synthetic front start",
            "x_max": float(ex.max()), "x_p999": float(np.quantile(ex, 0.999)),
            "T_max": float(eT.max()), "T_p999": float(np.quantile(eT, 0.999)),
            "bar": 1e-9 if precision == "fp64" else 1e-4}


def bench_batch(args, torch, binding, synth) -> dict:
    """Batched form: the generated set of uneven grids (n uniform in 32..160,
    uniform or lognormal media, Q log-uniform in 1e47..1e50) advanced together,
    one graph replay per step; beside it the FP64 single-grid path on a
    sample of the same grids, one grid at a time."""
    specs = synth.batch_specs(args.batch_grids, seed=0, precision=args.precision)
    tick = time.time()
    nHs = [synth.density(s) for s in specs]
    print(f"# batch: {len(specs)} grids, {sum(s.ncells for s in specs) / 1e6:.1f} M cells, "
          f"densities in {time.time() - tick:.1f} s", file=sys.stderr, flush=True)
    bt = binding.Batch(specs, precision=args.precision)
    bt.load(nHs, T0s=[s.T0 for s in specs], t_end=[s.t_end for s in specs])
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        bt.step_o2()
    torch.cuda.synchronize()
    _, n0, _ = bt.state()
    bt.work_counters(reset=True)   # the timed steps' work only
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        bt.step_o2()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    _, n1, _ = bt.state()
    cells = sum(s.ncells * (b - a) for s, a, b in zip(specs, n0, n1))
    value = cells / (ms * 1e-3)
    work = bt.work_counters(reset=True)
    tile = bt.raytrace_tile
    bt.close()
    del bt
    torch.cuda.empty_cache()
    # FP64 single-grid path on a sample of the same grids
    sample = specs[:args.batch_fp64_sample]
    tot_cells, tot_ms = 0.0, 0.0
    for s, nH in zip(sample, nHs):
        g = binding.Grid(s, precision="fp64")
        g.load(nH, 1.0, T0=s.T0)
        g.step_o2(s.t_end)
        torch.cuda.synchronize()
        a, b2 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(3):
            g.step_o2(s.t_end)
        b2.record(stream)
        torch.cuda.synchronize()
        tot_cells += 3 * s.ncells
        tot_ms += a.elapsed_time(b2)
        g.close()
    fp64_plain = tot_cells / (tot_ms * 1e-3)
    # the whole batched step against the FP32 issue rate (counted flops, as
    # for the single grid: Newton iterations from the work counters, two
    # micro-integration set-ups and raytraces per cell-update) and against HBM
    # (seven words per cell-update)
    flops = work["newton"] * FLOP_NEWTON + 2 * cells * (FLOP_CELL_SETUP + FLOP_SWEEP_CELL)
    achieved = flops / (ms * 1e-3) / 1e12
    step_gbs = STEP_WORDS * word_bytes(args.precision) * cells / (ms * 1e-3) / 1e9
    roofline = {"bound": "alu", "kernel": "whole batched step (timestep, micro-physics, "
                                          "re-solve, raytrace)",
                "achieved": round(achieved, 3), "peak": VALU_PEAK[args.precision],
                "unit": "TFLOP/s", "frac": round(achieved / VALU_PEAK[args.precision], 5),
                "peak_note": VALU_PEAK_NOTE, "traffic": None,
                "flops_per_step": flops / args.steps,
                "hbm_of_step": {"bytes_per_cell_update": STEP_WORDS * word_bytes(args.precision),
                                "achieved": round(step_gbs, 2), "peak": HBM_PEAK_GBS,
                                "unit": "GB/s", "frac": round(step_gbs / HBM_PEAK_GBS, 5)}}
    return {
        "metric": "cell-updates/s of the batched A3 step, 64 uneven grids",
        "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": dtype_name(args.precision),
        "data": "synthetic",
        "config": {"workload": f"batch of {len(specs)} grids, n uniform in 32..160, uniform or "
                               "lognormal media, Q log-uniform 1e47..1e50, 1e5 K blackbody table, "
                               "T evolving, A3-dt02, from a neutral start",
                   "cells": sum(s.ncells for s in specs), "precision": args.precision,
                   "raytrace_tile": tile,
                   "fp64_single_grid_rate": fp64_plain,
                   "fp64_single_grid_sample": len(sample),
                   "ratio_to_fp64_single_grid": value / fp64_plain,
                   "fp64_resolved_frac": work["resolved_fp64"] / max(1, cells)},
        "roofline": roofline,
    }


def bench_hardening(args, torch, binding, synth) -> dict:
    """Spectral-hardening runs of Sect. 4 (37 500 K blackbody; cell optical
    depth 1, 3, 10, 30 with n_H = 10, 100, 1000): the twelve grids advanced as
    one batch, timed over K steps from the neutral start; then each run is
    taken to 0.1 t_rec with dt02 and, in a second batch, with four times
    smaller steps (K4 = 1/16), and the front radii are compared."""
    INF = synth.INF
    specs = synth.hardening_specs(args.precision)
    nHs = [synth.density(s) for s in specs]
    stream = torch.cuda.current_stream()

    def make(K):
        sp = [s.with_(K=K, t_end=args.hardening_trec * s.t_rec) for s in specs]
        b = binding.Batch(sp, precision=args.precision)
        b.load(nHs, T0s=[s.T0 for s in sp], t_end=[s.t_end for s in sp])
        return b

    bt = make(synth.EXPLICIT_CRITERIA["dt02"])
    for _ in range(args.warmup):
        bt.step_o2()
    torch.cuda.synchronize()
    _, n0, _ = bt.state()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        bt.step_o2()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    _, n1, _ = bt.state()
    cells = sum(s.ncells * (b - a) for s, a, b in zip(specs, n0, n1))
    value = cells / (ms * 1e-3)
    tick = time.time()
    bt.run()
    _, steps_dt02, _ = bt.state()
    r_dt02 = [d["r_ion"] for d in bt.diagnostics()]
    print(f"# hardening: dt02 runs to {args.hardening_trec} t_rec in {time.time() - tick:.1f} s",
          file=sys.stderr, flush=True)
    bt.close()
    tick = time.time()
    ref = make((INF, INF, INF, 1.0 / 16))
    ref.run()
    r_ref = [d["r_ion"] for d in ref.diagnostics()]
    print(f"# hardening: reference runs in {time.time() - tick:.1f} s", file=sys.stderr, flush=True)
    ref.close()
    runs = []
    for s, a, b2, k in zip(specs, r_dt02, r_ref, steps_dt02):
        RS = 150.0 / (s.nH_mean * synth.SIGMA0)
        runs.append({"dtau0": round(s.dx * s.nH_mean * synth.SIGMA0, 6), "nH": s.nH_mean,
                     "n": s.n[0], "steps_dt02": int(k), "r_ion_over_RS": a / RS,
                     "rel_err_vs_K4_1_16": a / b2 - 1})
    return {
        "metric": "cell-updates/s of the batched A3 step, spectral-hardening runs",
        "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": dtype_name(args.precision),
        "data": "synthetic",
        "config": {"workload": "12 grids: 37500 K blackbody table, cell optical depth 1, 3, 10, 30 "
                               "x n_H 10, 100, 1000 (tau_S 150, Q ~ 1/n_H), corner source, T "
                               "evolving from 50 K, A3-dt02, from a neutral start",
                   "cells": sum(s.ncells for s in specs), "precision": args.precision,
                   "runs_to_trec": args.hardening_trec, "runs": runs},
    }


def bench_a1(args, torch, binding, synth) -> dict:
    """Algorithm 1 (implicit, time-averaged attenuation) on the same 256^3
    clumpy medium as the default workload, with Table 1's implicit dt02
    (steps of a tenth of the recombination time), from the state the A3
    pre-evolution reaches at 0.1 t_rec."""
    INF = synth.INF
    spec = synth.cfg3(n=args.n).with_(precision=args.precision)
    g = binding.Grid(spec, precision=args.precision)
    g.load(synth.density(spec), 1.0, T0=spec.T0)
    g.run(args.pre_trec * spec.t_rec, check_every=16)
    t0, n0, _ = g.state()
    ga = binding.Grid(spec.with_(K=(0.1, INF, INF, INF)), precision=args.precision)
    for k in ("nH", "x", "E", "tau"):
        getattr(ga, k).copy_(getattr(g, k))
    ga.set_time(t0, n0)
    g.close()
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        ga.step_a1(1e30)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        ga.step_a1(1e30)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    _, _, dt = ga.state()
    ga.close()
    return {
        "metric": "cell-updates/s of algorithm 1 steps at 256^3",
        "value": spec.ncells * args.steps / (ms * 1e-3), "unit": "cell-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": dtype_name(args.precision), "data": "synthetic",
        "config": {"workload": f"cfg3 clumpy medium {args.n}^3, algorithm 1 with implicit dt02 "
                               f"(K1 = 0.1), from the A3 state at {args.pre_trec} t_rec",
                   "precision": args.precision, "dt_over_trec": dt / spec.t_rec},
    }


def bench_sources(args, torch, binding, synth) -> dict:
    """The same 256^3 clumpy medium lit by four point sources (the central
    one and three off-centre ones of half its rate), A3 steps from the state
    the pre-evolution reaches at 0.1 t_rec."""
    n = args.n
    base = synth.cfg3(n=n).with_(precision=args.precision)
    more = tuple(((v[0] * n // 256, v[1] * n // 256, v[2] * n // 256), 0.5 * base.Q)
                 for v in ((64, 64, 64), (192, 80, 160), (100, 200, 48)))
    spec = base.with_(more_sources=more)
    g = binding.Grid(spec, precision=args.precision)
    g.load(synth.density(spec), 1.0, T0=spec.T0)
    g.run(args.pre_trec * spec.t_rec, check_every=16)
    stream = torch.cuda.current_stream()
    t_end = 1e30
    for _ in range(args.warmup):
        g.step_o2(t_end)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        g.step_o2(t_end)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    d = g.diagnostics()
    g.close()
    return {
        "metric": "cell-updates/s of A3 steps at 256^3 with four point sources",
        "value": spec.ncells * args.steps / (ms * 1e-3), "unit": "cell-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": dtype_name(args.precision), "data": "synthetic",
        "config": {"workload": f"cfg3 clumpy medium {n}^3 lit by 4 point sources (central "
                               f"5e48 /s and three of 2.5e48 /s), A3-dt02 from {args.pre_trec} t_rec",
                   "precision": args.precision, "octants": d["octants"]},
    }


def bench_serve(args, torch, binding, synth) -> dict:
    """Served form: Poisson arrivals of single-grid requests submitted to the
    library's server at their arrival times; latency from submission to
    completion."""
    import numpy as np
    reqs = synth.poisson_requests(args.serve_requests, rate=args.serve_rate, seed=5651,
                                  nmin=args.serve_nmin, nmax=args.serve_nmax,
                                  n_outlier=2 * args.serve_nmax, p_outlier=args.serve_outliers,
                                  precision=args.precision)
    reqs = [(t, synth.GridSpec(**{**s.__dict__, "t_end": args.serve_trec * s.t_rec})) for t, s in reqs]
    tick = time.time()
    nHs = [synth.density(s) for _, s in reqs]
    print(f"# serve: {len(reqs)} requests, densities in {time.time() - tick:.1f} s",
          file=sys.stderr, flush=True)
    srv = binding.Server(precision=args.precision, hbm_budget=0, max_active=args.serve_max_active,
                         steps_per_tick=args.serve_steps_per_tick)
    # warm-up: a few requests of the same kind (other seed) run to completion
    # first, so the timed stream sees a server whose rate tables and raytrace
    # tiles are set up (a serving workload has a warm-up period)
    warm = synth.poisson_requests(args.serve_warmup, rate=args.serve_rate, seed=15651,
                                  nmin=args.serve_nmin, nmax=args.serve_nmax, p_outlier=0.0,
                                  precision=args.precision) if args.serve_warmup > 0 else []
    wt = []
    for _, s in warm:
        s = synth.GridSpec(**{**s.__dict__, "t_end": args.serve_trec * s.t_rec})
        wt.append(srv.submit(s, synth.density(s), T0=s.T0, t_end=s.t_end))
    while wt:
        wt = [tk for tk in wt if srv.poll(tk)[0] == binding.PI_PENDING]
        time.sleep(0.002)
    base = srv.stats()
    pending, done = {}, {}
    t0 = time.perf_counter()
    i = 0
    last = t0
    while i < len(reqs) or pending:
        now = time.perf_counter() - t0
        while i < len(reqs) and reqs[i][0] <= now:
            s = reqs[i][1]
            pending[srv.submit(s, nHs[i], T0=s.T0, t_end=s.t_end)] = i
            i += 1
        for tk in list(pending):
            st, info, _, _ = srv.poll(tk)
            if st != binding.PI_PENDING:
                done[pending.pop(tk)] = (st, info)
        if time.perf_counter() - last > 20:
            last = time.perf_counter()
            print(f"# serve: {len(done)} done, {len(pending)} pending, {now:.0f} s",
                  file=sys.stderr, flush=True)
        time.sleep(0.002)
    wall = time.perf_counter() - t0
    stats = srv.stats()
    for k in ("completed", "cell_updates", "busy_s", "steps", "rebuilds"):
        stats[k] -= base[k]   # the timed stream only
    srv.close()
    lat = np.array([info["latency_s"] for st, info in done.values()])
    que = np.array([info["queue_s"] for st, info in done.values()])
    ok = sum(1 for st, _ in done.values() if st == binding.PI_OK)
    # offered load: the cell-updates the stream asks for per second of arrivals
    span = reqs[-1][0] if reqs else 1.0
    return {
        "metric": "served A3 solves: cell-updates/s and p50/p99 latency",
        "value": stats["cell_updates"] / wall, "unit": "cell-updates/s", "n_gpus": 1,
        "steps": int(stats["steps"]), "warmup": args.serve_warmup,
        "ms_per_step": 1e3 * stats["busy_s"] / max(1, stats["steps"]),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": dtype_name(args.precision), "data": "synthetic",
        "config": {"workload": f"{len(reqs)} requests, Poisson arrivals at {args.serve_rate}/s, n "
                               f"uniform in {args.serve_nmin}..{args.serve_nmax} "
                               f"({100 * args.serve_outliers:g}% at {2 * args.serve_nmax}), source "
                               f"in the central half, uniform or lognormal media of mean 1..100 "
                               f"cm^-3, Q 1e47..1e50 /s, cfg2 physics, each to {args.serve_trec} "
                               f"t_rec(mean)",
                   "completed_ok": ok, "wall_s": wall, "busy_s": stats["busy_s"],
                   "offered_cell_updates_per_s": stats["cell_updates"] / max(span, 1e-9),
                   "latency_p50_s": float(np.quantile(lat, 0.5)),
                   "latency_p99_s": float(np.quantile(lat, 0.99)),
                   "queue_p50_s": float(np.quantile(que, 0.5)),
                   "queue_p99_s": float(np.quantile(que, 0.99)),
                   "batch_rebuilds": int(stats["rebuilds"])},
    }


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--precision", default="mixed", choices=["fp64", "fp32", "mixed", "mixed_front"])
    ap.add_argument("--front-steps", type=int, default=6,
                    help="default workload: steps timed with the FP64 front cells (mixed_front) "
                         "from the same state; 0 skips")
    ap.add_argument("--pre-trec", type=float, default=0.1,
                    help="untimed evolution before timing, in units of t_rec")
    ap.add_argument("--pre-steps-max", type=int, default=400)
    ap.add_argument("--phase-reps", type=int, default=4,
                    help="back-to-back launches per phase in the phase timing")
    ap.add_argument("--phase-steps", type=int, default=3,
                    help="extra steps timed phase by phase after the timed region")
    ap.add_argument("--cpu-sample-n", type=int, default=48,
                    help="single-thread CPU baseline (and error check) at this n^3")
    ap.add_argument("--cpu-budget", type=float, default=10.0)
    ap.add_argument("--cpu-omp-n", type=int, default=128,
                    help="OpenMP CPU baseline leg at this n^3")
    ap.add_argument("--cpu-omp-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--raytrace-tile", default="auto", choices=["auto", "4", "8", "16", "persistent"],
                    help="raytrace variant of the timed grid (auto: the library's tuning on its "
                         "first raytrace)")
    ap.add_argument("--no-serve", action="store_true",
                    help="default workload: skip the served-stream leg (p50/p99 latency)")
    ap.add_argument("--omp-leg", nargs=2, type=int, metavar=("N", "STEPS"), default=None,
                    help=argparse.SUPPRESS)
    ap.add_argument("--workload", default="cfg3",
                    choices=["cfg3", "batch", "serve", "hardening", "a1", "sources"],
                    help="cfg3: the 256^3 single grid (default); batch / serve: the batched and "
                         "served forms (their own JSON line)")
    ap.add_argument("--hardening-trec", type=float, default=1.0,
                    help="hardening workload: accuracy runs end at this many t_rec")
    ap.add_argument("--batch-grids", type=int, default=64)
    ap.add_argument("--batch-fp64-sample", type=int, default=8)
    # the served stream: config 5's sizes and run length (n 48..256, each to
    # 2 t_rec) at an arrival rate the GPU sustains (2 /s; config 5 names
    # 20 /s, above this GPU's throughput for such requests), without the 1%
    # of 512^3 outliers unless --serve-outliers says otherwise
    ap.add_argument("--serve-requests", type=int, default=120)
    ap.add_argument("--serve-warmup", type=int, default=4,
                    help="requests run to completion before the timed stream (not counted)")
    ap.add_argument("--serve-rate", type=float, default=2.0)
    ap.add_argument("--serve-nmin", type=int, default=48)
    ap.add_argument("--serve-nmax", type=int, default=256)
    ap.add_argument("--serve-trec", type=float, default=2.0)
    ap.add_argument("--serve-outliers", type=float, default=0.0,
                    help="fraction of requests at twice nmax (config 5: 0.01)")
    ap.add_argument("--serve-max-active", type=int, default=64)
    ap.add_argument("--serve-steps-per-tick", type=int, default=4)
    ap.add_argument("--time-tiles", action="store_true",
                    help="also time one raytrace with each tile edge (in config.raytrace_ms_by_tile)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (a known-size "
                         "reference for hardware traffic counters)")
    args = ap.parse_args()
    if args.omp_leg:
        return omp_leg(*args.omp_leg)

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (grids "
              "and octants would shard across GPUs with no exchange but two FP64 scalars "
              "per step); run with --gpus 1", file=sys.stderr)
        return 2

    import torch

    from paper_1201_5651_amd import binding, synth

    torch.cuda.set_device(0)
    if args.workload != "cfg3":
        fn = {"batch": bench_batch, "serve": bench_serve, "hardening": bench_hardening,
              "a1": bench_a1, "sources": bench_sources}[args.workload]
        print(json.dumps(fn(args, torch, binding, synth)))
        return 0
    spec = synth.cfg3(n=args.n)
    nH = synth.density(spec)
    g = binding.Grid(spec, precision=args.precision)
    if args.raytrace_tile != "auto":
        g.raytrace_tile = (binding.PI_TILE_PERSISTENT if args.raytrace_tile == "persistent"
                           else int(args.raytrace_tile))
    g.load(nH, 1.0, T0=spec.T0)
    t_end = 1e30   # open-ended: every step is a full step

    # untimed pre-evolution to the benchmark state
    t_pre = args.pre_trec * spec.t_rec
    pre = 0
    tick = time.time()
    while pre < args.pre_steps_max:
        burst = min(25, args.pre_steps_max - pre)
        for _ in range(burst):
            g.step_o2(t_pre)
        t, n, _ = g.state()
        pre = n
        print(f"# pre-evolution: {pre} steps, t = {t / spec.t_rec:.4f} t_rec, "
              f"{time.time() - tick:.1f} s", file=sys.stderr, flush=True)
        if t >= t_pre:
            break
    t_start, n_start, _ = g.state()

    for _ in range(args.warmup):
        g.step_o2(t_end)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        g.step_o2(t_end)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    ms_step = ms / args.steps
    value = spec.ncells * args.steps / (ms * 1e-3)

    work = g.work_counters(reset=True)   # over pre-evolution + warm-up + timed steps

    # phase-by-phase timing of the same launches (same stream, HIP events):
    # each phase is launched `phase_reps` times back to back between two events
    # on inputs it does not modify, so that the per-launch figure carries no
    # event overhead.  predictor and corrector are the step's two halves, each
    # the micro-physics followed by the raytrace of its result (pi_chem_raytrace:
    # one fused launch when the grid's raytrace is the persistent one, and for
    # mixed precision the double re-solve and the conditional second raytrace
    # after it).  The corrector's repetitions write their state to the
    # half-step buffers and their columns to tau (both rewritten before they
    # are read again); one untimed corrector then moves state n on as in a
    # step.  raytrace_alone: the raytrace by itself, for reference.
    phases = {"timestep": 0.0, "predictor": 0.0, "corrector": 0.0, "raytrace_alone": 0.0}
    R = args.phase_reps
    P_N, P_H = binding.PI_BUF_N, binding.PI_BUF_HALF
    timed = {
        "timestep": lambda: g.timestep(t_end),
        "predictor": lambda: g.chem_raytrace(0.5, P_N, P_N, P_H, P_H, use_device_dt=True),
        "corrector": lambda: g.chem_raytrace(1.0, P_H, P_N, P_H, P_N, use_device_dt=True),
        "raytrace_alone": lambda: g.raytrace(P_N, P_N),
    }
    g.work_counters(reset=True)
    work_phase = {}
    for _ in range(args.phase_steps):
        for k, fn in timed.items():
            if k == "raytrace_alone":
                # the step's own corrector (untimed, counters excluded)
                w = g.work_counters(reset=True)
                for c, v in w.items():
                    work_phase[c] = work_phase.get(c, 0) + v
                g.chem_raytrace(1.0, P_H, P_N, P_N, P_N, use_device_dt=True)
                torch.cuda.synchronize()
                g.work_counters(reset=True)
            a, b2 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(R):
                fn()
            b2.record(stream)
            torch.cuda.synchronize()
            phases[k] += a.elapsed_time(b2) / (R * args.phase_steps)
    chem_launches = 2 * R * args.phase_steps
    if args.calib_copy_mib > 0:
        nel = args.calib_copy_mib * 2**20 // 4
        src = torch.ones(nel, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    tiles_ms = None
    if args.time_tiles:
        tuned = g.raytrace_tile
        tiles_ms = {}
        for edge in (4, 8, 16):
            g.raytrace_tile = edge
            g.raytrace()
            a, b2 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(10):
                g.raytrace()
            b2.record(stream)
            torch.cuda.synchronize()
            tiles_ms[edge] = a.elapsed_time(b2) / 10
        g.raytrace_tile = tuned
    diag = g.diagnostics()
    t_now, n_now, _ = g.state()

    # the same state advanced with the ionisation-front cells in double
    front_leg = None
    if args.front_steps > 0 and args.precision == "mixed":
        gf = binding.Grid(spec, precision="mixed_front")
        for k in ("nH", "x", "E", "tau"):
            getattr(gf, k).copy_(getattr(g, k))
        gf.set_time(t_now, n_now)
        gf.raytrace_tile = g.raytrace_tile
        gf.step_o2(t_end)
        gf.work_counters(reset=True)
        torch.cuda.synchronize()
        a, b2 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(args.front_steps):
            gf.step_o2(t_end)
        b2.record(stream)
        torch.cuda.synchronize()
        fms = a.elapsed_time(b2) / args.front_steps
        wf = gf.work_counters(reset=True)
        front_leg = {"precision": "mixed_front", "dtype": dtype_name("mixed_front"),
                     "detail": PRECISION_DETAIL["mixed_front"], "steps": args.front_steps,
                     "ms_per_step": fms, "value": spec.ncells / (fms * 1e-3),
                     "fp64_resolved_frac": wf["resolved_fp64"] / (2 * args.front_steps * spec.ncells)}
        gf.close()

    W = word_bytes(args.precision)
    N = spec.ncells
    newton_per_launch = work_phase["newton"] / chem_launches
    fused = g.raytrace_tile == binding.PI_TILE_PERSISTENT and args.precision in ("fp32", "mixed")
    # algorithmic bytes per launch: a half step (micro-physics and the raytrace
    # of its result) reads n_H, x, E, tau and writes x, E, tau (7 words per
    # cell); the timestep reads n_H, x, E, tau (4 words); a raytrace alone reads
    # n_H, x and writes tau (3 words)
    alg = {"predictor": 7 * W * N, "corrector": 7 * W * N, "timestep": 4 * W * N,
           "raytrace_alone": 3 * W * N}
    hbm = {k: alg[k] / (phases[k] * 1e-3) / 1e9 for k in phases}
    dom = max(("timestep", "predictor", "corrector"), key=phases.get)
    # the whole step against HBM: seven words per cell-update
    step_gbs = STEP_WORDS * W * N / (ms_step * 1e-3) / 1e9
    hbm_view = {"kernel": dom, "achieved": round(hbm[dom], 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(hbm[dom] / HBM_PEAK_GBS, 5),
                "bytes_per_launch": alg[dom]}
    step_view = {"bytes_per_cell_update": STEP_WORDS * W, "achieved": round(step_gbs, 2),
                 "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(step_gbs / HBM_PEAK_GBS, 5)}
    if fused:
        kname = "k_chem_sweep" + (" (+ k_chem_fix, conditional k_sweep_persist)"
                                  if args.precision == "mixed" else "")
    else:
        kname = "k_chem" + (" + k_chem_fix" if args.precision in ("mixed", "mixed_front") else "") \
                + " + raytrace"
    if dom != "timestep":
        # a half step is bound by the vector arithmetic of the micro-physics:
        # a few words of HBM per cell against hundreds of flops
        flops = newton_per_launch * FLOP_NEWTON + N * (FLOP_CELL_SETUP + FLOP_SWEEP_CELL)
        t_half = 0.5 * (phases["predictor"] + phases["corrector"])
        achieved = flops / (t_half * 1e-3) / 1e12
        peak = VALU_PEAK[args.precision]
        roofline = {"bound": "alu", "kernel": kname + " (" + dom + ")",
                    "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                    "frac": round(achieved / peak, 5), "peak_note": VALU_PEAK_NOTE,
                    "traffic": measured_traffic() if (args.precision == "mixed" and args.n == 256
                                                      and fused) else None,
                    "flops_per_launch": flops, "launch_ms": round(t_half, 4)}
    else:
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(hbm[dom], 2),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(hbm[dom] / HBM_PEAK_GBS, 5),
                    "traffic": None}
    roofline["hbm_of_dominant"] = hbm_view
    roofline["hbm_of_step"] = step_view
    roofline["phase_ms"] = {k: round(v, 4) for k, v in phases.items()}
    roofline["raytrace_alone_hbm"] = {"achieved": round(hbm["raytrace_alone"], 2), "unit": "GB/s",
                                      "frac": round(hbm["raytrace_alone"] / HBM_PEAK_GBS, 5)}

    out = {
        "metric": "cell-updates/s per raytrace+chemistry step at 256^3; p50/p99 batched solve latency",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype_name(args.precision),
        "data": "synthetic",
        "config": {
            "workload": f"cfg3 clumpy medium {args.n}^3: lognormal n_H (sigma_ln 1, k^-11/3, seed "
                        f"1201), mean 5 cm^-3, central 1e5 K blackbody Q=5e48/s, 64-node rate "
                        f"table, T evolving, A3-dt02, pre-evolved to {args.pre_trec} t_rec",
            "n": args.n, "precision": args.precision, "pre_steps": int(n_start),
            "t_start_trec": t_start / spec.t_rec, "t_end_trec": t_now / spec.t_rec,
            "r_ion_cells": diag["r_ion"] / spec.dx, "n_sub": spec.n_sub,
            "raytrace_tile": g.raytrace_tile,
            "raytrace_ms_by_tile": tiles_ms,
            "substeps_per_cell_update": (work_phase["accepted"] + work_phase["rejected"])
            / (spec.ncells * chem_launches / 2),
            "rejected_frac": work_phase["rejected"]
            / max(1, work_phase["accepted"] + work_phase["rejected"]),
            "fallbacks_per_cell_update": work_phase["fallbacks"] / (spec.ncells * chem_launches / 2),
            "newton_per_cell_update": work_phase["newton"] / (spec.ncells * chem_launches / 2),
            "fp64_resolved_frac": work_phase["resolved_fp64"] / (spec.ncells * chem_launches),
            "precision_detail": PRECISION_DETAIL[args.precision],
        },
        "roofline": roofline,
    }
    if front_leg is not None:
        out["front_fp64"] = front_leg
    g.close()
    del g
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        print("# cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"], (k, pb, st) = cpu_baseline(args.cpu_sample_n, args.cpu_budget,
                                                        args.cpu_omp_n, args.cpu_omp_steps)
        # the headline's kernels against the oracle's steps of that sample
        out["error_vs_oracle"] = error_vs_oracle(torch, binding, args.cpu_sample_n, k, pb, st,
                                                 args.precision)
    if not args.no_serve:
        print("# served stream", file=sys.stderr, flush=True)
        sv = bench_serve(args, torch, binding, synth)
        c = sv["config"]
        out["latency"] = {"p50_s": c["latency_p50_s"], "p99_s": c["latency_p99_s"],
                          "queue_p50_s": c["queue_p50_s"], "queue_p99_s": c["queue_p99_s"],
                          "cell_updates_per_s": sv["value"],
                          "offered_cell_updates_per_s": c["offered_cell_updates_per_s"],
                          "requests": args.serve_requests, "completed_ok": c["completed_ok"],
                          "stream": c["workload"], "wall_s": c["wall_s"]}
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
