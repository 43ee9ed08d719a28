"""Throughput of the DG shallow-water hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp64|fp32]

Workload (default): 512x512x2 triangulation of a 100 km square, nodes jittered
by U(-0.2h, 0.2h) (seed 2), uniform order p = 2, bathymetry
10 m + 3990 m (1 + sin(2 pi x/L) cos(2 pi y/L))/2, lake at rest, west edge
open and forced by a 0.5 m tide of period 44712 s, Coriolis 3.19e-5 1/s,
quadratic friction 0.009.  A step is one SSP-RK2 step (two stages) of the
whole hot path: volume + source + edge fluxes + stage update + u H = q.
Metric: DOF-updates per second per RK stage, DOF = 3 * sum_e K(p_e).
Inputs are resident in HBM before the timed region.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
K_OF_P = (1, 3, 6, 10)


def stage_bytes_per_element(p: int, word: int, nv: int, ne: int) -> float:
    """Algorithmic HBM bytes one element moves in one stage kernel (average of
    the two SSP-RK2 stages): read c (3K) and u (2K), read c^n (3K) in the
    second stage only, write c (3K) and u (2K); geometry: 3 vertex ids, 3
    neighbour ids, 1 packed neighbour-edge byte, and the element's share of
    the 32-byte vertex records.  Neighbour coefficients are counted once (as
    their owner's read): they are served from cache."""
    K = K_OF_P[p]
    state = (3 * K + 2 * K + 0.5 * 3 * K + 3 * K + 2 * K) * word
    geo = 3 * 4 + 3 * 4 + 1 + 32.0 * nv / ne
    return state + geo


def cpu_baseline(p: int, budget_s: float = 15.0):
    """The FP64 oracle (single thread) on a bounded sample of the same workload:
    the same problem family on a coarser mesh, timed over whole SSP-RK2 steps."""
    from oracle.oracle import Oracle
    from paper_2311_11348_amd import inputs as I
    n = 64
    prob = I.config_c2(n=n, p=p)
    orc = Oracle.from_problem(prob)
    c0 = orc.project(prob.ic)
    dt = prob.dt()
    t0 = time.perf_counter()
    c = orc.step(c0, 1, dt)
    one = time.perf_counter() - t0
    steps = max(1, int(budget_s / max(one, 1e-3)))
    t0 = time.perf_counter()
    orc.step(c, steps, dt, t0=dt)
    el = time.perf_counter() - t0
    dof = 3 * K_OF_P[p] * prob.mesh.ne
    return {"value": dof * 2 * steps / el, "unit": "DOF-updates/s per RK stage", "cores": 1,
            "kind": "oracle",
            "sample": f"{n}x{n}x2 mesh of the same workload family ({prob.mesh.ne} elements, p={p}), "
                      f"{steps} SSP-RK2 steps, FP64, single thread, {el:.1f} s"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--p", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (instances and "
              "meshes shard without communication across GPUs, see the design notes)",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch
    from paper_2311_11348_amd import inputs as I
    from paper_2311_11348_amd import swe

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    prec = swe.SWE_FP64 if args.precision == "fp64" else swe.SWE_FP32_WB
    word = 8 if prec == swe.SWE_FP64 else 4
    prob = I.config_c2(n=args.n, p=args.p)
    stream = torch.cuda.Stream()
    print(f"bench: building {prob.mesh.ne} elements, p={args.p}, {args.precision}", file=sys.stderr, flush=True)
    ctx = swe.context_for(prob, precision=prec, stream_base=stream.cuda_stream)
    ctx.set_state_fn(prob.ic)
    dt = prob.dt()
    ctx.step(args.warmup, dt)
    ctx.sync()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t_wall0 = time.perf_counter()
    ev0.record(stream)
    ctx.step(args.steps, dt)
    ev1.record(stream)
    ctx.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall0
    gpu_ms = ev0.elapsed_time(ev1)
    ne, nv = prob.mesh.ne, prob.mesh.nv
    dof = 3 * K_OF_P[args.p] * ne
    stages = 2 * args.steps
    value = dof * stages / (gpu_ms * 1e-3)
    launch_s = gpu_ms * 1e-3 / stages
    bpe = stage_bytes_per_element(args.p, word, nv, ne)
    achieved = bpe * ne / launch_s / 1e9
    out = {
        "metric": "DOF-updates/s per RK stage",
        "value": value,
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": gpu_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == swe.SWE_FP64 else "f32 (f64 bathymetry terms)",
        "data": "synthetic",
        "config": {"workload": f"tidal: {args.n}x{args.n}x2 jittered triangulation, {ne} elements, "
                               f"p={args.p} uniform, sin*cos bathymetry 10-4000 m, west tide",
                   "elements": ne, "order": args.p, "dof": dof, "precision": args.precision},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_stage (fused volume+source+edges+RK+u-solve)",
                     "bytes_per_launch": bpe * ne, "avg_launch_us": launch_s * 1e6},
        "wall_s": wall,
    }
    if not args.no_cpu_baseline:
        print("bench: timing the oracle on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.p)
    ctx.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
