"""Throughput of the DG shallow-water hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
                    [--workload default|tidal|tsunami|static32|dambreak|batched|served|shallow]

default: the tidal headline below (value, roofline, compute roofline, the
  FP64 path beside it, the oracle on the host), with the tsunami, batched and
  served workloads as extra keys of the same line (tsunami timed over at
  least 200 steps, batched over at least 20 steps of every instance, served
  on a 30 s trace); each extra leg that fails records its error instead.
tidal: the headline alone: 512x512x2 triangulation of a 100 km square, nodes jittered
  by U(-0.2h, 0.2h) (seed 2), uniform order p = 2, bathymetry
  10 m + 3990 m (1 + sin(2 pi x/L) cos(2 pi y/L))/2, lake at rest, west edge
  open and forced by a 0.5 m tide of period 44712 s, Coriolis 3.19e-5 1/s,
  quadratic friction 0.009.  The headline value is the FP32 path (FP32 state
  and bulk arithmetic, FP64 bathymetry terms); the FP64 path is measured on
  the same workload and reported beside it.
tsunami: 256x256x2 jittered (seed 3), linear shelf 4000 m -> 50 m, 2 m hump,
  orders in {1,2,3} re-chosen every step by the indicator (threshold 1e-3 m),
  base order 1; the order-separated FP32 path (FP64 bathymetry terms), with
  the order-partitioned FP64 path beside it.
static32: the tidal mesh with base order 1 and every 32nd element at order 2,
  order-separated on two streams, FP32 path.
dambreak: the paper's radial dam break on 1024x1024x2 = 2,097,152 jittered
  triangles of [0,5]^2 (g = 1, h_b = 0.5 m, walls, linear friction), 100
  steps of 1e-5 s as in its static runs: uniform p0, p1, p2 (fused kernel)
  and every 32nd element at the higher order (p0-1, p1-2; order-partitioned
  and order-separated), then dynamic orders (this library's indicator,
  threshold 1e-2 m, the CFL step, 400 steps), FP64 and FP32, each beside the
  paper's own time per stage on its hardware (context).  The value is static
  1/32 p1-2, order-partitioned, FP64.
batched: 64 independent instances (seeds 4000+i), log-uniform 16k-500k
  elements, p in {1,2,3}, tidal or hump, random smooth bathymetry, 300 steps
  each; FP32 and FP64 batched against the plain FP64 solver run one instance
  at a time; reports DOF-updates/s and solves/s.
shallow: the minimum depth control: 512x512x2 jittered mesh (seed 8), bottom
  1 m -> 0.5 m, a -0.6 m Gaussian depression in the middle (0.15 m deep at
  its centre), uniform p = 2, FP32 and FP64 steps with the control
  (h_min = 0.25 m, acting around the depression) and without it.
served: Poisson arrivals (20 req/s for 120 s, seed 5), 8k-260k elements,
  p in {1,2,3}, 200-2000 steps; continuous batching with admission by
  footprint; reports solves/s with p50/p99 latency, then the capacity of
  the batched FP32 server and of the plain FP64 solver on the first 100
  requests offered at once.

A step is one SSP-RK2 step (two stages) of the whole hot path: volume +
source + edge fluxes + stage update + u H = q (+ order update when adaptive).
Metric: DOF-updates per second per RK stage, DOF = 3 * sum_e K(p_e).  Inputs
are resident in HBM before the timed region.  Prints one JSON line.

roofline: the headline kernel's algorithmic bytes per launch (11.5 K words +
100 B per element and stage) over its average launch time in the timed
region (HIP events on the library stream; every launch there is that
kernel), against 8 TB/s; traffic: the HBM bytes its counters read per launch
(a committed counter summary of the same kernel sources), over the same
time.  compute: the method's floating-point operations per launch over the
same time, against the vector peaks.  cpu_baseline: the FP64 oracle on the
host's cores (one process per usable core, up to 16), with a single-process
figure beside it.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
K_OF_P = (1, 3, 6, 10)


def stage_bytes_per_element(p: int, word: int) -> float:
    """Algorithmic HBM bytes one element moves in one RK stage, the practical
    figure of the scope table's measurement row: read c (3K), read c^n (3K)
    in the second stage only (1.5K on average), write c (3K), and the stored
    velocity u (write 2K, read 2K): 11.5 K words, plus G = 100 B of geometry
    (about 80 B of FP64 geometry and 16 B of neighbour ids and codes)."""
    return 11.5 * K_OF_P[p] * word + 100.0


def kernel_bytes_per_element(p: int, word: int, nv: int, ne: int) -> float:
    """The same stage as this library's fused kernel moves it: read c (3K) and
    u (2K), c^n (3K) in stage 2, write c (3K) and u (2K); 3 vertex ids, 3
    neighbour ids, 1 packed neighbour-edge byte and the element's share of
    the 32-byte vertex records (geometry is rebuilt from the vertices, not
    stored).  Neighbour coefficients are counted once, as their owner's read."""
    K = K_OF_P[p]
    state = (3 * K + 2 * K + 0.5 * 3 * K + 3 * K + 2 * K) * word
    geo = 3 * 4 + 3 * 4 + 1 + 32.0 * nv / ne
    return state + geo


# Vector peaks of the MI355X (256 CUs at 2.4 GHz): FP32 157.3 TFLOP/s with
# packed FP32 FMAs, which this library's kernels are built without (half that
# rate per issued instruction), FP64 78.6 TFLOP/s.
FP32_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6


def compute_roofline(p: int, fp32: bool, ne: int, launch_s: float) -> dict:
    """Operations of one stage launch (the method's contractions with the
    reference tensors' exact zero patterns, each edge flux once, see
    paper_2311_11348_amd/flops.py) over the launch time, against the vector
    peak of the bulk precision; the FP64 part of the FP32 path is priced at
    the FP64 rate."""
    from paper_2311_11348_amd import flops as F
    f = F.stage_flops(p)
    bulk = f["total"] * ne
    f64 = f["fp64"] * ne

    def mixed_peak(fp32_rate):
        # the rate at which the launch's work completes at peak: the bulk at
        # the bulk precision's rate, the FP64 part at the FP64 rate
        if not fp32:
            return FP64_PEAK_TFLOPS
        return (bulk + f64) / (bulk / fp32_rate + f64 / FP64_PEAK_TFLOPS)
    peak = mixed_peak(FP32_PEAK_TFLOPS)
    unpacked = mixed_peak(FP32_PEAK_TFLOPS / 2)
    achieved = (bulk + f64) / launch_s / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
            "frac_of_unpacked_peak": achieved / unpacked,
            "flop_per_element": f["total"] + f["fp64"], "fp64_flop_per_element": f["fp64"],
            "flop_per_launch": bulk + f64,
            "peak_note": "vector peaks (FP32 157.3 TFLOP/s with packed FMAs, 78.6 without, which is how "
                         "the kernels are built; FP64 78.6), mixed by the FP64 share of the work on the "
                         "FP32 path"}


def host_description() -> dict:
    """The host the oracle legs run on: logical CPUs, the ones this process
    may use, and the CPU model and socket count from /proc/cpuinfo."""
    model, sockets = None, set()
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name") and model is None:
                    model = line.split(":", 1)[1].strip()
                elif line.startswith("physical id"):
                    sockets.add(line.split(":", 1)[1].strip())
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "usable": len(os.sched_getaffinity(0)), "model": model,
            "sockets": len(sockets) or None}


KERNEL_SOURCES = ("paper_2311_11348_amd/csrc/swe_kernels.hip", "paper_2311_11348_amd/csrc/swe_internal.h",
                  "paper_2311_11348_amd/csrc/swe_tables.h", "paper_2311_11348_amd/build.py")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_stage_p2_tidal512_traffic.txt")
BATCH_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "batched64_traffic.txt")


def kernel_source_hash() -> str:
    """SHA-256 over the sources and build flags that determine the kernels' code."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _traffic_counts(path):
    """key = value lines of a committed PMC summary, or None when it is
    missing or was taken on other kernel sources."""
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if "=" in line and not line.lstrip().startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_hash") != kernel_source_hash():
        return None
    return kv


def _scaled_bytes(kv, kernels):
    """HBM bytes per dispatch of each kernel (FETCH_SIZE and WRITE_SIZE, each
    scaled by what the same counter reads for a copy of known size)."""
    fs = float(kv["copy_bytes"]) / (float(kv["copy_fetch_kib"]) * 1024.0)
    ws = float(kv["copy_bytes"]) / (float(kv["copy_write_kib"]) * 1024.0)
    vals = []
    for k in kernels:
        f, w = kv.get(f"fetch_kib[{k}]"), kv.get(f"write_kib[{k}]")
        if f is None or w is None:
            return None
        vals.append(float(f) * 1024.0 * fs + float(w) * 1024.0 * ws)
    return vals


def measured_traffic(kernels):
    """HBM bytes per launch of the given kernels from the committed PMC summary
    (FETCH_SIZE and WRITE_SIZE runs, each scaled by what the same counter reads
    for a copy kernel of known size), averaged over the kernels; None when the
    summary is missing or the kernel sources changed since it was taken."""
    kv = _traffic_counts(TRAFFIC_FILE)
    vals = _scaled_bytes(kv, kernels) if kv else None
    return sum(vals) / len(vals) if vals else None


def measured_batch_traffic(kernels):
    """HBM bytes of one batch step: the sum over the step's stage launches
    (the given kernels, one launch each per step), from the batched PMC
    summary; None when missing, stale, or a kernel is not in it."""
    kv = _traffic_counts(BATCH_TRAFFIC_FILE)
    vals = _scaled_bytes(kv, kernels) if kv else None
    return sum(vals) if vals else None


def copy_calibration(nbytes: int = 1 << 30, reps: int = 3) -> None:
    """An elementwise copy of nbytes (read nbytes, write nbytes), for scaling
    the HBM byte counters of a profiled run."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    del src, dst


ORACLE_SAMPLE_N = 64


def _oracle_sample(p: int):
    from oracle.oracle import Oracle
    from paper_2311_11348_amd import inputs as I
    prob = I.config_c2(n=ORACLE_SAMPLE_N, p=p)
    orc = Oracle.from_problem(prob)
    c0 = orc.project(prob.ic)
    return prob, orc, c0


def _oracle_worker(p, steps, start, results):
    """One oracle process of the all-core leg: set up, wait at the start
    barrier, run `steps` SSP-RK2 steps, report the elapsed time."""
    prob, orc, c0 = _oracle_sample(p)
    dt = prob.dt()
    start.wait()
    t0 = time.perf_counter()
    orc.step(c0, steps, dt)
    results.put(time.perf_counter() - t0)


def cpu_baseline(p: int, budget_s: float = 10.0) -> dict:
    """The FP64 oracle on the host, on a bounded sample of the headline
    workload: the tidal problem family on a 64x64x2 mesh (8192 elements, the
    same order, bathymetry, forcing and physics), whole SSP-RK2 steps, scaled
    to DOF-updates per second per stage.  First one process on one core
    (about budget_s seconds), then one independent oracle process per usable
    core, started together, each running the same number of steps (the
    oracle is single-threaded and unchanged; its elements are computed one
    after another).  Runs before the GPU is initialised: the worker processes
    are forked from this one."""
    import multiprocessing as mp
    prob, orc, c0 = _oracle_sample(p)
    dt = prob.dt()
    t0 = time.perf_counter()
    c = orc.step(c0, 1, dt)
    one = time.perf_counter() - t0
    steps = max(1, int(budget_s / max(one, 1e-3)))
    t0 = time.perf_counter()
    orc.step(c, steps, dt, t0=dt)
    el = time.perf_counter() - t0
    dof = 3 * K_OF_P[p] * prob.mesh.ne
    single = dof * 2 * steps / el
    host = host_description()
    nproc = min(16, host["usable"] or 1)
    ctx = mp.get_context("fork")
    start, results = ctx.Barrier(nproc + 1), ctx.Queue()
    procs = [ctx.Process(target=_oracle_worker, args=(p, steps, start, results)) for _ in range(nproc)]
    for pr in procs:
        pr.start()
    start.wait()              # every worker has set up: they start together
    times = [results.get() for _ in procs]
    for pr in procs:
        pr.join()
    allcore = nproc * dof * 2 * steps / max(times)
    return {"value": allcore, "unit": "DOF-updates/s", "cores": nproc, "kind": "oracle",
            "sample": f"{ORACLE_SAMPLE_N}x{ORACLE_SAMPLE_N}x2 mesh of the tidal workload family "
                      f"({prob.mesh.ne} elements, p={p}), {steps} SSP-RK2 steps per process, FP64; "
                      f"{nproc} independent oracle processes at once (slowest {max(times):.1f} s); "
                      f"single process {el:.1f} s",
            "single_thread": {"value": single, "cores": 1, "seconds": el},
            "host": host}


def timed_steps(ctx, stream, steps, dt):
    import torch
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    ctx.step(steps, dt)
    ev1.record(stream)
    ctx.sync()
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1)


def run_uniform(prob, precision, steps, warmup):
    """Fused full-order stage kernel on a uniform-order workload."""
    import torch
    from paper_2311_11348_amd import swe
    stream = torch.cuda.Stream()
    ctx = swe.context_for(prob, precision=precision, stream_base=stream.cuda_stream)
    ctx.set_state_fn(prob.ic)
    dt = prob.dt()
    ctx.step(warmup, dt)
    ctx.sync()
    torch.cuda.synchronize()
    ms = timed_steps(ctx, stream, steps, dt)
    ctx.close()
    p = int(prob.p_max)
    ne, nv = prob.mesh.ne, prob.mesh.nv
    word = 8 if precision == swe.SWE_FP64 else 4
    dof = 3 * K_OF_P[p] * ne
    # every launch of the timed region is this kernel (two per step, back to back
    # on the library stream), so the event-timed region / launches is its
    # average launch duration, launch gaps included
    launch_s = ms * 1e-3 / (2 * steps)
    bpe = stage_bytes_per_element(p, word)
    kbpe = kernel_bytes_per_element(p, word, nv, ne)
    achieved = bpe * ne / launch_s / 1e9
    real = "double" if word == 8 else "float"
    traffic = measured_traffic([f"k_stage_sh<{p}, {real}, {m}>" for m in (1, 2)]) if p == 2 and ne == 524288 else None
    return {"value": dof / launch_s, "ms_per_step": ms / steps,
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS,
                         "traffic": traffic / 1e9 / launch_s if traffic is not None else None,
                         "traffic_bytes_per_launch": traffic,
                         "kernel": f"k_stage_sh<{p},{real}> (fused stage, edge fluxes shared within a block)"
                                   if p >= 1 else f"k_stage<{p},{real}> (fused stage, element gather)",
                         "bytes_per_element": bpe, "bytes_per_launch": bpe * ne,
                         "bytes_note": "11.5 K words + 100 B per element and stage (stored velocity, "
                                       "c^n read in the second stage only)",
                         "kernel_bytes_per_launch": kbpe * ne,
                         "frac_kernel_bytes": kbpe * ne / launch_s / 1e9 / HBM_PEAK_GBS,
                         "avg_launch_us": launch_s * 1e6, "launches_timed": 2 * steps},
            "compute": compute_roofline(p, word == 4, ne, launch_s)}


def run_separated(prob, precision, steps, warmup, separate=1, chunk=50, hetero=0):
    """Order-separated scheme (separate=1: base + corrections joined by an
    epilogue; hetero=1: the corrections on the host's cores) or
    order-partitioned scheme (separate=2: base elements and each order's
    listed elements), optionally adaptive.  A static order map runs the
    base and list work on two graph branches, an adaptive one as one chain
    per step.  DOF counts follow the order map, read between timed chunks."""
    import numpy as np
    import torch
    from paper_2311_11348_amd import swe
    stream = torch.cuda.Stream()
    stream2 = torch.cuda.Stream()
    ctx = swe.context_for(prob, precision=precision, separate=separate, stream_base=stream.cuda_stream,
                          stream_corr=stream2.cuda_stream, hetero=hetero)
    ctx.set_state_fn(prob.ic)
    dt = prob.dt()
    ctx.step(warmup, dt)
    ctx.sync()
    torch.cuda.synchronize()
    done, ms, dof_stages = 0, 0.0, 0.0
    kdist = np.zeros(4)
    while done < steps:
        n = min(chunk, steps - done)
        p = ctx.order()
        K = np.asarray(K_OF_P)[p]
        ms += timed_steps(ctx, stream, n, dt)
        p2 = ctx.order()
        K2 = np.asarray(K_OF_P)[p2]
        dof_stages += 3 * 0.5 * (K.sum() + K2.sum()) * 2 * n
        kdist += np.bincount(p2, minlength=4)
        done += n
    ctx.close()
    frac = kdist / kdist.sum()
    return {"value": dof_stages / (ms * 1e-3), "ms_per_step": ms / steps,
            "order_fractions": {f"p{i}": float(frac[i]) for i in range(4) if frac[i] > 0}}


# The paper's times per RK stage (ms) for the dam break on 2,097,152
# triangles (Fig. flow_non-separated, the separated-kernel figure and
# Tab. timings): Jetson AGX Xavier (ARM-AGX: 3 Carmel cores + integrated Volta
# GPU) and 2x EPYC 7742 + Quadro RTX 6000 (AMD-RTX).  Context, not targets.
DAMBREAK_PAPER_MS = {
    "p0": {"ARM-AGX GPU": 28.86, "ARM-AGX CPU": 55.11},
    "p1": {"ARM-AGX GPU": 174.55, "ARM-AGX CPU": 342.31},
    "p2": {"ARM-AGX GPU": 806.55, "ARM-AGX CPU": 1425.03},
    "p0-1 1/32": {"ARM-AGX GPU unseparated": 118.87, "ARM-AGX GPU separated": 144.55,
                  "ARM-AGX CPU+GPU separated": 127.40, "AMD-RTX CPU separated": 24.85,
                  "AMD-RTX GPU separated": 16.12, "AMD-RTX CPU+GPU separated": 101.0},
    "p1-2 1/32": {"ARM-AGX CPU unseparated": 517.70, "ARM-AGX GPU separated": 714.25,
                  "ARM-AGX CPU+GPU separated": 460.01, "AMD-RTX CPU separated": 68.05,
                  "AMD-RTX GPU separated": 72.39, "AMD-RTX CPU+GPU separated": 222.2},
    # dynamic runs: averaged over 12,500 steps, with the paper's own indicator
    # (about 1/482 and 1/172 of the elements at the higher order)
    "p0-1 dynamic": {"ARM-AGX GPU unseparated": 59.80, "ARM-AGX GPU separated": 74.44,
                     "ARM-AGX CPU+GPU separated": 88.1, "ARM-AGX CPU unseparated": 110.92,
                     "ARM-AGX CPU separated": 123.94},
    "p1-2 dynamic": {"ARM-AGX GPU unseparated": 270.92, "ARM-AGX GPU separated": 310.16,
                     "ARM-AGX CPU+GPU separated": 292.7, "ARM-AGX CPU unseparated": 416.16,
                     "ARM-AGX CPU separated": 432.64},
}
DAMBREAK_TAU = 1e-2     # indicator threshold (m) of the dynamic setups
DAMBREAK_HETERO_STEPS = 10   # timed steps of the heterogeneous rows (each stage waits for the host)
DAMBREAK_DYN_STEPS = 400


def run_dambreak(steps, warmup, n=1024, only=None):
    """The radial dam break: uniform orders on the fused stage kernel, the
    statically adaptive 1/32 setups on the order-partitioned and
    order-separated schemes; FP64 and FP32 (``only``: that setup alone)."""
    import numpy as np
    from paper_2311_11348_amd import inputs as I
    from paper_2311_11348_amd import swe
    out = {}
    setups = [("p0", 0, 0, 0), ("p1", 1, 1, 0), ("p2", 2, 2, 0), ("p0-1 1/32", 0, 1, 32), ("p1-2 1/32", 1, 2, 32)]
    for name, lo, hi, every in setups:
        if only is not None and name != only:
            continue
        prob = I.config_dambreak(n=n, p_lo=lo, p_hi=hi, every=every)
        dof = 3 * sum(K_OF_P[q] * c for q, c in enumerate(np.bincount(prob.p, minlength=4)))
        row = {"dof_per_stage": int(dof)}
        for prec, tag in ((swe.SWE_FP64, "fp64"), (swe.SWE_FP32_WB, "fp32")):
            print(f"bench: dambreak {name} {tag} ({prob.mesh.ne} elements)", file=sys.stderr, flush=True)
            if every == 0:
                r = run_uniform(prob, prec, steps, warmup)
                row[tag] = {"scheme": "fused", "ms_per_stage": r["ms_per_step"] / 2, "value": r["value"],
                            "hbm_frac": r["roofline"]["frac"], "kernel": r["roofline"]["kernel"]}
            else:
                for sep, scheme in ((2, "partitioned"), (1, "separated")):
                    r = run_separated(prob, prec, steps, warmup, separate=sep)
                    row[f"{tag}_{scheme}"] = {"ms_per_stage": r["ms_per_step"] / 2, "value": r["value"]}
                # the paper's heterogeneous run: the separated scheme's
                # correction on the host's cores, the base pass on the GPU
                print(f"bench: dambreak {name} {tag} heterogeneous", file=sys.stderr, flush=True)
                r = run_separated(prob, prec, DAMBREAK_HETERO_STEPS, 2, separate=1, hetero=1,
                                  chunk=DAMBREAK_HETERO_STEPS)
                row[f"{tag}_hetero"] = {"ms_per_stage": r["ms_per_step"] / 2, "value": r["value"],
                                        "host_threads": len(os.sched_getaffinity(0)),
                                        "scheme": "separated; correction on the host's cores, base on the GPU"}
        row["paper_ms_per_stage"] = DAMBREAK_PAPER_MS[name]
        out[name] = row
    # dynamic orders: this library's indicator (threshold DAMBREAK_TAU), the
    # CFL step, DAMBREAK_DYN_STEPS timed steps from the start of the run
    for name, lo, hi in (("p0-1 dynamic", 0, 1), ("p1-2 dynamic", 1, 2)):
        if only is not None and name != only:
            continue
        prob = I.config_dambreak(n=n, p_lo=lo, p_hi=hi, dt_fixed=None, adapt_tau=DAMBREAK_TAU)
        row = {"tau_m": DAMBREAK_TAU, "dt_s": prob.dt(), "timed_steps": DAMBREAK_DYN_STEPS}
        for prec, tag in ((swe.SWE_FP64, "fp64"), (swe.SWE_FP32_WB, "fp32")):
            for sep, scheme in ((2, "partitioned"), (1, "separated")):
                print(f"bench: dambreak {name} {tag} {scheme} ({prob.mesh.ne} elements)", file=sys.stderr,
                      flush=True)
                r = run_separated(prob, prec, DAMBREAK_DYN_STEPS, warmup, separate=sep)
                row[f"{tag}_{scheme}"] = {"ms_per_stage": r["ms_per_step"] / 2, "value": r["value"],
                                         "order_fractions": r["order_fractions"]}
        row["paper_ms_per_stage"] = DAMBREAK_PAPER_MS[name]
        out[name] = row
    return out


BATCH_SOLVE_STEPS = 300      # steps of one batched solve in the batched workload


def run_batched(count, steps, warmup):
    """Many independent instances: FP32 and FP64 batched (tile-per-block
    kernels, step graph, autotuned tiles) and the plain FP64 solver (one
    instance at a time, one ordinary launch per stage, on the same FP64
    contexts once they have left the batch).  Each leg runs warmup steps,
    then `steps` timed steps of every instance; solves per second are for
    the workload's 300-step solves at the timed rate.  Inputs are resident
    before timing."""
    import numpy as np
    import torch
    from paper_2311_11348_amd import inputs as I
    from paper_2311_11348_amd import swe
    t_prep = time.perf_counter()
    probs = I.config_c4(count)
    print(f"bench: {count} instances generated in {time.perf_counter() - t_prep:.1f} s, "
          f"{sum(p.mesh.ne for p in probs)} elements", file=sys.stderr, flush=True)
    stream = torch.cuda.Stream()
    dofs = np.array([3 * K_OF_P[p.p_max] * p.mesh.ne for p in probs], dtype=np.float64)
    dts = [p.dt() for p in probs]

    def elapsed(fn):
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        fn()
        ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1)

    def contexts(prec):
        out, t0 = [], time.perf_counter()
        for i, p in enumerate(probs):
            c = swe.context_for(p, precision=prec, stream_base=stream.cuda_stream)
            c.set_state_fn(p.ic)
            out.append(c)
            if i % 16 == 15:
                print(f"bench: {i + 1} contexts (precision {prec}) in {time.perf_counter() - t0:.1f} s",
                      file=sys.stderr, flush=True)
        return out

    def batched(prec, ctxs):
        t0 = time.perf_counter()
        budget = sum(swe.swe_footprint_bytes(c.ne, p.p_max, prec) for c, p in zip(ctxs, probs)) + (8 << 30)
        b = swe.Batch(precision=prec, budget_bytes=budget, max_instances=count, stream=stream.cuda_stream)
        slots = [b.admit(c, steps + warmup, dt) for c, dt in zip(ctxs, dts)]
        b.tune(reps=3)
        tiles = {p: b.tile_config(p) for p in range(4)}
        b.tick(warmup)
        b.sync()
        print(f"bench: batched precision {prec} ready after {time.perf_counter() - t0:.1f} s",
              file=sys.stderr, flush=True)
        ms = elapsed(lambda: b.tick(steps))
        done = b.poll()
        assert len(done) == count and not any(f for _, f in done), done
        out = []
        for s_, c in zip(slots, ctxs):
            b.retire(s_)
            out.append(c.state()[0][:, 0].copy())
        b.close()
        return ms, out, tiles

    def plain_fp64(ctxs):
        ms, out = 0.0, []
        for p, dt, c in zip(probs, dts, ctxs):
            c.set_state_fn(p.ic)
            c.step(warmup, dt)
            c.sync()
            torch.cuda.synchronize()
            ms += elapsed(lambda: c.step(steps, dt))
            c.sync()
            out.append(c.state()[0][:, 0].copy())
        return ms, out

    c32 = contexts(swe.SWE_FP32_WB)
    ms32, xi32, tiles = batched(swe.SWE_FP32_WB, c32)
    for c in c32:
        c.close()
    c64 = contexts(swe.SWE_FP64)
    ms64, xi64, _ = batched(swe.SWE_FP64, c64)
    print("bench: plain FP64 solver, one instance at a time", file=sys.stderr, flush=True)
    msp, xip = plain_fp64(c64)
    for c in c64:
        c.close()
    d64 = max(float(np.linalg.norm(a - b) / np.linalg.norm(b)) for a, b in zip(xi64, xip))
    err = max(float(np.linalg.norm(a - b) / np.linalg.norm(b)) for a, b in zip(xi32, xi64))
    upd = dofs.sum() * 2 * steps
    k = np.bincount([p.p_max for p in probs], minlength=4)
    word_bytes = {w: sum(p.mesh.ne * stage_bytes_per_element(p.p_max, w) for p in probs) * 2 * steps for w in (4, 8)}
    ach = word_bytes[4] / (ms32 * 1e-3) / 1e9

    def leg(ms, word):
        return {"solves_per_s": count / (ms / steps * BATCH_SOLVE_STEPS * 1e-3), "value": upd / (ms * 1e-3),
                "ms_per_step": ms / steps, "hbm_gbs": word_bytes[word] / (ms * 1e-3) / 1e9}
    kinds = {p: ("shared edge fluxes, 256-element tiles" if t[2] else f"element gather, {t[0]}-element tiles")
             for p, t in tiles.items() if k[p] > 0}
    # HBM bytes of one FP32 step: both stage launches of every order class
    names = [f"k_batch_stage_sh<{p}, float, {m}>" if tiles[p][2] else f"k_batch_stage<{p}, float, {m}, {tiles[p][0]}>"
             for p in sorted(kinds) for m in (1, 2)]
    step_bytes = measured_batch_traffic(names)
    kernel = "; ".join(f"p{p}: k_batch_stage{'_sh' if tiles[p][2] else ''}<{p},float> ({kinds[p]})"
                       for p in sorted(kinds))
    return {"value": upd / (ms32 * 1e-3), "ms_per_step": ms32 / steps,
            "solves_per_s": leg(ms32, 4)["solves_per_s"],
            "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": ach / HBM_PEAK_GBS,
                         "traffic": step_bytes / (ms32 / steps * 1e-3) / 1e9 if step_bytes else None,
                         "traffic_bytes_per_step": step_bytes,
                         "kernel": kernel + " + k_batch_clock, whole step (one launch per order class and stage)"},
            "fp32_batched": leg(ms32, 4), "fp64_batched": leg(ms64, 8), "plain_fp64": leg(msp, 8),
            "speedup_solves_vs_plain_fp64": msp / ms32,
            "fp32_xi_rel_l2_vs_fp64_max": err, "fp64_batched_vs_plain_xi_rel_l2_max": d64,
            "solve_steps": BATCH_SOLVE_STEPS, "timed_steps": steps,
            "tiles": {f"p{p}": {"tile": t[0], "grid": t[1], "kernel": kinds[p]}
                      for p, t in tiles.items() if k[p] > 0},
            "elements": int(sum(p.mesh.ne for p in probs)),
            "orders": {f"p{p}": int(k[p]) for p in range(4) if k[p] > 0}}


def run_served(duration, rate, capacity_requests, tick_steps):
    """Continuous batching over a Poisson request trace (FP32 with FP64
    well-balancing), then the capacity of the batched FP32 server and of the
    plain FP64 solver on the same first requests, all offered at once."""
    import torch
    from paper_2311_11348_amd import inputs as I
    from paper_2311_11348_amd import swe
    from paper_2311_11348_amd.serve import GpuExecutor, PlainExecutor, requests_from_trace, serve
    stream = torch.cuda.Stream()
    trace = I.request_trace(rate=rate, duration=duration)
    reqs = requests_from_trace(trace)
    budget = 64 << 30
    print(f"bench: served trace {len(reqs)} requests over {duration} s", file=sys.stderr, flush=True)
    last = [0.0]

    def progress(t, n):
        if t - last[0] > 10.0:
            last[0] = t
            print(f"bench: t={t:.0f} s, {n} resident", file=sys.stderr, flush=True)
    ex = GpuExecutor(swe.SWE_FP32_WB, budget, max_instances=1024, stream=stream.cuda_stream, keep_state=False)
    st = serve(reqs, ex, tick_steps=tick_steps, on_tick=progress)
    ex.close()
    main = st.summary()
    print(f"bench: served {main}", file=sys.stderr, flush=True)
    cap = []
    for mk in ("batched_fp32", "plain_fp64"):
        sub = requests_from_trace([dataclasses.replace(t, arrival=0.0) for t in trace[:capacity_requests]])
        if mk == "batched_fp32":
            e = GpuExecutor(swe.SWE_FP32_WB, budget, max_instances=1024, stream=stream.cuda_stream,
                            keep_state=False)
            s2 = serve(sub, e, tick_steps=tick_steps, on_tick=progress)
            e.close()
        else:
            e = PlainExecutor(swe.SWE_FP64, budget_bytes=budget, keep_state=False)
            s2 = serve(sub, e, tick_steps=1 << 30, on_tick=progress)
        sm = s2.summary()
        print(f"bench: capacity {mk} {sm}", file=sys.stderr, flush=True)
        cap.append((mk, sm))
    return main, dict(cap)


def tidal_leg(args, I, swe):
    """The headline: the tidal workload, FP32 path with the FP64 path beside it."""
    n = args.n or 512
    prob = I.config_c2(n=n, p=args.p)
    print(f"bench: tidal {prob.mesh.ne} elements p={args.p}", file=sys.stderr, flush=True)
    r32 = run_uniform(prob, swe.SWE_FP32_WB, args.steps, args.warmup)
    r64 = run_uniform(prob, swe.SWE_FP64, args.steps, args.warmup)
    return dict(value=r32["value"], ms_per_step=r32["ms_per_step"], dtype="f32 (f64 bathymetry terms)",
                config={"workload": f"tidal: {n}x{n}x2 jittered triangulation, {prob.mesh.ne} elements, "
                                    f"p={args.p} uniform, sin*cos bathymetry 10-4000 m, west tide",
                        "elements": prob.mesh.ne, "order": args.p, "dof": 3 * K_OF_P[args.p] * prob.mesh.ne},
                roofline=r32["roofline"], compute=r32["compute"],
                fp64={"value": r64["value"], "ms_per_step": r64["ms_per_step"], "dtype": "f64",
                      "roofline": r64["roofline"], "compute": r64["compute"]})


def shallow_leg(n, steps, warmup, I, swe):
    """Uniform p = 2 steps on the shallow depression with and without the
    minimum depth control (FP32 and FP64): time per stage and the control's
    share of it."""
    import torch
    prob = I.config_shallow(n=n, p=2)
    print(f"bench: shallow {prob.mesh.ne} elements", file=sys.stderr, flush=True)
    dof = 3 * K_OF_P[2] * prob.mesh.ne
    out = {}
    for prec, name in ((swe.SWE_FP32_WB, "fp32"), (swe.SWE_FP64, "fp64")):
        row = {}
        for h_min in (prob.h_min, 0.0):
            stream = torch.cuda.Stream()
            ctx = swe.context_for(prob, precision=prec, stream_base=stream.cuda_stream, h_min=h_min)
            ctx.set_state_fn(prob.ic)
            dt = prob.dt()
            ctx.step(warmup, dt)
            ctx.sync()
            torch.cuda.synchronize()
            ms = timed_steps(ctx, stream, steps, dt)
            ctx.close()
            row["control" if h_min > 0 else "no_control"] = {"us_per_stage": ms * 1e3 / (2 * steps),
                                                             "value": dof * 2 * steps / (ms * 1e-3)}
        row["control_share"] = 1.0 - row["no_control"]["us_per_stage"] / row["control"]["us_per_stage"]
        out[name] = row
    return {"value": out["fp32"]["control"]["value"], "ms_per_step": 2 * out["fp32"]["control"]["us_per_stage"] / 1e3,
            "dtype": "f32 (f64 bathymetry terms)", "h_min": prob.h_min, **out,
            "config": f"shallow: {n}x{n}x2 jittered, bottom 1 -> 0.5 m, -0.6 m depression, p=2, "
                      f"minimum depth control h_min = {prob.h_min} m"}


def tsunami_leg(n, steps, warmup, I, swe):
    """The p-adaptive workload in the precision it is specified in (FP32 bulk,
    FP64 bathymetry and mass terms) on the paper's order-separated scheme,
    with the order-partitioned FP64 path beside it."""
    prob = I.config_c3(n=n)
    print(f"bench: tsunami {prob.mesh.ne} elements adaptive", file=sys.stderr, flush=True)
    rs = run_separated(prob, swe.SWE_FP32_WB, steps, warmup, separate=1)
    # FP32 order-partitioned stepping with orders up to 3 is switched off (see
    # the library's configuration checks): the partitioned scheme runs in FP64
    r = run_separated(I.config_c3(n=n), swe.SWE_FP64, steps, warmup, separate=2)
    return {"value": rs["value"], "ms_per_step": rs["ms_per_step"], "dtype": "f32 (f64 bathymetry terms)",
            "timed_steps": steps,
            "scheme": "order-separated (base pass over every element, corrections of the listed elements, "
                      "epilogues; one graph chain per step)",
            "order_fractions": rs["order_fractions"],
            "partitioned_fp64": {"value": r["value"], "ms_per_step": r["ms_per_step"], "dtype": "f64",
                                 "order_fractions": r["order_fractions"],
                                 "scheme": "order-partitioned (base pass over the unlisted elements, then the "
                                           "listed elements of every order; one graph chain per step)"},
            "config": f"tsunami: {n}x{n}x2 jittered, shelf 4000-50 m, 2 m hump, p in {{1,2,3}} by the "
                      "indicator (1e-3 m) before every step, base p=1"}


def served_leg(duration, rate, capacity, tick_steps, swe):
    main_s, cap = run_served(duration, rate, capacity, tick_steps)
    return {"solves_per_s": main_s["solves_per_s"], "p50_latency_s": main_s["p50_latency_s"],
            "p99_latency_s": main_s["p99_latency_s"], "served": main_s, "capacity": cap,
            "speedup_solves_vs_plain_fp64": cap["batched_fp32"]["solves_per_s"]
            / max(cap["plain_fp64"]["solves_per_s"], 1e-30),
            "config": f"served: Poisson {rate:g} req/s for {duration:g} s, 8k-260k elements log-uniform, "
                      "p in {1,2,3}, 200-2000 steps, tidal or hump; FP32 with FP64 bathymetry terms; "
                      f"admission by resident footprint (64 GiB); {tick_steps} steps per tick; capacity "
                      f"legs: the first {capacity} requests offered at once"}


def guarded(name, fn):
    """Run one extra leg of the default line; a failure is recorded, not raised."""
    t0 = time.perf_counter()
    try:
        r = fn()
    except Exception as e:   # noqa: BLE001 - the headline line must still print
        print(f"bench: {name} leg failed: {e!r}", file=sys.stderr, flush=True)
        r = {"error": repr(e)}
    r["wall_s"] = time.perf_counter() - t0
    return r


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", choices=["default", "tidal", "tsunami", "static32", "dambreak", "batched",
                                           "served", "shallow"], default="default",
                    help="default: the tidal headline with the tsunami, batched and (shortened) served "
                         "workloads as extra keys; tidal: the headline alone")
    ap.add_argument("--instances", type=int, default=64)
    ap.add_argument("--duration", type=float, default=120.0)
    ap.add_argument("--rate", type=float, default=20.0)
    ap.add_argument("--capacity-requests", type=int, default=100)
    ap.add_argument("--tick-steps", type=int, default=50)
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--p", type=int, default=2)
    ap.add_argument("--served-duration", type=float, default=30.0,
                    help="length of the request trace of the default line's served leg (s)")
    ap.add_argument("--setup", default=None,
                    help="dambreak workload: run this setup alone (e.g. 'p1-2 1/32', 'p0-1 dynamic')")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="default workload without the extra legs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a 1 GiB elementwise copy first (scales PMC byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (instances and "
              "meshes would shard without a collective in the time loop; see the design notes)",
              file=sys.stderr)
        return 2

    t_wall0 = time.perf_counter()
    cpu = None
    if args.workload in ("default", "tidal") and not args.no_cpu_baseline:
        # the oracle legs fork worker processes: before anything initialises the GPU
        print("bench: timing the oracle on the host", file=sys.stderr, flush=True)
        cpu = cpu_baseline(args.p)

    import numpy as np
    import torch
    from paper_2311_11348_amd import inputs as I
    from paper_2311_11348_amd import swe

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    out = {"metric": "DOF-updates/s per RK stage", "unit": "DOF-updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "data": "synthetic"}
    if args.copy_calibration:
        copy_calibration()
    if args.workload in ("default", "tidal"):
        out.update(tidal_leg(args, I, swe))
        if cpu is not None:
            out["cpu_baseline"] = cpu
        if args.workload == "default" and not args.no_extras:
            # the other workloads of the method's measurement plan, at the
            # driver's step counts where they are timed per step
            out["tsunami"] = guarded("tsunami", lambda: tsunami_leg(256, max(args.steps, 200), max(args.warmup, 5),
                                                                    I, swe))
            out["batched"] = guarded("batched", lambda: run_batched(args.instances, max(args.steps, 20), 2))
            out["served"] = guarded("served", lambda: served_leg(args.served_duration, args.rate,
                                                                 args.capacity_requests, args.tick_steps, swe))
    elif args.workload == "shallow":
        n = args.n or 512
        r = shallow_leg(n, args.steps, args.warmup, I, swe)
        out.update(value=r.pop("value"), ms_per_step=r.pop("ms_per_step"), dtype=r.pop("dtype"),
                   config={"workload": r.pop("config"), "elements": 2 * n * n}, **r)
    elif args.workload == "tsunami":
        n = args.n or 256
        r = tsunami_leg(n, args.steps, args.warmup, I, swe)
        out.update(value=r.pop("value"), ms_per_step=r.pop("ms_per_step"), dtype=r.pop("dtype"),
                   config={"workload": r.pop("config"), "elements": 2 * n * n}, **r)
    elif args.workload == "dambreak":
        steps = args.steps if args.steps != 500 else 100
        n = args.n or 1024
        rows = run_dambreak(steps, args.warmup, n=n, only=args.setup)
        key = args.setup or "p1-2 1/32"
        head = rows[key].get("fp64_partitioned") or rows[key].get("fp64")
        best_ms = min(rows[key]["paper_ms_per_stage"].values()) if "paper_ms_per_stage" in rows[key] else None
        out.update(steps=steps, value=head["value"], ms_per_step=2 * head["ms_per_stage"], dtype="f64",
                   vs_baseline=best_ms / head["ms_per_stage"] if n == 1024 and key == "p1-2 1/32" else None,
                   baseline={"what": f"the paper's fastest time per stage for {key} on 2,097,152 triangles, "
                                     "on its own hardware", "ms": best_ms},
                   config={"workload": f"dambreak: {n}x{n}x2 jittered triangulation of [0,5]^2, "
                                       f"{2 * n * n} elements, g=1, h_b=0.5 m, linear friction, dt=1e-5 s; "
                                       "headline: every 32nd element p=2, base p=1, order-partitioned, FP64",
                           "elements": 2 * n * n}, setups=rows)
    elif args.workload == "batched":
        steps = args.steps if args.steps != 500 else 300
        r = run_batched(args.instances, steps, args.warmup)
        out.update(steps=steps, value=r.pop("value"), ms_per_step=r.pop("ms_per_step"),
                   dtype="f32 (f64 bathymetry terms)", roofline=r.pop("roofline"),
                   config={"workload": f"batched: {args.instances} independent instances, log-uniform "
                                       "16k-500k elements, p in {1,2,3}, tidal or hump, random smooth "
                                       f"bathymetry 50-4000 m, {steps} steps each, one tile per block",
                           **{k: r.pop(k) for k in ("elements", "orders", "tiles")}}, **r)
    elif args.workload == "served":
        main_s, cap = run_served(args.duration, args.rate, args.capacity_requests, args.tick_steps)
        out.update(metric="served solves/s", unit="solves/s", value=main_s["solves_per_s"],
                   ms_per_step=None, steps=None, warmup=None, dtype="f32 (f64 bathymetry terms)",
                   p50_latency_s=main_s["p50_latency_s"], p99_latency_s=main_s["p99_latency_s"],
                   served=main_s, capacity=cap,
                   speedup_solves_vs_plain_fp64=cap["batched_fp32"]["solves_per_s"]
                   / max(cap["plain_fp64"]["solves_per_s"], 1e-30),
                   config={"workload": f"served: Poisson {args.rate:g} req/s for {args.duration:g} s, "
                                       "8k-260k elements log-uniform, p in {1,2,3}, 200-2000 steps, "
                                       "tidal or hump; admission by resident footprint (64 GiB); "
                                       f"{args.tick_steps} steps per tick; capacity legs: first "
                                       f"{args.capacity_requests} requests offered at once"})
    else:
        n = args.n or 512
        prob = I.config_c2(n=n, p=2)
        prob.p_base = 1
        prob.p = np.full(prob.mesh.ne, 1, np.int8)
        prob.p[::32] = 2
        print(f"bench: static32 {prob.mesh.ne} elements", file=sys.stderr, flush=True)
        r = run_separated(prob, swe.SWE_FP32_WB, args.steps, args.warmup, separate=2)
        rs = run_separated(prob, swe.SWE_FP32_WB, args.steps, args.warmup, separate=1)
        out.update(value=r["value"], ms_per_step=r["ms_per_step"], dtype="f32 (f64 bathymetry terms)",
                   config={"workload": f"static32: tidal {n}x{n}x2 mesh, base p=1, every 32nd element p=2, "
                                       "order-partitioned",
                           "elements": prob.mesh.ne, "order_fractions": r["order_fractions"]},
                   separated={"value": rs["value"], "ms_per_step": rs["ms_per_step"],
                              "scheme": "base + corrections on a second stream, joined by epilogues"})
    out["wall_s"] = time.perf_counter() - t_wall0
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
