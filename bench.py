"""Throughput of the DG shallow-water hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
                    [--workload tidal|tsunami|static32|dambreak|batched|served]

tidal (default): 512x512x2 triangulation of a 100 km square, nodes jittered
  by U(-0.2h, 0.2h) (seed 2), uniform order p = 2, bathymetry
  10 m + 3990 m (1 + sin(2 pi x/L) cos(2 pi y/L))/2, lake at rest, west edge
  open and forced by a 0.5 m tide of period 44712 s, Coriolis 3.19e-5 1/s,
  quadratic friction 0.009.  The headline value is the FP32 path (FP32 state
  and bulk arithmetic, FP64 bathymetry terms); the FP64 path is measured on
  the same workload and reported beside it.
tsunami: 256x256x2 jittered (seed 3), linear shelf 4000 m -> 50 m, 2 m hump,
  orders in {1,2,3} re-chosen every step by the indicator (threshold 1e-3 m),
  base order 1; order-partitioned FP64 path, with the order-separated FP32
  path (corrections on a second stream) beside it.
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
served: Poisson arrivals (20 req/s for 120 s, seed 5), 8k-260k elements,
  p in {1,2,3}, 200-2000 steps; continuous batching with admission by
  footprint; reports solves/s with p50/p99 latency, then the capacity of
  the batched FP32 server and of the plain FP64 solver on the first 100
  requests offered at once.

A step is one SSP-RK2 step (two stages) of the whole hot path: volume +
source + edge fluxes + stage update + u H = q (+ order update when adaptive).
Metric: DOF-updates per second per RK stage, DOF = 3 * sum_e K(p_e).  Inputs
are resident in HBM before the timed region.  Prints one JSON line.
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


def stage_bytes_per_element(p: int, word: int, nv: int, ne: int) -> float:
    """Algorithmic HBM bytes one element moves in one fused stage kernel
    (average of the two SSP-RK2 stages): read c (3K) and u (2K), read c^n (3K)
    in the second stage only, write c (3K) and u (2K); geometry: 3 vertex ids,
    3 neighbour ids, 1 packed neighbour-edge byte and the element's share of
    the 32-byte vertex records.  Neighbour coefficients are counted once, as
    their owner's read (they are served from cache)."""
    K = K_OF_P[p]
    state = (3 * K + 2 * K + 0.5 * 3 * K + 3 * K + 2 * K) * word
    geo = 3 * 4 + 3 * 4 + 1 + 32.0 * nv / ne
    return state + geo


KERNEL_SOURCES = ("paper_2311_11348_amd/csrc/swe_kernels.hip", "paper_2311_11348_amd/csrc/swe_internal.h",
                  "paper_2311_11348_amd/csrc/swe_tables.h", "paper_2311_11348_amd/build.py")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_stage_p2_tidal512_traffic.txt")


def kernel_source_hash() -> str:
    """SHA-256 over the sources and build flags that determine the kernels' code."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernels):
    """HBM bytes per launch of the given kernels from the committed PMC summary
    (FETCH_SIZE and WRITE_SIZE runs, each scaled by what the same counter reads
    for a copy kernel of known size), averaged over the kernels; None when the
    summary is missing or the kernel sources changed since it was taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            if "=" in line and not line.lstrip().startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_hash") != kernel_source_hash():
        return None
    fs = float(kv["copy_bytes"]) / (float(kv["copy_fetch_kib"]) * 1024.0)
    ws = float(kv["copy_bytes"]) / (float(kv["copy_write_kib"]) * 1024.0)
    vals = []
    for k in kernels:
        f, w = kv.get(f"fetch_kib[{k}]"), kv.get(f"write_kib[{k}]")
        if f is None or w is None:
            return None
        vals.append(float(f) * 1024.0 * fs + float(w) * 1024.0 * ws)
    return sum(vals) / len(vals)


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


def cpu_baseline(p: int, budget_s: float = 15.0):
    """The FP64 oracle (single thread) on a bounded sample of the same workload:
    the same problem family on a 64x64x2 mesh, timed over whole SSP-RK2 steps."""
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
    return {"value": dof * 2 * steps / el, "unit": "DOF-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{n}x{n}x2 mesh of the tidal workload family ({prob.mesh.ne} elements, p={p}), "
                      f"{steps} SSP-RK2 steps, FP64, single thread, {el:.1f} s"}


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
    launch_s = ms * 1e-3 / (2 * steps)
    bpe = stage_bytes_per_element(p, word, nv, ne)
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
                         "bytes_per_launch": bpe * ne, "avg_launch_us": launch_s * 1e6}}


def run_separated(prob, precision, steps, warmup, separate=1, chunk=50):
    """Order-separated scheme (separate=1: base + corrections joined by an
    epilogue) or order-partitioned scheme (separate=2: base elements and each
    order's listed elements on parallel branches), optionally adaptive.
    DOF counts follow the order map, read between timed chunks."""
    import numpy as np
    import torch
    from paper_2311_11348_amd import swe
    stream = torch.cuda.Stream()
    stream2 = torch.cuda.Stream()
    ctx = swe.context_for(prob, precision=precision, separate=separate, stream_base=stream.cuda_stream,
                          stream_corr=stream2.cuda_stream)
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
DAMBREAK_DYN_STEPS = 400


def run_dambreak(steps, warmup, n=1024):
    """The radial dam break: uniform orders on the fused stage kernel, the
    statically adaptive 1/32 setups on the order-partitioned and
    order-separated schemes; FP64 and FP32."""
    import numpy as np
    from paper_2311_11348_amd import inputs as I
    from paper_2311_11348_amd import swe
    out = {}
    setups = [("p0", 0, 0, 0), ("p1", 1, 1, 0), ("p2", 2, 2, 0), ("p0-1 1/32", 0, 1, 32), ("p1-2 1/32", 1, 2, 32)]
    for name, lo, hi, every in setups:
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
        row["paper_ms_per_stage"] = DAMBREAK_PAPER_MS[name]
        out[name] = row
    # dynamic orders: this library's indicator (threshold DAMBREAK_TAU), the
    # CFL step, DAMBREAK_DYN_STEPS timed steps from the start of the run
    for name, lo, hi in (("p0-1 dynamic", 0, 1), ("p1-2 dynamic", 1, 2)):
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


def run_batched(count, steps, warmup):
    """Many independent instances: FP32 and FP64 batched (tile-per-block
    kernels, step graph, autotuned tiles) and the plain FP64 solver (one
    instance at a time, one ordinary launch per stage).  Every instance runs
    warmup + steps steps; the timed region holds the last ``steps`` of all of
    them.  Inputs are resident before timing."""
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

    def batched(prec):
        t0 = time.perf_counter()
        ctxs = []
        for p in probs:
            c = swe.context_for(p, precision=prec)
            c.set_state_fn(p.ic)
            ctxs.append(c)
        budget = sum(swe.swe_footprint_bytes(c.ne, p.p_max, prec) for c, p in zip(ctxs, probs)) + (1 << 30)
        b = swe.Batch(precision=prec, budget_bytes=budget, max_instances=count, stream=stream.cuda_stream)
        slots = [b.admit(c, steps + warmup, dt) for c, dt in zip(ctxs, dts)]
        b.tune(reps=3)
        tiles = {p: b.tile_config(p) for p in range(4)}
        b.tick(warmup)
        b.sync()
        print(f"bench: batched precision {prec} ready after {time.perf_counter() - t0:.1f} s",
              file=sys.stderr, flush=True)

        def run():
            b.tick(steps)
        ms = elapsed(run)
        done = b.poll()
        assert len(done) == count and not any(f for _, f in done), done
        out = []
        for s, c in zip(slots, ctxs):
            b.retire(s)
            out.append(c.state()[0][:, 0].copy())
            c.close()
        b.close()
        return ms, out, tiles

    def plain_fp64():
        ms, out = 0.0, []
        for p, dt in zip(probs, dts):
            c = swe.context_for(p, precision=swe.SWE_FP64, stream_base=stream.cuda_stream)
            c.set_state_fn(p.ic)
            c.step(warmup, dt)
            c.sync()
            torch.cuda.synchronize()

            def run():
                c.step(steps, dt)
            ms += elapsed(run)
            c.sync()
            out.append(c.state()[0][:, 0].copy())
            c.close()
        return ms, out

    ms32, xi32, tiles = batched(swe.SWE_FP32_WB)
    ms64, xi64, _ = batched(swe.SWE_FP64)
    msp, xip = plain_fp64()
    d64 = max(float(np.linalg.norm(a - b) / np.linalg.norm(b)) for a, b in zip(xi64, xip))
    err = max(float(np.linalg.norm(a - b) / np.linalg.norm(b)) for a, b in zip(xi32, xi64))
    upd = dofs.sum() * 2 * steps
    word_bytes = {4: 0.0, 8: 0.0}
    for w in word_bytes:
        word_bytes[w] = sum(p.mesh.ne * stage_bytes_per_element(p.p_max, w, p.mesh.nv, p.mesh.ne)
                            for p in probs) * 2 * steps
    ach = word_bytes[4] / (ms32 * 1e-3) / 1e9

    def leg(ms, word):
        return {"solves_per_s": count / (ms * 1e-3), "value": upd / (ms * 1e-3), "ms_total": ms,
                "hbm_gbs": word_bytes[word] / (ms * 1e-3) / 1e9}
    k = np.bincount([p.p_max for p in probs], minlength=4)
    return {"value": upd / (ms32 * 1e-3), "ms_per_step": ms32 / steps,
            "solves_per_s": count / (ms32 * 1e-3),
            "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": ach / HBM_PEAK_GBS, "traffic": None,
                         "kernel": "k_batch_stage<P,float> over all orders + k_batch_clock (whole step)"},
            "fp64_batched": leg(ms64, 8), "plain_fp64": leg(msp, 8),
            "speedup_solves_vs_plain_fp64": msp / ms32,
            "fp32_xi_rel_l2_vs_fp64_max": err, "fp64_batched_vs_plain_xi_rel_l2_max": d64,
            "tiles": {f"p{p}": {"tile": t[0], "grid": t[1], "kernel": "shared edge fluxes" if t[2] else "element gather"}
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
            e = PlainExecutor(swe.SWE_FP64, stream=stream.cuda_stream, keep_state=False)
            s2 = serve(sub, e, tick_steps=1 << 30, on_tick=progress)
        sm = s2.summary()
        print(f"bench: capacity {mk} {sm}", file=sys.stderr, flush=True)
        cap.append((mk, sm))
    return main, dict(cap)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", choices=["tidal", "tsunami", "static32", "dambreak", "batched", "served"],
                    default="tidal")
    ap.add_argument("--instances", type=int, default=64)
    ap.add_argument("--duration", type=float, default=120.0)
    ap.add_argument("--rate", type=float, default=20.0)
    ap.add_argument("--capacity-requests", type=int, default=100)
    ap.add_argument("--tick-steps", type=int, default=50)
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--p", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a 1 GiB elementwise copy first (scales PMC byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (instances and "
              "meshes would shard without a collective in the time loop; see the design notes)",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch
    from paper_2311_11348_amd import inputs as I
    from paper_2311_11348_amd import swe

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    t_wall0 = time.perf_counter()
    out = {"metric": "DOF-updates/s per RK stage", "unit": "DOF-updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "data": "synthetic"}
    if args.copy_calibration:
        copy_calibration()
    if args.workload == "tidal":
        n = args.n or 512
        prob = I.config_c2(n=n, p=args.p)
        print(f"bench: tidal {prob.mesh.ne} elements p={args.p}", file=sys.stderr, flush=True)
        r32 = run_uniform(prob, swe.SWE_FP32_WB, args.steps, args.warmup)
        r64 = run_uniform(prob, swe.SWE_FP64, args.steps, args.warmup)
        out.update(value=r32["value"], ms_per_step=r32["ms_per_step"], dtype="f32 (f64 bathymetry terms)",
                   config={"workload": f"tidal: {n}x{n}x2 jittered triangulation, {prob.mesh.ne} elements, "
                                       f"p={args.p} uniform, sin*cos bathymetry 10-4000 m, west tide",
                           "elements": prob.mesh.ne, "order": args.p, "dof": 3 * K_OF_P[args.p] * prob.mesh.ne},
                   roofline=r32["roofline"],
                   fp64={"value": r64["value"], "ms_per_step": r64["ms_per_step"], "dtype": "f64",
                         "roofline": r64["roofline"]})
        if not args.no_cpu_baseline:
            print("bench: timing the oracle on the host", file=sys.stderr, flush=True)
            out["cpu_baseline"] = cpu_baseline(args.p)
    elif args.workload == "tsunami":
        n = args.n or 256
        prob = I.config_c3(n=n)
        print(f"bench: tsunami {prob.mesh.ne} elements adaptive", file=sys.stderr, flush=True)
        # FP32 order-partitioned stepping with orders up to 3 is switched off
        # (see the library's configuration checks): the partitioned scheme
        # runs in FP64 (the faster of the two here), the order-separated
        # scheme in FP32 beside it
        r = run_separated(prob, swe.SWE_FP64, args.steps, args.warmup, separate=2)
        rs = run_separated(I.config_c3(n=n), swe.SWE_FP32_WB, args.steps, args.warmup, separate=1)
        out.update(value=r["value"], ms_per_step=r["ms_per_step"], dtype="f64",
                   config={"workload": f"tsunami: {n}x{n}x2 jittered, shelf 4000-50 m, 2 m hump, "
                                       "p in {1,2,3} by indicator (1e-3 m), base p=1; order-partitioned "
                                       "(base elements and each order's listed elements on parallel branches)",
                           "elements": prob.mesh.ne, "order_fractions": r["order_fractions"]},
                   separated_fp32={"value": rs["value"], "ms_per_step": rs["ms_per_step"],
                                   "dtype": "f32 (f64 bathymetry terms)",
                                   "scheme": "base + corrections on a second stream, joined by epilogues"})
    elif args.workload == "dambreak":
        steps = args.steps if args.steps != 500 else 100
        n = args.n or 1024
        rows = run_dambreak(steps, args.warmup, n=n)
        head = rows["p1-2 1/32"]["fp64_partitioned"]
        best_ms = min(rows["p1-2 1/32"]["paper_ms_per_stage"].values())
        out.update(steps=steps, value=head["value"], ms_per_step=2 * head["ms_per_stage"], dtype="f64",
                   vs_baseline=best_ms / head["ms_per_stage"] if n == 1024 else None,
                   baseline={"what": "the paper's fastest time per stage for static 1/32 p1-2 on 2,097,152 "
                                     "triangles (AMD-RTX, CPU, separated), on its own hardware", "ms": best_ms},
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
