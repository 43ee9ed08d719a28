"""Serving on the GPU: requests arriving while others run are admitted as
memory frees up and advanced together; each request's result in the mix
matches the oracle run of the same request (FP64 within 1e-12 relative L2,
FP32 elevation within 1e-5) and is bitwise its result computed alone (the
same kernels round identically inside and outside the batch); a failing
request fails alone; the device memory the service holds stays within the
batch budget plus the staging budget of prepared requests."""
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2311_11348_amd import inputs as I
from paper_2311_11348_amd import swe
from paper_2311_11348_amd.serve import GpuExecutor, requests_from_trace, serve

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def trace(count, seed, n_lo=300, n_hi=2500, steps=(20, 60), gap=0.01):
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    for i in range(count):
        t += rng.exponential(gap)
        out.append(I.Request(arrival=t, seed=seed * 100 + i,
                             n_elements_target=float(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi)))),
                             p=int(rng.integers(1, 4)), steps=int(rng.integers(*steps)),
                             tidal=bool(rng.integers(0, 2))))
    return requests_from_trace(out)


def oracle_state(prob):
    """A request's initial state projected by the oracle."""
    return Oracle.from_problem(prob).project(prob.ic)


class OracleRuns:
    """The served trace's requests run by the oracle from the oracle's
    projection of their initial states (once, one thread per request)."""

    def __init__(self):
        self.reqs = trace(10, seed=11)
        self.poisoned = 4

        def one(r):
            prob = I.request_problem(r.spec)
            orc = Oracle.from_problem(prob)
            return orc.step(orc.project(prob.ic), r.spec.steps, prob.dt())
        todo = [r for i, r in enumerate(self.reqs) if i != self.poisoned]
        with ThreadPoolExecutor(max_workers=len(todo)) as pool:
            refs = list(pool.map(one, todo))
        self.ref = {r.rid: c for r, c in zip(todo, refs)}


@pytest.fixture(scope="module")
def oracle_runs():
    say("oracle runs of the served requests")
    return OracleRuns()


def alone(spec, precision):
    prob = I.request_problem(spec)
    with swe.context_for(prob, precision=precision) as ctx:
        ctx.set_state(oracle_state(prob))
        ctx.step(spec.steps, prob.dt())
        ctx.sync()
        c, _ = ctx.state()
    return c


@pytest.mark.parametrize("precision", [swe.SWE_FP64, swe.SWE_FP32_WB])
def test_served_equals_alone(precision, oracle_runs):
    reqs = trace(10, seed=11)
    reqs[oracle_runs.poisoned].poisoned = True
    fps = sorted(swe.swe_footprint_bytes(r.elements, r.spec.p, precision) for r in reqs)
    budget = sum(fps[-3:])                      # at most a few resident at once: forces queueing
    ex = GpuExecutor(precision, budget, max_instances=16, init_state=oracle_state)
    try:
        st = serve(reqs, ex, tick_steps=16, prep_threads=4)
    finally:
        ex.close()
    s = st.summary()
    say(f"precision {precision}: {s}")
    assert st.max_used <= budget
    assert len(st.results) == len(reqs)
    for r, q in zip(st.results, reqs):
        if q.poisoned:
            assert not r.ok and "depth" in r.error
            continue
        assert r.ok, (r.rid, r.error)
        ref = alone(q.spec, precision)
        eq = np.array_equal(r.state, ref)
        orc = oracle_runs.ref[r.rid]
        err = np.linalg.norm(r.state - orc) / np.linalg.norm(orc)
        exi = np.linalg.norm((r.state - orc)[:, 0]) / np.linalg.norm(orc[:, 0])
        say(f"  request {r.rid}: ne={q.elements} p={q.spec.p} steps={q.spec.steps} "
            f"latency {r.latency * 1e3:.1f} ms equal={eq} vs oracle rel L2 {err:.2e}, xi {exi:.2e}")
        assert eq, r.rid
        if precision == swe.SWE_FP64:
            assert err < 1e-12, r.rid
        else:
            assert exi < 1e-5, r.rid


def test_served_device_memory_within_budget():
    """Twelve requests of 40k-100k elements arriving at once, FP32: the
    device memory in use (hipMemGetInfo, sampled at every tick and after the
    run) stays below the batch budget (three of the largest footprints) plus
    the staging budget of prepared requests, the one request being retired
    and a margin for the runtime's own allocations; every request
    completes, and the batch holds nothing once the trace is done."""
    import torch
    torch.cuda.init()
    torch.cuda.synchronize()
    prec = swe.SWE_FP32_WB
    reqs = trace(12, seed=23, n_lo=40e3, n_hi=100e3, steps=(30, 60), gap=1e-6)
    fps = [swe.swe_footprint_bytes(r.elements, r.spec.p, prec) for r in reqs]
    budget = sum(sorted(fps)[-3:])
    stage = budget // 3
    margin = 128 << 20
    free0, _ = torch.cuda.mem_get_info()
    peak = [0]

    def sample(*_):
        free, _ = torch.cuda.mem_get_info()
        peak[0] = max(peak[0], free0 - free)
    ex = GpuExecutor(prec, budget, max_instances=16, keep_state=False)
    try:
        st = serve(reqs, ex, tick_steps=10, prep_threads=4, on_tick=sample, stage_budget=stage)
        sample()
        held = ex.batch.free_bytes()
    finally:
        ex.close()
    bound = budget + stage + max(fps) + margin
    say(f"served memory: peak {peak[0] / 2**20:.0f} MiB, bound {bound / 2**20:.0f} MiB (budget "
        f"{budget / 2**20:.0f}, staging {stage / 2**20:.0f}, largest request {max(fps) / 2**20:.0f} MiB), "
        f"max staged {st.max_staged / 2**20:.0f} MiB, summary {st.summary()}")
    assert all(r.ok for r in st.results)
    assert held == budget
    assert peak[0] <= bound
