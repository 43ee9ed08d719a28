"""Serving on the GPU: requests arriving while others run are admitted as
memory frees up and advanced together; each request's result in the mix is
bitwise its result computed alone (the same kernels round identically inside
and outside the batch), a failing request fails alone, and the resident
footprint never exceeds the budget."""
import sys

import numpy as np
import pytest

from paper_2311_11348_amd import inputs as I
from paper_2311_11348_amd import swe
from paper_2311_11348_amd.serve import GpuExecutor, requests_from_trace, serve

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def trace(count, seed):
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    for i in range(count):
        t += rng.exponential(0.01)
        out.append(I.Request(arrival=t, seed=seed * 100 + i, n_elements_target=float(np.exp(rng.uniform(np.log(300), np.log(4000)))),
                             p=int(rng.integers(1, 4)), steps=int(rng.integers(20, 90)), tidal=bool(rng.integers(0, 2))))
    return requests_from_trace(out)


def alone(spec, precision):
    prob = I.request_problem(spec)
    with swe.context_for(prob, precision=precision) as ctx:
        ctx.set_state_fn(prob.ic)
        ctx.step(spec.steps, prob.dt())
        ctx.sync()
        c, _ = ctx.state()
    return c


@pytest.mark.parametrize("precision", [swe.SWE_FP64, swe.SWE_FP32_WB])
def test_served_equals_alone(precision):
    reqs = trace(10, seed=11 + precision)
    reqs[4].poisoned = True
    fps = sorted(swe.swe_footprint_bytes(r.elements, r.spec.p, precision) for r in reqs)
    budget = sum(fps[-3:])                      # at most a few resident at once: forces queueing
    ex = GpuExecutor(precision, budget, max_instances=16)
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
        say(f"  request {r.rid}: ne={q.elements} p={q.spec.p} steps={q.spec.steps} "
            f"latency {r.latency * 1e3:.1f} ms equal={eq}")
        assert eq, r.rid
