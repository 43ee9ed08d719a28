"""Continuous-batching scheduler on the host, against a timing-model executor:
every request finishes exactly once, admission is FIFO and never exceeds the
footprint budget, latency accounting is consistent, and a failing request
(bad input, a run that fails, a footprint that can never fit) fails alone."""
import numpy as np

from paper_2311_11348_amd import inputs as I
from paper_2311_11348_amd.serve import FakeExecutor, Request, requests_from_trace, serve


def small_trace(count, seed=1, steps=(5, 40)):
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    for i in range(count):
        t += rng.exponential(0.002)
        out.append(I.Request(arrival=t, seed=i, n_elements_target=float(rng.uniform(200, 5000)),
                             p=int(rng.integers(1, 4)), steps=int(rng.integers(*steps)),
                             tidal=bool(rng.integers(0, 2))))
    return requests_from_trace(out)


def test_all_complete_fifo_within_budget():
    reqs = small_trace(40)
    budget = 100 * 12000
    ex = FakeExecutor(budget, bytes_per_element=100, step_time=1e-5)
    st = serve(reqs, ex, tick_steps=7, prep_threads=4)
    assert [r.rid for r in st.results] == list(range(40))
    assert all(r.ok for r in st.results)
    assert ex.admitted == sorted(ex.admitted)          # FIFO by arrival
    assert ex.max_used <= budget and st.max_used == ex.max_used
    assert ex.used == 0 and not ex.left
    for r in st.results:
        assert r.arrival <= r.admitted <= r.done
    s = st.summary()
    assert s["completed"] == 40 and s["failed"] == 0
    assert s["p50_latency_s"] <= s["p99_latency_s"]
    assert s["solves_per_s"] > 0


def test_failures_are_isolated():
    reqs = small_trace(20, seed=2)
    reqs[3].poisoned = True                               # fails during its run
    reqs[7].spec.steps = 0                                # fails in preparation
    reqs[11].spec.n_elements_target = 1e7                 # can never fit
    budget = 100 * 20000
    ex = FakeExecutor(budget, bytes_per_element=100)
    st = serve(reqs, ex, tick_steps=5, prep_threads=2)
    bad = {3, 7, 11}
    for r in st.results:
        assert r.ok == (r.rid not in bad), (r.rid, r.error)
    assert "budget" in st.results[11].error
    assert 11 in ex.discarded
    assert ex.used == 0


def test_tick_granularity():
    """A request of S steps needs ceil(S / tick) ticks while resident."""
    spec = I.Request(arrival=0.0, seed=0, n_elements_target=800.0, p=1, steps=23, tidal=False)
    ex = FakeExecutor(10**9)
    st = serve([Request(0, spec)], ex, tick_steps=5)
    assert st.ticks == 5 and st.results[0].ok


def test_staging_budget_bounds_prepared_requests():
    """Prepared requests hold device memory until admitted: their summed
    footprints stay within the staging budget (one request is always let
    through), and every request still completes."""
    reqs = small_trace(60, seed=3, steps=(20, 60))
    for r in reqs:
        r.spec.arrival = 0.0                         # all at once: preparation would run far ahead
    budget = 100 * 15000
    stage = 100 * 6000
    ex = FakeExecutor(budget, bytes_per_element=100, step_time=2e-5)
    st = serve(reqs, ex, tick_steps=5, prep_threads=8, stage_budget=stage)
    assert all(r.ok for r in st.results)
    biggest = max(ex.footprint(r) for r in reqs)
    assert ex.max_prepared <= max(stage, biggest)
    assert st.max_staged <= max(stage, biggest)
    assert ex.prepared == 0 and ex.used == 0
    # without the bound, preparation runs ahead of admission
    ex2 = FakeExecutor(budget, bytes_per_element=100, step_time=2e-5)
    serve(reqs, ex2, tick_steps=5, prep_threads=8, stage_budget=1 << 60)
    assert ex2.max_prepared > stage
