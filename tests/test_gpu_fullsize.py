"""Parity at the benchmarked sizes, in the benchmarked launch configuration.

The tidal workload's full mesh (512x512x2 = 524,288 elements, p = 2): the
right-hand side of a random state and two SSP-RK2 steps through swe_step (the
fused stage kernels the benchmark times) against the oracle on every element.
The tsunami workload's full mesh (131,072 elements): order-separated adaptive
steps against the oracle's adaptive steps (identical order maps).  The batched
workload's first instances at full size: batched bitwise equal to alone.
"""
import sys

import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2311_11348_amd import inputs as I
from paper_2311_11348_amd import swe

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_max_err(a, b):
    assert np.all(np.isfinite(a)), "non-finite values in the GPU result"
    return max(np.max(np.abs(a[:, j] - b[:, j])) / np.max(np.abs(b[:, j])) for j in range(3))


class Tidal:
    """The tidal mesh, a random state and the oracle's results on it (computed once)."""

    def __init__(self):
        self.prob = I.config_c2(n=512, p=2)
        self.orc = Oracle.from_problem(self.prob)
        self.c = I.random_state(self.prob.mesh, self.prob.p, 2, seed=512, hb_vertex=self.prob.hb_vertex,
                                xi_amp=1.0, q_amp=20.0)
        self._rhs = self._step = None

    def rhs(self):
        if self._rhs is None:
            self._rhs = self.orc.rhs(777.0, self.c)
        return self._rhs

    def step(self):
        if self._step is None:
            self._step = self.orc.step(self.c, 2, self.prob.dt(), t0=100.0)
        return self._step


@pytest.fixture(scope="module")
def tidal():
    return Tidal()


@pytest.mark.parametrize("precision,tol", [(swe.SWE_FP64, 1e-12), (swe.SWE_FP32_WB, 1e-4)])
def test_tidal_rhs_full_size(tidal, precision, tol):
    prob, c = tidal.prob, tidal.c
    ref = tidal.rhs()
    with swe.context_for(prob, precision=precision) as ctx:
        got = ctx.rhs(777.0, c)
    err = rel_max_err(got, ref)
    say(f"tidal full size rhs precision={precision}: ne={prob.mesh.ne} max rel err {err:.2e}")
    assert err < tol


@pytest.mark.parametrize("precision,tol", [(swe.SWE_FP64, 1e-12), (swe.SWE_FP32_WB, 1e-5)])
def test_tidal_step_full_size(tidal, precision, tol):
    """Two SSP-RK2 steps through the stage kernels the benchmark times."""
    prob, c = tidal.prob, tidal.c
    dt = prob.dt()
    ref = tidal.step()
    with swe.context_for(prob, precision=precision) as ctx:
        ctx.set_state(c, t0=100.0)
        ctx.step(2, dt)
        ctx.sync()
        got, t = ctx.state()
    assert abs(t - (100.0 + 2 * dt)) < 1e-9 * t
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    exi = np.linalg.norm((got - ref)[:, 0]) / np.linalg.norm(ref[:, 0])
    say(f"tidal full size 2 steps precision={precision}: rel L2 {err:.2e}, xi {exi:.2e}")
    assert err < tol and exi < tol


class Tsunami:
    """The tsunami mesh at full size and the oracle's three adaptive steps
    from its initial state (computed once)."""
    steps = 3

    def __init__(self):
        self.prob = I.config_c3(n=256)
        self.orc = Oracle.from_problem(self.prob)
        self.c0 = self.orc.project(self.prob.ic)
        self.dt = self.prob.dt()
        self._ref = None

    def ref(self):
        if self._ref is None:
            prob, orc, dt = self.prob, self.orc, self.dt
            ref = self.c0
            for s in range(self.steps):
                # the order decision of each step must not be within rounding of a threshold
                ind = orc.indicator(s * dt, ref)
                for thr in (prob.adapt_tau, prob.adapt_tau / 10):
                    assert np.min(np.abs(ind - thr)) / thr > 1e-9
                ref = orc.step(ref, 1, dt, t0=s * dt, adapt=True, tau=prob.adapt_tau, p_lo=1, p_hi=3)
            self._ref = (ref, orc.order())
        return self._ref


@pytest.fixture(scope="module")
def tsunami():
    return Tsunami()


def test_tsunami_adaptive_full_size(tsunami):
    ref, pref = tsunami.ref()
    with swe.context_for(tsunami.prob, separate=1) as ctx:
        ctx.set_state(tsunami.c0)
        ctx.step(tsunami.steps, tsunami.dt)
        ctx.sync()
        got, _ = ctx.state()
        pgot = ctx.order()
    counts = np.bincount(pref, minlength=4)
    say(f"tsunami full size: orders p1/p2/p3 = {counts[1]}/{counts[2]}/{counts[3]}, "
        f"maps equal {np.array_equal(pgot, pref)}")
    assert counts[2] + counts[3] > 0
    assert np.array_equal(pgot, pref)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    say(f"  rel L2 {err:.2e}")
    assert err < 1e-12


def test_tsunami_adaptive_full_size_fp32(tsunami):
    """The FP32 order-separated adaptive path the benchmark times, at full
    size: order maps agreeing on at least 99 % of the elements and the
    elevation within 1e-5 relative L2 of the oracle after three steps."""
    ref, pref = tsunami.ref()
    with swe.context_for(tsunami.prob, precision=swe.SWE_FP32_WB, separate=1) as ctx:
        ctx.set_state(tsunami.c0)
        ctx.step(tsunami.steps, tsunami.dt)
        ctx.sync()
        got, _ = ctx.state()
        pgot = ctx.order()
    assert np.all(np.isfinite(got))
    agree = float(np.mean(pgot == pref))
    exi = np.linalg.norm((got - ref)[:, 0]) / np.linalg.norm(ref[:, 0])
    say(f"tsunami full size FP32 separated: map agreement {agree:.5f}, xi rel L2 {exi:.2e}")
    assert agree >= 0.99
    assert exi < 1e-5


@pytest.mark.parametrize("precision", [swe.SWE_FP32_WB, swe.SWE_FP64])
def test_batched_full_size_equals_alone(precision):
    probs = I.config_c4(6)
    steps = 4
    alone = []
    for p in probs:
        with swe.context_for(p, precision=precision) as ctx:
            ctx.set_state_fn(p.ic)
            ctx.step(steps, p.dt())
            ctx.sync()
            alone.append(ctx.state()[0])
    ctxs = []
    for p in probs:
        ctx = swe.context_for(p, precision=precision)
        ctx.set_state_fn(p.ic)
        ctxs.append(ctx)
    with swe.Batch(precision=precision, budget_bytes=32 << 30, max_instances=8) as b:
        slots = [b.admit(c, steps, p.dt()) for c, p in zip(ctxs, probs)]
        b.tune(reps=2)
        b.tick(steps)
        done = b.poll()
        assert sorted(s for s, f in done if not f) == sorted(slots)
        for s in slots:
            b.retire(s)
    for i, (ctx, ref) in enumerate(zip(ctxs, alone)):
        got, _ = ctx.state()
        say(f"instance {i}: ne={ctx.ne} p={probs[i].p_max} equal={np.array_equal(got, ref)}")
        assert np.array_equal(got, ref), i
        ctx.close()


@pytest.mark.parametrize("precision,bound", [(swe.SWE_FP32_WB, 1e-6), (swe.SWE_FP64, 1e-11)])
def test_lake_at_rest_full_size(precision, bound):
    """The tidal mesh at full size (524,288 elements, p = 2, bathymetry
    10-4000 m) with a flat surface 0.5 m above the datum at rest and the
    open west edge held at 0.5 m: 50 steps through the benchmarked stage
    kernels keep the surface within the bound (FP32 path: 1e-6 m) and the
    momentum at rest."""
    prob = I.config_c2(n=512, p=2)
    prob.forcing = I.Forcing([0.5], [0.0], [np.pi / 2])
    p = 2
    Href = 0.5 + prob.hb_vertex.max()
    dt = 0.2 * prob.mesh.inscribed_diameters().min() / ((2 * p + 1) * np.sqrt(9.81 * Href))
    with swe.context_for(prob, precision=precision) as ctx:
        ctx.set_state_fn(I.ic_rest(0.5))
        before, _ = ctx.state()
        ctx.step(50, dt)
        ctx.sync()
        got, _ = ctx.state()
    sa = np.sqrt(prob.mesh.areas())
    dev = got[:, 0] - before[:, 0]
    # |xi(x) - xi0(x)| <= sum_i |c_i| max|phi_i| / sqrt(2 area); max|phi_i| < 6 for p <= 3
    drift = np.max(np.sum(np.abs(dev), axis=1) * 6.0 / (np.sqrt(2.0) * sa))
    qmax = np.max(np.abs(got[:, 1:]) / sa[:, None, None])
    say(f"lake at rest full size precision={precision}: surface drift bound {drift:.2e} m, |q| coefficient {qmax:.2e}")
    assert drift <= bound
    assert qmax <= 1e3 * bound
