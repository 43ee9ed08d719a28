"""Batched instances: each instance's result inside a batch (persistent
launches over all resident instances, captured step replayed, membership
changing between ticks, autotuned tiles) matches the oracle run of the same
instance (FP64 within 1e-12 relative L2, FP32 elevation within 1e-5) and is
bitwise the result of the same instance run on its own; admission respects
the footprint budget."""
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2311_11348_amd import inputs as I
from paper_2311_11348_amd import swe

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make_instances(count, seed, n_lo=200, n_hi=6000):
    probs = []
    for i in range(count):
        prob = I.config_instance(seed * 100 + i, n_lo=n_lo, n_hi=n_hi)
        probs.append(prob)
    return probs


def ctx_for(prob, precision, c0=None):
    ctx = swe.context_for(prob, precision=precision)
    if c0 is None:
        ctx.set_state_fn(prob.ic)
    else:
        ctx.set_state(c0)
    return ctx


class OracleRuns:
    """The mixed-size instances of the batch test, their initial states
    projected by the oracle and the oracle's runs of each (computed once, one
    thread per instance: the oracle releases the interpreter lock)."""

    def __init__(self):
        self.probs = make_instances(6, seed=7)
        self.steps = [30, 17, 25, 40, 9, 33]
        self.c0, self.ref = [], []

        def one(args):
            prob, n = args
            orc = Oracle.from_problem(prob)
            c0 = orc.project(prob.ic)
            return c0, orc.step(c0, n, prob.dt())
        with ThreadPoolExecutor(max_workers=6) as pool:
            for c0, ref in pool.map(one, zip(self.probs, self.steps)):
                self.c0.append(c0)
                self.ref.append(ref)


@pytest.fixture(scope="module")
def oracle_runs():
    say("oracle runs of the batch instances")
    return OracleRuns()


@pytest.mark.parametrize("precision", [swe.SWE_FP64, swe.SWE_FP32_WB])
def test_batch_equals_alone(precision, oracle_runs):
    probs, steps, c0s = oracle_runs.probs, oracle_runs.steps, oracle_runs.c0
    dts = [p.dt() for p in probs]
    alone = []
    for prob, n, dt, c0 in zip(probs, steps, dts, c0s):
        ctx = ctx_for(prob, precision, c0)
        ctx.step(n, dt)
        ctx.sync()
        alone.append(ctx.state())
        ctx.close()
    ctxs = [ctx_for(p, precision, c0) for p, c0 in zip(probs, c0s)]
    with swe.Batch(precision=precision, budget_bytes=8 << 30, max_instances=16) as b:
        slots = [b.admit(c, n, dt) for c, n, dt in zip(ctxs[:4], steps[:4], dts[:4])]
        b.tick(5)
        slots += [b.admit(c, n, dt) for c, n, dt in zip(ctxs[4:], steps[4:], dts[4:])]   # join mid-run
        b.tick(10)
        b.tune(reps=2)
        b.tick(50)
        b.sync()
        for s, n in zip(slots, steps):
            left, t, failed = b.query(s)
            assert left == 0 and not failed
        for s in slots:
            b.retire(s)
        assert b.resident() == 0
    for i, (ctx, (ref, tref)) in enumerate(zip(ctxs, alone)):
        got, t = ctx.state()
        orc = oracle_runs.ref[i]
        err = np.linalg.norm(got - orc) / np.linalg.norm(orc)
        exi = np.linalg.norm((got - orc)[:, 0]) / np.linalg.norm(orc[:, 0])
        say(f"instance {i}: ne={ctx.ne} p={probs[i].p_max} equal={np.array_equal(got, ref)} t={t:.3f}/{tref:.3f} "
            f"vs oracle rel L2 {err:.2e}, xi {exi:.2e}")
        assert np.array_equal(got, ref), i
        assert t == tref
        if precision == swe.SWE_FP64:
            assert err < 1e-12, i
        else:
            assert exi < 1e-5, i
        ctx.close()


@pytest.mark.parametrize("precision", [swe.SWE_FP64, swe.SWE_FP32_WB])
def test_batch_kernels_equal_alone(precision):
    """Each kernel choice of the batch (element gather with 64- and 256-element
    tiles, shared edge fluxes on 256-element tiles where the order has it)
    gives every instance bitwise its result alone.  Sizes span several tiles
    with ragged ends; every order 1-3 is present."""
    probs = []
    seed = 300
    while len({p.p_max for p in probs}) < 3 or len(probs) < 6:
        prob = I.config_instance(seed, n_lo=300, n_hi=9000)
        seed += 1
        if sum(q.p_max == prob.p_max for q in probs) < 2:
            probs.append(prob)
    steps = 12
    alone = []
    for prob in probs:
        ctx = ctx_for(prob, precision)
        ctx.step(steps, prob.dt())
        ctx.sync()
        alone.append(ctx.state()[0])
        ctx.close()
    choices = [(64, False), (256, False), (256, True)]
    for tile, shared in choices:
        ctxs = [ctx_for(p, precision) for p in probs]
        with swe.Batch(precision=precision, budget_bytes=8 << 30, max_instances=8) as b:
            slots = [b.admit(c, steps, p.dt()) for c, p in zip(ctxs, probs)]
            used = {}
            for p in range(4):
                sh = shared and p >= 1
                b.set_tile(p, tile, sh)
                used[p] = b.tile_config(p)
            b.tick(steps)
            b.sync()
            for s in slots:
                b.retire(s)
        say(f"tile {tile} shared {shared}: " + ", ".join(f"p{p} {used[p]}" for p in (1, 2, 3)))
        for i, (ctx, ref) in enumerate(zip(ctxs, alone)):
            got, _ = ctx.state()
            eq = np.array_equal(got, ref)
            if not eq:
                say(f"  instance {i} ne={ctx.ne} p={probs[i].p_max}: max diff {np.max(np.abs(got - ref)):.3e}")
            assert eq, (tile, shared, i)
            ctx.close()


def test_batch_admission_budget():
    probs = make_instances(3, seed=9)
    ctxs = [ctx_for(p, swe.SWE_FP32_WB) for p in probs]
    need = [swe.swe_footprint_bytes(c.ne, p.p_max, swe.SWE_FP32_WB) for c, p in zip(ctxs, probs)]
    budget = need[0] + need[1] // 2
    with swe.Batch(precision=swe.SWE_FP32_WB, budget_bytes=budget, max_instances=4) as b:
        s0 = b.admit(ctxs[0], 3, probs[0].dt())
        with pytest.raises(swe.SweError) as ei:
            b.admit(ctxs[1], 3, probs[1].dt())
        assert ei.value.status == swe.SWE_ENOMEM
        with pytest.raises(swe.SweError):
            ctxs[0].step(1, 1.0)       # resident contexts refuse their own stepping
        b.tick(3)
        b.retire(s0)
        assert b.free_bytes() == budget
        with pytest.raises(swe.SweError):      # precision mismatch
            fp64 = ctx_for(probs[2], swe.SWE_FP64)
            b.admit(fp64, 1, 1.0)
    for c in ctxs:
        c.close()
