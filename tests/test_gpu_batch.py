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


def mixed_members():
    """Members with per-element orders beside uniform ones: a static random
    order map (tidal family, orders 1-3), the dam break's every-32nd map
    (p1-2), the tsunami with orders from the indicator (1-3), the dam break
    with orders from the indicator (p0-1), and uniform p1 and p3 instances
    sharing those members' pools."""
    out = []
    prob = I.config_c2(n=14, p=3, seed=31)
    prob.p = np.random.default_rng(31).integers(1, 4, prob.mesh.ne).astype(np.int8)
    out.append(("static random p1-3", prob, 21))
    out.append(("dam break 1/32 p1-2", I.config_dambreak(n=16, p_lo=1, p_hi=2, every=32, dt_fixed=None), 17))
    out.append(("tsunami adaptive p1-3", I.config_c3(n=18), 25))
    out.append(("dam break adaptive p0-1", I.config_dambreak(n=16, p_lo=0, p_hi=1, dt_fixed=None, adapt_tau=1e-2), 14))
    uni1 = I.config_instance(911, n_lo=300, n_hi=900)
    uni1.p[:] = 1
    uni1.p_max = uni1.p_base = 1
    out.append(("uniform p1", uni1, 19))
    uni3 = I.config_instance(912, n_lo=300, n_hi=900)
    uni3.p[:] = 3
    uni3.p_max = uni3.p_base = 3
    out.append(("uniform p3", uni3, 12))
    return out


@pytest.mark.parametrize("precision", [swe.SWE_FP64, swe.SWE_FP32_WB])
def test_batch_mixed_order_members(precision):
    """Mixed-order members in one batch with uniform ones (members joining
    mid-run, the tuner choosing kernels): each member's result matches the
    oracle (FP64 state within 1e-12 relative L2 and identical order maps;
    FP32 elevation within 1e-5 and maps agreeing on 99 % of the elements)
    and is bitwise its result alone."""
    cases = mixed_members()
    refs, c0s = [], []

    def oracle_run(args):
        _, prob, n = args
        orc = Oracle.from_problem(prob)
        c0 = orc.project(prob.ic)
        ref = orc.step(c0, n, prob.dt(), adapt=bool(prob.adapt), tau=prob.adapt_tau, p_lo=prob.p_base,
                       p_hi=prob.p_max)
        return c0, ref, orc.order()
    with ThreadPoolExecutor(max_workers=len(cases)) as pool:
        res = list(pool.map(oracle_run, cases))
    alone = []
    for (name, prob, n), (c0, _, _) in zip(cases, res):
        with ctx_for(prob, precision, c0) as ctx:
            ctx.step(n, prob.dt())
            ctx.sync()
            alone.append((ctx.state()[0], ctx.order()))
    ctxs = [ctx_for(prob, precision, r[0]) for (_, prob, _), r in zip(cases, res)]
    with swe.Batch(precision=precision, budget_bytes=4 << 30, max_instances=8) as b:
        slots = [b.admit(c, n, prob.dt()) for c, (_, prob, n) in zip(ctxs[:3], cases[:3])]
        b.tick(4)
        slots += [b.admit(c, n, prob.dt()) for c, (_, prob, n) in zip(ctxs[3:], cases[3:])]
        b.tune(reps=2)
        used = {p: b.tile_config(p) for p in range(4)}
        b.tick(40)
        b.sync()
        for s in slots:
            left, _, failed = b.query(s)
            assert left == 0 and not failed
            b.retire(s)
    say(f"mixed-order batch precision={precision}: kernels {used}")
    for (name, prob, n), ctx, (_, ref, pref), (al, pal) in zip(cases, ctxs, res, alone):
        got, _ = ctx.state()
        pgot = ctx.order()
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        exi = np.linalg.norm((got - ref)[:, 0]) / np.linalg.norm(ref[:, 0])
        agree = float(np.mean(pgot == pref))
        hi = int((pref > prob.p_base).sum())
        say(f"  {name}: ne={ctx.ne} steps={n} above base order {hi}, maps agree {agree:.4f}, equal alone "
            f"{np.array_equal(got, al)}, vs oracle rel L2 {err:.2e}, xi {exi:.2e}")
        assert np.array_equal(got, al) and np.array_equal(pgot, pal), name
        if precision == swe.SWE_FP64:
            assert np.array_equal(pgot, pref), name
            assert err < 1e-12, name
        else:
            assert agree >= 0.99, name
            assert exi < 1e-5, name
        ctx.close()
    assert not used[1][2] and not used[2][2] and not used[3][2]   # those classes hold per-element orders
