"""Listed-element kernels on long lists: the kernels that reach order 3 take
every list by teams of waves over a grid sized for the longest possible
list; kernels up to order 2 take a list of more than 16,384 entries one
element per thread and a shorter one by teams, in the same launch.  Static
and indicator-driven order maps on 32,768 elements with more than 16,384
listed elements of one order, against the oracle (FP64 within 1e-12
relative L2, identical order maps; FP32 elevation within 1e-5)."""
import sys

import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2311_11348_amd import inputs as I
from paper_2311_11348_amd import swe

pytestmark = pytest.mark.gpu

N = 128          # 32,768 elements
TEAM_MAX = 16384


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def static_case(name):
    """The tidal family with a seeded random static order map: 70 % of the
    elements at order 3 (orders 1-3), or 60 % at order 2 (orders 1-2)."""
    rng = np.random.default_rng(71)
    if name == "p1-3 mostly 3":
        prob = I.config_c2(n=N, p=3, seed=71)
        u = rng.random(prob.mesh.ne)
        prob.p = np.where(u < 0.7, 3, np.where(u < 0.85, 2, 1)).astype(np.int8)
    else:
        prob = I.config_c2(n=N, p=2, seed=72)
        prob.p = np.where(rng.random(prob.mesh.ne) < 0.6, 2, 1).astype(np.int8)
    prob.p_base = 1
    return prob


def listed_counts(prob):
    """Entries of each order's list of the separated and partitioned schemes:
    elements above the base order, or next to one."""
    m, p, b = prob.mesh, prob.p, prob.p_base
    nb = Oracle.from_problem(prob).neighbours()[0]
    above = p > b
    near = np.array([above[e] or any(n >= 0 and above[n] for n in nb[e]) for e in range(m.ne)])
    return np.bincount(p[near], minlength=4)


CASES = [("p1-3 mostly 3", swe.SWE_FP64, 1), ("p1-3 mostly 3", swe.SWE_FP64, 2),
         ("p1-3 mostly 3", swe.SWE_FP32_WB, 1),
         ("p1-2 mostly 2", swe.SWE_FP64, 1), ("p1-2 mostly 2", swe.SWE_FP64, 2),
         ("p1-2 mostly 2", swe.SWE_FP32_WB, 1), ("p1-2 mostly 2", swe.SWE_FP32_WB, 2)]


@pytest.fixture(scope="module")
def oracle_static():
    out = {}
    for name in ("p1-3 mostly 3", "p1-2 mostly 2"):
        prob = static_case(name)
        orc = Oracle.from_problem(prob)
        c0 = orc.project(prob.ic)
        dt = prob.dt()
        say(f"oracle: {name}")
        out[name] = (prob, c0, dt, orc.step(c0, 3, dt))
    return out


@pytest.mark.parametrize("name,precision,separate", CASES)
def test_static_long_lists(name, precision, separate, oracle_static):
    prob, c0, dt, ref = oracle_static[name]
    counts = listed_counts(prob)
    assert counts.max() > TEAM_MAX, "one list must be longer than a team kernel's short list"
    with swe.context_for(prob, precision=precision, separate=separate) as ctx:
        ctx.set_state(c0)
        ctx.step(3, dt)
        ctx.sync()
        got, _ = ctx.state()
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    exi = np.linalg.norm((got - ref)[:, 0]) / np.linalg.norm(ref[:, 0])
    say(f"{name} precision={precision} separate={separate}: list lengths by order {counts.tolist()}, "
        f"rel L2 {err:.2e}, xi {exi:.2e}")
    assert np.all(np.isfinite(got))
    if precision == swe.SWE_FP64:
        assert err < 1e-12
    else:
        assert exi < 1e-5


@pytest.mark.parametrize("separate", [1, 2])
def test_adaptive_long_lists(separate):
    """A random initial state (linear modes) on the tsunami family: the
    indicator puts every element with a jump of at least tau at order 3, so
    the device-built order-3 list holds almost every element."""
    prob = I.config_c3(n=N)
    orc = Oracle.from_problem(prob)
    p0 = np.full(prob.mesh.ne, 1)
    c0 = I.random_state(prob.mesh, p0, prob.p_max, seed=73, hb_vertex=prob.hb_vertex, xi_amp=0.5, q_amp=5.0)
    dt, steps = prob.dt(), 3
    ref = orc.step(c0, steps, dt, adapt=True, tau=prob.adapt_tau, p_lo=1, p_hi=3)
    pref = orc.order()
    counts = np.bincount(pref, minlength=4)
    assert counts[3] > TEAM_MAX
    with swe.context_for(prob, separate=separate) as ctx:
        ctx.set_state(c0)
        ctx.step(steps, dt)
        ctx.sync()
        got, _ = ctx.state()
        pgot = ctx.order()
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    say(f"adaptive separate={separate}: orders p1/p2/p3 = {counts[1]}/{counts[2]}/{counts[3]}, "
        f"maps equal {np.array_equal(pgot, pref)}, rel L2 {err:.2e}")
    assert np.array_equal(pgot, pref)
    assert err < 1e-12
