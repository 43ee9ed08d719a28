"""Adaptive steps whose correction lists are longer than the teams take.

Below order 3 a list of more than 16,384 entries is corrected one element
per thread, and in an adaptive step graph (one chain per step) the
correction kernel also joins the base part and finishes the listed
elements' stage, the sum the epilogue kernel forms otherwise.  The tsunami
family on 128 x 128 x 2 elements with orders 1-2 and a threshold so small
that most elements take order 2 gives such a list.  The step graph must
equal kernel-by-kernel launches (which join in the epilogue) bit for bit,
and both the oracle's adaptive run (FP64, identical order maps)."""
import sys

import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2311_11348_amd import inputs as I
from paper_2311_11348_amd import swe

pytestmark = pytest.mark.gpu

TAU = 1e-9


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def problem(n=128):
    prob = I.config_c3(n=n)
    prob.p_max = 2
    prob.p = np.ones(prob.mesh.ne, np.int8)
    prob.adapt, prob.adapt_tau = 1, TAU
    return prob


def run(prob, c0, steps, dt, graph):
    with swe.context_for(prob, precision=swe.SWE_FP64, separate=1, step_graph=graph) as ctx:
        ctx.set_state(c0)
        ctx.step(1, dt)
        ctx.step(steps - 1, dt)
        ctx.sync()
        c, _ = ctx.state()
        p = ctx.order()
    return c, p


def test_long_lists_in_adaptive_chain():
    prob = problem()
    orc = Oracle.from_problem(prob)
    c0 = orc.project(prob.ic)
    dt, steps = prob.dt(), 3
    c = c0
    for s in range(steps):
        ind = orc.indicator(s * dt, c)
        assert np.min(np.abs(ind - TAU)) / TAU > 1e-9, s
        c = orc.step(c, 1, dt, t0=s * dt, adapt=True, tau=TAU, p_lo=1, p_hi=2)
    ref, pref = c, orc.order()
    n2 = int(np.sum(pref == 2))
    say(f"long lists: {prob.mesh.ne} elements, {n2} at order 2 after {steps} steps")
    assert n2 > 16384
    cg, pg = run(prob, c0, steps, dt, 2)
    cl, pl = run(prob, c0, steps, dt, 0)
    err = np.linalg.norm(cg - ref) / np.linalg.norm(ref)
    say(f"  graph vs launches equal {np.array_equal(cg, cl)}, vs oracle rel L2 {err:.2e}, "
        f"maps equal {np.array_equal(pg, pref)}")
    assert np.array_equal(pg, pref) and np.array_equal(pl, pref)
    assert np.array_equal(cg, cl)
    assert err < 1e-12
