"""Order-partitioned scheme (separate = 2): every element's full stage computed
by the kernel of its order class, the base kernel skipping listed elements.
It computes the same right-hand side as the fused and separated schemes, so
runs match the oracle (static mixed orders, adaptive runs with identical order
maps) and the separated scheme."""
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


def mixed_problem(n=20, b=1, pm=3, seed=8):
    prob = I.config_c2(n=n, p=pm, seed=seed)
    prob.p_base = b
    rng = np.random.default_rng(seed)
    prob.p = rng.integers(b, pm + 1, prob.mesh.ne).astype(np.int8)
    prob.p[rng.random(prob.mesh.ne) < 0.6] = b          # mostly base order, scattered higher orders
    return prob


@pytest.mark.parametrize("b,pm", [(0, 1), (1, 2), (1, 3), (2, 3), (0, 3)])
def test_partitioned_static_fp64(b, pm):
    prob = mixed_problem(b=b, pm=pm)
    orc = Oracle.from_problem(prob)
    c0 = I.random_state(prob.mesh, prob.p, pm, seed=40 + pm, hb_vertex=prob.hb_vertex, xi_amp=0.5, q_amp=5.0)
    dt = prob.dt()
    ref = orc.step(c0, 20, dt, t0=5.0)
    with swe.context_for(prob, separate=2) as ctx:
        ctx.set_state(c0, t0=5.0)
        ctx.step(20, dt)
        ctx.sync()
        got, _ = ctx.state()
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    say(f"partitioned b={b} pm={pm}: rel L2 {err:.2e}")
    assert err < 1e-12


@pytest.mark.parametrize("graph", [0, 1])
def test_partitioned_adaptive_fp64(graph):
    prob = I.config_c3(n=24)
    orc = Oracle.from_problem(prob)
    c0 = orc.project(prob.ic)
    dt = prob.dt()
    ref = orc.step(c0, 30, dt, adapt=True, tau=prob.adapt_tau, p_lo=1, p_hi=3)
    with swe.context_for(prob, separate=2, step_graph=graph) as ctx:
        ctx.set_state(c0)
        ctx.step(30, dt)
        ctx.sync()
        got, _ = ctx.state()
        pgot = ctx.order()
    assert np.array_equal(pgot, orc.order())
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    counts = np.bincount(pgot, minlength=4)
    say(f"partitioned adaptive graph={graph}: p1/p2/p3 {counts[1]}/{counts[2]}/{counts[3]}, rel L2 {err:.2e}")
    assert counts[2] + counts[3] > 0
    assert err < 1e-12


@pytest.mark.skip(reason="FP32 order-partitioned stepping with orders up to 3 is switched off: one run of it "
                         "aborted on the device and no cause has been found in the source")
def test_partitioned_matches_separated_fp32():
    prob = I.config_c3(n=32)
    orc = Oracle.from_problem(prob)
    c0 = orc.project(prob.ic)
    dt = prob.dt()
    out = {}
    for sep in (1, 2):
        with swe.context_for(prob, precision=swe.SWE_FP32_WB, separate=sep) as ctx:
            ctx.set_state(c0)
            ctx.step(40, dt)
            ctx.sync()
            out[sep] = (ctx.state()[0], ctx.order())
    agree = np.mean(out[1][1] == out[2][1])
    err = np.linalg.norm((out[1][0] - out[2][0])[:, 0]) / np.linalg.norm(out[1][0][:, 0])
    say(f"fp32 partitioned vs separated: order agreement {agree:.4f}, xi rel L2 {err:.2e}")
    assert agree > 0.99 and err < 1e-5
