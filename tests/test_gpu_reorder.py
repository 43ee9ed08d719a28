"""A static order map replaced during a run.

Setting a static order map on a separated context renumbers the elements
(unlisted first, then the listed elements of each order); a second map
renumbers an already renumbered mesh.  Three steps under one map, a new map,
three more steps, against the oracle doing the same (the state kept and
truncated to the new orders between the two runs, as the interface defines),
in the order-separated and order-partitioned schemes, FP64.
"""
import dataclasses
import sys

import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2311_11348_amd import inputs as I
from paper_2311_11348_amd import swe

pytestmark = pytest.mark.gpu

K_OF_P = np.array([1, 3, 6, 10])


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("separate", [1, 2])
def test_second_order_map_matches_oracle(separate):
    prob = I.config_c2(n=20, p=2)
    prob.p_base = 1
    ne = prob.mesh.ne
    map_a = np.full(ne, 1, np.int8)
    map_a[::5] = 2
    map_b = np.full(ne, 1, np.int8)
    map_b[3::7] = 2
    prob_a = dataclasses.replace(prob, p=map_a)
    prob_b = dataclasses.replace(prob, p=map_b)
    dt, steps = prob.dt(), 3
    c0 = I.random_state(prob.mesh, map_a, 2, seed=21, hb_vertex=prob.hb_vertex, xi_amp=0.5, q_amp=5.0)
    # oracle: three steps under map A, truncate to map B, three more steps
    o_a = Oracle.from_problem(prob_a)
    c1 = o_a.step(c0, steps, dt, t0=0.0)
    c1 = c1 * (np.arange(c1.shape[2])[None, None, :] < K_OF_P[map_b][:, None, None])
    o_b = Oracle.from_problem(prob_b)
    ref = o_b.step(c1, steps, dt, t0=steps * dt)
    with swe.context_for(prob_a, separate=separate) as ctx:
        ctx.set_state(c0)
        ctx.step(steps, dt)
        ctx.sync()
        ctx.set_order(map_b)
        assert np.array_equal(ctx.order(), map_b)
        ctx.step(steps, dt)
        ctx.sync()
        got, t = ctx.state()
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    say(f"second order map, separate={separate}: rel L2 {err:.2e}, t={t:.4f}")
    assert abs(t - 2 * steps * dt) < 1e-12
    assert err < 1e-12
