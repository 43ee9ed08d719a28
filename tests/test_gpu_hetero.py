"""Heterogeneous stages (the paper's CPU + GPU co-execution of the
order-separated scheme): the GPU's base pass over every element and the
host's correction of the listed elements, joined on the GPU.  Results match
the oracle (FP64 within 1e-12 relative L2, FP32 elevation within 1e-5) and
the GPU-only order-separated run, on the dam break's static 1/32 maps and a
random static order map of the tidal family, with open and land edges."""
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


def cases():
    tidal = I.config_c2(n=18, p=3, seed=41)
    tidal.p_base = 1
    tidal.p = np.random.default_rng(41).integers(1, 4, tidal.mesh.ne).astype(np.int8)
    tidal.p[np.random.default_rng(42).random(tidal.mesh.ne) < 0.7] = 1
    return {"dam break p1-2 1/32": I.config_dambreak(n=16, p_lo=1, p_hi=2, every=32, dt_fixed=None),
            "dam break p0-1 1/32": I.config_dambreak(n=16, p_lo=0, p_hi=1, every=32, dt_fixed=None),
            "tidal random p1-3": tidal}


@pytest.mark.parametrize("name", ["dam break p1-2 1/32", "dam break p0-1 1/32", "tidal random p1-3"])
@pytest.mark.parametrize("precision", [swe.SWE_FP64, swe.SWE_FP32_WB])
def test_hetero_matches_oracle(name, precision):
    prob = cases()[name]
    orc = Oracle.from_problem(prob)
    c0 = orc.project(prob.ic)
    dt, steps = prob.dt(), 12
    ref = orc.step(c0, steps, dt, t0=3.0)
    out = {}
    for hetero in (0, 1):
        with swe.context_for(prob, precision=precision, separate=1, hetero=hetero, host_threads=4) as ctx:
            ctx.set_state(c0, t0=3.0)
            ctx.step(5, dt)
            ctx.step(steps - 5, dt)
            ctx.sync()
            out[hetero] = ctx.state()
    got, t = out[1]
    assert abs(t - (3.0 + steps * dt)) < 1e-12 * t
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    exi = np.linalg.norm((got - ref)[:, 0]) / np.linalg.norm(ref[:, 0])
    gpu = np.linalg.norm(got - out[0][0]) / np.linalg.norm(out[0][0])
    say(f"hetero {name} precision={precision}: {int((prob.p > prob.p_base).sum())} of {prob.mesh.ne} above "
        f"base order; vs oracle rel L2 {err:.2e}, xi {exi:.2e}; vs GPU-only separated {gpu:.2e}")
    assert np.all(np.isfinite(got))
    if precision == swe.SWE_FP64:
        assert err < 1e-12 and gpu < 1e-13
    else:
        assert exi < 1e-5 and gpu < 1e-5


def test_hetero_needs_a_static_order_map():
    prob = cases()["dam break p1-2 1/32"]
    cfg = swe.Config(p_base=1, p_max=2, g=1.0, separate=1, hetero=1)
    with swe.Context(cfg) as ctx:
        ctx.set_mesh(prob.mesh.vxy, prob.mesh.tri, prob.mesh.tag)
        ctx.set_bathymetry(prob.hb_vertex)
        with pytest.raises(swe.SweError) as ei:
            ctx.step(1, 1e-5)
        assert ei.value.status == swe.SWE_EINVAL and "static order map" in str(ei.value)
