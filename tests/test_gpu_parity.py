"""HIP path vs the FP64 oracle, element by element, through the C ABI.

Sizes span several 256-element tiles plus a ragged tail; inputs are seeded and
identical on both sides (the oracle projects the initial data, both receive
the same coefficient array).
"""
import math
import sys

import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2311_11348_amd import inputs as I
from paper_2311_11348_amd import swe

pytestmark = pytest.mark.gpu

RHS_TOL_FP64 = 1e-12     # max-norm error relative to the max-norm of each component
STEP_TOL_FP64 = 1e-12    # relative L2 after a run


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def problem(n=20, p=2, seed=5, open_west=True, friction=2, fc=3.19e-5, bathy=None, jitter=0.2):
    mesh = I.structured_mesh(n, jitter=jitter, seed=seed, open_west=open_west)
    bathy = bathy or I.bathy_sincos()
    hb = bathy(mesh.vxy[:, 0], mesh.vxy[:, 1])
    forcing = I.Forcing([0.3, 0.1], [2 * math.pi / 44712.0, 2 * math.pi / 3000.0], [0.2, 1.0]) if open_west else I.Forcing()
    return I.Problem(name="t", mesh=mesh, hb_vertex=hb, ic=I.ic_rest(), p=np.full(mesh.ne, p, np.int8),
                     p_base=p, p_max=p, f_coriolis=fc, friction=friction, friction_coef=0.009 if friction == 2 else 1e-4,
                     forcing=forcing, bathy=bathy)


def rel_max_err(a, b):
    assert np.all(np.isfinite(a)), "non-finite values in the GPU result"
    assert np.all(np.isfinite(b)), "non-finite values in the reference"
    out = 0.0
    for j in range(3):
        s = np.max(np.abs(b[:, j]))
        if s > 0:
            out = max(out, np.max(np.abs(a[:, j] - b[:, j])) / s)
    return out


@pytest.mark.parametrize("p", [0, 1, 2, 3])
@pytest.mark.parametrize("friction", [1, 2])
def test_rhs_parity_fp64(p, friction):
    prob = problem(n=20, p=p, friction=friction)
    say(f"rhs parity p={p} friction={friction} ne={prob.mesh.ne}")
    orc = Oracle.from_problem(prob)
    c = I.random_state(prob.mesh, prob.p, p, seed=100 + p, hb_vertex=prob.hb_vertex, xi_amp=1.0, q_amp=20.0)
    ref = orc.rhs(1234.5, c)
    with swe.context_for(prob) as ctx:
        got = ctx.rhs(1234.5, c)
    err = rel_max_err(got, ref)
    say("  err", err)
    assert err < RHS_TOL_FP64


@pytest.mark.parametrize("p", [0, 1, 2, 3])
def test_usolve_parity_fp64(p):
    prob = problem(n=20, p=p)
    orc = Oracle.from_problem(prob)
    c = I.random_state(prob.mesh, prob.p, p, seed=200 + p, hb_vertex=prob.hb_vertex, xi_amp=1.0, q_amp=20.0)
    ref = orc.usolve(c)
    with swe.context_for(prob) as ctx:
        got = ctx.usolve(c)
    err = max(np.max(np.abs(got[:, j] - ref[:, j])) / np.max(np.abs(ref[:, j])) for j in range(2))
    say(f"usolve p={p} err {err}")
    assert err < 1e-13


def test_c1_run_fp64():
    """C1: 32x32x2, p = 1, flat 10 m, 0.1 m bump, land walls, 100 steps."""
    prob = I.config_c1()
    orc = Oracle.from_problem(prob)
    c0 = orc.project(prob.ic)
    dt = prob.dt()
    say(f"c1 ne={prob.mesh.ne} dt={dt}")
    ref = orc.step(c0, prob.steps, dt)
    with swe.context_for(prob) as ctx:
        ctx.set_state(c0)
        ctx.step(prob.steps, dt)
        ctx.sync()
        got, t = ctx.state()
    assert abs(t - prob.steps * dt) < 1e-9 * t
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    say("  c1 rel L2", err)
    assert err < STEP_TOL_FP64
    dxi = np.linalg.norm((got - ref)[:, 0]) / np.linalg.norm(ref[:, 0])
    assert dxi < STEP_TOL_FP64


@pytest.mark.parametrize("p", [1, 2, 3])
def test_run_parity_fp64_open_boundary(p):
    """Jittered mesh, sin*cos bathymetry, tide on the west edge, friction + Coriolis."""
    prob = problem(n=16, p=p)
    orc = Oracle.from_problem(prob)
    c0 = orc.project(I.ic_gaussian(0.5, 2e4, 5e4, 5e4))
    dt = 0.2 * prob.mesh.inscribed_diameters().min() / ((2 * p + 1) * math.sqrt(9.81 * 4001))
    ref = orc.step(c0, 20, dt, t0=100.0)
    with swe.context_for(prob) as ctx:
        ctx.set_state(c0, t0=100.0)
        ctx.step(20, dt)
        ctx.sync()
        got, _ = ctx.state()
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    say(f"run p={p} rel L2 {err}")
    assert err < STEP_TOL_FP64


def test_mixed_order_fused_fp64():
    """Per-element orders in {0..3} through the fused full-order kernel (masked)."""
    prob = problem(n=16, p=3)
    rng = np.random.default_rng(7)
    pe = rng.integers(0, 4, prob.mesh.ne).astype(np.int8)
    prob.p = pe
    prob.p_base = 0
    orc = Oracle.from_problem(prob)
    c = I.random_state(prob.mesh, pe, 3, seed=77, hb_vertex=prob.hb_vertex, xi_amp=1.0, q_amp=20.0)
    ref = orc.rhs(10.0, c)
    with swe.context_for(prob) as ctx:
        got = ctx.rhs(10.0, c)
        assert np.array_equal(ctx.order(), pe)
    err = rel_max_err(got, ref)
    say("mixed fused err", err)
    assert err < RHS_TOL_FP64


def test_mass_and_lake_at_rest_gpu_fp64():
    prob = problem(n=16, p=2, open_west=False)
    orc = Oracle.from_problem(prob)
    c0 = orc.project(I.ic_rest(0.5))
    Href = 0.5 + prob.hb_vertex.max()
    dt = 0.2 * prob.mesh.inscribed_diameters().min() / (5 * math.sqrt(9.81 * Href))
    with swe.context_for(prob) as ctx:
        ctx.set_state(c0)
        m0 = ctx.mass()
        ctx.step(100, dt)
        ctx.sync()
        got, _ = ctx.state()
        m1 = ctx.mass()
    sa = np.sqrt(prob.mesh.areas())
    assert abs(m1 - m0) <= 1e-12 * np.sum(np.abs(c0[:, 0, 0]) * sa)
    assert abs(m0 - orc.mass(c0)) <= 1e-13 * abs(m0)
    # xi stays 0.5, q stays 0 (coefficient bound: |f(x)| <= sum_i |c_i| max|phi_i| / sqrt(2 a))
    dev = got.copy()
    dev[:, 0, 0] -= 0.5 * sa
    bound = np.max(np.sum(np.abs(dev), axis=2) * 4.0 / sa[:, None])
    say("lake at rest bound", bound)
    assert bound <= 1e-12 * Href * math.sqrt(9.81 * Href)


def test_determinism_fp64():
    prob = problem(n=16, p=2)
    c = I.random_state(prob.mesh, prob.p, 2, seed=9, hb_vertex=prob.hb_vertex, xi_amp=1.0, q_amp=5.0)
    dt = 0.1
    outs = []
    for _ in range(2):
        with swe.context_for(prob) as ctx:
            ctx.set_state(c)
            ctx.step(10, dt)
            ctx.sync()
            outs.append(ctx.state()[0])
    assert np.array_equal(outs[0], outs[1])
