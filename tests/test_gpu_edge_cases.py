"""Degenerate and invalid inputs through the C-ABI on the device.

A one-element mesh (every edge land, or one edge open) and a two-element
mesh at every order and both precisions against the oracle; meshes the
library must refuse (clockwise or zero-area triangles, vertex ids out of
range, an edge shared by three triangles, empty meshes); states it must
refuse (non-finite coefficients) or flag during a run (non-positive mean
depth), and recovery from the failed state; zero-step and bad-step calls.
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


def tiny_problem(p, ne, open_edge=False):
    """One triangle, or two sharing their diagonal, 10 km across, bathymetry
    20-60 m, a smooth elevation and momentum field."""
    vxy = np.array([[0.0, 0.0], [1e4, 0.0], [0.0, 1e4], [1e4, 1e4]])
    tri = np.array([[0, 1, 2]] if ne == 1 else [[0, 1, 2], [1, 3, 2]], np.int32)
    vxy = vxy[: 3 if ne == 1 else 4]
    tag = np.zeros((ne, 3), np.int8)
    if ne == 2:
        tag[0, 0] = -1          # the shared diagonal (opposite vertex 0 of the first triangle)
        tag[1, 1] = -1          # ... and opposite vertex 3 of the second
    if open_edge:
        tag[0, 1] = 1           # the west edge (x = 0) is open sea
    mesh = I.Mesh(vxy=vxy, tri=tri, tag=tag)
    hb = np.array([20.0, 40.0, 60.0, 35.0])[: mesh.nv]

    def ic(x, y):
        xi = 0.3 * np.sin(x / 4e3) * np.cos(y / 5e3)
        return xi, 2.0 + 0.1 * x / 1e4, -1.0 + 0.2 * y / 1e4

    prob = I.Problem(name=f"tiny{ne}", mesh=mesh, hb_vertex=hb, ic=ic, p=np.full(ne, p, np.int8), p_base=p,
                     p_max=p, f_coriolis=1e-4, friction=I.FRICTION_QUADRATIC, friction_coef=0.003)
    if open_edge:
        prob.forcing = I.tide_forcing()
    return prob


@pytest.mark.parametrize("ne,open_edge", [(1, False), (1, True), (2, False), (2, True)])
@pytest.mark.parametrize("p", [0, 1, 2, 3])
@pytest.mark.parametrize("precision", [swe.SWE_FP64, swe.SWE_FP32_WB])
def test_tiny_meshes_match_oracle(precision, p, ne, open_edge):
    prob = tiny_problem(p, ne, open_edge)
    orc = Oracle.from_problem(prob)
    c0 = orc.project(prob.ic)
    rhs_ref = orc.rhs(5.0, c0)
    dt = 0.5
    ref = orc.step(c0, 3, dt, t0=5.0)
    with swe.context_for(prob, precision=precision) as ctx:
        rhs = ctx.rhs(5.0, c0)
        ctx.set_state(c0, t0=5.0)
        ctx.step(3, dt)
        ctx.sync()
        got, t = ctx.state()
    tol_rhs, tol_run = (1e-12, 1e-12) if precision == swe.SWE_FP64 else (1e-4, 1e-5)
    # per-component scale, floored where a component vanishes (p = 0, all land: no mass flux)
    floor = 1e-9 * np.max(np.abs(rhs_ref))
    scale = [max(np.max(np.abs(rhs_ref[:, j])), floor) for j in range(3)]
    e_rhs = max(np.max(np.abs(rhs[:, j] - rhs_ref[:, j])) / scale[j] for j in range(3))
    e_run = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    say(f"precision={precision} p={p} ne={ne} open={open_edge}: rhs {e_rhs:.2e}, 3 steps {e_run:.2e}")
    assert abs(t - (5.0 + 3 * dt)) < 1e-12
    assert e_rhs < tol_rhs and e_run < tol_run


def ctx_p1():
    return swe.Context(swe.Config(precision=swe.SWE_FP64, p_base=1, p_max=1))


def expect_status(fn, status):
    with pytest.raises(swe.SweError) as ei:
        fn()
    assert ei.value.status == status, str(ei.value)
    say(f"  refused: {ei.value}")


def test_meshes_refused():
    sq = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0], [1.0, 1.0]])
    cases = {
        "clockwise": (sq[:3], np.array([[0, 2, 1]], np.int32)),
        "zero area": (np.array([[0.0, 0.0], [1.0, 0.0], [2.0, 0.0]]), np.array([[0, 1, 2]], np.int32)),
        "vertex id out of range": (sq[:3], np.array([[0, 1, 3]], np.int32)),
        "negative vertex id": (sq[:3], np.array([[0, 1, -1]], np.int32)),
        # edge 1-2 shared by three counter-clockwise triangles
        "edge of three triangles": (np.vstack([sq, [[2.0, 2.0]]]),
                                    np.array([[0, 1, 2], [1, 3, 2], [1, 4, 2]], np.int32)),
        "empty": (sq[:3], np.zeros((0, 3), np.int32)),
    }
    for name, (vxy, tri) in cases.items():
        say(name)
        with ctx_p1() as ctx:
            expect_status(lambda: ctx.set_mesh(vxy, tri), swe.SWE_EINVAL)


def test_states_and_steps_refused_and_recovered():
    prob = tiny_problem(1, 2)
    orc = Oracle.from_problem(prob)
    c0 = orc.project(prob.ic)
    with swe.context_for(prob) as ctx:
        bad = c0.copy()
        bad[1, 2, 0] = np.nan
        expect_status(lambda: ctx.set_state(bad), swe.SWE_EINVAL)
        ctx.set_state(c0)
        before, _ = ctx.state()       # the upload's scaling rounds: compare with what the device holds
        expect_status(lambda: ctx.step(1, 0.0), swe.SWE_EINVAL)
        expect_status(lambda: ctx.step(1, -1.0), swe.SWE_EINVAL)
        expect_status(lambda: ctx.step(1, float("inf")), swe.SWE_EINVAL)
        expect_status(lambda: ctx.step(-1, 0.5), swe.SWE_EINVAL)
        ctx.step(0, 0.5)                      # nothing to do
        ctx.sync()
        same, t = ctx.state()
        assert np.array_equal(same, before) and t == 0.0
        # every element dry: the run flags it, the context refuses to step on
        dry = c0.copy()
        dry[:, 0, 0] = -500.0 * np.sqrt(prob.mesh.areas())
        ctx.set_state(dry)
        ctx.step(1, 0.5)
        expect_status(ctx.sync, swe.SWE_ESTATE)
        expect_status(lambda: ctx.step(1, 0.5), swe.SWE_ESTATE)
        # a new state clears the failed state
        ctx.set_state(c0)
        ctx.step(2, 0.5)
        ctx.sync()
        got, _ = ctx.state()
    ref = orc.step(c0, 2, 0.5)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-12


def isolated_triangles(count, p, seed=11):
    """count disjoint triangles (every edge land): 3 edge items per element,
    more than the shared-flux kernel takes per block."""
    rng = np.random.default_rng(seed)
    vxy, tri = [], []
    for i in range(count):
        x0, y0 = (i % 20) * 1.2e4, (i // 20) * 1.2e4
        a = rng.uniform(5e3, 9e3)
        vxy += [[x0, y0], [x0 + a, y0 + 1e3], [x0 + 2e3, y0 + a]]
        tri.append([3 * i, 3 * i + 1, 3 * i + 2])
    vxy, tri = np.array(vxy), np.array(tri, np.int32)
    mesh = I.Mesh(vxy=vxy, tri=tri, tag=np.zeros((count, 3), np.int8))
    hb = rng.uniform(20.0, 80.0, len(vxy))

    def ic(x, y):
        return 0.2 * np.sin(x / 3e3) * np.cos(y / 4e3), 1.0 + 0.0 * x, -0.5 + 0.0 * y

    return I.Problem(name="isolated", mesh=mesh, hb_vertex=hb, ic=ic, p=np.full(count, p, np.int8), p_base=p,
                     p_max=p, f_coriolis=1e-4)


@pytest.mark.parametrize("precision", [swe.SWE_FP64, swe.SWE_FP32_WB])
def test_too_many_items_fall_back_to_gather(precision):
    """A mesh whose blocks hold more edge items than the shared-flux kernel
    takes runs on the element-gather kernel: alone against the oracle, and in
    a batch (its order then falls back for every member) bitwise equal to
    alone, beside an ordinary member of the same order."""
    p = 2
    prob = isolated_triangles(300, p)
    orc = Oracle.from_problem(prob)
    c0 = orc.project(prob.ic)
    dt, steps = 0.5, 6
    ref = orc.step(c0, steps, dt)
    other = I.config_instance(301, n_lo=2000, n_hi=4000)
    other.p_max = other.p_base = p
    other.p = np.full(other.mesh.ne, p, np.int8)
    with swe.context_for(prob, precision=precision) as ctx:
        ctx.set_state(c0)
        ctx.step(steps, dt)
        ctx.sync()
        alone_iso, _ = ctx.state()
    with swe.context_for(other, precision=precision) as ctx:
        ctx.set_state_fn(other.ic)
        ctx.step(steps, other.dt())
        ctx.sync()
        alone_other, _ = ctx.state()
    tol = 1e-12 if precision == swe.SWE_FP64 else 1e-5
    err = np.linalg.norm(alone_iso - ref) / np.linalg.norm(ref)
    say(f"isolated triangles precision={precision}: rel L2 vs oracle {err:.2e}")
    assert err < tol
    c_iso = swe.context_for(prob, precision=precision)
    c_iso.set_state(c0)
    c_oth = swe.context_for(other, precision=precision)
    c_oth.set_state_fn(other.ic)
    with swe.Batch(precision=precision, budget_bytes=4 << 30, max_instances=4) as b:
        s1 = b.admit(c_oth, steps, other.dt())
        s2 = b.admit(c_iso, steps, dt)
        b.set_tile(p, 256, True)          # asked for, but a member has no edge items
        tile, _, shared = b.tile_config(p)
        say(f"  batch order {p}: tile {tile}, shared {shared}")
        assert not shared
        b.tick(steps)
        b.sync()
        b.retire(s1)
        b.retire(s2)
    got_iso, _ = c_iso.state()
    got_oth, _ = c_oth.state()
    c_iso.close()
    c_oth.close()
    assert np.array_equal(got_iso, alone_iso)
    assert np.array_equal(got_oth, alone_other)
