"""Edge-item layouts of the shared-flux stage kernel against the oracle.

A block's edge items are grouped by kind (in-block pairs, outside
neighbours, land, open).  While the block still fits in its 512 slots with
every kind starting on a run of 64 (one wave's lanes), empty slots go before
each kind; otherwise the kinds follow each other unpadded.  The tidal,
tsunami and dam-break meshes of the other tests give padded blocks.  A grid
of walled islands of 3 x 3 squares gives blocks with many land items, which
fit only unpadded.  The host-side count below follows the library's element
order (Morton order of the centroids, each axis scaled to 16 bits, ties by
index) to check that the mesh has such blocks and that every block still
fits (so the shared-flux kernel, not the gather kernel, runs).  The
right-hand side and a short run then match the oracle."""
import sys

import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2311_11348_amd import inputs as I
from paper_2311_11348_amd import swe

pytestmark = pytest.mark.gpu

BLOCK, SLOTS, WAVE = 256, 512, 64


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def islands(g=10, m=3, size=5e3, gap=2e3, p=2, seed=21):
    """g x g islands of m x m squares (two triangles each), walled all round."""
    vxy, tri, tag = [], [], []
    nv = 0
    for j in range(g):
        for i in range(g):
            isl = I.structured_mesh(m, length=size, jitter=0.15, seed=seed + j * g + i)
            vxy.append(isl.vxy + [i * (size + gap), j * (size + gap)])
            tri.append(isl.tri + nv)
            tag.append(isl.tag)
            nv += len(isl.vxy)
    mesh = I.Mesh(vxy=np.concatenate(vxy), tri=np.concatenate(tri).astype(np.int32),
                  tag=np.concatenate(tag).astype(np.int8))
    x, y = mesh.vxy[:, 0], mesh.vxy[:, 1]
    hb = 30.0 + 20.0 * np.sin(x / 9e3) * np.cos(y / 7e3)

    def ic(x, y):
        return 0.3 * np.sin(x / 4e3) * np.cos(y / 5e3), 2.0 + 0.0 * x, -1.0 + 0.0 * y

    return I.Problem(name="islands", mesh=mesh, hb_vertex=hb, ic=ic, p=np.full(mesh.ne, p, np.int8), p_base=p,
                     p_max=p, f_coriolis=1e-4)


def spread16(v):
    v = v.astype(np.uint64) & 0xFFFF
    v = (v | (v << 8)) & 0x00FF00FF
    v = (v | (v << 4)) & 0x0F0F0F0F
    v = (v | (v << 2)) & 0x33333333
    v = (v | (v << 1)) & 0x55555555
    return v


def block_layouts(mesh):
    """Per block: (slots used unpadded, slots used with every kind on a run of 64)."""
    vxy, tri = mesh.vxy, mesh.tri
    ne = len(tri)
    a, b, d = vxy[tri[:, 0]], vxy[tri[:, 1]], vxy[tri[:, 2]]
    c = (a + b + d) / 3.0
    lo, hi = c.min(axis=0), c.max(axis=0)
    q = ((c - lo) * (65535.0 / (hi - lo))).astype(np.uint32)
    key = spread16(q[:, 0]) | (spread16(q[:, 1]) << np.uint64(1))
    order = np.lexsort((np.arange(ne), key))        # element at each new position
    new = np.empty(ne, np.int64)
    new[order] = np.arange(ne)
    owner = {}
    for e in range(ne):
        for k in range(3):
            owner.setdefault(tuple(sorted((tri[e][(k + 1) % 3], tri[e][(k + 2) % 3]))), []).append(e)
    counts = np.zeros(((ne + BLOCK - 1) // BLOCK, 4), np.int64)   # pairs, outside, land, open
    for es in owner.values():
        if len(es) == 1:
            counts[new[es[0]] // BLOCK, 2] += 1       # every boundary edge here is land
            continue
        i, j = sorted(new[e] for e in es)
        if i // BLOCK == j // BLOCK:
            counts[i // BLOCK, 0] += 1
        else:
            counts[i // BLOCK, 1] += 1
            counts[j // BLOCK, 1] += 1
    out = []
    for row in counts:
        padded = 0
        for n in row:
            if n:
                padded = (padded + WAVE - 1) // WAVE * WAVE + int(n)
        out.append((int(row.sum()), padded))
    return out


def test_island_blocks_fall_back_to_unpadded_items():
    """Host-side only: the island mesh has blocks that fit unpadded but not
    padded, and every block fits one way or the other."""
    lay = block_layouts(islands().mesh)
    unpadded = sum(1 for u, pd in lay if pd > SLOTS)
    say(f"islands: {len(lay)} blocks, slots unpadded/padded {lay}")
    assert all(min(u, pd) <= SLOTS for u, pd in lay)
    assert unpadded >= 3


@pytest.mark.parametrize("p", [1, 2, 3])
def test_island_rhs_matches_oracle(p):
    prob = islands(p=p)
    orc = Oracle.from_problem(prob)
    c = I.random_state(prob.mesh, prob.p, p, seed=300 + p, hb_vertex=prob.hb_vertex, xi_amp=0.5, q_amp=5.0)
    ref = orc.rhs(0.0, c)
    with swe.context_for(prob) as ctx:
        got = ctx.rhs(0.0, c)
    assert np.all(np.isfinite(got))
    err = max(np.max(np.abs(got[:, j] - ref[:, j])) / np.max(np.abs(ref[:, j])) for j in range(3))
    say(f"islands p={p}: RHS max error relative to each component's max {err:.2e}")
    assert err < 1e-12


@pytest.mark.parametrize("precision", [swe.SWE_FP64, swe.SWE_FP32_WB])
def test_island_run_matches_oracle(precision):
    prob = islands(p=2)
    orc = Oracle.from_problem(prob)
    c0 = orc.project(prob.ic)
    dt, steps = prob.dt(), 10
    ref = orc.step(c0, steps, dt)
    with swe.context_for(prob, precision=precision) as ctx:
        ctx.set_state(c0)
        ctx.step(steps, dt)
        ctx.sync()
        got, _ = ctx.state()
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    exi = np.linalg.norm((got - ref)[:, 0]) / np.linalg.norm(ref[:, 0])
    say(f"islands run precision={precision}: rel L2 {err:.2e}, xi {exi:.2e}")
    if precision == swe.SWE_FP64:
        assert err < 1e-12
    else:
        assert exi < 1e-5
