"""Pins of the oracle's minimum depth control (a reading of the paper's
"minimum depth control to avoid negative depths", a kernel its code runs,
Sec. "Performance results"; the paper gives no formula, so the reading is a
mass-conserving scaling of each element's deviation of the total depth from
its mean, H' = mean H + theta (H - mean H), with theta bringing H up to h_min
at the element's vertices and edge midpoints, the momentum's deviation scaled
by the same theta).

Each pin checks values fixed by hand (linear and quadratic fields on one
triangle, whose point values and means are known exactly) or an invariant
(means kept, h_min reached at every check point, untouched states), and each
fails on a plausible mistake planted in a private copy of the oracle source.
"""
import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2311_11348_amd import inputs as I
from tests.test_oracle_terms import assert_catches

# check points of the reference triangle (0,0), (1,0), (0,1): vertices and edge midpoints
CHECK = [(0.0, 0.0), (1.0, 0.0), (0.0, 1.0), (0.5, 0.5), (0.0, 0.5), (0.5, 0.0)]


def one_triangle(hb, p):
    """The reference triangle itself as a one-element mesh (all land)."""
    vxy = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    tri = np.array([[0, 1, 2]], np.int32)
    tag = np.zeros((1, 3), np.int8)
    return Oracle(vxy, np.asarray(hb, float), tri, tag, p, g=9.81)


def depths(o, c, hb, pts=CHECK):
    """Total depth xi + h_b at points of the one-element mesh."""
    out = np.zeros(5)
    H = []
    for x, y in pts:
        o.L.orc_eval(o.h, c.ctypes.data_as(np.ctypeslib.ctypes.POINTER(np.ctypeslib.ctypes.c_double)),
                     0, x, y, out.ctypes.data_as(np.ctypeslib.ctypes.POINTER(np.ctypeslib.ctypes.c_double)))
        H.append(out[0] + hb[0] * (1 - x - y) + hb[1] * x + hb[2] * y)
    return np.array(H)


def projected(o, xi, U=None, V=None):
    """L2 projection of point functions onto the element's space (exact for polynomials of its degree)."""
    def f(x, y):
        z = np.zeros_like(x)
        return (xi(x, y), (U or (lambda a, b: z))(x, y), (V or (lambda a, b: z))(x, y))
    return np.ascontiguousarray(o.project(f))


def test_linear_surface_flat_bottom():
    """h_b = 1, xi = -0.8 + 0.8 x + 1.6 y: depths 0.2, 1.0, 1.8 at the
    vertices, mean 1.0.  With h_min = 0.5, theta = (1 - 0.5) / (1 - 0.2) =
    0.625: the vertex depths become 0.5, 1.0, 1.5 and the midpoints their
    averages; the mean stays 1."""
    hb = [1.0, 1.0, 1.0]
    o = one_triangle(hb, 2)
    c = projected(o, lambda x, y: -0.8 + 0.8 * x + 1.6 * y, lambda x, y: 2.0 + x, lambda x, y: -1.0 + y)
    assert np.allclose(depths(o, c, hb)[:3], [0.2, 1.0, 1.8], atol=1e-13)
    c2, n = o.depth_limit(c, 0.5)
    assert n == 1
    H = depths(o, c2, hb)
    assert np.allclose(H, [0.5, 1.0, 1.5, 1.25, 1.0, 0.75], atol=1e-12), H
    # the momentum's deviation from its mean scaled by theta, its mean kept
    assert c2[0, 1, 0] == c[0, 1, 0] and c2[0, 2, 0] == c[0, 2, 0]
    assert np.allclose(c2[0, 1, 1:], 0.625 * c[0, 1, 1:], rtol=1e-14, atol=1e-15)
    assert np.allclose(c2[0, 2, 1:], 0.625 * c[0, 2, 1:], rtol=1e-14, atol=1e-15)


def test_flat_surface_sloping_bottom():
    """xi = 0 over h_b = 0.1, 1, 1 at the vertices: depths 0.1, 1, 1, mean 0.7.
    With h_min = 0.3, theta = 0.4 / 0.6 = 2/3: H becomes 0.3, 0.9, 0.9 at the
    vertices, so xi (the only thing that can change) takes a slope,
    xi = 0.2, -0.1, -0.1 there."""
    hb = [0.1, 1.0, 1.0]
    o = one_triangle(hb, 1)
    c = projected(o, lambda x, y: 0.0 * x)
    c2, n = o.depth_limit(c, 0.3)
    assert n == 1
    H = depths(o, c2, hb)
    assert np.allclose(H[:3], [0.3, 0.9, 0.9], atol=1e-12), H
    assert abs(c2[0, 0, 0]) < 1e-15     # the mean of xi (the mass) is still 0


def test_minimum_at_an_edge_midpoint():
    """h_b = 1, xi = -3.6 x y: 0 at the vertices and at two edge midpoints,
    -0.9 at the midpoint of the edge opposite the origin; mean xi = -0.3.
    The vertices alone see no shallow point; the midpoint's depth 0.1 sets
    theta = (0.7 - 0.4) / (0.7 - 0.1) = 0.5 for h_min = 0.4."""
    hb = [1.0, 1.0, 1.0]
    o = one_triangle(hb, 2)
    c = projected(o, lambda x, y: -3.6 * x * y)
    assert np.allclose(depths(o, c, hb), [1.0, 1.0, 1.0, 0.1, 1.0, 1.0], atol=1e-12)
    c2, n = o.depth_limit(c, 0.4)
    assert n == 1
    H = depths(o, c2, hb)
    assert np.allclose(H, [0.85, 0.85, 0.85, 0.4, 0.85, 0.85], atol=1e-12), H


def test_untouched_when_deep_enough():
    """Every check point at least h_min deep: the state is returned bitwise."""
    hb = [1.0, 1.0, 1.0]
    o = one_triangle(hb, 3)
    c = projected(o, lambda x, y: -0.8 + 0.8 * x + 1.6 * y + 0.1 * x * y * y)
    c2, n = o.depth_limit(c, 0.1)
    assert n == 0 and np.array_equal(c2, c)


def shallow_state(n=12, p=2, seed=9):
    """A jittered mesh over a flat 1 m bottom with a random state whose
    elevation reaches down to about -0.95 m (depths near and below 0.1 m)."""
    mesh = I.structured_mesh(n, jitter=0.2, seed=seed)
    hb = np.full(mesh.nv, 1.0)
    o = Oracle(mesh.vxy, hb, mesh.tri, mesh.tag, p)
    c = I.random_state(mesh, np.full(mesh.ne, p), p, seed=seed, hb_vertex=hb, xi_amp=0.6, q_amp=1.0,
                       decay=1.0)
    return o, mesh, hb, c


def check_point_depths(o, mesh, hb, c):
    """Depth at each element's six check points, and the element means."""
    H = np.zeros((mesh.ne, 6))
    out = np.zeros(5)
    P = lambda a: a.ctypes.data_as(np.ctypeslib.ctypes.POINTER(np.ctypeslib.ctypes.c_double))
    for e in range(mesh.ne):
        v = mesh.vxy[mesh.tri[e]]
        h3 = hb[mesh.tri[e]]
        for j, (a, b) in enumerate(CHECK):
            x, y = v[0] + a * (v[1] - v[0]) + b * (v[2] - v[0])
            o.L.orc_eval(o.h, P(c), e, x, y, P(out))
            H[e, j] = out[0] + h3[0] * (1 - a - b) + h3[1] * a + h3[2] * b
    mean = c[:, 0, 0] / np.sqrt(mesh.areas()) + hb[mesh.tri].mean(axis=1)
    return H, mean


def test_means_kept_and_h_min_reached():
    """On a random shallow state: the elements' means of xi, U and V are kept
    bitwise; every element whose mean depth exceeds h_min reaches at least
    h_min at all six check points; an element below h_min on average is
    made flat (its depth equal to its mean at every check point)."""
    o, mesh, hb, c = shallow_state()
    h_min = 0.5
    H0, _ = check_point_depths(o, mesh, hb, c)
    c2, n = o.depth_limit(c, h_min)
    assert n == int(np.sum(H0.min(axis=1) < h_min)) and n > 10
    assert np.array_equal(c2[:, :, 0], c[:, :, 0])
    H, mean = check_point_depths(o, mesh, hb, c2)
    deep = mean > h_min
    assert np.all(H[deep].min(axis=1) >= h_min - 1e-12)
    if np.any(~deep):
        assert np.allclose(H[~deep], mean[~deep, None], atol=1e-12)


def test_order_zero_untouched():
    o, mesh, hb, c = shallow_state(p=1)
    o.set_order(np.zeros(mesh.ne, np.int32))
    c0 = c.copy()
    c0[:, :, 1:] = 0.0
    c2, n = o.depth_limit(c0, 0.5)
    assert n == 0 and np.array_equal(c2, c0)


def test_step_applies_the_control_after_every_stage():
    """With the control on, a step equals the hand-composed stages (RK
    update, control, RK update, control) built from the oracle's own RHS."""
    o, mesh, hb, c = shallow_state(n=8, p=2)
    h_min, dt = 0.3, 2e-4
    ref = Oracle(mesh.vxy, hb, mesh.tri, mesh.tag, 2)
    c1, _ = ref.depth_limit(c + dt * ref.rhs(0.0, c), h_min)
    c2, _ = ref.depth_limit(0.5 * c + 0.5 * (c1 + dt * ref.rhs(dt, c1)), h_min)
    o.set_depth_limit(h_min)
    got = o.step(c, 1, dt)
    assert np.allclose(got, c2, rtol=0, atol=1e-14 * np.abs(c2).max())


# ----------------------------------------------------------- planted mistakes
def test_catches_missing_bathymetry_term(tmp_path):
    """xi's deviation scaled alone, as if h_b were flat."""
    assert_catches(tmp_path, "ce[n] = theta * ce[n] + (n < 3 ? (theta - 1.0) * bq[n] : 0.0);",
                   "ce[n] = theta * ce[n];", test_flat_surface_sloping_bottom)


def test_catches_vertices_only(tmp_path):
    assert_catches(tmp_path, "for (int j = 0; j < 6; ++j) {\n        basis_eval(Ke, px[j]",
                   "for (int j = 0; j < 3; ++j) {\n        basis_eval(Ke, px[j]", test_minimum_at_an_edge_midpoint)


def test_catches_wrong_theta(tmp_path):
    """theta from the ratio of depths instead of their distances to the mean."""
    assert_catches(tmp_path, "? (Hm - h_min) / (Hm - Hlow) : 0.0;", "? Hlow / h_min : 0.0;",
                   test_linear_surface_flat_bottom)


def test_catches_momentum_left_alone(tmp_path):
    assert_catches(tmp_path, "        ce[K + n] *= theta;\n", "", test_linear_surface_flat_bottom)


def test_catches_control_skipped_in_the_first_stage(tmp_path):
    assert_catches(tmp_path, "if (o->h_min > 0.0) orc_depth_limit(h, c1, o->h_min);", "",
                   test_step_applies_the_control_after_every_stage)
