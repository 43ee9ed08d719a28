"""Synthetic workloads against the numbers the paper prints for them."""
import numpy as np

from paper_2311_11348_amd import inputs as I

K_OF_P = np.array([1, 3, 6, 10])


def test_dambreak_matches_the_papers_counts():
    """Sec. "Radial dam break": 2,097,152 triangles; the statically adaptive
    setups (every 32nd element at the higher order) have 6,684,672 (p0-1) and
    19,464,192 (p1-2) degrees of freedom per stage, as the paper's tables list;
    uniform p0, p1, p2 have 6,291,456, 18,874,368 and 37,748,736."""
    expect = {(0, 1, 32): 6_684_672, (1, 2, 32): 19_464_192, (0, 0, 0): 6_291_456, (1, 1, 0): 18_874_368,
              (2, 2, 0): 37_748_736}
    for (lo, hi, every), dof in expect.items():
        prob = I.config_dambreak(n=1024, p_lo=lo, p_hi=hi, every=every)
        assert prob.mesh.ne == 2_097_152
        assert 3 * int(K_OF_P[prob.p].sum()) == dof
        assert prob.p_base == lo and prob.p_max == hi
    prob = I.config_dambreak(n=1024)
    assert prob.g == 1.0 and prob.f_coriolis == 1e-5
    assert prob.friction == I.FRICTION_LINEAR and prob.friction_coef == 1e-4
    assert prob.dt() == 1e-5
    assert np.all(prob.hb_vertex == 0.5)
    assert prob.mesh.vxy.min() == 0.0 and prob.mesh.vxy.max() == 5.0
    assert np.all(prob.mesh.tag[prob.mesh.tag >= 0] == I.TAG_LAND)        # walls only
    xi, U, V = prob.ic(np.array([2.5, 2.5 + 0.49, 2.5 + 0.51, 0.0]), np.array([2.5, 2.5, 2.5, 0.0]))
    assert xi[0] == 2.5 and abs(xi[1] - (2.0 + 0.5 * np.exp(-15 * 0.49 ** 2))) < 1e-15
    assert xi[2] == 1.0 and xi[3] == 1.0 and not U.any() and not V.any()
