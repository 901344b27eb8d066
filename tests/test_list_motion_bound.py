"""The neighbour-list rebuild rule: between a list's build and now, the
distance between a gel point g and an indenter triangle drops by at most
|g_now - (M (g_build - t_build) + t_now)| + theta D_build, where M = R_now
R_build^T is the indenter's rotation since the build (angle theta) and D_build
the distance at the build. Checked on random rigid motions, triangles and gel
motions with the oracle's exact point-triangle distance."""

import numpy as np

from oracle.distance import point_triangle


def _rot(axis, ang):
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + np.sin(ang) * K + (1 - np.cos(ang)) * K @ K


def test_distance_drop_is_bounded_by_relative_motion():
    rng = np.random.default_rng(3)
    worst = 0.0
    for _ in range(4000):
        Y = rng.uniform(-1.0, 1.0, (3, 3))                       # indenter triangle, local frame
        Rb = _rot(rng.standard_normal(3), rng.uniform(0, np.pi))
        tb = rng.uniform(-1.0, 1.0, 3)
        theta = rng.uniform(0.0, 0.2)
        Rn = _rot(rng.standard_normal(3), theta) @ Rb
        tn = tb + rng.uniform(-0.3, 0.3, 3)
        g = rng.uniform(-1.5, 1.5, 3)
        gn = g + rng.uniform(-0.2, 0.2, 3)
        Wb, Wn = Y @ Rb.T + tb, Y @ Rn.T + tn
        Db = point_triangle(g, *Wb)["d"][0]
        Dn = point_triangle(gn, *Wn)["d"][0]
        M = Rn @ Rb.T
        rel = np.linalg.norm(gn - (M @ (g - tb) + tn))
        bound = rel + theta * Db
        assert Db - Dn <= bound + 1e-12, (Db, Dn, bound)
        worst = max(worst, (Db - Dn) / bound if bound > 0 else 0.0)
    assert worst > 0.5                                         # the bound is not vacuous


def test_gel_static_indenter_translating_gives_the_translation():
    """A gel point at rest and an indenter translating by dt: relative motion |dt|."""
    g = np.array([0.3, -0.2, 0.1])
    tb, tn = np.zeros(3), np.array([0.0, 0.0, -0.05])
    rel = np.linalg.norm(g - (np.eye(3) @ (g - tb) + tn))
    assert np.isclose(rel, 0.05)
