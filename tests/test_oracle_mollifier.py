"""Pins of the oracle's optional edge-edge mollifier (IPC's smoothing of the
edge-edge barrier as two edges turn parallel; the contact model of Supp. A
follows IPC): the cross-product derivatives against the vector cross product
written out, the mollifier's closed form at its ends, and the mollified
barrier's gradient, Hessian and pose coupling against central differences on a
one-tet gel under a nearly parallel indenter edge."""

import numpy as np
import pytest

from oracle.barrier import (EDGE_MOLLIFIER_REL, edge_cross_derivatives, edge_mollifier,
                            edge_mollifier_d1, edge_mollifier_d2)
from oracle.geometry import GelGeometry, IndenterGeometry
from oracle.problem import EE, StepProblem

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _cross_sq(z):
    a = z[3:6] - z[0:3]
    b = z[9:12] - z[6:9]
    w = np.array([a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]])
    return float(w @ w)


def test_cross_derivatives_match_differences_of_the_cross_product():
    rng = np.random.default_rng(5)
    Z = rng.normal(size=(6, 4, 3))
    c, g, H = edge_cross_derivatives(Z)
    h = 1e-5
    for n in range(len(Z)):
        z = Z[n].ravel()
        assert abs(c[n] - _cross_sq(z)) <= 1e-12 * max(1.0, abs(c[n]))
        gfd = np.zeros(12)
        Hfd = np.zeros((12, 12))
        for i in range(12):
            e = np.zeros(12)
            e[i] = h
            gfd[i] = (_cross_sq(z + e) - _cross_sq(z - e)) / (2 * h)
            # the gradient (pinned just above) is cubic in z: its central
            # difference is exact up to h^2 times a constant third derivative
            gp = edge_cross_derivatives((z + e).reshape(1, 4, 3))[1][0]
            gm = edge_cross_derivatives((z - e).reshape(1, 4, 3))[1][0]
            Hfd[i] = (gp - gm) / (2 * h)
        assert np.allclose(g[n], gfd, rtol=1e-7, atol=1e-7)
        assert np.allclose(H[n], Hfd, rtol=1e-7, atol=1e-7)
        assert np.allclose(H[n], H[n].T, rtol=0, atol=1e-12)


def test_edge_mollifier_ends_and_derivatives():
    eps = 0.37
    assert edge_mollifier(0.0, eps) == 0.0
    assert edge_mollifier(eps, eps) == 1.0 and edge_mollifier(2 * eps, eps) == 1.0
    assert edge_mollifier_d1(eps, eps) == 0.0 and edge_mollifier_d1(3 * eps, eps) == 0.0
    # C^1 at eps from below, slope 2/eps at 0, monotone on [0, eps]
    assert abs(float(edge_mollifier(eps * (1 - 1e-9), eps)) - 1.0) < 1e-15
    assert abs(float(edge_mollifier_d1(eps * (1 - 1e-9), eps))) < 1e-8
    assert float(edge_mollifier_d1(0.0, eps)) == pytest.approx(2.0 / eps)
    c = np.linspace(0.0, eps, 201)
    assert np.all(np.diff(edge_mollifier(c, eps)) > 0)
    h = 1e-7
    for c0 in (0.05, 0.2, 0.33):
        fd1 = (edge_mollifier(c0 + h, eps) - edge_mollifier(c0 - h, eps)) / (2 * h)
        fd2 = (edge_mollifier_d1(c0 + h, eps) - edge_mollifier_d1(c0 - h, eps)) / (2 * h)
        assert float(edge_mollifier_d1(c0, eps)) == pytest.approx(float(fd1), rel=1e-7)
        assert float(edge_mollifier_d2(c0, eps)) == pytest.approx(float(fd2), rel=1e-7)


def _scene(theta, mollify, height=0.03):
    """One tet whose top face lies in z = 0 with the edge x0 -> x1 on the x axis,
    and a triangle indenter whose lowest edge crosses that edge's midpoint at
    `height` above it, turned by `theta` about z."""
    X = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.3, 0.3, -1.0]])
    gel = GelGeometry(X, np.array([[0, 2, 1, 3]]), np.array([False, False, False, True]))
    Y = np.array([[-0.4, 0.0, 0.0], [0.4, 0.0, 0.0], [0.0, 0.1, 0.6]])
    ind = IndenterGeometry(Y, np.array([[0, 1, 2]]))
    prob = StepProblem(gel, ind, 1.0, 0.3, 0.0, 1e-3, 0.05, 10.0, ee_mollifier=mollify)
    prob.set_pose(np.array([0.5, 0.0, height, np.cos(theta / 2), 0.0, 0.0, np.sin(theta / 2)]))
    return prob


def _rest(prob):
    return prob.gel.X.copy()


def test_mollified_scene_has_an_edge_pair_below_the_threshold():
    prob = _scene(0.02, True)
    x = _rest(prob)
    pairs, res = prob.active(x)
    ee = np.nonzero(pairs["kind"] == EE)[0]
    eps = EDGE_MOLLIFIER_REL * 1.0 * 0.8 ** 2
    c = edge_cross_derivatives(res["Z"][ee])[0]
    assert np.any(c < eps)
    # the mollifier lowers the edge-edge barrier of that pair and nothing else
    plain = _scene(0.02, False)
    assert prob.energy(x) < plain.energy(x)
    far = _scene(0.5, True)
    assert far.energy(x) == pytest.approx(_scene(0.5, False).energy(x), rel=1e-14)


def test_parallel_edges_have_no_edge_edge_potential():
    """Exactly parallel edges: c = 0, so the mollified edge-edge terms vanish;
    the energy approaches that value continuously as theta -> 0."""
    x = _rest(_scene(0.0, True))
    prob = _scene(0.0, True)
    pairs, res = prob.active(x)
    val = prob.pair_terms(pairs, res, order=0)[0]
    ee = pairs["kind"] == EE
    par = np.zeros(len(ee), bool)
    if np.any(ee):
        par[ee] = edge_cross_derivatives(res["Z"][ee])[0] < 1e-20
    assert np.any(par)
    assert np.all(val[par] == 0.0)
    e0 = prob.energy(x)
    for th in (1e-3, 1e-4, 1e-5):
        assert abs(_scene(th, True).energy(x) - e0) < 2e3 * th ** 2 * abs(e0) + 1e-12


@pytest.mark.parametrize("theta", [0.0, 0.01, 0.02, 0.1])
def test_mollified_gradient_and_hessian_match_differences(theta):
    prob = _scene(theta, True)
    rng = np.random.default_rng(11)
    x = _rest(prob) + 1e-3 * rng.normal(size=(4, 3)) * (~prob.gel.fixed)[:, None]
    g = prob.gradient(x).ravel()
    H = prob.hessian(x, project=False).toarray()
    h = 1e-6
    free = np.repeat(~prob.gel.fixed, 3)
    for i in np.nonzero(free)[0]:
        e = np.zeros(12)
        e[i] = h
        xp, xm = x + e.reshape(4, 3), x - e.reshape(4, 3)
        fd = (prob.energy(xp) - prob.energy(xm)) / (2 * h)
        assert fd == pytest.approx(g[i], rel=1e-6, abs=1e-8)
        hd = (prob.gradient(xp).ravel() - prob.gradient(xm).ravel()) / (2 * h)
        assert np.allclose(H[i][free], hd[free], rtol=1e-5, atol=1e-6)
    # the diagonal, curvature and preconditioner paths read the same blocks
    assert np.allclose(prob.diag(x).ravel(), np.diag(H))
    p = rng.normal(size=(4, 3))
    assert prob.curvature(x, p) == pytest.approx(float(p.ravel() @ H @ p.ravel()), rel=1e-12)


def test_mollified_pose_coupling_matches_differences():
    """lambda^T d g / d pose (the adjoint's pose term) against central
    differences of the gradient under pose offsets."""
    from oracle.adjoint import _pose_mixed_terms, offset_pose
    prob = _scene(0.015, True)
    rng = np.random.default_rng(2)
    x = _rest(prob) + 1e-3 * rng.normal(size=(4, 3)) * (~prob.gel.fixed)[:, None]
    lam = rng.normal(size=(4, 3)) * (~prob.gel.fixed)[:, None]
    got = _pose_mixed_terms(prob, x, lam)
    pose = prob.pose.copy()
    h = 1e-6
    for a in range(6):
        dt = np.zeros(3)
        dw = np.zeros(3)
        (dt if a < 3 else dw)[a % 3] = h
        prob.set_pose(offset_pose(pose, dt, dw))
        gp = prob.gradient(x)
        prob.set_pose(offset_pose(pose, -dt, -dw))
        gm = prob.gradient(x)
        prob.set_pose(pose)
        fd = float(np.sum(lam * (gp - gm))) / (2 * h)
        assert got[a] == pytest.approx(fd, rel=1e-5, abs=1e-7)


def test_threshold_is_relative_to_the_rest_lengths():
    """eps_x = 1e-3 |a_rest|^2 |b_rest|^2: for the two edges in one plane,
    c = |a|^2 |b|^2 sin^2(theta), so the mollifier acts exactly when
    sin^2(theta) < 1e-3, whatever the edge lengths."""
    th = np.arcsin(np.sqrt(EDGE_MOLLIFIER_REL))
    x = _rest(_scene(0.0, True))
    assert _scene(1.02 * th, True).energy(x) == pytest.approx(_scene(1.02 * th, False).energy(x), rel=1e-14)
    assert _scene(0.98 * th, True).energy(x) < _scene(0.98 * th, False).energy(x)
