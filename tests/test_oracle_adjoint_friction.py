"""Pins of the oracle's friction adjoint (gradients through the friction lag
of a load-step sequence):
* the derivative of the lagged friction gradient with respect to the lag
  points, per pair, against central differences of its definition, for every
  pair kind and closest-point region, sticking and sliding;
* every per-step term (material, friction coefficient, pose offset through
  the current and the lag pose, carry to the previous state) against central
  differences of the step gradient itself;
* the whole sequence adjoint against central differences of the forward
  simulation (Newton to 1e-12 mm at theta +- h)."""

import dataclasses

import numpy as np
import pytest

from oracle.adjoint import (N_THETA, adjoint_sequence, lag_objective, lag_objective_grad,
                            offset_pose, step_adjoint_terms)
from oracle.problem import EE, FV, VF
from oracle.sim import build, simulate
from scenes.configs import micro_press

DHAT, KAPPA, EPS_V, MU_F = 0.05, 1e3, 1e-3, 0.5
TILT = np.array([0.99996192, 0.00610865, 0.00436331, 0.0])


def _plate_scene():
    q = TILT / np.linalg.norm(TILT)
    return micro_press(mesh="micro3", indenter="plate", depth=0.08, n_steps=2, mu_f=MU_F,
                       shear=(0.05, 0.02), n_shear=2, xy=(0.1, -0.05), q=tuple(q))


def _tri():
    return np.array([[0.0, 0.0, 0.0], [1.0, 0.1, 0.0], [0.2, 0.9, 0.05]])


def _point_over(tri, bary, h):
    nrm = np.cross(tri[1] - tri[0], tri[2] - tri[0])
    nrm /= np.linalg.norm(nrm)
    return bary @ tri + h * nrm


def _pair_cases(rng):
    """(Zp (4,3), kind) covering VF/FV interiors, edges and vertices, and EE
    interiors and an end point; every pair closer than dhat."""
    cases = []
    tri = _tri()
    for bary in ([0.3, 0.3, 0.4], [0.5, 0.53, -0.03], [1.02, -0.01, -0.01]):
        for kind in (VF, FV):
            h = rng.uniform(0.005, 0.02)
            p = _point_over(tri, np.array(bary), h)
            cases.append((np.vstack([p[None], tri]), kind))
    a0, a1 = np.array([0.0, 0.0, 0.0]), np.array([1.0, 0.2, 0.0])
    cases.append((np.stack([a0, a1, [0.4, -0.5, 0.02], [0.6, 0.6, 0.03]]), EE))
    cases.append((np.stack([a0, a1, [1.02, -0.5, 0.01], [1.04, 0.6, 0.015]]), EE))
    for Zp, kind in cases:
        d = np.linalg.norm(np.einsum("ni,nid->nd", *_closest_c(Zp, kind)))
        assert 0.0 < d < 0.9 * DHAT, (kind, d)
    return cases


def _closest_c(Zp, kind):
    from oracle.adjoint import _closest
    _, c, _, _ = _closest(Zp[None], np.array([kind]))
    return c, Zp[None]


def _is_gel(kind):
    return np.array({VF: [1, 0, 0, 0], FV: [0, 1, 1, 1], EE: [1, 1, 0, 0]}[kind], dtype=bool)


@pytest.mark.parametrize("slide", [0.3, 5.0])
def test_lag_objective_gradient_matches_differences(slide):
    rng = np.random.default_rng(7)
    for Zp, kind in _pair_cases(rng):
        Zp = Zp[None]
        kinds = np.array([kind])
        is_gel = _is_gel(kind)[None]
        Z = Zp + slide * EPS_V * rng.standard_normal((1, 4, 3))
        ell = rng.standard_normal((1, 4, 3)) * is_gel[:, :, None]
        args = (kinds, is_gel, ell, MU_F, KAPPA, DHAT, EPS_V)
        G = lag_objective_grad(Zp, Z, *args)[0]
        fd = np.zeros((4, 3))
        h = 1e-7
        for i in range(4):
            for c in range(3):
                P, M = Zp.copy(), Zp.copy()
                P[0, i, c] += h
                M[0, i, c] -= h
                fd[i, c] = (lag_objective(P, Z, *args)[0] - lag_objective(M, Z, *args)[0]) / (2 * h)
        scale = np.abs(fd).max()
        assert scale > 0
        assert np.allclose(G, fd, rtol=1e-5, atol=1e-6 * scale), (kind, G, fd)


@pytest.fixture(scope="module")
def plate_run():
    w = _plate_scene()
    env = w.envs[0]
    r = simulate(w.meshes[env.mesh], w.indenters[env.indenter], env, mode="newton", tol=1e-12)
    return w, env, r


def _step_gradient(w, env, x, xp, theta):
    """Gradient of Pi_s at x with the lag at (xp, q_{s-1}) for a perturbed theta,
    the pose offset applied to both poses."""
    dE, dnu, dmu, dt, dw, s = theta
    e = dataclasses.replace(env, E=env.E + dE, nu=env.nu + dnu, mu_f=env.mu_f + dmu)
    _, _, prob = build(w.meshes[e.mesh], w.indenters[e.indenter], e)
    prob.set_lag(xp, offset_pose(env.poses[s - 1], dt, dw))
    prob.set_pose(offset_pose(env.poses[s], dt, dw))
    return prob.gradient(x)


def test_step_terms_match_differences(plate_run):
    w, env, r = plate_run
    gel, _, prob = build(w.meshes[env.mesh], w.indenters[env.indenter], env)
    s = 4                                    # a shear step: friction lag with every pair kind
    xs = [gel.X] + r.x
    x, xp = xs[s], xs[s - 1]
    rng = np.random.default_rng(5)
    lam_x = rng.standard_normal(x.shape)
    lam_x[gel.fixed] = 0.0
    prob.set_lag(xp, env.poses[s - 1])
    prob.set_pose(env.poses[s])
    theta, carry = step_adjoint_terms(prob, x, xp, env.poses[s - 1], lam_x)
    z3 = np.zeros(3)
    hs = [env.E * 1e-6, env.nu * 1e-6, 1e-6] + [1e-6] * 6
    for i, h in enumerate(hs):
        def q(sgn):
            v = np.zeros(N_THETA)
            v[i] = sgn * h
            return float(np.sum(lam_x * _step_gradient(w, env, x, xp, (v[0], v[1], v[2], v[3:6], v[6:9], s))))
        fd = (q(+1) - q(-1)) / (2 * h)
        assert -theta[i] == pytest.approx(fd, rel=2e-5, abs=1e-7 * max(1.0, abs(fd))), (i, -theta[i], fd)
    # carry: d/de lambda^T g_s(x; lag at xp + e v) = -carry . v
    v = rng.standard_normal(x.shape)
    v[gel.fixed] = 0.0
    h = 1e-7
    gp = _step_gradient(w, env, x, xp + h * v, (0.0, 0.0, 0.0, z3, z3, s))
    gm = _step_gradient(w, env, x, xp - h * v, (0.0, 0.0, 0.0, z3, z3, s))
    fd = float(np.sum(lam_x * (gp - gm))) / (2 * h)
    assert -float(np.sum(carry * v)) == pytest.approx(fd, rel=2e-5), (float(np.sum(carry * v)), fd)
    assert np.all(carry[gel.fixed] == 0.0)


def test_frictionless_sequence_reduces_to_the_last_step():
    """Without friction only the last step carries the loss: earlier steps' rhs is
    zero, so the sequence adjoint equals the single-step one."""
    w = micro_press(mesh="micro3", indenter="sphere_small", depth=0.15, n_steps=3, xy=(0.12, -0.07))
    env = w.envs[0]
    r = simulate(w.meshes[env.mesh], w.indenters[env.indenter], env, mode="newton", tol=1e-12)
    gel, _, prob = build(w.meshes[env.mesh], w.indenters[env.indenter], env)
    rng = np.random.default_rng(2)
    du = np.zeros((3, len(gel.marker_w), 3))
    du[-1] = rng.standard_normal(du[-1].shape)
    g_seq = adjoint_sequence(prob, [gel.X] + r.x, env.poses, du)
    _, _, p1 = build(w.meshes[env.mesh], w.indenters[env.indenter], env)
    from oracle.adjoint import adjoint_gradient
    p1.set_pose(env.poses[-1])
    g_one, _ = adjoint_gradient(p1, r.x[-1], du[-1], x_prev=r.x[-2], pose_prev=env.poses[-2])
    assert np.allclose(g_seq, g_one, rtol=1e-9, atol=1e-12 * np.abs(g_one).max())


@pytest.mark.slow
def test_sequence_adjoint_matches_central_differences(plate_run):
    w, env, r0 = plate_run
    gel, _, prob = build(w.meshes[env.mesh], w.indenters[env.indenter], env)
    rng = np.random.default_rng(17)
    n_m = len(gel.marker_w)
    S = len(env.poses) - 1
    tgt = 0.02 * rng.standard_normal((S, n_m, 3))
    wts = np.zeros(S)
    wts[-1], wts[1] = 1.0, 0.5               # loss on the last step and on the last press step

    def loss(theta):
        dE, dnu, dmu, dt, dw = theta
        e = dataclasses.replace(env, E=env.E + dE, nu=env.nu + dnu, mu_f=env.mu_f + dmu,
                                poses=np.stack([offset_pose(p, dt, dw) for p in env.poses]))
        r = simulate(w.meshes[e.mesh], w.indenters[e.indenter], e, mode="newton", tol=1e-12)
        return sum(0.5 * wts[s] * float(np.sum((r.markers[s] - tgt[s]) ** 2)) for s in range(S))

    du = np.stack([wts[s] * (r0.markers[s] - tgt[s]) for s in range(S)])
    grad = adjoint_sequence(prob, [gel.X] + r0.x, env.poses, du)
    hs = [env.E * 1e-6, env.nu * 1e-6, 1e-6] + [1e-6] * 6
    fd = np.zeros(N_THETA)
    for i, h in enumerate(hs):
        def off(sgn):
            v = np.zeros(N_THETA)
            v[i] = sgn * h
            return (v[0], v[1], v[2], v[3:6], v[6:9])
        fd[i] = (loss(off(+1)) - loss(off(-1))) / (2 * h)
    scale = np.abs(fd).max()
    for i in range(N_THETA):
        assert abs(grad[i] - fd[i]) <= 1e-4 * max(abs(fd[i]), 1e-3 * scale), (i, grad[i], fd[i])
    # the lag matters here: dropping the carry changes the answer
    assert np.abs(fd[2]) > 1e-3 * scale
