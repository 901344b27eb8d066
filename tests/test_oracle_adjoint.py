"""Pins of the oracle adjoint (marker-loss gradients at a frictionless
equilibrium) against central finite differences of the whole forward
simulation: Newton to 1e-12 mm at theta +- h for every parameter."""

import dataclasses

import numpy as np
import pytest

from oracle.adjoint import adjoint_gradient, lame_partials, marker_vjp, offset_pose
from oracle.sim import build, simulate
from scenes.configs import micro_press


def _loss_and_state(w, env, theta_off, u_target):
    dE, dnu, dmu, dt, dw = theta_off
    e = dataclasses.replace(env, E=env.E + dE, nu=env.nu + dnu, mu_f=env.mu_f + dmu,
                            poses=np.stack([offset_pose(p, dt, dw) for p in env.poses]))
    r = simulate(w.meshes[e.mesh], w.indenters[e.indenter], e, mode="newton", tol=1e-12)
    u = r.markers[-1]
    return 0.5 * float(np.sum((u - u_target) ** 2)), r


def test_lame_partials_match_differences():
    E, nu, h = 0.3, 0.45, 1e-7
    def lame(E, nu):
        return E / (2 * (1 + nu)), E * nu / ((1 + nu) * (1 - 2 * nu))
    dmu_dE, dlam_dE, dmu_dnu, dlam_dnu = lame_partials(E, nu)
    fd_E = (np.array(lame(E + h, nu)) - np.array(lame(E - h, nu))) / (2 * h)
    fd_nu = (np.array(lame(E, nu + h)) - np.array(lame(E, nu - h))) / (2 * h)
    assert np.allclose([dmu_dE, dlam_dE], fd_E, rtol=1e-7)
    assert np.allclose([dmu_dnu, dlam_dnu], fd_nu, rtol=1e-7)


def test_marker_vjp_is_the_transpose_of_the_marker_map():
    w = micro_press(mesh="micro3")
    env = w.envs[0]
    gel, _, _ = build(w.meshes[env.mesh], w.indenters[env.indenter], env)
    rng = np.random.default_rng(3)
    dx = rng.standard_normal((gel.n_v, 3))
    du = rng.standard_normal((len(gel.marker_w), 3))
    lhs = np.sum(du * (gel.markers(gel.X + dx)))
    rhs = np.sum(marker_vjp(gel, du) * dx)
    assert lhs == pytest.approx(rhs, rel=1e-12)


@pytest.mark.slow
def test_adjoint_gradient_matches_central_differences():
    w = micro_press(mesh="micro3", indenter="sphere_small", depth=0.15, n_steps=3, xy=(0.12, -0.07),
                    q=(0.9990482, 0.0, 0.0436194, 0.0))
    env = w.envs[0]
    rng = np.random.default_rng(11)
    n_m = len(w.meshes[env.mesh].markers)
    u_target = 0.02 * rng.standard_normal((n_m, 3))
    zero = (0.0, 0.0, 0.0, np.zeros(3), np.zeros(3))
    L0, r0 = _loss_and_state(w, env, zero, u_target)
    gel, ind, prob = build(w.meshes[env.mesh], w.indenters[env.indenter], env)
    prob.set_pose(env.poses[-1])
    grad, _ = adjoint_gradient(prob, r0.x[-1], r0.markers[-1] - u_target,
                               x_prev=r0.x[-2], pose_prev=env.poses[-2])
    steps = [env.E * 1e-6, env.nu * 1e-6, 1e-6] + [1e-6] * 6
    fd = np.zeros(9)
    for i, h in enumerate(steps):
        def off(sgn):
            v = np.zeros(9)
            v[i] = sgn * h
            return (v[0], v[1], v[2], v[3:6], v[6:9])
        Lp, _ = _loss_and_state(w, env, off(+1), u_target)
        Lm, _ = _loss_and_state(w, env, off(-1), u_target)
        fd[i] = (Lp - Lm) / (2 * h)
    scale = np.abs(fd).max()
    for i in range(9):
        assert abs(grad[i] - fd[i]) <= 1e-4 * max(abs(fd[i]), 1e-3 * scale), (i, grad[i], fd[i])
