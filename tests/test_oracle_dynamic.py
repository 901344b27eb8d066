"""Pins of the oracle's dynamic (implicit-Euler) form: the inertia term
1/2 sum_v m_v / h^2 |x_v - xhat_v|^2 with lumped masses and the inertial
prediction xhat = x^t + h v^t."""

import dataclasses

import numpy as np
import pytest

from oracle.newton import newton_solve
from oracle.sim import build, lumped_mass, simulate
from scenes.configs import micro_press


def _scene():
    return micro_press(mesh="micro3", indenter="sphere_small", depth=0.15, n_steps=3)


def test_lumped_mass_sums_to_the_volume():
    w = _scene()
    env = w.envs[0]
    gel, _, _ = build(w.meshes[env.mesh], w.indenters[env.indenter], env)
    m = lumped_mass(gel)
    assert m.sum() == pytest.approx(gel.vol.sum(), rel=1e-14)
    assert np.all(m > 0)


def test_inertia_derivatives_match_differences():
    w = _scene()
    env = w.envs[0]
    gel, _, prob = build(w.meshes[env.mesh], w.indenters[env.indenter], env)
    prob.set_pose(env.poses[0])                        # clear of the gel: elastic + inertia only
    rng = np.random.default_rng(1)
    free = np.nonzero(~gel.fixed)[0]
    x = gel.X.copy()
    x[free] += 0.01 * rng.standard_normal((len(free), 3))
    wv = rng.uniform(0.5, 2.0, gel.n_v)
    xh = gel.X + 0.02 * rng.standard_normal(gel.X.shape)
    prob.set_inertia(wv, xh)
    g = prob.gradient(x)
    h = 1e-6
    for v in free[:8]:
        for a in range(3):
            xp, xm = x.copy(), x.copy()
            xp[v, a] += h
            xm[v, a] -= h
            fd = (prob.energy(xp) - prob.energy(xm)) / (2 * h)
            assert fd == pytest.approx(g[v, a], rel=1e-6, abs=1e-9)
    # the inertia part of the gradient and diagonal in closed form
    prob2 = build(w.meshes[env.mesh], w.indenters[env.indenter], env)[2]
    prob2.set_pose(env.poses[0])
    gi = g - prob2.gradient(x)
    assert np.allclose(gi[free], (wv[:, None] * (x - xh))[free], rtol=1e-12, atol=1e-14)
    di = prob.diag(x) - prob2.diag(x)
    assert np.allclose(di[free], np.repeat(wv[free, None], 3, axis=1), rtol=1e-12)
    p = np.zeros_like(x)
    p[free] = rng.standard_normal((len(free), 3))
    assert prob.curvature(x, p) - prob2.curvature(x, p) == pytest.approx(
        float(np.sum(wv[free] * np.einsum("nd,nd->n", p[free], p[free]))), rel=1e-10)


def test_prediction_at_the_equilibrium_leaves_it_unmoved():
    """With xhat equal to the quasi-static equilibrium the inertia term's
    gradient vanishes there, so the dynamic minimiser is the same point for any
    mass."""
    w = _scene()
    env = w.envs[0]
    r = simulate(w.meshes[env.mesh], w.indenters[env.indenter], env, mode="newton", tol=1e-12)
    gel, _, prob = build(w.meshes[env.mesh], w.indenters[env.indenter], env)
    prob.set_pose(env.poses[-1])
    g_static = np.abs(prob.gradient(r.x[-1])).max()
    prob.set_inertia(np.full(gel.n_v, 50.0), r.x[-1])
    assert np.abs(prob.gradient(r.x[-1])).max() <= g_static + 1e-15
    rng = np.random.default_rng(4)
    x0 = r.x[-1].copy()
    x0[~gel.fixed] += 2e-4 * rng.standard_normal((int((~gel.fixed).sum()), 3))
    xn, info = newton_solve(prob, x0, tol=1e-12)
    assert info["converged"]
    assert np.abs(xn - r.x[-1]).max() <= 1e-9


def test_long_time_step_reduces_to_quasi_static_and_mass_matters():
    w = _scene()
    env = w.envs[0]
    q = simulate(w.meshes[env.mesh], w.indenters[env.indenter], env, mode="newton", tol=1e-12)
    d_long = simulate(w.meshes[env.mesh], w.indenters[env.indenter], env, mode="newton", tol=1e-12,
                      dynamic=dict(density=1e-9, dt=1e3))
    assert max(np.abs(a - b).max() for a, b in zip(q.markers, d_long.markers)) <= 1e-9
    heavy = simulate(w.meshes[env.mesh], w.indenters[env.indenter], env, mode="newton", tol=1e-12,
                     dynamic=dict(density=1e-3, dt=1e-2))
    assert max(np.abs(a - b).max() for a, b in zip(q.markers, heavy.markers)) >= 1e-4
