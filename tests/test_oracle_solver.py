"""Pins for the oracle's step energy and minimiser on tiny scenes: finite
differences of the assembled energy (elastic + barrier + lagged friction),
an independent quasi-Newton minimisation, zero gradient, feasibility, no
interpenetration, path independence, recovery after unloading (the paper's
"recovers original state post-contact", Sec. 5.1) and mirror symmetry."""

import numpy as np
import pytest
from scipy.optimize import minimize

from oracle.geometry import slerp_pose
from oracle.newton import newton_solve
from oracle.pncg import pncg_solve
from oracle.problem import StepProblem
from oracle.sim import build, simulate
from scenes.configs import micro_press


def _scene(**kw):
    w = micro_press(**kw)
    env = w.envs[0]
    return w.meshes[env.mesh], w.indenters[env.indenter], env


@pytest.fixture(scope="module")
def pressed():
    mesh, ind, env = _scene(mesh="micro3", indenter="sphere_small", depth=0.15, n_steps=3)
    res = simulate(mesh, ind, env, mode="newton")
    gel, indg, prob = build(mesh, ind, env)
    prob.set_pose(env.poses[-1])
    return mesh, ind, env, res, prob


@pytest.fixture(scope="module")
def friction_state():
    mesh, ind, env = _scene(mesh="micro3", indenter="sphere_small", depth=0.12, n_steps=2,
                            mu_f=0.5, shear=(0.05, 0.02), n_shear=2)
    res = simulate(mesh, ind, env, mode="newton", n_steps=3)
    gel, indg, prob = build(mesh, ind, env)
    prob.set_lag(res.x[-1], env.poses[3])
    prob.set_pose(env.poses[4])
    return prob, res.x[-1]


def test_zero_gradient_and_feasibility(pressed):
    mesh, ind, env, res, prob = pressed
    x = res.x[-1]
    g = prob.gradient(x)
    assert np.abs(g).max() < 1e-9
    assert prob.feasible(x)
    pairs, geo = prob.active(x)
    assert len(pairs["idx"]) > 0, "the scene must be in contact"
    assert np.all(geo["d"] > 0) and np.all(geo["d"] < prob.dhat)
    _, Eb, _ = prob.energy_parts(x)
    assert Eb > 0


def _seg_tri_intersect(p0, p1, a, b, c):
    e1, e2 = b - a, c - a
    d = p1 - p0
    h = np.cross(d, e2)
    det = e1 @ h
    if abs(det) < 1e-300:
        return False
    f = 1.0 / det
    s = p0 - a
    u = f * (s @ h)
    if u < 0 or u > 1:
        return False
    q = np.cross(s, e1)
    v = f * (d @ q)
    if v < 0 or u + v > 1:
        return False
    t = f * (e2 @ q)
    return 0 <= t <= 1


def test_no_interpenetration(pressed):
    mesh, ind, env, res, prob = pressed
    x = res.x[-1]
    gel = prob.gel
    Y = prob.Yw
    for (i, j) in gel.surf_edges:
        for t in prob.ind.tris:
            assert not _seg_tri_intersect(x[i], x[j], *Y[t])
    for (i, j) in prob.ind.edges:
        for t in gel.boundary_tris_all:
            assert not _seg_tri_intersect(Y[i], Y[j], *x[t])


def test_independent_quasi_newton_agrees(pressed):
    mesh, ind, env, res, prob = pressed
    x_star = res.x[-1]
    free = ~prob.gel.fixed
    rng = np.random.default_rng(3)
    x0 = x_star.copy()
    x0[free] += 2e-4 * rng.standard_normal((free.sum(), 3))
    assert np.isfinite(prob.energy(x0))

    def f(z):
        x = x_star.copy()
        x[free] = z.reshape(-1, 3)
        e = prob.energy(x)
        if not np.isfinite(e):
            return 1e30, np.zeros_like(z)
        return e, prob.gradient(x)[free].ravel()

    # a box of +-0.01 mm keeps every trial point feasible (d_min ~ dhat here)
    z0 = x0[free].ravel()
    r = minimize(f, z0, jac=True, method="L-BFGS-B", bounds=list(zip(z0 - 0.01, z0 + 0.01)),
                 options=dict(ftol=0, gtol=1e-13, maxiter=20000, maxcor=50))
    xs = x_star.copy()
    xs[free] = r.x.reshape(-1, 3)
    # L-BFGS stops at the energy's rounding floor, about 1e-8 mm away
    assert np.abs(xs - x_star).max() < 5e-8
    assert prob.energy(x_star) <= prob.energy(xs) + 1e-15


def test_energy_gradient_hessian_consistent_with_friction(friction_state):
    prob, x = friction_state
    assert prob.lag is not None and len(prob.lag["lam"]) > 0
    rng = np.random.default_rng(5)
    free = np.nonzero(~prob.gel.fixed)[0]
    xr = x.copy()
    xr[free] += 1e-4 * rng.standard_normal((len(free), 3))
    g = prob.gradient(xr)
    _, _, Ef = prob.energy_parts(xr)
    assert Ef > 0
    h = 1e-7
    for v in free[:12]:
        for a in range(3):
            xp, xm = xr.copy(), xr.copy()
            xp[v, a] += h
            xm[v, a] -= h
            fd = (prob.energy(xp) - prob.energy(xm)) / (2 * h)
            assert fd == pytest.approx(g[v, a], rel=2e-5, abs=2e-9)
    # curvature equals the second difference of the energy along a random direction
    p = np.zeros_like(x)
    p[free] = rng.standard_normal((len(free), 3))
    h = 1e-5
    fd2 = (prob.energy(xr + h * p) - 2 * prob.energy(xr) + prob.energy(xr - h * p)) / h ** 2
    assert fd2 == pytest.approx(prob.curvature(xr, p), rel=1e-4)
    # diagonal equals the first difference of the gradient per DOF
    dg = prob.diag(xr)
    h = 1e-7
    for v in free[:10]:
        for a in range(3):
            xp, xm = xr.copy(), xr.copy()
            xp[v, a] += h
            xm[v, a] -= h
            fd = (prob.gradient(xp)[v, a] - prob.gradient(xm)[v, a]) / (2 * h)
            assert fd == pytest.approx(dg[v, a], rel=1e-4, abs=1e-6)


def test_path_independence_without_friction():
    mesh, ind, env = _scene(mesh="micro3", indenter="sphere_small", depth=0.15, n_steps=3)
    r3 = simulate(mesh, ind, env, mode="newton")
    env1 = type(env)(**{**env.__dict__})
    env1.poses = env.poses[[0, 3]]
    r1 = simulate(mesh, ind, env1, mode="newton")
    assert np.abs(r3.x[-1] - r1.x[-1]).max() < 1e-9


def test_recovers_rest_state_after_unloading():
    mesh, ind, env = _scene(mesh="micro3", indenter="sphere_small", depth=0.15, n_steps=2)
    env.poses = np.concatenate([env.poses, env.poses[:1]])  # retract to the start pose
    r = simulate(mesh, ind, env, mode="newton")
    assert np.abs(r.x[1] - mesh.X).max() > 1e-3
    assert np.abs(r.x[-1] - mesh.X).max() < 1e-10


def test_mirror_symmetry_about_the_diagonal():
    # the Kuhn split uses all six axis permutations, so a square gel is invariant
    # under x <-> y; so is an icosphere turned to put a mirror plane on x = y.
    # (A flat plate over the whole top is no good here: its barrier pairs make
    # lateral forces with several equilibria, which break the symmetry.)
    mesh, ind, env = _scene(mesh="micro3", indenter="sphere_sym", depth=0.15, n_steps=2,
                            xy=(0.0, 0.0))
    r = simulate(mesh, ind, env, mode="newton")
    x = r.x[-1]
    X = mesh.X
    swapped = X[:, [1, 0, 2]]
    perm = np.array([np.argmin(np.linalg.norm(X - s, axis=1)) for s in swapped])
    u = x - X
    assert np.abs(u).max() > 1e-3
    assert np.abs(u[perm][:, [1, 0, 2]] - u).max() < 1e-10


def test_pncg_reference_reaches_the_newton_minimiser(pressed):
    mesh, ind, env, res, prob = pressed
    r = simulate(mesh, ind, env, mode="pncg", tol=1e-10)
    assert np.abs(r.x[-1] - res.x[-1]).max() < 1e-8
    assert np.abs(r.markers[-1] - res.markers[-1]).max() < 1e-8


def test_preconditioner_diagonal_clamps_negative_pair_entries():
    """precond_diag is the exact diagonal with each contact pair's contribution
    clamped at zero: equal to diag without contact, never below it, positive on
    the free DOFs, and different from it where a close pair's b' grad^2 d term
    makes the exact entry smaller (edge-edge pairs of a pressed plate)."""
    from oracle.sim import build, simulate
    from scenes.configs import micro_press
    q = np.array([0.99996192, 0.00610865, 0.00436331, 0.0])
    w = micro_press(mesh="micro3", indenter="plate", depth=0.08, n_steps=2, xy=(0.1, -0.05),
                    q=tuple(q / np.linalg.norm(q)))
    env = w.envs[0]
    r = simulate(w.meshes[env.mesh], w.indenters[env.indenter], env, mode="newton", tol=1e-12)
    gel, _, prob = build(w.meshes[env.mesh], w.indenters[env.indenter], env)
    free = ~gel.fixed
    prob.set_pose(env.poses[0])                       # clear of the gel: no pair
    assert np.array_equal(prob.precond_diag(gel.X), prob.diag(gel.X))
    # the pressed state with the plate lowered by 0.7 d_min: every pair much
    # closer than at equilibrium (a state a solve passes through)
    x = r.x[-1]
    prob.set_pose(env.poses[-1])
    pose = env.poses[-1].copy()
    pose[2] -= 0.7 * prob.d_min(x)
    prob.set_pose(pose)
    assert len(prob.active(x)[0]["idx"]) > 0 and prob.d_min(x) > 0.0
    dg, pd = prob.diag(x), prob.precond_diag(x)
    assert np.all(pd >= dg - 1e-12 * np.abs(dg).max())
    assert np.all(pd[free] > 0.0)
    assert np.any(pd[free] > dg[free] + 1e-9 * np.abs(dg).max())   # the clamp binds
    # what is left after removing the elastic part is a sum of clamped pair entries
    el = StepProblem(prob.gel, prob.ind, 1.0, 0.25, 0.0, prob.eps_v, prob.dhat, prob.kappa)
    el.mu, el.lam = prob.mu, prob.lam
    el.set_pose(np.array([0.0, 0.0, 1e3, 1.0, 0.0, 0.0, 0.0]))     # indenter far away
    assert len(el.active(x)[0]["idx"]) == 0
    assert np.all(pd - el.diag(x) >= -1e-12 * np.abs(dg).max())
