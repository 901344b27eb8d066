"""Pins of the oracle's optional gel self-contact (barriers between gel surface
primitives that share no vertex): the candidate set against an all-pairs loop
with exact distances, the energy's gradient and Hessian against differences
with self pairs active, the conservative step bound with both sides moving, and
the scene itself: with the option the two blocks stay apart under the load
that makes them overlap without it."""

import itertools

import numpy as np
import pytest

from oracle.ccd import ccd_step
from oracle.distance import edge_edge, point_triangle
from oracle.problem import GEE, GVF
from oracle.sim import build, simulate
from scenes.configs import self_contact_press


def _scene(self_contact=True):
    w = self_contact_press(depth=0.3, xy=(-0.45, 0.0), mu_f=0.0)
    env = w.envs[0]
    gel, ind, prob = build(w.meshes["two_block"], w.indenters["sphere_small"], env, self_contact=self_contact)
    return w, env, gel, prob


def _squeezed(gel, amount=0.035):
    """Rest positions with the first block's upper right wall pushed towards the
    second block by up to `amount` mm (so the gap narrows below dhat there)."""
    x = gel.X.copy()
    nA = gel.n_v // 2
    xa = x[:nA]
    wall = xa[:, 0].max()
    push = amount * np.clip(1.0 - (wall - xa[:, 0]) / 0.5, 0.0, 1.0) * (xa[:, 2] / xa[:, 2].max())
    x[:nA, 0] += push * (~gel.fixed[:nA])
    return x


def test_self_contact_candidates_equal_an_all_pairs_loop():
    w, env, gel, prob = _scene()
    prob.set_pose(env.poses[0])
    x = _squeezed(gel)
    thr = 0.06
    pairs = prob.candidates(x, thr)
    res = prob.pair_geometry(x, pairs)
    got = {(int(k), tuple(int(v) for v in i)): d for k, i, d in zip(pairs["kind"], pairs["idx"], res["d"])
           if k in (GVF, GEE) and d < thr}
    ref = {}
    for v in gel.surf_verts:
        for t in gel.surf_tris:
            if v in t:
                continue
            d = point_triangle(x[v][None], x[t[0]][None], x[t[1]][None], x[t[2]][None])["d"][0]
            if d < thr:
                ref[(GVF, (int(v), int(t[0]), int(t[1]), int(t[2])))] = d
    for i, j in itertools.combinations(range(len(gel.surf_edges)), 2):
        a, b = gel.surf_edges[i], gel.surf_edges[j]
        if len(set(a.tolist()) & set(b.tolist())):
            continue
        d = edge_edge(x[a[0]][None], x[a[1]][None], x[b[0]][None], x[b[1]][None])["d"][0]
        if d < thr:
            ref[(GEE, (int(a[0]), int(a[1]), int(b[0]), int(b[1])))] = d
    assert len(ref) > 0 and set(got) == set(ref)
    assert max(abs(got[k] - ref[k]) for k in ref) <= 1e-15


def test_self_contact_gradient_and_hessian_match_differences():
    """At a squeezed state with a small random perturbation: facing walls of
    the structured blocks have parallel edges, where the edge-edge distance is
    not differentiable; the perturbation moves the state off that set."""
    w, env, gel, prob = _scene()
    prob.set_pose(env.poses[0])
    rng = np.random.default_rng(3)
    x = _squeezed(gel) + 2e-3 * rng.standard_normal(gel.X.shape) * (~gel.fixed.astype(bool))[:, None]
    pairs, res = prob.active(x)
    assert np.any(np.isin(pairs["kind"], (GVF, GEE)))
    g = prob.gradient(x).ravel()
    H = prob.hessian(x, project=False).tocsr()
    free = np.repeat(~gel.fixed.astype(bool), 3)
    # the active self pairs' vertices, plus a few others
    act = np.unique(pairs["idx"][np.isin(pairs["kind"], (GVF, GEE))])
    dofs = [3 * v + c for v in act[:8] for c in range(3) if free[3 * v + c]]
    dofs += list(rng.choice(np.nonzero(free)[0], 6, replace=False))
    h = 1e-7
    for i in dofs:
        e = np.zeros(x.size)
        e[i] = h
        xp, xm = x + e.reshape(x.shape), x - e.reshape(x.shape)
        fd = (prob.energy(xp) - prob.energy(xm)) / (2 * h)
        assert fd == pytest.approx(g[i], rel=1e-5, abs=1e-7)
        hd = (prob.gradient(xp).ravel() - prob.gradient(xm).ravel()) / (2 * h)
        row = H.getrow(i).toarray().ravel()
        assert np.allclose(row[free], hd[free], rtol=1e-4, atol=1e-4 * np.abs(row).max())


def test_conservative_step_keeps_self_pairs_apart_when_both_sides_move():
    """Two gel walls moving towards each other at equal speed: the step bound
    stops them with each self pair at >= 10% of its gap (the rate is the sum of
    the two sides' speeds, not the larger one)."""
    w, env, gel, prob = _scene()
    prob.set_pose(env.poses[0])
    x = gel.X.copy()
    nA = gel.n_v // 2
    dx = np.zeros_like(x)
    free = ~gel.fixed.astype(bool)
    dx[:nA][free[:nA], 0] = 1.0
    dx[nA:][free[nA:], 0] = -1.0
    t = ccd_step(prob, x, dx, 0.2)
    xt = x + t * dx
    pairs = prob.candidates(xt, 0.2)
    sel = np.isin(pairs["kind"], (GVF, GEE))
    d = prob.pair_geometry(xt, {"idx": pairs["idx"][sel], "kind": pairs["kind"][sel]})["d"]
    assert 0.0 < t < 0.04                       # the walls start 0.08 mm apart
    assert d.min() >= 0.1 * 0.08 * 0.999


def test_self_contact_keeps_the_blocks_apart_where_plain_contact_lets_them_overlap():
    """Press and a sliding push towards the second block (the stored scene's
    load): with self-contact every gel surface pair stays at a positive distance
    and some are active; without it the first block's wall passes into the
    second block's."""
    w = self_contact_press(depth=0.3, xy=(-0.45, 0.0), mu_f=0.8, shear=(0.25, 0.0), n_shear=3)
    env = w.envs[0]
    g = w.meshes["two_block"]
    nA = g.n_verts // 2
    x_plain = simulate(g, w.indenters["sphere_small"], env, mode="newton", n_steps=4).x[-1]
    xb_min = g.X[nA:, 0].min()
    top = g.X[:nA, 2] > g.thickness - 1e-9
    assert x_plain[:nA][top, 0].max() > xb_min + 0.01     # overlap without self-contact
    r = simulate(g, w.indenters["sphere_small"], env, mode="newton", n_steps=4, self_contact=True)
    gel, ind, prob = build(g, w.indenters["sphere_small"], env, self_contact=True)
    prob.set_pose(env.poses[4])
    pairs = prob.candidates(r.x[-1], 0.3)
    sel = np.isin(pairs["kind"], (GVF, GEE))
    d = prob.pair_geometry(r.x[-1], {"idx": pairs["idx"][sel], "kind": pairs["kind"][sel]})["d"]
    assert d.min() > 0.0 and np.sum(d < prob.dhat) > 0


def test_self_contact_with_the_edge_mollifier_matches_differences():
    """Both options on: the facing walls' parallel gel edges are mollified
    edge-edge pairs (the threshold from both gel edges' rest lengths); the
    energy's gradient and Hessian still match differences."""
    from oracle.barrier import EDGE_MOLLIFIER_REL, edge_cross_derivatives
    w = self_contact_press(depth=0.3, xy=(-0.45, 0.0), mu_f=0.0)
    env = w.envs[0]
    gel, ind, prob = build(w.meshes["two_block"], w.indenters["sphere_small"], env, self_contact=True,
                           ee_mollifier=True)
    plain = build(w.meshes["two_block"], w.indenters["sphere_small"], env, self_contact=True)[2]
    for q in (prob, plain):
        q.set_pose(env.poses[0])
    rng = np.random.default_rng(8)
    x = _squeezed(gel) + 2e-4 * rng.standard_normal(gel.X.shape) * (~gel.fixed.astype(bool))[:, None]
    pairs, res = prob.active(x)
    gee = np.nonzero(pairs["kind"] == GEE)[0]
    idx = pairs["idx"][gee]
    eps = EDGE_MOLLIFIER_REL * np.sum((gel.X[idx[:, 1]] - gel.X[idx[:, 0]]) ** 2, 1) * \
        np.sum((gel.X[idx[:, 3]] - gel.X[idx[:, 2]]) ** 2, 1)
    assert np.sum(edge_cross_derivatives(res["Z"][gee])[0] < eps) > 0
    assert prob.energy(x) < plain.energy(x)
    g = prob.gradient(x).ravel()
    free = np.repeat(~gel.fixed.astype(bool), 3)
    act = np.unique(idx)
    h = 1e-7
    for i in [3 * v + c for v in act[:6] for c in range(3) if free[3 * v + c]]:
        e = np.zeros(x.size)
        e[i] = h
        xp, xm = x + e.reshape(x.shape), x - e.reshape(x.shape)
        assert (prob.energy(xp) - prob.energy(xm)) / (2 * h) == pytest.approx(g[i], rel=1e-5, abs=1e-7)
