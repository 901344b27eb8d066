"""Pins of the oracle's lagged friction term and contact enumeration against
physics and brute force, not against the oracle's own formulas.

Friction (Supp. A, eqs. friction_energy and friction_mollifier): with the lag
taken at (x_{s-1}, q_{s-1}), D_s = mu_f sum_k lambda_k f(|T_k Delta_k|), where
Delta_k is the relative tangential displacement of the gel's closest point
with respect to the indenter's since the lag, and f(s) = s beyond eps_v with
f(0) = eps_v / 3. Two rigid cases fix the term completely:
  * gel and indenter translated together: nothing slides, so every Delta_k
    vanishes, D = mu_f sum lambda_k eps_v / 3 and the friction force is zero;
  * the indenter slid by u (|T_k u| >> eps_v) over a frozen gel: every pair is
    in the Coulomb regime, D = mu_f sum lambda_k |T_k u|, and the friction
    force pair k puts on the gel has magnitude mu_f lambda_k and points along
    T_k u (it opposes the gel's slip -u relative to the indenter); reversing
    the slide reverses it.

Contact set (Supp. A, eq. ipc_energy; every gel-surface/indenter pair closer
than dhat, duplicates kept): the oracle's box-filtered enumeration must equal
an all-pairs loop over (surface vertex, indenter triangle), (surface triangle,
indenter vertex) and (surface edge, indenter edge) with exact distances.
"""

import os

import numpy as np
import pytest

from oracle.distance import edge_edge, point_triangle
from oracle.problem import EE, FV, VF
from oracle.sim import build

HERE = os.path.dirname(os.path.abspath(__file__))


def _hover_scene(mu_f=0.5):
    """The slightly tilted flat-ended peg hovering within dhat of the 484-vertex
    gel: VF, FV and EE pairs are all active at rest."""
    from scenes.configs import DHAT, peg_press_484v, pose_at_depth
    w = peg_press_484v(mu_f=mu_f)
    g = w.meshes["c1"]
    ind = w.indenters["peg4"]
    env = w.envs[0]
    p0 = env.poses[0]
    hover = pose_at_depth(ind, p0[3:], p0[:2], -0.3 * DHAT, g.thickness)
    gel, _, prob = build(g, ind, env)
    return gel, prob, gel.X.copy(), hover


def _friction_gradient(prob, x):
    """Gradient of D alone: the full gradient minus the one without the lag."""
    lag = prob.lag
    g_all = prob.gradient(x)
    prob.lag = None
    g_wo = prob.gradient(x)
    prob.lag = lag
    return g_all - g_wo


def _sub_lag(lag, k):
    out = dict(lag)
    for key in ("idx", "a", "b", "n", "lam"):
        out[key] = lag[key][k:k + 1]
    return out


def test_hover_scene_lags_every_pair_kind():
    gel, prob, x0, hover = _hover_scene()
    prob.set_lag(x0, hover)
    prob.set_pose(hover)
    pairs, _ = prob.active(x0)
    kinds = set(np.unique(pairs["kind"]).tolist())
    assert kinds == {VF, FV, EE}
    assert len(prob.lag["lam"]) == len(pairs["idx"]) > 0
    assert np.all(prob.lag["lam"] > 0)


def test_rigid_co_motion_does_not_slide():
    gel, prob, x0, hover = _hover_scene()
    prob.set_lag(x0, hover)
    lam = prob.lag["lam"]
    for u in ([0.03, -0.02, 0.0], [0.0, 0.0, 0.01], [-0.2, 0.1, 0.05]):
        u = np.asarray(u)
        x = x0 + u                     # every gel point moves by u ...
        pose = hover.copy()
        pose[:3] += u                  # ... and so does the indenter
        prob.set_pose(pose)
        _, _, TD, s = prob._friction_terms(x)
        assert np.abs(TD).max() <= 1e-15 * max(1.0, np.abs(x).max())
        _, _, Ef = prob.energy_parts(x)
        assert Ef == pytest.approx(prob.mu_f * lam.sum() * prob.eps_v / 3.0, rel=1e-12)
        gf = _friction_gradient(prob, x)
        # against the force scale of one pair mu_f lambda_k
        assert np.abs(gf).max() <= 1e-9 * prob.mu_f * lam.max()


@pytest.mark.parametrize("u", [(0.02, 0.0, 0.0), (0.012, -0.015, 0.0), (-0.01, 0.02, 0.001)])
def test_slide_past_eps_gives_the_coulomb_force(u):
    gel, prob, x0, hover = _hover_scene()
    prob.set_lag(x0, hover)
    lag = prob.lag
    u = np.asarray(u)
    assert not np.any(gel.fixed[lag["idx"][lag["idx"] < gel.n_v]])  # top-surface pairs only

    def slid(sign):
        pose = hover.copy()
        pose[:3] += sign * u
        prob.set_pose(pose)
        return x0  # frozen gel

    x = slid(+1.0)
    n = lag["n"]
    Tu = u[None, :] - np.einsum("kd,d->k", n, u)[:, None] * n      # T_k u
    tu = np.linalg.norm(Tu, axis=1)
    assert np.all(tu > 5.0 * prob.eps_v)                            # Coulomb regime everywhere
    _, _, TD, s = prob._friction_terms(x)
    assert np.allclose(s, tu, rtol=1e-12)
    _, _, Ef = prob.energy_parts(x)
    assert Ef == pytest.approx(prob.mu_f * np.sum(lag["lam"] * tu), rel=1e-12)

    rng = np.random.default_rng(3)
    picks = []
    n_gel = (lag["idx"] < gel.n_v).sum(axis=1)
    kind_of = np.select([n_gel == 1, n_gel == 3], [VF, FV], EE)
    for kd in (VF, FV, EE):
        ids = np.nonzero(kind_of == kd)[0]
        picks += list(rng.choice(ids, size=min(3, len(ids)), replace=False))
    assert len(picks) >= 3
    for k in picks:
        prob.lag = _sub_lag(lag, k)
        forces = []
        for sign in (+1.0, -1.0):
            xk = slid(sign)
            F = -_friction_gradient(prob, xk).sum(axis=0)   # total force on the gel's points
            forces.append(F)
        prob.lag = lag
        F, Fr = forces
        mag = prob.mu_f * lag["lam"][k]
        assert np.linalg.norm(F) == pytest.approx(mag, rel=1e-10)
        assert float(F @ Tu[k]) / tu[k] == pytest.approx(mag, rel=1e-10)   # along +T_k u
        assert np.allclose(Fr, -F, rtol=0, atol=1e-12 * mag)               # reversed slide


def _brute_force_active(prob, x, Yw, thr):
    """Every (kind, four point ids) with exact distance < thr, by looping over
    all primitive pairs in chunks (no spatial filter of any kind)."""
    gel, ind, nv = prob.gel, prob.ind, prob.nv
    pts = np.concatenate([x, Yw])
    out = {}

    def run(kind, A, B):
        # A: (na, ka) point ids of gel-side/indenter-side primitive, B likewise
        na, nb = len(A), len(B)
        ia, ib = np.meshgrid(np.arange(na), np.arange(nb), indexing="ij")
        ia, ib = ia.ravel(), ib.ravel()
        for s0 in range(0, len(ia), 200000):
            sa, sb = A[ia[s0:s0 + 200000]], B[ib[s0:s0 + 200000]]
            idx = np.concatenate([sa, sb], axis=1)
            Z = pts[idx]
            if kind == EE:
                d = edge_edge(Z[:, 0], Z[:, 1], Z[:, 2], Z[:, 3])["d"]
            else:
                d = point_triangle(Z[:, 0], Z[:, 1], Z[:, 2], Z[:, 3])["d"]
            for j in np.nonzero(d < thr)[0]:
                out[(kind, *map(int, idx[j]))] = float(d[j])

    run(VF, gel.surf_verts[:, None], nv + ind.tris)
    run(FV, nv + np.arange(len(ind.Y))[:, None], gel.surf_tris)
    run(EE, gel.surf_edges, nv + ind.edges)
    return out


def _oracle_active(prob, x):
    pairs, geo = prob.active(x)
    return {(int(k), *map(int, i)): float(d) for k, i, d in zip(pairs["kind"], pairs["idx"], geo["d"])}


@pytest.mark.parametrize("step", [4, 9])
def test_active_set_equals_all_pairs_loop_sphere_press(step):
    from scenes.configs import sphere_press_484v
    gold = np.load(os.path.join(HERE, "golden", "sphere_press_484v_newton.npz"))
    w = sphere_press_484v()
    env = w.envs[0]
    gel, ind, prob = build(w.meshes["c1"], w.indenters["sphere3"], env)
    x, pose = gold["x"][step], gold["poses"][step + 1]
    prob.set_pose(pose)
    got = _oracle_active(prob, x)
    ref = _brute_force_active(prob, x, prob.Yw, prob.dhat)
    assert len(ref) > 0 and len(ref) == int(gold["n_active"][step])
    assert got.keys() == ref.keys()
    assert max(abs(got[k] - ref[k]) for k in ref) <= 1e-15


def test_active_set_and_candidates_equal_all_pairs_loop_every_kind():
    gel, prob, x0, hover = _hover_scene(mu_f=0.0)
    rng = np.random.default_rng(5)
    x = x0.copy()
    x[gel.free] += 2e-4 * rng.standard_normal((gel.free.sum(), 3))
    prob.set_pose(hover)
    got = _oracle_active(prob, x)
    ref = _brute_force_active(prob, x, prob.Yw, prob.dhat)
    assert {k[0] for k in ref} == {VF, FV, EE}
    assert got.keys() == ref.keys()
    assert max(abs(got[k] - ref[k]) for k in ref) <= 1e-15
    # the wider candidate set (CCD uses 2 dhat) holds every pair within its radius
    cand = prob.candidates(x, 2.0 * prob.dhat)
    have = {(int(k), *map(int, i)) for k, i in zip(cand["kind"], cand["idx"])}
    wide = _brute_force_active(prob, x, prob.Yw, 2.0 * prob.dhat)
    assert set(wide) <= have
