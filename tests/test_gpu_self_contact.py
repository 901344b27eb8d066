"""Gel self-contact on the GPU against the oracle with the same option, on the
two-block scene (two gel blocks 0.08 mm apart, a small sphere pressing the
first next to the gap and sliding it towards the second): one evaluation with
self-contact pairs active, a friction sequence against the oracle's Newton
minimiser, and the sequence adjoint at the GPU's own states. The coarse list's
margin is widened to 16 dhat so that the primitives of both facing walls lie
in the region where the library searches self-contact pairs."""

import os

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_28475_amd import t2r
    return t2r


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda:0")


def _sim(t2r, w, **opts):
    from paper_2603_28475_amd.sim import Sim
    return Sim.from_workload(w, t2r.default_opts(self_contact=1, outer_radius=16.0, **opts))


def _oracle(w, env):
    from oracle.sim import build
    return build(w.meshes[env.mesh], w.indenters[env.indenter], env, self_contact=True)


def _scene(**kw):
    from scenes.configs import self_contact_press
    return self_contact_press(depth=0.3, xy=(-0.45, 0.0), **kw)


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def test_eval_with_self_contact_matches_oracle():
    """The first block's upper wall pushed to within dhat of the second's, plus
    a small random perturbation; the sphere hovers above the gap."""
    t2r = _gpu()
    from oracle.problem import GEE, GVF
    w = _scene(mu_f=0.0)
    env = w.envs[0]
    gel, _, prob = _oracle(w, env)
    x = gel.X.copy()
    nA = gel.n_v // 2
    xa = x[:nA]
    push = 0.035 * np.clip(1.0 - (xa[:, 0].max() - xa[:, 0]) / 0.5, 0.0, 1.0) * (xa[:, 2] / xa[:, 2].max())
    free = ~gel.fixed.astype(bool)
    x[:nA, 0] += push * free[:nA]
    rng = np.random.default_rng(3)
    x += 2e-3 * rng.standard_normal(x.shape) * free[:, None]
    p = rng.standard_normal(x.shape) * free[:, None]
    pose = env.poses[0]
    prob.set_pose(pose)
    pairs, _ = prob.active(x)
    n_self = int(np.isin(pairs["kind"], (GVF, GEE)).sum())
    assert n_self > 0
    print(f"two-block squeezed state, {n_self} self-contact pairs active, t2r_eval", flush=True)
    sim = _sim(t2r, w)
    g = torch.zeros(x.shape, dtype=torch.float64, device="cuda:0")
    d = torch.zeros_like(g)
    sc = torch.zeros(8, dtype=torch.float64, device="cuda:0")
    sim.ctx.eval(0, _dev(x), pose, d_p=_dev(p), d_grad=g, d_diag=d, d_scalars=sc)
    torch.cuda.synchronize()
    g, d, sc = g.cpu().numpy(), d.cpu().numpy(), sc.cpu().numpy()
    assert int(sc[3]) == len(pairs["idx"])
    assert sc[0] == pytest.approx(prob.energy(x), rel=1e-12)
    assert _rel(g, prob.gradient(x)) < 1e-11
    assert _rel(d[free], prob.precond_diag(x)[free]) < 1e-11
    assert sc[1] == pytest.approx(prob.curvature(x, p), rel=1e-11)


def _run(t2r, w, record=False, **opts):
    env = w.envs[0]
    S = env.poses.shape[0] - 1
    sim = _sim(t2r, w, **opts)
    if record:
        sim.record(S)
    xs, ms = [], []
    for s in range(1, S + 1):
        m, st = sim.step(env.poses[s][None], want_x=True)
        torch.cuda.synchronize()
        assert int(st.cpu()[0]) & 1, (s, sim.stats()[0])
        xs.append(sim.x.cpu().numpy().copy())
        ms.append(m.cpu().numpy().copy())
    return sim, xs, ms


def test_self_contact_friction_sequence_matches_newton_oracle():
    """Three press steps and three sliding steps towards the second block with
    friction 0.8, against the oracle's Newton minimiser with self-contact (stored
    by tests/golden/make_golden.py); self-contact pairs are active at every step."""
    t2r = _gpu()
    w = _scene(mu_f=0.8, shear=(0.25, 0.0), n_shear=3)
    gold = np.load(os.path.join(HERE, "golden", "self_contact_friction_newton.npz"))
    assert np.all(gold["n_self"] > 0)
    print("two-block friction sequence with self-contact", flush=True)
    _, xs, ms = _run(t2r, w, tol=1e-10, substep_tol=1e-8, max_iters=400000)
    for s in range(len(xs)):
        assert np.abs(xs[s] - gold["x"][s]).max() <= 1e-6, s
        assert np.abs(ms[s] - gold["markers"][s]).max() <= 1e-6, s


@pytest.mark.parametrize("mollify", [0, 1])
def test_backward_sequence_with_self_contact_matches_oracle_adjoint(mollify):
    """With and without the edge-edge mollifier (the facing walls' edge pairs
    are nearly parallel, so the mollified Hessian terms of gel-gel edge pairs
    enter the adjoint's products)."""
    t2r = _gpu()
    from oracle.adjoint import adjoint_sequence
    from oracle.sim import build
    w = _scene(mu_f=0.8, shear=(0.25, 0.0), n_shear=3)
    env = w.envs[0]
    print(f"two-block friction sequence with self-contact (mollifier {mollify}), backward_sequence vs oracle",
          flush=True)
    sim, xs, ms = _run(t2r, w, record=True, tol=1e-11, substep_tol=1e-11, max_iters=400000,
                       ee_mollifier=mollify)
    rng = np.random.default_rng(6)
    S = len(ms)
    du = np.zeros((S,) + ms[0].shape)
    du[2] = 0.5 * (ms[2] - 0.02 * rng.standard_normal(ms[2].shape))
    du[S - 1] = ms[S - 1] - 0.02 * rng.standard_normal(ms[S - 1].shape)
    g = sim.backward_sequence(du)
    torch.cuda.synchronize()
    st = sim.stats()[0]
    assert st["status"] & 1 and st["residual"] <= 1e-10, st
    gel, _, prob = build(w.meshes[env.mesh], w.indenters[env.indenter], env, self_contact=True,
                         ee_mollifier=bool(mollify))
    ref = adjoint_sequence(prob, [gel.X] + xs, env.poses, du)
    got = g.cpu().numpy()[0]
    scale = np.abs(ref).max()
    assert np.all(np.abs(got - ref) <= 1e-6 * np.maximum(np.abs(ref), 1e-3 * scale)), (got, ref)


def test_eval_with_self_contact_and_edge_mollifier_matches_oracle():
    """Both options on at a squeezed state whose facing walls have nearly
    parallel gel edges: mollified gel-gel edge pairs (threshold from both gel
    edges' rest lengths) against the oracle with the same options."""
    t2r = _gpu()
    from oracle.barrier import EDGE_MOLLIFIER_REL, edge_cross_derivatives
    from oracle.problem import GEE
    from oracle.sim import build
    from paper_2603_28475_amd.sim import Sim
    w = _scene(mu_f=0.0)
    env = w.envs[0]
    gel, _, prob = build(w.meshes[env.mesh], w.indenters[env.indenter], env, self_contact=True,
                         ee_mollifier=True)
    x = gel.X.copy()
    nA = gel.n_v // 2
    xa = x[:nA]
    push = 0.035 * np.clip(1.0 - (xa[:, 0].max() - xa[:, 0]) / 0.5, 0.0, 1.0) * (xa[:, 2] / xa[:, 2].max())
    free = ~gel.fixed.astype(bool)
    x[:nA, 0] += push * free[:nA]
    rng = np.random.default_rng(8)
    x += 2e-4 * rng.standard_normal(x.shape) * free[:, None]
    p = rng.standard_normal(x.shape) * free[:, None]
    pose = env.poses[0]
    prob.set_pose(pose)
    pairs, res = prob.active(x)
    gee = np.nonzero(pairs["kind"] == GEE)[0]
    idx = pairs["idx"][gee]
    eps = EDGE_MOLLIFIER_REL * np.sum((gel.X[idx[:, 1]] - gel.X[idx[:, 0]]) ** 2, 1) * \
        np.sum((gel.X[idx[:, 3]] - gel.X[idx[:, 2]]) ** 2, 1)
    n_moll = int(np.sum(edge_cross_derivatives(res["Z"][gee])[0] < eps))
    assert n_moll > 0
    print(f"two-block squeezed state, {n_moll} mollified gel-gel edge pairs, t2r_eval", flush=True)
    sim = Sim.from_workload(w, t2r.default_opts(self_contact=1, ee_mollifier=1, outer_radius=16.0))
    g = torch.zeros(x.shape, dtype=torch.float64, device="cuda:0")
    d = torch.zeros_like(g)
    sc = torch.zeros(8, dtype=torch.float64, device="cuda:0")
    sim.ctx.eval(0, _dev(x), pose, d_p=_dev(p), d_grad=g, d_diag=d, d_scalars=sc)
    torch.cuda.synchronize()
    g, d, sc = g.cpu().numpy(), d.cpu().numpy(), sc.cpu().numpy()
    assert int(sc[3]) == len(pairs["idx"])
    assert sc[0] == pytest.approx(prob.energy(x), rel=1e-12)
    assert _rel(g, prob.gradient(x)) < 1e-11
    assert _rel(d[free], prob.precond_diag(x)[free]) < 1e-11
    assert sc[1] == pytest.approx(prob.curvature(x, p), rel=1e-11)
