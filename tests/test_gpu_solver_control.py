"""GPU checks through the C ABI of the solver's control paths against the FP64
oracle: the mixed-precision kernel terms, the PNCG iterates one iteration at a
time, every per-env outcome bit a caller can force, and the HIP-graph step
(including a re-capture after the layout changed) against the oracle's Newton
path.
"""

import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_28475_amd import t2r
    return t2r


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda:0")


def _build(t2r, workload, envs=None, stream=None, **opts):
    from paper_2603_28475_amd.sim import Sim
    return Sim.from_workload(workload, t2r.default_opts(**opts), envs=envs, stream=stream)


def _oracle_problem(workload, env):
    from oracle.sim import build
    return build(workload.meshes[env.mesh], workload.indenters[env.indenter], env)


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _state(sim):
    """(positions (n_v, 3), pose (7,)) of the single env of `sim`."""
    st = torch.empty(sim.ctx.state_size(), dtype=torch.float64, device="cuda:0")
    sim.ctx.get_state(st)
    torch.cuda.synchronize()
    a = st.cpu().numpy()
    nv = sim.n_v[0]
    return a[:3 * nv].reshape(nv, 3), a[3 * nv:3 * nv + 7]


def _set_state(sim, x, pose):
    sim.ctx.set_state(_dev(np.concatenate([np.asarray(x).ravel(), np.asarray(pose)])))
    torch.cuda.synchronize()


def _eval(t2r, w, x, pose, p, precision):
    sim = _build(t2r, w, precision=precision)
    nv = x.shape[0]
    g = torch.zeros((nv, 3), dtype=torch.float64, device="cuda:0")
    d = torch.zeros_like(g)
    sc = torch.zeros(8, dtype=torch.float64, device="cuda:0")
    sim.ctx.eval(0, _dev(x), pose, d_p=_dev(p), d_grad=g, d_diag=d, d_scalars=sc)
    torch.cuda.synchronize()
    return g.cpu().numpy(), d.cpu().numpy(), sc.cpu().numpy()


def test_eval_mixed_precision_matches_oracle():
    """precision = 1 (rest-shape inverses and volumes stored as FP32; element
    gradient, diagonal and curvature in FP32; F, J, ln J and the energy in FP64
    from the FP32 rest data; distances, barrier and sums FP64) against the FP64
    oracle at perturbed states of the sphere press and of the peg hovering with
    every pair kind active: energy within 1e-6 relative (the FP32 rest data
    carry a relative rounding of 2^-24 = 6e-8 per entry, which enters the
    strain energy through F), gradient, diagonal and p^T H p within 1e-5
    relative (FP32 rounding of the element terms, about 1e-7 per term, summed
    over up to 24 tets per vertex)."""
    t2r = _gpu()
    from scenes.configs import DHAT, peg_press_484v, pose_at_depth, sphere_press_484v
    gold = np.load(os.path.join(HERE, "golden", "sphere_press_484v_newton.npz"))
    rng = np.random.default_rng(17)
    w1 = sphere_press_484v()
    g = w1.meshes["c1"]
    free = g.fixed == 0
    x = gold["x"][6].copy()
    x[free] += 2e-4 * rng.standard_normal((free.sum(), 3))
    w2 = peg_press_484v(mu_f=0.0)
    ind = w2.indenters["peg4"]
    p0 = w2.envs[0].poses[0]
    hover = pose_at_depth(ind, p0[3:], p0[:2], -0.3 * DHAT, g.thickness)
    x2 = g.X.copy()
    x2[free] += 2e-4 * rng.standard_normal((free.sum(), 3))
    for w, xs, pose in ((w1, x, gold["poses"][7]), (w2, x2, hover)):
        p = np.zeros_like(xs)
        p[free] = rng.standard_normal((free.sum(), 3))
        gm, dm, scm = _eval(t2r, w, xs, pose, p, precision=1)
        _, _, prob = _oracle_problem(w, w.envs[0])
        prob.set_pose(pose)
        assert scm[4] == 1.0 and int(scm[3]) > 0
        assert scm[0] == pytest.approx(prob.energy(xs), rel=1e-6)
        assert _rel(gm, prob.gradient(xs)) < 1e-5
        assert _rel(dm[free], prob.precond_diag(xs)[free]) < 1e-5
        assert scm[1] == pytest.approx(prob.curvature(xs, p), rel=1e-5)


def _squashed_state(g, j_target=1e-9):
    """Rest positions with one free top vertex pushed straight down until the
    first of its tets reaches volume ratio J = j_target (bisection on the CPU),
    every tet still positive."""
    from oracle import elastic
    Dm_inv = np.linalg.inv(np.stack([(g.X[t[1:]] - g.X[t[0]]).T for t in g.tets]))
    top = np.flatnonzero((g.X[:, 2] == g.X[:, 2].max()) & (g.fixed == 0))
    v = top[np.argmin(np.abs(g.X[top, 0] - 1.0) + np.abs(g.X[top, 1] + 1.0))]
    lo, hi = 0.0, float(g.X[:, 2].max())

    def jmin(dz):
        x = g.X.copy()
        x[v, 2] -= dz
        return float(np.linalg.det(elastic.deformation_gradients(x, g.tets, Dm_inv)).min()), x

    for _ in range(200):
        mid = 0.5 * (lo + hi)
        j, _ = jmin(mid)
        if j > j_target:
            lo = mid
        else:
            hi = mid
    j, x = jmin(lo)
    assert 0.0 < j < 10 * j_target
    return x, j


def test_eval_mixed_precision_with_a_squashed_tet_matches_oracle():
    """A tet squashed to J ~ 1e-9 (a free top vertex pushed into the element
    layer below it): the mixed path computes that tet's gradient, diagonal and
    curvature in FP64 (in FP32 the cofactors lose the sign of det F as J -> 0),
    so the bars of the mixed path still hold: energy 1e-6, gradient, diagonal
    and p^T H p 1e-5 relative to the FP64 oracle."""
    t2r = _gpu()
    from scenes.configs import sphere_press_484v
    w = sphere_press_484v()
    g = w.meshes["c1"]
    free = g.fixed == 0
    x, j = _squashed_state(g)
    rng = np.random.default_rng(29)
    p = np.zeros_like(x)
    p[free] = rng.standard_normal((free.sum(), 3))
    pose = w.envs[0].poses[0]
    gm, dm, scm = _eval(t2r, w, x, pose, p, precision=1)
    _, _, prob = _oracle_problem(w, w.envs[0])
    prob.set_pose(pose)
    assert scm[4] == 1.0
    assert scm[0] == pytest.approx(prob.energy(x), rel=1e-6)
    # the squashed tet's vertices (gradient ~1e10) and the rest, each to its own scale
    from oracle import elastic
    J = np.linalg.det(elastic.deformation_gradients(x, prob.gel.tets, prob.gel.Dm_inv))
    sq = np.zeros(len(x), dtype=bool)
    sq[prob.gel.tets[J < 0.1].ravel()] = True
    go, do = prob.gradient(x), prob.precond_diag(x)
    for mask in (sq & free, ~sq & free):
        assert mask.any()
        assert _rel(gm[mask], go[mask]) < 1e-5
        assert _rel(dm[mask], do[mask]) < 1e-5
    assert scm[1] == pytest.approx(prob.curvature(x, p), rel=1e-5)


def test_pncg_iterates_match_oracle_reference_one_iteration_at_a_time():
    """From a perturbed equilibrium of the sphere press, with the indenter held at
    its pose (one solve, no continuation), max_iters = k stops the GPU solve after
    k PNCG iterations; its positions equal the oracle's PNCG reference after k
    iterations from the same start (same preconditioner, Dai-Kou beta, analytic
    and CCD step bounds, Armijo halving) within 1e-10 relative to the
    displacement from the start, for k = 1..4; the halving and restart counts
    are equal too. (The per-iteration scalars are sums over about 1,400 DOFs
    accumulated in a different order on the two sides, about 1e-13 relative
    each, and the recurrence carries them on: after four iterations the two
    agree to about 1e-12; a wrong step length or beta moves the iterate by
    1e-3 or more.)"""
    t2r = _gpu()
    from oracle.pncg import pncg_solve
    from scenes.configs import sphere_press_484v
    w = sphere_press_484v()
    gold = np.load(os.path.join(HERE, "golden", "sphere_press_484v_newton.npz"))
    free = w.meshes["c1"].fixed == 0
    rng = np.random.default_rng(23)
    pose = gold["poses"][5]
    x0 = gold["x"][4].copy()
    x0[free] += 1e-3 * rng.standard_normal((free.sum(), 3))
    _, _, prob = _oracle_problem(w, w.envs[0])
    prob.set_pose(pose)
    assert np.isfinite(prob.energy(x0))
    for k in (1, 2, 3, 4):
        sim = _build(t2r, w, tol=1e-12, substep_tol=1e-12, max_iters=k, warm_start=0)
        _set_state(sim, x0, pose)
        _, status = sim.step(pose[None])
        torch.cuda.synchronize()
        st = int(status.cpu()[0])
        assert st & t2r.ENV_MAXITER and not st & t2r.ENV_CONVERGED, st
        xg, qg = _state(sim)
        stats = sim.stats()[0]
        assert stats["iters"] == k and stats["substeps"] == 1
        rec = []
        xo, info = pncg_solve(prob, x0, tol=1e-12, max_iters=k, record=rec)
        assert info["iters"] == k and len(rec) == k
        assert _rel(xg - x0, xo - x0) < 1e-10, k
        assert stats["halvings"] == info["halvings"] and stats["restarts"] == info["restarts"]
        np.testing.assert_array_equal(qg, pose)


def test_max_iters_reports_maxiter_and_keeps_the_state():
    """max_iters = 1 through three press steps: every solve stops after one
    iteration; the steps report T2R_ENV_MAXITER without T2R_ENV_CONVERGED, the
    env keeps the state it reached (not rolled back: the gel moved), and that
    state is feasible at the env's pose (the target pose, or the continuation
    pose reached if the substeps ran out first)."""
    t2r = _gpu()
    from scenes.configs import sphere_press_484v
    w = sphere_press_484v()
    env = w.envs[0]
    sim = _build(t2r, w, tol=1e-10, substep_tol=1e-10, max_iters=1, max_substeps=200)
    seq = np.ascontiguousarray(env.poses[1:4][:, None, :])
    _, status = sim.step_sequence(seq)
    torch.cuda.synchronize()
    st = int(status.cpu().numpy()[-1, 0])
    assert st & t2r.ENV_MAXITER and not st & t2r.ENV_CONVERGED, st
    assert not st & (t2r.ENV_INFEASIBLE | t2r.ENV_PAIR_OVERFLOW | t2r.ENV_BUDGET), st
    x, q = _state(sim)
    if not st & t2r.ENV_SUBSTEPS:
        np.testing.assert_array_equal(q, env.poses[3])
    _, _, prob = _oracle_problem(w, env)
    prob.set_pose(q)
    assert np.isfinite(prob.energy(x)) and prob.d_min(x) > 0.0
    assert np.abs(x - w.meshes["c1"].X).max() > 1e-4  # it moved


def test_infeasible_start_reports_infeasible_and_rolls_back():
    """A start state with inverted tets (a free top vertex pushed 1 mm down,
    through the element layer below it): the load step reports
    T2R_ENV_INFEASIBLE, and positions and pose stay as they were."""
    t2r = _gpu()
    from scenes.configs import sphere_press_484v
    w = sphere_press_484v()
    env = w.envs[0]
    g = w.meshes["c1"]
    x0 = g.X.copy()
    top = np.flatnonzero((g.X[:, 2] == g.X[:, 2].max()) & (g.fixed == 0))
    v = top[np.argmax(np.abs(g.X[top, 0]) + np.abs(g.X[top, 1]))]  # a corner, far from the sphere
    x0[v, 2] -= 1.0
    _, _, prob = _oracle_problem(w, env)
    prob.set_pose(env.poses[0])
    assert not np.isfinite(prob.energy(x0))  # J <= 0 somewhere
    sim = _build(t2r, w, tol=1e-8)
    _set_state(sim, x0, env.poses[0])
    _, status = sim.step(env.poses[1][None])
    torch.cuda.synchronize()
    st = int(status.cpu()[0])
    assert st & t2r.ENV_INFEASIBLE and not st & t2r.ENV_CONVERGED, st
    x, q = _state(sim)
    np.testing.assert_array_equal(x, x0)
    np.testing.assert_array_equal(q, env.poses[0])


def test_max_substeps_reports_substeps_and_keeps_the_pose_reached():
    """max_substeps = 1 on a load step whose continuation needs several advances
    (no warm start): the step reports T2R_ENV_SUBSTEPS without
    T2R_ENV_CONVERGED; the env keeps the equilibrium of the intermediate pose it
    reached, which becomes its pose (strictly between the start and the target
    along the press), and the oracle's Newton started there does not move it."""
    t2r = _gpu()
    from oracle.newton import newton_solve
    from scenes.configs import sphere_press_484v
    w = sphere_press_484v(n_steps=2)  # 0.3 mm per load step
    env = w.envs[0]
    sim = _build(t2r, w, tol=1e-10, substep_tol=1e-10, max_substeps=1, warm_start=0)
    _, status = sim.step(env.poses[1][None])
    torch.cuda.synchronize()
    st = int(status.cpu()[0])
    assert st & t2r.ENV_SUBSTEPS and not st & t2r.ENV_CONVERGED, st
    assert sim.stats()[0]["substeps"] == 1
    x, q = _state(sim)
    z0, z1 = env.poses[0][2], env.poses[1][2]
    assert min(z0, z1) < q[2] < max(z0, z1)
    np.testing.assert_allclose(q[:2], env.poses[1][:2], atol=1e-12)
    _, _, prob = _oracle_problem(w, env)
    prob.set_pose(q)
    xn, info = newton_solve(prob, x, tol=1e-12)
    assert info["converged"] and np.abs(xn - x).max() <= 1e-6


def test_evaluation_budget_stops_the_env_and_rolls_back():
    """max_evals = 5 evaluation passes per env and launch: a press that needs
    more stops with T2R_ENV_BUDGET and T2R_ENV_MAXITER, is rolled back to its
    previous state and pose, and later load steps of the same launch stop at
    once; the env's evaluation count stays within the budget plus one line
    search. A budget that suffices changes nothing."""
    t2r = _gpu()
    from scenes.configs import sphere_press_484v
    w = sphere_press_484v()
    env = w.envs[0]
    gold = np.load(os.path.join(HERE, "golden", "sphere_press_484v_newton.npz"))
    sim = _build(t2r, w, tol=1e-10, substep_tol=1e-10, max_evals=5)
    seq = np.ascontiguousarray(env.poses[1:4][:, None, :])
    _, status = sim.step_sequence(seq)
    torch.cuda.synchronize()
    st = status.cpu().numpy()[:, 0]
    assert all(s & t2r.ENV_BUDGET and s & t2r.ENV_MAXITER and not s & t2r.ENV_CONVERGED for s in st), st
    ev = sim.stats()[0]["evals"]
    assert 5 <= ev <= 5 + 32, ev
    x, q = _state(sim)
    np.testing.assert_array_equal(x, w.meshes["c1"].X)
    np.testing.assert_array_equal(q, env.poses[0])
    ok = _build(t2r, w, tol=1e-10, substep_tol=1e-10, max_evals=100000)
    m, status = ok.step_sequence(seq)
    torch.cuda.synchronize()
    assert np.all(status.cpu().numpy() & t2r.ENV_CONVERGED)
    assert np.abs(m.cpu().numpy()[:, :, :] - gold["markers"][:3]).max() <= 1e-6


def test_graph_step_matches_newton_oracle_and_recaptures_after_layout_change():
    """Sim.graph_step (a captured HIP graph replayed per load step, eager library
    calls between replays) through the 10-step sphere press: markers within
    1e-6 mm of the oracle's Newton minimiser at every step. Half way, the pair
    capacity is changed (the library reallocates its lists): the layout
    generation moves and the next graph_step captures again instead of
    replaying launches that point at freed lists. Recording a tape refuses the
    graph step."""
    t2r = _gpu()
    from scenes.configs import sphere_press_484v
    w = sphere_press_484v()
    env = w.envs[0]
    gold = np.load(os.path.join(HERE, "golden", "sphere_press_484v_newton.npz"))
    side = torch.cuda.Stream()
    sim = _build(t2r, w, stream=side, tol=1e-10, substep_tol=1e-10, max_iters=200000)
    gens = []
    for s in range(1, 11):
        if s == 6:
            sim.ctx.set_pair_capacity(2 * sim.ctx.gel_info(0)["pair_capacity"])
        m, st = sim.graph_step(env.poses[s][None])
        side.synchronize()
        gens.append(sim._graph_gen)
        assert len(sim.stats()) == 1  # eager library call between replays
        assert int(st.cpu()[0]) & t2r.ENV_CONVERGED, s
        assert np.abs(m.cpu().numpy() - gold["markers"][s - 1]).max() <= 1e-6, s
    assert len(set(gens[:5])) == 1 and len(set(gens[5:])) == 1 and gens[5] > gens[4]
    sim.record(2)
    with pytest.raises(RuntimeError):
        sim.graph_step(env.poses[10][None])


def test_library_memory_comes_from_torch_caching_allocator():
    """Sim routes the library's device allocations through torch's caching
    allocator (t2r_set_allocator): torch's allocated-bytes counter grows by the
    library's buffers at the first GPU call and drops back when the Sim is
    closed; a Sim with torch_memory=False allocates outside torch and steps to
    the same markers."""
    t2r = _gpu()
    from paper_2603_28475_amd.sim import Sim
    from scenes.configs import peg_batch_5k
    w = peg_batch_5k(n_envs=8, n_steps=2)
    poses = np.stack([e.poses for e in w.envs])
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    sim = Sim.from_workload(w, t2r.default_opts(tol=1e-8, precision=0))
    m, st = sim.step(poses[:, 1])
    torch.cuda.synchronize()
    grown = torch.cuda.memory_allocated() - base
    assert grown > 20e6, grown  # pair lists, friction records, state vectors of 8 envs (about 38 MB)
    assert np.all(st.cpu().numpy() & t2r.ENV_CONVERGED)
    m_torch = m.cpu().numpy().copy()
    sim.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() - base < 5e6  # the Sim's own output tensors remain
    plain = Sim.from_workload(w, t2r.default_opts(tol=1e-8, precision=0), torch_memory=False)
    before = torch.cuda.memory_allocated()
    m2, st2 = plain.step(poses[:, 1])
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() - before < 10e6  # only the outputs are torch's
    assert np.abs(m2.cpu().numpy() - m_torch).max() <= 1e-6
