"""Deterministic mode and checkpoints on the GPU: one evaluation in
deterministic mode against atomic mode (1e-12) and against itself (bitwise);
a friction sequence repeated in two contexts (bitwise, and at the oracle's
Newton result to 1e-6 mm); resuming from a checkpoint (bitwise); a batched env
against its own single-env launch (bitwise)."""

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


def _sim(t2r, w, envs=None, **opts):
    from paper_2603_28475_amd.sim import Sim
    return Sim.from_workload(w, t2r.default_opts(**opts), envs=envs)


def _eval(t2r, w, x, pose, p, lag, det):
    sim = _sim(t2r, w, deterministic=det)
    nv = x.shape[0]
    g = torch.zeros((nv, 3), dtype=torch.float64, device="cuda:0")
    d = torch.zeros_like(g)
    sc = torch.zeros(8, dtype=torch.float64, device="cuda:0")
    sim.ctx.eval(0, _dev(x), pose, d_p=_dev(p), d_x_lag=_dev(lag[0]), pose_lag=lag[1], d_grad=g, d_diag=d,
                 d_scalars=sc)
    torch.cuda.synchronize()
    return g.cpu().numpy(), d.cpu().numpy(), sc.cpu().numpy()


def test_deterministic_eval_matches_atomic_mode_and_repeats():
    t2r = _gpu()
    from scenes.configs import DHAT, peg_press_484v, pose_at_depth
    w = peg_press_484v(mu_f=0.5)
    g = w.meshes["c1"]
    ind = w.indenters["peg4"]
    p0 = w.envs[0].poses[0]
    hover = pose_at_depth(ind, p0[3:], p0[:2], -0.3 * DHAT, g.thickness)
    rng = np.random.default_rng(4)
    free = g.fixed == 0
    x0 = g.X.copy()
    x0[free] += 2e-4 * rng.standard_normal((free.sum(), 3))
    x = x0.copy()
    x[free] += 3e-4 * rng.standard_normal((free.sum(), 3))
    pose = hover.copy()
    pose[:2] += (0.02, 0.01)
    p = np.zeros_like(x0)
    p[free] = rng.standard_normal((free.sum(), 3))
    print("peg hover state with a friction lag, t2r_eval deterministic vs atomic", flush=True)
    ga, da, sa = _eval(t2r, w, x, pose, p, (x0, hover), 0)
    gd, dd, sd = _eval(t2r, w, x, pose, p, (x0, hover), 1)
    gd2, dd2, sd2 = _eval(t2r, w, x, pose, p, (x0, hover), 1)
    assert int(sd[6]) > 0 and int(sd[3]) > 0            # friction pairs and active pairs
    assert np.array_equal(gd, gd2) and np.array_equal(dd, dd2) and np.array_equal(sd, sd2)
    assert sd[0] == pytest.approx(sa[0], rel=1e-12) and sd[1] == pytest.approx(sa[1], rel=1e-12)
    assert np.abs(gd - ga).max() <= 1e-12 * np.abs(ga).max()
    assert np.abs(dd - da).max() <= 1e-12 * np.abs(da).max()


def _run(sim, poses, s0, s1):
    xs, ms = [], []
    for s in range(s0, s1):
        m, st = sim.step(poses[:, s], want_x=True)
        torch.cuda.synchronize()
        assert np.all(st.cpu().numpy() & 1), (s, sim.stats())
        xs.append(sim.x.cpu().numpy().copy())
        ms.append(m.cpu().numpy().copy())
    return xs, ms


def test_deterministic_sequence_repeats_and_resumes_bit_for_bit():
    """The peg friction scene (three press and two shear steps) in deterministic
    mode: two contexts give identical bits at every step, and the Newton
    oracle's equilibria to 1e-6 mm; a third context loading the second's
    checkpoint after step 2 repeats steps 3-5 bit for bit."""
    t2r = _gpu()
    from scenes.configs import peg_press_484v
    w = peg_press_484v(mu_f=0.5, shear=(0.1, 0.05), n_shear=2)
    gold = np.load(os.path.join(HERE, "golden", "peg_press_484v_friction_newton.npz"))
    poses = np.stack([e.poses for e in w.envs])
    opts = dict(tol=1e-10, substep_tol=1e-8, max_iters=400000, deterministic=1)
    print("peg friction sequence, deterministic mode, run A", flush=True)
    xa, ma = _run(_sim(t2r, w, **opts), poses, 1, poses.shape[1])
    assert np.abs(np.array(xa) - gold["x"]).max() <= 1e-6
    print("run B to step 2, checkpoint, then steps 3-5", flush=True)
    sb = _sim(t2r, w, **opts)
    xb, mb = _run(sb, poses, 1, 3)
    ck = sb.save_checkpoint()
    xb2, mb2 = _run(sb, poses, 3, poses.shape[1])
    for a, b in zip(xa, xb + xb2):
        assert np.array_equal(a, b)
    for a, b in zip(ma, mb + mb2):
        assert np.array_equal(a, b)
    print("run C from the checkpoint", flush=True)
    sc = _sim(t2r, w, **opts)
    sc.load_checkpoint(ck)
    xc, mc = _run(sc, poses, 3, poses.shape[1])
    for a, b in zip(xa[2:], xc):
        assert np.array_equal(a, b)
    for a, b in zip(ma[2:], mc):
        assert np.array_equal(a, b)


def _small_uneven(n_steps=2):
    """Three envs over two gel sizes (484 and 32 vertices) and three indenters."""
    from scenes.configs import INDENTERS, NU, EnvSpec, Workload, mesh_class, press_schedule
    meshes = {k: mesh_class(k) for k in ("c1", "micro3")}
    inds = {k: INDENTERS[k]() for k in ("sphere3", "peg4", "sphere_small")}
    combos = [("c1", "sphere3", (0.3, -0.2), 0.3), ("micro3", "sphere_small", (0.1, -0.05), 0.12),
              ("c1", "peg4", (-0.2, 0.1), 0.25)]
    envs = []
    for mk, ik, xy, depth in combos:
        poses = press_schedule(inds[ik], (1.0, 0.0, 0.0, 0.0), xy, depth, meshes[mk].thickness, n_steps)
        envs.append(EnvSpec(mk, ik, 0.3, NU, 0.0, poses))
    return Workload("small_uneven", 0, meshes, inds, envs, "f64", 1e-6, "3 envs, 2 gel sizes, 3 indenters")


def test_deterministic_batched_env_equals_its_single_env_launch_bit_for_bit():
    """Three envs over two gel sizes and three indenters in one launch: each
    env's positions equal those of its own single-env launch exactly (same
    workgroup shape)."""
    t2r = _gpu()
    w = _small_uneven()
    opts = dict(tol=1e-8, substep_tol=1e-8, max_iters=400000, deterministic=1, block_size=256)
    seq = lambda idx: np.ascontiguousarray(np.stack([w.envs[i].poses[1:] for i in idx]).transpose(1, 0, 2))
    print("small uneven batch, deterministic mode, batched launch", flush=True)
    sim = _sim(t2r, w, **opts)
    _, st = sim.step_sequence(seq(range(len(w.envs))), want_x=True)
    torch.cuda.synchronize()
    assert np.all(st.cpu().numpy() & 1), st
    xb = [a.cpu().numpy().copy() for a in sim.split_x()]
    for i in range(len(w.envs)):
        print(f"single-env launch of env {i}", flush=True)
        one = _sim(t2r, w, envs=[i], **opts)
        _, st1 = one.step_sequence(seq([i]), want_x=True)
        torch.cuda.synchronize()
        assert np.all(st1.cpu().numpy() & 1)
        assert np.array_equal(xb[i], one.x.cpu().numpy())
