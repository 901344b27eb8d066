"""Oracle load-step sequence with indenter continuation. Test infrastructure only.

The paper does not say how a moving rigid indenter avoids starting a solve in
intersection. Reading: within load step s the indenter pose is interpolated
from q_{s-1} to q_s (translation linear, rotation slerp) over tau in [0, 1],
and tau advances by the largest increment that moves every indenter point by
at most 1/2 min(dhat, d_min), where d_min is the current smallest gel/indenter
distance. A rigid motion moves every point of a triangle by at most the
largest vertex displacement, and that is bounded by |dt| + theta r_max for a
translation dt, a rotation by angle theta and the largest local vertex radius
r_max. Each intermediate pose is solved; the last one (tau = 1) gives x*_s.
Only the indenter moves during an advance, so no distance drops below half
its value and every start is feasible. Without friction x*_s depends only on
q_s; with lagged friction only on (q_s, x_{s-1}, q_{s-1}).
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .geometry import GelGeometry, IndenterGeometry, rotation_angle_between, slerp_pose
from .newton import newton_solve
from .pncg import pncg_solve
from .problem import StepProblem


@dataclass
class SimResult:
    x: list = field(default_factory=list)          # x*_s, (N_v, 3) per step
    markers: list = field(default_factory=list)    # (n_m, 3) per step
    substeps: list = field(default_factory=list)
    iters: list = field(default_factory=list)
    energy: list = field(default_factory=list)
    d_min: list = field(default_factory=list)
    n_active: list = field(default_factory=list)


def build(gel_mesh, indenter, env, ee_mollifier=False, self_contact=False):
    gel = GelGeometry(gel_mesh.X, gel_mesh.tets, gel_mesh.fixed, gel_mesh.markers)
    ind = IndenterGeometry(indenter.Y, indenter.tris)
    prob = StepProblem(gel, ind, env.E, env.nu, env.mu_f, env.eps_v, env.dhat, env.kappa,
                       ee_mollifier=ee_mollifier, self_contact=self_contact)
    return gel, ind, prob


def continuation_increment(prob, x, pose_a, pose_b, tau, d_min):
    """Largest d_tau per the bound 1/2 min(dhat, d_min) on indenter point motion."""
    dt = np.linalg.norm(np.asarray(pose_b[:3]) - np.asarray(pose_a[:3]))
    theta = rotation_angle_between(pose_a, pose_b)
    rate = dt + theta * prob.ind.r_max
    if rate == 0.0:
        return 1.0 - tau
    return 0.5 * min(prob.dhat, d_min) / rate


def lumped_mass(gel):
    """Per-vertex volume share sum_{e contains v} V_e / 4 (the lumped mass over the density)."""
    m = np.zeros(gel.n_v)
    np.add.at(m, gel.tets, np.repeat(gel.vol[:, None] / 4.0, 4, axis=1))
    return m


def simulate(gel_mesh, indenter, env, mode="newton", tol=None, n_steps=None,
             max_substeps=10000, pncg_kw=None, x_start=None, verbose=False, dynamic=None,
             ee_mollifier=False, self_contact=False):
    """Run the load steps of `env` (a scenes.EnvSpec). mode: 'newton' or 'pncg'.
    dynamic: None (quasi-static) or dict(density=rho, dt=h) for the implicit-Euler
    form: each step adds 1/2 |x - xhat|^2_M / h^2 with the lumped mass M = rho V/4
    per vertex and xhat = x^t + h v^t, and then v = (x - x^t) / h (v^0 = 0).
    ee_mollifier: weight edge-edge barriers by the parallel-edge mollifier;
    self_contact: barriers between gel surface primitives too."""
    gel, ind, prob = build(gel_mesh, indenter, env, ee_mollifier=ee_mollifier, self_contact=self_contact)
    poses = np.asarray(env.poses, dtype=np.float64)
    S = poses.shape[0] - 1 if n_steps is None else n_steps
    x = gel.X.copy() if x_start is None else np.array(x_start, dtype=np.float64)
    out = SimResult()
    vel = np.zeros_like(x)
    if dynamic is not None:
        w_dyn = dynamic["density"] * lumped_mass(gel) / dynamic["dt"] ** 2
    for s in range(1, S + 1):
        q0, q1 = poses[s - 1], poses[s]
        x_t = x.copy()
        if dynamic is not None:
            prob.set_inertia(w_dyn, x_t + dynamic["dt"] * vel)
        prob.set_lag(x, q0)
        tau, nsub, iters = 0.0, 0, 0
        while tau < 1.0:
            prob.set_pose(slerp_pose(q0, q1, tau))
            dm = prob.d_min(x)
            dtau = continuation_increment(prob, x, q0, q1, tau, dm)
            tau = min(1.0, tau + dtau)
            prob.set_pose(slerp_pose(q0, q1, tau))
            if mode == "newton":
                x, info = newton_solve(prob, x, tol=1e-12 if tol is None else tol)
            else:
                x, info = pncg_solve(prob, x, tol=1e-6 if tol is None else tol, **(pncg_kw or {}))
            iters += info["iters"]
            nsub += 1
            if verbose:
                print(f"step {s} tau={tau:.4f} iters={info['iters']} conv={info['converged']}")
            if nsub >= max_substeps:
                raise RuntimeError("too many substeps")
        if dynamic is not None:
            vel = (x - x_t) / dynamic["dt"]
            vel[gel.fixed] = 0.0
        out.x.append(x.copy())
        out.markers.append(gel.markers(x))
        out.substeps.append(nsub)
        out.iters.append(iters)
        out.energy.append(prob.energy(x))
        out.d_min.append(prob.d_min(x))
        out.n_active.append(len(prob.active(x)[0]["idx"]))
    return out
