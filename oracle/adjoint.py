"""Oracle adjoint of a marker loss at a frictionless equilibrium.
Test infrastructure only.

Parameters theta = (E, nu, mu_f, dt_x, dt_y, dt_z, dw_x, dw_y, dw_z): the
material of the env, its friction coefficient, and a rigid offset of the
indenter pose that moves every indenter point to
    y_j(dt, dw) = exp([dw]x) (y_j - t) + t + dt
(translation dt; rotation vector dw about the indenter origin t), with the
derivative taken at dt = dw = 0.

The last load step's equilibrium x* has g(x*; theta) = 0 on the free DOFs, so
by implicit differentiation
    dL/dtheta = -lambda^T dg/dtheta,   H(x*) lambda = dL/dx,
with H the exact (unprojected) Hessian of Pi_s on the free DOFs (a direct
sparse solve here). Without friction (mu_f = 0) the last step's equilibrium
depends on theta only through that step, because the lag enters Pi_s with the
factor mu_f; for the same reason dg/dmu_f at mu_f = 0 is the lagged friction
gradient with unit coefficient, the lag taken at the previous equilibrium
(x_{s-1}, q_{s-1}).

Parity unpinned by the paper (it has no gradients): pinned by central finite
differences of the whole forward simulation in the tests.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .barrier import barrier_d1, barrier_d2
from .distance import distance_derivatives
from .elastic import element_gradient
from .problem import StepProblem

N_THETA = 9


def marker_vjp(gel, dL_du):
    """dL/dx (N_v, 3) of a loss on the marker displacements u_m = sum_k w_mk (x - X)_{t_mk}."""
    out = np.zeros((gel.n_v, 3))
    np.add.at(out, gel.marker_tris, gel.marker_w[:, :, None] * np.asarray(dL_du)[:, None, :])
    return out


def lame_partials(E, nu):
    """d(mu, lambda)/dE and d(mu, lambda)/dnu for mu = E/(2(1+nu)), lambda = E nu/((1+nu)(1-2nu))."""
    dmu_dE = 1.0 / (2.0 * (1.0 + nu))
    dlam_dE = nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    dmu_dnu = -E / (2.0 * (1.0 + nu) ** 2)
    dlam_dnu = E * (1.0 + 2.0 * nu * nu) / ((1.0 + nu) ** 2 * (1.0 - 2.0 * nu) ** 2)
    return dmu_dE, dlam_dE, dmu_dnu, dlam_dnu


def _elastic_gradient(prob, x, mu, lam):
    g = prob.gel
    out = np.zeros_like(x)
    np.add.at(out, g.tets, element_gradient(x, g.tets, g.Dm_inv, g.vol, mu, lam))
    out[g.fixed] = 0.0
    return out


def _unit_friction_gradient(prob, x, x_prev, pose_prev):
    """Gradient of the lagged friction term with coefficient 1 (lag at x_prev, pose_prev)."""
    unit = StepProblem(prob.gel, prob.ind, 1.0, 0.25, 1.0, prob.eps_v, prob.dhat, prob.kappa)
    unit.mu, unit.lam = 0.0, 0.0          # elastic part off
    unit.set_lag(x_prev, pose_prev)
    unit.set_pose(prob.pose)
    if unit.lag is None or len(unit.lag["lam"]) == 0:
        return np.zeros_like(x)
    full = unit.gradient(x)
    # remove the barrier part: the same problem without the lag
    unit.lag = None
    return full - unit.gradient(x)


def _pose_mixed_terms(prob, x, lam_x):
    """lambda^T (d g / d theta_pose) for the six pose directions (barrier term)."""
    pairs, res = prob.active(x)
    out = np.zeros(6)
    if len(pairs["idx"]) == 0:
        return out
    d, grad, Hd = distance_derivatives(res["Z"], res["c"], res["Cw"], res["k"])
    b1 = barrier_d1(d, prob.dhat)
    b2 = barrier_d2(d, prob.dhat)
    gf = grad.reshape(-1, 12)
    Hb = prob.kappa * (b2[:, None, None] * np.einsum("ni,nj->nij", gf, gf) + b1[:, None, None] * Hd)
    gel_pt = pairs["idx"] < prob.nv
    P1 = np.where(gel_pt[:, :, None], lam_x[np.where(gel_pt, pairs["idx"], 0)], 0.0).reshape(-1, 12)
    t = prob.pose[:3]
    Zind = res["Z"]                               # world points of the pair
    for a in range(6):
        e = np.zeros(3)
        e[a % 3] = 1.0
        if a < 3:
            dy = np.broadcast_to(e, Zind.shape)
        else:
            dy = np.cross(e[None, None, :], Zind - t[None, None, :])
        P2 = np.where(gel_pt[:, :, None], 0.0, dy).reshape(-1, 12)
        out[a] = float(np.einsum("ni,nij,nj->", P1, Hb, P2))
    return out


def adjoint_gradient(prob, x, dL_du, x_prev=None, pose_prev=None):
    """dL/dtheta (9,) at the frictionless equilibrium x of `prob` (pose set).
    x_prev, pose_prev: the previous equilibrium, for the mu_f derivative."""
    if prob.lag is not None and prob.mu_f != 0.0:
        raise ValueError("the oracle adjoint covers frictionless equilibria")
    gel = prob.gel
    free = np.repeat(~gel.fixed, 3)
    H = prob.hessian(x, project=False).tocsc()[free][:, free]
    rhs = marker_vjp(gel, dL_du).ravel()[free]
    lam = spla.spsolve(H.tocsc(), rhs)
    lam_full = np.zeros(3 * gel.n_v)
    lam_full[free] = lam
    lam_x = lam_full.reshape(-1, 3)
    E = prob.mu * (3 * prob.lam + 2 * prob.mu) / (prob.lam + prob.mu)
    nu = prob.lam / (2 * (prob.lam + prob.mu))
    dmu_dE, dlam_dE, dmu_dnu, dlam_dnu = lame_partials(E, nu)
    g_mu = _elastic_gradient(prob, x, 1.0, 0.0)
    g_lam = _elastic_gradient(prob, x, 0.0, 1.0)
    c_mu, c_lam = float(np.sum(lam_x * g_mu)), float(np.sum(lam_x * g_lam))
    out = np.zeros(N_THETA)
    out[0] = -(c_mu * dmu_dE + c_lam * dlam_dE)
    out[1] = -(c_mu * dmu_dnu + c_lam * dlam_dnu)
    if x_prev is not None:
        out[2] = -float(np.sum(lam_x * _unit_friction_gradient(prob, x, x_prev, pose_prev)))
    out[3:] = -_pose_mixed_terms(prob, x, lam_x)
    return out, lam_x


def quat_from_rotvec(w):
    w = np.asarray(w, dtype=np.float64)
    a = float(np.linalg.norm(w))
    if a == 0.0:
        return np.array([1.0, 0.0, 0.0, 0.0])
    return np.concatenate([[np.cos(0.5 * a)], np.sin(0.5 * a) * w / a])


def quat_mul(p, q):
    w1, x1, y1, z1 = p
    w2, x2, y2, z2 = q
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                     w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                     w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def offset_pose(pose, dt, dw):
    """The pose whose indenter points are exp([dw]x)(y - t) + t + dt."""
    pose = np.asarray(pose, dtype=np.float64)
    q = pose[3:] / np.linalg.norm(pose[3:])
    return np.concatenate([pose[:3] + np.asarray(dt, dtype=np.float64), quat_mul(quat_from_rotvec(dw), q)])
