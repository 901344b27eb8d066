"""Oracle adjoint of a marker loss through a sequence of load steps.
Test infrastructure only.

Parameters theta = (E, nu, mu_f, dt_x, dt_y, dt_z, dw_x, dw_y, dw_z): the
material of the env, its friction coefficient, and a rigid offset of every
indenter pose of the sequence that moves each indenter point to
    y_j(dt, dw) = exp([dw]x) (y_j - t) + t + dt
(translation dt; rotation vector dw about that pose's indenter origin t),
with the derivative taken at dt = dw = 0.

Load step s has the equilibrium x_s with g_s(x_s; x_{s-1}, q_{s-1}, q_s,
theta) = 0 on the free DOFs, where the friction term is lagged at
(x_{s-1}, q_{s-1}) (lambda_k, closest-point weights and normal of every pair
closer than dhat there). Implicit differentiation, last step first:
    H_s lambda_s = a_s,   a_s = W^T dL/du_s - (d g_{s+1} / d x_s)^T lambda_{s+1},
    dL/dtheta = - sum_s lambda_s^T d g_s / d theta,
with H_s the exact (unprojected) Hessian of Pi_s on the free DOFs (a direct
sparse solve here). d g_s / d theta collects the elastic term (E, nu), the
friction term with unit coefficient (mu_f), and the pose offset through the
indenter points at q_s (barrier and friction) and at q_{s-1} (the lag). The
carry (d g_s / d x_{s-1})^T lambda_s is the gradient with respect to the lag
points of Q_s = lambda_s^T g_s, taken through lambda_k(d), the normal, the
closest-point weights and the relative displacement (lag_objective_grad).
The state before the first step of the sequence is taken as given.

Parity unpinned by the paper (it has no gradients): pinned by central finite
differences of Q per pair and of the whole forward simulation in the tests.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .barrier import barrier_d1, barrier_d2, mollifier_d1
from .distance import distance_derivatives, edge_edge, point_triangle
from .elastic import element_gradient
from .problem import EE, FV, StepProblem

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
    _, _, Hb = prob.pair_terms(pairs, res, order=2)
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


# ---------------------------------------------------------------- friction lag
def _closest(Zp, kind):
    """Closest-point data (d, c, Cw, k) of pairs with points Zp (n,4,3)."""
    n = len(Zp)
    d, c = np.zeros(n), np.zeros((n, 4))
    Cw, k = np.zeros((n, 4, 2)), np.zeros(n, np.int64)
    for sel, fn in ((kind != EE, point_triangle), (kind == EE, edge_edge)):
        if np.any(sel):
            r = fn(Zp[sel, 0], Zp[sel, 1], Zp[sel, 2], Zp[sel, 3])
            d[sel], c[sel], Cw[sel], k[sel] = r["d"], r["c"], r["Cw"], r["k"]
    return d, c, Cw, k


def _phi(s, eps):
    """f'(s)/s of the friction mollifier, and its derivative in s."""
    s = np.asarray(s, dtype=np.float64)
    inner = s < eps
    with np.errstate(divide="ignore", invalid="ignore"):
        phi = np.where(inner, -s / eps ** 2 + 2.0 / eps, 1.0 / np.where(s > 0, s, 1.0))
        dphi = np.where(inner, -1.0 / eps ** 2, -1.0 / np.where(s > 0, s, 1.0) ** 2)
    return phi, dphi


def lag_objective(Zp, Z, kind, is_gel, ell, mu_f, kappa, dhat, eps_v):
    """Q_k = sum over the gel points i of ell_i . g_i for each friction pair k:
    the pair's friction gradient at the current points Z (n,4,3), contracted
    with ell (n,4,3), as a function of the lag points Zp (n,4,3).
    g_i = mu_f lambda_k phi(s) a_i u with lambda_k = -kappa b'(d(Zp)), a_i the
    signed closest-point weight of gel point i, u the tangential part of the
    relative displacement and phi = f'(s)/s (Supp. A, eqs. friction_energy,
    friction_mollifier)."""
    d, c, _, _ = _closest(Zp, kind)
    sig = np.where(kind == FV, -1.0, 1.0)
    r = np.einsum("ni,nid->nd", c, Zp)
    nvec = sig[:, None] * r / d[:, None]
    lam = -kappa * barrier_d1(d, dhat)
    Delta = sig[:, None] * np.einsum("ni,nid->nd", c, Z - Zp)
    u = Delta - np.einsum("nd,nd->n", nvec, Delta)[:, None] * nvec
    phi, _ = _phi(np.linalg.norm(u, axis=1), eps_v)
    Lb = np.einsum("ni,nid->nd", c * is_gel, ell)
    return mu_f * lam * phi * sig * np.einsum("nd,nd->n", Lb, u)


def lag_objective_grad(Zp, Z, kind, is_gel, ell, mu_f, kappa, dhat, eps_v):
    """Gradient of lag_objective with respect to the lag points Zp, (n,4,3).

    Reverse-mode chain rule through d = |r|, n = sig r/d, lambda(d), the
    relative displacement Delta = sig sum_i c_i (Z_i - Zp_i), u = (I - n n^T)
    Delta, phi(|u|), and the closest-point weights c(w(Zp)), whose free
    parameters w move with Zp by the implicit-function theorem on the
    optimality condition D^T r = 0 (D_a = sum_i Cw_ia Zp_i):
        (D^T D) dw = - sum_i (Cw_ia r + c_i D_a) . dZp_i."""
    d, c, Cw, k = _closest(Zp, kind)
    n = len(d)
    sig = np.where(kind == FV, -1.0, 1.0)
    r = np.einsum("ni,nid->nd", c, Zp)
    rh = r / d[:, None]
    nvec = sig[:, None] * rh
    b1 = barrier_d1(d, dhat)
    b2 = barrier_d2(d, dhat)
    lam = -kappa * b1
    dZ = Z - Zp
    Delta = sig[:, None] * np.einsum("ni,nid->nd", c, dZ)
    nD = np.einsum("nd,nd->n", nvec, Delta)
    u = Delta - nD[:, None] * nvec
    s = np.linalg.norm(u, axis=1)
    phi, dphi = _phi(s, eps_v)
    Lb = np.einsum("ni,nid->nd", c * is_gel, ell)
    C = sig * np.einsum("nd,nd->n", Lb, u)
    # adjoints of Q = mu_f lam phi C
    lam_b = mu_f * phi * C
    phi_b = mu_f * lam * C
    C_b = mu_f * lam * phi
    d_b = lam_b * (-kappa * b2)
    s_b = phi_b * dphi
    with np.errstate(divide="ignore", invalid="ignore"):
        uh = np.where(s[:, None] > 0, u / np.where(s > 0, s, 1.0)[:, None], 0.0)
    u_b = (C_b * sig)[:, None] * Lb + s_b[:, None] * uh
    Lb_b = (C_b * sig)[:, None] * u
    nu_b = np.einsum("nd,nd->n", nvec, u_b)
    Delta_b = u_b - nu_b[:, None] * nvec
    n_b = -nD[:, None] * u_b - nu_b[:, None] * Delta
    rh_b = sig[:, None] * n_b
    r_b = (rh_b - np.einsum("nd,nd->n", rh, rh_b)[:, None] * rh) / d[:, None] + d_b[:, None] * rh
    c_b = sig[:, None] * np.einsum("nd,nid->ni", Delta_b, dZ) \
        + is_gel * np.einsum("nd,nid->ni", Lb_b, ell) + np.einsum("nd,nid->ni", r_b, Zp)
    Zp_b = (-sig[:, None] * c)[:, :, None] * Delta_b[:, None, :] + c[:, :, None] * r_b[:, None, :]
    # closest-point parameters: c = c(w), w = w(Zp)
    D = np.einsum("nia,nid->nad", Cw, Zp)
    M = np.einsum("nad,nbd->nab", D, D)
    for a in range(2):
        unused = k <= a
        M[unused, a, :] = 0.0
        M[unused, :, a] = 0.0
        M[unused, a, a] = 1.0
    w_b = np.einsum("ni,nia->na", c_b, Cw)
    for a in range(2):
        w_b[k <= a, a] = 0.0
    m = np.linalg.solve(M, w_b[:, :, None])[:, :, 0]
    Zp_b -= np.einsum("nia,nd,na->nid", Cw, r, m) + np.einsum("ni,nad,na->nid", c, D, m)
    return Zp_b


def _lag_pairs(prob, x_prev, pose_prev):
    """The pairs of the friction lag at (x_{s-1}, q_{s-1}) and their points."""
    Yp = prob.ind.world(pose_prev)
    pairs = prob.candidates(x_prev, prob.dhat, Yw=Yp)
    res = prob.pair_geometry(x_prev, pairs, Yw=Yp)
    act = (res["d"] < prob.dhat) & (pairs["kind"] < 3)   # self-contact pairs carry no friction
    return pairs["idx"][act], pairs["kind"][act], res["Z"][act], Yp


def _pose_directions(Y, t):
    """dY/dtheta_a (6, n, 3): translations e_a and rotations e_a x (y - t)."""
    out = np.zeros((6,) + Y.shape)
    for a in range(3):
        e = np.zeros(3)
        e[a] = 1.0
        out[a] = e
        out[3 + a] = np.cross(e[None, :], Y - t[None, :])
    return out


def _friction_pose_terms(prob, x, lam_x):
    """lambda^T (d g_f / d theta_pose) through the indenter points at the
    current pose (the relative displacement of the lagged friction term)."""
    L = prob.lag
    out = np.zeros(6)
    if L is None or len(L["lam"]) == 0:
        return out
    gel_pt, gid, TD, s = prob._friction_terms(x)
    eps = prob.eps_v
    phi, dphi = _phi(s, eps)
    corr = s * dphi
    with np.errstate(divide="ignore", invalid="ignore"):
        uh = np.where(s[:, None] > 0, TD / np.where(s > 0, s, 1.0)[:, None], 0.0)
    nvec = L["n"]
    q1 = np.einsum("ni,nid->nd", L["a"] * gel_pt, lam_x[gid])
    yid = np.where(gel_pt, 0, L["idx"] - prob.nv)
    dirs = _pose_directions(prob.Yw, prob.pose[:3])
    w = prob.mu_f * L["lam"]
    for a in range(6):
        q2 = -np.einsum("ni,nid->nd", L["b"] * ~gel_pt, dirs[a][yid])
        hq = phi * (np.einsum("nd,nd->n", q1, q2) - np.einsum("nd,nd->n", nvec, q1) * np.einsum("nd,nd->n", nvec, q2)) \
            + corr * np.einsum("nd,nd->n", uh, q1) * np.einsum("nd,nd->n", uh, q2)
        out[a] = float(np.sum(w * hq))
    return out


def step_adjoint_terms(prob, x, xp, pose_prev, lam_x):
    """For one load step with prob's pose q_s set and lag at (xp, pose_prev):
    returns (-lambda^T dg_s/dtheta (9,), -(dg_s/dx_{s-1})^T lambda (N_v, 3))."""
    gel = prob.gel
    E = prob.mu * (3 * prob.lam + 2 * prob.mu) / (prob.lam + prob.mu)
    nu = prob.lam / (2 * (prob.lam + prob.mu))
    dmu_dE, dlam_dE, dmu_dnu, dlam_dnu = lame_partials(E, nu)
    out = np.zeros(N_THETA)
    g_mu = _elastic_gradient(prob, x, 1.0, 0.0)
    g_lam = _elastic_gradient(prob, x, 0.0, 1.0)
    c_mu, c_lam = float(np.sum(lam_x * g_mu)), float(np.sum(lam_x * g_lam))
    out[0] = -(c_mu * dmu_dE + c_lam * dlam_dE)
    out[1] = -(c_mu * dmu_dnu + c_lam * dlam_dnu)
    out[2] = -float(np.sum(lam_x * _unit_friction_gradient(prob, x, xp, pose_prev)))
    out[3:] = -_pose_mixed_terms(prob, x, lam_x) - _friction_pose_terms(prob, x, lam_x)
    carry = np.zeros((gel.n_v, 3))
    if prob.mu_f != 0.0:
        idx, kind, Zp, Yp = _lag_pairs(prob, xp, pose_prev)
        if len(idx):
            is_gel = idx < prob.nv
            pts = np.concatenate([x, prob.Yw], axis=0)
            ell = np.where(is_gel[:, :, None], lam_x[np.where(is_gel, idx, 0)], 0.0)
            G = lag_objective_grad(Zp, pts[idx], kind, is_gel, ell, prob.mu_f, prob.kappa,
                                   prob.dhat, prob.eps_v)
            np.add.at(carry, np.where(is_gel, idx, 0), -G * is_gel[:, :, None])
            dirs = _pose_directions(Yp, np.asarray(pose_prev[:3], dtype=np.float64))
            yid = np.where(is_gel, 0, idx - prob.nv)
            for a in range(6):
                out[3 + a] -= float(np.sum(G * (~is_gel)[:, :, None] * dirs[a][yid]))
    carry[gel.fixed] = 0.0
    return out, carry


def adjoint_sequence(prob, xs, poses, dL_du):
    """dL/dtheta (9,) of a loss on the markers of load steps 1..S.

    prob: a StepProblem of the env (material, mu_f, dhat, kappa, eps_v);
    xs: [x_0, ..., x_S] the equilibria (x_0 the state before step 1);
    poses: (S+1, 7) the indenter poses q_0..q_S; dL_du: (S, n_m, 3)."""
    gel = prob.gel
    S = len(xs) - 1
    free = np.repeat(~gel.fixed, 3)
    out = np.zeros(N_THETA)
    carry = np.zeros((gel.n_v, 3))
    for s in range(S, 0, -1):
        x, xp = xs[s], xs[s - 1]
        prob.set_lag(xp, poses[s - 1])
        prob.set_pose(poses[s])
        H = prob.hessian(x, project=False).tocsc()[free][:, free]
        rhs = (marker_vjp(gel, dL_du[s - 1]) + carry).ravel()[free]
        lam = np.zeros(3 * gel.n_v)
        lam[free] = spla.spsolve(H.tocsc(), rhs)
        theta, carry = step_adjoint_terms(prob, x, xp, poses[s - 1], lam.reshape(-1, 3))
        out += theta
    return out
