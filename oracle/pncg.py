"""Oracle PNCG reference: preconditioned Dai-Kou nonlinear CG on the step energy.
Test infrastructure only.

From Supp. A (eqs. dk_direction and step_size) with these readings:
  * P_k = diag(H(x_k))^-1, re-evaluated at every iterate, from the exact
    (unprojected) diagonal with each contact pair's contribution clamped at
    zero (StepProblem.precond_diag: close pairs make the exact entry negative
    in the tangential directions); entries are floored at 1e-12 mu max_v sum_e V_e |g_i|^2
    (a fixed fraction of the largest rest-state stiffness of a free vertex) so
    the inverse exists; the floor is per env, not per iterate, so the kernels
    can apply P in the same pass that finishes diag.
  * p_0 = -P_0 g_0;  p_{k+1} = -P_{k+1} g_{k+1} + beta_k p_k with
        beta_k = g_{k+1}^T P_{k+1} y_k / (y_k^T p_k)
                 - (y_k^T P_{k+1} y_k / y_k^T p_k) (p_k^T g_{k+1} / y_k^T p_k),
    y_k = g_{k+1} - g_k; beta is reset to 0 when y_k^T p_k <= 1e-30, and the
    direction is reset to -P g when it is not a descent direction.
  * alpha_up = dhat / (2 |p|_inf) (component max over free DOFs) and
    alpha_bar = -g^T p / p^T H p (infinite when p^T H p <= 0);
    alpha = min(alpha_up, alpha_bar, alpha_ccd) where alpha_ccd is the
    conservative CCD step over pairs closer than 2 dhat.
  * The trial point is accepted when it is feasible (every J > 0, every
    d > 0) and, if armijo is on, Pi drops by at least 1e-4 alpha |g^T p| up to
    a rounding guard 1e-13 (mu sum_e V_e + |Pi|) (the elastic energy scale plus
    the energy's magnitude, which barrier terms of close pairs dominate in
    contact, so that rounding noise in Pi cannot stall the search near
    convergence);
    otherwise alpha is halved, at most 30 times.
  * Convergence: |P g|_inf <= tol (mm), the Jacobi-Newton displacement estimate.
"""

from __future__ import annotations

import time

import numpy as np

from .ccd import ccd_step

ARMIJO_C = 1e-4
ENERGY_GUARD = 1e-13
DIAG_FLOOR = 1e-12
YP_MIN = 1e-30
MAX_HALVINGS = 30


def _precond(prob, x, free):
    dg = prob.precond_diag(x)
    floor = DIAG_FLOOR * prob.diag_scale
    P = 1.0 / np.maximum(dg, floor)
    P[~free] = 0.0
    return P


def pncg_solve(prob, x0, tol=1e-6, max_iters=100000, armijo=True, record=None, deadline=None):
    """Run PNCG from the feasible x0. Returns (x, info). `record` collects per-iteration data.
    deadline: a time.perf_counter() value after which no further iteration starts
    (for bounded timing runs; info["timed_out"] is then set)."""
    x = np.array(x0, dtype=np.float64)
    free = ~prob.gel.fixed
    E = prob.energy(x)
    if not np.isfinite(E):
        raise ValueError("PNCG start is infeasible")
    g = prob.gradient(x)
    P = _precond(prob, x, free)
    p = -P * g
    info = dict(iters=0, converged=False, restarts=0, halvings=0)
    k = 0
    for k in range(max_iters + 1):
        res = float(np.abs(P * g).max())
        if res <= tol:
            info["converged"] = True
            break
        if k == max_iters:
            break
        if deadline is not None and time.perf_counter() > deadline:
            info["timed_out"] = True
            break
        pinf = float(np.abs(p).max())
        gp = float(np.sum(g * p))
        curv = prob.curvature(x, p)
        a_up = prob.dhat / (2.0 * pinf)
        a_bar = -gp / curv if curv > 0 else np.inf
        alpha = min(a_up, a_bar)
        L = float(np.linalg.norm(p, axis=1).max())
        a_ccd = ccd_step(prob, x, p, alpha, thr=2.0 * prob.dhat)
        alpha = min(alpha, a_ccd)
        rec = dict(k=k, E=E, res=res, pinf=pinf, gp=gp, curv=curv, a_up=a_up, a_bar=a_bar,
                   a_ccd=a_ccd)
        ok = False
        for h in range(MAX_HALVINGS + 1):
            xt = x + alpha * p
            Et = prob.energy(xt)
            if np.isfinite(Et) and (not armijo or
                                    Et <= E + ARMIJO_C * alpha * gp + ENERGY_GUARD * (prob.energy_ref + abs(E))):
                ok = True
                break
            alpha *= 0.5
            info["halvings"] += 1
        if not ok:
            info["failed"] = "line search"
            break
        x, E = xt, Et
        g1 = prob.gradient(x)
        P1 = _precond(prob, x, free)
        y = g1 - g
        yp = float(np.sum(y * p))
        if yp > YP_MIN:
            beta = float(np.sum(g1 * P1 * y)) / yp - \
                (float(np.sum(y * P1 * y)) / yp) * (float(np.sum(p * g1)) / yp)
        else:
            beta = 0.0
        p1 = -P1 * g1 + beta * p
        if float(np.sum(g1 * p1)) >= 0.0:
            p1 = -P1 * g1
            info["restarts"] += 1
            beta = 0.0
        rec.update(alpha=alpha, beta=beta, yp=yp)
        if record is not None:
            record.append(rec)
        g, P, p = g1, P1, p1
    info["iters"] = k
    info["energy"] = E
    info["res"] = float(np.abs(P * g).max())
    return x, info
