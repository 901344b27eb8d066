"""Oracle ground-truth minimiser: projected Newton with a CCD-bounded line search.
Test infrastructure only.

This is the standard IPC solver route (Newton + CCD line search) that the
paper names as accurate but expensive (Sec. 3.1; Supp. A after the Hessian).
Element and pair Hessian blocks are eigen-clamped to PSD, the step is the
sparse (or dense) solve H_psd dx = -g over the free DOFs, its length is capped
so that no vertex moves more than dhat, CCD keeps every pair at >= 10% of its
gap, and Armijo backtracking (c = 1e-4) with a relative rounding guard ensures
decrease. It stops when |dx|_inf <= tol.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from .ccd import ccd_step

ARMIJO_C = 1e-4
ENERGY_GUARD = 1e-13
EXACT_NEAR = 1e-4   # mm: switch to the exact Hessian once steps are this small


def _solve(H, g, require_pd):
    """Return -H^-1 g; with require_pd, None unless H is positive definite."""
    n = g.shape[0]
    if n <= 3000:
        A = H.toarray()
        if require_pd:
            try:
                cf = sla.cho_factor(A)
            except np.linalg.LinAlgError:
                return None
            return -sla.cho_solve(cf, g)
        return -sla.solve(A, g, assume_a="sym")
    if require_pd:
        # symmetric permutation with diagonal pivots only: U's diagonal is D of
        # P H P^T = L D L^T, so H is positive definite iff every entry is positive
        try:
            lu = spla.splu(H.tocsc(), permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                           options=dict(SymmetricMode=True))
        except RuntimeError:
            return None
        if np.any(lu.U.diagonal() <= 0):
            return None
        return -lu.solve(g)
    return -spla.splu(H.tocsc()).solve(g)


def newton_solve(prob, x0, tol=1e-12, max_iter=200, verbose=False):
    """Minimise prob.energy from the feasible x0. Returns (x, info)."""
    x = np.array(x0, dtype=np.float64)
    free = ~prob.gel.fixed
    fdof = np.repeat(free, 3)
    E = prob.energy(x)
    if not np.isfinite(E):
        raise ValueError("Newton start is infeasible")
    info = dict(iters=0, converged=False, step_inf=np.inf)
    stall = 0
    prev_step = np.inf
    for it in range(max_iter):
        g = prob.gradient(x).ravel()
        gf = g[fdof]
        dxf = None
        if prev_step < EXACT_NEAR:
            # close to the minimiser the exact Hessian is positive definite there:
            # use it (Cholesky must succeed) for the quadratic final convergence
            Hx = prob.hessian(x, project=False)[fdof][:, fdof]
            dxf = _solve(Hx, gf, require_pd=True)
        if dxf is None:
            H = prob.hessian(x, project=True)[fdof][:, fdof]
            dxf = _solve(H, gf, require_pd=False)
        dx = np.zeros(3 * prob.nv)
        dx[fdof] = dxf
        dx = dx.reshape(-1, 3)
        step_inf = float(np.abs(dx).max())
        info["iters"] = it
        info["step_inf"] = step_inf
        if step_inf <= tol:
            info["converged"] = True
            break
        L = float(np.linalg.norm(dx, axis=1).max())
        alpha = min(1.0, prob.dhat / L)
        # self-contact pairs close at up to twice the largest speed
        rate = 2.02 if getattr(prob, "self_contact", False) else 1.01
        alpha = ccd_step(prob, x, dx, alpha, thr=prob.dhat + rate * alpha * L)
        gdx = float(g @ dx.ravel())
        accepted = False
        for _ in range(80):
            xt = x + alpha * dx
            Et = prob.energy(xt)
            if np.isfinite(Et) and Et <= E + ARMIJO_C * alpha * gdx + ENERGY_GUARD * prob.energy_ref:
                accepted = True
                break
            alpha *= 0.5
        if not accepted:
            info["failed"] = "line search"
            break
        prev_step = step_inf
        x, E = xt, Et
        if verbose:
            print(f"newton it {it} |dx|={step_inf:.3e} alpha={alpha:.3e} E={E:.12e}")
        if alpha * step_inf < 1e-15:
            stall += 1
            if stall > 3:
                info["failed"] = "stalled"
                break
    info["energy"] = E
    return x, info
