"""Oracle conservative continuous collision step. Test infrastructure only.

Within one solve the indenter is static and gel vertex i moves along
x_i + t dx_i. Every point of a primitive is a convex combination of its
vertices, so the distance of a pair can shrink at most at rate
l = max |dx_i| over the pair's gel vertices; for a self-contact pair, whose two
primitives both move, at most at the sum of that maximum over each side. Starting from d_0 and advancing
by t += (d(t) - g)/l therefore never brings the pair below the gap
g = GAP_FRACTION * d_0: this is additive conservative advancement (the
additive-CCD idea of codimensional IPC, cited by the paper for IPC).
"""

from __future__ import annotations

import numpy as np

from .distance import edge_edge, point_triangle

GAP_FRACTION = 0.1
MAX_ADVANCE = 500


def ccd_step(prob, x, dx, alpha_max, thr=None):
    """Largest t <= alpha_max (conservative) keeping every pair at >= 10% of its gap.

    Only pairs closer than `thr` at t = 0 are checked; the caller guarantees that
    pairs farther away cannot reach zero within alpha_max (|alpha_max dx| < thr).
    """
    L = float(np.linalg.norm(dx, axis=1).max()) if len(dx) else 0.0
    if L == 0.0 or alpha_max <= 0.0:
        return alpha_max
    if thr is None:  # self-contact pairs close at up to twice the largest speed
        thr = prob.dhat + (2.02 if getattr(prob, "self_contact", False) else 1.01) * alpha_max * L
    pairs = prob.candidates(x, thr)
    if len(pairs["idx"]) == 0:
        return alpha_max
    nv = prob.nv
    idx = pairs["idx"]
    gel_pt = idx < nv
    vel = np.where(gel_pt[:, :, None], dx[np.where(gel_pt, idx, 0)], 0.0)
    speed = np.linalg.norm(vel, axis=2)
    lpair = speed.max(axis=1)
    kind = pairs["kind"]
    gvf, gee = kind == 3, kind == 4       # self-contact: both sides move
    lpair[gvf] = speed[gvf, 0] + speed[gvf, 1:].max(axis=1)
    lpair[gee] = speed[gee, :2].max(axis=1) + speed[gee, 2:].max(axis=1)
    d0 = prob.pair_geometry(x, pairs)["d"]
    if np.any(d0 <= 0):
        return 0.0
    gap = GAP_FRACTION * d0
    t = np.zeros(len(d0))
    d = d0.copy()
    done = (lpair == 0.0) | (lpair * alpha_max <= d0 - gap)
    t[done] = alpha_max
    active = ~done
    for _ in range(MAX_ADVANCE):
        if not np.any(active):
            break
        ia = np.nonzero(active)[0]
        # remaining travel cannot close the gap: the full step is safe
        fin = lpair[ia] * (alpha_max - t[ia]) <= d[ia] - gap[ia]
        t[ia[fin]] = alpha_max
        active[ia[fin]] = False
        ia = ia[~fin]
        if len(ia) == 0:
            break
        t[ia] = t[ia] + (d[ia] - gap[ia]) / lpair[ia]
        sub = {"idx": idx[ia], "kind": pairs["kind"][ia]}
        d[ia] = _dist_at(prob, x, dx, sub, t[ia])
        stall = (d[ia] - gap[ia]) <= 1e-3 * (d0[ia] - gap[ia])
        active[ia[stall]] = False
    return float(min(alpha_max, t.min()))


def _dist_at(prob, x, dx, pairs, t):
    """Distance of each pair when gel vertices sit at x + t_k dx (t per pair)."""
    pts = np.concatenate([x, prob.Yw], axis=0)
    vel = np.concatenate([dx, np.zeros_like(prob.Yw)], axis=0)
    idx = pairs["idx"]
    Z = pts[idx] + t[:, None, None] * vel[idx]
    d = np.zeros(len(idx))
    pt = ~np.isin(pairs["kind"], (2, 4))  # point-triangle kinds; 2 and 4 are edge-edge
    if np.any(pt):
        d[pt] = point_triangle(Z[pt, 0], Z[pt, 1], Z[pt, 2], Z[pt, 3])["d"]
    ee = ~pt
    if np.any(ee):
        d[ee] = edge_edge(Z[ee, 0], Z[ee, 1], Z[ee, 2], Z[ee, 3])["d"]
    return d
