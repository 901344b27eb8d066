"""Oracle distances between closed primitives and their derivatives.
Test infrastructure only.

d_k in the barrier (Supp. A, eq. ipc_energy) is read as the exact Euclidean
distance between closed primitives: point-triangle and segment-segment.

Closest points are found by the textbook convex-minimisation argument: the
squared distance is a convex quadratic in the barycentric parameters, so the
minimum over the closed primitive is either the unconstrained stationary
point (if it lies inside) or the minimum over the primitive's boundary, which
reduces to point-segment problems.

Each result carries a coefficient vector c over the four involved points Z
(r = sum_i c_i Z_i is the vector between the two closest points, d = |r|), the
derivative Cw = dc/dw of c with respect to the k free barycentric parameters w
of the active feature (k = 2 face/edge-edge interior, 1 edge, 0 vertex), so
that derivatives follow from the value function d^2(Z) = min_w |sum c_i(w) Z_i|^2:
  grad_{Z_i} d = c_i r / d                                    (envelope theorem)
  Hess(d^2) = phi_ZZ - phi_Zw phi_ww^-1 phi_wZ                (implicit function)
with phi = |r|^2, phi_ZiZj = 2 c_i c_j I, phi_wawb = 2 D_a.D_b,
phi_Ziwa = 2 (Cw_ia r + c_i D_a), D_a = sum_i Cw_ia Z_i, and
Hess(d) = Hess(d^2)/(2d) - grad d grad d^T / d.
"""

from __future__ import annotations

import numpy as np

PARALLEL_SIN2 = 1e-14  # relative sin^2 threshold below which edge-edge is treated as parallel


def _dot(a, b):
    return np.einsum("...i,...i->...", a, b)


def _point_segment(p, a, b):
    """Closest point on segment [a,b] to p: returns (dist, s) with s clamped to [0,1]."""
    e = b - a
    ee = _dot(e, e)
    s = np.clip(_dot(p - a, e) / ee, 0.0, 1.0)
    r = p - (a + s[:, None] * e)
    return np.sqrt(_dot(r, r)), s


def point_triangle(p, t0, t1, t2):
    """Distance from points p to triangles (t0,t1,t2), all (n,3).

    Returns dict(d, c, Cw, k) over the point order [p, t0, t1, t2], with
    r = p - closest point on the triangle.
    """
    p, t0, t1, t2 = (np.asarray(v, dtype=np.float64).reshape(-1, 3) for v in (p, t0, t1, t2))
    n = p.shape[0]
    e1, e2, v = t1 - t0, t2 - t0, p - t0
    a11, a12, a22 = _dot(e1, e1), _dot(e1, e2), _dot(e2, e2)
    b1, b2 = _dot(v, e1), _dot(v, e2)
    det = a11 * a22 - a12 * a12
    s = (b1 * a22 - b2 * a12) / det
    t = (a11 * b2 - a12 * b1) / det
    inside = (s >= 0) & (t >= 0) & (s + t <= 1)

    d = np.empty(n)
    c = np.zeros((n, 4))
    Cw = np.zeros((n, 4, 2))
    k = np.zeros(n, dtype=np.int64)

    # interior
    ii = inside
    r = v[ii] - s[ii, None] * e1[ii] - t[ii, None] * e2[ii]
    d[ii] = np.sqrt(_dot(r, r))
    c[ii] = np.stack([np.ones(ii.sum()), -(1 - s[ii] - t[ii]), -s[ii], -t[ii]], axis=1)
    Cw[ii, :, 0] = [0.0, 1.0, -1.0, 0.0]
    Cw[ii, :, 1] = [0.0, 1.0, 0.0, -1.0]
    k[ii] = 2

    # boundary: the three edges
    oo = ~inside
    if np.any(oo):
        P, A = p[oo], (t0[oo], t1[oo], t2[oo])
        cand = []
        for (ia, ib) in ((0, 1), (1, 2), (2, 0)):
            dist, sp = _point_segment(P, A[ia], A[ib])
            cand.append((dist, sp, ia, ib))
        dists = np.stack([cnd[0] for cnd in cand], axis=1)
        best = np.argmin(dists, axis=1)
        idx = np.nonzero(oo)[0]
        for j, (dist, sp, ia, ib) in enumerate(cand):
            sel = best == j
            rows = idx[sel]
            ss = sp[sel]
            d[rows] = dist[sel]
            c[rows, 0] = 1.0
            c[rows, 1 + ia] = -(1.0 - ss)
            c[rows, 1 + ib] = -ss
            inner = (ss > 0.0) & (ss < 1.0)
            Cw[rows[inner], 1 + ia, 0] = 1.0
            Cw[rows[inner], 1 + ib, 0] = -1.0
            k[rows[inner]] = 1
    return dict(d=d, c=c, Cw=Cw, k=k)


def edge_edge(a0, a1, b0, b1):
    """Distance between segments [a0,a1] and [b0,b1], all (n,3).

    Returns dict(d, c, Cw, k) over the point order [a0, a1, b0, b1], with
    r = (closest point on a) - (closest point on b).
    """
    a0, a1, b0, b1 = (np.asarray(v, dtype=np.float64).reshape(-1, 3) for v in (a0, a1, b0, b1))
    n = a0.shape[0]
    ea, eb, w0 = a1 - a0, b1 - b0, a0 - b0
    A, B, C = _dot(ea, ea), _dot(ea, eb), _dot(eb, eb)
    Dd, Ee = _dot(ea, w0), _dot(eb, w0)
    det = A * C - B * B
    nonpar = det > PARALLEL_SIN2 * A * C
    with np.errstate(divide="ignore", invalid="ignore"):
        s = (B * Ee - C * Dd) / det
        t = (A * Ee - B * Dd) / det
    inside = nonpar & (s >= 0) & (s <= 1) & (t >= 0) & (t <= 1)

    d = np.empty(n)
    c = np.zeros((n, 4))
    Cw = np.zeros((n, 4, 2))
    k = np.zeros(n, dtype=np.int64)

    ii = inside
    r = w0[ii] + s[ii, None] * ea[ii] - t[ii, None] * eb[ii]
    d[ii] = np.sqrt(_dot(r, r))
    c[ii] = np.stack([1 - s[ii], s[ii], -(1 - t[ii]), -t[ii]], axis=1)
    Cw[ii, :, 0] = [-1.0, 1.0, 0.0, 0.0]
    Cw[ii, :, 1] = [0.0, 0.0, 1.0, -1.0]
    k[ii] = 2

    oo = ~inside
    if np.any(oo):
        idx = np.nonzero(oo)[0]
        A0, A1, B0, B1 = a0[oo], a1[oo], b0[oo], b1[oo]
        # four point-vs-segment subproblems on the boundary of [0,1]^2
        sub = [
            ("a", 0, _point_segment(A0, B0, B1)),   # a0 vs segment b
            ("a", 1, _point_segment(A1, B0, B1)),   # a1 vs segment b
            ("b", 0, _point_segment(B0, A0, A1)),   # b0 vs segment a
            ("b", 1, _point_segment(B1, A0, A1)),   # b1 vs segment a
        ]
        dists = np.stack([sb[2][0] for sb in sub], axis=1)
        best = np.argmin(dists, axis=1)
        for j, (side, end, (dist, sp)) in enumerate(sub):
            sel = best == j
            rows = idx[sel]
            ss = sp[sel]
            d[rows] = dist[sel]
            inner = (ss > 0.0) & (ss < 1.0)
            if side == "a":
                # r = a_end - (b0 + ss (b1 - b0))
                c[rows, end] = 1.0
                c[rows, 2] = -(1.0 - ss)
                c[rows, 3] = -ss
                Cw[rows[inner], 2, 0] = 1.0
                Cw[rows[inner], 3, 0] = -1.0
            else:
                # r = (a0 + ss (a1 - a0)) - b_end
                c[rows, 0] = 1.0 - ss
                c[rows, 1] = ss
                c[rows, 2 + end] = -1.0
                Cw[rows[inner], 0, 0] = -1.0
                Cw[rows[inner], 1, 0] = 1.0
            k[rows[inner]] = 1
    return dict(d=d, c=c, Cw=Cw, k=k)


def distance_derivatives(Z, c, Cw, k):
    """Gradient (n,4,3) and Hessian (n,12,12) of d with respect to the 4 points Z (n,4,3)."""
    Z = np.asarray(Z, dtype=np.float64)
    n = Z.shape[0]
    r = np.einsum("ni,nid->nd", c, Z)
    d = np.sqrt(_dot(r, r))
    nhat = r / d[:, None]
    grad = c[:, :, None] * nhat[:, None, :]
    D = np.einsum("nia,nid->nad", Cw, Z)                       # (n,2,3)
    phi_ww = 2.0 * np.einsum("nad,nbd->nab", D, D)
    for a in range(2):
        unused = k <= a
        phi_ww[unused, a, :] = 0.0
        phi_ww[unused, :, a] = 0.0
        phi_ww[unused, a, a] = 1.0
    inv = np.linalg.inv(phi_ww)
    phi_zw = 2.0 * (Cw[:, :, :, None] * r[:, None, None, :] + c[:, :, None, None] * D[:, None, :, :])
    # phi_zw: (n, 4 points, 2 params, 3 axes)
    I3 = np.eye(3)
    H2 = 2.0 * np.einsum("ni,nj,de->nidje", c, c, I3)
    H2 = H2 - np.einsum("niad,nab,njbe->nidje", phi_zw, inv, phi_zw)
    H2 = H2.reshape(n, 12, 12)
    gflat = grad.reshape(n, 12)
    Hd = H2 / (2.0 * d[:, None, None]) - np.einsum("ni,nj->nij", gflat, gflat) / d[:, None, None]
    return d, grad, Hd
