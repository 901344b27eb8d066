"""Oracle log-barrier b(d) and friction mollifier f(s). Test infrastructure only.

Barrier (Supp. A, eq. ipc_energy and the sentence after it): a C^2 log barrier
that activates below dhat. Reading: the IPC barrier on the unsquared distance,
    b(d) = -(d - dhat)^2 ln(d / dhat)   for 0 < d < dhat,
    b(d) = 0 for d >= dhat,  b(d) = +inf for d <= 0.

Mollifier (Supp. A, eq. friction_mollifier):
    f(s) = -s^3 / (3 eps^2) + s^2 / eps + eps / 3   for s < eps,   f(s) = s otherwise.

Edge-edge mollifier (option; Supp. A follows IPC, whose edge-edge barrier is
multiplied by a mollifier of the edges' cross product so that it stays smooth
as two edges turn parallel, where their closest points jump):
    m(c) = -c^2 / eps_x^2 + 2 c / eps_x   for c < eps_x,   m(c) = 1 otherwise,
with c = |a x b|^2 for the edge vectors a, b and eps_x = 1e-3 |a_rest|^2 |b_rest|^2
(reading: the rest lengths of the gel edge and of the rigid indenter edge).
m(0) = 0 and m is C^1 at eps_x (m = 1, m' = 0 there).
"""

from __future__ import annotations

import numpy as np


def barrier(d, dhat):
    d = np.asarray(d, dtype=np.float64)
    out = np.zeros_like(d)
    out[d <= 0] = np.inf
    m = (d > 0) & (d < dhat)
    dm = d[m]
    out[m] = -(dm - dhat) ** 2 * np.log(dm / dhat)
    return out


def barrier_d1(d, dhat):
    d = np.asarray(d, dtype=np.float64)
    out = np.zeros_like(d)
    m = (d > 0) & (d < dhat)
    dm = d[m]
    out[m] = -2.0 * (dm - dhat) * np.log(dm / dhat) - (dm - dhat) ** 2 / dm
    return out


def barrier_d2(d, dhat):
    d = np.asarray(d, dtype=np.float64)
    out = np.zeros_like(d)
    m = (d > 0) & (d < dhat)
    dm = d[m]
    out[m] = -2.0 * np.log(dm / dhat) - 4.0 * (dm - dhat) / dm + (dm - dhat) ** 2 / dm ** 2
    return out


def mollifier(s, eps):
    s = np.asarray(s, dtype=np.float64)
    return np.where(s < eps, -s ** 3 / (3 * eps ** 2) + s ** 2 / eps + eps / 3.0, s)


def mollifier_d1(s, eps):
    s = np.asarray(s, dtype=np.float64)
    return np.where(s < eps, -s ** 2 / eps ** 2 + 2.0 * s / eps, 1.0)


def mollifier_d2(s, eps):
    s = np.asarray(s, dtype=np.float64)
    return np.where(s < eps, -2.0 * s / eps ** 2 + 2.0 / eps, 0.0)


EDGE_MOLLIFIER_REL = 1e-3


def edge_mollifier(c, eps):
    c = np.asarray(c, dtype=np.float64)
    return np.where(c < eps, -c * c / eps ** 2 + 2.0 * c / eps, 1.0)


def edge_mollifier_d1(c, eps):
    c = np.asarray(c, dtype=np.float64)
    return np.where(c < eps, -2.0 * c / eps ** 2 + 2.0 / eps, 0.0)


def edge_mollifier_d2(c, eps):
    c = np.asarray(c, dtype=np.float64)
    return np.where(c < eps, -2.0 / eps ** 2, 0.0)


def edge_cross_derivatives(Z):
    """c = |a x b|^2 with a = z1 - z0, b = z3 - z2 for the points Z (n, 4, 3), and
    its gradient (n, 12) and Hessian (n, 12, 12) with respect to the 4 points.
    With c = |a|^2 |b|^2 - (a.b)^2: dc/da = 2 |b|^2 a - 2 (a.b) b,
    dc/db = 2 |a|^2 b - 2 (a.b) a, d2c/da2 = 2 |b|^2 I - 2 b b^T,
    d2c/db2 = 2 |a|^2 I - 2 a a^T, d2c/da db = 4 a b^T - 2 b a^T - 2 (a.b) I."""
    Z = np.asarray(Z, dtype=np.float64)
    n = Z.shape[0]
    a = Z[:, 1] - Z[:, 0]
    b = Z[:, 3] - Z[:, 2]
    aa = np.einsum("nd,nd->n", a, a)
    bb = np.einsum("nd,nd->n", b, b)
    ab = np.einsum("nd,nd->n", a, b)
    c = aa * bb - ab * ab
    ga = 2.0 * bb[:, None] * a - 2.0 * ab[:, None] * b
    gb = 2.0 * aa[:, None] * b - 2.0 * ab[:, None] * a
    grad = np.concatenate([-ga, ga, -gb, gb], axis=1)
    I3 = np.eye(3)[None]
    Haa = 2.0 * bb[:, None, None] * I3 - 2.0 * np.einsum("ni,nj->nij", b, b)
    Hbb = 2.0 * aa[:, None, None] * I3 - 2.0 * np.einsum("ni,nj->nij", a, a)
    Hab = 4.0 * np.einsum("ni,nj->nij", a, b) - 2.0 * np.einsum("ni,nj->nij", b, a) - 2.0 * ab[:, None, None] * I3
    # a = z1 - z0, b = z3 - z2: the point Hessian is S^T [[Haa, Hab], [Hab^T, Hbb]] S
    sa = np.array([-1.0, 1.0, 0.0, 0.0])
    sb = np.array([0.0, 0.0, -1.0, 1.0])
    H = (np.einsum("i,j,nde->nidje", sa, sa, Haa) + np.einsum("i,j,nde->nidje", sb, sb, Hbb)
         + np.einsum("i,j,nde->nidje", sa, sb, Hab) + np.einsum("i,j,nde->nidje", sb, sa, Hab.transpose(0, 2, 1)))
    return c, grad, H.reshape(n, 12, 12)

