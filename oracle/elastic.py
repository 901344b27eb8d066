"""Oracle hyperelastic term Psi(x) = sum_e V_e psi(F_e). Test infrastructure only.

The paper names a "hyperelastic potential Psi" on a tetrahedral mesh
(Supp. A, eq. varopt) without its form. Reading: compressible neo-Hookean
with the log-determinant barrier on volume,
    psi(F) = mu/2 (|F|^2 - 3) - mu ln J + lam/2 (ln J)^2,  J = det F,
and psi = +inf for J <= 0, with the Lame parameters from (E, nu):
    mu = E / (2 (1 + nu)),  lam = E nu / ((1 + nu)(1 - 2 nu)).
F_e = D_s(x) Dm_inv with D_s = [x1-x0, x2-x0, x3-x0].

Everything here is written from these definitions: the gradient is
V P(F) Dm_inv^T with the first Piola stress P = dpsi/dF, and the element
Hessian is V * J^T M J with M the 9x9 second derivative of psi in F and J the
(constant) 9x12 map from vertex positions to F. Diagonal Hessian entries and
p^T H p are read off that full matrix, not from any shortcut.
"""

from __future__ import annotations

import numpy as np


def lame(E, nu):
    mu = E / (2.0 * (1.0 + nu))
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    return mu, lam


def deformation_gradients(x, tets, Dm_inv):
    xt = x[tets]
    Ds = np.stack([xt[:, 1] - xt[:, 0], xt[:, 2] - xt[:, 0], xt[:, 3] - xt[:, 0]], axis=2)
    return Ds @ Dm_inv


def psi(F, mu, lam):
    """Energy density per element; +inf where det F <= 0."""
    J = np.linalg.det(F)
    out = np.full(J.shape, np.inf)
    ok = J > 0
    lnJ = np.log(J[ok])
    I1 = np.einsum("nij,nij->n", F[ok], F[ok])
    out[ok] = 0.5 * mu * (I1 - 3.0) - mu * lnJ + 0.5 * lam * lnJ ** 2
    return out


def first_piola(F, mu, lam):
    """P(F) = mu (F - F^-T) + lam ln J F^-T."""
    J = np.linalg.det(F)
    FinvT = np.transpose(np.linalg.inv(F), (0, 2, 1))
    return mu * (F - FinvT) + lam * np.log(J)[:, None, None] * FinvT


def d2psi_matrix(F, mu, lam):
    """9x9 matrix M with  M[(a,b),(c,d)] = d^2 psi / dF_ab dF_cd.

    From psi: d^2psi[A,B] = mu A:B + (mu - lam ln J) tr(F^-1 A F^-1 B)
                            + lam tr(F^-1 A) tr(F^-1 B).
    With A = e_a e_b^T, B = e_c e_d^T: tr(F^-1 A) = Finv[b,a] and
    tr(F^-1 A F^-1 B) = Finv[b,c] Finv[d,a].
    """
    n = F.shape[0]
    Finv = np.linalg.inv(F)
    lnJ = np.log(np.linalg.det(F))
    I = np.eye(3)
    term1 = mu * np.einsum("ac,bd->abcd", I, I)[None]
    term2 = (mu - lam * lnJ)[:, None, None, None, None] * np.einsum("nbc,nda->nabcd", Finv, Finv)
    term3 = lam * np.einsum("nba,ndc->nabcd", Finv, Finv)
    return (term1 + term2 + term3).reshape(n, 9, 9)


def _dF_dx(Dm_inv):
    """Constant map dF/dx: (n, 9, 12) with columns ordered (vertex i, axis c).

    F_ab = sum_i (x_i - x_0)_a G[i-1, b]  =>  dF_ab/d(x_i)_c = delta_ac Gfull[i, b]
    with Gfull rows g_0 = -(g_1 + g_2 + g_3), g_i = row i-1 of Dm_inv.
    """
    n = Dm_inv.shape[0]
    Gfull = np.concatenate([-Dm_inv.sum(axis=1, keepdims=True), Dm_inv], axis=1)  # (n,4,3)
    Jm = np.zeros((n, 3, 3, 4, 3))
    for a in range(3):
        Jm[:, a, :, :, a] = np.transpose(Gfull, (0, 2, 1))  # [n, b, i]
    return Jm.reshape(n, 9, 12)


def element_energy(x, tets, Dm_inv, vol, mu, lam):
    F = deformation_gradients(x, tets, Dm_inv)
    return vol * psi(F, mu, lam)


def element_gradient(x, tets, Dm_inv, vol, mu, lam):
    """(n, 4, 3) per-element gradient blocks: vertex i gets V P g_i."""
    F = deformation_gradients(x, tets, Dm_inv)
    P = first_piola(F, mu, lam)
    H = vol[:, None, None] * (P @ np.transpose(Dm_inv, (0, 2, 1)))  # columns = V P g_i, i=1..3
    g123 = np.transpose(H, (0, 2, 1))
    g0 = -g123.sum(axis=1, keepdims=True)
    return np.concatenate([g0, g123], axis=1)


def element_hessian(x, tets, Dm_inv, vol, mu, lam):
    """(n, 12, 12) exact element Hessians V J^T M J."""
    F = deformation_gradients(x, tets, Dm_inv)
    M = d2psi_matrix(F, mu, lam)
    Jm = _dF_dx(Dm_inv)
    return vol[:, None, None] * np.einsum("nki,nkl,nlj->nij", Jm, M, Jm)


def psd_project(H):
    """Clamp the eigenvalues of each symmetric block to >= 0."""
    w, Q = np.linalg.eigh(0.5 * (H + np.transpose(H, (0, 2, 1))))
    w = np.maximum(w, 0.0)
    return np.einsum("nij,nj,nkj->nik", Q, w, Q)
