"""Oracle per-step energy Pi(x) with its derivatives. Test infrastructure only.

Quasi-static reading of Supp. A, eq. ipc_energy: the inertia term is dropped
and h^2 Psi becomes Psi, so each load step is the equilibrium
    x*_s = argmin_x  Pi_s(x) = Psi(x) + kappa sum_{k in C(x)} b(d_k(x)) + D_s(x)
over the free vertices (the bottom face stays at rest).

C(x) holds every gel-surface/indenter pair closer than dhat: gel vertex vs
indenter triangle, indenter vertex vs gel triangle, gel edge vs indenter edge.
With the option self_contact it also holds every pair of gel surface
primitives closer than dhat that share no vertex: gel vertex vs gel triangle
and gel edge vs gel edge (Supp. A applies the barrier between all surface
primitives). Shared-feature duplicates are kept (plain IPC enumeration). With
the option ee_mollifier the edge-edge terms are kappa m(c) b(d), m the
edge-edge mollifier of barrier.py (smooth as the edges turn parallel);
without it kappa b(d). Self-contact pairs carry no friction (reading).

Friction (Supp. A, eqs. friction_energy, friction_mollifier) is lagged once per
load step at the previous equilibrium (x_{s-1}, q_{s-1}): for each pair active
there, lambda_k = -kappa b'(d_k), the closest-point weights a_k (gel side) and
c_k (indenter side), n_k the unit vector from the indenter's closest point to
the gel's, T_k = I - n_k n_k^T, and
    Delta_k(x) = sum_i a_ki (x_i - x_{s-1,i}) - sum_j c_kj (y_j(q) - y_j(q_{s-1})),
    D_s(x) = mu_f sum_k lambda_k f(|T_k Delta_k(x)|).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .barrier import (EDGE_MOLLIFIER_REL, barrier, barrier_d1, barrier_d2, edge_cross_derivatives,
                      edge_mollifier, edge_mollifier_d1, edge_mollifier_d2, mollifier, mollifier_d1,
                      mollifier_d2)
from .distance import distance_derivatives, edge_edge, point_triangle
from .elastic import (element_energy, element_gradient, element_hessian, lame, psd_project)
from .geometry import GelGeometry, IndenterGeometry

VF, FV, EE = 0, 1, 2
GVF, GEE = 3, 4      # gel vertex vs gel triangle, gel edge vs gel edge (self-contact)
EDGE_KINDS = (EE, GEE)


def _aabb(P):
    """P: (n, m, 3) primitive points -> (lo, hi)."""
    return P.min(axis=1), P.max(axis=1)


def _pairs_by_aabb(lo_a, hi_a, lo_b, hi_b, thr, chunk=4096):
    """All (i, j) whose per-axis box gaps are all < thr (necessary for distance < thr)."""
    out_i, out_j = [], []
    if len(lo_a) == 0 or len(lo_b) == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    for s in range(0, len(lo_a), chunk):
        la, ha = lo_a[s:s + chunk], hi_a[s:s + chunk]
        gap = np.maximum(la[:, None, :] - hi_b[None, :, :], lo_b[None, :, :] - ha[:, None, :])
        ok = np.all(gap < thr, axis=2)
        i, j = np.nonzero(ok)
        out_i.append(i + s)
        out_j.append(j)
    return np.concatenate(out_i), np.concatenate(out_j)


class StepProblem:
    """Energy of one load step at a fixed indenter pose (and fixed friction lag)."""

    def __init__(self, gel: GelGeometry, ind: IndenterGeometry, E, nu, mu_f=0.0,
                 eps_v=1e-3, dhat=0.05, kappa=1e3, ee_mollifier=False, self_contact=False):
        self.gel, self.ind = gel, ind
        self.ee_mollifier = bool(ee_mollifier)
        self.self_contact = bool(self_contact)
        self.mu, self.lam = lame(E, nu)
        self.mu_f, self.eps_v, self.dhat, self.kappa = mu_f, eps_v, dhat, kappa
        self.nv = gel.n_v
        # natural energy scale mu * total volume: the rounding guard of the
        # line-search energy test is a fixed multiple of it
        self.energy_ref = float(self.mu * gel.vol.sum())
        # preconditioner floor: a fixed fraction of the largest rest-state
        # stiffness mu * sum_e V_e |g_i|^2 over free vertices
        G = np.concatenate([-gel.Dm_inv.sum(axis=1, keepdims=True), gel.Dm_inv], axis=1)
        s = np.zeros(gel.n_v)
        np.add.at(s, gel.tets, gel.vol[:, None] * np.einsum("nid,nid->ni", G, G))
        self.diag_scale = float(self.mu * s[~gel.fixed].max())
        self.pose = None
        self.Yw = None
        self.lag = None
        self.inertia = None

    # ---------------------------------------------------------------- inertia
    def set_inertia(self, w, xhat):
        """Dynamic form (Supp. A, eq. ipc_energy with its inertia term): adds
        1/2 sum_v w_v |x_v - xhat_v|^2, w_v = m_v / h^2 with the lumped mass m_v
        and xhat = x^t + h v^t the inertial prediction. None turns it off."""
        self.inertia = None if w is None else (np.asarray(w, dtype=np.float64),
                                               np.asarray(xhat, dtype=np.float64))

    def _inertia_energy(self, x):
        if self.inertia is None:
            return 0.0
        w, xh = self.inertia
        free = ~self.gel.fixed
        r = (x - xh)[free]
        return 0.5 * float(np.sum(w[free] * np.einsum("nd,nd->n", r, r)))

    # ---------------------------------------------------------------- pose / lag
    def set_pose(self, pose):
        self.pose = np.asarray(pose, dtype=np.float64)
        self.Yw = self.ind.world(self.pose)

    def set_lag(self, x_prev, pose_prev):
        """Friction lag at the previous equilibrium (x_{s-1}, q_{s-1})."""
        if self.mu_f == 0.0:
            self.lag = None
            return
        Yp = self.ind.world(pose_prev)
        pairs = self.candidates(x_prev, self.dhat, Yw=Yp)
        res = self.pair_geometry(x_prev, pairs, Yw=Yp)
        act = (res["d"] < self.dhat) & (pairs["kind"] < GVF)   # self-contact pairs: no friction
        idx, kind = pairs["idx"][act], pairs["kind"][act]
        d, c = res["d"][act], res["c"][act]
        Z = res["Z"][act]
        sign = np.where(kind == FV, -1.0, 1.0)
        r = np.einsum("ni,nid->nd", c, Z)
        nvec = sign[:, None] * r / d[:, None]
        gel_pt = idx < self.nv
        a = np.where(gel_pt, sign[:, None] * c, 0.0)
        b = np.where(gel_pt, 0.0, -sign[:, None] * c)
        lam = -self.kappa * barrier_d1(d, self.dhat)
        self.lag = dict(idx=idx, a=a, b=b, n=nvec, lam=lam, x_prev=x_prev.copy(),
                        Y_prev=Yp)

    # ---------------------------------------------------------------- contact
    def _points(self, x, Yw):
        return np.concatenate([x, Yw], axis=0)

    def candidates(self, x, thr, Yw=None):
        """Pairs whose closed primitives may be closer than thr (exact AABB filter)."""
        Yw = self.Yw if Yw is None else Yw
        g, ind, nv = self.gel, self.ind, self.nv
        ilo, ihi = Yw.min(axis=0), Yw.max(axis=0)
        out_idx, out_kind = [], []

        def near_ind(P):  # gel primitives whose box is within thr of the indenter box
            lo, hi = _aabb(P)
            gap = np.maximum(lo - ihi, ilo - hi)
            return np.all(gap < thr, axis=1)

        # gel vertex vs indenter triangle
        sv = g.surf_verts
        Pv = x[sv][:, None, :]
        mv = near_ind(Pv)
        sv = sv[mv]
        if len(sv):
            T = Yw[ind.tris]
            i, j = _pairs_by_aabb(x[sv], x[sv], *_aabb(T), thr)
            idx = np.stack([sv[i], nv + ind.tris[j, 0], nv + ind.tris[j, 1], nv + ind.tris[j, 2]], 1)
            out_idx.append(idx)
            out_kind.append(np.full(len(i), VF))
        # indenter vertex vs gel triangle
        st = g.surf_tris
        Pt = x[st]
        mt = near_ind(Pt)
        st = st[mt]
        if len(st):
            lo, hi = _aabb(x[st])
            i, j = _pairs_by_aabb(lo, hi, Yw, Yw, thr)
            idx = np.stack([nv + j, st[i, 0], st[i, 1], st[i, 2]], 1)
            out_idx.append(idx)
            out_kind.append(np.full(len(i), FV))
        # gel edge vs indenter edge
        se = g.surf_edges
        Pe = x[se]
        me = near_ind(Pe)
        se = se[me]
        if len(se):
            lo, hi = _aabb(x[se])
            ie = ind.edges
            lo2, hi2 = _aabb(Yw[ie])
            i, j = _pairs_by_aabb(lo, hi, lo2, hi2, thr)
            idx = np.stack([se[i, 0], se[i, 1], nv + ie[j, 0], nv + ie[j, 1]], 1)
            out_idx.append(idx)
            out_kind.append(np.full(len(i), EE))
        if self.self_contact:
            # gel surface vertex vs gel surface triangle not containing it
            sv, st = g.surf_verts, g.surf_tris
            if len(sv) and len(st):
                lo, hi = _aabb(x[st])
                i, j = _pairs_by_aabb(x[sv], x[sv], lo, hi, thr)
                keep = np.all(st[j] != sv[i][:, None], axis=1)
                i, j = i[keep], j[keep]
                out_idx.append(np.stack([sv[i], st[j, 0], st[j, 1], st[j, 2]], 1))
                out_kind.append(np.full(len(i), GVF))
            # gel surface edge pairs (each unordered pair once) sharing no vertex
            se = g.surf_edges
            if len(se) > 1:
                lo, hi = _aabb(x[se])
                i, j = _pairs_by_aabb(lo, hi, lo, hi, thr)
                keep = (i < j) & np.all(se[i][:, :, None] != se[j][:, None, :], axis=(1, 2))
                i, j = i[keep], j[keep]
                out_idx.append(np.stack([se[i, 0], se[i, 1], se[j, 0], se[j, 1]], 1))
                out_kind.append(np.full(len(i), GEE))
        if out_idx:
            idx = np.concatenate(out_idx).astype(np.int64)
            kind = np.concatenate(out_kind)
        else:
            idx = np.zeros((0, 4), np.int64)
            kind = np.zeros(0, np.int64)
        return dict(idx=idx, kind=kind)

    def pair_geometry(self, x, pairs, Yw=None):
        Yw = self.Yw if Yw is None else Yw
        pts = self._points(x, Yw)
        idx, kind = pairs["idx"], pairs["kind"]
        n = len(idx)
        Z = pts[idx] if n else np.zeros((0, 4, 3))
        d = np.zeros(n)
        c = np.zeros((n, 4))
        Cw = np.zeros((n, 4, 2))
        k = np.zeros(n, np.int64)
        ee = np.isin(kind, EDGE_KINDS)
        pt = ~ee
        if np.any(pt):
            r = point_triangle(Z[pt, 0], Z[pt, 1], Z[pt, 2], Z[pt, 3])
            d[pt], c[pt], Cw[pt], k[pt] = r["d"], r["c"], r["Cw"], r["k"]
        if np.any(ee):
            r = edge_edge(Z[ee, 0], Z[ee, 1], Z[ee, 2], Z[ee, 3])
            d[ee], c[ee], Cw[ee], k[ee] = r["d"], r["c"], r["Cw"], r["k"]
        return dict(d=d, c=c, Cw=Cw, k=k, Z=Z)

    def active(self, x):
        pairs = self.candidates(x, self.dhat)
        res = self.pair_geometry(x, pairs)
        act = res["d"] < self.dhat
        return {"idx": pairs["idx"][act], "kind": pairs["kind"][act]}, \
            {k: v[act] for k, v in res.items()}

    def d_min(self, x, thr=None):
        thr = self.dhat if thr is None else thr
        pairs = self.candidates(x, thr)
        if len(pairs["idx"]) == 0:
            return np.inf
        return float(self.pair_geometry(x, pairs)["d"].min())

    def pair_terms(self, pairs, res, order=2):
        """Per active pair: the barrier potential kappa b(d) (edge-edge pairs:
        kappa m(c) b(d) with the mollifier on), its gradient (n, 12) and Hessian
        (n, 12, 12) with respect to the pair's four points (gel and indenter),
        up to derivative `order`."""
        d = res["d"]
        n = len(d)
        val = self.kappa * barrier(d, self.dhat)
        if order == 0 and not self.ee_mollifier:
            return val, None, None
        _, grad, Hd = distance_derivatives(res["Z"], res["c"], res["Cw"], res["k"])
        b1 = barrier_d1(d, self.dhat)
        g = grad.reshape(n, 12)
        G = self.kappa * b1[:, None] * g
        H = None
        if order >= 2:
            b2 = barrier_d2(d, self.dhat)
            H = self.kappa * (b2[:, None, None] * np.einsum("ni,nj->nij", g, g) + b1[:, None, None] * Hd)
        if self.ee_mollifier:
            ee = np.nonzero(np.isin(pairs["kind"], EDGE_KINDS))[0]
            if len(ee):
                idx = pairs["idx"][ee]
                # rest positions: the gel's, or the indenter's local ones
                rest = lambda i: np.where((i < self.nv)[:, None], self.gel.X[np.minimum(i, self.nv - 1)],
                                          self.ind.Y[np.maximum(i - self.nv, 0)])
                ar = rest(idx[:, 1]) - rest(idx[:, 0])
                br = rest(idx[:, 3]) - rest(idx[:, 2])
                eps = EDGE_MOLLIFIER_REL * np.einsum("nd,nd->n", ar, ar) * np.einsum("nd,nd->n", br, br)
                c, gc, Hc = edge_cross_derivatives(res["Z"][ee])
                m, m1, m2 = edge_mollifier(c, eps), edge_mollifier_d1(c, eps), edge_mollifier_d2(c, eps)
                b = barrier(d[ee], self.dhat)
                be1 = b1[ee]
                ge = g[ee]
                if H is not None:
                    He = H[ee]
                    H[ee] = (m[:, None, None] * He
                             + self.kappa * (m1 * be1)[:, None, None] * (np.einsum("ni,nj->nij", gc, ge)
                                                                         + np.einsum("ni,nj->nij", ge, gc))
                             + self.kappa * (m2 * b)[:, None, None] * np.einsum("ni,nj->nij", gc, gc)
                             + self.kappa * (m1 * b)[:, None, None] * Hc)
                G[ee] = m[:, None] * G[ee] + self.kappa * (m1 * b)[:, None] * gc
                val[ee] = m * val[ee]
        return val, G, H

    # ---------------------------------------------------------------- friction
    def _friction_terms(self, x):
        L = self.lag
        gel_pt = L["idx"] < self.nv
        gid = np.where(gel_pt, L["idx"], 0)
        yid = np.where(gel_pt, 0, L["idx"] - self.nv)
        dx = (x[gid] - L["x_prev"][gid]) * gel_pt[:, :, None]
        dy = (self.Yw[yid] - L["Y_prev"][yid]) * (~gel_pt)[:, :, None]
        Delta = np.einsum("ni,nid->nd", L["a"], dx) - np.einsum("ni,nid->nd", L["b"], dy)
        nv_ = L["n"]
        TD = Delta - np.einsum("nd,nd->n", nv_, Delta)[:, None] * nv_
        s = np.linalg.norm(TD, axis=1)
        return gel_pt, gid, TD, s

    # ---------------------------------------------------------------- energy
    def energy(self, x):
        g = self.gel
        Ee = element_energy(x, g.tets, g.Dm_inv, g.vol, self.mu, self.lam)
        if not np.all(np.isfinite(Ee)):
            return np.inf
        pairs, res = self.active(x)
        if np.any(res["d"] <= 0):
            return np.inf
        Eb = self.pair_terms(pairs, res, order=0)[0].sum()
        Ef = 0.0
        if self.lag is not None and len(self.lag["lam"]):
            _, _, _, s = self._friction_terms(x)
            Ef = self.mu_f * np.sum(self.lag["lam"] * mollifier(s, self.eps_v))
        return float(Ee.sum() + Eb + Ef + self._inertia_energy(x))

    def energy_parts(self, x):
        g = self.gel
        Ee = element_energy(x, g.tets, g.Dm_inv, g.vol, self.mu, self.lam).sum()
        pairs, res = self.active(x)
        Eb = self.pair_terms(pairs, res, order=0)[0].sum()
        Ef = 0.0
        if self.lag is not None and len(self.lag["lam"]):
            _, _, _, s = self._friction_terms(x)
            Ef = self.mu_f * np.sum(self.lag["lam"] * mollifier(s, self.eps_v))
        return float(Ee), float(Eb), float(Ef)

    def gradient(self, x):
        g = self.gel
        out = np.zeros_like(x)
        ge = element_gradient(x, g.tets, g.Dm_inv, g.vol, self.mu, self.lam)
        np.add.at(out, g.tets, ge)
        pairs, res = self.active(x)
        if len(pairs["idx"]):
            _, G, _ = self.pair_terms(pairs, res, order=1)
            gel_pt = pairs["idx"] < self.nv
            contrib = G.reshape(-1, 4, 3) * gel_pt[:, :, None]
            np.add.at(out, np.where(gel_pt, pairs["idx"], 0), contrib)
        if self.lag is not None and len(self.lag["lam"]):
            gel_pt, gid, TD, s = self._friction_terms(x)
            with np.errstate(divide="ignore", invalid="ignore"):
                fos = np.where(s < self.eps_v, -s / self.eps_v ** 2 + 2.0 / self.eps_v,
                               1.0 / np.where(s > 0, s, 1.0))
            w = self.mu_f * self.lag["lam"] * fos
            contrib = (w[:, None, None] * self.lag["a"][:, :, None] * TD[:, None, :]) * gel_pt[:, :, None]
            np.add.at(out, gid, contrib)
        if self.inertia is not None:
            wi, xh = self.inertia
            out += wi[:, None] * (x - xh)
        out[self.gel.fixed] = 0.0
        return out

    def _blocks(self, x, project):
        """Yield (term, dof_index (n,m), blocks (n,m,m)) for every Hessian
        contribution; term is 'elastic', 'barrier' or 'friction'."""
        g = self.gel
        He = element_hessian(x, g.tets, g.Dm_inv, g.vol, self.mu, self.lam)
        if project:
            He = psd_project(He)
        dof = (3 * g.tets[:, :, None] + np.arange(3)[None, None, :]).reshape(-1, 12)
        yield "elastic", dof, He
        pairs, res = self.active(x)
        if len(pairs["idx"]):
            _, _, Hb = self.pair_terms(pairs, res, order=2)
            gel_pt = pairs["idx"] < self.nv
            mask = np.repeat(gel_pt, 3, axis=1).astype(np.float64)
            Hb = Hb * mask[:, :, None] * mask[:, None, :]
            if project:
                Hb = psd_project(Hb)
            dof = (3 * np.where(gel_pt, pairs["idx"], 0)[:, :, None] + np.arange(3)).reshape(-1, 12)
            yield "barrier", dof, Hb
        if self.lag is not None and len(self.lag["lam"]):
            gel_pt, gid, TD, s = self._friction_terms(x)
            eps = self.eps_v
            nvec = self.lag["n"]
            T = np.eye(3)[None] - np.einsum("ni,nj->nij", nvec, nvec)
            with np.errstate(divide="ignore", invalid="ignore"):
                uhat = np.where(s[:, None] > 0, TD / np.where(s > 0, s, 1.0)[:, None], 0.0)
                fos = np.where(s < eps, -s / eps ** 2 + 2.0 / eps, 1.0 / np.where(s > 0, s, 1.0))
                corr = np.where(s < eps, -s / eps ** 2, -1.0 / np.where(s > 0, s, 1.0))
            HD = fos[:, None, None] * T + corr[:, None, None] * np.einsum("ni,nj->nij", uhat, uhat)
            HD = (self.mu_f * self.lag["lam"])[:, None, None] * HD
            a = self.lag["a"] * gel_pt
            Hf = np.einsum("ni,nj,nde->nidje", a, a, HD).reshape(-1, 12, 12)
            if project:
                Hf = psd_project(Hf)
            dof = (3 * gid[:, :, None] + np.arange(3)).reshape(-1, 12)
            yield "friction", dof, Hf
        if self.inertia is not None:
            wi, _ = self.inertia
            free = np.nonzero(~g.fixed)[0]
            dof = 3 * free[:, None] + np.arange(3)[None, :]
            yield "inertia", dof, wi[free][:, None, None] * np.eye(3)[None]

    def hessian(self, x, project=True):
        n = 3 * self.nv
        rows, cols, vals = [], [], []
        for _, dof, H in self._blocks(x, project):
            m = dof.shape[1]
            rows.append(np.repeat(dof, m, axis=1).ravel())
            cols.append(np.tile(dof, (1, m)).ravel())
            vals.append(H.reshape(len(H), -1).ravel())
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(n, n))

    def diag(self, x):
        """Exact (unprojected) diagonal of the Hessian, (N_v, 3)."""
        out = np.zeros(3 * self.nv)
        for _, dof, H in self._blocks(x, project=False):
            np.add.at(out, dof, np.einsum("nii->ni", H))
        return out.reshape(-1, 3)

    def precond_diag(self, x):
        """Diagonal of the Jacobi preconditioner P = diag(H)^-1 (Supp. A), (N_v, 3):
        the exact diagonal with each contact pair's contribution to an entry
        clamped at zero. For a close pair kappa b'(d) d^2d/dx^2 is negative in the
        directions tangent to the contact, and outweighs kappa b''(d) (dd/dx)^2
        there, so the exact entry can be negative, which a Jacobi preconditioner
        cannot use. Elastic and friction contributions are kept as they are."""
        out = np.zeros(3 * self.nv)
        for term, dof, H in self._blocks(x, project=False):
            dd = np.einsum("nii->ni", H)
            if term == "barrier":
                dd = np.maximum(dd, 0.0)
            np.add.at(out, dof, dd)
        return out.reshape(-1, 3)

    def curvature(self, x, p):
        """p^T H(x) p with the exact Hessian."""
        pf = np.asarray(p, dtype=np.float64).ravel()
        tot = 0.0
        for _, dof, H in self._blocks(x, project=False):
            pv = pf[dof]
            tot += float(np.einsum("ni,nij,nj->", pv, H, pv))
        return tot

    def feasible(self, x):
        g = self.gel
        Ee = element_energy(x, g.tets, g.Dm_inv, g.vol, self.mu, self.lam)
        if not np.all(np.isfinite(Ee)):
            return False
        return self.d_min(x) > 0.0
