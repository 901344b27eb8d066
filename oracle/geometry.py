"""Oracle geometry: rest shape per tet, gel surface primitives, marker embedding,
indenter poses. Test infrastructure only (see package docstring).

Readings:
  * Contact acts between "all surface primitives" (Supp. A, first paragraph);
    here gel-surface primitives against the indenter only. A primitive whose
    vertices are all fixed (bottom face) can never move and is dropped.
  * Markers (Sec. 3.2, last paragraph) are embedded barycentrically in the
    top-face triangle that contains their rest xy; on a tie the lowest
    triangle id wins (the interpolation is continuous, so the result agrees).
"""

from __future__ import annotations

import numpy as np


def quat_to_matrix(q) -> np.ndarray:
    """Rotation matrix of quaternion (w, x, y, z), normalised first."""
    q = np.asarray(q, dtype=np.float64)
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([
        [w * w + x * x - y * y - z * z, 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), w * w - x * x + y * y - z * z, 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), w * w - x * x - y * y + z * z],
    ])


def slerp_pose(p0, p1, tau: float) -> np.ndarray:
    """Pose between p0 and p1: translation linear in tau, rotation by slerp."""
    p0 = np.asarray(p0, dtype=np.float64)
    p1 = np.asarray(p1, dtype=np.float64)
    t = (1.0 - tau) * p0[:3] + tau * p1[:3]
    q0 = p0[3:] / np.linalg.norm(p0[3:])
    q1 = p1[3:] / np.linalg.norm(p1[3:])
    c = float(np.dot(q0, q1))
    if c < 0.0:
        q1, c = -q1, -c
    c = min(c, 1.0)
    theta = np.arccos(c)
    if theta < 1e-12:
        q = (1.0 - tau) * q0 + tau * q1
    else:
        q = (np.sin((1.0 - tau) * theta) * q0 + np.sin(tau * theta) * q1) / np.sin(theta)
    return np.concatenate([t, q / np.linalg.norm(q)])


def rotation_angle_between(p0, p1) -> float:
    """Angle of the relative rotation between the orientations of two poses."""
    q0 = np.asarray(p0[3:], dtype=np.float64)
    q1 = np.asarray(p1[3:], dtype=np.float64)
    c = abs(float(np.dot(q0 / np.linalg.norm(q0), q1 / np.linalg.norm(q1))))
    return 2.0 * np.arccos(min(1.0, c))


class GelGeometry:
    """Rest-shape quantities of a tetrahedral gel.

    Dm_inv[e] = inverse of [X1-X0, X2-X0, X3-X0]; vol[e] = det(Dm)/6 > 0.
    surf_tris / surf_edges / surf_verts: boundary primitives not entirely fixed.
    """

    def __init__(self, X, tets, fixed, markers_xy=None):
        self.X = np.asarray(X, dtype=np.float64)
        self.tets = np.asarray(tets, dtype=np.int64)
        self.fixed = np.asarray(fixed).astype(bool)
        self.n_v = self.X.shape[0]
        Xt = self.X[self.tets]
        Dm = np.stack([Xt[:, 1] - Xt[:, 0], Xt[:, 2] - Xt[:, 0], Xt[:, 3] - Xt[:, 0]], axis=2)
        det = np.linalg.det(Dm)
        if np.any(det <= 0):
            raise ValueError("tet with non-positive rest volume")
        self.vol = det / 6.0
        self.Dm_inv = np.linalg.inv(Dm)
        self._surface()
        self.free = ~self.fixed
        if markers_xy is not None:
            self.embed_markers(markers_xy)

    def _surface(self):
        faces = {}
        # each tet face, oriented outward: opposite-vertex rule on a positive tet
        local = [(1, 2, 3), (0, 3, 2), (0, 1, 3), (0, 2, 1)]
        for t in self.tets:
            for f in local:
                tri = (int(t[f[0]]), int(t[f[1]]), int(t[f[2]]))
                key = tuple(sorted(tri))
                if key in faces:
                    faces[key] = None
                else:
                    faces[key] = tri
        tris = [tri for tri in faces.values() if tri is not None]
        tris = [t for t in tris if not all(self.fixed[list(t)])]
        self.surf_tris = np.array(sorted(tris), dtype=np.int64).reshape(-1, 3)
        all_tris = [tri for tri in faces.values() if tri is not None]
        edges = set()
        for a, b, c in all_tris:
            for u, v in ((a, b), (b, c), (c, a)):
                edges.add((min(u, v), max(u, v)))
        edges = [e for e in edges if not (self.fixed[e[0]] and self.fixed[e[1]])]
        self.surf_edges = np.array(sorted(edges), dtype=np.int64).reshape(-1, 2)
        verts = sorted({v for tri in all_tris for v in tri})
        verts = [v for v in verts if not self.fixed[v]]
        self.surf_verts = np.array(verts, dtype=np.int64)
        self.boundary_tris_all = np.array(sorted(all_tris), dtype=np.int64).reshape(-1, 3)

    def embed_markers(self, markers_xy):
        """Barycentric embedding of marker xy in the top-face triangles."""
        ztop = self.X[:, 2].max()
        T = self.surf_tris
        top = T[np.all(np.abs(self.X[T][:, :, 2] - ztop) < 1e-9, axis=1)]
        tris, weights = [], []
        for m in np.asarray(markers_xy, dtype=np.float64):
            found = None
            for t in top:
                A = self.X[t[0], :2]
                B = self.X[t[1], :2]
                C = self.X[t[2], :2]
                M = np.array([B - A, C - A]).T
                st = np.linalg.solve(M, m - A)
                w = np.array([1.0 - st.sum(), st[0], st[1]])
                if np.all(w >= -1e-12):
                    found = (t, w)
                    break
            if found is None:
                raise ValueError(f"marker {m} outside the top face")
            tris.append(found[0])
            weights.append(found[1])
        self.marker_tris = np.array(tris, dtype=np.int64)
        self.marker_w = np.array(weights, dtype=np.float64)
        self.marker_ref = np.einsum("mk,mkd->md", self.marker_w, self.X[self.marker_tris])

    def markers(self, x) -> np.ndarray:
        """Marker displacement u_m = sum_i w_mi (x_i - X_i), shape (n_m, 3)."""
        u = x - self.X
        return np.einsum("mk,mkd->md", self.marker_w, u[self.marker_tris])


class IndenterGeometry:
    """Rigid indenter: local vertices, triangles and unique edges."""

    def __init__(self, Y, tris):
        self.Y = np.asarray(Y, dtype=np.float64)
        self.tris = np.asarray(tris, dtype=np.int64)
        edges = set()
        for a, b, c in self.tris:
            for u, v in ((a, b), (b, c), (c, a)):
                edges.add((min(int(u), int(v)), max(int(u), int(v))))
        self.edges = np.array(sorted(edges), dtype=np.int64)
        self.r_max = float(np.linalg.norm(self.Y, axis=1).max())

    def world(self, pose) -> np.ndarray:
        R = quat_to_matrix(pose[3:])
        return self.Y @ R.T + np.asarray(pose[:3], dtype=np.float64)
