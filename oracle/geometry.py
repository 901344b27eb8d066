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


# ---------------------------------------------------------------------------
# Indenter motion from a physics engine (Sec. 3.3, Integrating to Physics
# Engine): per engine step the object's pose relative to the sensor at its
# start and end gives a constant linear and angular velocity.
# ---------------------------------------------------------------------------
def _qmul(a, b):
    w1, x1, y1, z1 = np.moveaxis(a, -1, 0)
    w2, x2, y2, z2 = np.moveaxis(b, -1, 0)
    return np.stack([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2], axis=-1)


def relative_velocity(p0, p1, dt):
    """Constant linear and world-frame angular velocity (rad/s) carrying pose p0
    to p1 in time dt: v = (t1 - t0) / dt, w = axis * angle / dt of the shortest
    rotation q1 q0^-1. Shapes (..., 7) -> ((..., 3), (..., 3))."""
    p0 = np.asarray(p0, dtype=np.float64)
    p1 = np.asarray(p1, dtype=np.float64)
    if not dt > 0:
        raise ValueError("dt must be positive")
    v = (p1[..., :3] - p0[..., :3]) / dt
    q0 = p0[..., 3:] / np.linalg.norm(p0[..., 3:], axis=-1, keepdims=True)
    q1 = p1[..., 3:] / np.linalg.norm(p1[..., 3:], axis=-1, keepdims=True)
    dq = _qmul(q1, q0 * np.array([1.0, -1.0, -1.0, -1.0]))
    dq = np.where(dq[..., :1] < 0, -dq, dq)
    s = np.linalg.norm(dq[..., 1:], axis=-1, keepdims=True)
    angle = 2.0 * np.arctan2(s, dq[..., :1])
    axis = np.divide(dq[..., 1:], s, out=np.zeros_like(dq[..., 1:]), where=s > 0)
    return v, axis * angle / dt


def advance_pose(p0, v, w, tau):
    """Pose after moving p0 for time tau at linear velocity v and world-frame
    angular velocity w: t = t0 + v tau, q = exp(w tau) q0."""
    p0 = np.asarray(p0, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    t = p0[..., :3] + v * tau
    rate = np.linalg.norm(w, axis=-1, keepdims=True)
    half = 0.5 * rate * tau
    axis = np.divide(w, rate, out=np.zeros_like(w), where=rate > 0)
    dq = np.concatenate([np.cos(half), np.sin(half) * axis], axis=-1)
    q = _qmul(dq, p0[..., 3:] / np.linalg.norm(p0[..., 3:], axis=-1, keepdims=True))
    return np.concatenate([t, q / np.linalg.norm(q, axis=-1, keepdims=True)], axis=-1)


def top_face_vertices(X, surface_tris):
    """Ascending ids of the vertices of the boundary triangles that lie on the
    top face (largest z)."""
    X = np.asarray(X, dtype=np.float64)
    tris = np.asarray(surface_tris)
    zt = X[:, 2].max()
    on = np.all(np.abs(X[tris, 2] - zt) <= 1e-9 * (1.0 + abs(zt)), axis=1)
    return np.unique(tris[on])


def knn_marker_map(X, top_vertices, markers_xy, k=3, power=1.0):
    """The k-nearest-neighbour marker map (Sec. 3.2: marker displacements from the
    k nearest nodes of the initial mesh, with weights; k and the weights are not
    given). Reading: the k <= 3 top-face vertices nearest to the marker's rest xy
    (ties by vertex id) with weights 1 / distance^power summing to 1; a marker on
    a vertex (within 1e-12 mm) takes that vertex alone. Returns vertex and weight
    arrays [n_m][3]; unused slots repeat the nearest vertex with weight 0."""
    X = np.asarray(X, dtype=np.float64)
    top = np.sort(np.asarray(top_vertices, dtype=np.int64))
    M = np.asarray(markers_xy, dtype=np.float64).reshape(-1, 2)
    vertex = np.zeros((len(M), 3), dtype=np.int32)
    weight = np.zeros((len(M), 3))
    for m, (mx, my) in enumerate(M):
        d = np.hypot(X[top, 0] - mx, X[top, 1] - my)
        order = sorted(range(len(top)), key=lambda j: (d[j], top[j]))[:k]
        vertex[m, :] = top[order[0]]
        if d[order[0]] <= 1e-12:
            weight[m, 0] = 1.0
            continue
        w = np.array([1.0 / d[j] ** power for j in order])
        vertex[m, :k] = top[order]
        weight[m, :k] = w / w.sum()
    return vertex, weight

