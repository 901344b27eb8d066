"""Rigid indenter surface meshes in their local frames.

Each indenter is a closed, outward-oriented triangle mesh. Its local origin is
the rotation centre used by the pose: world point = R(q) y_local + t.
The shapes follow the workloads the paper uses (a sphere-like indenter, an
end-on cylindrical peg and a hexagonal nut; Sec. 5.2 and the RL tasks of
Sec. 5.3).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Indenter:
    """Y: (n_v, 3) float64 local vertices (mm); tris: (n_f, 3) int32, outward CCW."""

    Y: np.ndarray
    tris: np.ndarray
    name: str = ""

    @property
    def n_verts(self) -> int:
        return int(self.Y.shape[0])

    @property
    def n_tris(self) -> int:
        return int(self.tris.shape[0])


def rigid_set(parts, offsets, name: str = "") -> Indenter:
    """Several closed meshes that move together as one rigid body (a fixture
    with several pins, fingers of one tool): their union, part k shifted by
    offsets[k] in the common local frame."""
    Ys, Ts, n = [], [], 0
    for ind, off in zip(parts, offsets):
        Ys.append(np.asarray(ind.Y, dtype=np.float64) + np.asarray(off, dtype=np.float64))
        Ts.append(np.asarray(ind.tris, dtype=np.int32) + n)
        n += len(ind.Y)
    return Indenter(Y=np.concatenate(Ys), tris=np.concatenate(Ts).astype(np.int32), name=name)


def icosphere(radius: float = 3.0, level: int = 2, yaw: float = 0.0) -> Indenter:
    """Icosahedron subdivided `level` times, vertices projected to the sphere.

    level 2 gives 162 vertices and 320 triangles. Local origin = centre.
    The plane x = 0 is a mirror plane of the base icosahedron; yaw = -pi/4
    turns it into the plane x = y, making the mesh symmetric under x <-> y.
    """
    t = (1.0 + 5.0 ** 0.5) / 2.0
    V = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0),
         (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    F = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
         (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
         (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
         (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    verts = [np.array(v, dtype=np.float64) / np.linalg.norm(v) for v in V]
    faces = list(F)
    for _ in range(level):
        cache = {}

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    Y = np.array(verts) * radius
    c, s_ = np.cos(yaw), np.sin(yaw)
    Y = Y @ np.array([[c, -s_, 0.0], [s_, c, 0.0], [0.0, 0.0, 1.0]]).T
    tris = np.array(faces, dtype=np.int32)
    return Indenter(Y=Y, tris=tris, name=f"sphere_r{radius:g}")


def _disk_rings(n_seg: int, n_rings: int, radius: float, z: float):
    """Centre vertex followed by n_rings rings of n_seg vertices (radii k/n_rings)."""
    pts = [np.array([0.0, 0.0, z])]
    ang = 2.0 * np.pi * np.arange(n_seg) / n_seg
    for k in range(1, n_rings + 1):
        r = radius * k / n_rings
        pts += list(np.stack([r * np.cos(ang), r * np.sin(ang), np.full(n_seg, z)], axis=1))
    return pts


def end_on_peg(radius: float = 4.0, length: float = 10.0, n_seg: int = 64,
               n_rings: int = 8) -> Indenter:
    """Cylindrical peg with its axis along local z, flat pressing cap at z = 0.

    Each cap is a centre fan plus (n_rings - 1) quad rings; the side wall is one
    ring of quads. 64 segments and 8 rings give 1026 vertices, 2048 triangles.
    Local origin = centre of the pressing (bottom) cap.
    """
    bot = _disk_rings(n_seg, n_rings, radius, 0.0)
    top = _disk_rings(n_seg, n_rings, radius, length)
    nb = len(bot)
    Y = np.array(bot + top, dtype=np.float64)

    def ring(k, j, off):  # vertex j of ring k (k >= 1)
        return off + 1 + (k - 1) * n_seg + (j % n_seg)

    tris = []
    for off, up in ((0, False), (nb, True)):
        for j in range(n_seg):
            a, b = ring(1, j, off), ring(1, j + 1, off)
            tris.append((off, a, b) if up else (off, b, a))
        for k in range(1, n_rings):
            for j in range(n_seg):
                a, b = ring(k, j, off), ring(k, j + 1, off)
                c, d = ring(k + 1, j, off), ring(k + 1, j + 1, off)
                if up:
                    tris += [(a, c, d), (a, d, b)]
                else:
                    tris += [(a, d, c), (a, b, d)]
    for j in range(n_seg):
        a, b = ring(n_rings, j, 0), ring(n_rings, j + 1, 0)
        c, d = ring(n_rings, j, nb), ring(n_rings, j + 1, nb)
        tris += [(a, b, d), (a, d, c)]
    return Indenter(Y=Y, tris=np.array(tris, dtype=np.int32), name=f"peg_r{radius:g}")


def hex_nut(across_flats: float = 8.0, thickness: float = 4.7, hole_diameter: float = 4.2,
            n_ang: int = 96, n_rad: int = 6, n_z: int = 2) -> Indenter:
    """Hexagonal nut lying flat: annular faces at z = 0 and z = thickness.

    Around the axis, n_ang angular stations (16 per hexagon side by default)
    join a point on the hole circle to the point on the hexagon at the same
    polar angle; n_rad radial rings split that span, n_z rings split the walls.
    Defaults give 1536 vertices and 3072 triangles (genus 1).
    Local origin = centre of the bottom face.
    """
    R_hex = across_flats / np.sqrt(3.0)  # circumradius
    r_h = hole_diameter / 2.0
    ang = 2.0 * np.pi * np.arange(n_ang) / n_ang
    # point on the hexagon (corners at angles k*60 deg) along direction ang
    sector = np.floor(ang / (np.pi / 3.0))
    a0 = sector * np.pi / 3.0
    c0 = np.stack([np.cos(a0), np.sin(a0)], 1) * R_hex
    c1 = np.stack([np.cos(a0 + np.pi / 3), np.sin(a0 + np.pi / 3)], 1) * R_hex
    d = np.stack([np.cos(ang), np.sin(ang)], 1)
    e = c1 - c0
    # solve c0 + s e = lam d
    det = e[:, 0] * (-d[:, 1]) - e[:, 1] * (-d[:, 0])
    s = ((0 - c0[:, 0]) * (-d[:, 1]) - (0 - c0[:, 1]) * (-d[:, 0])) / det
    outer = c0 + s[:, None] * e
    inner = d * r_h
    verts = []
    idx = {}

    def add(key, p):
        idx[key] = len(verts)
        verts.append(p)

    for face, z in (("b", 0.0), ("t", thickness)):
        for k in range(n_rad + 1):
            w = k / n_rad
            for j in range(n_ang):
                xy = (1 - w) * inner[j] + w * outer[j]
                add((face, k, j), np.array([xy[0], xy[1], z]))
    for wall, src in (("in", inner), ("out", outer)):
        for m in range(1, n_z):
            z = thickness * m / n_z
            for j in range(n_ang):
                add((wall, m, j), np.array([src[j][0], src[j][1], z]))

    def wall_vid(wall, m, j):
        j %= n_ang
        if m == 0:
            return idx[("b", 0 if wall == "in" else n_rad, j)]
        if m == n_z:
            return idx[("t", 0 if wall == "in" else n_rad, j)]
        return idx[(wall, m, j)]

    tris = []
    for face in ("b", "t"):
        for k in range(n_rad):
            for j in range(n_ang):
                a = idx[(face, k, j)]
                b = idx[(face, k, (j + 1) % n_ang)]
                c = idx[(face, k + 1, j)]
                dd = idx[(face, k + 1, (j + 1) % n_ang)]
                if face == "t":  # normal +z: CCW seen from above
                    tris += [(a, c, dd), (a, dd, b)]
                else:
                    tris += [(a, dd, c), (a, b, dd)]
    for wall in ("in", "out"):
        for m in range(n_z):
            for j in range(n_ang):
                a, b = wall_vid(wall, m, j), wall_vid(wall, m, j + 1)
                c, dd = wall_vid(wall, m + 1, j), wall_vid(wall, m + 1, j + 1)
                if wall == "out":  # outward normal points away from the axis
                    tris += [(a, b, dd), (a, dd, c)]
                else:
                    tris += [(a, dd, b), (a, c, dd)]
    return Indenter(Y=np.array(verts, dtype=np.float64), tris=np.array(tris, dtype=np.int32),
                    name=f"nut_af{across_flats:g}")


def flat_plate(half: float = 2.0, z0: float = 0.0, n: int = 3) -> Indenter:
    """A thin square plate [-half,half]^2 x [z0, z0+0.5] on an n x n grid.

    Each grid cell is split along its x = -y diagonal, so the bottom face is
    symmetric under the swap x <-> y (symmetry tests rely on this) and its
    edges are not collinear with the x = y diagonals of a Kuhn gel's top face.
    """
    g = np.linspace(-half, half, n + 1)
    verts, tris = [], []
    for z in (z0, z0 + 0.5):
        for j in range(n + 1):
            for i in range(n + 1):
                verts.append((g[i], g[j], z))
    m = (n + 1) * (n + 1)

    def v(i, j, top):
        return i + (n + 1) * j + (m if top else 0)

    for top in (False, True):
        for j in range(n):
            for i in range(n):
                a, b, c, d = v(i, j, top), v(i + 1, j, top), v(i, j + 1, top), v(i + 1, j + 1, top)
                if top:
                    tris += [(a, b, c), (b, d, c)]
                else:
                    tris += [(a, c, b), (b, c, d)]
    # side walls
    border = [(i, 0) for i in range(n)] + [(n, j) for j in range(n)] + \
             [(n - i, n) for i in range(n)] + [(0, n - j) for j in range(n)]
    for k in range(len(border)):
        i0, j0 = border[k]
        i1, j1 = border[(k + 1) % len(border)]
        a, b = v(i0, j0, False), v(i1, j1, False)
        c, d = v(i0, j0, True), v(i1, j1, True)
        tris += [(a, b, d), (a, d, c)]
    return Indenter(Y=np.array(verts, dtype=np.float64), tris=np.array(tris, dtype=np.int32),
                    name="plate")


def rotation_matrix(q) -> np.ndarray:
    """Rotation matrix of the unit quaternion q = (w, x, y, z)."""
    w, x, y, z = (float(v) for v in q)
    n = (w * w + x * x + y * y + z * z) ** 0.5
    w, x, y, z = w / n, x / n, y / n, z / n
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def quat_from_axis_angle(axis, angle) -> np.ndarray:
    axis = np.asarray(axis, dtype=np.float64)
    axis = axis / np.linalg.norm(axis)
    h = 0.5 * angle
    return np.array([np.cos(h), *(np.sin(h) * axis)])


def quat_mul(a, b) -> np.ndarray:
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([
        w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
        w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
        w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
        w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2,
    ])
