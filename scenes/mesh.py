"""Tetrahedral gel pads: a hex grid split into six Kuhn tetrahedra per hex, or
an unstructured Delaunay tetrahedralisation of the same box.

The paper meshes the sensor gel with tetrahedra (Supp. A, first paragraph)
and reports a "pseudo-structured" mesh for its throughput figure (Sec. 5.1,
"Parallel Performance"). A box split hex-by-hex into the six tetrahedra of
the Kuhn (Freudenthal) subdivision is such a mesh: every hex uses the same
main diagonal, so neighbouring hexes share conforming faces.
"""

from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class GelMesh:
    """A gel pad in its rest configuration.

    X      : (N_v, 3) float64 rest positions in mm; box [-W/2,W/2]x[-D/2,D/2]x[0,T]
    tets   : (N_t, 4) int32 vertex ids, every tet positively oriented
    fixed  : (N_v,) uint8, 1 for vertices on the bottom face z = 0
    size   : (W, D, T) in mm
    cells  : (nx, ny, nz) hexes
    markers: (n_m, 2) float64 marker rest xy on the top face z = T
    """

    X: np.ndarray
    tets: np.ndarray
    fixed: np.ndarray
    size: tuple
    cells: tuple
    markers: np.ndarray
    name: str = ""

    @property
    def n_verts(self) -> int:
        return int(self.X.shape[0])

    @property
    def n_tets(self) -> int:
        return int(self.tets.shape[0])

    @property
    def thickness(self) -> float:
        return float(self.size[2])


def _perm_sign(p) -> int:
    s = 1
    p = list(p)
    for i in range(len(p)):
        for j in range(i + 1, len(p)):
            if p[i] > p[j]:
                s = -s
    return s


def hex_kuhn_gel(size, cells, markers_xy=(7, 7), name: str = "") -> GelMesh:
    """Box gel of `size` = (W, D, T) mm meshed with `cells` = (nx, ny, nz) hexes.

    Vertex (i, j, k) has id i + (nx+1) * (j + (ny+1) * k): x fastest, then y,
    then z, so the top face is the last (nx+1)(ny+1) vertices.
    Each hex with lowest corner c is split into the six tetrahedra
    [c, c+e_a, c+e_a+e_b, c+e_a+e_b+e_c] for the permutations (a, b, c) of the
    axes; odd permutations swap the last two vertices so that every tet has a
    positive signed volume.
    """
    W, D, T = (float(s) for s in size)
    nx, ny, nz = (int(n) for n in cells)
    xs = np.linspace(-W / 2, W / 2, nx + 1)
    ys = np.linspace(-D / 2, D / 2, ny + 1)
    zs = np.linspace(0.0, T, nz + 1)
    Zg, Yg, Xg = np.meshgrid(zs, ys, xs, indexing="ij")
    X = np.stack([Xg.ravel(), Yg.ravel(), Zg.ravel()], axis=1).astype(np.float64)

    def vid(i, j, k):
        return i + (nx + 1) * (j + (ny + 1) * k)

    unit = np.eye(3, dtype=np.int64)
    local = []
    for perm in itertools.permutations(range(3)):
        c0 = np.zeros(3, dtype=np.int64)
        c1 = c0 + unit[perm[0]]
        c2 = c1 + unit[perm[1]]
        c3 = c2 + unit[perm[2]]
        tet = [c0, c1, c2, c3]
        if _perm_sign(perm) < 0:
            tet = [c0, c1, c3, c2]
        local.append(tet)
    local = np.array(local)  # (6, 4, 3) corner offsets

    ii, jj, kk = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    base = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1)  # (nhex, 3)
    # order hexes z-slowest like the vertices
    order = np.lexsort((base[:, 0], base[:, 1], base[:, 2]))
    base = base[order]
    corners = base[:, None, None, :] + local[None, :, :, :]  # (nhex, 6, 4, 3)
    tets = vid(corners[..., 0], corners[..., 1], corners[..., 2]).reshape(-1, 4).astype(np.int32)
    fixed = (np.abs(X[:, 2]) < 1e-12).astype(np.uint8)
    mk = marker_grid((W, D), markers_xy)
    return GelMesh(X=X, tets=tets, fixed=fixed, size=(W, D, T), cells=(nx, ny, nz),
                   markers=mk, name=name)


def marker_grid(size_xy, counts) -> np.ndarray:
    """Marker rest xy on a uniform grid of cell centres over the top face.

    counts = (n_x, n_y); marker (i, j) sits at
    (-W/2 + (i + 1/2) W/n_x, -D/2 + (j + 1/2) D/n_y); x varies fastest.
    """
    W, D = (float(s) for s in size_xy)
    n_x, n_y = (int(c) for c in counts)
    mx = -W / 2 + (np.arange(n_x) + 0.5) * W / n_x
    my = -D / 2 + (np.arange(n_y) + 0.5) * D / n_y
    Yg, Xg = np.meshgrid(my, mx, indexing="ij")
    return np.stack([Xg.ravel(), Yg.ravel()], axis=1).astype(np.float64)


def delaunay_gel(size, cells, markers_xy=(7, 7), seed: int = 0, jitter: float = 0.3,
                 q_min: float = 0.1, max_rounds: int = 100, name: str = "") -> GelMesh:
    """Unstructured box gel: the Delaunay tetrahedralisation of a jittered point
    set, with a lower bound on tet quality.

    The paper contrasts its pseudo-structured mesh with an unstructured one
    (Sec. 5.1, "Parallel Performance"). This builds the latter kind without a
    mesh generator: the (nx+1)(ny+1)(nz+1) grid points of `cells` over the box
    are moved by independent uniform offsets of up to `jitter` cells along
    every axis in which they are interior (box corners stay, edge points move
    along their edge, face points within their face), so the box faces stay
    planar, and scipy's Delaunay tetrahedralises them. Tets whose normalised
    volume-to-edge quality 6 sqrt(2) V / l_rms^3 (1 for a regular tet) is
    below `q_min` are slivers: their movable points are drawn again and the
    point set re-triangulated until none is left (at most `max_rounds` times,
    else ValueError). Every tet is returned positively oriented.
    """
    from scipy.spatial import Delaunay

    W, D, T = (float(s) for s in size)
    nx, ny, nz = (int(n) for n in cells)
    n = np.array([nx, ny, nz])
    h = np.array([W / nx, D / ny, T / nz])
    kk, jj, ii = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    ijk = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1)   # x fastest, like hex_kuhn_gel
    movable = (ijk > 0) & (ijk < n)
    P0 = ijk * h + np.array([-W / 2, -D / 2, 0.0])
    rng = np.random.default_rng(seed)
    J = rng.uniform(-jitter, jitter, P0.shape)
    for _ in range(max_rounds):
        X = P0 + J * h * movable
        tets = Delaunay(X).simplices.astype(np.int64)
        q = tet_quality(X, tets)
        bad = np.abs(q) < q_min
        if not bad.any():
            break
        vs = np.unique(tets[bad])
        J[vs] = rng.uniform(-jitter, jitter, (len(vs), 3))
    else:
        raise ValueError(f"no sliver-free tetrahedralisation after {max_rounds} rounds")
    neg = q < 0
    tets[neg] = tets[neg][:, [0, 1, 3, 2]]
    fixed = (np.abs(X[:, 2]) < 1e-12).astype(np.uint8)
    return GelMesh(X=X, tets=tets.astype(np.int32), fixed=fixed, size=(W, D, T), cells=(nx, ny, nz),
                   markers=marker_grid((W, D), markers_xy), name=name)


def tet_quality(X, tets) -> np.ndarray:
    """Signed 6 sqrt(2) V / l_rms^3 per tet: 1 for a regular tet, 0 when flat."""
    P = np.asarray(X)[np.asarray(tets)]
    e = [P[:, a] - P[:, b] for a, b in ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))]
    l_rms = np.sqrt(np.mean([np.einsum("ij,ij->i", v, v) for v in e], axis=0))
    vol = np.einsum("ij,ij->i", P[:, 1] - P[:, 0], np.cross(P[:, 2] - P[:, 0], P[:, 3] - P[:, 0])) / 6.0
    return 6.0 * np.sqrt(2.0) * vol / l_rms ** 3


# Mesh classes used by the workloads: (size mm, hexes, marker grid).
MESH_CLASSES = {
    "c1": ((8.0, 8.0, 2.0), (10, 10, 3), (7, 7)),
    "2k": ((20.0, 16.0, 4.0), (20, 16, 5), (11, 9)),
    "5k": ((20.0, 16.0, 4.0), (25, 20, 8), (11, 9)),
    "12k": ((20.0, 16.0, 4.0), (40, 32, 8), (11, 9)),
    "micro1": ((1.0, 1.0, 1.0), (1, 1, 1), (2, 2)),
    "micro2": ((2.0, 2.0, 1.0), (2, 2, 1), (2, 2)),
    "micro3": ((3.0, 3.0, 1.0), (3, 3, 1), (3, 3)),
}


# Unstructured classes "<name>u": the same box, grid and markers as class
# <name>, tetrahedralised by delaunay_gel (seed 0) instead of the Kuhn split.
_UNSTRUCTURED = {}


def mesh_class(name: str) -> GelMesh:
    if name.endswith("u") and name[:-1] in MESH_CLASSES:
        if name not in _UNSTRUCTURED:
            size, cells, mk = MESH_CLASSES[name[:-1]]
            _UNSTRUCTURED[name] = delaunay_gel(size, cells, mk, seed=0, name=name)
        return _UNSTRUCTURED[name]
    size, cells, mk = MESH_CLASSES[name]
    return hex_kuhn_gel(size, cells, mk, name=name)
