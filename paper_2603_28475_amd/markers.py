"""Marker maps of the gel's top face.

The paper builds the marker map with the k nearest mesh nodes of each marker
in the initial mesh and interpolates marker displacements from those nodes
with weights (Sec. 3.1, Tactile Representation); it gives neither k nor the
weights. `knn_marker_map` reads them as k <= 3 nearest top-face vertices in
the rest xy plane with inverse-distance weights normalised to sum 1 (a marker
on a node takes that node alone). The result is a linear marker map for
`Context.set_gel_markers` (t2r_set_gel_markers); the library's default map
is the barycentric one of the top-face triangle under each marker.
"""

from __future__ import annotations

import numpy as np


def knn_marker_map(X, top_vertices, markers_xy, k=3, power=1.0):
    """(vertex [n_m][3], weight [n_m][3]) of the k-nearest-neighbour map.
    X: rest positions (n_v, 3); top_vertices: candidate vertex ids (the top
    face); markers_xy: (n_m, 2) rest positions of the markers; k <= 3
    (unused slots get weight 0 on the nearest node)."""
    if not 1 <= k <= 3:
        raise ValueError("k must be 1, 2 or 3 (three nodes per marker on the device)")
    X = np.asarray(X, dtype=np.float64)
    top = np.asarray(top_vertices, dtype=np.int64)
    M = np.asarray(markers_xy, dtype=np.float64).reshape(-1, 2)
    d = np.linalg.norm(X[top][None, :, :2] - M[:, None, :], axis=2)      # (n_m, n_top)
    order = np.argsort(d, axis=1, kind="stable")[:, :k]
    vid = top[order]
    dk = np.take_along_axis(d, order, axis=1)
    w = np.zeros_like(dk)
    on_node = dk[:, 0] <= 1e-12
    w[on_node, 0] = 1.0
    inv = 1.0 / np.maximum(dk[~on_node], 1e-300) ** power
    w[~on_node] = inv / inv.sum(axis=1, keepdims=True)
    vertex = np.repeat(vid[:, :1], 3, axis=1)
    weight = np.zeros((len(M), 3))
    vertex[:, :k] = vid
    weight[:, :k] = w
    return vertex.astype(np.int32), weight
