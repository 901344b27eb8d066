"""Pins of the unstructured (Delaunay) gel meshes: an exact, conforming
partition of the box into positively oriented tets with planar box faces, a
closed genus-0 boundary, the empty-circumsphere property checked by brute
force, the quality bound, the fixed bottom face and the marker embedding; and
the host library's surface extraction and tiling of them against the
oracle's."""

import itertools
from collections import Counter

import numpy as np
import pytest

from oracle.geometry import GelGeometry
from scenes.mesh import delaunay_gel, mesh_class, tet_quality


def _faces(tets):
    c = Counter()
    for t in tets:
        for f in itertools.combinations(sorted(int(v) for v in t), 3):
            c[f] += 1
    return c


@pytest.mark.parametrize("name", ["micro3u", "c1u"])
def test_delaunay_gel_is_a_conforming_partition_of_the_box(name):
    g = mesh_class(name)
    W, D, T = g.size
    nx, ny, nz = g.cells
    assert g.n_verts == (nx + 1) * (ny + 1) * (nz + 1)
    q = tet_quality(g.X, g.tets)
    assert np.all(q >= 0.1)                               # positive and not a sliver
    geo = GelGeometry(g.X, g.tets, g.fixed, g.markers)
    assert geo.vol.sum() == pytest.approx(W * D * T, rel=1e-12)
    faces = _faces(g.tets)
    assert max(faces.values()) == 2                       # conforming: no face in three tets
    bnd = np.array([f for f, k in faces.items() if k == 1])
    # every boundary face lies on one of the six box planes, and they tile them
    P = g.X[bnd]
    lo, hi = np.array([-W / 2, -D / 2, 0.0]), np.array([W / 2, D / 2, T])
    on = [(np.all(np.abs(P[:, :, a] - b) < 1e-12, axis=1)) for a in range(3) for b in (lo[a], hi[a])]
    assert np.all(np.sum(on, axis=0) == 1)
    area = 0.5 * np.linalg.norm(np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]), axis=1)
    assert area.sum() == pytest.approx(2 * (W * D + W * T + D * T), rel=1e-12)
    # closed genus-0 boundary
    edges = {tuple(sorted(e)) for t in bnd for e in ((t[0], t[1]), (t[1], t[2]), (t[0], t[2]))}
    assert len(np.unique(bnd)) - len(edges) + len(bnd) == 2
    assert len(geo.boundary_tris_all) == len(bnd)
    # bottom face fixed, nothing else; markers embedded in the top face
    assert g.fixed.sum() == (nx + 1) * (ny + 1)
    assert np.all(np.abs(g.X[g.fixed.astype(bool), 2]) < 1e-15)
    assert np.allclose(geo.marker_ref[:, :2], g.markers, atol=1e-12)
    assert np.allclose(geo.marker_ref[:, 2], T, atol=1e-12)


@pytest.mark.parametrize("name", ["micro3u", "c1u"])
def test_delaunay_gel_has_empty_circumspheres(name):
    """No mesh vertex lies strictly inside any tet's circumsphere (brute force)."""
    g = mesh_class(name)
    X = g.X
    P = X[g.tets]
    A = 2.0 * (P[:, 1:] - P[:, :1])                                        # (n_t, 3, 3)
    b = np.sum(P[:, 1:] ** 2, axis=2) - np.sum(P[:, :1] ** 2, axis=2)     # (n_t, 3)
    c = np.linalg.solve(A, b[..., None])[..., 0]
    r2 = np.sum((P[:, 0] - c) ** 2, axis=1)
    d2 = np.sum((X[None, :, :] - c[:, None, :]) ** 2, axis=2)              # (n_t, n_v)
    inside = d2 < r2[:, None] * (1.0 - 1e-9)
    assert not inside.any(), np.argwhere(inside)[:5]


def test_delaunay_gel_is_deterministic_and_differs_from_the_kuhn_split():
    a = delaunay_gel((3.0, 3.0, 1.0), (3, 3, 1), (3, 3), seed=4)
    b = delaunay_gel((3.0, 3.0, 1.0), (3, 3, 1), (3, 3), seed=4)
    assert np.array_equal(a.X, b.X) and np.array_equal(a.tets, b.tets)
    k = mesh_class("micro3")
    assert a.n_verts == k.n_verts and not np.allclose(a.X, k.X)
    # the jitter keeps the box faces in place
    assert np.array_equal(np.sort(a.X[:, 2])[[0, -1]], [0.0, 1.0])


def test_quality_of_the_regular_tet_is_one():
    s = np.sqrt(2.0) / 2
    X = np.array([[1, 0, -s], [-1, 0, -s], [0, 1, s], [0, -1, s]], dtype=np.float64)
    q = tet_quality(X, np.array([[0, 1, 2, 3]]))
    assert abs(abs(q[0]) - 1.0) < 1e-14
    assert tet_quality(X, np.array([[0, 1, 3, 2]]))[0] == pytest.approx(-q[0])


@pytest.mark.parametrize("name", ["c1u", "5ku"])
def test_host_library_surface_and_tiles_of_unstructured_gels(name):
    from paper_2603_28475_amd import t2r
    g = mesh_class(name)
    ctx = t2r.Context()
    gid = ctx.add_gel(g.X, g.tets, g.fixed, g.markers)
    info = ctx.gel_info(gid)
    geo = GelGeometry(g.X, g.tets, g.fixed, g.markers)
    assert info["n_v"] == g.n_verts and info["n_t"] == g.n_tets
    assert (info["n_sv"], info["n_se"], info["n_sf"]) == (len(geo.surf_verts), len(geo.surf_edges),
                                                          len(geo.surf_tris))
    assert info["n_fixed"] == int(g.fixed.sum())
    tri, w = ctx.gel_markers(gid)
    assert np.allclose(np.einsum("mk,mkd->md", w, g.X[tri]), geo.marker_ref, atol=1e-12)
    assert info["n_tiles"] >= -(-g.n_tets // 1024)
