"""Pins for the inputs and the oracle's mesh preprocessing: grid counts of the
hex-to-tet split, closed surfaces (Euler characteristic), orientation, marker
embedding (Sec. 3.2 reading: barycentric in the top-face triangle)."""

import numpy as np
import pytest

from oracle.geometry import GelGeometry, IndenterGeometry, quat_to_matrix, slerp_pose
from scenes.configs import INDENTERS, sphere_press_484v
from scenes.mesh import mesh_class


@pytest.mark.parametrize("name,nv,nt,nsv,nsf,nse", [
    ("c1", 484, 1800, 322, 640, 960),
    ("2k", 2142, 9600, 1002, 2000, 3000),
    ("5k", 4914, 24000, 1722, 3440, 5160),
])
def test_grid_counts_and_surface(name, nv, nt, nsv, nsf, nse):
    g = mesh_class(name)
    assert (g.n_verts, g.n_tets) == (nv, nt)
    nx, ny, nz = g.cells
    assert nv == (nx + 1) * (ny + 1) * (nz + 1) and nt == 6 * nx * ny * nz
    geo = GelGeometry(g.X, g.tets, g.fixed)
    allt = geo.boundary_tris_all
    assert len(allt) == 4 * (nx * ny + nx * nz + ny * nz)
    verts = np.unique(allt)
    edges = {tuple(sorted(e)) for t in allt for e in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0]))}
    assert len(verts) - len(edges) + len(allt) == 2  # closed genus-0 surface
    assert (len(verts), len(allt), len(edges)) == (nsv, nsf, nse)
    # dropping the all-fixed primitives of the bottom face
    assert len(geo.surf_verts) == nsv - (nx + 1) * (ny + 1)
    assert len(geo.surf_tris) == nsf - 2 * nx * ny
    assert len(geo.surf_edges) == nse - (nx * (ny + 1) + ny * (nx + 1) + nx * ny)
    assert np.all(geo.vol > 0)
    assert geo.vol.sum() == pytest.approx(np.prod(g.size), rel=1e-12)


def test_marker_embedding_reproduces_marker_positions():
    w = sphere_press_484v()
    g = w.meshes["c1"]
    geo = GelGeometry(g.X, g.tets, g.fixed, g.markers)
    assert geo.marker_w.shape == (49, 3)
    assert np.all(geo.marker_w >= -1e-12)
    assert np.allclose(geo.marker_w.sum(axis=1), 1.0)
    assert np.allclose(geo.marker_ref[:, :2], g.markers, atol=1e-12)
    assert np.allclose(geo.marker_ref[:, 2], g.size[2])
    assert np.allclose(geo.markers(g.X), 0.0)
    # a rigid translation of the gel moves every marker by the same vector
    assert np.allclose(geo.markers(g.X + [0.1, -0.2, 0.3]), [0.1, -0.2, 0.3])


@pytest.mark.parametrize("name,nv,nf,chi", [("sphere3", 162, 320, 2), ("peg4", 1026, 2048, 2),
                                            ("nut8", 1536, 3072, 0)])
def test_indenters_are_closed_and_outward(name, nv, nf, chi):
    ind = INDENTERS[name]()
    geo = IndenterGeometry(ind.Y, ind.tris)
    assert (len(geo.Y), len(geo.tris)) == (nv, nf)
    assert len(geo.Y) - len(geo.edges) + len(geo.tris) == chi
    Y, T = geo.Y, geo.tris
    vol = np.einsum("ni,ni->n", Y[T[:, 0]], np.cross(Y[T[:, 1]], Y[T[:, 2]])).sum() / 6
    assert vol > 0


def test_poses_and_slerp():
    q = np.array([np.cos(0.3), 0, np.sin(0.3), 0])
    R = quat_to_matrix(q)
    assert np.allclose(R @ R.T, np.eye(3)) and np.linalg.det(R) == pytest.approx(1)
    p0 = np.array([0, 0, 0, 1, 0, 0, 0.0])
    p1 = np.array([1, 2, 3, *q])
    assert np.allclose(slerp_pose(p0, p1, 0.0), p0)
    assert np.allclose(slerp_pose(p0, p1, 1.0), p1)
    mid = slerp_pose(p0, p1, 0.5)
    assert np.allclose(mid[:3], [0.5, 1, 1.5])
    assert np.allclose(mid[3:], [np.cos(0.15), 0, np.sin(0.15), 0])
    # schedule: lowest indenter vertex 2 dhat above the gel at step 0, 0.6 mm deep at the end
    w = sphere_press_484v()
    env = w.envs[0]
    ind = w.indenters["sphere3"]
    for s, depth in ((0, -0.1), (10, 0.6)):
        Yw = ind.Y @ quat_to_matrix(env.poses[s][3:]).T + env.poses[s][:3]
        assert 2.0 - Yw[:, 2].min() == pytest.approx(depth, abs=1e-12)
