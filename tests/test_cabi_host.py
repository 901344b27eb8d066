"""CPU checks of the C-ABI library: it loads, exports every entry point of
include/t2r.h, and its host-side preprocessing (validation, surface
extraction, marker embedding) agrees with the oracle. No GPU call is made."""

import ctypes
import os
import re

import numpy as np
import pytest
import torch

from oracle.geometry import GelGeometry
from scenes.configs import INDENTERS, sphere_press_484v
from scenes.mesh import mesh_class

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _t2r():
    from paper_2603_28475_amd import t2r
    return t2r


def test_library_exports_every_declared_symbol():
    t2r = _t2r()
    header = open(os.path.join(ROOT, "include", "t2r.h")).read()
    names = set(re.findall(r"\b(t2r_[a-z_]+)\s*\(", header))
    names -= {"t2r_alloc_fn", "t2r_free_fn"}
    assert len(names) >= 20
    lib = ctypes.CDLL(t2r.LIB_PATH)
    for n in sorted(names):
        assert hasattr(lib, n), n
    assert {s[0] for s in t2r.SIGNATURES} == names


@pytest.mark.parametrize("name", ["c1", "5k"])
def test_surface_and_markers_agree_with_oracle(name):
    t2r = _t2r()
    g = mesh_class(name)
    ctx = t2r.Context()
    gid = ctx.add_gel(g.X, g.tets, g.fixed, g.markers)
    info = ctx.gel_info(gid)
    geo = GelGeometry(g.X, g.tets, g.fixed, g.markers)
    assert info["n_v"] == g.n_verts and info["n_t"] == g.n_tets
    assert info["n_sv"] == len(geo.surf_verts)
    assert info["n_se"] == len(geo.surf_edges)
    assert info["n_sf"] == len(geo.surf_tris)
    assert info["n_fixed"] == int(g.fixed.sum())
    tri, w = ctx.gel_markers(gid)
    # the interpolated rest positions must coincide (triangles may differ on ties)
    ref_lib = np.einsum("mk,mkd->md", w, g.X[tri])
    assert np.allclose(ref_lib, geo.marker_ref, atol=1e-12)
    assert np.all(w >= -1e-12) and np.allclose(w.sum(axis=1), 1.0)
    # every tet lands in exactly one tile, tiles respect the LDS limits
    assert info["n_tiles"] >= -(-g.n_tets // 1024)  # at most 1024 tets per tile


def test_invalid_inputs_are_rejected_on_the_host():
    t2r = _t2r()
    g = mesh_class("micro2")
    ctx = t2r.Context()
    bad = g.tets.copy()
    bad[0] = bad[0][[0, 2, 1, 3]]
    with pytest.raises(t2r.T2RError) as e:
        ctx.add_gel(g.X, bad, g.fixed, g.markers)
    assert e.value.code == t2r.T2R_E_ARG and "inverted" in str(e.value)
    bad = g.tets.copy()
    bad[3, 2] = g.n_verts
    with pytest.raises(t2r.T2RError):
        ctx.add_gel(g.X, bad, g.fixed, g.markers)
    X = np.concatenate([g.X, [[9.0, 9.0, 9.0]]])
    with pytest.raises(t2r.T2RError) as e:
        ctx.add_gel(X, g.tets, np.concatenate([g.fixed, [0]]), g.markers)
    assert "belongs to no tet" in str(e.value)
    with pytest.raises(t2r.T2RError) as e:
        ctx.add_gel(g.X, g.tets, g.fixed, np.array([[50.0, 0.0]]))
    assert "outside the top face" in str(e.value)
    gid = ctx.add_gel(g.X, g.tets, g.fixed, g.markers)
    ind = INDENTERS["sphere_small"]()
    iid = ctx.add_indenter(ind.Y, ind.tris)
    pose = np.array([[0, 0, 2.0, 1, 0, 0, 0]])
    with pytest.raises(t2r.T2RError):
        ctx.add_envs([gid], [iid], [(0.3, 0.7, 0, 1e-3, 0.05, 1e3)], pose)   # nu >= 0.5
    with pytest.raises(t2r.T2RError):
        ctx.add_envs([gid], [iid + 1], [(0.3, 0.45, 0, 1e-3, 0.05, 1e3)], pose)
    with pytest.raises(t2r.T2RError):
        ctx.add_envs([gid], [iid], [(0.3, 0.45, 0, 1e-3, 0.05, 1e3)], pose * np.nan)
    assert ctx.add_envs([gid], [iid], [(0.3, 0.45, 0, 1e-3, 0.05, 1e3)], pose) == 0
    assert ctx.env_count() == (1, g.n_verts)
    assert ctx.state_size() == 3 * g.n_verts + 7
    with pytest.raises(t2r.T2RError) as e:
        ctx.backward(None, None)
    assert e.value.code == t2r.T2R_E_ARG            # no outputs
    fr = ctx.add_envs([gid], [iid], [(0.3, 0.45, 0.5, 1e-3, 0.05, 1e3)], pose)
    assert fr == 1
    with pytest.raises(t2r.T2RError) as e:
        ctx.backward(None, None)
    assert e.value.code == t2r.T2R_E_UNSUPPORTED     # friction: needs the sequence adjoint
    assert ctx.tape_length() == -1                   # not recording
    with pytest.raises(t2r.T2RError) as e:
        ctx.record(-1)
    assert e.value.code == t2r.T2R_E_ARG
    with pytest.raises(t2r.T2RError) as e:
        ctx.backward_sequence(1, None, None)
    assert e.value.code == t2r.T2R_E_ARG            # no outputs
    host = torch.zeros(4, dtype=torch.float64)       # never dereferenced: rejected first
    with pytest.raises(t2r.T2RError) as e:
        ctx.backward_sequence(1, host, host)
    assert e.value.code == t2r.T2R_E_STATE          # no tape


def test_invalid_options_are_rejected():
    t2r = _t2r()
    for kw in ({"tol": 0.0}, {"precision": 3}, {"block_size": 100}, {"block_size": 1024}, {"max_substeps": 0},
               {"dynamic": 2}, {"dynamic": 1, "dt": 0.0}, {"dynamic": 1, "density": -1.0}, {"ee_mollifier": 2},
               {"outer_radius": 1.5}, {"outer_radius": 65.0}, {"outer_radius": float("nan")}):
        with pytest.raises(t2r.T2RError):
            t2r.Context(t2r.default_opts(**kw))
    o = t2r.default_opts()
    assert o.tol == 1e-6 and o.armijo == 1 and o.max_iters > 0
    assert o.dynamic == 0 and o.dt > 0.0 and o.density == 1.1e-9
    assert o.max_evals == 200000 and o.ee_mollifier == 0 and o.outer_radius == 0.0
    t2r.Context(t2r.default_opts(dynamic=1, dt=1e-3, density=1e-9))   # a valid dynamic set
    t2r.Context(t2r.default_opts(ee_mollifier=1, outer_radius=10.0))


def test_options_struct_layout_matches_the_library():
    """t2r_default_opts writes every field of the C struct: into a buffer larger
    than the binding's struct, it leaves the bytes past the binding's size alone
    and sets the last field the binding knows."""
    import ctypes
    t2r = _t2r()
    n = ctypes.sizeof(t2r.SolverOpts)
    buf = (ctypes.c_ubyte * (n + 64))(*([0xA5] * (n + 64)))
    t2r.lib.t2r_default_opts(ctypes.cast(buf, ctypes.POINTER(t2r.SolverOpts)))
    assert bytes(buf[n:]) == bytes([0xA5] * 64)
    o = t2r.SolverOpts.from_buffer(buf)
    assert o.outer_radius == 0.0 and o.max_evals == 200000


def test_workload_classes_build_on_the_host():
    t2r = _t2r()
    w = sphere_press_484v(n_envs=3)
    ctx = t2r.Context()
    gid = ctx.add_gel(*(getattr(w.meshes["c1"], k) for k in ("X", "tets", "fixed", "markers")))
    ind = w.indenters["sphere3"]
    iid = ctx.add_indenter(ind.Y, ind.tris)
    first = ctx.add_envs([gid] * 3, [iid] * 3, [e.material() for e in w.envs],
                         np.stack([e.poses[0] for e in w.envs]))
    assert first == 0 and ctx.env_count()[0] == 3


def test_options_roundtrip_and_capacity_rule():
    t2r = _t2r()
    ctx = t2r.Context()
    o = ctx.get_opts()
    assert o.block_size == 0 and o.pair_capacity == 0
    o.block_size = 512
    o.tol = 1e-8
    ctx.set_opts(o)
    assert ctx.get_opts().block_size == 512 and ctx.get_opts().tol == 1e-8
    bad = ctx.get_opts()
    bad.block_size = 100
    with pytest.raises(t2r.T2RError):
        ctx.set_opts(bad)
    assert ctx.get_opts().block_size == 512
    for name in ("c1", "5k"):
        g = mesh_class(name)
        gid = ctx.add_gel(g.X, g.tets, g.fixed, g.markers)
        info = ctx.gel_info(gid)
        assert info["pair_capacity"] == max(8192, 3 * (info["n_sv"] + info["n_se"] + info["n_sf"]))
    ctx.set_pair_capacity(5000)
    assert ctx.gel_info(gid)["pair_capacity"] == 5000


def test_marker_map_replacement_and_knn_map():
    """t2r_set_gel_markers validates and replaces a gel's map before the first GPU
    call. t2r_set_gel_markers_knn builds the paper's k-nearest-neighbour map in
    the library; it equals the oracle's kNN map (same vertices, weights to
    1e-15) for k = 1, 2, 3 and two weight powers, its weights sum to 1 in
    order of distance, and a marker on a node takes it alone."""
    t2r = _t2r()
    from oracle.geometry import GelGeometry, knn_marker_map, top_face_vertices
    g = mesh_class("c1")
    top = top_face_vertices(g.X, GelGeometry(g.X, g.tets, g.fixed, g.markers).boundary_tris_all)
    rng = np.random.default_rng(4)
    M = np.concatenate([np.asarray(g.markers), g.X[top[:2], :2], rng.uniform(-3.9, 3.9, (20, 2))])
    for k in (1, 2, 3):
        for power in (1.0, 2.0):
            ctx = t2r.Context()
            gid = ctx.add_gel(g.X, g.tets, g.fixed, g.markers)
            ctx.set_gel_markers_knn(gid, M, k=k, power=power)
            vert, wt = ctx.gel_markers(gid)
            ov, ow = knn_marker_map(g.X, top, M, k=k, power=power)
            assert np.array_equal(vert, ov), (k, power)
            assert np.abs(wt - ow).max() <= 1e-15, (k, power)
            assert np.allclose(wt.sum(axis=1), 1.0) and np.all(wt >= 0.0)
            d = np.linalg.norm(g.X[vert][:, :, :2] - M[:, None, :], axis=2)
            if k == 3:
                assert np.all(d[:, 0] <= d[:, 1] + 1e-15) and np.all(d[:, 1] <= d[:, 2] + 1e-15)
            on = len(g.markers)  # the two markers placed on nodes
            assert np.all(wt[on:on + 2, 0] == 1.0) and np.all(vert[on:on + 2, 0] == top[:2])
    ctx = t2r.Context()
    gid = ctx.add_gel(g.X, g.tets, g.fixed, g.markers)
    for bad in (dict(k=0), dict(k=4), dict(power=0.0)):
        with pytest.raises(t2r.T2RError) as e:
            ctx.set_gel_markers_knn(gid, M, **{"k": 3, "power": 1.0, **bad})
        assert e.value.code == t2r.T2R_E_ARG
    vert, wt = knn_marker_map(g.X, top, np.asarray(g.markers), k=3)
    ctx.set_gel_markers(gid, vert, wt)
    tri2, w2 = ctx.gel_markers(gid)
    assert np.array_equal(tri2, vert) and np.allclose(w2, wt)
    for bad in ((vert + g.n_verts, wt), (vert, wt * np.nan)):
        with pytest.raises(t2r.T2RError) as e:
            ctx.set_gel_markers(gid, *bad)
        assert e.value.code == t2r.T2R_E_ARG


def test_device_code_has_no_function_calls():
    """Every device function of the kernels is force-inlined, so the compiled
    kernels contain no calls. A call is the one place where a kernel's private
    state crosses a calling convention (caller-saved registers, a callee stack
    frame in scratch); the adjoint kernel's result once changed with the layout
    of its private state while one helper was a real call, and matched the
    oracle again once that helper was inlined."""
    csrc = os.path.join(ROOT, "paper_2603_28475_amd", "csrc")
    for f in ("t2r_kernels.hip", "t2r_math.h"):
        src = open(os.path.join(csrc, f)).read()
        for m in re.finditer(r"^[^\n/]*__device__[^\n;{]*\(", src, re.M):
            decl = m.group(0)
            if "__global__" in decl or "constexpr" in decl or "__align__" in decl:
                continue  # kernels, constants and device arrays
            assert "__forceinline__" in decl, f"{f}: {decl.strip()}"


def test_static_backward_refuses_a_tape_beyond_its_workspace_before_any_gpu_use():
    """t2r_backward_static keeps its tape in a fixed 2^21-double workspace: a
    context whose tape would not fit (800 envs of the 484-vertex gel need
    2 x (800 x 1,452 + 800 x 7) doubles) is refused with T2R_E_ARG and a message
    naming the sizes, before any GPU call."""
    t2r = _t2r()
    w = sphere_press_484v(n_envs=800, n_steps=1)
    ctx = t2r.Context(t2r.default_opts(), None)
    g = w.meshes["c1"]
    gid = ctx.add_gel(g.X, g.tets, g.fixed, g.markers)
    iid = ctx.add_indenter(w.indenters["sphere3"].Y, w.indenters["sphere3"].tris)
    ctx.add_envs([gid] * 800, [iid] * 800, [e.material() for e in w.envs], np.stack([e.poses[0] for e in w.envs]))
    with pytest.raises(t2r.T2RError) as ei:
        ctx.backward_static(torch.zeros(1, dtype=torch.float64), torch.zeros(1, dtype=torch.float64))
    assert ei.value.code == t2r.T2R_E_ARG
    assert "static workspace holds 2097152" in str(ei.value)


def test_autotune_key_counts_batch_composition():
    """The autotune cache key (Sim.tune_key) depends on the batch's composition
    by gel and indenter class, not on the envs' order or poses. Host only: the
    key is computed without any GPU call (device name stubbed)."""
    import torch
    from paper_2603_28475_amd.sim import Sim
    from scenes.configs import uneven_small
    w = uneven_small(n_steps=2)
    orig = torch.cuda.get_device_name
    torch.cuda.get_device_name = lambda dev=None: "stub"
    try:
        def key(order):
            s = Sim.__new__(Sim)
            s.ctx = _t2r().Context()
            s.device = torch.device("cpu")
            gid = {n: s.ctx.add_gel(g.X, g.tets, g.fixed, g.markers) for n, g in w.meshes.items()}
            s.ind_sizes = {i: (len(w.indenters[n].Y), len(w.indenters[n].tris))
                           for i, n in enumerate(w.indenters)}
            iid = {n: i for i, n in enumerate(w.indenters)}
            s.env_gel = [gid[w.envs[k].mesh] for k in order]
            s.env_ind = [iid[w.envs[k].indenter] for k in order]
            return s.tune_key(4)
        assert key([0, 1, 2, 3]) == key([3, 2, 1, 0])
        assert key([0, 1, 2, 3]) != key([0, 1, 2, 2])
        assert key([0, 1, 2, 3]) != key([0, 1, 2])
    finally:
        torch.cuda.get_device_name = orig
