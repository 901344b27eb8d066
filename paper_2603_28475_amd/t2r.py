"""ctypes binding of the t2r C ABI (include/t2r.h): argument marshalling only.

Every step of the solve runs in the HIP kernels of libt2r.so; this module
passes host arrays and torch device pointers through. If the library is
missing the import fails loudly: there is no CPU fallback.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libt2r.so")

T2R_OK, T2R_E_ARG, T2R_E_NOMEM, T2R_E_HIP, T2R_E_STATE, T2R_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
ENV_CONVERGED, ENV_MAXITER, ENV_INFEASIBLE, ENV_NONFINITE = 1, 2, 4, 8
ENV_PAIR_OVERFLOW, ENV_LINESEARCH, ENV_SUBSTEPS, ENV_SKIPPED = 16, 32, 64, 128
ENV_BUDGET = 256


class Material(C.Structure):
    _fields_ = [("E", C.c_double), ("nu", C.c_double), ("mu_f", C.c_double),
                ("eps_v", C.c_double), ("dhat", C.c_double), ("kappa", C.c_double)]


class SolverOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("substep_tol", C.c_double), ("max_iters", C.c_int32),
                ("max_substeps", C.c_int32), ("precision", C.c_int32),
                ("pair_capacity", C.c_int32), ("armijo", C.c_int32), ("block_size", C.c_int32),
                ("warm_start", C.c_int32), ("dynamic", C.c_int32), ("dt", C.c_double),
                ("density", C.c_double), ("max_evals", C.c_int32),
                ("ee_mollifier", C.c_int32), ("outer_radius", C.c_double), ("deterministic", C.c_int32),
                ("self_contact", C.c_int32)]


class EnvStats(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("substeps", C.c_int32),
                ("restarts", C.c_int32), ("halvings", C.c_int32), ("reculls", C.c_int32),
                ("n_candidates", C.c_int32), ("n_active", C.c_int32), ("n_friction", C.c_int32),
                ("max_solve_iters", C.c_int32), ("outer_builds", C.c_int32),
                ("n_outer", C.c_int32), ("d_min", C.c_double), ("residual", C.c_double),
                ("energy", C.c_double), ("phase_ms", C.c_double * 10), ("list_fill", C.c_double),
                ("evals", C.c_int32), ("reserved", C.c_int32)]


class T2RError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"t2r error {code}: {msg}")
        self.code = code


_P = C.c_void_p
_PD = C.POINTER(C.c_double)
_PI = C.POINTER(C.c_int32)

# (name, restype, argtypes) for every entry point of include/t2r.h
SIGNATURES = [
    ("t2r_default_opts", None, [C.POINTER(SolverOpts)]),
    ("t2r_create", C.c_int32, [C.POINTER(_P), C.POINTER(SolverOpts), _P]),
    ("t2r_destroy", None, [_P]),
    ("t2r_last_error", C.c_char_p, [_P]),
    ("t2r_set_allocator", C.c_int32, [_P, _P, _P, _P]),
    ("t2r_add_gel", C.c_int32, [_P, C.c_int32, _PD, C.c_int32, _PI, C.POINTER(C.c_uint8),
                                C.c_int32, _PD, _PI]),
    ("t2r_gel_info", C.c_int32, [_P, C.c_int32, _PI]),
    ("t2r_gel_markers", C.c_int32, [_P, C.c_int32, _PI, _PD]),
    ("t2r_add_indenter", C.c_int32, [_P, C.c_int32, _PD, C.c_int32, _PI, _PI]),
    ("t2r_add_envs", C.c_int32, [_P, C.c_int32, _PI, _PI, C.POINTER(Material), _PD, _PI]),
    ("t2r_env_count", C.c_int32, [_P, _PI, C.POINTER(C.c_int64)]),
    ("t2r_set_materials", C.c_int32, [_P, C.c_int32, _PI, C.POINTER(Material)]),
    ("t2r_step", C.c_int32, [_P, _P, _P, _P, _P, _P]),
    ("t2r_step_sequence", C.c_int32, [_P, C.c_int32, _P, _P, _P, _P, _P]),
    ("t2r_eval", C.c_int32, [_P, C.c_int32, _P, _P, _P, _PD, _PD, _P, _P, _P]),
    ("t2r_get_stats", C.c_int32, [_P, _P, C.c_size_t]),
    ("t2r_state_size", C.c_int32, [_P, C.POINTER(C.c_int64)]),
    ("t2r_get_state", C.c_int32, [_P, _P]),
    ("t2r_checkpoint_size", C.c_int32, [_P, C.POINTER(C.c_int64)]),
    ("t2r_save_checkpoint", C.c_int32, [_P, _P]),
    ("t2r_load_checkpoint", C.c_int32, [_P, _P]),
    ("t2r_set_state", C.c_int32, [_P, _P]),
    ("t2r_reset_envs", C.c_int32, [_P, _PI, C.c_int32]),
    ("t2r_set_pair_capacity", C.c_int32, [_P, C.c_int32]),
    ("t2r_get_opts", C.c_int32, [_P, C.POINTER(SolverOpts)]),
    ("t2r_set_opts", C.c_int32, [_P, C.POINTER(SolverOpts)]),
    ("t2r_backward", C.c_int32, [_P, _P, _P]),
    ("t2r_record", C.c_int32, [_P, C.c_int32]),
    ("t2r_tape_length", C.c_int32, [_P, C.POINTER(C.c_int32)]),
    ("t2r_backward_sequence", C.c_int32, [_P, C.c_int32, _P, _P]),
    ("t2r_tape_read", C.c_int32, [_P, C.c_int32, _P]),
    ("t2r_set_gel_markers", C.c_int32, [_P, C.c_int32, C.c_int32, _PI, _PD]),
    ("t2r_layout_generation", C.c_int32, [_P, C.POINTER(C.c_int64)]),
    ("t2r_backward_static", C.c_int32, [_P, _P, _P]),
    ("t2r_set_gel_markers_knn", C.c_int32, [_P, C.c_int32, C.c_int32, _PD, C.c_int32, C.c_double]),
    ("t2r_step_velocity", C.c_int32, [_P, C.c_int32, C.c_double, _P, _P, _P, _P, _P]),
    ("t2r_step_relative", C.c_int32, [_P, C.c_int32, _P, _P, _P, _P, _P, _P]),
    ("t2r_set_pose_offsets", C.c_int32, [_P, C.c_int32, _PI, _PD]),
    ("t2r_set_densities", C.c_int32, [_P, C.c_int32, _PI, _PD]),
]


def load_library(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2603_28475_amd.build` "
                          "(there is no CPU fallback)")
    lib = C.CDLL(path)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = load_library()


def _dptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def _tptr(t):
    """Device pointer of a torch tensor (or None)."""
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def default_opts(**kw) -> SolverOpts:
    o = SolverOpts()
    lib.t2r_default_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Context:
    """Owns one t2r context; methods mirror the C entry points."""

    def __init__(self, opts: SolverOpts | None = None, stream=None):
        self.handle = C.c_void_p()
        s = C.c_void_p(stream) if stream else None
        code = lib.t2r_create(C.byref(self.handle), C.byref(opts) if opts is not None else None, s)
        if code != T2R_OK:
            raise T2RError(code, "t2r_create failed")

    def close(self):
        if self.handle:
            lib.t2r_destroy(self.handle)
            self.handle = C.c_void_p()
        self._alloc_cbs = None

    def set_allocator(self, alloc, free):
        """Routes every device allocation of the context through alloc(nbytes) -> int
        pointer (0 on failure) and free(ptr) (t2r_set_allocator); before the first
        GPU call. The callbacks live as long as the context."""
        a = _ALLOC_FN(lambda n, user: alloc(int(n)))
        f = _FREE_FN(lambda ptr, user: free(int(ptr)) if ptr else None)
        self.check(lib.t2r_set_allocator(self.handle, C.cast(a, C.c_void_p), C.cast(f, C.c_void_p), None))
        self._alloc_cbs = (a, f)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_error(self) -> str:
        return lib.t2r_last_error(self.handle).decode()

    def check(self, code):
        if code != T2R_OK:
            raise T2RError(code, self.last_error())
        return code

    # -- classes and envs (host only) -------------------------------------
    def add_gel(self, X, tets, fixed, markers) -> int:
        X = np.ascontiguousarray(X, dtype=np.float64)
        tets = np.ascontiguousarray(tets, dtype=np.int32)
        fixed = np.ascontiguousarray(fixed, dtype=np.uint8)
        markers = np.ascontiguousarray(markers, dtype=np.float64).reshape(-1, 2)
        gid = C.c_int32()
        self.check(lib.t2r_add_gel(self.handle, X.shape[0], _dptr(X, C.c_double), tets.shape[0],
                                   _dptr(tets, C.c_int32), _dptr(fixed, C.c_uint8), markers.shape[0],
                                   _dptr(markers, C.c_double), C.byref(gid)))
        return gid.value

    def gel_info(self, gid) -> dict:
        out = np.zeros(10, np.int32)
        self.check(lib.t2r_gel_info(self.handle, gid, _dptr(out, C.c_int32)))
        keys = ["n_v", "n_t", "n_sv", "n_se", "n_sf", "n_m", "n_tiles", "n_top", "n_fixed", "pair_capacity"]
        return dict(zip(keys, out.tolist()))

    def gel_markers(self, gid):
        n_m = self.gel_info(gid)["n_m"]
        tri = np.zeros((n_m, 3), np.int32)
        w = np.zeros((n_m, 3), np.float64)
        self.check(lib.t2r_gel_markers(self.handle, gid, _dptr(tri, C.c_int32), _dptr(w, C.c_double)))
        return tri, w

    def set_gel_markers(self, gid, vertex, weight):
        vertex = np.ascontiguousarray(vertex, dtype=np.int32).reshape(-1, 3)
        weight = np.ascontiguousarray(weight, dtype=np.float64).reshape(-1, 3)
        self.check(lib.t2r_set_gel_markers(self.handle, gid, len(vertex), _dptr(vertex, C.c_int32),
                                           _dptr(weight, C.c_double)))

    def set_gel_markers_knn(self, gid, markers_xy, k=3, power=1.0):
        m = np.ascontiguousarray(markers_xy, dtype=np.float64).reshape(-1, 2)
        self.check(lib.t2r_set_gel_markers_knn(self.handle, gid, len(m), _dptr(m, C.c_double), int(k),
                                               float(power)))

    def add_indenter(self, Y, tris) -> int:
        Y = np.ascontiguousarray(Y, dtype=np.float64)
        tris = np.ascontiguousarray(tris, dtype=np.int32)
        iid = C.c_int32()
        self.check(lib.t2r_add_indenter(self.handle, Y.shape[0], _dptr(Y, C.c_double), tris.shape[0],
                                        _dptr(tris, C.c_int32), C.byref(iid)))
        return iid.value

    def add_envs(self, gel_ids, ind_ids, mats, pose0) -> int:
        n = len(gel_ids)
        g = np.ascontiguousarray(gel_ids, dtype=np.int32)
        i = np.ascontiguousarray(ind_ids, dtype=np.int32)
        m = (Material * n)(*[Material(*mt) for mt in mats])
        p = np.ascontiguousarray(pose0, dtype=np.float64).reshape(n, 7)
        first = C.c_int32()
        self.check(lib.t2r_add_envs(self.handle, n, _dptr(g, C.c_int32), _dptr(i, C.c_int32), m,
                                    _dptr(p, C.c_double), C.byref(first)))
        return first.value

    def set_materials(self, env_ids, mats):
        n = len(env_ids)
        ids = np.ascontiguousarray(env_ids, dtype=np.int32)
        m = (Material * n)(*[Material(*mt) for mt in mats])
        self.check(lib.t2r_set_materials(self.handle, n, _dptr(ids, C.c_int32), m))

    def env_count(self):
        n = C.c_int32()
        v = C.c_int64()
        self.check(lib.t2r_env_count(self.handle, C.byref(n), C.byref(v)))
        return n.value, v.value

    def state_size(self) -> int:
        n = C.c_int64()
        self.check(lib.t2r_state_size(self.handle, C.byref(n)))
        return n.value

    def layout_generation(self) -> int:
        n = C.c_int64()
        self.check(lib.t2r_layout_generation(self.handle, C.byref(n)))
        return n.value

    def set_pair_capacity(self, cap):
        self.check(lib.t2r_set_pair_capacity(self.handle, cap))

    def get_opts(self) -> SolverOpts:
        o = SolverOpts()
        self.check(lib.t2r_get_opts(self.handle, C.byref(o)))
        return o

    def set_opts(self, opts: SolverOpts):
        self.check(lib.t2r_set_opts(self.handle, C.byref(opts)))

    # -- GPU entry points (torch tensors on the context's device) -----------
    def step(self, d_pose, d_mask=None, d_markers=None, d_x=None, d_status=None):
        self.check(lib.t2r_step(self.handle, _tptr(d_pose), _tptr(d_mask), _tptr(d_markers),
                                _tptr(d_x), _tptr(d_status)))

    def step_sequence(self, n_steps, d_poses, d_mask=None, d_markers=None, d_x=None, d_status=None):
        self.check(lib.t2r_step_sequence(self.handle, int(n_steps), _tptr(d_poses), _tptr(d_mask),
                                         _tptr(d_markers), _tptr(d_x), _tptr(d_status)))

    def step_velocity(self, n_steps, dt, d_vel, d_mask=None, d_markers=None, d_x=None, d_status=None):
        self.check(lib.t2r_step_velocity(self.handle, int(n_steps), float(dt), _tptr(d_vel), _tptr(d_mask),
                                         _tptr(d_markers), _tptr(d_x), _tptr(d_status)))

    def step_relative(self, n_steps, d_rel0, d_rel1, d_mask=None, d_markers=None, d_x=None, d_status=None):
        self.check(lib.t2r_step_relative(self.handle, int(n_steps), _tptr(d_rel0), _tptr(d_rel1), _tptr(d_mask),
                                         _tptr(d_markers), _tptr(d_x), _tptr(d_status)))

    def set_densities(self, env_ids, density):
        ids = np.ascontiguousarray(env_ids, dtype=np.int32)
        rho = np.ascontiguousarray(density, dtype=np.float64).reshape(-1)
        self.check(lib.t2r_set_densities(self.handle, len(ids), _dptr(ids, C.c_int32), _dptr(rho, C.c_double)))

    def set_pose_offsets(self, env_ids, offsets):
        ids = np.ascontiguousarray(env_ids, dtype=np.int32)
        off = np.ascontiguousarray(offsets, dtype=np.float64).reshape(-1, 6)
        self.check(lib.t2r_set_pose_offsets(self.handle, len(ids), _dptr(ids, C.c_int32), _dptr(off, C.c_double)))

    def eval(self, env, d_x, pose, d_p=None, d_x_lag=None, pose_lag=None, d_grad=None, d_diag=None,
             d_scalars=None):
        pose = np.ascontiguousarray(pose, dtype=np.float64)
        pl = None if pose_lag is None else np.ascontiguousarray(pose_lag, dtype=np.float64)
        self.check(lib.t2r_eval(self.handle, env, _tptr(d_x), _tptr(d_p), _tptr(d_x_lag),
                                _dptr(pose, C.c_double), None if pl is None else _dptr(pl, C.c_double),
                                _tptr(d_grad), _tptr(d_diag), _tptr(d_scalars)))

    def get_stats(self) -> list:
        n, _ = self.env_count()
        arr = (EnvStats * n)()
        self.check(lib.t2r_get_stats(self.handle, C.cast(arr, C.c_void_p), C.sizeof(arr)))
        out = []
        for s in arr:
            d = {f: getattr(s, f) for f, _ in EnvStats._fields_}
            d["phase_ms"] = list(s.phase_ms)
            out.append(d)
        return out

    def get_state(self, d_state):
        self.check(lib.t2r_get_state(self.handle, _tptr(d_state)))

    def set_state(self, d_state):
        self.check(lib.t2r_set_state(self.handle, _tptr(d_state)))

    def checkpoint_size(self) -> int:
        n = C.c_int64()
        self.check(lib.t2r_checkpoint_size(self.handle, C.byref(n)))
        return n.value

    def save_checkpoint(self, d_buf):
        self.check(lib.t2r_save_checkpoint(self.handle, _tptr(d_buf)))

    def load_checkpoint(self, d_buf):
        self.check(lib.t2r_load_checkpoint(self.handle, _tptr(d_buf)))

    def reset_envs(self, ids):
        a = np.ascontiguousarray(ids, dtype=np.int32)
        self.check(lib.t2r_reset_envs(self.handle, _dptr(a, C.c_int32), len(a)))

    def backward(self, d_dL_du, d_grad):
        self.check(lib.t2r_backward(self.handle, _tptr(d_dL_du), _tptr(d_grad)))

    def backward_static(self, d_dL_du, d_grad):
        self.check(lib.t2r_backward_static(self.handle, _tptr(d_dL_du), _tptr(d_grad)))

    def record(self, max_steps):
        self.check(lib.t2r_record(self.handle, int(max_steps)))

    def tape_length(self):
        n = C.c_int32(0)
        self.check(lib.t2r_tape_length(self.handle, C.byref(n)))
        return n.value

    def tape_read(self, entry, d_state):
        self.check(lib.t2r_tape_read(self.handle, int(entry), _tptr(d_state)))

    def backward_sequence(self, n_steps, d_dL_du, d_grad):
        self.check(lib.t2r_backward_sequence(self.handle, int(n_steps), _tptr(d_dL_du), _tptr(d_grad)))
