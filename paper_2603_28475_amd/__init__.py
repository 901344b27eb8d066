"""MI355X-native PNCG-IPC visuotactile gel solver (Tac2Real hot path).

The solver is the HIP library libt2r.so behind the C ABI in include/t2r.h;
`t2r` is its ctypes binding and `Sim` a torch-facing convenience wrapper.
"""

from .t2r import Context, SolverOpts, Material, T2RError, default_opts, lib  # noqa: F401


def Sim(*args, **kwargs):  # noqa: N802 - imported lazily so the binding loads without torch
    from .sim import Sim as _Sim
    return _Sim(*args, **kwargs)
