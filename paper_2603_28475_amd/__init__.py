"""MI355X-native PNCG-IPC visuotactile gel solver (Tac2Real hot path).

The solver is the HIP library libt2r.so behind the C ABI in include/t2r.h;
`t2r` is its ctypes binding and `Sim` a torch-facing convenience wrapper.
Both load lazily, so `python -m paper_2603_28475_amd.build` works before the
library exists (or while an older build is in place).
"""

_BINDING = ("Context", "SolverOpts", "Material", "T2RError", "default_opts", "lib")


def __getattr__(name):
    if name in _BINDING:
        from . import t2r
        return getattr(t2r, name)
    if name == "Sim":
        from .sim import Sim
        return Sim
    raise AttributeError(name)
