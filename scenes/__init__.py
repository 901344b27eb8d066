"""Seeded synthetic scenes: gel meshes, rigid indenters, marker layouts and pose schedules.

This package only generates inputs. It holds none of the solver's arithmetic
(no energies, distances, preconditioners or surface extraction) so that the
CPU oracle and the HIP path can both consume the same inputs without sharing
any of the method's code.

Units throughout: mm, N, MPa (N/mm^2). Poses are 7-vectors
(tx, ty, tz, qw, qx, qy, qz) mapping indenter-local points y to world points
R(q) y + t.
"""

from .mesh import GelMesh, hex_kuhn_gel, marker_grid
from .indenters import Indenter, icosphere, end_on_peg, hex_nut
from .configs import Workload, EnvSpec, make_workload, WORKLOADS

__all__ = [
    "GelMesh", "hex_kuhn_gel", "marker_grid",
    "Indenter", "icosphere", "end_on_peg", "hex_nut",
    "Workload", "EnvSpec", "make_workload", "WORKLOADS",
]
