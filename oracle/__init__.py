"""FP64 CPU oracle for the PNCG-IPC quasi-static gel solve (Tac2Real, Supp. A).

TEST INFRASTRUCTURE ONLY. Nothing on the product path may import, call or
execute anything in this package: only the tests, the smoke check and the
benchmark's CPU-baseline leg use it. It shares no code with the HIP library
and does not import it; both consume the seeded inputs of `scenes`.

What it computes (readings of the paper are listed per module):
  * the per-step energy  Pi(x) = sum_e V_e psi(F_e) + kappa sum_k b(d_k) + D(x)
    (Supp. A, eq. ipc_energy without the inertia term: quasi-static),
  * its exact gradient, diagonal Hessian and curvature p^T H p,
  * the minimiser x* of Pi by projected Newton with a CCD-bounded line search
    (the standard IPC route the paper contrasts PNCG with, Sec. 3.1),
  * a step-by-step PNCG reference (Supp. A, eqs. dk_direction and step_size),
  * marker displacements interpolated from the deformed mesh (Sec. 3.2).
"""

from .geometry import GelGeometry, IndenterGeometry, quat_to_matrix, slerp_pose
from .elastic import lame, psi, first_piola, element_energy, element_gradient, element_hessian
from .barrier import barrier, barrier_d1, barrier_d2
from .distance import point_triangle, edge_edge, distance_derivatives
from .problem import StepProblem
from .newton import newton_solve
from .pncg import pncg_solve
from .sim import simulate, SimResult

__all__ = [
    "GelGeometry", "IndenterGeometry", "quat_to_matrix", "slerp_pose",
    "lame", "psi", "first_piola", "element_energy", "element_gradient", "element_hessian",
    "barrier", "barrier_d1", "barrier_d2",
    "point_triangle", "edge_edge", "distance_derivatives",
    "StepProblem", "newton_solve", "pncg_solve", "simulate", "SimResult",
]
