"""torch.autograd access to the adjoint (t2r_backward_sequence).

MarkerTrajectory.apply(theta, sim, poses) returns the marker displacements of
every load step of a scripted trajectory, (S, sum n_m, 3), as a differentiable
function of per-env parameters theta = (E, nu, mu_f, dt_x, dt_y, dt_z, dw_x,
dw_y, dw_z): material, friction coefficient and a rigid offset applied by the
library to every pose of the trajectory (t2r_set_pose_offsets: the indenter
point R Y + t becomes exp([dw]x) R Y + t + dt). The forward sets the materials
and offsets, resets the envs, records a tape and runs the trajectory in one
launch; the backward differentiates through every step (and the friction lag
between them) with t2r_backward_sequence, which reports the gradient with
respect to the offset itself. MarkerField.apply returns the last step only.
The offsets stay set on the Sim after the forward.
"""

from __future__ import annotations

import numpy as np
import torch


class MarkerTrajectory(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, sim, poses):
        th = theta.detach().cpu().numpy().astype(np.float64)
        n = sim.n_env
        ids = list(range(n))
        sim.ctx.set_materials(ids, [(th[i, 0], th[i, 1], th[i, 2], *sim.mats[i][3:]) for i in range(n)])
        sim.ctx.set_pose_offsets(ids, th[:, 3:9])
        sim.ctx.reset_envs(ids)
        seq = np.asarray(poses, dtype=np.float64)
        sim.record(seq.shape[0])
        markers, status = sim.step_sequence(seq)
        ctx.sim = sim
        ctx.status = status
        return markers.clone()

    @staticmethod
    def backward(ctx, grad_u):
        g = ctx.sim.backward_sequence(grad_u.contiguous())
        return g.cpu().to(torch.float64), None, None


class MarkerField:
    """Marker displacements of the last load step of the trajectory."""

    @staticmethod
    def apply(theta, sim, poses):
        return MarkerTrajectory.apply(theta, sim, poses)[-1]
