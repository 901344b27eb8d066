"""torch.autograd access to the adjoint (t2r_backward_sequence).

MarkerTrajectory.apply(theta, sim, poses) returns the marker displacements of
every load step of a scripted trajectory, (S, sum n_m, 3), as a differentiable
function of per-env parameters theta = (E, nu, mu_f, dt_x, dt_y, dt_z, dw_x,
dw_y, dw_z): material, friction coefficient and a rigid offset applied to every
pose of the trajectory (the indenter point y becomes exp([dw]x) R Y + t + dt).
The forward resets the envs, applies the materials and offsets, records a tape
and runs the trajectory in one launch; the backward differentiates through
every step (and the friction lag between them) with t2r_backward_sequence and
maps its rotation gradient, taken for an incremental rotation at the offset
pose, to dw through the left Jacobian of SO(3). MarkerField.apply returns the
last step only.
"""

from __future__ import annotations

import numpy as np
import torch


def _quat_from_rotvec(w):
    a = float(np.linalg.norm(w))
    if a == 0.0:
        return np.array([1.0, 0.0, 0.0, 0.0])
    return np.concatenate([[np.cos(0.5 * a)], np.sin(0.5 * a) * np.asarray(w) / a])


def _quat_mul(p, q):
    w1, x1, y1, z1 = p
    w2, x2, y2, z2 = q
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def _left_jacobian(w):
    """J_l(w) with exp([w + d]x) = exp([J_l(w) d]x) exp([w]x) to first order."""
    w = np.asarray(w, dtype=np.float64)
    a = float(np.linalg.norm(w))
    K = np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])
    if a < 1e-8:
        return np.eye(3) + 0.5 * K
    return np.eye(3) + (1.0 - np.cos(a)) / a ** 2 * K + (a - np.sin(a)) / a ** 3 * (K @ K)


def offset_poses(poses, theta):
    """poses (S, n_env, 7), theta (n_env, 9) -> poses with each env's rigid offset."""
    out = np.array(poses, dtype=np.float64, copy=True)
    for e in range(out.shape[1]):
        dq = _quat_from_rotvec(theta[e, 6:9])
        for s in range(out.shape[0]):
            q = out[s, e, 3:] / np.linalg.norm(out[s, e, 3:])
            out[s, e, 3:] = _quat_mul(dq, q)
            out[s, e, :3] += theta[e, 3:6]
    return out


class MarkerTrajectory(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, sim, poses):
        th = theta.detach().cpu().numpy().astype(np.float64)
        n = sim.n_env
        mats = [(th[i, 0], th[i, 1], th[i, 2], *sim.mats[i][3:]) for i in range(n)]
        sim.ctx.set_materials(list(range(n)), mats)
        sim.ctx.reset_envs(list(range(n)))
        # the start pose (the friction lag pose of the first step) takes the offset too
        state = torch.empty(sim.ctx.state_size(), dtype=torch.float64, device=sim.device)
        sim.ctx.get_state(state)
        sim.stream.synchronize()
        st = state.cpu().numpy()
        off = 0
        for e in range(n):
            off += 3 * sim.n_v[e]
            st[off:off + 7] = offset_poses(st[off:off + 7][None, None, :], th[e:e + 1])[0, 0]
            off += 7
        with torch.cuda.stream(sim.stream):
            state.copy_(torch.from_numpy(st))
        sim.ctx.set_state(state)
        seq = offset_poses(np.asarray(poses, dtype=np.float64), th)
        sim.record(seq.shape[0])
        markers, status = sim.step_sequence(seq)
        ctx.sim = sim
        ctx.theta = th
        ctx.status = status
        return markers.clone()

    @staticmethod
    def backward(ctx, grad_u):
        g = ctx.sim.backward_sequence(grad_u.contiguous()).cpu().numpy()
        for e in range(g.shape[0]):
            g[e, 6:9] = _left_jacobian(ctx.theta[e, 6:9]).T @ g[e, 6:9]
        return torch.as_tensor(g, dtype=torch.float64), None, None


class MarkerField:
    """Marker displacements of the last load step of the trajectory."""

    @staticmethod
    def apply(theta, sim, poses):
        return MarkerTrajectory.apply(theta, sim, poses)[-1]
