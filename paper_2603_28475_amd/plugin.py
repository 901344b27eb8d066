"""The plugin surface towards a physics engine, and the policy's tactile
observation.

Per physics step the engine reports where the grasped object sits relative
to the sensor at the start and at the end of the step; that motion, as a
linear and an angular velocity, drives the tactile simulation, whose marker
displacement field is handed back as part of the observation (Sec. 3.3,
"Integrating to Physics Engine"). The policy sees the field of one finger as
a 7 x 9 grid of in-plane displacements (Sec. 5.3, online RL).

Poses are (t_x, t_y, t_z, q_w, q_x, q_y, q_z) of the indenter (the object) in
the gel's frame, as everywhere in this package. The velocity integration is
host-side pose arithmetic on a few numbers per env; every load step runs in
the library.
"""

from __future__ import annotations

import numpy as np


def _qmul(a, b):
    w1, x1, y1, z1 = np.moveaxis(a, -1, 0)
    w2, x2, y2, z2 = np.moveaxis(b, -1, 0)
    return np.stack([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2], axis=-1)


def _qconj(q):
    return q * np.array([1.0, -1.0, -1.0, -1.0])


def relative_velocity(p0, p1, dt):
    """Constant linear and angular velocity (world-frame, rad/s) that carry pose
    p0 to pose p1 in time dt: v = (t1 - t0) / dt, and w = axis * angle / dt of
    the shortest rotation q1 q0^-1. Shapes (..., 7) -> ((..., 3), (..., 3))."""
    p0 = np.asarray(p0, dtype=np.float64)
    p1 = np.asarray(p1, dtype=np.float64)
    if not dt > 0:
        raise ValueError("dt must be positive")
    v = (p1[..., :3] - p0[..., :3]) / dt
    q0 = p0[..., 3:] / np.linalg.norm(p0[..., 3:], axis=-1, keepdims=True)
    q1 = p1[..., 3:] / np.linalg.norm(p1[..., 3:], axis=-1, keepdims=True)
    dq = _qmul(q1, _qconj(q0))
    dq = np.where(dq[..., :1] < 0, -dq, dq)                  # q and -q: take the short way
    s = np.linalg.norm(dq[..., 1:], axis=-1, keepdims=True)
    angle = 2.0 * np.arctan2(s, dq[..., :1])
    axis = np.divide(dq[..., 1:], s, out=np.zeros_like(dq[..., 1:]), where=s > 0)
    return v, axis * angle / dt


def advance_pose(p0, v, w, tau):
    """Pose after moving p0 for time tau at linear velocity v and world-frame
    angular velocity w: t = t0 + v tau, q = exp(w tau) q0."""
    p0 = np.asarray(p0, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    t = p0[..., :3] + v * tau
    rate = np.linalg.norm(w, axis=-1, keepdims=True)
    half = 0.5 * rate * tau
    axis = np.divide(w, rate, out=np.zeros_like(w), where=rate > 0)
    dq = np.concatenate([np.cos(half), np.sin(half) * axis], axis=-1)
    q = _qmul(dq, p0[..., 3:])
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    return np.concatenate([t, q], axis=-1)


def observation(markers, n_env, grid=(7, 9)):
    """The policy's tactile observation: the in-plane (x, y) components of the
    marker displacements of every env as (n_env, n_x, n_y, 2), where the gel's
    markers lie on an n_x x n_y grid listed x fastest (scenes.mesh.marker_grid).
    A view of `markers` ((n_env * n_x * n_y, 3)); no arithmetic."""
    n_x, n_y = grid
    if markers.shape[-2] != n_env * n_x * n_y:
        raise ValueError(f"{markers.shape[-2]} markers are not {n_env} grids of {n_x} x {n_y}")
    return markers.view(n_env, n_y, n_x, 3)[..., :2].transpose(1, 2)


class TactilePlugin:
    """Drives a Sim from the engine's relative motion, one engine step at a time.

    `sim` must hold envs whose gels all carry an n_x x n_y marker grid;
    `poses0` ((n_env, 7)) are the indenter poses the envs start from (the
    poses they were built with). Each engine step of length dt is split into
    `substeps` load steps along the constant-velocity motion, run in one
    launch; the observation is that of the last one."""

    def __init__(self, sim, poses0, grid=(7, 9), substeps=1):
        if any(m != grid[0] * grid[1] for m in sim.n_m):
            raise ValueError(f"every env needs {grid[0]} x {grid[1]} markers, got {sorted(set(sim.n_m))}")
        if substeps < 1:
            raise ValueError("substeps must be >= 1")
        self.sim = sim
        self.grid = tuple(grid)
        self.substeps = int(substeps)
        self.pose = np.array(poses0, dtype=np.float64).reshape(sim.n_env, 7)

    def substep_poses(self, v, w, dt):
        """The load-step targets (substeps, n_env, 7) of one engine step."""
        return np.stack([advance_pose(self.pose, v, w, dt * (k + 1) / self.substeps)
                         for k in range(self.substeps)])

    def step_velocity(self, v, w, dt):
        """Moves every indenter at (v, w) ((n_env, 3) each) for dt. Returns
        (observation (n_env, n_x, n_y, 2), status (substeps, n_env)), device
        tensors, not synchronised."""
        poses = self.substep_poses(v, w, dt)
        markers, status = self.sim.step_sequence(poses)
        self.pose = poses[-1]
        return observation(markers[-1], self.sim.n_env, self.grid), status

    def step_relative(self, rel0, rel1, dt):
        """One engine step given the object's pose relative to the sensor at its
        start and end ((n_env, 7) each): the velocities of that motion drive the
        tactile step."""
        v, w = relative_velocity(rel0, rel1, dt)
        return self.step_velocity(v, w, dt)
