"""The plugin surface towards a physics engine, and the policy's tactile
observation.

Per physics step the engine reports where the grasped object sits relative
to the sensor at the start and at the end of the step, or the object's
velocity; that motion drives the tactile simulation (Sec. 3.3, "Integrating
to Physics Engine"), and the marker displacement field is handed back as
part of the observation. The policy sees the field of one finger as a 7 x 9
grid of in-plane displacements (Sec. 5.3, online RL).

The pose integration of the motion runs in the library (t2r_step_velocity,
t2r_step_relative); this module only marshals arrays and reshapes the marker
output into the observation.
"""

from __future__ import annotations

import numpy as np
import torch


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

    `sim` must hold envs whose gels all carry an n_x x n_y marker grid. Each
    engine step is split into `substeps` load steps along the constant-velocity
    motion from every env's current pose, all in one launch; the observation is
    that of the last one."""

    def __init__(self, sim, grid=(7, 9), substeps=1):
        if any(m != grid[0] * grid[1] for m in sim.n_m):
            raise ValueError(f"every env needs {grid[0]} x {grid[1]} markers, got {sorted(set(sim.n_m))}")
        if substeps < 1:
            raise ValueError("substeps must be >= 1")
        self.sim = sim
        self.grid = tuple(grid)
        self.substeps = int(substeps)

    def _buffers(self):
        markers = torch.zeros((self.substeps, sum(self.sim.n_m), 3), dtype=torch.float64, device=self.sim.device)
        status = torch.zeros((self.substeps, self.sim.n_env), dtype=torch.int32, device=self.sim.device)
        return markers, status

    def _dev(self, a, width):
        t = torch.as_tensor(np.asarray(a, dtype=np.float64) if not torch.is_tensor(a) else a,
                            dtype=torch.float64, device=self.sim.device).contiguous()
        if tuple(t.shape) != (self.sim.n_env, width):
            raise ValueError(f"expected ({self.sim.n_env}, {width}), got {tuple(t.shape)}")
        return t

    def step_velocity(self, v, w, dt):
        """Moves every indenter at linear velocity v and world-frame angular
        velocity w ((n_env, 3) each, mm/s and rad/s) for dt seconds
        (t2r_step_velocity). Returns (observation (n_env, n_x, n_y, 2), status
        (substeps, n_env)), device tensors, not synchronised."""
        vw = self._dev(np.concatenate([np.asarray(v, dtype=np.float64), np.asarray(w, dtype=np.float64)], axis=1)
                       if not torch.is_tensor(v) else torch.cat([v, w], dim=1), 6)
        markers, status = self._buffers()
        self.sim.ctx.step_velocity(self.substeps, dt, vw, None, markers, None, status)
        return observation(markers[-1], self.sim.n_env, self.grid), status

    def step_relative(self, rel0, rel1):
        """One engine step given the object's pose relative to the sensor at its
        start and end ((n_env, 7) each, t2r_step_relative): that motion, applied
        to every env's current pose. Returns as step_velocity."""
        markers, status = self._buffers()
        self.sim.ctx.step_relative(self.substeps, self._dev(rel0, 7), self._dev(rel1, 7), None, markers, None,
                                   status)
        return observation(markers[-1], self.sim.n_env, self.grid), status
