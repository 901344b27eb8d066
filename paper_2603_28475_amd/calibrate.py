"""Calibration of the gel's parameters against marker-field recordings.

The paper fits (E, nu, rho, mu) by minimising the mean squared error between
simulated and recorded marker displacement fields over K frames of N
indenters (Sec. 4.2, eqs. loss_function and optimization_problem) with
CMA-ES, popsize 12, the parameters normalised to [0, 1] over fixed ranges
(Supp., Results for Parameters Calibration). Two drivers over the batched
solver:

* `cmaes_fit`: every generation runs popsize x N envs (one per candidate and
  indenter) through the recorded protocol in one batched launch.
* `gradient_fit`: bounded L-BFGS on the normalised parameters with the exact
  gradient of the same loss from the adjoint through the whole protocol
  (autograd.MarkerTrajectory).

The CMA-ES is the (mu/mu_w, lambda) strategy with cumulative step-size
adaptation and rank-one plus rank-mu covariance updates, as set out in
N. Hansen, "The CMA Evolution Strategy: A Tutorial" (2016); a candidate
outside the unit box is drawn again.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch

from scenes.configs import protocol_poses  # noqa: F401  (the recording protocol, re-exported)

# The paper's ranges (Supp., table of parameter ranges): E in Pa there, here MPa
# (1e4..2e5 Pa = 0.01..0.2 MPa); rho is given without a unit as 1e-3..5e-3, read
# as g/mm^3 (1,000..5,000 kg/m^3, around a silicone gel's 1,100); the library
# takes t/mm^3, RHO_TO_LIB times these values.
PAPER_RANGES = {"E": (0.01, 0.2), "nu": (0.4, 0.497), "mu_f": (0.25, 2.5), "density": (1e-3, 5e-3)}
RHO_TO_LIB = 1e-6


@dataclass
class Params:
    """The calibrated parameters (a subset of E, nu, mu_f, density) and their
    ranges; `to_unit` / `from_unit` map to and from [0, 1]."""
    names: tuple = ("E", "nu", "mu_f")
    ranges: dict = field(default_factory=lambda: dict(PAPER_RANGES))

    def lo_hi(self):
        lo = np.array([self.ranges[n][0] for n in self.names])
        hi = np.array([self.ranges[n][1] for n in self.names])
        return lo, hi

    def to_unit(self, v):
        lo, hi = self.lo_hi()
        return (np.asarray(v, dtype=np.float64) - lo) / (hi - lo)

    def from_unit(self, u):
        lo, hi = self.lo_hi()
        return lo + np.clip(np.asarray(u, dtype=np.float64), 0.0, 1.0) * (hi - lo)


def mse(markers, target):
    """Mean over frames and indenters of the squared marker-field error (one
    indenter per leading index of the env axis)."""
    return float(((markers - target) ** 2).sum(axis=-1).sum(axis=-1).mean())


class CMAES:
    """(mu/mu_w, lambda)-CMA-ES in the unit box."""

    def __init__(self, x0, sigma0=0.3, popsize=12, seed=0):
        self.n = n = len(x0)
        self.lam = popsize
        self.mu = popsize // 2
        w = np.log(self.mu + 0.5) - np.log(np.arange(1, self.mu + 1))
        self.w = w / w.sum()
        self.mueff = 1.0 / np.sum(self.w ** 2)
        self.cc = (4 + self.mueff / n) / (n + 4 + 2 * self.mueff / n)
        self.cs = (self.mueff + 2) / (n + self.mueff + 5)
        self.c1 = 2 / ((n + 1.3) ** 2 + self.mueff)
        self.cmu = min(1 - self.c1, 2 * (self.mueff - 2 + 1 / self.mueff) / ((n + 2) ** 2 + self.mueff))
        self.damps = 1 + 2 * max(0.0, math.sqrt((self.mueff - 1) / (n + 1)) - 1) + self.cs
        self.chin = math.sqrt(n) * (1 - 1 / (4 * n) + 1 / (21 * n * n))
        self.m = np.asarray(x0, dtype=np.float64).copy()
        self.sigma = sigma0
        self.C = np.eye(n)
        self.pc = np.zeros(n)
        self.ps = np.zeros(n)
        self.B = np.eye(n)
        self.D = np.ones(n)
        self.gen = 0
        self.rng = np.random.default_rng(seed)

    def ask(self):
        """popsize candidates (lambda, n) in [0, 1]: a sample outside the box is
        drawn again (at most 100 times, then clipped), so that every evaluated
        point is the sample the update uses."""
        self._z = self.rng.standard_normal((self.lam, self.n))
        for k in range(self.lam):
            for _ in range(100):
                x = self.m + self.sigma * (self.B @ (self.D * self._z[k]))
                if np.all((x >= 0.0) & (x <= 1.0)):
                    break
                self._z[k] = self.rng.standard_normal(self.n)
        self._y = (self._z * self.D) @ self.B.T
        return np.clip(self.m + self.sigma * self._y, 0.0, 1.0)

    def tell(self, losses):
        idx = np.argsort(losses)[:self.mu]
        y_w = self.w @ self._y[idx]
        z_w = self.w @ self._z[idx]
        self.m = self.m + self.sigma * y_w
        self.ps = (1 - self.cs) * self.ps + math.sqrt(self.cs * (2 - self.cs) * self.mueff) * (self.B @ z_w)
        self.gen += 1
        hsig = (np.linalg.norm(self.ps) / math.sqrt(1 - (1 - self.cs) ** (2 * self.gen)) / self.chin
                < 1.4 + 2 / (self.n + 1))
        self.pc = (1 - self.cc) * self.pc + hsig * math.sqrt(self.cc * (2 - self.cc) * self.mueff) * y_w
        rank_mu = (self._y[idx].T * self.w) @ self._y[idx]
        self.C = ((1 - self.c1 - self.cmu) * self.C + self.c1 * (np.outer(self.pc, self.pc)
                  + (1 - hsig) * self.cc * (2 - self.cc) * self.C) + self.cmu * rank_mu)
        self.sigma *= math.exp((self.cs / self.damps) * (np.linalg.norm(self.ps) / self.chin - 1))
        self.C = 0.5 * (self.C + self.C.T)
        d2, self.B = np.linalg.eigh(self.C)
        self.D = np.sqrt(np.maximum(d2, 1e-20))


def _set_and_run(sim, mats, poses_env):
    """Resets every env, applies per-env materials and runs the protocol poses
    (S, n_env, 7) in one launch; returns markers (S, sum n_m, 3) on the host."""
    n = sim.n_env
    sim.ctx.set_materials(list(range(n)), mats)
    sim.ctx.reset_envs(list(range(n)))
    markers, status = sim.step_sequence(poses_env)
    sim.stream.synchronize()
    return markers.cpu().numpy(), status.cpu().numpy()


def cmaes_fit(sim, base_mats, poses, target, params: Params, x0_unit, generations=80, popsize=12,
              sigma0=0.3, seed=0, log=None):
    """CMA-ES over `params` for N indenters. `sim` holds popsize x N envs, env
    k * N + i running indenter i for candidate k; base_mats: the N indenters'
    materials (the calibrated entries are replaced; a calibrated density is set
    per env, which the dynamic form reads); poses: (S, N, 7);
    target: (S, N, n_m, 3) recorded marker fields. Returns (best values, best
    loss, loss per generation)."""
    N = len(base_mats)
    assert sim.n_env == popsize * N
    es = CMAES(x0_unit, sigma0, popsize, seed)
    poses_env = np.ascontiguousarray(np.tile(poses, (1, popsize, 1)))
    n_m = target.shape[2]
    best, best_loss, history = None, math.inf, []
    for g in range(generations):
        cand = es.ask()
        mats, dens = [], []
        for k in range(popsize):
            vals = dict(zip(params.names, params.from_unit(cand[k])))
            for i in range(N):
                m = list(base_mats[i])
                for j, key in enumerate(("E", "nu", "mu_f")):
                    if key in vals:
                        m[j] = float(vals[key])
                mats.append(tuple(m))
                dens.append(float(vals["density"]) * RHO_TO_LIB if "density" in vals else 0.0)
        if "density" in params.names:  # per-candidate density of the dynamic form
            sim.ctx.set_densities(list(range(sim.n_env)), dens)
        markers, status = _set_and_run(sim, mats, poses_env)
        markers = markers.reshape(markers.shape[0], popsize, N, n_m, 3)
        losses = np.array([mse(markers[:, k], target) for k in range(popsize)])
        losses[~np.all(status.reshape(status.shape[0], popsize, N) & 1, axis=(0, 2))] = math.inf
        es.tell(losses)
        k = int(np.argmin(losses))
        if losses[k] < best_loss:
            best_loss, best = float(losses[k]), params.from_unit(cand[k])
        history.append(float(losses[k]))
        if log:
            log(f"generation {g}: best {losses[k]:.3e} sigma {es.sigma:.3e}")
    return best, best_loss, history


def gradient_fit(sim, poses, target, params: Params, x0_unit, steps=40, log=None):
    """Bounded L-BFGS (scipy L-BFGS-B) on the unit-box parameters with the exact
    gradient of the MSE loss from the adjoint through the whole protocol.
    `sim` holds the N indenters' envs; poses (S, N, 7); target (S, N, n_m, 3).
    Only E, nu and mu_f can be fitted here. Returns (values, loss per
    evaluation)."""
    from scipy.optimize import minimize

    from .autograd import MarkerTrajectory
    N = sim.n_env
    lo, hi = params.lo_hi()
    idx = {"E": 0, "nu": 1, "mu_f": 2}
    sel = [idx[n] for n in params.names]
    base = np.array([[m[0], m[1], m[2], 0, 0, 0, 0, 0, 0] for m in sim.mats], dtype=np.float64)
    tgt = torch.as_tensor(target.reshape(target.shape[0], -1, 3), device=sim.device)
    S = target.shape[0]
    history = []

    def fun(u):
        uu = torch.tensor(np.clip(u, 0.0, 1.0), dtype=torch.float64, requires_grad=True)
        vals = torch.as_tensor(lo) + uu * torch.as_tensor(hi - lo)
        theta = torch.as_tensor(base).clone()
        theta[:, sel] = vals[None, :].expand(N, -1)
        m = MarkerTrajectory.apply(theta, sim, poses)
        loss = ((m - tgt) ** 2).sum(dim=-1).sum() / (S * N)
        loss.backward()
        L = loss.item()
        history.append(L)
        if log:
            log(f"evaluation {len(history)}: loss {L:.3e} values {vals.detach().numpy()}")
        return L, uu.grad.numpy().copy()

    res = minimize(fun, np.asarray(x0_unit, dtype=np.float64), jac=True, method="L-BFGS-B",
                   bounds=[(0.0, 1.0)] * len(sel), options=dict(maxiter=steps, ftol=1e-15, gtol=1e-12))
    return params.from_unit(res.x), history
