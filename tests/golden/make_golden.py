"""Writes the stored expected values used by the GPU parity tests.

Calls only the CPU oracle (oracle/) on the seeded scenes (scenes/); nothing
here comes from the HIP path. The paper prints no worked numeric example, so
these values are pinned by the oracle's own tests (finite differences, closed
forms, brute force, invariants), not by the paper.

    python tests/golden/make_golden.py
"""

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.sim import simulate  # noqa: E402
from scenes.configs import (calibration_micro, micro_press, peg_press_484v, self_contact_press,  # noqa: E402
                            sphere_press_484v, two_finger_grasp, two_pin_press)

CALIB_THETA = (0.12, 0.45, 0.6)        # hidden (E MPa, nu, mu_f) of the calibration recordings
CALIB_DYNAMIC = dict(density=2.5e-9, dt=2e-4)  # hidden density (t/mm^3) of the dynamic recordings


def sphere_press():
    w = sphere_press_484v()
    env = w.envs[0]
    t = time.time()
    r = simulate(w.meshes["c1"], w.indenters["sphere3"], env, mode="newton")
    np.savez_compressed(os.path.join(HERE, "sphere_press_484v_newton.npz"),
                        x=np.array(r.x), markers=np.array(r.markers), poses=env.poses,
                        n_active=np.array(r.n_active), d_min=np.array(r.d_min))
    print(f"sphere_press_484v: {time.time() - t:.1f}s, active {r.n_active}")


def micro_friction():
    w = micro_press(mesh="micro3", indenter="sphere_small", depth=0.12, n_steps=3, mu_f=0.5,
                    shear=(0.06, 0.03), n_shear=3)
    env = w.envs[0]
    t = time.time()
    r = simulate(w.meshes["micro3"], w.indenters["sphere_small"], env, mode="newton")
    np.savez_compressed(os.path.join(HERE, "micro3_friction_newton.npz"),
                        x=np.array(r.x), markers=np.array(r.markers), poses=env.poses,
                        n_active=np.array(r.n_active))
    print(f"micro3_friction: {time.time() - t:.1f}s, active {r.n_active}")


def peg_press_friction():
    """Every pair kind active (tilted flat-ended peg), lagged friction and shear."""
    w = peg_press_484v(mu_f=0.5, shear=(0.1, 0.05), n_shear=2)
    env = w.envs[0]
    t = time.time()
    r = simulate(w.meshes["c1"], w.indenters["peg4"], env, mode="newton")
    np.savez_compressed(os.path.join(HERE, "peg_press_484v_friction_newton.npz"),
                        x=np.array(r.x), markers=np.array(r.markers), poses=env.poses,
                        n_active=np.array(r.n_active), d_min=np.array(r.d_min))
    print(f"peg_press_484v_friction: {time.time() - t:.1f}s, active {r.n_active}")


def peg_press_friction_unstructured():
    """The same scene on the unstructured (Delaunay) version of the 484-vertex
    gel; the mesh itself is stored too, so that a test can check that it
    regenerates bit for bit."""
    w = peg_press_484v(mu_f=0.5, shear=(0.1, 0.05), n_shear=2, mesh="c1u")
    env = w.envs[0]
    g = w.meshes["c1u"]
    t = time.time()
    r = simulate(g, w.indenters["peg4"], env, mode="newton")
    np.savez_compressed(os.path.join(HERE, "peg_press_484v_unstructured_friction_newton.npz"),
                        x=np.array(r.x), markers=np.array(r.markers), poses=env.poses,
                        n_active=np.array(r.n_active), d_min=np.array(r.d_min),
                        mesh_X=g.X, mesh_tets=g.tets)
    print(f"peg_press_484v_unstructured_friction: {time.time() - t:.1f}s, active {r.n_active}")


def peg_press_mollified():
    """The tilted peg scene with lagged friction and shear, edge-edge barriers
    weighted by the parallel-edge mollifier; per step, the number of edge-edge
    pairs below the mollifier's threshold is stored too."""
    from oracle.barrier import EDGE_MOLLIFIER_REL, edge_cross_derivatives
    from oracle.problem import EE
    from oracle.sim import build
    w = peg_press_484v(mu_f=0.5, shear=(0.1, 0.05), n_shear=2)
    env = w.envs[0]
    t = time.time()
    r = simulate(w.meshes["c1"], w.indenters["peg4"], env, mode="newton", ee_mollifier=True)
    gel, ind, prob = build(w.meshes["c1"], w.indenters["peg4"], env, ee_mollifier=True)
    n_moll = []
    for s, x in enumerate(r.x):
        prob.set_pose(env.poses[s + 1])
        pairs, res = prob.active(x)
        ee = np.nonzero(pairs["kind"] == EE)[0]
        idx = pairs["idx"][ee]
        ar = gel.X[idx[:, 1]] - gel.X[idx[:, 0]]
        br = ind.Y[idx[:, 3] - prob.nv] - ind.Y[idx[:, 2] - prob.nv]
        eps = EDGE_MOLLIFIER_REL * np.sum(ar * ar, 1) * np.sum(br * br, 1)
        n_moll.append(int(np.sum(edge_cross_derivatives(res["Z"][ee])[0] < eps)))
    np.savez_compressed(os.path.join(HERE, "peg_press_484v_mollifier_friction_newton.npz"),
                        x=np.array(r.x), markers=np.array(r.markers), poses=env.poses,
                        n_active=np.array(r.n_active), d_min=np.array(r.d_min), n_mollified=np.array(n_moll))
    print(f"peg_press_484v_mollifier_friction: {time.time() - t:.1f}s, active {r.n_active}, mollified {n_moll}")


def self_contact_friction():
    """Two gel blocks 0.08 mm apart; a small sphere presses the first next to
    the gap and slides it towards the second with friction 0.8: gel surface
    pairs of the two blocks come within dhat (self-contact on)."""
    from oracle.problem import GEE, GVF
    from oracle.sim import build
    w = self_contact_press(depth=0.3, xy=(-0.45, 0.0), mu_f=0.8, shear=(0.25, 0.0), n_shear=3)
    env = w.envs[0]
    g = w.meshes["two_block"]
    t = time.time()
    r = simulate(g, w.indenters["sphere_small"], env, mode="newton", self_contact=True)
    gel, ind, prob = build(g, w.indenters["sphere_small"], env, self_contact=True)
    n_self = []
    for s, x in enumerate(r.x):
        prob.set_pose(env.poses[s + 1])
        pairs, _ = prob.active(x)
        n_self.append(int(np.isin(pairs["kind"], (GVF, GEE)).sum()))
    np.savez_compressed(os.path.join(HERE, "self_contact_friction_newton.npz"),
                        x=np.array(r.x), markers=np.array(r.markers), poses=env.poses,
                        n_active=np.array(r.n_active), n_self=np.array(n_self))
    print(f"self_contact_friction: {time.time() - t:.1f}s, active {r.n_active}, self {n_self}")


def two_finger():
    """The two finger sensors of a parallel gripper closing on one sphere held
    off-centre, with friction: each sensor's env against the oracle's Newton."""
    w = two_finger_grasp()
    t = time.time()
    xs, ms = [], []
    for env in w.envs:
        r = simulate(w.meshes["micro3"], w.indenters["sphere_small"], env, mode="newton", tol=1e-12)
        xs.append(np.array(r.x))
        ms.append(np.array(r.markers))
    np.savez_compressed(os.path.join(HERE, "two_finger_grasp_newton.npz"), x=np.stack(xs), markers=np.stack(ms),
                        poses=np.stack([e.poses for e in w.envs]))
    print(f"two_finger: {time.time() - t:.1f}s")


def two_pin():
    """Two pins of one rigid fixture pressed and slid with friction on the
    32-vertex gel; per step, the number of active pairs on each pin."""
    from oracle.sim import build
    w = two_pin_press()
    env = w.envs[0]
    t = time.time()
    r = simulate(w.meshes["micro3"], w.indenters["two_pin"], env, mode="newton", tol=1e-12)
    gel, ind, prob = build(w.meshes["micro3"], w.indenters["two_pin"], env)
    half = len(ind.Y) // 2
    per_pin = []
    for s, x in enumerate(r.x):
        prob.set_pose(env.poses[s + 1])
        idx = prob.active(x)[0]["idx"]
        ind_ids = idx[idx >= prob.nv] - prob.nv
        per_pin.append([int(np.any(ind_ids < half)), int(np.any(ind_ids >= half))])
    np.savez_compressed(os.path.join(HERE, "two_pin_press_newton.npz"), x=np.array(r.x),
                        markers=np.array(r.markers), poses=env.poses, pins_in_contact=np.array(per_pin))
    print(f"two_pin: {time.time() - t:.1f}s, pins in contact {per_pin}")


def calibration_targets():
    """Synthetic recordings for the calibration driver: the oracle's Newton
    marker fields of the calibration scene (two indenters, the recording
    protocol) at hidden parameters, quasi-static and in the dynamic form."""
    w, poses = calibration_micro(CALIB_THETA)
    t = time.time()
    out = {}
    for key, dyn in (("static", None), ("dynamic", CALIB_DYNAMIC)):
        ms = []
        for env in w.envs:
            r = simulate(w.meshes[env.mesh], w.indenters[env.indenter], env, mode="newton", tol=1e-12,
                         dynamic=dyn)
            ms.append(np.array(r.markers))
        out[key] = np.stack(ms, axis=1)     # (S, 2 indenters, n_m, 3)
    np.savez_compressed(os.path.join(HERE, "calibration_micro3_newton.npz"), poses=poses,
                        theta=np.array(CALIB_THETA), density=CALIB_DYNAMIC["density"], dt=CALIB_DYNAMIC["dt"],
                        **out)
    print(f"calibration_targets: {time.time() - t:.1f}s")


if __name__ == "__main__":
    which = sys.argv[1:] or ["micro_friction", "sphere_press", "peg_press_friction",
                             "peg_press_friction_unstructured", "calibration_targets", "peg_press_mollified",
                             "self_contact_friction", "two_finger", "two_pin"]
    for name in which:
        globals()[name]()
