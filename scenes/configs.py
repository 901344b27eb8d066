"""Seeded workload recipes: which gel, which indenter, which material and which
pose schedule each environment gets.

Every random draw for environment `e` of workload number `k` comes from
numpy.random.default_rng(SeedSequence([k, e])), so any subset of
environments can be regenerated on its own.

A pose schedule holds S+1 poses: pose[0] is the starting pose (indenter lowest
point 2*dhat above the gel top, i.e. press depth -2*dhat) and pose[s] is the
target of load step s. Press depth delta is measured as the gel thickness
minus the lowest world z of the indenter's vertices.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .indenters import (Indenter, end_on_peg, flat_plate, hex_nut, icosphere,
                        quat_from_axis_angle, quat_mul, rigid_set, rotation_matrix)
from .mesh import GelMesh, hex_kuhn_gel, marker_grid, mesh_class

DHAT = 0.05      # mm
KAPPA = 1.0e3    # N/mm
EPS_V = 1.0e-3   # mm per step
NU = 0.45


@dataclass
class EnvSpec:
    mesh: str
    indenter: str
    E: float
    nu: float
    mu_f: float
    poses: np.ndarray                 # (S+1, 7)
    eps_v: float = EPS_V
    dhat: float = DHAT
    kappa: float = KAPPA
    extra: dict = field(default_factory=dict)

    def material(self):
        return (self.E, self.nu, self.mu_f, self.eps_v, self.dhat, self.kappa)


@dataclass
class Workload:
    name: str
    number: int
    meshes: dict                      # name -> GelMesh
    indenters: dict                   # name -> Indenter
    envs: list                        # [EnvSpec]
    precision: str = "f64"            # "f64" or "mixed"
    tol: float = 1e-6                 # mm, on the preconditioned gradient
    description: str = ""

    @property
    def n_steps(self) -> int:
        return int(self.envs[0].poses.shape[0] - 1)


INDENTERS = {
    "sphere3": lambda: icosphere(3.0, 2),
    "peg4": lambda: end_on_peg(4.0, 10.0, 64, 8),
    "nut8": lambda: hex_nut(8.0, 4.7, 4.2),
    "plate": lambda: flat_plate(2.0, 0.0, 3),
    "sphere_small": lambda: icosphere(0.6, 1),
    "sphere_sym": lambda: icosphere(0.6, 1, yaw=-np.pi / 4),
    "two_pin": lambda: rigid_set([icosphere(0.5, 1), icosphere(0.5, 1, yaw=0.3)],
                                 [(-0.75, -0.3, 0.0), (0.75, 0.35, 0.1)], name="two_pin"),
}


def pose_at_depth(ind: Indenter, q, xy, depth: float, thickness: float) -> np.ndarray:
    """Pose with rotation q whose lowest indenter vertex sits `depth` below the gel top."""
    R = rotation_matrix(q)
    zmin = float((ind.Y @ R.T)[:, 2].min())
    tz = thickness - depth - zmin
    return np.array([xy[0], xy[1], tz, *q], dtype=np.float64)


def press_schedule(ind, q, xy, depth, thickness, n_press, dhat=DHAT,
                   shear=(0.0, 0.0), n_shear=0, clearance=None) -> np.ndarray:
    """Pose 0 `clearance` above the gel (default 2 dhat), then n_press steps to
    `depth`, then n_shear in-plane steps adding up to `shear`."""
    poses = [pose_at_depth(ind, q, xy, -(2.0 * dhat if clearance is None else clearance), thickness)]
    for s in range(1, n_press + 1):
        poses.append(pose_at_depth(ind, q, xy, depth * s / n_press, thickness))
    last = poses[-1].copy()
    for s in range(1, n_shear + 1):
        p = last.copy()
        p[0] += shear[0] * s / n_shear
        p[1] += shear[1] * s / n_shear
        poses.append(p)
    return np.stack(poses)


def _rng(k, e):
    return np.random.default_rng(np.random.SeedSequence([k, e]))


def _yaw_tilt(yaw, tilt):
    return quat_mul(quat_from_axis_angle((0, 0, 1), yaw), quat_from_axis_angle((0, 1, 0), tilt))


def sphere_press_484v(n_envs: int = 1, n_steps: int = 10) -> Workload:
    """Plain single env: 8x8x2 mm gel (484 v, 1800 t), r=3 mm icosphere pressed
    0.6 mm in 10 steps at a seeded xy offset in [-1,1]^2 mm; E=0.3, nu=0.45, no friction."""
    g = mesh_class("c1")
    ind = INDENTERS["sphere3"]()
    envs = []
    for e in range(n_envs):
        r = _rng(1, e)
        xy = r.uniform(-1.0, 1.0, 2)
        poses = press_schedule(ind, (1.0, 0, 0, 0), xy, 0.6, g.thickness, n_steps)
        envs.append(EnvSpec("c1", "sphere3", 0.3, NU, 0.0, poses))
    return Workload("sphere_press_484v", 1, {"c1": g}, {"sphere3": ind}, envs, "f64", 1e-6,
                    "1 env, 8x8x2 mm gel 10x10x3 hexes, icosphere r=3 pressed 0.6 mm in 10 steps")


def peg_press_484v(tilt_deg: float = 1.0, depth: float = 0.3, n_steps: int = 3, mu_f: float = 0.0,
                   shear=(0.0, 0.0), n_shear: int = 0, mesh: str = "c1") -> Workload:
    """Small parity scene with every pair kind active: the 8x8x2 mm gel (484 v)
    pressed by the end-on peg r=4 mm, tilted a little so that its flat face, its
    rim edges and its rim vertices all come within dhat of the gel. mesh "c1u":
    the same gel tetrahedralised unstructured."""
    assert mesh in ("c1", "c1u")
    g = mesh_class(mesh)
    ind = INDENTERS["peg4"]()
    q = _yaw_tilt(0.3, np.deg2rad(tilt_deg))
    poses = press_schedule(ind, q, (0.5, -0.3), depth, g.thickness, n_steps, shear=shear,
                           n_shear=n_shear)
    env = EnvSpec(mesh, "peg4", 0.3, NU, mu_f, poses)
    return Workload("peg_press_484v" + ("u" if mesh == "c1u" else ""), 6, {mesh: g}, {"peg4": ind}, [env],
                    "f64", 1e-6,
                    "1 env, 484-vertex gel, slightly tilted end-on peg")


def peg_press_shear_12k(n_envs: int = 1) -> Workload:
    """Single env, 20x16x4 mm gel with 40x32x8 hexes (12,177 v, 61,440 t), end-on peg
    r=4 mm with tilt U[-5,5] deg and yaw U[0,360) deg; 20 press steps to 0.8 mm then
    20 shear steps totalling +0.5 mm along x; E U[0.2,0.5] MPa, mu=0.5."""
    g = mesh_class("12k")
    ind = INDENTERS["peg4"]()
    envs = []
    for e in range(n_envs):
        r = _rng(2, e)
        tilt = np.deg2rad(r.uniform(-5.0, 5.0))
        yaw = np.deg2rad(r.uniform(0.0, 360.0))
        E = r.uniform(0.2, 0.5)
        poses = press_schedule(ind, _yaw_tilt(yaw, tilt), (0.0, 0.0), 0.8, g.thickness, 20,
                               shear=(0.5, 0.0), n_shear=20)
        envs.append(EnvSpec("12k", "peg4", E, NU, 0.5, poses))
    return Workload("peg_press_shear_12k", 2, {"12k": g}, {"peg4": ind}, envs, "f64", 1e-6,
                    "1 env, 12k-vertex gel, tilted peg, 0.8 mm press + 0.5 mm shear, friction 0.5")


def peg_batch_5k(n_envs: int = 2048, n_steps: int = 20, precision: str = "mixed",
                 mesh: str = "5k") -> Workload:
    """Uniform batch: n_envs x 5k-vertex gels (4,914 v, 24,000 t), peg at xy U[-2,2]^2 mm,
    yaw U[0,360) deg, 20 press steps to depth U[0.3,1.0] mm, E U[0.2,0.5], mu U[0.3,0.8].
    mesh "5ku": the same box and points tetrahedralised unstructured (27,063 t)."""
    assert mesh in ("5k", "5ku")
    g = mesh_class(mesh)
    ind = INDENTERS["peg4"]()
    envs = []
    for e in range(n_envs):
        r = _rng(3, e)
        xy = r.uniform(-2.0, 2.0, 2)
        yaw = np.deg2rad(r.uniform(0.0, 360.0))
        depth = r.uniform(0.3, 1.0)
        E = r.uniform(0.2, 0.5)
        mu = r.uniform(0.3, 0.8)
        poses = press_schedule(ind, _yaw_tilt(yaw, 0.0), xy, depth, g.thickness, n_steps)
        envs.append(EnvSpec(mesh, "peg4", E, NU, mu, poses))
    return Workload(f"peg_batch_{n_envs}x{mesh}", 3, {mesh: g}, {"peg4": ind}, envs, precision, 1e-6,
                    f"{n_envs} envs, 5k-vertex gels ({'unstructured' if mesh == '5ku' else 'Kuhn'}), "
                    f"peg, {n_steps} press steps")


def mixed_batch(n_envs: int = 512, n_steps: int = 20, precision: str = "mixed") -> Workload:
    """Uneven batch: gel class uniform over {2k, 5k, 12k}, indenter uniform over
    {sphere r=3, peg r=4, hex nut 8 mm across flats}; pose and press as the uniform batch."""
    meshes = {k: mesh_class(k) for k in ("2k", "5k", "12k")}
    inds = {k: INDENTERS[k]() for k in ("sphere3", "peg4", "nut8")}
    envs = []
    for e in range(n_envs):
        r = _rng(4, e)
        mk = ("2k", "5k", "12k")[int(r.integers(0, 3))]
        ik = ("sphere3", "peg4", "nut8")[int(r.integers(0, 3))]
        xy = r.uniform(-2.0, 2.0, 2)
        yaw = np.deg2rad(r.uniform(0.0, 360.0))
        depth = r.uniform(0.3, 1.0)
        E = r.uniform(0.2, 0.5)
        mu = r.uniform(0.3, 0.8)
        poses = press_schedule(inds[ik], _yaw_tilt(yaw, 0.0), xy, depth,
                               meshes[mk].thickness, n_steps)
        envs.append(EnvSpec(mk, ik, E, NU, mu, poses))
    return Workload(f"mixed_batch_{n_envs}", 4, meshes, inds, envs, precision, 1e-6,
                    f"{n_envs} envs over 3 gel sizes and 3 indenters")


def uneven_small(n_steps: int = 4, precision: str = "f64") -> Workload:
    """Small uneven batch for parity: two gel sizes (484 and 2,142 vertices) and
    all three indenter shapes in one batch, seeded poses, 0.3 mm press."""
    meshes = {k: mesh_class(k) for k in ("c1", "2k")}
    inds = {k: INDENTERS[k]() for k in ("sphere3", "peg4", "nut8")}
    combos = [("c1", "sphere3"), ("2k", "peg4"), ("c1", "nut8"), ("2k", "sphere3")]
    envs = []
    for e, (mk, ik) in enumerate(combos):
        r = _rng(7, e)
        xy = r.uniform(-0.5, 0.5, 2)
        yaw = np.deg2rad(r.uniform(0.0, 360.0))
        E = r.uniform(0.2, 0.5)
        poses = press_schedule(inds[ik], _yaw_tilt(yaw, np.deg2rad(1.0)), xy, 0.3, meshes[mk].thickness,
                               n_steps)
        envs.append(EnvSpec(mk, ik, E, NU, 0.0, poses))
    return Workload("uneven_small", 7, meshes, inds, envs, precision, 1e-6,
                    "4 envs over 2 gel sizes and 3 indenters")


def adjoint_peg_5k(n_envs: int = 64) -> Workload:
    """64 x 5k-vertex gels, peg: 10 press steps to 0.6 mm then 10 shear steps of 0.5 mm
    total. Hidden per-env parameters theta* (E, nu, mu, pose offset) are drawn here and
    kept in EnvSpec.extra; the gradient is evaluated at a perturbed theta_0."""
    g = mesh_class("5k")
    ind = INDENTERS["peg4"]()
    envs = []
    for e in range(n_envs):
        r = _rng(5, e)
        E = r.uniform(0.2, 0.5)
        nu = r.uniform(0.40, 0.48)
        mu = r.uniform(0.3, 0.8)
        dt = r.uniform(-0.2, 0.2, 3)
        dw = np.deg2rad(r.uniform(-2.0, 2.0, 3))
        # pose 0 starts 0.6 mm above the gel: the rigid offsets (|dt_z| <= 0.3 mm,
        # tilts of up to 3 deg over the 4 mm peg radius) move every pose,
        # the start pose included, and it must stay clear of the gel
        poses = press_schedule(ind, (1.0, 0, 0, 0), (0.0, 0.0), 0.6, g.thickness, 10,
                               shear=(0.5, 0.0), n_shear=10, clearance=0.6)
        theta_star = dict(E=E, nu=nu, mu=mu, dt=dt, dw=dw)
        theta0 = dict(E=1.2 * E, nu=nu - 0.02, mu=mu + 0.1, dt=dt + 0.1, dw=dw + np.deg2rad(1.0))
        envs.append(EnvSpec("5k", "peg4", theta0["E"], theta0["nu"], theta0["mu"], poses,
                            extra=dict(theta_star=theta_star, theta0=theta0)))
    return Workload(f"adjoint_{n_envs}x5k", 5, {"5k": g}, {"peg4": ind}, envs, "f64", 1e-6,
                    f"{n_envs} envs, adjoint of marker loss")


def micro_press(mesh: str = "micro2", indenter: str = "sphere_small", depth: float = 0.15,
                n_steps: int = 3, xy=(0.1, -0.05), E: float = 0.3, nu: float = NU,
                mu_f: float = 0.0, shear=(0.0, 0.0), n_shear: int = 0, q=(1.0, 0, 0, 0)) -> Workload:
    """Tiny scene for brute-force checks: a 1- to 9-hex gel and a small indenter."""
    g = mesh_class(mesh)
    ind = INDENTERS[indenter]()
    poses = press_schedule(ind, q, xy, depth, g.thickness, n_steps, shear=shear, n_shear=n_shear)
    env = EnvSpec(mesh, indenter, E, nu, mu_f, poses)
    return Workload(f"micro_{mesh}_{indenter}", 0, {mesh: g}, {indenter: ind}, [env], "f64", 1e-10,
                    "micro scene")


def two_block_gel(size=(1.5, 1.5, 1.0), cells=(3, 3, 2), gap: float = 0.08, markers=(3, 3)) -> GelMesh:
    """Two box gels side by side along x, `gap` mm apart, both fixed at the bottom:
    one gel mesh whose surfaces can meet (self-contact scenes). Markers on the
    first block's top face."""
    a = hex_kuhn_gel(size, cells, markers)
    off = np.array([size[0] / 2 + gap / 2, 0.0, 0.0])
    X = np.concatenate([a.X - off, a.X + off])
    tets = np.concatenate([a.tets, a.tets + a.n_verts]).astype(np.int32)
    fixed = np.concatenate([a.fixed, a.fixed])
    mk = marker_grid(size[:2], markers) - off[:2]
    return GelMesh(X=X, tets=tets, fixed=fixed, size=(2 * size[0] + gap, size[1], size[2]), cells=cells,
                   markers=mk, name="two_block")


def self_contact_press(depth: float = 0.3, n_steps: int = 3, xy=(-0.3, 0.0), gap: float = 0.08,
                       mu_f: float = 0.0, shear=(0.0, 0.0), n_shear: int = 0) -> Workload:
    """Self-contact scene: a small sphere (r = 0.6 mm) presses the first of two
    gel blocks next to the gap between them, so that the block's side wall bulges
    towards the second block's."""
    g = two_block_gel(gap=gap)
    ind = INDENTERS["sphere_small"]()
    poses = press_schedule(ind, (1.0, 0.0, 0.0, 0.0), xy, depth, g.thickness, n_steps, shear=shear,
                           n_shear=n_shear)
    env = EnvSpec("two_block", "sphere_small", 0.3, NU, mu_f, poses)
    return Workload("self_contact_press", 0, {"two_block": g}, {"sphere_small": ind}, [env], "f64", 1e-6,
                    "1 env, two gel blocks with a gap, small sphere pressing next to the gap")


def two_pin_press(n_steps: int = 3, depth: float = 0.2, mu_f: float = 0.5, shear=(0.1, 0.05),
                  n_shear: int = 2) -> Workload:
    """Two small spheres held in one rigid fixture (one indenter made of two
    closed meshes, the second 0.1 mm higher) pressed into the 32-vertex gel and
    slid with friction: two separate contact patches that move together."""
    g = mesh_class("micro3")
    ind = INDENTERS["two_pin"]()
    poses = press_schedule(ind, _yaw_tilt(0.2, 0.0), (0.0, 0.0), depth, g.thickness, n_steps, shear=shear,
                           n_shear=n_shear)
    env = EnvSpec("micro3", "two_pin", 0.3, NU, mu_f, poses)
    return Workload("two_pin_press", 0, {"micro3": g}, {"two_pin": ind}, [env], "f64", 1e-6,
                    "1 env, two pins of one rigid fixture on the 32-vertex gel")


def gripper_sensor_frames(w: float):
    """Frames of two sensors facing each other across a parallel gripper: sensor
    k's gel bottom centre sits at (-w, 0, 0) (k = 0) or (+w, 0, 0) (k = 1) of the
    gripper frame, its gel normal (local +z) pointing at the gripper's centre.
    Returns [(centre, unit quaternion)] for the two sensors."""
    s = math.sqrt(0.5)
    return [(np.array([-w, 0.0, 0.0]), np.array([s, 0.0, s, 0.0])),     # local z -> gripper +x
            (np.array([w, 0.0, 0.0]), np.array([s, 0.0, -s, 0.0]))]     # local z -> gripper -x


def object_in_sensor(obj_t, obj_q, centre, q_sensor) -> np.ndarray:
    """The object's pose (t, q) relative to a sensor: the frame change
    R_s^T (t - c), q_s^-1 q."""
    qc = np.array([q_sensor[0], -q_sensor[1], -q_sensor[2], -q_sensor[3]])
    t = rotation_matrix(q_sensor).T @ (np.asarray(obj_t, dtype=np.float64) - centre)
    q = _qmul(qc, np.asarray(obj_q, dtype=np.float64))
    return np.concatenate([t, q / np.linalg.norm(q)])


def two_finger_grasp(n_steps: int = 3, squeeze: float = 0.12, obj_t=(0.04, 0.2, -0.15),
                     obj_yaw_deg: float = 20.0, mu_f: float = 0.5) -> Workload:
    """A parallel gripper with a sensor on each finger closing on one small
    sphere (r = 0.6 mm) held off the gripper's centre (`obj_t`): one env per
    sensor gel (the 32-vertex gel), each driven by the object's pose relative
    to its own sensor as the fingers close until the gels are squeezed by about
    `squeeze` mm. The sensors see different poses because of the offset."""
    g = mesh_class("micro3")
    ind = INDENTERS["sphere_small"]()
    r = float(np.linalg.norm(ind.Y, axis=1).max())
    q_obj = quat_from_axis_angle((1, 0, 0), math.radians(obj_yaw_deg))
    w0 = g.thickness + r + 2.0 * DHAT + abs(obj_t[0])
    w1 = g.thickness + r - squeeze
    envs = []
    for k in range(2):
        poses = []
        for i in range(n_steps + 1):
            w = w0 + (w1 - w0) * i / n_steps
            c, qs = gripper_sensor_frames(w)[k]
            poses.append(object_in_sensor(obj_t, q_obj, c, qs))
        envs.append(EnvSpec("micro3", "sphere_small", 0.3, NU, mu_f, np.array(poses)))
    return Workload("two_finger_grasp", 0, {"micro3": g}, {"sphere_small": ind}, envs, "f64", 1e-6,
                    "2 envs: the two finger sensors of a parallel gripper on one sphere")


WORKLOADS = {
    "sphere_press_484v": sphere_press_484v,
    "peg_press_shear_12k": peg_press_shear_12k,
    "peg_batch_5k": peg_batch_5k,
    "mixed_batch": mixed_batch,
    "adjoint_peg_5k": adjoint_peg_5k,
    "micro_press": micro_press,
    "peg_press_484v": peg_press_484v,
    "uneven_small": uneven_small,
}


def make_workload(name: str, **kw) -> Workload:
    return WORKLOADS[name](**kw)


def protocol_poses(pose0, press=1.0, slide=1.0, rotate_deg=2.0, d_press=0.1, d_slide=0.1, d_rot_deg=0.5,
                   slide_axis=(1.0, 0.0, 0.0)):
    """The recording protocol as poses (S, 7) after `pose0` (the indenter just
    touching): press by `press` mm in `d_press` steps, slide by `slide` mm along
    `slide_axis`, rotate by `rotate_deg` about the vertical axis."""
    pose0 = np.asarray(pose0, dtype=np.float64)
    out = []
    p = pose0.copy()
    for _ in range(int(round(press / d_press))):
        p = p.copy()
        p[2] -= d_press
        out.append(p)
    ax = np.asarray(slide_axis, dtype=np.float64)
    for _ in range(int(round(slide / d_slide))):
        p = p.copy()
        p[:3] += d_slide * ax
        out.append(p)
    h = math.radians(d_rot_deg) / 2
    dq = np.array([math.cos(h), 0.0, 0.0, math.sin(h)])
    for _ in range(int(round(rotate_deg / d_rot_deg))):
        p = p.copy()
        p[3:] = _qmul(dq, p[3:])
        out.append(p)
    return np.stack(out)


def _qmul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def calibration_micro(theta, n_copies: int = 1):
    """The calibration scene: the 32-vertex gel with a small sphere and a tilted
    plate (N = 2 indenters), friction, driven by the recording protocol scaled to
    the 1 mm gel (press 0.2 mm, slide 0.1 mm, rotate 1 deg, in 0.05 mm, 0.05 mm
    and 0.5 deg steps); theta = (E, nu, mu_f); n_copies of the pair of envs.
    Returns (workload, poses (S, 2, 7) of the protocol after pose 0)."""
    import dataclasses
    q = np.array([0.99996192, 0.00610865, 0.00436331, 0.0])
    ws = micro_press(mesh="micro3", indenter="sphere_small", depth=0.1, n_steps=1)
    wp = micro_press(mesh="micro3", indenter="plate", depth=0.05, n_steps=1, xy=(0.1, -0.05),
                     q=tuple(q / np.linalg.norm(q)))
    envs, poses = [], []
    for wk in (ws, wp):
        e = wk.envs[0]
        P = protocol_poses(e.poses[0], press=0.2, slide=0.1, rotate_deg=1.0, d_press=0.05, d_slide=0.05)
        poses.append(P)
        envs.append(dataclasses.replace(e, E=theta[0], nu=theta[1], mu_f=theta[2],
                                        poses=np.concatenate([e.poses[:1], P])))
    w = dataclasses.replace(ws, name="calibration_micro3",
                            indenters={"sphere_small": INDENTERS["sphere_small"](), "plate": INDENTERS["plate"]()},
                            envs=envs * n_copies)
    return w, np.stack(poses, axis=1)

