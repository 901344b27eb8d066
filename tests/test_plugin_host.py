"""Host-side pins of the oracle's pose integration for the physics-engine
input (the velocities of a pose change and their integration are inverse to
each other and agree with closed forms), the plugin's argument checks, and
the observation: the in-plane marker field laid out as the n_x x n_y marker
grid."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.geometry import advance_pose, relative_velocity  # noqa: E402
from paper_2603_28475_amd.plugin import TactilePlugin, observation  # noqa: E402
from scenes.indenters import quat_from_axis_angle, quat_mul  # noqa: E402
from scenes.mesh import marker_grid  # noqa: E402


def _random_poses(rng, n):
    t = rng.uniform(-2, 2, (n, 3))
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return np.concatenate([t, q], axis=1)


def _same_rotation(qa, qb):
    return np.all(np.abs(np.abs(np.sum(qa * qb, axis=-1)) - 1.0) < 1e-12)


def test_velocity_integration_inverts_the_velocity_of_a_pose_change():
    rng = np.random.default_rng(3)
    p0, p1 = _random_poses(rng, 50), _random_poses(rng, 50)
    dt = 0.0125
    v, w = relative_velocity(p0, p1, dt)
    p = advance_pose(p0, v, w, dt)
    assert np.allclose(p[:, :3], p1[:, :3], atol=1e-12)
    assert _same_rotation(p[:, 3:], p1[:, 3:])
    # the shortest rotation: |w| dt <= pi, and q1 given as -q1 changes nothing
    assert np.all(np.linalg.norm(w, axis=1) * dt <= np.pi + 1e-12)
    v2, w2 = relative_velocity(p0, np.concatenate([p1[:, :3], -p1[:, 3:]], axis=1), dt)
    assert np.allclose(v2, v) and np.allclose(w2, w, atol=1e-12)


def test_velocities_of_closed_form_motions():
    dt = 0.02
    q0 = quat_from_axis_angle((0, 1, 0), 0.3)
    p0 = np.array([0.1, -0.2, 3.0, *q0])
    # a turn by 0.05 rad about the world z axis and a slide along x
    q1 = quat_mul(quat_from_axis_angle((0, 0, 1), 0.05), q0)
    p1 = np.array([0.15, -0.2, 2.9, *q1])
    v, w = relative_velocity(p0, p1, dt)
    assert np.allclose(v, [0.05 / dt, 0.0, -0.1 / dt], atol=1e-12)
    assert np.allclose(w, [0.0, 0.0, 0.05 / dt], atol=1e-10)
    # no motion, no velocity
    v0, w0 = relative_velocity(p0, p0, dt)
    assert np.all(v0 == 0) and np.allclose(w0, 0.0, atol=1e-15)
    with pytest.raises(ValueError):
        relative_velocity(p0, p1, 0.0)


def test_two_half_steps_equal_one_step():
    rng = np.random.default_rng(8)
    p0 = _random_poses(rng, 10)
    v, w = rng.standard_normal((10, 3)), rng.standard_normal((10, 3))
    a = advance_pose(advance_pose(p0, v, w, 0.05), v, w, 0.05)
    b = advance_pose(p0, v, w, 0.1)
    assert np.allclose(a[:, :3], b[:, :3], atol=1e-13) and _same_rotation(a[:, 3:], b[:, 3:])


def test_observation_is_the_in_plane_field_on_the_marker_grid():
    n_env, grid = 3, (7, 9)
    xy = marker_grid((8.0, 9.0), grid)                          # x fastest
    m = np.concatenate([np.concatenate([xy + 100 * e, np.full((63, 1), -1.0)], axis=1)
                        for e in range(n_env)])
    obs = observation(torch.as_tensor(m), n_env, grid)
    assert tuple(obs.shape) == (n_env, 7, 9, 2)
    for e in range(n_env):
        for i in range(7):
            for j in range(9):
                assert np.array_equal(obs[e, i, j].numpy(), m[e * 63 + j * 7 + i, :2])
    # x grows along the first grid axis, y along the second
    assert np.all(np.diff(obs[0, :, 0, 0].numpy()) > 0) and np.all(np.diff(obs[0, 0, :, 1].numpy()) > 0)
    with pytest.raises(ValueError):
        observation(torch.zeros((62, 3)), 1, grid)


class _FakeSim:
    def __init__(self, n_env, n_m):
        self.n_env, self.n_m = n_env, [n_m] * n_env


def test_plugin_checks_its_marker_grid_and_substeps():
    TactilePlugin(_FakeSim(4, 63), substeps=5)
    with pytest.raises(ValueError):
        TactilePlugin(_FakeSim(2, 49))
    with pytest.raises(ValueError):
        TactilePlugin(_FakeSim(2, 63), substeps=0)


def test_two_finger_sensor_poses_describe_one_object():
    """The two finger sensors' envs of the grasp scene see one rigid object:
    mapping each sensor's relative pose back through its frame gives the same
    gripper-frame pose at every step, and the object centre's heights above
    the two gels' bottoms add up to the finger gap 2 w."""
    from scenes.configs import gripper_sensor_frames, two_finger_grasp
    from scenes.indenters import rotation_matrix
    w = two_finger_grasp(n_steps=4)
    g = w.meshes["micro3"]
    r = float(np.linalg.norm(w.indenters["sphere_small"].Y, axis=1).max())
    w0 = g.thickness + r + 2 * 0.05 + 0.04
    w1 = g.thickness + r - 0.12
    for i in range(5):
        wi = w0 + (w1 - w0) * i / 4
        frames = gripper_sensor_frames(wi)
        back = []
        for (c, qs), env in zip(frames, w.envs):
            t = rotation_matrix(qs) @ env.poses[i, :3] + c
            Rg = rotation_matrix(qs) @ rotation_matrix(env.poses[i, 3:])
            back.append((t, Rg))
        assert np.allclose(back[0][0], back[1][0], atol=1e-12)
        assert np.allclose(back[0][1], back[1][1], atol=1e-12)
        assert w.envs[0].poses[i, 2] + w.envs[1].poses[i, 2] == pytest.approx(2 * wi, abs=1e-12)


def test_rigid_set_is_the_union_of_its_parts():
    """A fixture of several pins is one indenter: the union of the parts'
    meshes, each shifted by its offset, triangle ids renumbered into the union."""
    from scenes.indenters import icosphere, rigid_set
    a, b = icosphere(0.5, 1), icosphere(0.4, 1, yaw=0.3)
    u = rigid_set([a, b], [(-1.0, 0.0, 0.0), (1.0, 0.5, 0.2)])
    na = len(a.Y)
    assert np.allclose(u.Y[:na], a.Y + [-1.0, 0.0, 0.0]) and np.allclose(u.Y[na:], b.Y + [1.0, 0.5, 0.2])
    assert np.array_equal(u.tris[:len(a.tris)], a.tris) and np.array_equal(u.tris[len(a.tris):], b.tris + na)
