"""Pins for the oracle's barrier, mollifier and primitive distances (Supp. A,
eqs. ipc_energy, friction_energy, friction_mollifier): closed-form properties,
brute-force minimisation over barycentric grids and finite differences."""

import numpy as np
import pytest
from scipy.optimize import minimize

from oracle.barrier import (barrier, barrier_d1, barrier_d2, mollifier, mollifier_d1,
                            mollifier_d2)
from oracle.distance import distance_derivatives, edge_edge, point_triangle

DHAT = 0.05


def test_barrier_vanishes_with_two_derivatives_at_dhat():
    d = np.array([DHAT, DHAT * 1.5, 1.0])
    assert np.all(barrier(d, DHAT) == 0)
    assert np.all(barrier_d1(d, DHAT) == 0)
    assert np.all(barrier_d2(d, DHAT) == 0)
    # one-sided limits also vanish (C^2 at dhat)
    e = DHAT * (1 - 1e-7)
    assert abs(barrier(np.array([e]), DHAT)[0]) < 1e-22
    assert abs(barrier_d1(np.array([e]), DHAT)[0]) < 1e-14
    assert abs(barrier_d2(np.array([e]), DHAT)[0]) < 1e-5


def test_barrier_sign_and_blow_up():
    d = np.linspace(1e-6, DHAT * (1 - 1e-9), 200)
    assert np.all(barrier(d, DHAT) > 0)
    assert np.all(barrier_d1(d, DHAT) < 0)
    assert np.all(barrier_d2(d, DHAT) > 0)
    assert barrier(np.array([1e-12]), DHAT)[0] > 1e-2
    assert np.isinf(barrier(np.array([0.0]), DHAT)[0])


def test_barrier_derivatives_by_central_differences():
    d = np.linspace(0.002, 0.049, 40)
    h = 1e-8
    fd1 = (barrier(d + h, DHAT) - barrier(d - h, DHAT)) / (2 * h)
    fd2 = (barrier_d1(d + h, DHAT) - barrier_d1(d - h, DHAT)) / (2 * h)
    assert np.allclose(fd1, barrier_d1(d, DHAT), rtol=1e-6, atol=1e-12)
    assert np.allclose(fd2, barrier_d2(d, DHAT), rtol=1e-6, atol=1e-9)


def test_mollifier_is_c1_at_eps_and_matches_differences():
    eps = 1e-3
    assert mollifier(np.array([eps]), eps)[0] == pytest.approx(eps)
    lo = eps * (1 - 1e-9)
    assert mollifier(np.array([lo]), eps)[0] == pytest.approx(eps, rel=1e-8)
    assert mollifier_d1(np.array([lo]), eps)[0] == pytest.approx(1.0, rel=1e-8)
    assert mollifier(np.array([0.0]), eps)[0] == pytest.approx(eps / 3)
    assert mollifier_d1(np.array([0.0]), eps)[0] == 0.0
    s = np.linspace(1e-5, 0.99 * eps, 30)
    h = 1e-10
    assert np.allclose((mollifier(s + h, eps) - mollifier(s - h, eps)) / (2 * h),
                       mollifier_d1(s, eps), rtol=1e-5)
    assert np.allclose((mollifier_d1(s + h, eps) - mollifier_d1(s - h, eps)) / (2 * h),
                       mollifier_d2(s, eps), rtol=1e-4)


def _brute_pt(p, a, b, c):
    best = np.inf
    n = 200
    for i in range(n + 1):
        s = i / n
        t = np.linspace(0, 1 - s, n + 1 - i)
        q = a + s * (b - a) + t[:, None] * (c - a)
        best = min(best, np.linalg.norm(q - p, axis=1).min())

    def f(w):
        s, t = w
        return np.sum((a + s * (b - a) + t * (c - a) - p) ** 2)
    res = minimize(f, [1 / 3, 1 / 3], method="SLSQP", bounds=[(0, 1), (0, 1)],
                   constraints=[{"type": "ineq", "fun": lambda w: 1 - w[0] - w[1]}],
                   options=dict(ftol=1e-20, maxiter=500))
    return min(best, np.sqrt(res.fun))


def _brute_ee(a0, a1, b0, b1):
    def f(w):
        s, t = w
        return np.sum((a0 + s * (a1 - a0) - b0 - t * (b1 - b0)) ** 2)
    best = np.inf
    for s0 in (0.1, 0.5, 0.9):
        for t0 in (0.1, 0.5, 0.9):
            res = minimize(f, [s0, t0], method="L-BFGS-B", bounds=[(0, 1), (0, 1)],
                           options=dict(ftol=1e-22, gtol=1e-14, maxiter=1000))
            best = min(best, np.sqrt(res.fun))
    return best


def test_point_triangle_matches_brute_force():
    rng = np.random.default_rng(11)
    for _ in range(60):
        a, b, c = rng.standard_normal((3, 3))
        p = rng.standard_normal(3) * 1.5
        d = point_triangle(p, a, b, c)["d"][0]
        assert d == pytest.approx(_brute_pt(p, a, b, c), abs=1e-7)
        assert d <= _brute_pt(p, a, b, c) + 1e-12


def test_edge_edge_matches_brute_force():
    rng = np.random.default_rng(12)
    for _ in range(60):
        a0, a1, b0, b1 = rng.standard_normal((4, 3))
        d = edge_edge(a0, a1, b0, b1)["d"][0]
        assert d == pytest.approx(_brute_ee(a0, a1, b0, b1), abs=1e-8)


def test_special_cases():
    # point above the interior of a triangle: the plane distance
    a, b, c = np.array([0, 0, 0.]), np.array([1, 0, 0.]), np.array([0, 1, 0.])
    r = point_triangle(np.array([0.2, 0.3, 0.7]), a, b, c)
    assert r["d"][0] == pytest.approx(0.7, abs=1e-15) and r["k"][0] == 2
    # point beyond a vertex: the vertex distance
    r = point_triangle(np.array([-1.0, -1.0, 1.0]), a, b, c)
    assert r["d"][0] == pytest.approx(np.sqrt(3.0)) and r["k"][0] == 0
    # crossing perpendicular segments separated by 0.3 in z
    r = edge_edge(np.array([-1, 0, 0.]), np.array([1, 0, 0.]),
                  np.array([0, -1, 0.3]), np.array([0, 1, 0.3]))
    assert r["d"][0] == pytest.approx(0.3, abs=1e-15) and r["k"][0] == 2
    # parallel overlapping segments at distance 0.25
    r = edge_edge(np.array([0, 0, 0.]), np.array([1, 0, 0.]),
                  np.array([0.5, 0.25, 0.]), np.array([1.5, 0.25, 0.]))
    assert r["d"][0] == pytest.approx(0.25, abs=1e-15)
    # parallel disjoint segments: endpoint distance
    r = edge_edge(np.array([0, 0, 0.]), np.array([1, 0, 0.]),
                  np.array([2, 1, 0.]), np.array([3, 1, 0.]))
    assert r["d"][0] == pytest.approx(np.sqrt(2.0), abs=1e-15)


def _fd_check(kind, seed, n=40):
    rng = np.random.default_rng(seed)
    fn = point_triangle if kind == "pt" else edge_edge
    checked = 0
    for _ in range(n):
        Z = rng.standard_normal((4, 3))
        r = fn(Z[0], Z[1], Z[2], Z[3])
        d, grad, H = distance_derivatives(Z[None], r["c"], r["Cw"], r["k"])
        h = 1e-6
        ok = True
        for j in range(12):
            Zp, Zm = Z.copy(), Z.copy()
            Zp.flat[j] += h
            Zm.flat[j] -= h
            rp, rm = fn(*Zp), fn(*Zm)
            if rp["k"][0] != r["k"][0] or rm["k"][0] != r["k"][0]:
                ok = False  # feature change inside the stencil: derivatives jump there
                break
            fd = (rp["d"][0] - rm["d"][0]) / (2 * h)
            assert fd == pytest.approx(grad[0].flat[j], rel=1e-6, abs=1e-8)
            _, gp, _ = distance_derivatives(Zp[None], rp["c"], rp["Cw"], rp["k"])
            _, gm, _ = distance_derivatives(Zm[None], rm["c"], rm["Cw"], rm["k"])
            fdH = (gp[0] - gm[0]).ravel() / (2 * h)
            assert np.allclose(fdH, H[0][:, j], rtol=1e-4, atol=1e-6)
        checked += ok
    assert checked > n // 3


@pytest.mark.parametrize("kind,seed", [("pt", 21), ("ee", 22)])
def test_distance_derivatives_by_finite_differences(kind, seed):
    _fd_check(kind, seed)


def test_point_plane_hessian_vanishes_in_the_point():
    # the distance from a point to a fixed plane is affine in the point
    a, b, c = np.array([0, 0, 0.]), np.array([1, 0, 0.]), np.array([0, 1, 0.])
    Z = np.array([[0.2, 0.3, 0.7], a, b, c])
    r = point_triangle(*Z)
    _, g, H = distance_derivatives(Z[None], r["c"], r["Cw"], r["k"])
    assert np.abs(H[0][:3, :3]).max() < 1e-14
    assert np.allclose(g[0, 0], [0, 0, 1])


def test_point_point_hessian_closed_form():
    # d = |p - q| has Hessian (I - n n^T)/d in p
    a, b, c = np.array([0, 0, 0.]), np.array([1, 0, 0.]), np.array([0, 1, 0.])
    p = np.array([-0.6, -0.8, 0.0])
    Z = np.array([p, a, b, c])
    r = point_triangle(*Z)
    assert r["k"][0] == 0
    d, g, H = distance_derivatives(Z[None], r["c"], r["Cw"], r["k"])
    n = p / np.linalg.norm(p)
    assert np.allclose(H[0][:3, :3], (np.eye(3) - np.outer(n, n)) / d[0], atol=1e-14)
