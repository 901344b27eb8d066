"""Pins for the oracle's neo-Hookean term (reading of the hyperelastic potential
in Supp. A, eq. varopt): closed forms, finite differences, invariances and the
small-strain limit of textbook linear elasticity."""

import numpy as np
import pytest

from oracle.elastic import (d2psi_matrix, element_energy, element_gradient, element_hessian,
                            first_piola, lame, psi)

E, NU = 0.3, 0.45
MU, LAM = lame(E, NU)


def _random_tets(n, seed, scale=0.3):
    rng = np.random.default_rng(seed)
    X = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float)
    Xs, xs = [], []
    for _ in range(n):
        A = np.eye(3) + 0.2 * rng.standard_normal((3, 3))
        if np.linalg.det(A) < 0.3:
            A = np.eye(3)
        Xr = X @ A.T + rng.standard_normal(3)
        F = np.eye(3) + scale * rng.standard_normal((3, 3))
        if np.linalg.det(F) < 0.2:
            F = np.eye(3) + 0.05 * rng.standard_normal((3, 3))
        Xs.append(Xr)
        xs.append(Xr @ F.T + rng.standard_normal(3))
    Xall = np.concatenate(Xs)
    xall = np.concatenate(xs)
    tets = np.arange(4 * n).reshape(n, 4)
    Xt = Xall[tets]
    Dm = np.stack([Xt[:, 1] - Xt[:, 0], Xt[:, 2] - Xt[:, 0], Xt[:, 3] - Xt[:, 0]], axis=2)
    return xall, tets, np.linalg.inv(Dm), np.linalg.det(Dm) / 6.0


def test_lame_recovers_young_and_poisson():
    # textbook isotropic identities: E = mu(3 lam + 2 mu)/(lam + mu), nu = lam / (2 (lam + mu))
    for e, nu in [(0.3, 0.45), (0.2, 0.4), (1e4, 0.497)]:
        mu, lam = lame(e, nu)
        assert mu * (3 * lam + 2 * mu) / (lam + mu) == pytest.approx(e, rel=1e-12)
        assert lam / (2 * (lam + mu)) == pytest.approx(nu, rel=1e-12)


def test_rest_state_is_stress_free():
    F = np.eye(3)[None]
    assert psi(F, MU, LAM)[0] == 0.0
    assert np.abs(first_piola(F, MU, LAM)).max() < 1e-15


def test_rotation_invariance():
    rng = np.random.default_rng(1)
    F = np.eye(3)[None] + 0.3 * rng.standard_normal((50, 3, 3))
    F = F[np.linalg.det(F) > 0.2]
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    assert np.allclose(psi(Q[None] @ F, MU, LAM), psi(F, MU, LAM), rtol=1e-12, atol=1e-14)


def test_inverted_element_has_infinite_energy():
    F = np.diag([1.0, 1.0, -0.5])[None]
    assert np.isinf(psi(F, MU, LAM)[0])


def test_small_strain_limit_is_linear_elasticity():
    # d^2 psi at F = I equals 2 mu |sym dF|^2 + lam (tr dF)^2 (isotropic linear elasticity)
    rng = np.random.default_rng(2)
    M = d2psi_matrix(np.eye(3)[None], MU, LAM)[0]
    for _ in range(10):
        dF = rng.standard_normal((3, 3))
        sym = 0.5 * (dF + dF.T)
        lin = 2 * MU * np.sum(sym * sym) + LAM * np.trace(dF) ** 2
        assert dF.ravel() @ M @ dF.ravel() == pytest.approx(lin, rel=1e-12)


def test_gradient_matches_central_differences():
    x, tets, Dmi, vol = _random_tets(20, 3)
    g = element_gradient(x, tets, Dmi, vol, MU, LAM)
    h = 1e-6
    for e in range(20):
        for i in range(4):
            for a in range(3):
                xp, xm = x.copy(), x.copy()
                xp[tets[e, i], a] += h
                xm[tets[e, i], a] -= h
                fd = (element_energy(xp, tets, Dmi, vol, MU, LAM)[e]
                      - element_energy(xm, tets, Dmi, vol, MU, LAM)[e]) / (2 * h)
                assert fd == pytest.approx(g[e, i, a], rel=1e-6, abs=1e-9)


def test_hessian_matches_differences_of_gradient():
    x, tets, Dmi, vol = _random_tets(10, 4)
    H = element_hessian(x, tets, Dmi, vol, MU, LAM)
    h = 1e-6
    for e in range(10):
        for i in range(4):
            for a in range(3):
                xp, xm = x.copy(), x.copy()
                xp[tets[e, i], a] += h
                xm[tets[e, i], a] -= h
                fd = (element_gradient(xp, tets, Dmi, vol, MU, LAM)[e]
                      - element_gradient(xm, tets, Dmi, vol, MU, LAM)[e]).ravel() / (2 * h)
                col = H[e][:, 3 * i + a]
                assert np.allclose(fd, col, rtol=1e-5, atol=1e-8)


def test_diagonal_matches_independent_closed_form():
    # diag entry (vertex i, axis a) = V [mu |g_i|^2 + (mu + lam (1 - ln J)) ((F^-T g_i)_a)^2]
    x, tets, Dmi, vol = _random_tets(30, 5)
    H = element_hessian(x, tets, Dmi, vol, MU, LAM)
    xt = x[tets]
    Ds = np.stack([xt[:, 1] - xt[:, 0], xt[:, 2] - xt[:, 0], xt[:, 3] - xt[:, 0]], axis=2)
    F = Ds @ Dmi
    J = np.linalg.det(F)
    FinvT = np.transpose(np.linalg.inv(F), (0, 2, 1))
    G = np.concatenate([-Dmi.sum(axis=1, keepdims=True), Dmi], axis=1)  # rows g_0..g_3
    for e in range(30):
        for i in range(4):
            gi = G[e, i]
            v = FinvT[e] @ gi
            for a in range(3):
                cf = vol[e] * (MU * gi @ gi + (MU + LAM * (1 - np.log(J[e]))) * v[a] ** 2)
                assert H[e, 3 * i + a, 3 * i + a] == pytest.approx(cf, rel=1e-11)


def test_rigid_translation_and_rotation_give_zero_force_and_torque():
    x, tets, Dmi, vol = _random_tets(15, 6)
    g = element_gradient(x, tets, Dmi, vol, MU, LAM)
    assert np.abs(g.sum(axis=1)).max() < 1e-12
    torque = np.cross(x[tets], g).sum(axis=1)
    assert np.abs(torque).max() < 1e-11


def test_curvature_is_second_directional_derivative():
    x, tets, Dmi, vol = _random_tets(10, 7)
    H = element_hessian(x, tets, Dmi, vol, MU, LAM)
    rng = np.random.default_rng(8)
    p = rng.standard_normal(x.shape)
    h = 1e-4
    e0 = element_energy(x, tets, Dmi, vol, MU, LAM).sum()
    ep = element_energy(x + h * p, tets, Dmi, vol, MU, LAM).sum()
    em = element_energy(x - h * p, tets, Dmi, vol, MU, LAM).sum()
    fd = (ep - 2 * e0 + em) / h ** 2
    curv = sum(p[tets[e]].ravel() @ H[e] @ p[tets[e]].ravel() for e in range(10))
    assert fd == pytest.approx(curv, rel=1e-5)
