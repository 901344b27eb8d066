"""Host pins of the calibration driver: the CMA-ES (Hansen's (mu/mu_w,
lambda) strategy) reaches the known minimum of test functions in the unit
box, and the recording protocol has the paper's increments."""

import math

import numpy as np

from paper_2603_28475_amd.calibrate import CMAES, Params, protocol_poses


def _run(f, x0, gens, seed=0):
    es = CMAES(x0, sigma0=0.3, popsize=12, seed=seed)
    best = math.inf
    for _ in range(gens):
        c = es.ask()
        assert np.all((c >= 0.0) & (c <= 1.0))
        l = np.array([f(x) for x in c])
        best = min(best, l.min())
        es.tell(l)
    return best, es.m


def test_cmaes_finds_the_minimum_of_a_shifted_quadratic():
    xs = np.array([0.3, 0.7, 0.55, 0.2])
    scale = np.array([1.0, 10.0, 100.0, 3.0])
    best, m = _run(lambda x: float(np.sum(scale * (x - xs) ** 2)), np.full(4, 0.5), 150)
    assert best < 1e-12
    assert np.abs(m - xs).max() < 1e-5


def test_cmaes_follows_a_curved_valley():
    # Rosenbrock in the unit box, minimum at (0.5, 0.5) after a shift
    def f(x):
        a, b = 4 * x[0] - 1, 4 * x[1] - 1
        return (1 - a) ** 2 + 100 * (b - a * a) ** 2
    best, m = _run(f, np.array([0.1, 0.9]), 200, seed=1)
    assert best < 1e-10
    assert np.allclose(m, [0.5, 0.5], atol=1e-4)


def test_protocol_and_normalisation():
    p0 = np.array([0.0, 0.0, 2.0, 1.0, 0.0, 0.0, 0.0])
    P = protocol_poses(p0)
    assert P.shape == (10 + 10 + 4, 7)
    assert np.allclose(P[9, 2], 1.0) and np.allclose(P[19, 0], 1.0)
    w = P[-1, 3]
    assert math.isclose(2 * math.degrees(math.acos(w)), 2.0, rel_tol=1e-12)
    pr = Params()
    v = np.array([0.05, 0.45, 1.0])
    assert np.allclose(pr.from_unit(pr.to_unit(v)), v)
