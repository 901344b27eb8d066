"""Oracle log-barrier b(d) and friction mollifier f(s). Test infrastructure only.

Barrier (Supp. A, eq. ipc_energy and the sentence after it): a C^2 log barrier
that activates below dhat. Reading: the IPC barrier on the unsquared distance,
    b(d) = -(d - dhat)^2 ln(d / dhat)   for 0 < d < dhat,
    b(d) = 0 for d >= dhat,  b(d) = +inf for d <= 0.

Mollifier (Supp. A, eq. friction_mollifier):
    f(s) = -s^3 / (3 eps^2) + s^2 / eps + eps / 3   for s < eps,   f(s) = s otherwise.
"""

from __future__ import annotations

import numpy as np


def barrier(d, dhat):
    d = np.asarray(d, dtype=np.float64)
    out = np.zeros_like(d)
    out[d <= 0] = np.inf
    m = (d > 0) & (d < dhat)
    dm = d[m]
    out[m] = -(dm - dhat) ** 2 * np.log(dm / dhat)
    return out


def barrier_d1(d, dhat):
    d = np.asarray(d, dtype=np.float64)
    out = np.zeros_like(d)
    m = (d > 0) & (d < dhat)
    dm = d[m]
    out[m] = -2.0 * (dm - dhat) * np.log(dm / dhat) - (dm - dhat) ** 2 / dm
    return out


def barrier_d2(d, dhat):
    d = np.asarray(d, dtype=np.float64)
    out = np.zeros_like(d)
    m = (d > 0) & (d < dhat)
    dm = d[m]
    out[m] = -2.0 * np.log(dm / dhat) - 4.0 * (dm - dhat) / dm + (dm - dhat) ** 2 / dm ** 2
    return out


def mollifier(s, eps):
    s = np.asarray(s, dtype=np.float64)
    return np.where(s < eps, -s ** 3 / (3 * eps ** 2) + s ** 2 / eps + eps / 3.0, s)


def mollifier_d1(s, eps):
    s = np.asarray(s, dtype=np.float64)
    return np.where(s < eps, -s ** 2 / eps ** 2 + 2.0 * s / eps, 1.0)


def mollifier_d2(s, eps):
    s = np.asarray(s, dtype=np.float64)
    return np.where(s < eps, -2.0 * s / eps ** 2 + 2.0 / eps, 0.0)
