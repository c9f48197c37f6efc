"""Penalty-barrier function of Ben-Tal and Zibulevsky, Section 3.1 eq. (3.8):

    phi(t) = t + t^2/2                                         t >= t_hat
    phi(t) = -(1+t_hat)^2 log((1 + 2 t_hat - t)/(1 + t_hat))
             + t_hat + t_hat^2/2                               t <  t_hat

The paper sets t_hat = -1/2 (pure logarithmic branch).  The derivatives are
differentiated by hand from the two branches.
"""
from __future__ import annotations

import numpy as np

TAU_HAT = -0.5


def phi(t, that: float = TAU_HAT):
    t = np.asarray(t, dtype=np.float64)
    quad = t + 0.5 * t * t
    a = (1.0 + that) ** 2
    arg = np.where(t < that, (1.0 + 2.0 * that - t) / (1.0 + that), 1.0)
    logb = -a * np.log(arg) + that + 0.5 * that * that
    return np.where(t >= that, quad, logb)


def dphi(t, that: float = TAU_HAT):
    t = np.asarray(t, dtype=np.float64)
    a = (1.0 + that) ** 2
    den = np.where(t < that, 1.0 + 2.0 * that - t, 1.0)
    return np.where(t >= that, 1.0 + t, a / den)


def d2phi(t, that: float = TAU_HAT):
    t = np.asarray(t, dtype=np.float64)
    a = (1.0 + that) ** 2
    den = np.where(t < that, 1.0 + 2.0 * that - t, 1.0)
    return np.where(t >= that, np.ones_like(t), a / (den * den))


def phi_diff(t, dt, that: float = TAU_HAT):
    """phi(t + dt) - phi(t) formed without subtracting two values of phi
    where both points lie on one branch: dt (1 + t + dt/2) on the quadratic
    branch, -(1+t_hat)^2 log1p(-dt / (1 + 2 t_hat - t)) on the logarithmic
    one (both exact rearrangements of eq. (3.8)); points on different
    branches take the plain difference."""
    t = np.asarray(t, dtype=np.float64)
    dt = np.asarray(dt, dtype=np.float64)
    t1 = t + dt
    a = (1.0 + that) ** 2
    quad = dt * (1.0 + t + 0.5 * dt)
    both_log = (t < that) & (t1 < that)
    den = np.where(both_log, 1.0 + 2.0 * that - t, 1.0)
    logd = -a * np.log1p(np.where(both_log, -dt / den, 0.0))
    plain = phi(t1, that) - phi(t, that)
    return np.where((t >= that) & (t1 >= that), quad, np.where(both_log, logd, plain))
