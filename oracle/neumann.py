"""Closed-form Neumann solution of one-dimensional melting without subcooling.

Test infrastructure only.  The paper verifies the method against this
analytical solution (section 3.1, conduction melting problem; its Ref. [2]).
A semi-infinite solid at the melting temperature T_m is heated at y = 0 to
T_h.  The front sits at s(t) = 2*lam*sqrt(alpha*t), where lam solves

    lam * exp(lam**2) * erf(lam) = Ste / sqrt(pi),

and the liquid temperature is T(y, t) = T_h - (T_h - T_m) erf(eta) / erf(lam)
with eta = y / (2 sqrt(alpha t)).  The solid stays at T_m.
"""
from __future__ import annotations

import math

import numpy as np


def stefan_lambda(ste: float, tol: float = 1e-15) -> float:
    """Root of lam*exp(lam^2)*erf(lam) = Ste/sqrt(pi) by bisection."""
    if ste <= 0:
        raise ValueError("Stefan number must be positive")
    target = ste / math.sqrt(math.pi)

    def h(lam):
        return lam * math.exp(lam * lam) * math.erf(lam) - target

    lo, hi = 0.0, 1.0
    while h(hi) < 0:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if h(mid) < 0:
            lo = mid
        else:
            hi = mid
        if hi - lo < tol:
            break
    return 0.5 * (lo + hi)


def front(t, alpha: float, ste: float):
    lam = stefan_lambda(ste)
    return 2.0 * lam * np.sqrt(alpha * np.asarray(t, dtype=np.float64))


def temperature(y, t, alpha: float, ste: float, t_h: float = 1.0, t_m: float = 0.0):
    """Exact temperature at positions y and time t (liquid below the front,
    T_m above it)."""
    lam = stefan_lambda(ste)
    y = np.asarray(y, dtype=np.float64)
    eta = y / (2.0 * math.sqrt(alpha * t))
    erf = np.vectorize(math.erf)
    T = t_h - (t_h - t_m) * erf(eta) / math.erf(lam)
    s = 2.0 * lam * math.sqrt(alpha * t)
    return np.where(y < s, T, t_m)


def seed_time(s0: float, alpha: float, ste: float) -> float:
    """Time at which the exact front has reached s0."""
    lam = stefan_lambda(ste)
    return (s0 / (2.0 * lam)) ** 2 / alpha
