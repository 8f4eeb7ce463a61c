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


# ---------------------------------------------------------------- two phases
# Melting of a semi-infinite solid initially subcooled to T_c < T_m.  The
# solid conducts kappa times as well as the liquid with the same rho c
# (diffusivities alpha and alpha_s = kappa alpha; kappa = 1: equal
# properties).  Front s = 2 lam sqrt(alpha t); liquid
# T = T_h - (T_h - T_m) erf(eta) / erf(lam) with eta = y / (2 sqrt(alpha t));
# solid T = T_c + (T_m - T_c) erfc(eta_s) / erfc(nu lam) with
# eta_s = y / (2 sqrt(alpha_s t)), nu = sqrt(alpha / alpha_s).  The Stefan
# condition rho L ds/dt = k_s dT_s/dy - k_l dT_l/dy at y = s gives
#   lam sqrt(pi) = Ste_l exp(-lam^2) / erf(lam)
#                  - sqrt(kappa) Ste_s exp(-nu^2 lam^2) / erfc(nu lam)
# with Ste_l = c (T_h - T_m) / L and Ste_s = c (T_m - T_c) / L.

def two_phase_lambda(ste_l: float, ste_s: float, kappa: float = 1.0,
                     tol: float = 1e-15) -> float:
    """Root of the two-phase Stefan condition above."""
    if ste_l <= 0 or ste_s < 0 or kappa <= 0:
        raise ValueError("need Ste_l > 0, Ste_s >= 0 and kappa > 0")
    nu = 1.0 / math.sqrt(kappa)

    def h(lam):
        return (lam * math.sqrt(math.pi) - ste_l * math.exp(-lam * lam) / math.erf(lam)
                + math.sqrt(kappa) * ste_s * math.exp(-nu * nu * lam * lam) / math.erfc(nu * lam))

    lo, hi = 1e-12, 1.0
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


def two_phase_temperature(y, t, alpha, lam, t_h, t_m, t_c, kappa: float = 1.0):
    y = np.asarray(y, dtype=np.float64)
    alpha_s = kappa * alpha
    erf = np.vectorize(math.erf)
    erfc = np.vectorize(math.erfc)
    s = 2.0 * lam * math.sqrt(alpha * t)
    liquid = t_h - (t_h - t_m) * erf(y / (2.0 * math.sqrt(alpha * t))) / math.erf(lam)
    solid = t_c + (t_m - t_c) * erfc(y / (2.0 * math.sqrt(alpha_s * t))) / \
        math.erfc(lam * math.sqrt(alpha / alpha_s))
    return np.where(y < s, liquid, solid)
