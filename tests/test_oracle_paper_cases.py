"""Pins of the oracle on the paper's own workloads and their extensions: the
heated-wall Nusselt number (the paper's Fig. 4(b) and Fig. 5(b) plot it;
read as -H dT/da at the wall over T_h - T_m), the
conduction verification at the paper's other Stefan numbers (section 3.1:
Ste = 0.1, 0.5, 1), and melting into a subcooled solid with equal or
unequal phase conductivities (Eq. (6)'s solid term)
against the two-phase Neumann solution."""
import math

import numpy as np
import pytest

from oracle import OracleSim, neumann


def _set_profile(sim, heating, T_of_a, s):
    """Equilibrium g at rest with T(a) along the melt axis, per column."""
    n = sim.n
    w7 = sim.tables()["w7"]
    g = sim.g
    for a in range(n):
        T = T_of_a(a + 0.5)  # (n, n) per column: [other][x]
        for q in range(7):
            if heating == 0:
                g[q, :, a, :] = w7[q] * T      # g[q][z][y][x], column (z, x)
            else:
                g[q, a, :, :] = w7[q] * T      # column (y, x)
    sim.s[:] = s


@pytest.mark.parametrize("heating", [0, 1])
def test_quadratic_profile_gives_the_exact_wall_gradient(heating):
    """T = T_w + A a + B a^2 near the wall, per-column wall temperature: the
    quadratic through the wall and the first two centres is exact, so
    Nu = -n A / (T_h - T_m) in every column."""
    n = 12
    sim = OracleSim(n, flow=0, alpha=0.1, ste=0.1, heating=heating, t_h=1.0, t_m=0.2)
    rng = np.random.default_rng(3)
    Tw = 1.0 + 0.1 * rng.standard_normal((n, n))
    A = -0.3 + 0.05 * rng.standard_normal((n, n))
    B = 0.02
    sim.th[:] = Tw
    _set_profile(sim, heating, lambda a: Tw + A * a + B * a * a, s=8.0)
    nu = sim.wall_nusselt()
    np.testing.assert_allclose(nu, -n * A / (1.0 - 0.2), rtol=1e-12, atol=1e-12)


def test_thin_layer_uses_the_chord_to_the_front_and_no_liquid_gives_zero():
    n = 8
    sim = OracleSim(n, flow=0, alpha=0.1, ste=0.1, t_h=1.0, t_m=0.0)
    sim.th[:] = 1.0
    _set_profile(sim, 0, lambda a: np.full((n, n), 0.5), s=1.2)
    sim.s[0, 0] = 0.0
    sim.s[1, 1] = 1.5  # the second centre is not liquid (strict phase rule)
    nu = sim.wall_nusselt()
    assert nu[0, 0] == 0.0
    assert abs(nu[1, 1] - n / 1.5) <= 1e-12
    assert abs(nu[2, 2] - n / 1.2) <= 1e-12


@pytest.mark.parametrize("heating", [0, 1])
def test_conduction_nusselt_follows_the_neumann_solution(heating):
    """Wall flux of the Neumann solution: Nu = H / (erf(lam) sqrt(pi alpha t))."""
    n, ste = 24, 0.1
    o = OracleSim(n, flow=0, alpha=0.1, ste=ste, seed_profile=1, s0=2.0, heating=heating)
    alpha = o.derived().alpha
    t0 = neumann.seed_time(2.0, alpha, ste)
    lam = neumann.stefan_lambda(ste)
    for k in range(4):
        o.step(500)
        t = t0 + 500 * (k + 1)
        exact = n / (math.erf(lam) * math.sqrt(math.pi * alpha * t))
        nu = o.wall_nusselt()
        assert np.ptp(nu) <= 1e-12 * exact
        assert abs(nu.mean() / exact - 1.0) <= 5e-3, (t, nu.mean(), exact)


@pytest.mark.parametrize("ste,lam", [(0.5, 0.464786), (1.0, 0.620063)])
def test_conduction_at_the_papers_other_stefan_numbers(ste, lam):
    """Section 3.1 verifies Ste = 0.5 and 1 as well: the Neumann constants
    (to the 6 digits quoted) and the oracle's front after 1500 steps."""
    assert abs(neumann.stefan_lambda(ste) - lam) <= 5e-7
    n = 24
    o = OracleSim(n, flow=0, alpha=0.1, ste=ste, seed_profile=1, s0=2.0)
    alpha = o.derived().alpha
    t = neumann.seed_time(2.0, alpha, ste) + 1500
    o.step(1500)
    exact = float(neumann.front(t, alpha, ste))
    assert np.ptp(o.s) <= 1e-12
    # measured: 5.7e-4 (Ste = 0.5), 1.7e-3 (Ste = 1, the front nears the cold wall)
    assert abs(o.s.mean() - exact) <= 5e-3 * exact, (o.s.mean(), exact)


# ---------------------------------------------------------------- subcooled solid
@pytest.mark.parametrize("kappa", [1.0, 0.5, 2.0])
def test_two_phase_neumann_closed_form_solves_the_stefan_problem(kappa):
    """The two-phase similarity solution (subcooled solid; the solid conducts
    kappa times as well, same rho c): without subcooling its constant is the
    one-phase one; it solves the heat equation in each phase with that
    phase's diffusivity (central differences), is continuous at T_m on the
    front, and the jump of the flux k_s dT_s - k_l dT_l equals L ds/dt
    (Stefan condition in units where rho c = 1, k_l = alpha,
    L = (T_h - T_m) / Ste_l)."""
    assert abs(neumann.two_phase_lambda(0.1, 0.0, kappa) - neumann.stefan_lambda(0.1)) <= 1e-12
    t_h, t_m, t_c, ste_l, alpha = 1.0, 0.0, -0.5, 0.5, 0.3
    ste_s = ste_l * (t_m - t_c) / (t_h - t_m)
    lam = neumann.two_phase_lambda(ste_l, ste_s, kappa)
    assert lam < neumann.stefan_lambda(ste_l)  # subcooling slows the front
    T = lambda y, t: neumann.two_phase_temperature(y, t, alpha, lam, t_h, t_m, t_c, kappa)
    t, h, k = 7.0, 1e-3, 1e-4
    s = 2 * lam * math.sqrt(alpha * t)
    for y, a in ((0.3 * s, alpha), (0.8 * s, alpha), (1.2 * s, kappa * alpha),
                 (2.5 * s, kappa * alpha)):
        Tt = (T(y, t + k) - T(y, t - k)) / (2 * k)
        Tyy = (T(y + h, t) - 2 * T(y, t) + T(y - h, t)) / h ** 2
        assert abs(Tt - a * Tyy) <= 1e-5 * max(1.0, abs(Tt)), (y, Tt, a * Tyy)
    assert abs(T(s - 1e-9, t) - t_m) <= 1e-6 and abs(T(s + 1e-9, t) - t_m) <= 1e-6
    dl = (T(s - 1e-6, t) - T(s - 1e-6 - h, t)) / h   # liquid side gradient
    ds = (T(s + 1e-6 + h, t) - T(s + 1e-6, t)) / h   # solid side gradient
    L = (t_h - t_m) / ste_l
    v = lam * math.sqrt(alpha / t)                     # ds/dt
    flux = kappa * alpha * ds - alpha * dl
    assert abs(L * v - flux) <= 1e-3 * L * v, (L * v, flux)


@pytest.mark.parametrize("kappa,n", [(1.0, 48), (0.5, 48), (2.0, 64)])
def test_subcooled_conduction_follows_the_two_phase_solution(kappa, n):
    """Oracle, energy distribution only, T_c = -0.5 < T_m = 0 < T_h = 1,
    Ste = 0.1, conductivity ratio kappa, seeded with the two-phase profile at
    s0 = 2: the front (every column) and the temperature along the melt axis
    over 2000 steps (64^3 for kappa = 2: the faster solid would feel the cold
    wall of a 48^3 box)."""
    ste, t_c = 0.1, -0.5
    o = OracleSim(n, flow=0, alpha=0.1, ste=ste, seed_profile=2, s0=2.0, t_c=t_c, ks_kl=kappa)
    lam = neumann.two_phase_lambda(ste, ste * 0.5, kappa)
    alpha = o.derived().alpha
    t0 = (2.0 / (2 * lam)) ** 2 / alpha
    y = np.arange(n) + 0.5
    for k in range(4):
        o.step(500)
        t = t0 + 500 * (k + 1)
        exact = 2 * lam * math.sqrt(alpha * t)
        assert np.ptp(o.s) <= 1e-12
        # measured: <= 7.7e-4 after 500 steps, <= 1e-4 after 2000
        assert abs(o.s.mean() / exact - 1.0) <= 2e-3, (t, o.s.mean(), exact)
        T = o.fields()["T"][n // 2, :, n // 2]
        Tex = neumann.two_phase_temperature(y, t, alpha, lam, 1.0, 0.0, t_c, kappa)
        # away from the cold wall at y = n (the closed form is semi-infinite)
        assert np.abs(T - Tex)[:30].max() <= 3e-3
