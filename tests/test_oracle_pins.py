"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: the
velocity tables the paper prints (section 2, Eq. (3) and Eq. (5)), exact
matrix identities, textbook reductions (BGK, Guo forcing moments, shear-wave
and diffusion decay rates), the closed-form Neumann solution the paper uses
for verification (section 3.1), a manufactured front for Eq. (6), symmetry
and conservation invariants.
"""
import math

import numpy as np
import pytest

from conftest import golden_path
from oracle import OracleSim, neumann


def _load_velocities(name):
    rows = [list(map(int, ln.split())) for ln in open(golden_path(name))
            if ln.strip() and not ln.startswith("#")]
    return np.array(rows, dtype=np.int32).T  # (Q, 3)


@pytest.fixture(scope="module")
def tables(oracle_lib):
    return OracleSim(4, flow=1).tables()


# ---------------------------------------------------------------- lattices
def test_velocity_sets_match_paper(tables):
    np.testing.assert_array_equal(tables["e19"], _load_velocities("eq3_d3q19_velocities.txt"))
    np.testing.assert_array_equal(tables["e7"], _load_velocities("eq5_d3q7_velocities.txt"))


def test_opposites_and_weight_isotropy(tables):
    e19, e7 = tables["e19"].astype(float), tables["e7"].astype(float)
    np.testing.assert_array_equal(e19[tables["opp19"]], -e19)
    np.testing.assert_array_equal(e7[tables["opp7"]], -e7)
    w, w7 = tables["w19"], tables["w7"]
    assert abs(w.sum() - 1.0) < 1e-15 and abs(w7.sum() - 1.0) < 1e-15
    # second moment: c_s^2 = 1/3 (D3Q19), 1/4 (D3Q7)
    np.testing.assert_allclose(np.einsum("q,qa,qb->ab", w, e19, e19), np.eye(3) / 3, atol=1e-15)
    np.testing.assert_allclose(np.einsum("q,qa,qb->ab", w7, e7, e7), np.eye(3) / 4, atol=1e-15)
    # fourth-moment isotropy of D3Q19: sum w e_a e_b e_c e_d = (dd+dd+dd)/9
    d = np.eye(3)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
           + np.einsum("ad,bc->abcd", d, d)) / 9.0
    np.testing.assert_allclose(np.einsum("q,qa,qb,qc,qd->abcd", w, e19, e19, e19, e19), iso,
                               atol=1e-15)


# ---------------------------------------------------------------- moment bases
def test_m_is_orthogonal_and_inverted(tables):
    M, Minv = tables["M"], tables["Minv"]
    G = M @ M.T
    np.testing.assert_array_equal(G - np.diag(np.diag(G)), np.zeros((19, 19)))
    np.testing.assert_array_equal(
        np.diag(G), [19, 2394, 252, 10, 40, 10, 40, 10, 40, 36, 72, 12, 24, 4, 4, 4, 8, 8, 8])
    np.testing.assert_allclose(Minv @ M, np.eye(19), atol=1e-14)
    np.testing.assert_allclose(Minv, M.T / np.diag(G), atol=1e-15)
    # every entry is an integer (exact transform in any precision)
    np.testing.assert_array_equal(M, np.round(M))


def test_n_is_orthogonal_and_inverted(tables):
    N, Ninv = tables["N"], tables["Ninv"]
    G = N @ N.T
    np.testing.assert_array_equal(G - np.diag(np.diag(G)), np.zeros((7, 7)))
    np.testing.assert_array_equal(np.diag(G), [7, 2, 2, 2, 42, 12, 4])
    np.testing.assert_allclose(Ninv @ N, np.eye(7), atol=1e-15)


def _feq_incompressible(w, e, rho, u):
    eu = e @ u
    return w * (rho + 3 * eu + 4.5 * eu ** 2 - 1.5 * (u @ u))


def test_equilibrium_moments_are_moments_of_bgk_equilibrium(tables):
    rng = np.random.default_rng(1)
    M, N = tables["M"], tables["N"]
    e19, e7 = tables["e19"].astype(float), tables["e7"].astype(float)
    for _ in range(20):
        rho = 1 + 0.01 * rng.standard_normal()
        u = 0.05 * rng.standard_normal(3)
        T = rng.uniform(-1, 2)
        m_eq, n_eq = OracleSim.equilibrium_moments(rho, u, T, u)
        np.testing.assert_allclose(M @ _feq_incompressible(tables["w19"], e19, rho, u), m_eq,
                                   atol=2e-15)
        geq = tables["w7"] * T * (1 + 4 * (e7 @ u))
        np.testing.assert_allclose(N @ geq, n_eq, atol=2e-15)


def test_guo_force_moments(tables):
    """Guo forcing: zeroth moment 0, first F, second u F + F u; projected by M
    it has the closed form derived for the orthogonal basis."""
    sim = OracleSim(4, flow=1)
    e19 = tables["e19"].astype(float)
    rng = np.random.default_rng(2)
    for _ in range(10):
        u = 0.05 * rng.standard_normal(3)
        F = 1e-4 * rng.standard_normal(3)
        Fq = sim.guo_force(u, F)
        assert abs(Fq.sum()) < 1e-18
        np.testing.assert_allclose(e19.T @ Fq, F, atol=1e-18)
        np.testing.assert_allclose(np.einsum("q,qa,qb->ab", Fq, e19, e19),
                                   np.outer(u, F) + np.outer(F, u), atol=1e-18)
        uF = u @ F
        closed = np.array([
            0, 38 * uF, -11 * uF, F[0], -2 / 3 * F[0], F[1], -2 / 3 * F[1], F[2], -2 / 3 * F[2],
            2 * (3 * u[0] * F[0] - uF), -(3 * u[0] * F[0] - uF),
            2 * (u[1] * F[1] - u[2] * F[2]), -(u[1] * F[1] - u[2] * F[2]),
            u[0] * F[1] + u[1] * F[0], u[1] * F[2] + u[2] * F[1], u[0] * F[2] + u[2] * F[0],
            0, 0, 0])
        np.testing.assert_allclose(tables["M"] @ Fq, closed, atol=1e-18)


def test_equal_rates_reduce_to_bgk_with_guo_forcing(tables):
    """All relaxation rates equal to 1/tau: the MRT collision of Eq. (2) with
    the force term must equal the textbook BGK collision with Guo forcing."""
    sim = OracleSim(8, ra=1e4, pr=1.0, flow=1)
    d = sim.derived()
    tau = 0.77
    sim.set_rates(S=np.full(19, 1 / tau))
    e19 = tables["e19"].astype(float)
    w = tables["w19"]
    rng = np.random.default_rng(3)
    for _ in range(10):
        fin = w * (1 + 0.02 * rng.standard_normal(19))
        T = rng.uniform(0, 1)
        out = sim.collide_f_cell(fin, T)
        rho = fin.sum()
        F = np.array([0.0, 0.0, d.gbeta * (T - d.t0)])
        u = e19.T @ fin + 0.5 * F
        feq = _feq_incompressible(w, e19, rho, u)
        eu = e19 @ u
        Fq = w * (3 * ((e19 - u) @ F) + 9 * eu * (e19 @ F))
        bgk = fin - (fin - feq) / tau + (1 - 0.5 / tau) * Fq
        np.testing.assert_allclose(out, bgk, atol=1e-15)


def _uniform_collision_errors(tables, library=None):
    """Largest deviations of f and g from the collision of Eq. (2) and
    Eq. (4) with random distinct rates, after one oracle step of a lattice
    whose populations are the same in every cell: an interior cell pulls
    the same populations it holds, so it is left with the collision alone.
    Its moments must be m - S (m - m_eq) + (I - S/2) M F for f, with the
    equilibrium and the forcing of the textbook BGK and Guo forms projected
    by M, and n - Q (n - n_eq) for g with the D3Q7 equilibrium
    w_q T (1 + 4 e_q . u), u = j + F/2."""
    n = 6
    sim = OracleSim(n, ra=1e4, pr=1.0, ste=0.1, s0=float(n), flow=1, library=library)
    d = sim.derived()
    rng = np.random.default_rng(11)
    S = rng.uniform(0.6, 1.9, 19)
    Qr = rng.uniform(0.6, 1.9, 7)
    sim.set_rates(S=S, Q=Qr)
    M, N = tables["M"], tables["N"]
    w, w7 = tables["w19"], tables["w7"]
    e19, e7 = tables["e19"].astype(float), tables["e7"].astype(float)
    fin = w * (1 + 0.02 * rng.standard_normal(19))
    gin = w7 * 0.7 * (1 + 0.3 * rng.uniform(-1, 1, 7))
    sim.f[:] = fin[:, None, None, None]
    sim.g[:] = gin[:, None, None, None]
    sim.step(1)

    rho, T = fin.sum(), gin.sum()
    F = np.array([0.0, 0.0, d.gbeta * (T - d.t0)])
    u = e19.T @ fin + 0.5 * F
    feq = _feq_incompressible(w, e19, rho, u)
    eu = e19 @ u
    Fq = w * (3 * ((e19 - u) @ F) + 9 * eu * (e19 @ F))
    m = M @ fin
    f_exp = np.linalg.solve(M, m - S * (m - M @ feq) + (1 - 0.5 * S) * (M @ Fq))
    nn = N @ gin
    n_eq = N @ (w7 * T * (1 + 4 * (e7 @ u)))
    g_exp = np.linalg.solve(N, nn - Qr * (nn - n_eq))
    # the rates matter: the collision moves both distributions well above round-off
    assert np.abs(f_exp - fin).max() > 1e-5 and np.abs(g_exp - gin).max() > 1e-3

    inner = (slice(None), slice(1, n - 1), slice(1, n - 1), slice(1, n - 1))
    ef = float(np.abs(sim.f[inner] - f_exp[:, None, None, None]).max())
    eg = float(np.abs(sim.g[inner] - g_exp[:, None, None, None]).max())
    return ef, eg


def test_distinct_rates_relax_each_moment_by_its_own_rate(tables):
    """Eq. (2) and Eq. (4) with every rate different (the collision alone,
    above): round-off at every interior cell, within 20 ulps of the largest
    population (about 1/3) after the dense 19 x 19 transforms."""
    ef, eg = _uniform_collision_errors(tables)
    assert ef <= 1e-15 and eg <= 1e-15, (ef, eg)


# Planted mistakes for the pin above: (name, text in the oracle source,
# replacement).  Each text occurs exactly once in the step's collision.
COLLISION_MISTAKES = [
    ("rate of the next moment applied to each moment of f",
     "      ms[k] = m[k] - S->S[k] * (m[k] - me[k]) + (1.0 - 0.5 * S->S[k]) * Fm[k];\n",
     "      ms[k] = m[k] - S->S[(k + 1) % Q19] * (m[k] - me[k]) + (1.0 - 0.5 * S->S[k]) * Fm[k];\n"),
    ("forcing without the (I - S/2) factor",
     "      ms[k] = m[k] - S->S[k] * (m[k] - me[k]) + (1.0 - 0.5 * S->S[k]) * Fm[k];\n",
     "      ms[k] = m[k] - S->S[k] * (m[k] - me[k]) + Fm[k];\n"),
    ("velocity without the half force",
     "    uz = (jz + 0.5 * Fz) / rho0;\n",
     "    uz = jz / rho0;\n"),
    ("rates of g shifted by one moment",
     "  for (int k = 0; k < Q7; ++k) ns[k] = nm[k] - QR[k] * (nm[k] - ne[k]);\n",
     "  for (int k = 0; k < Q7; ++k) ns[k] = nm[k] - QR[(k + 1) % Q7] * (nm[k] - ne[k]);\n"),
]


def test_distinct_rates_pin_catches_planted_mistakes(tables, tmp_path):
    import os
    from oracle.oracle import _SRC, compile_oracle
    src = open(_SRC).read()
    for k, (name, old, new) in enumerate(COLLISION_MISTAKES):
        assert src.count(old) == 1, name
        path = os.path.join(tmp_path, f"mut{k}.c")
        with open(path, "w") as fh:
            fh.write(src.replace(old, new))
        lib = compile_oracle(path, os.path.join(tmp_path, f"libmut{k}.so"))
        ef, eg = _uniform_collision_errors(tables, library=lib)
        assert max(ef, eg) > 1e-8, (name, ef, eg)


def test_collision_conserves_mass_and_adds_force_momentum(tables):
    sim = OracleSim(8, ra=1e4, pr=1.0, flow=1)
    d = sim.derived()
    e19 = tables["e19"].astype(float)
    rng = np.random.default_rng(4)
    fin = tables["w19"] * (1 + 0.02 * rng.standard_normal(19))
    T = 0.9
    out = sim.collide_f_cell(fin, T)
    assert abs(out.sum() - fin.sum()) < 1e-15
    np.testing.assert_allclose(e19.T @ out - e19.T @ fin,
                               [0, 0, d.gbeta * (T - d.t0)], atol=1e-16)


# ---------------------------------------------------------------- parameters
def test_parameter_mapping_matches_eq7_and_table1():
    """Fo = alpha t / H^2 equals the paper's Eq. (7) form, and the two
    convection cases of Table 1 at equal lattice time have the Fourier-number
    ratio the paper quotes (1.00 vs 1.57, section 3.2)."""
    rows = [ln.split() for ln in open(golden_path("table1_convection_cases.txt"))
            if ln.strip() and not ln.startswith("#")]
    fo = {}
    for case, pr, ra, ste, fo_shown in rows:
        n, ma, t = 32, 0.1, 1000
        sim = OracleSim(n, ra=float(ra), pr=float(pr), ste=float(ste), ma=ma, flow=1)
        d = sim.derived()
        cs = 1 / math.sqrt(3)
        eq7 = t * math.sqrt(3) * cs / n * ma / math.sqrt(3 * float(ra) * float(pr))
        assert abs(d.alpha * t / n ** 2 - eq7) < 1e-15
        # Rayleigh and Prandtl numbers recovered from the lattice parameters
        ra_back = d.gbeta * 1.0 * n ** 3 / (d.nu * d.alpha)
        assert abs(ra_back / float(ra) - 1) < 1e-12
        assert abs(d.nu / d.alpha / float(pr) - 1) < 1e-12
        fo[int(case)] = (d.alpha * t / n ** 2, float(fo_shown))
    ratio = fo[2][0] / fo[1][0]  # Fo of case 2 over case 1 at equal lattice time
    assert abs(ratio - fo[2][1] / fo[1][1]) < 0.01 * ratio


# ---------------------------------------------------------------- Neumann
def test_neumann_closed_form_solves_the_stefan_problem():
    """The closed form itself: heat equation in the liquid, T(0)=T_h,
    T(s)=T_m, and the Stefan condition ds/dt = -alpha Ste/(T_h-T_m) dT/dy."""
    alpha, ste = 0.1, 0.1
    lam = neumann.stefan_lambda(ste)
    # small-Ste limit lam ~ sqrt(Ste/2)
    assert abs(neumann.stefan_lambda(1e-6) / math.sqrt(0.5e-6) - 1) < 1e-5
    t, hy, ht = 400.0, 1e-3, 1e-2
    s = neumann.front(t, alpha, ste)
    T = lambda y, tt: neumann.temperature(y, tt, alpha, ste)
    assert abs(T(0.0, t) - 1.0) < 1e-14
    y = 0.5 * s
    Tt = (T(y, t + ht) - T(y, t - ht)) / (2 * ht)
    Tyy = (T(y + hy, t) - 2 * T(y, t) + T(y - hy, t)) / hy ** 2
    assert abs(Tt - alpha * Tyy) < 1e-6 * abs(Tt)
    Ty_s = (T(s - 1e-6, t) - T(s - 2e-6, t)) / 1e-6
    ds_dt = (neumann.front(t + ht, alpha, ste) - neumann.front(t - ht, alpha, ste)) / (2 * ht)
    assert abs(ds_dt + alpha * ste * Ty_s) < 1e-5 * ds_dt
    assert abs(lam - 0.2200) < 5e-5


def _run_conduction(n, s0, steps, ste=0.1, alpha=0.1):
    sim = OracleSim(n, ste=ste, flow=0, alpha=alpha, s0=s0, seed_profile=1)
    sim.step(steps)
    t = neumann.seed_time(s0, alpha, ste) + steps
    return sim, t


def test_conduction_melting_tracks_neumann():
    """Conduction-controlled melting (section 3.1): 24^3, Ste = 0.1, 2000
    steps, energy distribution only."""
    n, alpha, ste = 24, 0.1, 0.1
    sim, t = _run_conduction(n, 1.0, 2000)
    s_exact = float(neumann.front(t, alpha, ste))
    assert abs(sim.s.mean() - s_exact) < 0.01
    # front is flat: x- and z-invariant to round-off
    assert sim.s.max() - sim.s.min() < 1e-12
    F = sim.fields()
    T = F["T"]
    assert np.abs(T - T[:, :, :1]).max() < 1e-12  # x-invariance
    assert np.abs(T - T[:1, :, :]).max() < 1e-12  # z-invariance
    y = np.arange(n) + 0.5
    Te = neumann.temperature(y, t, alpha, ste)
    assert np.abs(T[n // 2, :, n // 2] - Te).max() < 1e-3
    # solid stays at the melting temperature exactly (no subcooling)
    solid = y > sim.s.max()
    assert np.all(T[:, solid, :] == 0.0)
    # front-based liquid fraction equals s/H for a flat front
    assert abs(sim.liquid_fraction() - sim.s.mean() / n) < 1e-13


@pytest.mark.slow
def test_conduction_error_falls_with_resolution():
    errs = []
    for n, s0, steps in [(24, 1.0, 2000), (48, 2.0, 8000)]:
        sim, t = _run_conduction(n, s0, steps)
        errs.append(abs(sim.s.mean() - float(neumann.front(t, 0.1, 0.1))) / n)
    assert errs[1] < 0.5 * errs[0]


def test_conduction_larger_stefan_number_tracks_neumann():
    """Ste = 0.5 (also verified in section 3.1)."""
    n, alpha, ste = 24, 0.1, 0.5
    sim, t = _run_conduction(n, 1.5, 600, ste=ste)
    s_exact = float(neumann.front(t, alpha, ste))
    assert abs(sim.s.mean() - s_exact) < 0.02


# ---------------------------------------------------------------- Eq. (6)
def _manufactured_front(n, s_of_x, T_of_column, th=None):
    sim = OracleSim(n, ste=0.1, flow=0, alpha=0.1, s0=1.0)
    s = sim.s
    for x in range(n):
        s[:, x] = s_of_x(x)
    g = sim.g
    w7 = np.array([0.25] + [0.125] * 6)
    T = np.zeros((n, n, n))
    for x in range(n):
        T[:, :, x] = T_of_column(np.arange(n) + 0.5, s_of_x(x))[None, :]
    g[:] = w7[:, None, None, None] * T[None]
    if th is not None:
        for x in range(n):
            sim.th[:, x] = th(s_of_x(x))
    return sim


@pytest.mark.parametrize("s_base", [4.3, 6.0, 5.71])
def test_front_velocity_manufactured_tilted_plane(s_base):
    """Tilted front s = s0 + a x with a quadratic liquid profile
    T = T_m + A xi + B xi^2 (xi = s - y) and solid at T_m: Eq. (6) gives
    V = (1 + a^2) alpha Ste (0 - dT/dy)/(T_h - T_m) = (1 + a^2) alpha Ste A."""
    n, slope, A, B = 12, 0.13, 0.21, -0.017
    s_of_x = lambda x: s_base + slope * x
    prof = lambda y, s: np.where(y < s, A * (s - y) + B * (s - y) ** 2, 0.0)
    sim = _manufactured_front(n, s_of_x, prof)
    V = sim.front_velocity()
    alpha, ste = 0.1, 0.1
    expect = (1 + slope ** 2) * alpha * ste * A
    np.testing.assert_allclose(V[:, 1:-1], expect, rtol=1e-12)
    # mirrored slope at the side walls: half the one-sided difference
    np.testing.assert_allclose(V[:, 0], (1 + (slope / 2) ** 2) * alpha * ste * A, rtol=1e-12)


def test_front_velocity_uses_hot_wall_when_column_is_short():
    """With one usable liquid centre the heated-wall point closes the
    one-sided quadratic; a quadratic profile through the wall value is still
    differentiated exactly."""
    n, A, B = 10, 0.3, 0.05
    s_val = 1.7  # liquid centre at 0.5 has xi = 1.2; the wall at xi = 1.7
    prof = lambda y, s: np.where(y < s, A * (s - y) + B * (s - y) ** 2, 0.0)
    sim = _manufactured_front(n, lambda x: s_val, prof,
                              th=lambda s: A * s + B * s * s)
    V = sim.front_velocity()
    np.testing.assert_allclose(V, 0.1 * 0.1 * A, rtol=1e-12)


def test_front_velocity_skips_nearest_centre_closer_than_half():
    """Nearest liquid centre at xi < 1/2 is not used: a profile that is
    quadratic except at that centre still gives the exact gradient."""
    n, A, B = 10, 0.3, 0.05
    s_val = 5.8  # centre 5.5 at xi = 0.3 is skipped
    def prof(y, s):
        T = np.where(y < s, A * (s - y) + B * (s - y) ** 2, 0.0)
        return np.where(np.abs(y - 5.5) < 1e-9, 123.0, T)
    sim = _manufactured_front(n, lambda x: s_val, prof)
    np.testing.assert_allclose(sim.front_velocity(), 0.1 * 0.1 * A, rtol=1e-12)


# ---------------------------------------------------------------- bulk rates
def test_shear_wave_decay_gives_viscosity():
    """Periodic shear wave u_x = A sin(k y) decays as exp(-nu k^2 t) with
    nu = (1/s_nu - 1/2)/3, up to the scheme's O(k^2) dispersion."""
    n = 32
    sim = OracleSim(n, ra=1e4, pr=1.0, flow=1, periodic=True)
    d = sim.derived()
    t = sim.tables()
    e19 = t["e19"].astype(float)
    k = 2 * math.pi / n
    y = np.arange(n) + 0.5
    ux = 1e-3 * np.sin(k * y)
    u = np.zeros((3, n, n, n))
    u[0] = ux[None, :, None]
    eu = np.einsum("qa,azyx->qzyx", e19, u)
    f = t["w19"][:, None, None, None] * (1 + 3 * eu + 4.5 * eu ** 2 - 1.5 * (u ** 2).sum(0))
    sim.f[:] = f

    def amp():
        F = sim.fields()
        return (F["u"][0][0, :, 0] * np.sin(k * y)).sum() * 2 / n

    sim.step(50)
    a0 = amp()
    sim.step(300)
    a1 = amp()
    nu_meas = -math.log(a1 / a0) / (k * k * 300)
    assert abs(nu_meas / d.nu - 1) < 0.005
    assert abs(d.nu - (1 / d.s_nu - 0.5) / 3) < 1e-15


def test_sine_mode_decay_gives_diffusivity():
    """Periodic temperature mode decays as exp(-alpha k^2 t) with
    alpha = (1/q_j - 1/2)/4, up to the scheme's O(k^2) dispersion."""
    n = 32
    sim = OracleSim(n, ra=1e4, pr=1.0, flow=1, periodic=True)
    d = sim.derived()
    k = 2 * math.pi / n
    y = np.arange(n) + 0.5
    T = d.t0 + 1e-2 * np.sin(k * y)
    w7 = np.array([0.25] + [0.125] * 6)
    sim.g[:] = w7[:, None, None, None] * T[None, None, :, None]
    # the y-varying buoyancy drives u_z(y), which does not advect a
    # y-only temperature mode, so the mode decays by diffusion alone
    def amp():
        Tf = sim.fields()["T"][0, :, 0] - d.t0
        return (Tf * np.sin(k * y)).sum() * 2 / n

    sim.step(20)
    a0 = amp()
    sim.step(200)
    a1 = amp()
    al = -math.log(a1 / a0) / (k * k * 200)
    assert abs(al / d.alpha - 1) < 0.005
    assert abs(d.alpha - 0.25 * (1 / d.q_j - 0.5)) < 1e-15


# ---------------------------------------------------------------- walls
@pytest.mark.parametrize("s0", [6.0, 6.37, 5.81, 6.05, 6.95])
def test_steady_conduction_between_hot_wall_and_fixed_front(s0):
    """Front frozen (Ste = 0) at a fractional position: the steady liquid
    profile is the straight line from T_h at y = 0 to T_m at y = s.  The
    interpolated anti-bounce-back (both link-fraction branches) reproduces it
    to round-off."""
    n = 10
    sim = OracleSim(n, ste=0.0, flow=0, alpha=0.2, s0=s0)
    sim.step(4000)
    T = sim.fields()["T"][n // 2, :, n // 2]
    y = np.arange(n) + 0.5
    liq = y < s0
    lin = 1.0 + (0.0 - 1.0) * y / s0
    assert np.abs(T[liq] - lin[liq]).max() < 1e-12
    assert np.all(T[~liq] == 0.0)


def test_mass_changes_only_by_melted_cells():
    n = 16
    sim = OracleSim(n, ra=1e4, pr=1.0, ste=0.5, flow=1, s0=2.0)
    def liquid_mass():
        return sim.fields()["rho"].sum()
    m0 = liquid_mass()
    sim.step(300)
    assert sim.melted > 0
    assert abs(liquid_mass() - (m0 + sim.melted)) < 1e-10


def test_convection_mirror_symmetry_and_buoyancy_sign():
    """The cavity is mirror-symmetric in x: T symmetric, u_x antisymmetric.
    Hot liquid (T above the mean) rises (u_z > 0)."""
    n = 12
    sim = OracleSim(n, ra=1e5, pr=1.0, ste=0.5, flow=1, s0=4.0)
    sim.step(300)
    F = sim.fields()
    T, u = F["T"], F["u"]
    np.testing.assert_allclose(T, T[:, :, ::-1], atol=1e-13)
    np.testing.assert_allclose(u[0], -u[0][:, :, ::-1], atol=1e-15)
    np.testing.assert_allclose(u[2], u[2][:, :, ::-1], atol=1e-15)
    np.testing.assert_allclose(sim.s, sim.s[:, ::-1], atol=1e-14)
    liquid = F["rho"] > 0
    hot = liquid & (T > 0.5)
    assert u[2][hot].mean() > 0
    assert u[2][liquid & ~hot].mean() < 0
