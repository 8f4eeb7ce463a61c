"""Pins of the oracle's conservative front update: the front
of each column moves by the heat the lattice itself carried into the
interface (sent minus received over the interface links of the streaming),
divided by the latent heat L = (T_h - T_m) / Ste.  An alternative to the
gradient form of Eq. (6) from the same energy balance at the interface.
"""
import numpy as np
import pytest

from oracle import OracleSim, neumann

CONFIGS = [
    dict(flow=0, alpha=0.1, ste=0.1, seed_profile=1, s0=2.0),
    dict(flow=0, alpha=0.1, ste=0.1, seed_profile=2, s0=2.0, t_c=-0.5),
    dict(flow=1, ra=1e5, ste=0.5, s0=6.3),
    dict(flow=1, ra=1e5, ste=0.5, s0=6.3, heating=1, t_c=-0.3, ks_kl=2.0),
]


@pytest.mark.parametrize("kw", CONFIGS)
def test_energy_is_conserved_to_round_off(kw):
    """Sum of T over the cells + L sum of s - heat let in through the walls
    stays constant: the collisions conserve T, the streaming moves it, and
    every boundary link is accounted for (walls in W, the front in s)."""
    o = OracleSim(24, front_scheme=1, **kw)
    e0 = o.energy()
    for _ in range(3):
        o.step(200)
        drift = o.energy() - o.wall_heat() - e0
        assert abs(drift) <= 1e-11 * abs(e0), (kw, drift)
    assert o.wall_heat() != 0.0


@pytest.mark.parametrize("ste", [0.1, 0.5, 1.0])
def test_flux_front_follows_the_neumann_solution(ste):
    """Conduction melting, 24^3, Neumann seed at s0 = 2, 2000 steps
    (measured: within 1.9e-3 at every check)."""
    o = OracleSim(24, flow=0, alpha=0.1, ste=ste, seed_profile=1, s0=2.0, front_scheme=1)
    alpha = o.derived().alpha
    t0 = neumann.seed_time(2.0, alpha, ste)
    for k in range(4):
        o.step(500)
        exact = float(neumann.front(t0 + 500 * (k + 1), alpha, ste))
        assert np.ptp(o.s) <= 1e-12
        assert abs(o.s.mean() / exact - 1.0) <= 3e-3, (ste, k, o.s.mean(), exact)


def test_flux_and_gradient_fronts_agree_in_convection():
    """32^3, Ra = 1e5, Pr = 1, Ste = 0.5, 1500 steps: the two discretizations
    of the interface balance give the same liquid fraction to 2e-3
    (measured 4e-4)."""
    fl = {}
    for sch in (0, 1):
        o = OracleSim(32, ra=1e5, ste=0.5, s0=4.3, front_scheme=sch)
        o.step(1500)
        fl[sch] = o.liquid_fraction()
    assert abs(fl[1] / fl[0] - 1.0) <= 2e-3, fl


@pytest.mark.parametrize("kw", [
    dict(flow=0, alpha=0.1, ste=1.0, front_scheme=1),
    dict(flow=1, ra=1e5, ste=1.0, front_scheme=1),
    dict(flow=1, ra=1e5, ste=1.0, front_scheme=1, heating=1, t_c=-0.3),
    dict(flow=1, ra=1e5, ste=1.0, f_wall=1),
    dict(flow=1, ra=1e5, ste=1.0, f_wall=1, heating=1),
])
def test_reference_adjoint_on_a_rough_front(kw):
    """One-step dot-product identity <J v, w> = <v, J^T w> against central
    differences, from a state whose front heights are independent per column
    (every column's front in a different cell: lateral and diagonal links
    cross the front, and the heat of a lateral link is charged to the column
    of its solid cell)."""
    n = 10
    rng = np.random.default_rng(21)
    base = OracleSim(n, pr=1.0, s0=4.0, **kw)
    base.step(30)
    s0 = 2.2 + 4.6 * rng.random((n, n))
    f0, g0, th0 = base.f.copy(), base.g.copy(), base.th.copy()

    def clone(f, g, s, th):
        o = OracleSim(n, pr=1.0, s0=4.0, **kw)
        o.f[:] = f
        o.g[:] = g
        o.s[:] = s
        o.th[:] = th
        return o

    vf = rng.standard_normal(f0.shape) * 1e-2 * np.abs(f0).max()
    vg = rng.standard_normal(g0.shape) * 1e-2 * np.abs(g0).max()
    vs = rng.standard_normal(s0.shape)
    vth = rng.standard_normal(th0.shape)
    wf, wg, ws = (rng.standard_normal(a.shape) for a in (f0, g0, s0))
    if not kw["flow"]:
        vf[:] = 0.0
        wf[:] = 0.0
    a = clone(f0, g0, s0, th0)
    a.record(1)
    lf, lg, ls, lth = a.adjoint(wf, wg, ws)
    rhs = (vf * lf).sum() + (vg * lg).sum() + (vs * ls).sum() + (vth * lth).sum()
    eps = 1e-7
    out = []
    for sign in (1.0, -1.0):
        b = clone(f0 + sign * eps * vf, g0 + sign * eps * vg, s0 + sign * eps * vs,
                  th0 + sign * eps * vth)
        b.step(1)
        out.append((b.f.copy(), b.g.copy(), b.s.copy()))
    lhs = sum(((p - m) / (2 * eps) * w).sum() for p, m, w in zip(out[0], out[1], (wf, wg, ws)))
    assert abs(lhs - rhs) <= 1e-6 * abs(rhs), (lhs, rhs)
