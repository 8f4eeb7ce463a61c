"""Pins of the oracle's reference adjoint (reverse mode of its own step).

The adjoint is checked against central finite differences of the forward
oracle: the one-step dot-product identity <J v, w> = <v, J^T w> with random
directions in every input (f, g, front heights, hot-wall temperatures), and
the gradient of the liquid fraction after several steps with respect to the
hot-wall temperatures.  Phase and node selection are piecewise constant; the
perturbations are small enough not to move any of them.
"""
import numpy as np
import pytest

from oracle import OracleSim

HEAT = {"y0": 0, "z0": 1}


def _developed(n, steps, **kw):
    sim = OracleSim(n, **kw)
    sim.step(steps)
    return sim


def _clone(src, kw, f, g, s, th):
    sim = OracleSim(src.n, **kw)
    sim.f[:] = f
    sim.g[:] = g
    sim.s[:] = s
    sim.th[:] = th
    return sim


@pytest.mark.parametrize("case", [
    dict(flow=1, heating=0, ra=1e5, ste=1.0, s0=5.3),
    dict(flow=1, heating=1, ra=1e5, ste=1.0, s0=4.7),
    dict(flow=0, heating=0, alpha=0.1, ste=1.0, s0=5.3),
    dict(flow=1, heating=0, ra=1e5, ste=1.0, s0=5.3, t_c=-0.3, ks_kl=2.0),
    dict(flow=1, heating=0, ra=1e5, ste=1.0, s0=5.3, f_wall=1),
    dict(flow=1, heating=1, ra=1e5, ste=1.0, s0=4.7, f_wall=1),
    dict(flow=1, heating=0, ra=1e5, ste=1.0, s0=5.3, front_scheme=1),
    dict(flow=0, heating=1, alpha=0.1, ste=1.0, s0=4.7, front_scheme=1, t_c=-0.3),
])
def test_one_step_dot_product(case):
    n = 12
    kw = dict(pr=1.0, **case)
    base = _developed(n, 120, **kw)
    f0, g0, s0, th0 = base.f.copy(), base.g.copy(), base.s.copy(), base.th.copy()
    rng = np.random.default_rng(5)
    vf = rng.standard_normal(f0.shape) * 1e-2 * np.abs(f0).max()
    vg = rng.standard_normal(g0.shape) * 1e-2 * np.abs(g0).max()
    vs = rng.standard_normal(s0.shape)
    vth = rng.standard_normal(th0.shape)
    wf = rng.standard_normal(f0.shape)
    wg = rng.standard_normal(g0.shape)
    ws = rng.standard_normal(s0.shape)
    if not case["flow"]:
        vf[:] = 0.0
        wf[:] = 0.0

    # adjoint of one step at the base state
    a = _clone(base, kw, f0, g0, s0, th0)
    a.record(1)
    lf, lg, ls, lth = a.adjoint(wf, wg, ws)
    rhs = (vf * lf).sum() + (vg * lg).sum() + (vs * ls).sum() + (vth * lth).sum()

    eps = 1e-7
    out = []
    for sign in (1.0, -1.0):
        b = _clone(base, kw, f0 + sign * eps * vf, g0 + sign * eps * vg, s0 + sign * eps * vs,
                   th0 + sign * eps * vth)
        b.step(1)
        out.append((b.f.copy(), b.g.copy(), b.s.copy()))
    lhs = sum(((p - m) / (2 * eps) * w).sum() for p, m, w in zip(out[0], out[1], (wf, wg, ws)))
    assert abs(lhs - rhs) <= 1e-6 * abs(rhs), (lhs, rhs)


def test_gradient_of_liquid_fraction_matches_finite_differences():
    """d f_l(t + 40) / d T_h(x, z) from the reverse sweep against central
    differences for single columns and a random direction."""
    n = 12
    kw = dict(pr=1.0, flow=1, heating=0, ra=1e5, ste=1.0, s0=3.6)
    base = _developed(n, 60, **kw)
    f0, g0, s0 = base.f.copy(), base.g.copy(), base.s.copy()
    rng = np.random.default_rng(9)
    th0 = 1.0 + 0.1 * rng.standard_normal((n, n))
    steps = 40

    a = _clone(base, kw, f0, g0, s0, th0)
    a.record(steps)
    *_, grad = a.adjoint()
    assert np.abs(grad).max() > 0

    def J(th):
        b = _clone(base, kw, f0, g0, s0, th)
        b.step(steps)
        return b.liquid_fraction()

    # J is close to linear in T_h: a large step keeps the difference quotient
    # above the forward round-off (a 1e-5 step leaves ~2e-5 relative noise)
    eps = 1e-2
    for c in [(0, 0), (5, 6), (11, 3)]:
        e = np.zeros((n, n))
        e[c] = 1.0
        fd = (J(th0 + eps * e) - J(th0 - eps * e)) / (2 * eps)
        assert abs(fd - grad[c]) <= 1e-6 * abs(grad).max(), (c, fd, grad[c])
    d = rng.standard_normal((n, n))
    fd = (J(th0 + eps * d) - J(th0 - eps * d)) / (2 * eps)
    assert abs(fd - (grad * d).sum()) <= 1e-6 * abs(fd), (fd, (grad * d).sum())
