"""Pins of the oracle's interpolated no-slip of f at the front.

With f_wall = 1, a population whose source cell is solid bounces back from
the point where the front cuts the link, at fraction d of the link from the
cell's centre. The bounced value is interpolated linearly between this
cell's populations and, for d < 1/2, those of the cell behind it. The pins:

* Plane Poiseuille flow in the channel test mode. The two lateral axes are
  periodic and a uniform force acts along x. The heated wall sits at face 0
  and a frozen flat front at height s. For a front anywhere inside a cell
  (both branches of the interpolation), the steady profile converges to the
  closed form u(zeta) = F zeta (s - zeta) / (2 nu) at second order in the
  lattice spacing. Halfway bounce-back puts the wall at a cell face and
  converges only at first order.
* At d = 1/2 the interpolation reduces to halfway bounce-back, so the run is
  bitwise the same.
* The two heating axes (melt axis y or z) give the same channel profile.
* For every D3Q19 link that crosses a non-flat front, the closed-form link
  fraction agrees with a bisection on its geometric model.
"""
import numpy as np
import pytest

from oracle import OracleSim

U0 = 0.1 / np.sqrt(3.0)  # Ma = 0.1


def channel(n, s0, f_wall, heating=1, nu=1.0 / 6.0, umax=0.02):
    """Steady channel profile (mean over the lateral axes) and its closed form."""
    ra = (U0 * n / nu) ** 2  # with Pr = 1: nu = U0 n sqrt(Pr / Ra)
    fx = 8.0 * nu * umax / s0 ** 2
    o = OracleSim(n, ra=ra, pr=1.0, ste=0.0, s0=s0, heating=heating, flow=1, periodic=2,
                  f_wall=f_wall, body_fx=fx)
    nu_l = o.derived().nu
    # from rest, the slowest mode decays as exp(-pi^2 nu t / s^2): < 1e-8 is left
    o.step(int(2.0 * s0 * s0 / nu_l))
    ux = o.fields()["u"][0]  # [z][y][x]
    prof = ux.mean(axis=(1, 2)) if heating == 1 else ux.mean(axis=(0, 2))
    zeta = np.arange(n) + 0.5
    exact = fx / (2.0 * nu_l) * zeta * (s0 - zeta)
    return prof, exact, zeta < s0


def rel_err(n, s0, f_wall, **kw):
    prof, exact, liq = channel(n, s0, f_wall, **kw)
    return np.abs(prof[liq] - exact[liq]).max() / exact[liq].max()


@pytest.mark.parametrize("d", [0.3, 0.8])
def test_poiseuille_converges_at_second_order_for_a_front_inside_a_cell(d):
    """Top liquid cell at a, front at a + 1/2 + d: the d < 1/2 branch (cell
    behind) and the d >= 1/2 branch (own populations). Measured: d = 0.3:
    1.36e-2 -> 3.37e-3 from 12^3 to 24^3 (ratio 0.248); d = 0.8: 4.10e-3 ->
    1.09e-3 (0.265); halfway bounce-back 7.9e-2 and 1.1e-1 at 12^3, ratio 0.50."""
    e12 = rel_err(12, 9.5 + d, 1)
    e24 = rel_err(24, 19.5 + d, 1)
    assert e24 / e12 < 0.3, (e12, e24)
    assert e24 < 4e-3, e24
    h12 = rel_err(12, 9.5 + d, 0)
    assert h12 > 5.0 * e12, (h12, e12)


def test_half_link_interpolation_is_halfway_bounce_back():
    """A flat front at an integer height cuts every crossing link at d = 1/2;
    convection in the cavity (Ra = 1e5, front frozen) is then bitwise the
    same run with either rule."""
    runs = []
    for fw in (0, 1):
        o = OracleSim(16, ra=1e5, pr=1.0, ste=0.0, s0=10.0, flow=1, f_wall=fw)
        o.step(300)
        runs.append((o.f.copy(), o.g.copy()))
    assert np.abs(runs[0][0]).max() > 0.0
    assert np.array_equal(runs[0][0], runs[1][0])
    assert np.array_equal(runs[0][1], runs[1][1])


def test_both_melt_axes_give_the_same_channel_profile():
    """Melt axis z (heating 1) and y (heating 0): the same channel up to
    the order of the sums (pins the melt component of the link fraction)."""
    p1, _, liq = channel(12, 9.8, 1, heating=1)
    p0, _, _ = channel(12, 9.8, 1, heating=0)
    assert np.abs(p1 - p0).max() <= 1e-12 * np.abs(p1).max()
    assert np.abs(p1[~liq]).max() == 0.0  # solid cells carry no velocity


@pytest.mark.parametrize("heating", [0, 1])
def test_link_fraction_matches_bisection_on_the_front_model(heating):
    """Random fronts on 8^3. Along a link, the melt-axis height of the point
    and the front (linear between the two columns' heights) are both linear
    in t. Bisection on their difference must give the closed form to 1e-12,
    and every crossing link is cut once with 0 < d <= 1."""
    n = 8
    rng = np.random.default_rng(11 + heating)
    o = OracleSim(n, ste=0.0, s0=4.0, heating=heating, flow=1)
    s = 1.5 + 5.0 * rng.random((n, n))
    o.s[:, :] = s
    e19 = o.tables()["e19"]
    checked = 0
    for z in range(n):
        for y in range(n):
            for x in range(n):
                a, oc = (y, z) if heating == 0 else (z, y)
                if not a + 0.5 < s[oc, x]:
                    continue  # only liquid cells pull f
                for q in range(1, 19):
                    src = np.array([x, y, z]) - e19[q]
                    if np.any(src < 0) or np.any(src >= n):
                        continue
                    sa, so = (src[1], src[2]) if heating == 0 else (src[2], src[1])
                    s_src = s[so, src[0]]
                    if sa + 0.5 < s_src:
                        continue  # liquid source: regular pull
                    ea = src[1] - y if heating == 0 else src[2] - z

                    def phi(t):  # height of the point minus the front
                        return (a + 0.5 + t * ea) - (s[oc, x] + t * (s_src - s[oc, x]))

                    lo, hi = 0.0, 1.0
                    assert phi(lo) < 0.0 <= phi(hi)
                    for _ in range(80):
                        mid = 0.5 * (lo + hi)
                        if phi(mid) < 0.0:
                            lo = mid
                        else:
                            hi = mid
                    d = o.link_fraction19(x, y, z, q)
                    assert 0.0 < d <= 1.0
                    assert abs(d - hi) <= 1e-12, (x, y, z, q, d, hi)
                    checked += 1
    assert checked > 100
