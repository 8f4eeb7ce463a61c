"""Pins of the oracle's front condition of the energy distribution.

The front is the isotherm T = T_m that Eq. (6) moves (section 2). The oracle
imposes it on every D3Q7 link that crosses the front with the interpolated
anti-bounce-back of its reading R8, at the fraction of the link where the
front cuts it. Two pins fix that fraction and the interpolation from outside
the oracle:

* Geometry. Along a link, the melt-axis height of the point and the front
  (linear between the heights of the two columns) are both linear in the
  link parameter. Bisection on their difference gives the fraction. The test
  covers every D3Q7 link that crosses a rough random front, from liquid and
  from solid cells, in both heatings.
* A fixed point of the scheme. Take pure conduction (flow frozen) in a
  temperature field that is linear in space and equals T_m on a tilted plane
  front, continued through both phases. The discrete steady state of the
  D3Q7 MRT scheme is then known in closed form. Collision conserves T,
  relaxes the first moments at rate q_j and leaves the even moments at
  equilibrium. So the post-collision populations
      g*_q(x) = w_q [T(x) + (1 - 1/q_j) e_q . grad T]
  are reproduced by one step exactly, provided every streamed population
  equals the pull from the linear field continued across the walls. For a
  front at link fraction d (a plane, so the linear front model of the
  fraction is exact), both branches of the interpolated anti-bounce-back
  reproduce it (d < 1/2 through the cell behind, d >= 1/2 through the cell's
  own opposite population). The derivation holds for any q_j and d, so one
  step must leave every cell whose links stay off the adiabatic and far
  walls unchanged to round-off.

A mistake in the fraction (d taken as 1 - d across columns or along the melt
axis), in the branch weights, in the cell behind or in the wall value moves
the pulled value off the linear field. The last test plants each such
mistake in a copy of the oracle and checks that the fixed-point pin fails.
"""
import os

import numpy as np
import pytest

from oracle import OracleSim
from oracle.oracle import _SRC, compile_oracle

from linear_field import T_M, fixed_point_state, interior

N = 12


def _run_fixed_point(heating, library=None):
    o = OracleSim(N, flow=0, ste=0.0, alpha=0.1, t_h=1.0, t_c=T_M, t_m=T_M, s0=6.0,
                  heating=heating, library=library)
    tb = o.tables()
    q_j = o.derived().q_j
    g, s, th = fixed_point_state(N, heating, q_j, tb["w7"], tb["e7"])
    o.g[:] = g
    o.s[:] = s
    o.th[:] = th
    o.step(1)
    assert np.array_equal(o.s, s)  # Ste = 0 freezes the front
    m = interior(N, heating)
    return float(np.abs(o.g[:, m] - g[:, m]).max()), o, g


def _link_census(o, heating):
    """Interface links pulled by interior cells, by kind and branch."""
    n = o.n
    e7 = o.tables()["e7"]
    s = o.s
    m = interior(n, heating)

    def liquid(x, y, z):
        a, oc = (y, z) if heating == 0 else (z, y)
        return a + 0.5 < s[oc, x]

    counts = {}
    for z in range(n):
        for y in range(n):
            for x in range(n):
                if not m[z, y, x]:
                    continue
                lq = liquid(x, y, z)
                for q in range(1, 7):
                    sx, sy, sz = np.array([x, y, z]) - e7[q]
                    if not (0 <= sx < n and 0 <= sy < n and 0 <= sz < n):
                        continue
                    if liquid(sx, sy, sz) == lq:
                        continue
                    along = (e7[q][1] if heating == 0 else e7[q][2]) != 0
                    d = o.link_fraction7(x, y, z, q)
                    key = ("melt" if along else "lateral", "d<1/2" if d < 0.5 else "d>=1/2",
                           "liquid" if lq else "solid")
                    counts[key] = counts.get(key, 0) + 1
    return counts


@pytest.mark.parametrize("heating", [0, 1])
def test_linear_field_through_a_tilted_front_is_a_fixed_point(heating):
    err, o, g = _run_fixed_point(heating)
    assert err <= 1e-15 * 8, err
    # the pin exercises both branches along the melt axis and across
    # columns, from both phases
    counts = _link_census(o, heating)
    for kind in ("melt", "lateral"):
        for br in ("d<1/2", "d>=1/2"):
            for ph in ("liquid", "solid"):
                assert counts.get((kind, br, ph), 0) >= 4, counts
    # the field is not trivially uniform: the populations span the front
    assert np.ptp(g[0]) > 0.05


@pytest.mark.parametrize("heating", [0, 1])
def test_energy_link_fraction_matches_bisection_on_the_front_model(heating):
    """Rough random fronts on 8^3: for every D3Q7 link that crosses the
    front, from a liquid or a solid cell, the oracle's fraction equals a
    bisection on the geometric model to 1e-12 and lies in [0, 1]."""
    n = 8
    rng = np.random.default_rng(21 + heating)
    o = OracleSim(n, ste=0.0, s0=4.0, heating=heating, flow=0)
    s = 1.5 + 5.0 * rng.random((n, n))
    o.s[:, :] = s
    e7 = o.tables()["e7"]
    checked = {"liquid": 0, "solid": 0, "lateral": 0, "melt": 0}
    for z in range(n):
        for y in range(n):
            for x in range(n):
                a, oc = (y, z) if heating == 0 else (z, y)
                lq = a + 0.5 < s[oc, x]
                for q in range(1, 7):
                    src = np.array([x, y, z]) - e7[q]
                    if np.any(src < 0) or np.any(src >= n):
                        continue
                    sa, so = (src[1], src[2]) if heating == 0 else (src[2], src[1])
                    s_src = s[so, src[0]]
                    if (sa + 0.5 < s_src) == lq:
                        continue  # same phase: regular pull
                    ea = sa - a

                    def phi(t):  # height of the point minus the front
                        return (a + 0.5 + t * ea) - (s[oc, x] + t * (s_src - s[oc, x]))

                    lo, hi = 0.0, 1.0
                    sign0 = phi(lo) < 0.0
                    assert (phi(hi) < 0.0) != sign0
                    for _ in range(80):
                        mid = 0.5 * (lo + hi)
                        if (phi(mid) < 0.0) == sign0:
                            lo = mid
                        else:
                            hi = mid
                    d = o.link_fraction7(x, y, z, q)
                    assert 0.0 <= d <= 1.0
                    assert abs(d - hi) <= 1e-12, (x, y, z, q, d, hi)
                    checked["liquid" if lq else "solid"] += 1
                    checked["melt" if ea else "lateral"] += 1
    assert min(checked.values()) > 50, checked


# Planted mistakes: (name, text in the oracle source, replacement).  Each must
# occur exactly once, so a change of the oracle that moves the text fails
# here instead of passing silently.
MISTAKES = [
    ("fraction across columns taken as 1 - d",
     "  return (a - s[c]) / (s[cn] - s[c] - ea);\n",
     "  return ea ? (a - s[c]) / (s[cn] - s[c] - ea) : 1.0 - (a - s[c]) / (s[cn] - s[c]);\n"),
    ("fraction along the melt axis taken as 1 - d",
     "  return (a - s[c]) / (s[cn] - s[c] - ea);\n",
     "  return ea ? 1.0 - (a - s[c]) / (s[cn] - s[c] - ea) : (a - s[c]) / (s[cn] - s[c]);\n"),
    ("d < 1/2: the cell across the front in place of the cell behind",
     "      int bx = x + E7[q][0], by = y + E7[q][1], bz = z + E7[q][2];\n"
     "      wrap_lateral(S, &bx, &by, &bz);\n",
     "      int bx = x + E7[po][0], by = y + E7[po][1], bz = z + E7[po][2];\n"
     "      wrap_lateral(S, &bx, &by, &bz);\n"),
    ("d >= 1/2: the opposite population in place of the cell's own",
     "(2.0 * d - 1.0) / (2.0 * d) * g[q * nc + i] + w * p->t_m / d;",
     "(2.0 * d - 1.0) / (2.0 * d) * g[po * nc + i] + w * p->t_m / d;"),
    ("d >= 1/2: wall value weighted 1/(2d) instead of 1/d",
     "(2.0 * d - 1.0) / (2.0 * d) * g[q * nc + i] + w * p->t_m / d;",
     "(2.0 * d - 1.0) / (2.0 * d) * g[q * nc + i] + w * p->t_m / (2.0 * d);"),
    ("d < 1/2: weights of the two populations swapped",
     "          gl[q] = -(2.0 * d * g[po * nc + i] +\n"
     "                    (1.0 - 2.0 * d) * g[po * nc + cell_index(n, bx, by, bz)]) +\n",
     "          gl[q] = -((1.0 - 2.0 * d) * g[po * nc + i] +\n"
     "                    2.0 * d * g[po * nc + cell_index(n, bx, by, bz)]) +\n"),
]


def test_fixed_point_pin_catches_planted_mistakes(tmp_path):
    src = open(_SRC).read()
    for k, (name, old, new) in enumerate(MISTAKES):
        assert src.count(old) == 1, name
        path = os.path.join(tmp_path, f"mut{k}.c")
        with open(path, "w") as fh:
            fh.write(src.replace(old, new))
        lib = compile_oracle(path, os.path.join(tmp_path, f"libmut{k}.so"))
        errs = [_run_fixed_point(h, library=lib)[0] for h in (0, 1)]
        assert max(errs) > 1e-6, (name, errs)
