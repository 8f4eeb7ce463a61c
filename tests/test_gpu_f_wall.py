"""Parity of the interpolated no-slip of f at the front (f_wall = 1) with
the oracle, through the C ABI.

For a population whose source cell is solid, the GPU's general path bounces
back from the point where the front cuts the link, at fraction d. That fraction
is linear in both columns' fronts and uses the melt-axis step of the link,
diagonal links included. The rough random fronts below give every kind of
crossing link (along the melt axis, lateral, diagonal), both branches of the
interpolation, and cells with and without a liquid cell behind them.
Bars as for halfway bounce-back: FP64 at round-off, FP32 within
max|dT| <= 1e-5 and relative liquid-fraction error <= 1e-6.  (The adjoint with
this option is tested in test_gpu_adjoint.py.)
"""
import numpy as np
import pytest

from test_gpu_parity import _one_step_random, diffs, make_pair

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["f64", "f32", "f16s"])
@pytest.mark.parametrize("heating", ["y0", "z0"])
def test_one_step_random_state_72(prec, heating):
    """72^3 (a 64-lane tile and a ragged one), one step from a random state.
    FP64 gets a rough front (independent heights per column), the reduced
    precisions a smooth one (as for halfway bounce-back: the slope factor of
    Eq. (6) amplifies any rounding of T into the front on a rough one)."""
    front = (10.0, 50.0) if prec == "f64" else (30.0, 31.8)
    d = _one_step_random(72, prec, seed=5, heating=heating, front=front, f_wall=1)
    tol = {"f64": 1e-14, "f32": 2e-7, "f16s": 1e-3}[prec]
    tol_s = {"f64": 1e-12, "f32": 1e-6, "f16s": 1e-3}[prec]
    assert d["g"] <= tol and d["f"] <= tol and d["s"] <= tol_s, d


@pytest.mark.parametrize("heating,s0", [("y0", 23.3), ("z0", 10.6)])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_convection_melting_70(heating, s0, prec):
    """Full double MRT with buoyancy and a moving front, 70^3, 150 steps."""
    orc, gpu = make_pair(150, n=70, ra=1e5, pr=1.0, ste=0.5, s0=s0, heating=heating,
                         precision=prec, f_wall=1)
    d = diffs(orc, gpu)
    assert d["mask"] == 0, d
    if prec == "f64":
        assert d["T"] < 1e-12 and d["s"] < 1e-12 and d["u"] < 1e-14 and d["rho"] < 1e-13, d
    else:
        assert d["T"] <= 1e-5 and d["fl_rel"] <= 1e-6, d
        assert d["u"] <= 1e-6 and d["rho"] <= 1e-6, d
    gpu.close()


def test_interpolation_differs_from_halfway_where_the_front_is_inside_a_cell():
    """The same run with both rules: identical for a flat front at an integer
    height (every crossing link cut at d = 1/2), different for a front inside
    a cell."""
    from paper_1604_03478_amd import Config, Sim
    out = {}
    for s0 in (10.0, 10.3):
        for fw in (0, 1):
            sim = Sim(Config(n=32, ra=1e5, pr=1.0, ste=0.0, s0=s0, precision="f32", f_wall=fw))
            sim.step(200)
            out[(s0, fw)] = sim.get_populations()
            sim.close()
    from live_state import states_equal
    assert states_equal(out[(10.0, 0)], out[(10.0, 1)])
    assert not states_equal(out[(10.3, 0)], out[(10.3, 1)])
