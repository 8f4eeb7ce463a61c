"""Context state through the C ABI on the GPU: the instability report and
its recovery, the energy diagnostic against the oracle, and the invalidation
of a recorded run when the state or the hot wall changes under it."""
import numpy as np
import pytest

from oracle import OracleSim

pytestmark = pytest.mark.gpu


def test_instability_is_reported_until_load_state():
    """A non-finite population makes the next query return LBM_EUNSTABLE;
    from then on lbm_step returns LBM_ESTATE (and the queries keep
    reporting) until lbm_load_state restores a saved state, after which the
    run continues exactly as one that never saw the bad value.

    The planted values sit well away from the front (a liquid cell's f seven
    cells below it, a solid cell's g four cells above it), so one step
    spreads them only to the neighbouring cells and not into the nodes of
    Eq. (6), which lie within two cells of the front: the fronts stay
    finite."""
    from paper_1604_03478_amd import Config, LbmError, Sim
    from paper_1604_03478_amd.binding import LBM_ESTATE, LBM_EUNSTABLE
    cfg = Config(n=16, ra=1e5, pr=1.0, ste=0.5, s0=9.5, precision="f32")
    sim = Sim(cfg)
    sim.step(10)
    blob = sim.save_state()
    ref = Sim(cfg)
    ref.load_state(blob)
    ref.step(5)
    ref_pop = ref.get_populations()
    ref_fl = ref.liquid_fraction()
    ref.close()

    f, g, s = sim.get_populations()
    assert s.min() > 9.0 and s.max() < 10.0
    f[5, 3, 2, 8] = np.nan  # [q][z][y][x]: cell (8, 2, 3), liquid
    g[3, 8, 14, 5] = np.nan  # cell (5, 14, 8), solid
    sim.set_populations(f, g, s)
    sim.step(1)
    with pytest.raises(LbmError) as e:
        sim.liquid_fraction()
    assert e.value.code == LBM_EUNSTABLE
    with pytest.raises(LbmError) as e:
        sim.step(1)
    assert e.value.code == LBM_ESTATE
    with pytest.raises(LbmError) as e:
        sim.fields(which=("s",))
    assert e.value.code == LBM_EUNSTABLE
    with pytest.raises(LbmError) as e:
        sim.forward_ckpt(2, 1)
    assert e.value.code == LBM_ESTATE
    _, _, s_bad = sim.get_populations()
    assert np.isfinite(s_bad).all()  # the bad values did not reach the fronts

    sim.load_state(blob)
    assert sim.steps == 10
    sim.step(5)
    assert sim.liquid_fraction() == ref_fl
    from live_state import states_equal
    assert states_equal(sim.get_populations(), ref_pop)
    sim.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_energy_and_mass_diagnostics_match_the_oracle(prec):
    """lbm_diagnostics on a developed convecting state with T_m != 0 against
    the oracle: the thermal energy sum of (T - t_m) over all cells (the
    oracle's sum of T plus L sum(s), less L sum(s) and n^3 t_m), the liquid
    mass and the front sum.  Bars from the per-cell parity bars of the
    fields (T and rho: 1e-12 in FP64 storage, 1e-5 in FP32): in FP64 the
    per-cell differences (round-off, FMA contraction on the GPU) may share a
    sign, so N cells add up to N times the bar; in FP32 they are the
    zero-mean errors of stochastic rounding, so sqrt(N) times the bar.  The
    front sum: n^2 fronts at the FP64 round-off / FP32 front bars (1e-12,
    1e-5), summed the same way."""
    from paper_1604_03478_amd import Config, Sim
    kw = dict(ra=1e5, pr=1.0, ste=1.0, s0=4.4, t_h=1.0, t_c=0.2, t_m=0.2)
    n, steps = 40, 300  # melts 1600 cells
    orc = OracleSim(n, **kw)
    orc.step(steps)
    gpu = Sim(Config(n=n, precision=prec, **kw))
    gpu.step(steps)
    d = gpu.diagnostics()
    s_sum = float(orc.s.sum())
    e_ref = orc.energy() - orc.derived().latent * s_sum - n ** 3 * kw["t_m"]
    F = orc.fields()
    assert abs(e_ref - (F["T"] - kw["t_m"]).sum()) <= 1e-9 * abs(e_ref)
    N, NC = n ** 3, n ** 2
    bar = N * 1e-12 if prec == "f64" else np.sqrt(N) * 1e-5
    bar_s = NC * 1e-12 if prec == "f64" else np.sqrt(NC) * 1e-5
    res = {"energy": d["energy"] - e_ref, "mass": d["mass"] - F["rho"].sum(),
           "front_sum": d["front_sum"] - s_sum, "bar": bar, "bar_s": bar_s}
    print(prec, e_ref, res)
    assert d["melted"] == orc.melted and d["melted"] > 0
    assert abs(res["energy"]) <= bar, res
    assert abs(res["mass"]) <= bar, res
    assert abs(res["front_sum"]) <= bar_s, res
    gpu.close()


def test_adjoint_refuses_a_recorded_run_changed_underneath():
    """lbm_adjoint recomputes each segment with the current hot wall, so a
    hot-wall change, a state upload or a state restore after
    lbm_forward_ckpt invalidates the recorded run (LBM_ESTATE) until the
    next lbm_forward_ckpt."""
    from inputs import hot_wall_field
    from paper_1604_03478_amd import Config, LbmError, Sim
    from paper_1604_03478_amd.binding import LBM_ESTATE
    cfg = Config(n=12, ra=1e4, pr=1.0, ste=0.5, s0=3.3, precision="f64")
    sim = Sim(cfg)
    th = hot_wall_field(12, seed=5)
    sim.set_hot_wall(th)
    blob = sim.save_state()
    g_ok = None
    for change in ("none", "hot_wall", "populations", "load_state"):
        sim.load_state(blob)
        sim.set_hot_wall(th)
        sim.forward_ckpt(6, 2)
        if change == "hot_wall":
            sim.set_hot_wall(th)
        elif change == "populations":
            sim.set_populations(*sim.get_populations())
        elif change == "load_state":
            sim.load_state(sim.save_state())
        if change == "none":
            g_ok = sim.adjoint(1.0)
            assert np.abs(g_ok).max() > 0.0
            continue
        with pytest.raises(LbmError) as e:
            sim.adjoint(1.0)
        assert e.value.code == LBM_ESTATE, change
        sim.load_state(blob)
        sim.set_hot_wall(th)
        sim.forward_ckpt(6, 2)
        assert np.array_equal(sim.adjoint(1.0), g_ok)
    sim.close()


@pytest.mark.parametrize("prec", ["f64", "f32", "f16s", "bf16s"])
def test_forward_ckpt_continues_as_plain_steps(prec):
    """lbm_forward_ckpt hands the population buffers of each checkpointed
    state to its checkpoint and continues in others: the run it records, and
    every step after it, must equal plain lbm_step calls bit for bit (a
    segment length that does not divide the run, then a single segment, then
    a saved and reloaded state)."""
    from live_state import states_equal
    from paper_1604_03478_amd import Config, Sim
    cfg = Config(n=24, ra=1e5, pr=1.0, ste=1.0, s0=3.4, t_c=0.1, t_m=0.1, heating="z0",
                 precision=prec)
    a, b = Sim(cfg), Sim(cfg)
    a.step(10)
    b.step(10)
    fa = a.forward_ckpt(23, 5)
    b.step(23)
    assert fa == b.liquid_fraction()
    assert states_equal(a.get_populations(), b.get_populations(), "z0")
    a.step(7)
    b.step(7)
    assert states_equal(a.get_populations(), b.get_populations(), "z0")
    fa = a.forward_ckpt(4, 9)
    b.step(4)
    assert fa == b.liquid_fraction()
    g1 = a.adjoint(1.0)
    assert np.isfinite(g1).all()
    blob = a.save_state()
    a.step(5)
    b.step(5)
    assert states_equal(a.get_populations(), b.get_populations(), "z0")
    a.load_state(blob)
    a.step(5)
    assert a.steps == b.steps
    assert states_equal(a.get_populations(), b.get_populations(), "z0")
    a.close()
    b.close()
