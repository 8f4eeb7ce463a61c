"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Both sides start from the same parameters and build their initial state
independently; every comparison is element by element over the whole field
at sizes that span several 64-wide x tiles and 4-row y tiles with ragged
tails.  Tolerances: FP64 storage at round-off; FP32 storage within
max|dT| <= 1e-5 and relative liquid-fraction error <= 1e-6.
"""
import numpy as np
import pytest

from oracle import OracleSim

pytestmark = pytest.mark.gpu

HEAT = {"y0": 0, "z0": 1}


def make_pair(steps=0, **kw):
    from paper_1604_03478_amd import Config, Sim
    cfg = Config(**kw)
    orc = OracleSim(cfg.n, ra=cfg.ra, pr=cfg.pr, ste=cfg.ste, t_h=cfg.t_h, t_c=cfg.t_c,
                    t_m=cfg.t_m, ma=cfg.ma, alpha=cfg.alpha, s0=cfg.s0,
                    heating=HEAT[cfg.heating], flow=cfg.flow, seed_profile=cfg.seed_profile,
                    ks_kl=cfg.ks_kl, front_scheme=cfg.front_scheme, f_wall=cfg.f_wall)
    gpu = Sim(cfg)
    if steps:
        orc.step(steps)
        gpu.step(steps)
    return orc, gpu


def diffs(orc, gpu):
    Fo, Fg = orc.fields(), gpu.fields()
    liq = Fo["rho"] > 0
    return {
        "T": np.abs(Fo["T"] - Fg["T"]).max(),
        "s": np.abs(Fo["s"] - Fg["s"]).max(),
        "u": np.abs(Fo["u"] - Fg["u"]).max(),
        "rho": np.abs(Fo["rho"] - Fg["rho"]).max(),
        "mask": int(np.sum(liq != (Fg["rho"] > 0))),
        "fl_rel": abs(orc.liquid_fraction() - gpu.liquid_fraction()) / max(orc.liquid_fraction(), 1e-300),
    }


def test_initial_state_matches():
    for prec in ("f64", "f32"):
        orc, gpu = make_pair(n=20, flow=0, ste=0.1, s0=3.4, alpha=0.1, seed_profile=1,
                             precision=prec)
        d = diffs(orc, gpu)
        assert d["T"] < (1e-15 if prec == "f64" else 1e-7), d
        assert d["s"] == 0.0


@pytest.mark.parametrize("prec,tol_T,tol_s", [("f64", 1e-12, 1e-12), ("f32", 1e-5, 1e-5)])
def test_conduction_melting_24(prec, tol_T, tol_s):
    """Conduction-controlled melting, 24^3, D3Q7 only, Ste = 0.1, 2000
    steps, Neumann seed (the paper's verification case, section 3.1)."""
    orc, gpu = make_pair(2000, n=24, flow=0, ste=0.1, s0=1.0, alpha=0.1, seed_profile=1,
                         precision=prec)
    d = diffs(orc, gpu)
    assert d["T"] <= tol_T and d["s"] <= tol_s and d["mask"] == 0, d
    assert d["fl_rel"] <= (1e-13 if prec == "f64" else 1e-6), d


@pytest.mark.parametrize("heating,s0", [("y0", 23.3), ("z0", 10.6)])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_convection_melting_70(heating, s0, prec):
    """Full double MRT with buoyancy and a moving front, 70^3 (two x tiles,
    ragged y tiles), 150 steps."""
    orc, gpu = make_pair(150, n=70, ra=1e5, pr=1.0, ste=0.5, s0=s0, heating=heating,
                         precision=prec)
    d = diffs(orc, gpu)
    assert d["mask"] == 0, d
    if prec == "f64":
        assert d["T"] < 1e-12 and d["s"] < 1e-12 and d["u"] < 1e-14 and d["rho"] < 1e-13, d
    else:
        assert d["T"] <= 1e-5 and d["fl_rel"] <= 1e-6, d
        assert d["u"] <= 1e-6 and d["rho"] <= 1e-6, d


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_one_step_from_developed_state(prec):
    """Run the oracle into a developed convecting state with a curved front,
    hand the same state to both sides, take one step, compare."""
    from paper_1604_03478_amd import Config, Sim
    n = 36
    kw = dict(n=n, ra=1e5, pr=1.0, ste=1.0, s0=9.7)
    orc = OracleSim(n, ra=1e5, pr=1.0, ste=1.0, s0=9.7)
    orc.step(400)
    gpu = Sim(Config(**kw, precision=prec))
    gpu.set_populations(orc.f.copy(), orc.g.copy(), orc.s.copy())
    assert np.ptp(orc.s) > 0.02  # the front is not flat
    d0 = diffs(orc, gpu)
    assert d0["mask"] == 0
    orc.step(1)
    gpu.step(1)
    d = diffs(orc, gpu)
    if prec == "f64":
        assert d["T"] < 1e-14 and d["s"] < 1e-14 and d["u"] < 1e-16 and d["rho"] < 1e-15, d
    else:
        assert d["T"] < 1e-6 and d["s"] < 1e-7 and d["u"] < 1e-8, d


@pytest.mark.parametrize("n,s0", [(4, 1.5), (5, 0.0), (9, 9.0), (7, 3.5)])
def test_edge_sizes_and_fronts(n, s0):
    """Minimum size, ragged tiles, all-solid and all-liquid boxes, a front
    exactly on a cell face."""
    orc, gpu = make_pair(60, n=n, ra=1e3, pr=1.0, ste=0.5, s0=s0, precision="f64")
    d = diffs(orc, gpu)
    assert d["mask"] == 0 and d["T"] < 1e-13 and d["s"] < 1e-13 and d["u"] < 1e-15, d


def test_runs_are_bitwise_deterministic():
    from paper_1604_03478_amd import Config, Sim
    out = []
    from live_state import states_equal
    for _ in range(2):
        g = Sim(Config(n=40, ra=1e5, pr=1.0, ste=0.5, s0=11.2, precision="f32"))
        g.step(120)
        out.append(g.get_populations())
    assert states_equal(out[0], out[1])


def test_save_load_resume_is_bitwise():
    from paper_1604_03478_amd import Config, Sim
    cfg = Config(n=24, ra=1e5, pr=1.0, ste=0.5, s0=6.3, precision="f32")
    a = Sim(cfg)
    a.step(80)
    ref = a.get_populations()
    b = Sim(cfg)
    b.step(40)
    blob = b.save_state()
    c = Sim(cfg)
    c.load_state(blob)
    assert c.steps == 40
    c.step(40)
    from live_state import states_equal
    assert states_equal(ref, c.get_populations())


def test_mass_conservation_on_gpu():
    from paper_1604_03478_amd import Config, Sim
    g = Sim(Config(n=32, ra=1e5, pr=1.0, ste=1.0, s0=4.4, precision="f64"))
    m0 = g.diagnostics()["mass"]
    g.step(400)
    d = g.diagnostics()
    assert d["melted"] > 0
    assert abs(d["mass"] - (m0 + d["melted"])) < 1e-9
    # each reduction covers exactly its own array (the front has n^2 values)
    F = g.fields()
    assert abs(d["front_sum"] - F["s"].sum()) < 1e-9
    assert abs(d["mass"] - F["rho"].sum()) < 1e-9


@pytest.mark.parametrize("prec,unit_roundoff", [("f16s", 2.0 ** -11), ("bf16s", 2.0 ** -8)])
def test_sixteen_bit_shifted_storage(prec, unit_roundoff):
    """16-bit storage of the shifted populations with FP32 collision and
    stochastic rounding at the store, 40^3 convection melting (Ra = 1e5,
    Pr = 1, Ste = 0.5), 400 steps, against the FP64 oracle.  Bars from the
    zero-mean rounding noise:

    * T.  A stored deviation g_q - w_q T_ref (T in [0, 1], T_ref = 1/2) is at
      most 1/8 for the rest population and below 1/8 for the others (at most
      1/16 plus a small flux part), so its ulp is at most (1/8) 2u and
      (1/16) 2u (u the unit round-off).  Stochastic rounding leaves an error
      of zero mean and variance p (1 - p) ulp^2 <= ulp^2 / 4 per value, so a
      cell's T (the sum of 7 values) gets sigma_T <= u sqrt(1/64 + 6/256)
      per step.  Conserved T errors then spread: the variance left at a cell
      is sigma_T^2 times A = sum over k of the squared propagator after k
      steps, at most 1 for the first few steps and (8 pi alpha k)^(-3/2) by
      diffusion after, A <= 6 + (8 pi alpha)^(-3/2) 2 / sqrt(5) (17 at
      alpha = 0.0073).  The largest of 64 000 cells lies within 5 sigma:
      max |dT| <= 5 sigma_T sqrt(A), 2.0e-3 (FP16) and 1.6e-2 (BF16).
    * Front.  Eq. (6) turns node temperature errors into a velocity error of
      P K (dG_s - dG_l), K = alpha Ste / (t_h - t_m), P the slope factor,
      with |dG/dT| <= 3 and 0.6 at the two nodes of a side (nodes at 1/2 and
      3/2 from the front at worst): rms 4.33 sigma_T sqrt(A) P K per step,
      taken independent from step to step (sqrt(t) growth, as for the large
      configuration).  The largest of 1600 columns lies within 4.5 sigma.
    * Liquid fraction.  Equal error: the relative f_l error stays below a
      tenth of the discretization error of the same run, |f_l(40^3) -
      f_l(20^3)| / f_l at the same Fourier number (oracle), and never needs
      to be below the FP32 bar of 1e-6."""
    steps, n = 400, 40
    kw = dict(ra=1e5, pr=1.0, ste=0.5)
    orc, gpu = make_pair(steps, n=n, s0=11.2, precision=prec, **kw)
    d = diffs(orc, gpu)
    coarse = OracleSim(n // 2, s0=5.6, **kw)  # alpha halves: the same Fo in steps / 2
    coarse.step(steps // 2)
    fl = orc.liquid_fraction()
    disc = abs(coarse.liquid_fraction() - fl) / fl

    lat = gpu.lattice()
    alpha = lat["alpha"]
    sigma_T = unit_roundoff * np.sqrt(1.0 / 64 + 6.0 / 256)
    A = 6.0 + (8.0 * np.pi * alpha) ** -1.5 * 2.0 / np.sqrt(5.0)
    bar_T = 5.0 * sigma_T * np.sqrt(A)
    s = orc.s
    sx = np.gradient(s, axis=1)
    sz = np.gradient(s, axis=0)
    P = 1.0 + float((sx ** 2 + sz ** 2).max())
    K = alpha * kw["ste"] / 1.0
    bar_s = 4.5 * 4.33 * sigma_T * np.sqrt(A) * P * K * np.sqrt(steps)
    bar_fl = max(1e-6, 0.1 * disc)
    print(prec, d, {"bar_T": bar_T, "bar_s": bar_s, "bar_fl": bar_fl, "disc": disc, "P": P})
    assert d["mask"] == 0, d
    assert d["T"] <= bar_T, (d, bar_T)
    assert d["s"] <= bar_s, (d, bar_s)
    assert d["fl_rel"] <= bar_fl, (d, bar_fl)


def golden_path(name):
    from conftest import golden_path as gp
    return gp(name)


def _golden_conv64():
    import os
    path = golden_path("conv64_ra1e4_oracle.txt")
    if not os.path.exists(path) or not os.path.exists(golden_path("conv64_ra1e4_oracle_T.npy")):
        pytest.skip("golden file missing")
    fl, s, T, line = {}, {}, {}, {}
    for ln in open(path):
        if ln.startswith("#"):
            continue
        k, i, v = ln.split()
        {"fl": fl, "s": s, "T": T, "Tline": line}[k][int(i)] = float(v)
    return fl, s, T, line


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_convection_melting_64_full_run(prec):
    """The 64^3 convection-melting run (Ra = 1e4, Pr = 1, Ste = 0.1, 20000
    steps) against the FP64 oracle's stored trajectory.  FP64 storage: round
    off.  FP32 storage: max|dT| <= 1e-5 and relative liquid-fraction error
    <= 1e-6."""
    from paper_1604_03478_amd import Sim, presets
    fl, s, T, line = _golden_conv64()
    g = Sim(presets.conv64(prec).config)
    worst_fl = 0.0
    done = 0
    for st in sorted(fl):
        g.step(st - done)
        done = st
        worst_fl = max(worst_fl, abs(g.liquid_fraction() - fl[st]) / fl[st])
    F = g.fields()
    Tg = F["T"].reshape(-1)
    dT = max(abs(Tg[c] - v) for c, v in T.items())
    dline = max(abs(F["T"][32, y, 32] - v) for y, v in line.items())
    ds = max(abs(F["s"].reshape(-1)[c] - v) for c, v in s.items())
    # the whole final temperature field (written by the same script)
    T_full = np.load(golden_path("conv64_ra1e4_oracle_T.npy"), allow_pickle=False)
    dT_full = float(np.abs(F["T"] - T_full).max())
    res = {"fl_rel": worst_fl, "T": dT, "Tline": dline, "s": ds, "T_full": dT_full}
    print(prec, res)
    if prec == "f64":
        assert worst_fl <= 1e-12 and dT_full <= 1e-10 and ds <= 1e-10, res
    else:
        # FP32: the target tolerances on T and f_l; the front within 1e-5 cells
        assert worst_fl <= 1e-6 and dT_full <= 1e-5 and ds <= 1e-5, res
    assert dT <= dT_full and dline <= dT_full  # the sampled cells are part of the field


def _one_step_random(n, prec, seed, heating="y0", front=(0.0, None), flow=1, f_wall=0,
                     ste=2.0):
    """Hand the same seeded random state (rough front) to both sides, take
    one step, compare post-collision populations cell by cell."""
    from paper_1604_03478_amd import Config, Sim
    from inputs import random_state
    f, g, s = random_state(n, seed, flow=bool(flow), front=front)
    orc = OracleSim(n, ra=1e5, pr=1.0, ste=ste, s0=1.0, heating=HEAT[heating], flow=flow,
                    f_wall=f_wall)
    if flow:
        orc.f[:] = f
    orc.g[:] = g
    orc.s[:] = s
    gpu = Sim(Config(n=n, ra=1e5, pr=1.0, ste=ste, s0=1.0, heating=heating, flow=flow,
                     precision=prec, f_wall=f_wall))
    gpu.set_populations(f, g, s)
    del f, g
    orc.step(1)
    gpu.step(1)
    fg, gg, sg = gpu.get_populations()
    out = {"g": float(np.abs(gg - orc.g).max()), "s": float(np.abs(sg - orc.s).max())}
    if flow:
        a = np.arange(n) + 0.5
        if heating == "y0":
            liq = a[None, :, None] < orc.s[:, None, :]
        else:
            liq = a[:, None, None] < orc.s[None, :, :]
        out["f"] = float(np.abs(fg - orc.f)[:, liq].max())
        out["fscale"] = float(np.abs(orc.f[:, liq]).max())
    return out


# Bars of the one-step tests from a random state.  FP64: round-off.  FP32: a
# few ulps of the O(0.4) outputs.  FP16: the input rounding (half an ulp of
# values up to 0.4, 1e-4) carried through the collision, plus the output's
# stochastic rounding (under one ulp): 1e-3.  BF16 keeps 3 mantissa bits
# fewer than FP16 (unit round-off 2^-8 against 2^-11), so its bar is FP16's
# times 2^3.
ONE_STEP_TOL = {"f64": 1e-14, "f32": 2e-7, "f16s": 1e-3, "bf16s": 8e-3}
ONE_STEP_TOL_S = {"f64": 1e-12, "f32": 1e-6, "f16s": 1e-3, "bf16s": 8e-3}


@pytest.mark.parametrize("prec", ["f64", "f32", "f16s", "bf16s"])
@pytest.mark.parametrize("heating", ["y0", "z0"])
def test_one_step_random_state_128(prec, heating):
    """128^3: several workgroups of rows, the fast path and the general path
    near the front, one step from a random state.  FP64 gets a rough front
    (heights independent per column, many lateral interface links) and
    round-off bars.  The reduced precisions get a smooth front here: on a
    rough one the slope factor 1 + s_x^2 + s_z^2 of Eq. (6) reaches ~800 and
    amplifies any rounding of T into the front position (the rough front in
    reduced precision is covered with the front held fixed, below)."""
    front = (20.0, 60.0) if prec == "f64" else (40.0, 41.8)
    d = _one_step_random(128, prec, seed=7, heating=heating, front=front)
    tol = ONE_STEP_TOL[prec]
    assert d["g"] <= tol and d["f"] <= tol and d["s"] <= ONE_STEP_TOL_S[prec], d


@pytest.mark.parametrize("prec", ["f32", "f16s", "bf16s"])
@pytest.mark.parametrize("heating", ["y0", "z0"])
def test_one_step_random_rough_front_reduced_precision(prec, heating):
    """Reduced precisions on a rough front (independent heights per column
    in [20, 60]: every kind of lateral interface link, both branches of the
    interpolated anti-bounce-back), 128^3, the front held fixed (Ste = 0) so
    that the comparison is of the streamed and collided populations f and g
    themselves, at the bars above."""
    d = _one_step_random(128, prec, seed=5, heating=heating, front=(20.0, 60.0), ste=0.0)
    tol = ONE_STEP_TOL[prec]
    assert d["g"] <= tol and d["f"] <= tol and d["s"] == 0.0, d


@pytest.mark.parametrize("prec", ["f32", "f16s", "bf16s"])
def test_one_step_random_state_256(prec):
    """Full size, 256^3, in the launch configuration the benchmark times, one
    step from a random state, every cell (bars as at 128^3)."""
    d = _one_step_random(256, prec, seed=11, front=(100.0, 101.8))
    tol = ONE_STEP_TOL[prec]
    assert d["g"] <= tol and d["f"] <= tol, d
    assert d["s"] <= ONE_STEP_TOL_S[prec], d


@pytest.mark.parametrize("prec", ["f16s", "bf16s"])
@pytest.mark.parametrize("front", [(100.0, 101.8), (170.0, 171.8)], ids=["mostly_solid", "mostly_liquid"])
def test_one_step_random_state_264_two_workgroups_per_row(prec, front):
    """16-bit storage runs a row of up to 256 cells in one workgroup, so at
    264^3 every row takes two, the second with 8 live lanes.  The host picks
    the row order from the liquid fraction: above one half (front at ~0.65 n)
    both halves of a row go to one XCD, below it (~0.38 n) the halves are
    dispatched as separate row blocks.  Both orders, every cell, one step from
    a random state, at the one-step bars."""
    d = _one_step_random(264, prec, seed=13, heating="z0", front=front)
    tol = ONE_STEP_TOL[prec]
    assert d["g"] <= tol and d["f"] <= tol, d
    assert d["s"] <= ONE_STEP_TOL_S[prec], d


@pytest.mark.parametrize("prec,tol", [("f64", 1e-14), ("f32", 1e-7), ("f16s", 1e-3),
                                      ("bf16s", 8e-3)])
@pytest.mark.parametrize("heating", ["y0", "z0"])
def test_linear_field_through_a_tilted_front_is_a_fixed_point(prec, tol, heating):
    """The closed-form steady state of conduction in a linear temperature
    field that equals T_m on a tilted plane front (both phases, Ste = 0):
    one GPU step leaves every cell whose links stay off the adiabatic and
    far walls unchanged.  This pins the GPU's front condition of g, its
    link fractions across columns and along the melt axis and both
    interpolation branches, to the mathematics directly.  Bars: round-off
    (FP64); a few ulps of the stored values, below 0.3 (FP32); the one-step
    bars above for 16-bit storage."""
    from linear_field import T_M, fixed_point_state, interior
    from paper_1604_03478_amd import Config, Sim
    n = 40
    sim = Sim(Config(n=n, flow=0, ste=0.0, alpha=0.1, t_h=1.0, t_c=T_M, t_m=T_M, s0=1.0,
                     heating=heating, precision=prec))
    q_j = sim.lattice()["q_j"]
    from linear_field import E7, W7
    g, s, th = fixed_point_state(n, HEAT[heating], q_j, W7, E7)
    sim.set_populations(None, g, s)
    sim.set_hot_wall(th)
    sim.step(1)
    _, g1, s1 = sim.get_populations()
    sim.close()
    m = interior(n, HEAT[heating])
    err = float(np.abs(g1[:, m] - g[:, m]).max())
    assert np.array_equal(s1, s)
    assert err <= tol, err
