"""Graph replays of the step loop (lbm_set_graph) against kernel-by-kernel
launches, through the C ABI on the GPU.

The two must give the same state bit for bit: the replayed kernels are the
launched ones, and the step that seeds the stochastic rounding of FP32 and
16-bit storage comes from a device counter that the replays advance.  The
runs cross chunk boundaries, take odd remainders (which flip the buffer
parity, so the next chunk captures a graph from the other parity), query the
state between replays, switch the setting off and on, and pass the step at
which the first layer of cells melts (about step 70), so a phase switch and
the refill of f happen inside a replayed chunk."""
import numpy as np
import pytest

from live_state import states_equal

pytestmark = pytest.mark.gpu

CASES = [  # precision, heating, front_scheme, f_wall
    ("f64", "y0", 0, 0),
    ("f32", "y0", 0, 0),
    ("f32", "z0", 1, 1),
    ("f16s", "y0", 0, 0),
    ("f16s", "z0", 1, 0),
    ("bf16s", "y0", 0, 1),
]

# step() calls: with chunks of 8, 16 = 2 replays; 7 eager; 33 = 4 replays
# from the other parity + 1 eager; 1 eager; 8 = 1 replay; 40 = 5 replays
CALLS = [16, 7, 33, 1, 8, 40]


def _cfg(prec, heating, scheme, fwall):
    from paper_1604_03478_amd import Config
    return Config(n=40, ra=1e5, pr=1.0, ste=1.0, s0=4.4, t_c=0.1, t_m=0.1, heating=heating,
                  precision=prec, front_scheme=scheme, f_wall=fwall)


def _state(sim):
    return sim.get_populations()


@pytest.mark.parametrize("prec,heating,scheme,fwall", CASES)
def test_graph_replays_match_launches(prec, heating, scheme, fwall):
    from paper_1604_03478_amd import Sim
    cfg = _cfg(prec, heating, scheme, fwall)
    a = Sim(cfg)
    b = Sim(cfg)
    b.set_graph(8)
    for i, k in enumerate(CALLS):
        a.step(k)
        b.step(k)
        if i % 2:  # eager work and a synchronization between replays
            assert a.liquid_fraction() == b.liquid_fraction()
    assert a.steps == b.steps == sum(CALLS)
    assert b.diagnostics()["melted"] > 0  # cells melted inside the replayed run
    assert states_equal(_state(a), _state(b), heating)

    # off, then kernel timing (which launches one by one), then another chunk
    b.set_graph(0)
    a.step(10)
    b.step(10)
    b.set_graph(4)
    b.kernel_timing(True)
    a.step(8)
    b.step(8)
    ms, launches = b.kernel_time()
    assert launches == 8 and ms > 0
    b.kernel_timing(False)
    a.step(13)
    b.step(13)
    assert a.steps == b.steps
    assert a.liquid_fraction() == b.liquid_fraction()
    assert states_equal(_state(a), _state(b), heating)
    a.close()
    b.close()


def test_graph_on_a_caller_stream_and_after_load_state():
    """A context on a torch side stream replays on that stream; a saved
    state reloaded under an existing graph continues exactly as a fresh
    eager run from the same blob."""
    import torch
    from paper_1604_03478_amd import Sim
    cfg = _cfg("f16s", "y0", 0, 0)
    side = torch.cuda.Stream()
    a = Sim(cfg)
    b = Sim(cfg, stream=side)
    b.set_graph(6)
    a.step(30)
    b.step(30)
    assert states_equal(_state(a), _state(b), "y0")
    blob = a.save_state()
    a.step(50)
    b.load_state(blob)  # same parity as the graph was captured at
    b.step(50)
    assert b.steps == a.steps == 80
    assert states_equal(_state(a), _state(b), "y0")
    a.close()
    b.close()


def test_set_graph_rejects_bad_chunks():
    from paper_1604_03478_amd import LbmError, Sim
    from paper_1604_03478_amd.binding import LBM_EINVAL
    sim = Sim(_cfg("f32", "y0", 0, 0))
    for bad in (-2, 3, 4098):
        with pytest.raises(LbmError) as e:
            sim.set_graph(bad)
        assert e.value.code == LBM_EINVAL
    sim.set_graph(2)
    sim.step(5)
    assert sim.steps == 5
    sim.close()


def test_graph_setting_leaves_the_adjoint_unchanged():
    """lbm_forward_ckpt records every step and lbm_adjoint recomputes them,
    so both launch kernel by kernel whatever the graph setting; steps taken
    as replays before the recorded run reach the same state.  The gradient
    and the liquid fraction equal a context's without graphs bit for bit.
    The recorded run hands the context's population buffers to its
    checkpoints, so the replays after it capture a new graph: the states
    stay equal through them, and through a second recorded run."""
    from inputs import hot_wall_field
    from paper_1604_03478_amd import Sim
    cfg = _cfg("f32", "y0", 0, 0)
    out, sims = [], []
    for chunk in (0, 6):
        sim = Sim(cfg)
        sim.set_graph(chunk)
        sim.set_hot_wall(hot_wall_field(cfg.n, seed=2))
        sim.step(48)
        fl = sim.forward_ckpt(30, 7)
        out.append((fl, sim.adjoint(1.0)))
        sims.append(sim)
    assert out[0][0] == out[1][0]
    assert np.array_equal(out[0][1], out[1][1])
    assert np.linalg.norm(out[0][1]) > 0
    a, b = sims
    for k in (24, 13):
        a.step(k)
        b.step(k)
        assert states_equal(_state(a), _state(b), "y0")
    fa, fb = a.forward_ckpt(12, 5), b.forward_ckpt(12, 5)
    assert fa == fb
    assert np.array_equal(a.adjoint(1.0), b.adjoint(1.0))
    a.step(18)
    b.step(18)
    assert a.steps == b.steps
    assert states_equal(_state(a), _state(b), "y0")
    a.close()
    b.close()


def test_graph_follows_the_row_order_the_liquid_fraction_picks():
    """16-bit storage at 264^3 runs every row in two workgroups, and the host
    picks their order from the last known liquid fraction (both halves of a
    row on one XCD above one half, separate row blocks below).  A context with
    graphs captures in the order of its state, and a state handed over with
    the fraction on the other side of one half is replayed in the other order:
    the same states bit for bit as kernel-by-kernel launches throughout."""
    from inputs import random_state
    from paper_1604_03478_amd import Config, Sim
    n = 264
    cfg = Config(n=n, ra=1e5, pr=1.0, ste=0.1, s0=200.0, heating="z0", precision="f16s")
    a = Sim(cfg)
    b = Sim(cfg)
    b.set_graph(4)
    a.step(9)  # mostly liquid (f_l 0.76): paired order, two replays and one launch
    b.step(9)
    assert states_equal(_state(a), _state(b), "z0")
    for seed, front in ((3, (100.0, 101.8)), (4, (190.0, 191.8))):  # f_l 0.38, then 0.72
        f, g, s = random_state(n, seed, front=front)
        a.set_populations(f, g, s)
        b.set_populations(f, g, s)
        del f, g, s
        a.step(8)
        b.step(8)
        assert a.steps == b.steps
        assert states_equal(_state(a), _state(b), "z0")
    a.close()
    b.close()
