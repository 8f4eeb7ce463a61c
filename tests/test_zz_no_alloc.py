"""The allocation-free entry point lbm_diagnostics_noalloc against
lbm_diagnostics, through the C ABI: two calls in a row on two contexts, the
second with a smaller lattice, host and device outputs, and the sums against
host sums of the fields."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _run(n, steps, prec, heating):
    import torch
    from paper_1604_03478_amd import Config, Sim
    from paper_1604_03478_amd.binding import load_library
    lib = load_library()
    sim = Sim(Config(n=n, ra=1e5, pr=1.0, ste=1.0, s0=4.4, t_c=0.1, t_m=0.1,
                     heating=heating, precision=prec))
    sim.step(steps)
    ref = np.zeros(5)
    assert lib.lbm_diagnostics(sim._h, ref.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == 0
    out = np.full(5, np.nan)
    assert lib.lbm_diagnostics_noalloc(sim._h, out.ctypes.data_as(ctypes.c_void_p), 0) == 0
    dev = torch.full((5,), float("nan"), dtype=torch.float64, device="cuda")
    assert lib.lbm_diagnostics_noalloc(sim._h, ctypes.c_void_p(dev.data_ptr()), 1) == 0
    torch.cuda.synchronize()
    F = sim.fields(which=("T", "rho", "s"))
    sim.close()
    return ref, out, dev.cpu().numpy(), F


@pytest.mark.parametrize("first,second", [((40, 300, "f32", "y0"), (20, 200, "f64", "z0"))])
def test_noalloc_diagnostics_match_lbm_diagnostics(first, second):
    for n, steps, prec, heating in (first, second):
        ref, out, dev, F = _run(n, steps, prec, heating)
        assert ref[3] > 0  # cells melted, so every sum is exercised
        # the same reduction kernels: bit for bit
        assert np.array_equal(out, ref), (out, ref)
        assert np.array_equal(dev, ref), (dev, ref)
        # and the sums against host sums of the fields (FP64 round-off)
        assert abs(out[0] - F["rho"].sum()) <= 1e-12 * F["rho"].sum()
        assert abs(out[1] - (F["T"] - 0.1).sum()) <= 1e-12 * np.abs(F["T"] - 0.1).sum()
        assert abs(out[2] - F["s"].sum()) <= 1e-12 * F["s"].sum()
