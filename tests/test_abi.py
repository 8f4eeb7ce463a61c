"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function the public header declares, and rejects invalid parameters
before it touches a device."""
import ctypes
import os
import re

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "lbmmelt.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", text)))


def test_header_declares_the_four_core_entry_points():
    names = _declared()
    for core in ("lbm_init", "lbm_step", "lbm_liquid_fraction", "lbm_fields"):
        assert core in names


def test_library_exports_every_declared_symbol():
    from paper_1604_03478_amd.binding import EXPORTS, load_library
    lib = load_library()
    for name in _declared():
        assert hasattr(lib, name), name
    assert sorted(EXPORTS) == _declared()


def _params(**kw):
    from paper_1604_03478_amd.binding import Config
    base = dict(n=16, ra=1e4, pr=1.0, ste=0.1, t_h=1.0, t_c=0.0, t_m=0.0, ma=0.1, alpha=0.1,
                s0=1.0, heating="y0", flow=1, precision="f32", seed_profile=0)
    base.update(kw)
    return Config(**base).to_c()


@pytest.mark.parametrize("bad", [
    dict(n=3), dict(n=2000), dict(ma=0.3), dict(ma=0.0), dict(t_c=0.5), dict(t_h=0.0),
    dict(ste=-1.0), dict(s0=17.0), dict(s0=-0.1), dict(ra=0.0), dict(pr=-1.0),
    dict(flow=0, alpha=0.0), dict(seed_profile=1, ste=0.0), dict(seed_profile=2, ste=0.0), dict(seed_profile=3), dict(ks_kl=-1.0), dict(front_scheme=2), dict(f_wall=2), dict(n=1024, precision="f64"),
    dict(ra=1e12),  # viscous relaxation time too close to 1/2
])
def test_invalid_parameters_are_rejected(bad):
    from paper_1604_03478_amd.binding import LBM_EINVAL, load_library
    lib = load_library()
    p = _params(**bad)
    h = ctypes.c_void_p()
    rc = lib.lbm_init(ctypes.byref(p), None, ctypes.byref(h))
    assert rc == LBM_EINVAL
    assert not h.value
    assert len(lib.lbm_last_error()) > 0


def test_null_arguments_are_rejected():
    from paper_1604_03478_amd.binding import LBM_EINVAL, load_library
    lib = load_library()
    assert lib.lbm_init(None, None, None) == LBM_EINVAL
    assert lib.lbm_step(None, 1) == LBM_EINVAL
    v = ctypes.c_double()
    assert lib.lbm_liquid_fraction(None, ctypes.byref(v)) == LBM_EINVAL
    assert lib.lbm_fields(None, None, None, None, None) == LBM_EINVAL
    assert lib.lbm_get_schedule(None, None, 0) == LBM_EINVAL
    assert lib.lbm_step_replay(None, None, 1) == LBM_EINVAL
    assert lib.lbm_wall_nusselt(None, None) == LBM_EINVAL
    lib.lbm_destroy(None)


def test_bandwidth_ceiling_rejects_invalid_arguments():
    from paper_1604_03478_amd.binding import LBM_EINVAL, load_library
    lib = load_library()
    ms, nb = ctypes.c_double(), ctypes.c_double()
    args = (ctypes.byref(ms), ctypes.byref(nb))
    assert lib.lbm_bandwidth_ceiling(2, 64, 1, 1, 1, None, *args) == LBM_EINVAL
    assert lib.lbm_bandwidth_ceiling(0, 3, 1, 1, 1, None, *args) == LBM_EINVAL
    assert lib.lbm_bandwidth_ceiling(1, 64, 4, 1, 1, None, *args) == LBM_EINVAL
    assert lib.lbm_bandwidth_ceiling(1, 64, 1, 2, 1, None, *args) == LBM_EINVAL
    assert lib.lbm_bandwidth_ceiling(1, 64, 1, 1, 0, None, *args) == LBM_EINVAL
    assert lib.lbm_bandwidth_ceiling(1, 64, 1, 1, 1, None, None, None) == LBM_EINVAL
