"""lbmmelt: MI355X-native double-MRT lattice Boltzmann melting step.

The method (Li, Yang & Zhang, arXiv:1604.03478, section 2) runs in the HIP
library ``liblbmmelt.so`` behind the C ABI of ``include/lbmmelt.h``; this
package holds its sources (``csrc/``), its build and a thin ctypes binding.
"""
from .binding import Config, LbmError, LiquidFraction, Sim, load_library  # noqa: F401
from . import presets  # noqa: F401
