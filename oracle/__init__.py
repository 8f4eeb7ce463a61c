"""FP64 CPU oracle for the double-MRT lattice Boltzmann melting step.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and
the CPU-baseline leg of the benchmark import this package.  The product
library (the HIP path behind the C ABI) never imports, links or calls it, and
it shares no code with that path.

The arithmetic lives in ``lbm_oracle.c`` (plain C, IEEE double); this package
builds and wraps it with ctypes and adds the closed-form Neumann solution used
to pin it (``neumann.py``).
"""
from .oracle import OracleSim, build_oracle, oracle_library_path  # noqa: F401
from . import neumann  # noqa: F401
