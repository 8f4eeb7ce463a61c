"""ctypes wrapper around the FP64 C oracle (test infrastructure only).

The C source follows the paper's step order: pull-stream (Eq. (1) and Eq. (4)
left-hand sides), MRT collision of f (Eq. (2)) with the body force of Eq. (1),
MRT collision of g (Eq. (4)), then the interface velocity of Eq. (6) and the
phase switch.  This module only marshals arguments and exposes the state as
numpy views.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

from . import neumann

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def oracle_library_path() -> str:
    return _LIB


# gcc flags of the oracle: plain -O2, IEEE semantics (no fast-math, no
# contraction into fused multiply-adds), OpenMP over independent cells
CFLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
          "-std=c11"]


def compile_oracle(src: str, out: str, extra=()) -> str:
    """Compile an oracle source file into the shared library ``out``."""
    tmp = out + ".tmp"
    subprocess.run(["gcc", *CFLAGS, *extra, "-o", tmp, src, "-lm"], check=True)
    os.replace(tmp, out)
    return out


def build_oracle(force: bool = False) -> str:
    """Compile the oracle with gcc (CFLAGS)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        compile_oracle(_SRC, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int),
        ("ra", ctypes.c_double),
        ("pr", ctypes.c_double),
        ("ste", ctypes.c_double),
        ("t_h", ctypes.c_double),
        ("t_c", ctypes.c_double),
        ("t_m", ctypes.c_double),
        ("ma", ctypes.c_double),
        ("alpha_in", ctypes.c_double),
        ("s0", ctypes.c_double),
        ("heating", ctypes.c_int),
        ("flow", ctypes.c_int),
        ("seed_profile", ctypes.c_int),
        ("seed_lambda", ctypes.c_double),
        ("periodic", ctypes.c_int),
        ("ks_kl", ctypes.c_double),
        ("front_scheme", ctypes.c_int),
        ("f_wall", ctypes.c_int),
        ("body_fx", ctypes.c_double),
    ]


_libs = {}


def _load(path=None):
    """The oracle library (ctypes handle), loaded once per path.  ``path``
    names another build of the oracle source, for the tests that plant a
    mistake in a copy of it and check that a pin catches the mistake."""
    key = path or _LIB
    if key not in _libs:
        if path is None and not os.path.exists(_LIB):
            build_oracle()
        lib = ctypes.CDLL(key)
        P = ctypes.POINTER
        d, i, ll, vp = ctypes.c_double, ctypes.c_int, ctypes.c_longlong, ctypes.c_void_p
        dp = P(d)
        ip = P(i)
        lib.orc_sizeof_params.restype = i
        lib.orc_create.argtypes = [P(_Params)]
        lib.orc_create.restype = vp
        lib.orc_destroy.argtypes = [vp]
        lib.orc_step.argtypes = [vp, ll]
        lib.orc_liquid_fraction.argtypes = [vp]
        lib.orc_liquid_fraction.restype = d
        lib.orc_fields.argtypes = [vp, dp, dp, dp, dp, dp]
        lib.orc_front_velocity.argtypes = [vp, dp]
        for name in ("orc_f", "orc_g", "orc_s", "orc_th"):
            getattr(lib, name).argtypes = [vp]
            getattr(lib, name).restype = dp
        for name in ("orc_steps", "orc_melted", "orc_frozen"):
            getattr(lib, name).argtypes = [vp]
            getattr(lib, name).restype = ll
        lib.orc_derived.argtypes = [vp, dp]
        lib.orc_tables.argtypes = [vp, ip, ip, dp, dp, ip, ip, dp, dp, dp, dp, dp, dp]
        lib.orc_collide_f_cell.argtypes = [vp, dp, d, dp]
        lib.orc_set_rates.argtypes = [vp, dp, dp]
        lib.orc_equilibrium_moments.argtypes = [d, d, d, d, d, d, d, d, dp, dp]
        lib.orc_guo_force.argtypes = [vp, d, d, d, d, d, d, dp]
        lib.orc_record.argtypes = [vp, ll]
        lib.orc_adjoint.argtypes = [vp, dp, dp, dp, dp]
        lib.orc_wall_nusselt.argtypes = [vp, dp]
        for name in ("orc_link_fraction19", "orc_link_fraction7"):
            getattr(lib, name).argtypes = [vp, i, i, i, i]
            getattr(lib, name).restype = d
        lib.orc_energy.argtypes = [vp]
        lib.orc_energy.restype = d
        lib.orc_wall_heat.argtypes = [vp]
        lib.orc_wall_heat.restype = d
        lib.orc_threads.restype = i
        lib.orc_set_threads.argtypes = [i]
        assert lib.orc_sizeof_params() == ctypes.sizeof(_Params), "oracle params layout mismatch"
        _libs[key] = lib
    return _libs[key]


def threads() -> int:
    """OpenMP threads the oracle's cell loop uses."""
    return int(_load().orc_threads())


def set_threads(k: int) -> None:
    _load().orc_set_threads(int(k))


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


@dataclass
class Derived:
    nu: float
    alpha: float
    s_nu: float
    q_j: float
    q_e: float
    gbeta: float
    t0: float
    latent: float
    u0: float


class OracleSim:
    """One FP64 oracle simulation.

    Parameters mirror the problem statement of the paper's section 1: cube of
    edge ``n`` lattice units, hot wall at ``t_h``, cold wall at ``t_c``,
    melting temperature ``t_m``, and the dimensionless groups ``ra``, ``pr``,
    ``ste``.  ``heating`` 0 puts the hot wall at y=0 and the cold wall at y=n;
    1 puts it at z=0 with every other wall adiabatic.  ``flow`` 0 freezes the
    flow (energy distribution only).  ``f_wall`` 0 bounces f back halfway at
    the front, 1 interpolates the bounce-back to where the front cuts each
    link.  ``periodic`` selects a test mode: 1 (or True) a periodic box, all
    liquid, no walls and no front; 2 a channel, periodic across the two
    lateral axes, with the walls and a frozen front along the melt axis and
    the uniform force ``body_fx`` along x in place of the buoyancy.
    """

    def __init__(self, n, ra=1e4, pr=1.0, ste=0.1, t_h=1.0, t_c=0.0, t_m=0.0,
                 ma=0.1, alpha=0.1, s0=1.0, heating=0, flow=1, seed_profile=0,
                 periodic=False, ks_kl=1.0, front_scheme=0, f_wall=0, body_fx=0.0,
                 library=None):
        lib = _load(library)
        lam = 0.0
        if seed_profile == 1 and ste > 0:
            lam = neumann.stefan_lambda(ste)
        elif seed_profile == 2 and ste > 0:  # subcooled solid (two phases)
            lam = neumann.two_phase_lambda(ste, ste * (t_m - t_c) / (t_h - t_m), ks_kl)
        self.params = _Params(int(n), float(ra), float(pr), float(ste), float(t_h),
                              float(t_c), float(t_m), float(ma), float(alpha), float(s0),
                              int(heating), int(flow), int(seed_profile), float(lam),
                              int(periodic), float(ks_kl), int(front_scheme), int(f_wall),
                              float(body_fx))
        h = lib.orc_create(ctypes.byref(self.params))
        if not h:
            raise MemoryError("oracle allocation failed")
        self._h = h
        self._lib = lib
        self.n = int(n)
        self.ncell = self.n ** 3

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_destroy(h)
            self._h = None

    # ---- state views (re-fetched each time: the step swaps buffers) ----
    def _view(self, fn, count, shape):
        ptr = fn(self._h)
        return np.ctypeslib.as_array(ptr, shape=(count,)).reshape(shape)

    @property
    def f(self) -> np.ndarray:
        n = self.n
        return self._view(self._lib.orc_f, 19 * n ** 3, (19, n, n, n))

    @property
    def g(self) -> np.ndarray:
        n = self.n
        return self._view(self._lib.orc_g, 7 * n ** 3, (7, n, n, n))

    @property
    def s(self) -> np.ndarray:
        n = self.n
        return self._view(self._lib.orc_s, n * n, (n, n))

    @property
    def th(self) -> np.ndarray:
        n = self.n
        return self._view(self._lib.orc_th, n * n, (n, n))

    # ---- stepping and outputs ----
    def step(self, nsteps: int = 1) -> None:
        self._lib.orc_step(self._h, int(nsteps))

    @property
    def steps(self) -> int:
        return int(self._lib.orc_steps(self._h))

    @property
    def melted(self) -> int:
        return int(self._lib.orc_melted(self._h))

    def liquid_fraction(self) -> float:
        return float(self._lib.orc_liquid_fraction(self._h))

    def fields(self):
        n = self.n
        out = [np.zeros((n, n, n)) for _ in range(5)]
        self._lib.orc_fields(self._h, *[_dp(a) for a in out])
        T, ux, uy, uz, rho = out
        return {"T": T, "u": np.stack([ux, uy, uz]), "rho": rho, "s": self.s.copy()}

    def link_fraction19(self, x: int, y: int, z: int, q: int) -> float:
        """Fraction at which the front cuts the link from cell (x, y, z) to the
        source of its incoming D3Q19 direction q."""
        return float(self._lib.orc_link_fraction19(self._h, int(x), int(y), int(z), int(q)))

    def link_fraction7(self, x: int, y: int, z: int, q: int) -> float:
        """Fraction at which the front cuts the link from cell (x, y, z) to the
        source of its incoming D3Q7 direction q (the front condition of g)."""
        return float(self._lib.orc_link_fraction7(self._h, int(x), int(y), int(z), int(q)))

    def front_velocity(self) -> np.ndarray:
        V = np.zeros((self.n, self.n))
        self._lib.orc_front_velocity(self._h, _dp(V))
        return V

    def energy(self) -> float:
        """Sum of T over the cells plus L times the sum of the fronts."""
        return float(self._lib.orc_energy(self._h))

    def wall_heat(self) -> float:
        """Heat let in through the walls so far (front scheme 1 only)."""
        return float(self._lib.orc_wall_heat(self._h))

    def wall_nusselt(self) -> np.ndarray:
        """Local Nusselt number on the heated wall, per column (n x n)."""
        out = np.zeros((self.n, self.n))
        self._lib.orc_wall_nusselt(self._h, _dp(out))
        return out

    def derived(self) -> Derived:
        out = np.zeros(9)
        self._lib.orc_derived(self._h, _dp(out))
        return Derived(*[float(v) for v in out])

    def tables(self) -> dict:
        e19 = np.zeros((19, 3), dtype=np.int32)
        e7 = np.zeros((7, 3), dtype=np.int32)
        w19 = np.zeros(19)
        w7 = np.zeros(7)
        o19 = np.zeros(19, dtype=np.int32)
        o7 = np.zeros(7, dtype=np.int32)
        M = np.zeros((19, 19))
        Minv = np.zeros((19, 19))
        N = np.zeros((7, 7))
        Ninv = np.zeros((7, 7))
        S = np.zeros(19)
        Q = np.zeros(7)
        self._lib.orc_tables(self._h, _ip(e19), _ip(e7), _dp(w19), _dp(w7), _ip(o19),
                             _ip(o7), _dp(M), _dp(Minv), _dp(N), _dp(Ninv), _dp(S), _dp(Q))
        return dict(e19=e19, e7=e7, w19=w19, w7=w7, opp19=o19, opp7=o7, M=M, Minv=Minv,
                    N=N, Ninv=Ninv, S=S, Q=Q)

    def collide_f_cell(self, fin, T: float) -> np.ndarray:
        fin = np.ascontiguousarray(fin, dtype=np.float64)
        out = np.zeros(19)
        self._lib.orc_collide_f_cell(self._h, _dp(fin), float(T), _dp(out))
        return out

    def set_rates(self, S=None, Q=None) -> None:
        Sa = None if S is None else np.ascontiguousarray(S, dtype=np.float64)
        Qa = None if Q is None else np.ascontiguousarray(Q, dtype=np.float64)
        self._lib.orc_set_rates(self._h, None if Sa is None else _dp(Sa),
                                None if Qa is None else _dp(Qa))

    def guo_force(self, u, F) -> np.ndarray:
        out = np.zeros(19)
        self._lib.orc_guo_force(self._h, *[float(v) for v in u], *[float(v) for v in F],
                                _dp(out))
        return out

    # ---- reference adjoint ----
    def record(self, nsteps: int) -> None:
        """Step forward keeping every state (for the reverse sweep)."""
        rc = self._lib.orc_record(self._h, int(nsteps))
        if rc == -2:
            raise ValueError("the reference adjoint follows the cavity's walls (not the "
                             "channel test mode)")
        if rc != 0:
            raise MemoryError("oracle record allocation failed")

    def adjoint(self, lf=None, lg=None, ls=None):
        """Reverse sweep over the recorded run.  (lf, lg, ls): adjoint of the
        final state (default: that of the liquid fraction, ls = 1/n^3).
        Returns (lf0, lg0, ls0, lth): adjoint of the recorded initial state
        and the gradient with respect to the hot-wall temperatures."""
        n = self.n
        lf = np.zeros((19, n, n, n)) if lf is None else np.array(lf, dtype=np.float64)
        lg = np.zeros((7, n, n, n)) if lg is None else np.array(lg, dtype=np.float64)
        ls = np.full((n, n), 1.0 / n ** 3) if ls is None else np.array(ls, dtype=np.float64)
        lth = np.zeros((n, n))
        if self._lib.orc_adjoint(self._h, _dp(lf), _dp(lg), _dp(ls), _dp(lth)) != 0:
            raise RuntimeError("no recorded run")
        return lf, lg, ls, lth

    @staticmethod
    def equilibrium_moments(rho, j, T, u):
        lib = _load()
        m = np.zeros(19)
        nn = np.zeros(7)
        lib.orc_equilibrium_moments(float(rho), *[float(v) for v in j], float(T),
                                    *[float(v) for v in u], _dp(m), _dp(nn))
        return m, nn
