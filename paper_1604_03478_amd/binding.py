"""Python binding of liblbmmelt (the C ABI in include/lbmmelt.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  PyTorch supplies the HIP stream (and device memory where a
caller hands over tensors); it is imported before the library is loaded so
that both use the same HIP runtime.  There is no CPU fallback: a missing
library or a missing GPU is an error.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch  # noqa: F401  (must precede loading the library: one HIP runtime)

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblbmmelt.so")

PRECISIONS = {"f64": 0, "f32": 1, "f16s": 2, "bf16s": 3}
HEATING = {"y0": 0, "z0": 1}

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_EUNSTABLE, LBM_ESTATE = 0, -1, -2, -3, -4, -5
_STATUS = {LBM_EINVAL: "EINVAL", LBM_ENOMEM: "ENOMEM", LBM_EDEVICE: "EDEVICE",
           LBM_EUNSTABLE: "EUNSTABLE", LBM_ESTATE: "ESTATE"}


class LbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lbmmelt {_STATUS.get(code, code)}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("ra", ctypes.c_double),
        ("pr", ctypes.c_double),
        ("ste", ctypes.c_double),
        ("t_h", ctypes.c_double),
        ("t_c", ctypes.c_double),
        ("t_m", ctypes.c_double),
        ("ma", ctypes.c_double),
        ("alpha", ctypes.c_double),
        ("s0", ctypes.c_double),
        ("heating", ctypes.c_int32),
        ("flow", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("seed_profile", ctypes.c_int32),
        ("ks_kl", ctypes.c_double),
        ("front_scheme", ctypes.c_int32),
        ("f_wall", ctypes.c_int32),
    ]


class Lattice(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in
                ("u0", "nu", "alpha", "gbeta", "t0", "s_nu", "q_j", "q_e")]


EXPORTS = ("lbm_init", "lbm_destroy", "lbm_step", "lbm_liquid_fraction", "lbm_fields",
           "lbm_get_lattice", "lbm_get_step", "lbm_set_hot_wall", "lbm_set_populations",
           "lbm_get_populations", "lbm_diagnostics", "lbm_save_state", "lbm_load_state",
           "lbm_forward_ckpt", "lbm_adjoint", "lbm_get_schedule", "lbm_step_replay",
           "lbm_wall_nusselt", "lbm_kernel_timing", "lbm_kernel_time",
           "lbm_bandwidth_ceiling", "lbm_diagnostics_noalloc", "lbm_set_graph",
           "lbm_last_error")

_lib = None


def load_library(path: str = LIB_PATH):
    """Load liblbmmelt.so and declare its signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run __graft_entry__.build() first")
    lib = ctypes.CDLL(path)
    vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
    lib.lbm_init.argtypes = [ctypes.POINTER(Params), vp, ctypes.POINTER(vp)]
    lib.lbm_destroy.argtypes = [vp]
    lib.lbm_destroy.restype = None
    lib.lbm_step.argtypes = [vp, i64]
    lib.lbm_liquid_fraction.argtypes = [vp, dp]
    lib.lbm_fields.argtypes = [vp, vp, vp, vp, vp]
    lib.lbm_get_lattice.argtypes = [vp, ctypes.POINTER(Lattice)]
    lib.lbm_get_step.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    lib.lbm_set_hot_wall.argtypes = [vp, vp, i32]
    lib.lbm_set_populations.argtypes = [vp, vp, vp, vp]
    lib.lbm_get_populations.argtypes = [vp, vp, vp, vp]
    lib.lbm_diagnostics.argtypes = [vp, dp]
    lib.lbm_save_state.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_size_t)]
    lib.lbm_load_state.argtypes = [vp, vp, ctypes.c_size_t]
    lib.lbm_forward_ckpt.argtypes = [vp, i64, ctypes.c_int32, dp]
    lib.lbm_adjoint.argtypes = [vp, ctypes.c_double, vp, i32]
    lib.lbm_get_schedule.argtypes = [vp, vp, ctypes.c_size_t]
    lib.lbm_wall_nusselt.argtypes = [vp, dp]
    lib.lbm_step_replay.argtypes = [vp, vp, i64]
    lib.lbm_kernel_timing.argtypes = [vp, i32]
    lib.lbm_kernel_time.argtypes = [vp, dp, ctypes.POINTER(ctypes.c_int64)]
    lib.lbm_bandwidth_ceiling.argtypes = [i32, i32, i32, i32, i32, vp, dp, dp]
    lib.lbm_diagnostics_noalloc.argtypes = [vp, vp, i32]
    lib.lbm_set_graph.argtypes = [vp, i32]
    lib.lbm_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("lbm_destroy", "lbm_last_error"):
            getattr(lib, name).restype = i32
    _lib = lib
    return lib


def _check(rc: int):
    if rc != LBM_OK:
        raise LbmError(rc, load_library().lbm_last_error().decode())


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Config:
    n: int
    ra: float = 1e4
    pr: float = 1.0
    ste: float = 0.1
    t_h: float = 1.0
    t_c: float = 0.0
    t_m: float = 0.0
    ma: float = 0.1
    alpha: float = 0.1
    s0: float = 1.0
    heating: str = "y0"
    flow: int = 1
    precision: str = "f32"
    seed_profile: int = 0
    ks_kl: float = 1.0
    front_scheme: int = 0
    f_wall: int = 0

    def to_c(self) -> Params:
        return Params(int(self.n), float(self.ra), float(self.pr), float(self.ste),
                      float(self.t_h), float(self.t_c), float(self.t_m), float(self.ma),
                      float(self.alpha), float(self.s0), HEATING[self.heating], int(self.flow),
                      PRECISIONS[self.precision], int(self.seed_profile), float(self.ks_kl),
                      int(self.front_scheme), int(self.f_wall))


class Sim:
    """One simulation context on the current HIP device.

    ``stream``: a ``torch.cuda.Stream`` to enqueue on (default: torch's
    current stream of the current device).
    """

    def __init__(self, cfg: Config | None = None, stream=None, **kw):
        if cfg is None:
            cfg = Config(**kw)
        if not torch.cuda.is_available():
            raise RuntimeError("lbmmelt needs a HIP GPU; none is visible")
        self.cfg = cfg
        self._lib = load_library()
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self._params = cfg.to_c()
        h = ctypes.c_void_p()
        _check(self._lib.lbm_init(ctypes.byref(self._params), ctypes.c_void_p(stream.cuda_stream),
                                  ctypes.byref(h)))
        self._h = h
        self.n = cfg.n

    def close(self):
        if getattr(self, "_h", None):
            self._lib.lbm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- stepping ----
    def step(self, nsteps: int = 1) -> None:
        _check(self._lib.lbm_step(self._h, int(nsteps)))

    @property
    def steps(self) -> int:
        v = ctypes.c_int64()
        _check(self._lib.lbm_get_step(self._h, ctypes.byref(v)))
        return v.value

    def lattice(self) -> dict:
        L = Lattice()
        _check(self._lib.lbm_get_lattice(self._h, ctypes.byref(L)))
        return {k: getattr(L, k) for k, _ in Lattice._fields_}

    # ---- outputs ----
    def liquid_fraction(self) -> float:
        v = ctypes.c_double()
        _check(self._lib.lbm_liquid_fraction(self._h, ctypes.byref(v)))
        return v.value

    def fields(self, which=("T", "u", "rho", "s")) -> dict:
        """Macroscopic fields in FP64 (host); `which` selects the outputs."""
        n = self.n
        T = np.empty((n, n, n)) if "T" in which else None
        u = np.empty((3, n, n, n)) if "u" in which else None
        rho = np.empty((n, n, n)) if "rho" in which else None
        s = np.empty((n, n)) if "s" in which else None
        _check(self._lib.lbm_fields(self._h, _ptr(T), _ptr(u), _ptr(rho), _ptr(s)))
        out = {"T": T, "u": u, "rho": rho, "s": s}
        return {k: v for k, v in out.items() if v is not None}

    def wall_nusselt(self) -> np.ndarray:
        """Local Nusselt number on the heated wall, per column (n x n)."""
        out = np.empty((self.n, self.n))
        _check(self._lib.lbm_wall_nusselt(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def diagnostics(self) -> dict:
        out = np.zeros(5)
        _check(self._lib.lbm_diagnostics(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return {"mass": out[0], "energy": out[1], "front_sum": out[2], "melted": int(out[3]),
                "frozen": int(out[4])}

    def diagnostics_noalloc(self, device: bool = False):
        """lbm_diagnostics through the allocation-free entry point: a dict as
        diagnostics(), or (device=True) the 5 values in an FP64 tensor on the
        current device (enqueued on the context stream, not synchronized)."""
        if device:
            out = torch.empty(5, dtype=torch.float64,
                              device=torch.device("cuda", torch.cuda.current_device()))
            _check(self._lib.lbm_diagnostics_noalloc(self._h, ctypes.c_void_p(out.data_ptr()), 1))
            return out
        out = np.zeros(5)
        _check(self._lib.lbm_diagnostics_noalloc(self._h, _ptr(out), 0))
        return {"mass": out[0], "energy": out[1], "front_sum": out[2], "melted": int(out[3]),
                "frozen": int(out[4])}

    # ---- reverse mode ----
    def forward_ckpt(self, nsteps: int, every_k: int) -> float:
        """Run nsteps keeping a checkpoint every every_k steps; returns f_l."""
        fl = ctypes.c_double()
        _check(self._lib.lbm_forward_ckpt(self._h, int(nsteps), int(every_k), ctypes.byref(fl)))
        return fl.value

    def adjoint(self, dJ_dfl: float = 1.0, device: bool = False):
        """dJ/dT_h (n x n) for J = dJ_dfl * f_l of the last forward_ckpt run:
        a numpy array, or an FP64 torch tensor on the current device."""
        n = self.n
        if device:
            out = torch.empty((n, n), dtype=torch.float64,
                              device=torch.device("cuda", torch.cuda.current_device()))
            _check(self._lib.lbm_adjoint(self._h, float(dJ_dfl), ctypes.c_void_p(out.data_ptr()), 1))
            return out
        out = np.empty((n, n))
        _check(self._lib.lbm_adjoint(self._h, float(dJ_dfl), _ptr(out), 0))
        return out

    def schedule(self, nsteps: int) -> np.ndarray:
        """Schedule of the last forward_ckpt run of nsteps steps."""
        out = np.empty((nsteps + 1) * 3 * self.n * self.n, dtype=np.int32)
        _check(self._lib.lbm_get_schedule(self._h, _ptr(out), out.size))
        return out

    def step_replay(self, schedule: np.ndarray, nsteps: int) -> None:
        a = np.ascontiguousarray(schedule, dtype=np.int32)
        if a.size < (nsteps + 1) * 3 * self.n * self.n:
            raise ValueError("schedule too short")
        _check(self._lib.lbm_step_replay(self._h, _ptr(a), int(nsteps)))

    # ---- measurement ----
    def kernel_timing(self, enable: bool) -> None:
        _check(self._lib.lbm_kernel_timing(self._h, int(bool(enable))))

    def set_graph(self, steps: int) -> None:
        """Run step() in chunks of `steps` (even; 0: off) as HIP graph replays."""
        _check(self._lib.lbm_set_graph(self._h, int(steps)))

    def kernel_time(self):
        """(summed milliseconds, launches) of the timed stream-collide kernels."""
        ms = ctypes.c_double()
        k = ctypes.c_int64()
        _check(self._lib.lbm_kernel_time(self._h, ctypes.byref(ms), ctypes.byref(k)))
        return ms.value, k.value

    # ---- state ----
    def set_hot_wall(self, th) -> None:
        n = self.n
        if isinstance(th, torch.Tensor):
            t = th.detach().to(device=torch.device("cuda", torch.cuda.current_device()),
                               dtype=torch.float64).contiguous()
            if t.numel() != n * n:
                raise ValueError("hot-wall field must have n*n values")
            _check(self._lib.lbm_set_hot_wall(self._h, ctypes.c_void_p(t.data_ptr()), 1))
            self._th_keepalive = t  # the copy is enqueued on the stream
        else:
            a = np.ascontiguousarray(th, dtype=np.float64)
            if a.size != n * n:
                raise ValueError("hot-wall field must have n*n values")
            _check(self._lib.lbm_set_hot_wall(self._h, _ptr(a), 0))

    def set_populations(self, f, g, s) -> None:
        fa = None if f is None else np.ascontiguousarray(f, dtype=np.float64)
        ga = np.ascontiguousarray(g, dtype=np.float64)
        sa = np.ascontiguousarray(s, dtype=np.float64)
        _check(self._lib.lbm_set_populations(self._h, _ptr(fa), _ptr(ga), _ptr(sa)))

    def get_populations(self):
        n = self.n
        f = np.empty((19, n, n, n)) if self.cfg.flow else None
        g = np.empty((7, n, n, n))
        s = np.empty((n, n))
        _check(self._lib.lbm_get_populations(self._h, _ptr(f), _ptr(g), _ptr(s)))
        return f, g, s

    def save_state(self) -> bytes:
        size = ctypes.c_size_t(0)
        _check(self._lib.lbm_save_state(self._h, None, ctypes.byref(size)))
        buf = ctypes.create_string_buffer(size.value)
        _check(self._lib.lbm_save_state(self._h, buf, ctypes.byref(size)))
        return buf.raw[: size.value]

    def load_state(self, blob: bytes) -> None:
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(self._lib.lbm_load_state(self._h, buf, len(blob)))


CEILINGS = {"copy": 0, "pattern": 1}


def bandwidth_ceiling(which: str, n: int, precision: str = "f32", flow: int = 1, reps: int = 10,
                      stream=None):
    """(ms per launch, bytes per launch) of a bandwidth-ceiling kernel:
    "copy" (float4 copy of distribution-sized buffers) or "pattern" (the
    bare access pattern of the all-liquid step in its layout and launch)."""
    if not torch.cuda.is_available():
        raise RuntimeError("lbmmelt needs a HIP GPU; none is visible")
    lib = load_library()
    if stream is None:
        stream = torch.cuda.current_stream()
    ms, nbytes = ctypes.c_double(), ctypes.c_double()
    _check(lib.lbm_bandwidth_ceiling(CEILINGS[which], int(n), PRECISIONS[precision], int(flow),
                                     int(reps), ctypes.c_void_p(stream.cuda_stream),
                                     ctypes.byref(ms), ctypes.byref(nbytes)))
    return ms.value, nbytes.value


class LiquidFraction(torch.autograd.Function):
    """f_l after ``nsteps`` steps as a function of the hot-wall temperature
    field T_h (n x n tensor on the GPU, column layout of the front).

    forward: a fresh context from ``cfg`` at its initial state, T_h set, run
    with a checkpoint every ``every_k`` steps.  backward: the hand-written
    adjoint (recompute between checkpoints, transposed step in reverse)."""

    @staticmethod
    def forward(ctx, th, cfg, nsteps, every_k):
        sim = Sim(cfg)
        sim.set_hot_wall(th)
        fl = sim.forward_ckpt(int(nsteps), int(every_k))
        ctx.sim = sim
        ctx.th_dtype = th.dtype
        return torch.tensor(fl, dtype=torch.float64, device=th.device)

    @staticmethod
    def backward(ctx, grad_out):
        g = ctx.sim.adjoint(1.0, device=True)
        ctx.sim.close()
        return (grad_out * g).to(ctx.th_dtype), None, None, None
