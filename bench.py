#!/usr/bin/env python3
"""Throughput of the double-MRT melting step on one MI355X.

Metric: double-MRT MLUPS (million lattice-cell updates per second) and HBM
GB/s at 256^3, FP32 distributions, with the 16-bit shifted-storage path
reported beside it.

Workload (the timed step): one full step of the method - fused pull-stream +
MRT collide of f (D3Q19, Boussinesq force) and g (D3Q7), the interface
update of Eq. (6), the phase switch and the neighbourhood masks - on the
256^3 side-heated cavity (Ra = 1e5, Pr = 1, Ste = 0.1) in its all-liquid
state (front at the far wall), so that every cell runs the full double MRT
and moves 208 B (FP32).  The melting state of the same configuration
(front near the heated wall) is timed as well and reported separately.

Also reported: the 512^3 bottom-heated configuration in FP16 shifted storage
(`bottom512`), the adjoint timings (`adjoint`), two measured bandwidth
ceilings from the library's own kernels (`roofline.copy_ceiling_GBps`: a
float4 copy; `roofline.pattern_ceiling_GBps`: the bare access pattern of the
all-liquid step in the same layout and launch), and the equal-error leg
(`equal_error`: the melting run of the same configuration in FP64, FP32, FP16
and BF16 storage side by side for 2e4 steps, each format's liquid-fraction and
temperature errors against FP64 beside its throughput, and the
discretization band from FP64 at half resolution).

Output: one JSON line (see the contract in the repository notes).  The
roofline object uses the stream-collide kernel's average duration measured
live with HIP events on the stream it runs on; `traffic` comes from the
rocprofv3 counter summary under profiles/ when it was taken on the current
kernel source (else null).

Modes:
  (default)       the benchmark line
  --mode profile  a short run of one workload only, for rocprofv3: the
                  all-liquid benchmark state by default; --precision, --melting,
                  --case bottom512 --n 512 select the others
  --mode copy     a plain device copy of known size (counter calibration)
  --mode adjoint  the checkpointed forward run and the reverse sweep alone
                  (64^3 x 2000 steps with a checkpoint every 100, and
                  256^3 x 100 steps every 10), for rocprofv3
  --mode paper    the paper's two convection cases (Pr = 0.02, Ra = 25000 to
                  Fo = 1.00 and Ra = 10000 to Fo = 1.57) at --n (default 256)
  --mode precision
                  storage precision against an FP64 run of the same melting
                  configuration (256^3, 1e5 steps by default): liquid fraction
                  and temperature errors of FP32, FP16 and BF16 storage, each
                  with its throughput, plus an FP64 run at half resolution and
                  equal Fourier number for the discretization error
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
BYTES_PER_CELL = {"f32": 208, "f16s": 104, "bf16s": 104, "f64": 416}
# Algorithmic bytes per cell, FP32 storage and FP32 per-cell adjoints.  A
# forward step moves 208 B in a liquid cell and 56 B (g alone) in a solid one.
# A reverse step in a liquid cell: transposed collision (state 104 B and
# adjoint 104 B read, 104 B written) and transposed streaming (104 B read,
# 104 B written); in a solid cell only the g adjoint, 28 B read and 28 B
# written by each of the two, or 28 + 28 B in all where the streaming is
# paired with the next reverse collision (the bulk-solid rows of lattices
# above 128^3, in every step of a segment but its last).
FWD_BYTES_LIQUID, FWD_BYTES_SOLID = 208, 56
ADJ_BYTES_LIQUID = 312 + 208
ADJ_BYTES_SOLID, ADJ_BYTES_SOLID_PAIRED = 56 + 56, 28 + 28
ADJ_PAIR_MIN_N = 129
# sources the stream-collide kernel is compiled from
KERNEL_SRC = [os.path.join(ROOT, "paper_1604_03478_amd", "csrc", f)
              for f in ("lbm_kernels.hip", "lbm_device.h", "lbm_internal.h")]
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "stream_collide_f32_256_counters.md")


def workload_config(n: int, precision: str, all_liquid: bool):
    """The side-heated convection workload (preset conv256) at n^3."""
    from paper_1604_03478_amd import presets
    return presets.conv256(precision, all_liquid, n=n).config


def time_steps(sim, stream, steps: int):
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps  # ms per step


def kernel_ms(sim, steps: int):
    sim.kernel_timing(True)
    sim.step(steps)
    ms, launches = sim.kernel_time()
    sim.kernel_timing(False)
    return ms / launches


def measure(n, precision, all_liquid, steps, warmup, stream):
    from paper_1604_03478_amd import Sim
    sim = Sim(workload_config(n, precision, all_liquid), stream=stream)
    sim.step(warmup)
    ms = time_steps(sim, stream, steps)
    kms = kernel_ms(sim, max(10, min(steps, 200)))
    fl = sim.liquid_fraction()
    sim.close()
    return ms, kms, fl


def ceilings(n: int, stream, reps: int = 20):
    """Measured bandwidth ceilings (GB/s) from the library's ceiling kernels:
    a float4 copy of distribution-sized buffers, and the bare access pattern
    of the all-liquid step (every population pulled and stored, no
    arithmetic) in the step kernel's layout and launch, FP32 and FP16."""
    from paper_1604_03478_amd.binding import bandwidth_ceiling
    out = {}
    for key, which, prec in (("copy_f32", "copy", "f32"), ("pattern_f32", "pattern", "f32"),
                             ("pattern_f16s", "pattern", "f16s")):
        ms, nbytes = bandwidth_ceiling(which, n, prec, 1, reps, stream=stream)
        out[key] = {"GBps": round(nbytes / (ms * 1e-3) / 1e9, 1), "ms": round(ms, 5),
                    "bytes": nbytes}
    return out


def bottom_heated_512(stream, steps: int, warmup: int):
    """The large configuration: 512^3, hot wall z = 0 (every other wall
    adiabatic), Ra = 1e6, Pr = 1, Ste = 0.1, FP16 shifted storage with FP32
    collision and FP64 front and reductions.  Throughput of the all-liquid
    state (every cell moves 104 B) and of the initial melting state."""
    from paper_1604_03478_amd import Sim, presets
    n = 512
    out = {"workload": "convection melting 512^3, bottom-heated (hot z=0), Ra=1e6, Pr=1, "
                       "Ste=0.1, fp16 shifted storage, fp32 collide, fp64 front"}
    for key, liquid in (("all_liquid", True), ("melting_state", False)):
        cfg = presets.bottom512("f16s", all_liquid=liquid, n=n).config
        sim = Sim(cfg, stream=stream)
        sim.step(warmup)
        ms = time_steps(sim, stream, steps)
        kms = kernel_ms(sim, steps)
        fl = sim.liquid_fraction()
        sim.close()
        d = {"MLUPS": round(n ** 3 / (ms * 1e-3) / 1e6, 1), "ms_per_step": round(ms, 4),
             "kernel_ms": round(kms, 4), "liquid_fraction": round(fl, 6)}
        if key == "all_liquid":
            d["achieved_GBps"] = round(BYTES_PER_CELL["f16s"] * n ** 3 / (kms * 1e-3) / 1e9, 1)
        out[key] = d
    # the bare access pattern of the all-liquid step at this size (launch shape
    # and row order of the step kernel in that state)
    from paper_1604_03478_amd.binding import bandwidth_ceiling
    pms, nbytes = bandwidth_ceiling("pattern", n, "f16s", 1, 10, stream=stream)
    pat = nbytes / (pms * 1e-3) / 1e9
    out["all_liquid"]["pattern_ceiling_GBps"] = round(pat, 1)
    out["all_liquid"]["frac_of_pattern"] = round(out["all_liquid"]["achieved_GBps"] / pat, 4)
    return out


def large_run(stream, n: int, steps: int, sample: int = 1000):
    """The large configuration run to its end: n^3 (512), hot wall z = 0,
    Ra = 1e6, Pr = 1, Ste = 0.1, FP16 shifted storage, front seeded at s0 = 1.
    Whole-run throughput, the liquid fraction against the Fourier number, and
    HBM GB/s from the algorithmic bytes of each step: a liquid cell moves
    104 B, a solid one the 28 B of g; the liquid share is f_l, sampled every
    `sample` steps outside the timed part."""
    import torch
    from paper_1604_03478_amd import Sim, presets
    cfg = presets.bottom512("f16s", n=n).config
    sim = Sim(cfg, stream=stream)
    alpha = sim.lattice()["alpha"]
    done, t_gpu, nbytes, hist = 0, 0.0, 0.0, {}
    fl = sim.liquid_fraction()
    while done < steps:
        k = min(sample, steps - done)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(k)
        torch.cuda.synchronize()
        t_gpu += time.perf_counter() - t0
        fl_new = sim.liquid_fraction()
        nbytes += k * n ** 3 * (28.0 + 76.0 * 0.5 * (fl + fl_new))
        fl = fl_new
        done += k
        if done % 10000 == 0 or done == steps:
            hist[str(done)] = round(fl, 6)
            print(f"large: step {done} Fo {alpha * done / n ** 2:.4f} f_l {fl:.6f} "
                  f"{n ** 3 * done / t_gpu / 1e6:.0f} MLUPS", file=sys.stderr, flush=True)
    nu = sim.wall_nusselt()
    sim.close()
    return {"mode": "large", "workload": f"convection melting {n}^3, bottom-heated (hot z=0), "
            "Ra=1e6, Pr=1, Ste=0.1, fp16 shifted storage, fp32 collide, fp64 front, s0=1",
            "steps": done, "fo_end": round(alpha * done / n ** 2, 5), "seconds": round(t_gpu, 2),
            "MLUPS": round(n ** 3 * done / t_gpu / 1e6, 1),
            "algorithmic_GBps": round(nbytes / t_gpu / 1e9, 1),
            "liquid_fraction": hist, "nu_mean_end": round(float(nu.mean()), 4)}


def graph_timing(stream, reps: int = 3):
    """Steps launched kernel by kernel against the same steps run as replays
    of a captured graph (lbm_set_graph): ms per step, the two modes
    alternating `reps` times on a context each (the two stay in the same
    state) and each keeping its best."""
    from paper_1604_03478_amd import Sim
    out = []
    for n, prec, liquid, steps, chunk in ((64, "f32", False, 2000, 100),
                                          (64, "f16s", False, 2000, 100),
                                          (256, "f32", True, 200, 100),
                                          (256, "f16s", True, 200, 100)):
        sims = {m: Sim(workload_config(n, prec, liquid), stream=stream)
                for m in ("launch", "graph")}
        sims["graph"].set_graph(chunk)
        for sim in sims.values():
            sim.step(chunk)  # warm-up, and the capture
        best = {m: float("inf") for m in sims}
        for _ in range(reps):
            for m, sim in sims.items():
                best[m] = min(best[m], time_steps(sim, stream, steps))
        for sim in sims.values():
            sim.close()
        out.append({"n": n, "precision": prec, "state": "all-liquid" if liquid else "melting",
                    "steps": steps, "chunk": chunk,
                    "launch_ms_per_step": round(best["launch"], 5),
                    "graph_ms_per_step": round(best["graph"], 5),
                    "graph_speedup": round(best["launch"] / best["graph"], 4)})
    return out


def adjoint_timing(stream, n: int, steps: int, every: int):
    """Gradient of f_l after `steps` steps with respect to T_h(x, z), FP32
    storage, checkpoint every `every` steps: time of the checkpointed forward
    run, of the reverse sweep (recompute included) and of plain steps.  The
    pair runs twice; the figures are the second's, with its buffers in place
    (the first's, which allocates them, are reported as first_call), and the
    two gradients must agree bit for bit."""
    import numpy as np
    import torch
    from paper_1604_03478_amd import Sim, presets
    # C4 at 64^3; the C3 physics (Ra = 1e5) at other sizes
    p = presets.adj64("f32") if n == 64 else presets.conv256("f32", n=n)
    cfg = p.config
    th = 1.0 + 0.1 * np.random.default_rng(max(p.hot_wall_seed, 0)).standard_normal((n, n))
    sim = Sim(cfg, stream=stream)
    sim.set_hot_wall(th)
    blob = sim.save_state()
    plain = time_steps(sim, stream, steps)
    times = []
    for _ in range(2):  # the first pass also allocates the checkpoints and sweep buffers
        sim.load_state(blob)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.forward_ckpt(steps, every)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        grad = sim.adjoint(1.0, device=True)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        times.append(((t1 - t0) * 1e3, (t2 - t1) * 1e3, grad.clone()))
    if not torch.equal(times[0][2], times[1][2]):
        raise RuntimeError("the two reverse sweeps differ")
    fl = sim.liquid_fraction()
    sim.close()
    fwd, adj = times[1][0], times[1][1]
    # algorithmic bytes of the sweep, one recomputed forward step and one
    # reverse step per step, at the final (largest) liquid fraction; the
    # recompute runs beside the reverse steps, so only the sum is timed
    solid_rev = ADJ_BYTES_SOLID
    if n >= ADJ_PAIR_MIN_N:
        solid_rev = (ADJ_BYTES_SOLID_PAIRED * (every - 1) + ADJ_BYTES_SOLID) / every
    sweep_bytes = steps * n ** 3 * (fl * (FWD_BYTES_LIQUID + ADJ_BYTES_LIQUID)
                                    + (1.0 - fl) * (FWD_BYTES_SOLID + solid_rev))
    return {"n": n, "steps": steps, "every_k": every, "liquid_fraction": round(fl, 6),
            "plain_ms_per_step": round(plain, 4), "forward_ckpt_ms": round(fwd, 2),
            "adjoint_ms": round(adj, 2), "adjoint_over_forward": round(adj / (plain * steps), 2),
            "first_call": {"forward_ckpt_ms": round(times[0][0], 2),
                           "adjoint_ms": round(times[0][1], 2)},
            "sweep_ms_per_step": round(adj / steps, 4),
            "sweep_GBps_est": round(sweep_bytes / (adj * 1e-3) / 1e9, 1),
            "grad_norm": float(torch.linalg.norm(grad).item())}


def paper_cases(n: int, stream, f_wall: int = 0):
    """The paper's convection cases (section 3.2): Pr = 0.02, Ste = 0.1,
    side-heated cube, case 1 Ra = 25000 to Fo = 1.00, case 2 Ra = 10000 to
    Fo = 1.57 (the same lattice time), FP32 storage: throughput of the whole
    run and the quantities the paper discusses (liquid fraction against Fo,
    heated-wall Nusselt numbers, temperature stratification).  f_wall 1: the
    bounce-back of f interpolated to the front's position on each link."""
    import numpy as np
    import torch
    from paper_1604_03478_amd import Config, Sim
    out = {"mode": "paper", "n": n, "f_wall": f_wall,
           "workload": f"convection melting {n}^3, side-heated, "
           "Pr=0.02, Ste=0.1, fp32 storage, front seeded at s0=1"}
    for case, ra, fo_end in ((1, 25000.0, 1.00), (2, 10000.0, 1.57)):
        sim = Sim(Config(n=n, ra=ra, pr=0.02, ste=0.1, s0=1.0, precision="f32", f_wall=f_wall),
                  stream=stream)
        alpha = sim.lattice()["alpha"]
        fos = [f for f in (0.25, 0.5, 0.75, 1.0, 1.25, 1.57) if f <= fo_end + 1e-9]
        done, fl, t_gpu = 0, {}, 0.0
        for fo in fos:
            t = int(round(fo * n * n / alpha))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sim.step(t - done)
            torch.cuda.synchronize()
            t_gpu += time.perf_counter() - t0
            done = t
            fl[str(fo)] = round(sim.liquid_fraction(), 6)
            print(f"paper: case {case} Fo {fo} step {t} f_l {fl[str(fo)]}", file=sys.stderr,
                  flush=True)
        nu = sim.wall_nusselt()
        F = sim.fields(which=("T", "s"))
        T, s = F["T"], F["s"]
        depth = max(int(0.5 * s.min()), 1)
        Tm = T[:, depth, :]
        out[f"case{case}"] = {
            "ra": ra, "fo": fo_end, "steps": done, "MLUPS": round(n ** 3 * done / t_gpu / 1e6, 1),
            "liquid_fraction": fl, "nu_mean": round(float(nu.mean()), 4),
            "nu_mid_x": round(float(nu[:, n // 2].mean()), 4),
            "nu_side_x": round(float(0.5 * (nu[:, 0].mean() + nu[:, n - 1].mean())), 4),
            "T_liquid_top_quarter": round(float(Tm[3 * n // 4:].mean()), 4),
            "T_liquid_bottom_quarter": round(float(Tm[: n // 4].mean()), 4)}
        sim.close()
    print(json.dumps(out), flush=True)


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for path in KERNEL_SRC:
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_from_profile(n: int):
    """HBM bytes per stream-collide launch from the committed counter summary,
    if it was taken on the current kernel source."""
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None
    text = open(TRAFFIC_SUMMARY).read()
    src_hash = kernel_source_sha()
    m = re.search(r"kernel-source-sha256:\s*([0-9a-f]{64})", text)
    t = re.search(r"hbm-bytes-per-launch:\s*([0-9.eE+]+)", text)
    nn = re.search(r"lattice:\s*(\d+)", text)
    if not (m and t and nn) or m.group(1) != src_hash or int(nn.group(1)) != n:
        return None
    return float(t.group(1))


def cpu_baseline(n: int, steps: int):
    """The FP64 oracle, as it stands, on this host's cores: a bounded sample
    of the same workload (a few steps of the all-liquid 256^3 state) with all
    the threads OpenMP gives it, then one step on one thread."""
    from oracle import OracleSim
    from oracle import oracle as orc_mod
    orc_mod.build_oracle()
    orc = OracleSim(n, ra=1e5, pr=1.0, ste=0.1, t_h=1.0, t_c=0.0, t_m=0.0, ma=0.1,
                    s0=float(n), heating=0, flow=1)
    cores = orc_mod.threads()
    orc.step(1)  # first touch of the buffers
    t0 = time.perf_counter()
    orc.step(steps)
    el = time.perf_counter() - t0
    orc_mod.set_threads(1)
    t1 = time.perf_counter()
    orc.step(1)
    el1 = time.perf_counter() - t1
    orc_mod.set_threads(cores)
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    cpu = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": n ** 3 * steps / el / 1e6, "unit": "MLUPS", "cores": cores,
            "kind": "oracle", "value_1thread": n ** 3 / el1 / 1e6,
            "cpu_model": cpu, "host_cpus": os.cpu_count(),
            "oracle_build": "gcc " + " ".join(orc_mod.CFLAGS),
            "sample": f"{steps} steps of the {n}^3 all-liquid double-MRT state on {cores} "
                      f"threads ({n ** 3 * steps / 1e6:.1f}M FP64 cell updates, {el:.1f} s), "
                      f"then 1 step on 1 thread ({el1:.1f} s)"}


def precision_study(n: int, steps: int, stream, samples: int = 20, emit: bool = True):
    """Same melting run (side-heated, Ra = 1e5, Pr = 1, Ste = 0.1, front seeded
    at s0 = 1) in FP64, FP32, FP16 and BF16 storage side by side; errors
    against the FP64 run.  At every sample: the liquid fraction, and for each
    format the largest temperature difference; at the end, where it sits (its
    cell, its distance along the melt axis to the FP64 front, the largest
    difference more than two cells from the front) and the first sample at
    which it exceeded 1e-5.  The discretization band is the FP64 run at half
    resolution and the same Fourier number (half the steps)."""
    import numpy as np
    import torch
    from paper_1604_03478_amd import Sim
    every = max(1, steps // samples)
    precs = ("f64", "f32", "f16s", "bf16s")
    sims = {p: Sim(workload_config(n, p, False), stream=stream) for p in precs}
    t_gpu = {p: 0.0 for p in precs}
    fl = {p: [] for p in precs}
    first_1e5 = {p: None for p in precs[1:]}
    done = 0
    T = {}
    while done < steps:
        k = min(every, steps - done)
        for p in precs:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sims[p].step(k)
            torch.cuda.synchronize()
            t_gpu[p] += time.perf_counter() - t0
            fl[p].append(sims[p].liquid_fraction())
        done += k
        T = {p: sims[p].fields(which=("T",))["T"] for p in precs}
        for p in precs[1:]:
            if first_1e5[p] is None and float(np.abs(T[p] - T["f64"]).max()) > 1e-5:
                first_1e5[p] = done
        print(f"precision: step {done} fl " +
              " ".join(f"{p} {fl[p][-1]:.9f}" for p in precs), file=sys.stderr, flush=True)
    s64 = sims["f64"].fields(which=("s",))["s"]  # [z][x], melt axis y
    for p in precs:
        sims[p].close()
    # discretization band: FP64 at n/2, same Fourier number (t scales with n)
    half = n // 2
    sim = Sim(workload_config(half, "f64", False), stream=stream)
    sim.step(steps // 2)
    fl_half = sim.liquid_fraction()
    sim.close()
    ref = fl["f64"]
    out = {"mode": "precision", "n": n, "steps": steps, "workload":
           f"convection melting {n}^3, side-heated, Ra=1e5, Pr=1, Ste=0.1, s0=1",
           "fl_f64": ref[-1], "fl_f64_half_resolution": fl_half,
           "discretization_rel": abs(fl_half - ref[-1]) / ref[-1]}
    h = np.arange(n) + 0.5
    dist = np.abs(h[None, :, None] - s64[:, None, :])  # [z][y][x]: melt-axis distance to the front
    for p in precs[1:]:
        rel = [abs(a - b) / b for a, b in zip(fl[p], ref)]
        dT = np.abs(T[p] - T["f64"])
        z, y, x = np.unravel_index(int(np.argmax(dT)), dT.shape)
        far = dist > 2.0
        out[p] = {"fl_rel_err_final": rel[-1], "fl_rel_err_max": max(rel),
                  "max_abs_dT": float(dT.max()),
                  "max_abs_dT_at": {"x": int(x), "y": int(y), "z": int(z),
                                    "melt_axis_distance_to_front": round(float(dist[z, y, x]), 3)},
                  "max_abs_dT_beyond_2_cells_of_front": float(dT[far].max()),
                  "first_sample_dT_above_1e-5": first_1e5[p],
                  "mlups_melting_state": round(n ** 3 * steps / t_gpu[p] / 1e6, 1)}
    out["f64_mlups_melting_state"] = round(n ** 3 * steps / t_gpu["f64"] / 1e6, 1)
    band = max(out["f32"]["fl_rel_err_max"], 0.1 * out["discretization_rel"])
    out["equal_error_band"] = band
    for p in ("f16s", "bf16s"):
        out[p]["within_band"] = out[p]["fl_rel_err_max"] <= band
    if emit:
        print(json.dumps(out), flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--mode", choices=["bench", "profile", "copy", "precision", "adjoint",
                                       "paper", "large", "graph"], default="bench")
    ap.add_argument("--precision-steps", type=int, default=100000)
    ap.add_argument("--precision", choices=["f32", "f16s", "bf16s", "f64"], default="f32",
                    help="storage precision of --mode profile")
    ap.add_argument("--case", choices=["side256", "bottom512"], default="side256",
                    help="--mode profile: the side-heated benchmark configuration (Ra = 1e5) "
                         "or the bottom-heated large one (Ra = 1e6); --n sets the size")
    ap.add_argument("--melting", action="store_true",
                    help="--mode profile: the melting state (front at s0 = 1) instead of the "
                         "all-liquid one")
    ap.add_argument("--f-wall", type=int, choices=[0, 1], default=0,
                    help="--mode paper: 1 interpolates the no-slip of f to the front")
    ap.add_argument("--cpu-steps", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the 512^3 and adjoint legs")
    ap.add_argument("--no-equal-error", action="store_true",
                    help="skip the bounded precision (equal-error) leg")
    ap.add_argument("--equal-error-steps", type=int, default=20000,
                    help="steps of the equal-error leg at 256^3 (its 128^3 FP64 run takes "
                         "half as many)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU slab decomposition is a design, not an implementation.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()

    if args.mode == "copy":
        nbytes = 2 << 30
        with torch.cuda.stream(stream):
            src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
            dst = torch.empty_like(src)
            for _ in range(5):
                dst.copy_(src)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(10):
                dst.copy_(src)
            e1.record(stream)
            torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 10
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes,
                          "ms": ms, "GBps": 2 * nbytes / ms / 1e6}), flush=True)
        return

    if args.mode == "profile":
        from paper_1604_03478_amd import Sim, presets
        if args.case == "bottom512":  # the large configuration, hot wall z = 0
            cfg = presets.bottom512(args.precision, all_liquid=not args.melting, n=args.n).config
        else:
            cfg = workload_config(args.n, args.precision, not args.melting)
        sim = Sim(cfg, stream=stream)
        sim.step(args.warmup)
        ms = time_steps(sim, stream, args.steps)
        print(json.dumps({"mode": "profile", "case": args.case, "n": args.n,
                          "precision": args.precision, "melting": bool(args.melting),
                          "steps": args.steps, "ms_per_step": ms,
                          "liquid_fraction": sim.liquid_fraction()}), flush=True)
        return

    if args.mode == "precision":
        precision_study(args.n, args.precision_steps, stream)
        return

    if args.mode == "paper":
        paper_cases(args.n, stream, args.f_wall)
        return

    if args.mode == "large":  # --n 512 --steps 200000 for the full large configuration
        print(json.dumps(large_run(stream, args.n, args.steps)), flush=True)
        return

    if args.mode == "graph":
        print(json.dumps({"mode": "graph", "runs": graph_timing(stream)}), flush=True)
        return

    if args.mode == "adjoint":
        print(json.dumps({"mode": "adjoint",
                          "runs": [adjoint_timing(stream, 64, 2000, 100),
                                   adjoint_timing(stream, 256, 100, 10)]}), flush=True)
        return

    n, K, W = args.n, args.steps, args.warmup
    print(f"bench: {n}^3 all-liquid FP32, {W} warmup + {K} timed steps", file=sys.stderr,
          flush=True)
    ms, kms, fl = measure(n, "f32", True, K, W, stream)
    mlups = n ** 3 / (ms * 1e-3) / 1e6
    achieved = BYTES_PER_CELL["f32"] * n ** 3 / (kms * 1e-3) / 1e9
    traffic = traffic_from_profile(n)

    print("bench: 16-bit shifted storage and the melting state", file=sys.stderr, flush=True)
    ms16, kms16, _ = measure(n, "f16s", True, K, W, stream)
    msm, kmsm, flm = measure(n, "f32", False, K, W, stream)

    line = {
        "metric": "double-MRT MLUPS & HBM GB/s at 256^3; FP16-store vs FP32 at equal error",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {
            "workload": f"convection melting {n}^3, side-heated (hot y=0), Ra=1e5, Pr=1, "
                        "Ste=0.1, full double MRT (D3Q19 f + D3Q7 g), all-liquid state",
            "n": n, "cells": n ** 3, "liquid_fraction": round(fl, 6),
            "storage": "fp32 shifted", "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4),
            "traffic": traffic,
            "kernel": "k_stream_collide<float>",
            "kernel_ms": round(kms, 5),
            "bytes_per_cell": BYTES_PER_CELL["f32"],
        },
        "fp16s": {
            "value": round(n ** 3 / (ms16 * 1e-3) / 1e6, 1), "unit": "MLUPS",
            "ms_per_step": round(ms16, 5), "kernel_ms": round(kms16, 5),
            "achieved_GBps": round(BYTES_PER_CELL["f16s"] * n ** 3 / (kms16 * 1e-3) / 1e9, 1),
            "bytes_per_cell": BYTES_PER_CELL["f16s"],
        },
        "melting_state": {
            "value": round(n ** 3 / (msm * 1e-3) / 1e6, 1), "unit": "MLUPS",
            "liquid_fraction": round(flm, 6), "ms_per_step": round(msm, 5),
            "note": "front near the heated wall: solid cells move only g (56 B)",
        },
    }
    print("bench: bandwidth ceilings, equal-error leg, 512^3 bottom-heated fp16, adjoint",
          file=sys.stderr, flush=True)
    ceil = ceilings(n, stream)
    line["roofline"]["copy_ceiling_GBps"] = ceil["copy_f32"]["GBps"]
    line["roofline"]["frac_of_copy"] = round(achieved / ceil["copy_f32"]["GBps"], 4)
    line["roofline"]["pattern_ceiling_GBps"] = ceil["pattern_f32"]["GBps"]
    line["roofline"]["frac_of_pattern"] = round(achieved / ceil["pattern_f32"]["GBps"], 4)
    line["roofline"]["ceilings"] = ceil
    line["fp16s"]["pattern_ceiling_GBps"] = ceil["pattern_f16s"]["GBps"]
    line["fp16s"]["frac_of_pattern"] = round(
        line["fp16s"]["achieved_GBps"] / ceil["pattern_f16s"]["GBps"], 4)
    if not args.no_equal_error:
        line["equal_error"] = precision_study(n, args.equal_error_steps, stream, samples=10,
                                              emit=False)
    if not args.no_extras:
        line["bottom512"] = bottom_heated_512(stream, 100, 20)
        line["adjoint"] = [adjoint_timing(stream, 64, 2000, 100),
                           adjoint_timing(stream, 256, 100, 10)]
        line["graph"] = graph_timing(stream)
    if not args.no_cpu_baseline:
        print("bench: CPU oracle baseline", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(n, args.cpu_steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
