// Internal interface between the host context (lbm_capi.hip) and the gfx950
// kernels (lbm_kernels.hip) of liblbmmelt.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbmk {

// Storage precisions (same numbering as lbm_precision in the public header).
enum StoreKind { kF64 = 0, kF32 = 1, kF16S = 2, kBF16S = 3 };

// Everything a step kernel needs, in lattice units.  Distributions are
// stored shifted: f_q - w_q * rho0 (rho0 = 1) and g_q - w_q * tref with
// tref = (t_h + t_m)/2, the middle of the liquid temperature range, so every
// kernel works on small deviations from a rest state.
struct KParams {
  int n;           // cells per edge
  uint32_t ncell;  // n^3
  uint32_t pitch;  // elements of one direction row (>= n; rows start 128-byte aligned)
  int melt_z;      // 0: melt axis y (hot wall y=0, cold wall y=n); 1: axis z
  int flow;        // 0: energy distribution only
  double t0;       // buoyancy reference temperature
  double tref;     // storage shift of g: (t_h + t_m)/2
  double t_m;      // melting temperature (front Dirichlet value)
  double t_c;      // cold-wall temperature (melt axis y only)
  double gbeta;    // buoyancy: F_z = gbeta * (T - t0)
  double s_nu;     // shear rate of the D3Q19 MRT
  double q_j;      // heat-flux rate of the D3Q7 MRT
  double q_e;      // rate of the remaining D3Q7 moments
  double q_js;     // the same two rates in solid cells (solid diffusivity kappa * alpha)
  double q_es;
  double kappa;    // solid / liquid conductivity ratio of Eq. (6)
  int f_wall;      // 1: no-slip of f at the front interpolated to the link fraction
  double alpha;    // thermal diffusivity (front update)
  double ste;      // Stefan number (front update)
  double dT;       // nominal t_h - t_m (front update)
  uint32_t step;   // step counter (seeds the per-cell random stream of rounding)
  // Graph replays: the step counter in device memory, advanced by each step's
  // front kernel (launch_front's step_ctr); null: use step.
  const uint32_t* step_dev;
  // 16-bit storage with two workgroups per row: 1 keeps both halves of a row
  // on one XCD (the order for a mostly liquid lattice; results identical).
  int pair_rows;
  // ceil(2^32 / (n - 2)): the interior rows of the walls-first row order are
  // numbered without an integer division (recip32)
  uint32_t inv_nm2;
  // ceil(2^32 / n): cell, row and column indices split without an integer
  // division (div_n)
  uint32_t inv_n;
  // s_nu, gbeta, q_j, q_e, q_js, q_es, tref and tref - t0 rounded to FP32 on
  // the host (set_f32_params), for the kernels that collide in FP32: the
  // values a conversion in every wave would give
  float s_nu_f, gbeta_f, q_j_f, q_e_f, q_js_f, q_es_f, tref_f, dbuoy_f;
};

inline void set_f32_params(KParams& k) {
  k.s_nu_f = (float)k.s_nu;
  k.gbeta_f = (float)k.gbeta;
  k.q_j_f = (float)k.q_j;
  k.q_e_f = (float)k.q_e;
  k.q_js_f = (float)k.q_js;
  k.q_es_f = (float)k.q_es;
  k.tref_f = (float)k.tref;
  k.dbuoy_f = (float)(k.tref - k.t0);
}

// ceil(2^32 / d) for 2 <= d < 2^32.
inline uint32_t recip32(uint32_t d) { return (uint32_t)((0xFFFFFFFFull + d) / d); }

size_t store_bytes(int kind);

// Layout of a distribution with Q directions in HBM: row-interleaved.  For
// every lattice row (y, z), its Q direction rows of `pitch` elements (x
// fastest) lie next to each other; rows follow in (z, y) order.  Population
// q of cell (x, y, z) is element ((z n + y) Q + q) pitch + x.  A distribution
// takes Q * pitch * n^2 elements.
uint32_t row_pitch(int n, int kind);

// Whether the step kernel of a storage kind reads the precomputed 3x3
// neighbourhood min / max of the liquid counts (16-bit storage, one packed
// word per column); the others take it from the counts themselves.
inline bool uses_neighbourhood(int kind) { return store_bytes(kind) == 2; }

// One fused stream + collide pass over all cells: reads (fs, gs), writes
// (fd, gd).  cnt: liquid-cell count per column; cext: its min | max << 16
// over the 3x3 column neighbourhood (from launch_neighbourhood; read only
// for 16-bit storage, see uses_neighbourhood).  rowmax (16-bit storage, may be null):
// the largest 3x3 maximum of every row of columns, from launch_neighbourhood; with
// it the lattice rows whose stencils are all solid skip the per-cell phase
// loads (the same results bit for bit).  s: front per column.  th: hot-wall
// temperature per column.  flag: set to 1 when a non-finite value appears.
// ev_start / ev_stop (or null): events the kernel's dispatch records at its
// start and end (the kernel's own duration, with no separate event packets).
hipError_t launch_stream_collide(int kind, const KParams& P, const void* fs, void* fd,
                                 const void* gs, void* gd, const int* cnt, const uint32_t* cext,
                                 const int* rowmax, const double* s, const double* th, int* flag,
                                 hipStream_t st, hipEvent_t ev_start = nullptr,
                                 hipEvent_t ev_stop = nullptr);

// Interface update (Eq. (6)) of every column from the post-collision g, then
// the phase switch: s_new, cnt (in place), refill of f in newly liquid cells,
// per-column melt / freeze counters.  Schedule (each 3 * n^2 ints: liquid
// count, index of the first liquid node, index of the first solid node):
// record != null writes the one this step uses; replay != null makes the step
// use the given node indices and take the new liquid counts from
// replay_next (the following entry) instead of the new fronts.  heat != null
// (n^2 values from launch_front_heat) moves every front by heat * Ste /
// (t_h - t_m), the conservative form of the same balance, instead of Eq. (6).
// step_ctr (may be null): a device step counter that this launch advances by
// one; no kernel after it in the step reads the counter.
hipError_t launch_front(int kind, const KParams& P, const double* s_old, double* s_new,
                        int* cnt, const void* g, void* f, const double* th, int* melted,
                        int* frozen, int* flag, const int* replay, const int* replay_next,
                        int* record, const double* heat, uint32_t* step_ctr, hipStream_t st);

// cext: min | max << 16 of cnt over the 3x3 columns around each column (the
// columns in the box), for the fast-path test of the 16-bit step kernel;
// rowmax (n values, may be null): the largest max over each row of columns
// (all x for one value of the other lateral index).
hipError_t launch_neighbourhood(const KParams& P, const int* cnt, uint32_t* cext, int* rowmax,
                                hipStream_t st);

// *p = v (one thread).
hipError_t launch_set_u32(uint32_t* p, uint32_t v, hipStream_t st);

// cnt from s.
hipError_t launch_counts(const KParams& P, const double* s, int* cnt, hipStream_t st);

// Initial state: f at rest, g at equilibrium of seedT[a] (a the melt-axis
// coordinate; the host fills solid heights with t_c or the subcooled profile).
hipError_t launch_init(int kind, const KParams& P, const double* seedT, void* f, void* g,
                       hipStream_t st);

// Macroscopic fields in FP64 (any output may be null).
hipError_t launch_fields(int kind, const KParams& P, const void* f, const void* g, const int* cnt,
                         double* T, double* ux, double* uy, double* uz, double* rho,
                         hipStream_t st);

// Conversion between unshifted FP64 populations and the shifted storage.
// q_count = 19 (f) or 7 (g).
hipError_t launch_to_storage(int kind, const KParams& P, int q_count, const double* src, void* dst,
                             hipStream_t st);
hipError_t launch_from_storage(int kind, const KParams& P, int q_count, const void* src,
                               double* dst, hipStream_t st);

// Deterministic FP64 sum (fixed order; no atomics) of v[0..count) into
// out[0].  count must not exceed the number of elements v points to.
hipError_t launch_sum(const double* v, int64_t count, double* out, hipStream_t st);

}  // namespace lbmk
