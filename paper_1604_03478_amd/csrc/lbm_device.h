// Device-side helpers shared by the step kernels (lbm_kernels.hip) and the
// adjoint kernels (lbm_adjoint.hip): storage formats, arithmetic types,
// rounding at the store, and the two lattices.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_internal.h"



namespace lbmk {

// --------------------------------------------------------------- storage
// Arithmetic types of the collision: `type` for the flow (f, D3Q19),
// `gtype` for the energy distribution (g, D3Q7).  16-bit storage collides in
// FP32.  FP32 storage collides the flow in FP32 and the energy distribution
// in FP64 (rounded stochastically to FP32 at the store): temperature round
// off accumulated over 1e4+ steps is what moves the front, and the D3Q7 part
// is a small share of the arithmetic.
#ifndef LBM_F32_FLOW_T
#define LBM_F32_FLOW_T float
#endif
#ifndef LBM_F32_HEAT_T
#define LBM_F32_HEAT_T double
#endif
template <typename Ts> struct Compute { using type = float; using gtype = float; };
template <> struct Compute<double> { using type = double; using gtype = double; };
template <> struct Compute<float> { using type = LBM_F32_FLOW_T; using gtype = LBM_F32_HEAT_T; };

// Rounding of the collision result to the storage format.  With stochastic
// rounding the value is rounded up or down with probabilities proportional
// to its distance from the two neighbours (random bits added below the
// storage precision, then truncation toward zero), so the rounding error has
// zero mean even when the same value is stored step after step.
// Measured at 64^3 over 20000 steps against the FP64 oracle: FP16 storage
// with round-to-nearest drifts to a 1e-2 relative liquid-fraction error,
// with stochastic rounding 4.5e-6; FP32 storage with an FP64 energy collision
// and stochastic rounding stays at 1e-10.
#ifndef LBM_STOCHASTIC_ROUNDING
#define LBM_STOCHASTIC_ROUNDING 1
#endif

// Random bits of the rounding: one 32-bit hash per cell and step (a mix of
// the cell index and the step), then a Weyl sequence over the values the cell
// stores (each adds the 32-bit golden-ratio constant).  Every value's offset
// is uniform over the hash, so its rounding error has zero mean; within a
// cell the offsets are spread evenly (low discrepancy), and advancing the
// stream costs one integer add instead of a 32-bit multiply.  The hash is
// C. Wellons' published 32-bit integer mixer "lowbias32" (found by his
// hash-prospector search): two xor-shift / multiply rounds and a final
// xor-shift, with his shift amounts and multipliers.
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}
// The step that seeds a cell's hash: the kernel argument, or the counter in
// device memory that graph replays advance (a uniform scalar load).
__device__ __forceinline__ uint32_t step_of(const KParams& P) {
  return P.step_dev ? *P.step_dev : P.step;
}
// floor(k / n) for k < 2^30 (indices of cells, rows and columns) with the
// host's reciprocal ceil(2^32 / n): the multiply-high gives the quotient or
// one more, and one comparison corrects it.
__device__ __forceinline__ uint32_t div_n(uint32_t k, const KParams& P) {
  const uint32_t q = __umulhi(k, P.inv_n);
  return q - (q * (uint32_t)P.n > k ? 1u : 0u);
}

__device__ __forceinline__ uint32_t next_rand(uint32_t& st) {
  st += 0x9e3779b9u;
  return st;
}

template <typename Ts, typename C>
__device__ __forceinline__ Ts round_store(C v, uint32_t& rs) {
#if LBM_STOCHASTIC_ROUNDING
  if constexpr (sizeof(Ts) == 4 && sizeof(C) == 8) {
    uint64_t b = (uint64_t)__double_as_longlong(v);
    b += (uint64_t)(next_rand(rs) >> 3);  // 29 bits below FP32 precision
    b &= ~((1ull << 29) - 1);
    return static_cast<Ts>(__longlong_as_double((long long)b));
  } else if constexpr (sizeof(Ts) == 2 && sizeof(C) == 4) {
    uint32_t b = __float_as_uint(v);
    constexpr int drop = __is_same(Ts, _Float16) ? 13 : 16;  // bits below the 16-bit format
    b += next_rand(rs) >> (32 - drop);
    b &= ~((1u << drop) - 1);
    return static_cast<Ts>(__uint_as_float(b));
  }
#endif
  (void)rs;
  return static_cast<Ts>(v);
}

template <typename R, typename Ts>
__device__ __forceinline__ R load_as(const Ts* __restrict__ base, uint32_t i) {
  const Ts* p = reinterpret_cast<const Ts*>(reinterpret_cast<const char*>(base) +
                                            (uint32_t)(i * (uint32_t)sizeof(Ts)));
  return static_cast<R>(*p);
}
template <typename Ts>
__device__ __forceinline__ typename Compute<Ts>::type load(const Ts* __restrict__ base, uint32_t i) {
  return load_as<typename Compute<Ts>::type>(base, i);
}

template <typename Ts, typename C>
__device__ __forceinline__ void store(Ts* __restrict__ base, uint32_t i, C v) {
  Ts* p = reinterpret_cast<Ts*>(reinterpret_cast<char*>(base) + (uint32_t)(i * (uint32_t)sizeof(Ts)));
  *p = static_cast<Ts>(v);
}

// Population loads of the step kernel: every stored value is read once per
// step (the +-1 x shift of a row is caught by the workgroup's own loads), so
// they may bypass the caches as well.  Measured on MI355X at 256^3 (FP32,
// all liquid): 5.47 TB/s with non-temporal loads, 5.55 without; off.
#ifndef LBM_NT_LOADS
#define LBM_NT_LOADS 0
#endif
template <typename R, typename Ts>
__device__ __forceinline__ R load_stream(const Ts* __restrict__ base, uint32_t i) {
  const Ts* p = reinterpret_cast<const Ts*>(reinterpret_cast<const char*>(base) +
                                            (uint32_t)(i * (uint32_t)sizeof(Ts)));
#if LBM_NT_LOADS
  return static_cast<R>(__builtin_nontemporal_load(p));
#else
  return static_cast<R>(*p);
#endif
}

// Stores of the step kernel: written once, read only in the next step, so
// they bypass the caches (non-temporal).
template <typename Ts, typename C>
__device__ __forceinline__ void store_stream(Ts* __restrict__ base, uint32_t i, C v, uint32_t& rs) {
  Ts* p = reinterpret_cast<Ts*>(reinterpret_cast<char*>(base) + (uint32_t)(i * (uint32_t)sizeof(Ts)));
  __builtin_nontemporal_store(round_store<Ts>(v, rs), p);
}

// --------------------------------------------------------------- layout
// Row-interleaved distributions (see row_pitch): the Q direction rows of one
// lattice row (y, z) are contiguous, so the update of a row reads and writes a
// few contiguous blocks rather than Q arrays that lie far apart in HBM.
template <int Q, typename Ts>
__device__ __forceinline__ Ts* row_ptr(Ts* base, const KParams& P, int y, int z) {
  return base + ((uint64_t)z * (uint64_t)P.n + (uint64_t)y) * (uint64_t)Q * P.pitch;
}
__device__ __forceinline__ uint64_t pop_index(const KParams& P, int Q, int q, int x, int y,
                                              int z) {
  return (((uint64_t)z * P.n + y) * (uint64_t)Q + q) * P.pitch + x;
}

// --------------------------------------------------------------- lattices
// D3Q19 in the order of Eq. (3).
__host__ __device__ constexpr int ex19(int q) {
  return (q == 1 || q == 7 || q == 9 || q == 11 || q == 13) ? 1
       : (q == 2 || q == 8 || q == 10 || q == 12 || q == 14) ? -1 : 0;
}
__host__ __device__ constexpr int ey19(int q) {
  return (q == 3 || q == 7 || q == 8 || q == 15 || q == 17) ? 1
       : (q == 4 || q == 9 || q == 10 || q == 16 || q == 18) ? -1 : 0;
}
__host__ __device__ constexpr int ez19(int q) {
  return (q == 5 || q == 11 || q == 12 || q == 15 || q == 16) ? 1
       : (q == 6 || q == 13 || q == 14 || q == 17 || q == 18) ? -1 : 0;
}
__host__ __device__ constexpr int opp19(int q) {
  return q == 0 ? 0 : (q <= 6 ? (q % 2 ? q + 1 : q - 1)
                               : (q <= 10 ? 17 - q : (q <= 14 ? 25 - q : 33 - q)));
}
// D3Q7 in the order of Eq. (5).
__host__ __device__ constexpr int ex7(int q) { return q == 1 ? 1 : (q == 2 ? -1 : 0); }
__host__ __device__ constexpr int ey7(int q) { return q == 3 ? 1 : (q == 4 ? -1 : 0); }
__host__ __device__ constexpr int ez7(int q) { return q == 5 ? 1 : (q == 6 ? -1 : 0); }
__host__ __device__ constexpr int opp7(int q) { return q == 0 ? 0 : (q % 2 ? q + 1 : q - 1); }

static_assert(ex19(opp19(7)) == -1 && ey19(opp19(7)) == -1, "opp19");
static_assert(opp19(8) == 9 && opp19(11) == 14 && opp19(12) == 13 && opp19(15) == 18 &&
              opp19(16) == 17, "opp19");

constexpr double kW7Axis = 0.125;  // D3Q7 weight of the six moving directions
constexpr double kW7Rest = 0.25;

// --------------------------------------------------------------- launch order
// Largest workgroup of the step kernel (one lattice row, or part of one, per
// workgroup) for a storage format of `bytes` per value.
__host__ __device__ constexpr int step_block_max(size_t bytes) { return bytes == 2 ? 256 : 512; }

// One lattice row per workgroup, so the row pointers are uniform over it.
// The workgroups of the n x n rows are numbered r = blockIdx.z * n +
// blockIdx.y, the order in which they are dispatched; workgroup w runs on
// XCD w mod 8 (round-robin dispatch), each XCD with its own L2.
//
// Neighbouring rows share cache lines: at an x wall a cell bounces back its
// own outgoing population, the first or last value of a direction row whose
// other values a neighbouring row (y +- 1 or z +- 1, for the 8 diagonal
// directions with an x component) pulls.  On different XCDs those 8 lines
// per row are fetched twice (256^3: reads 1.041x the algorithmic bytes in
// FP32, 1.084x in FP16).  So where a workgroup covers a whole row
// (gridDim.x == 1) and n is a multiple of 8 L: the two z-wall planes first,
// then the planes z = 1 .. n-2 in order; within a plane, the workgroup at
// position j (on XCD j mod 8) takes a row of the XCD's runs of L consecutive
// rows (y = 8 L (m / L) + L c + m mod L, m = j / 8, c the XCD's run), so a
// row and most of its y neighbours share an L2, and the plane's workgroup
// count n, a multiple of 8, keeps its z neighbours on the same XCD.  The run
// an XCD takes rotates every 8 planes (c = (j + z / 8) mod 8): a front along
// y and the y walls put their slow rows in a few runs, and fixed runs per
// XCD left those XCDs with the slow rows of every plane (256^3 melting state
// 176 -> 210 us per step).  L = 0 stands for L = n / 8, one run per XCD and
// plane.  Measured against the order below, one box, medians of three:
// FP32 (L = 4) 256^3 all-liquid 601.6 -> 598.1 us, melting 178.5 -> 175.2,
// 64^3 melting 13.2 -> 11.7, reads 1.010x; FP16 (L = 0) all-liquid 290.6 ->
// 290.9 us, melting 103.4 -> 103.8, reads 1.012x (FP16 with L = 4: +0.7 and
// +1.5 %).
//
// Two workgroups per row (16-bit storage at 256 < n <= 512), n a multiple of 8, in
// the instantiation that asks for it (PAIR): workgroups w and w + 8 of every
// block of 16 take the two halves of one row, so a row sits on one XCD as
// well, and the same order follows.  The halves share the line where a
// shifted direction row crosses from one to the other.  That pays in a
// mostly liquid lattice (512^3 all-liquid FP16 2560 -> 2438 us) and costs in
// a mostly solid one, whose g-only rows share no lines (melting state 720 ->
// 773 us), so the host picks that instantiation from the liquid fraction it
// last knew (KParams::pair_rows): any order gives the same results bit for
// bit.  (A choice inside the kernel cost the melting state 2-21 %.)
//
// Otherwise (several workgroups per row, or other n): the 4n - 4 rows on the
// y and z walls, which always take the general path, come first, and the
// interior rows follow in z-major order.  In plane order the wall plane
// z = n - 1 came last, and its slow rows formed a tail: at 256^3 the melting
// step took 214 instead of 179 us (FP32), 167 instead of 141 us (FP16).
template <int L, bool PAIR = false>
__device__ __forceinline__ void step_row(const KParams& P, int& y, int& z, int& xb) {
  // No integer divisions: the grid is (row workgroups, n, n), so blockIdx.z
  // is the plane of row r = blockIdx.z n + blockIdx.y and blockIdx.y its
  // position j in the plane (the remapped r of the paired order stays in
  // plane blockIdx.z when n is a multiple of 8), and the walls-first order
  // divides by n - 2 with the host's reciprocal.
  const int n = P.n, bz = (int)blockIdx.z;
  int j = (int)blockIdx.y;
  xb = (int)blockIdx.x;
  bool xcd_order = gridDim.x == 1;
  if (PAIR && gridDim.x == 2 && (n & 7) == 0) {
    // two workgroups per row: workgroups w and w + 8 of each block of 16
    // (w = blockIdx.x + 2 r) take the two halves of row 8 (w / 16) + w mod 8,
    // so both run on its XCD; with 2 n a multiple of 16 that row is row
    // 8 (v / 16) + v mod 8 of plane blockIdx.z, v = blockIdx.x + 2 j
    const int v = (int)blockIdx.x + 2 * j;
    j = 8 * (v >> 4) + (v & 7);
    xb = (v >> 3) & 1;
    xcd_order = true;
  }
  if (xcd_order && (n & 7) == 0 && (L == 0 || ((n >> 3) % (L > 0 ? L : 1)) == 0)) {
    if (bz < 2) {  // the z-wall planes
      y = j;
      z = bz == 0 ? 0 : n - 1;
      return;
    }
    z = bz - 1;
    const int c = ((j & 7) + (z >> 3)) & 7;  // the XCD's run in this plane
    const int m = j >> 3;
    // L = 0: one run of n / 8 rows per XCD, and m < n / 8
    y = L > 0 ? (m / L) * (L << 3) + c * L + (m % L) : c * (n >> 3) + m;
    return;
  }
  const int r = bz * n + j, nw = 4 * n - 4;
  if (r < n) {
    y = r;
    z = 0;
  } else if (r < 2 * n) {
    y = r - n;
    z = n - 1;
  } else if (r < nw) {  // the y walls of the planes 0 < z < n - 1
    const int k = r - 2 * n;
    z = 1 + (k >> 1);
    y = (k & 1) ? n - 1 : 0;
  } else {
    const uint32_t k = (uint32_t)(r - nw), d = (uint32_t)(n - 2);
    uint32_t q = __umulhi(k, P.inv_nm2);  // floor(k / d) or one more
    q -= q * d > k ? 1u : 0u;
    z = 1 + (int)q;
    y = 1 + (int)(k - q * d);
  }
}

// The run length of the step kernels' row order for a storage format of
// `bytes` per value: 4 for FP32 and FP64, one run per XCD and plane for
// 16-bit storage.
template <typename Ts>
__host__ __device__ constexpr int row_run() { return sizeof(Ts) == 2 ? 0 : 4; }

// number of cells a in [0, n) with a + 1/2 < s (exact: s - 1/2 is exact in FP64)
__device__ __forceinline__ int count_liquid(double sv, int n) {
  double c = ceil(sv - 0.5);
  if (!(c > 0.0)) return 0;
  if (c > (double)n) return n;
  return (int)c;
}

}  // namespace lbmk
