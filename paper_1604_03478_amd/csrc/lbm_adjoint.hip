// Adjoint (reverse mode) of the double-MRT melting step on gfx950.
//
// For J = f_l after N steps (front-based liquid fraction), the reverse sweep
// propagates the adjoint lambda = dJ/dX of the state X = (f*, g*, s) from
// the last step to the first and accumulates dJ/dT_h for the hot-wall
// temperature of every column.  The forward step it reverses is the one of
// lbm_kernels.hip: pull-streaming (Eq. (1), Eq. (4)) with wall, solid and
// interpolated front conditions, MRT collisions (Eq. (2), Eq. (4)), front
// velocity from the interface energy balance (Eq. (6)), phase switch.  Phase
// masks and the node selection of Eq. (6) are piecewise constant in the
// state; the adjoint is that of the forward run's own schedule.
//
// Per step, in reverse order of the forward operations:
//   k_adj_partition     per column: liquid counts of state t, their extremes
//                       over 5x5 columns, and the largest count (the bound of
//                       the bulk-solid rows); launched by the host loop
//   k_adj_front         per column: s' = s + V(g*, s): adjoint into the node
//                       temperatures, into s and its neighbours, into T_h
//                       (the phase switch needs nothing: f of a solid cell
//                       is dead data and a melting cell is refilled, so the
//                       adjoint of f is kept only where the cell is liquid
//                       on both sides of a step); k_adj_front_heat instead
//                       for the conservative front update
//   k_adj_collide       per cell of the rows that hold a liquid cell:
//                       recomputes the pulled populations and applies the
//                       transposed collision Jacobian; k_adj_collide_solid
//                       the same for the all-solid rows, g only and
//                       without the state (linear at rest)
//   k_adj_stream        per cell: transposed streaming as a gather over every
//                       reader of each stored population (no atomics), on
//                       row slots over the rows outside the bulk solid;
//                       k_adj_stream_solid the bulk-solid rows (g only)
//   k_adj_interface     per column: dependence of the interpolated front
//                       conditions on the front through the link fractions,
//                       of the hot-wall condition on T_h, and the sum of the
//                       front part left by k_adj_front
// Adjoint arithmetic is FP64 for every storage format.  The per-cell
// adjoints of f and g are stored in FP64 with FP64 storage and in FP32
// otherwise (the state they are taken at is itself FP32 or coarser); the
// adjoints of the fronts and of T_h are FP64 throughout.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_device.h"
#include "lbm_adjoint.h"
#include "lbm_internal.h"

namespace lbmk {
namespace {

constexpr double kD19[19] = {19, 2394, 252, 10, 40, 10, 40, 10, 40, 36,
                             72, 12,   24,  4,  4,  4,  8,  8,  8};
constexpr double kD7[7] = {7, 2, 2, 2, 42, 12, 4};
// their reciprocals (a multiply instead of an FP64 divide per moment)
constexpr double kInvD19[19] = {1.0 / 19, 1.0 / 2394, 1.0 / 252, 1.0 / 10, 1.0 / 40, 1.0 / 10,
                                1.0 / 40, 1.0 / 10,   1.0 / 40,  1.0 / 36, 1.0 / 72, 1.0 / 12,
                                1.0 / 24, 1.0 / 4,    1.0 / 4,   1.0 / 4,  1.0 / 8,  1.0 / 8,
                                1.0 / 8};
constexpr double kInvD7[7] = {1.0 / 7, 1.0 / 2, 1.0 / 2, 1.0 / 2, 1.0 / 42, 1.0 / 12, 1.0 / 4};
static_assert(kInvD19[1] * kD19[1] > 0.999 && kInvD7[4] * kD7[4] > 0.999, "norms");

// m = M v for the orthogonal D3Q19 basis (integer structure, pairwise sums)
__device__ __forceinline__ void m19(const double (&f)[19], double (&m)[19]) {
  const double axp = f[1] + f[2], axm = f[1] - f[2];
  const double ayp = f[3] + f[4], aym = f[3] - f[4];
  const double azp = f[5] + f[6], azm = f[5] - f[6];
  const double a78 = f[7] + f[8], b78 = f[7] - f[8], a910 = f[9] + f[10], b910 = f[9] - f[10];
  const double Sxy = a78 + a910, Xxy = b78 + b910, Yxy = a78 - a910, Pxy = b78 - b910;
  const double a1112 = f[11] + f[12], b1112 = f[11] - f[12];
  const double a1314 = f[13] + f[14], b1314 = f[13] - f[14];
  const double Sxz = a1112 + a1314, Xxz = b1112 + b1314, Zxz = a1112 - a1314, Pxz = b1112 - b1314;
  const double a1516 = f[15] + f[16], b1516 = f[15] - f[16];
  const double a1718 = f[17] + f[18], b1718 = f[17] - f[18];
  const double Syz = a1516 + a1718, Yyz = b1516 + b1718, Zyz = a1516 - a1718, Pyz = b1516 - b1718;
  const double A = axp + ayp + azp, E = Sxy + Sxz + Syz;
  const double Ed = Sxy + Sxz - 2.0 * Syz;
  m[0] = f[0] + A + E;
  m[1] = -30.0 * f[0] - 11.0 * A + 8.0 * E;
  m[2] = 12.0 * f[0] - 4.0 * A + E;
  m[3] = axm + Xxy + Xxz;
  m[4] = -4.0 * axm + Xxy + Xxz;
  m[5] = aym + Yxy + Yyz;
  m[6] = -4.0 * aym + Yxy + Yyz;
  m[7] = azm + Zxz + Zyz;
  m[8] = -4.0 * azm + Zxz + Zyz;
  m[9] = 2.0 * axp - ayp - azp + Ed;
  m[10] = -4.0 * axp + 2.0 * ayp + 2.0 * azp + Ed;
  m[11] = ayp - azp + Sxy - Sxz;
  m[12] = -2.0 * ayp + 2.0 * azp + Sxy - Sxz;
  m[13] = Pxy;
  m[14] = Pyz;
  m[15] = Pxz;
  m[16] = Xxy - Xxz;
  m[17] = Yyz - Yxy;
  m[18] = Zxz - Zyz;
}

// f = M^T a
__device__ __forceinline__ void m19t(const double (&a)[19], double (&f)[19]) {
  const double Aax = a[0] - 11.0 * a[1] - 4.0 * a[2];
  const double Aed = a[0] + 8.0 * a[1] + a[2];
  f[0] = a[0] - 30.0 * a[1] + 12.0 * a[2];
  {
    const double c = Aax + 2.0 * a[9] - 4.0 * a[10], d = a[3] - 4.0 * a[4];
    f[1] = c + d;
    f[2] = c - d;
  }
  {
    const double c = Aax - a[9] + 2.0 * a[10] + a[11] - 2.0 * a[12], d = a[5] - 4.0 * a[6];
    f[3] = c + d;
    f[4] = c - d;
  }
  {
    const double c = Aax - a[9] + 2.0 * a[10] - a[11] + 2.0 * a[12], d = a[7] - 4.0 * a[8];
    f[5] = c + d;
    f[6] = c - d;
  }
  {
    const double b = Aed + a[9] + a[10] + a[11] + a[12], X = a[3] + a[4] + a[16],
                 Y = a[5] + a[6] - a[17];
    f[7] = b + X + Y + a[13];
    f[8] = b - X + Y - a[13];
    f[9] = b + X - Y - a[13];
    f[10] = b - X - Y + a[13];
  }
  {
    const double b = Aed + a[9] + a[10] - a[11] - a[12], X = a[3] + a[4] - a[16],
                 Z = a[7] + a[8] + a[18];
    f[11] = b + X + Z + a[15];
    f[12] = b - X + Z - a[15];
    f[13] = b + X - Z - a[15];
    f[14] = b - X - Z + a[15];
  }
  {
    const double b = Aed - 2.0 * a[9] - 2.0 * a[10], Y = a[5] + a[6] + a[17],
                 Z = a[7] + a[8] - a[18];
    f[15] = b + Y + Z + a[14];
    f[16] = b - Y + Z - a[14];
    f[17] = b + Y - Z - a[14];
    f[18] = b - Y - Z + a[14];
  }
}

// n = N g (D3Q7) and g = N^T b
__device__ __forceinline__ void m7(const double (&g)[7], double (&nm)[7]) {
  const double px = g[1] + g[2], py = g[3] + g[4], pz = g[5] + g[6];
  nm[0] = g[0] + px + py + pz;
  nm[1] = g[1] - g[2];
  nm[2] = g[3] - g[4];
  nm[3] = g[5] - g[6];
  nm[4] = 6.0 * g[0] - (px + py + pz);
  nm[5] = 2.0 * px - py - pz;
  nm[6] = py - pz;
}
__device__ __forceinline__ void m7t(const double (&b)[7], double (&g)[7]) {
  const double c1 = b[0] - b[4] + 2.0 * b[5];
  const double c3 = b[0] - b[4] - b[5] + b[6];
  const double c5 = b[0] - b[4] - b[5] - b[6];
  g[0] = b[0] + 6.0 * b[4];
  g[1] = c1 + b[1];
  g[2] = c1 - b[1];
  g[3] = c3 + b[2];
  g[4] = c3 - b[2];
  g[5] = c5 + b[3];
  g[6] = c5 - b[3];
}

// ---- geometry helpers ----
struct Geo {
  int n;
  uint32_t nn;
  __device__ uint32_t cell(int x, int y, int z) const {
    return (uint32_t)z * nn + (uint32_t)y * (uint32_t)n + (uint32_t)x;
  }
  __device__ bool in(int x, int y, int z) const {
    return (unsigned)x < (unsigned)n && (unsigned)y < (unsigned)n && (unsigned)z < (unsigned)n;
  }
};

template <bool MZ>
__device__ __forceinline__ int melt_of(int y, int z) { return MZ ? z : y; }
template <bool MZ>
__device__ __forceinline__ int col_of(int x, int y, int z, int n) { return (MZ ? y : z) * n + x; }
template <bool MZ>
__device__ __forceinline__ bool liquid_at(const int* cnt, int x, int y, int z, int n) {
  return melt_of<MZ>(y, z) < cnt[col_of<MZ>(x, y, z, n)];
}
template <bool MZ>
__device__ __forceinline__ uint32_t cell_in_column(int c, int a, const KParams& P) {
  const int n = P.n, o = (int)div_n((uint32_t)c, P), x = c - o * n;
  return MZ ? ((uint32_t)a * n + o) * n + x : ((uint32_t)o * n + a) * n + x;
}

// link fraction from cell (x,y,z) along direction (ex,ey,ez) to the front
template <bool MZ>
__device__ __forceinline__ double link_delta(const double* s, int x, int y, int z, int ex, int ey,
                                             int ez, int n) {
  const int c = col_of<MZ>(x, y, z, n);
  const double a = melt_of<MZ>(y, z) + 0.5;
  const bool along = MZ ? (ez != 0) : (ey != 0);
  if (along) return fabs(s[c] - a);
  const int cn = col_of<MZ>(x + ex, y + ey, z + ez, n);
  return (a - s[c]) / (s[cn] - s[c]);
}

// Conservative front update: the weight of the heat of the interface link of
// cell (x,y,z) whose incoming D3Q7 direction q has its source across the
// front.  A link along the melt axis is charged to its own column, a lateral
// one to the column of its solid cell.  wq: per-column weight.
template <bool MZ>
__device__ __forceinline__ double heat_weight(const double* wq, int x, int y, int z, int q,
                                              bool liquid, int n) {
  const bool along = MZ ? (ez7(q) != 0) : (ey7(q) != 0);
  return wq[(along || !liquid) ? col_of<MZ>(x, y, z, n)
                               : col_of<MZ>(x - ex7(q), y - ey7(q), z - ez7(q), n)];
}

// Fraction of the link from cell (x,y,z) to the source of its incoming D3Q19
// direction q at which the front cuts it, for the interpolated no-slip of f:
// the height on the melt axis and the front (linear between the two columns)
// meet there.  The forward step evaluates the same expression.  num and den
// return its numerator and denominator, d = num / den.
template <bool MZ>
__device__ __forceinline__ double frac19(const double* s, int x, int y, int z, int q, int n,
                                         double& num, double& den) {
  const int a = melt_of<MZ>(y, z);
  const double sc = s[col_of<MZ>(x, y, z, n)];
  const int ea = MZ ? ez19(q) : ey19(q);
  num = (a + 0.5) - sc;
  den = (s[col_of<MZ>(x - ex19(q), y - ey19(q), z - ez19(q), n)] - sc) + ea;
  return num / den;
}

// stored population q of linear cell i = (z n + y) n + x, in FP64 (the
// row-interleaved layout of a distribution with Q directions)
template <int Q, typename Ts>
__device__ __forceinline__ double sv3(const Ts* a, const KParams& P, int q, int x, int y, int z) {
  return (double)static_cast<typename Compute<Ts>::type>(
      a[(((uint64_t)z * (uint32_t)P.n + (uint32_t)y) * Q + q) * P.pitch + (uint32_t)x]);
}
template <int Q, typename Ts>
__device__ __forceinline__ double sv(const Ts* a, const KParams& P, int q, uint32_t i) {
  const uint32_t row = div_n(i, P), x = i - row * (uint32_t)P.n;
  return (double)static_cast<typename Compute<Ts>::type>(
      a[((uint64_t)row * Q + q) * P.pitch + x]);
}

// Fast-path test of the reverse kernels: away from the y and z walls, and
// every cell within two columns and two heights in one phase (the transposed
// streaming reaches the source of a neighbour's link, two cells away).
template <bool MZ>
__device__ __forceinline__ bool adj_fast(const int* cmin2, const int* cmax2, int x, int y, int z,
                                         int n) {
  const int a = melt_of<MZ>(y, z), c = col_of<MZ>(x, y, z, n);
  const bool interior = (y > 0) & (y < n - 1) & (z > 0) & (z < n - 1);
  return interior & (((a + 2) < cmin2[c]) | ((a - 2) >= cmax2[c]));
}

// What the transposed collision needs of the pulled populations: the
// collision is affine in them except through the equilibria and the force,
// which depend on T and u only, so its Jacobian is fixed by T - tref = sum g
// and j = sum e f (of the shifted populations; the shifts add nothing).
struct Macro {
  double Tt = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
  __device__ void add_g(double v) { Tt += v; }
  __device__ void add_f(int q, double v) {
    jx += ex19(q) * v;
    jy += ey19(q) * v;
    jz += ez19(q) * v;
  }
};

// Row partition of the reverse streaming.  With A = min(n - 1,
// max liquid count + 2), a row (height a along the melt axis, o across it)
// with A <= a < n - 1 and 0 < o < n - 1 is away from the walls and every
// cell within two columns and two heights of it is solid: the fast path
// with g alone.  The other rows (every height below A, the top height and
// the two side rows in between) take the full kernels; there are
// front_rows(A, n) of them, enumerated by front_row.
__device__ __forceinline__ bool bulk_solid_row(int a, int o, int A, int n) {
  return (a >= A) & (a < n - 1) & (o > 0) & (o < n - 1);
}
__device__ __forceinline__ int front_rows(int A, int n) { return A * n + n + 2 * (n - 1 - A); }
__device__ __forceinline__ void front_row(int r, int A, const KParams& P, int& a, int& o) {
  const int n = P.n;
  if (r < A * n) {
    a = (int)div_n((uint32_t)r, P);
    o = r - a * n;
  } else if (r < A * n + n) {
    a = n - 1;
    o = r - A * n;
  } else {
    const int k = r - A * n - n;
    a = A + (k >> 1);
    o = (k & 1) ? n - 1 : 0;
  }
}

// The bound A of the row partition from the largest liquid count m of the
// lattice.
__device__ __forceinline__ int row_bound(int m, int n) { return m + 2 < n - 1 ? m + 2 : n - 1; }

// The reverse collision needs no such margin: it is local to a cell, and a
// solid cell's needs no state (at rest the heat collision is linear in g).
// So every row at a height a >= m, all of whose cells are solid, takes the
// g-only kernel, wall rows included; the m n rows below (heights a < m,
// every o) take the full one.
__device__ __forceinline__ bool solid_collide_row(int a, int m) { return a >= m; }

// Pairing of two consecutive reverse steps (lattices above the shared-launch
// size).  A row that is bulk-solid for the transposed streaming of state t+1
// (largest liquid count ms) and at least three heights above the largest
// liquid count mc of state t, so that no node of state t's front adjoint lies
// in it, skips that streaming: the reverse collision of state t gathers the
// seven values from the neighbours' adjoints itself, the values the
// streaming would have stored.  56 instead of 112 bytes per cell in FP32.
__device__ __forceinline__ bool paired_row(int a, int o, int ms, int mc, int n) {
  return bulk_solid_row(a, o, row_bound(ms, n), n) && a >= mc + 3;
}

// Phase bookkeeping of the states of a segment, one state per grid plane z
// (state s[z]), in one pass over its columns: the liquid count of each column
// (from its front), the minimum and maximum count over the 5x5 columns around
// it (the columns in the box), and the largest count of the lattice.  The
// outputs of state z start at z n^2 (cnt, cmin2, cmax2) and at rmax[z].  None
// of this depends on the adjoints, so one launch serves a whole segment once
// its states are recomputed.  A workgroup covers kPartRows x 64 columns; its
// largest count is reduced in LDS and merged into rmax[z] by one atomic
// maximum (device-scope atomics on one address serialize, so there is one
// per workgroup), so rmax must be zero at launch.
constexpr int kPartRows = 8;
__global__ __launch_bounds__(64 * kPartRows) void k_adj_partition(
    const double* const* __restrict__ states, int* __restrict__ cnt, int* __restrict__ cmin2,
    int* __restrict__ cmax2, int* __restrict__ rmax, int n) {
  // counts of the (kPartRows + 4) x (64 + 4) columns the windows cover, each
  // computed once; -1 marks a column outside the box
  __shared__ int tile[kPartRows + 4][64 + 4];
  __shared__ int wmax[kPartRows];
  const int x0 = blockIdx.x * 64, o0 = blockIdx.y * kPartRows;
  const int tid = threadIdx.y * 64 + threadIdx.x;
  const size_t nn = (size_t)n * n, zofs = blockIdx.z * nn;
  const double* __restrict__ s = states[blockIdx.z];
  for (int i = tid; i < (kPartRows + 4) * (64 + 4); i += 64 * kPartRows) {
    const int r = i / (64 + 4), j = i - r * (64 + 4);
    const int oo = o0 + r - 2, xx = x0 + j - 2;
    const bool in = oo >= 0 && oo < n && xx >= 0 && xx < n;
    tile[r][j] = in ? count_liquid(s[oo * n + xx], n) : -1;
  }
  __syncthreads();
  const int x = x0 + threadIdx.x, o = o0 + threadIdx.y;
  int own = 0;
  if (x < n && o < n) {
    int lo = n, hi = 0;
#pragma unroll
    for (int r = 0; r < 5; ++r)
#pragma unroll
      for (int dx = 0; dx < 5; ++dx) {
        const int c = tile[threadIdx.y + r][threadIdx.x + dx];
        if (c < 0) continue;
        lo = c < lo ? c : lo;
        hi = c > hi ? c : hi;
      }
    own = tile[threadIdx.y + 2][threadIdx.x + 2];
    cnt[zofs + o * n + x] = own;
    cmin2[zofs + o * n + x] = lo;
    cmax2[zofs + o * n + x] = hi;
  }
  int m = own;  // lanes outside the box hold 0, below every count's maximum
  for (int w = 32; w > 0; w >>= 1) {
    const int v = __shfl_xor(m, w);
    m = v > m ? v : m;
  }
  if (threadIdx.x == 0) wmax[threadIdx.y] = m;
  __syncthreads();
  if (tid == 0) {
    for (int w = 1; w < kPartRows; ++w) m = wmax[w] > m ? wmax[w] : m;
    atomicMax(rmax + blockIdx.z, m);
  }
}

// pulled populations of a cell on the fast path: regular pulls, bounce-back
// at the adiabatic / no-slip x walls only
// (Each source index is selected before its load, and every load of a cell
// is issued before the first use, so the loads are in flight together.)
template <typename Ts, bool FLOW>
__device__ __forceinline__ void pull_fast(const Ts* f, const Ts* g, int x, int y, int z,
                                          bool liquid, const KParams& P, Macro& M) {
  using C = typename Compute<Ts>::type;
  const int n = P.n;
  Ts gv[7];
#pragma unroll
  for (int q = 0; q < 7; ++q) {
    const int sx = x - ex7(q);
    gv[q] = g[(unsigned)sx < (unsigned)n ? pop_index(P, 7, q, sx, y - ey7(q), z - ez7(q))
                                         : pop_index(P, 7, opp7(q), x, y, z)];
  }
#pragma unroll
  for (int q = 0; q < 7; ++q) M.add_g((double)static_cast<C>(gv[q]));
  if (FLOW && liquid) {
    Ts fv[19];
#pragma unroll
    for (int q = 1; q < 19; ++q) {  // the rest population carries no momentum
      const int sx = x - ex19(q);
      fv[q] = f[(unsigned)sx < (unsigned)n ? pop_index(P, 19, q, sx, y - ey19(q), z - ez19(q))
                                           : pop_index(P, 19, opp19(q), x, y, z)];
    }
#pragma unroll
    for (int q = 1; q < 19; ++q) M.add_f(q, (double)static_cast<C>(fv[q]));
  }
}

// Transposed streaming of one cell on the fast path (one phase all around):
// stored population p before the step was read by the regular pull of the
// neighbour x + e_p, or, at an x wall, by this cell's bounce-back into the
// reverse direction.  Indices first, then all Q loads, then the stores.
template <int Q, typename Lam>
__device__ __forceinline__ void push_fast(const Lam* __restrict__ lh, Lam* __restrict__ l0,
                                          const Geo& G, size_t nc, int x, int y, int z,
                                          uint32_t i) {
  Lam v[Q];
#pragma unroll
  for (int p = 0; p < Q; ++p) {
    const int ex = Q == 7 ? ex7(p) : ex19(p), ey = Q == 7 ? ey7(p) : ey19(p),
              ez = Q == 7 ? ez7(p) : ez19(p), q = Q == 7 ? opp7(p) : opp19(p);
    const bool in = (unsigned)(x + ex) < (unsigned)G.n;
    v[p] = lh[in ? (size_t)p * nc + G.cell(x + ex, y + ey, z + ez) : (size_t)q * nc + i];
  }
#pragma unroll
  for (int p = 0; p < Q; ++p) l0[(size_t)p * nc + i] = v[p];
}

// pulled (pre-collision) shifted populations of one cell (general path), in
// FP64, reduced to T and j
template <typename Ts, bool FLOW, bool MZ, bool EXT>
__device__ void pull_cell(const Ts* f, const Ts* g, const double* s, const double* th,
                          const int* cnt, int x, int y, int z, bool liquid, const KParams& P,
                          Macro& M) {
  const Geo G{P.n, (uint32_t)P.n * (uint32_t)P.n};
  const int n = P.n;
  const uint32_t i = G.cell(x, y, z);
  const double w = 0.125, wTm = w * (P.t_m - P.tref);
  // liquid counts of the 3x3 columns around this one, loaded together
  // (clamped at the walls; only in-box cells are asked for); the offsets are
  // constants of the unrolled loops, so each phase test reads a register
  const int o = MZ ? y : z;
  int nbc[9];
  {
    auto cl = [&](int v) { return v < 0 ? 0 : (v > n - 1 ? n - 1 : v); };
#pragma unroll
    for (int k = 0; k < 9; ++k) nbc[k] = cnt[cl(o + k / 3 - 1) * n + cl(x + k % 3 - 1)];
  }
  auto liq = [&](int X, int Y, int Z) -> bool {
    return melt_of<MZ>(Y, Z) < nbc[((MZ ? Y : Z) - o + 1) * 3 + (X - x) + 1];
  };
  // Every value the terms of g below may read is loaded first, for the seven
  // directions together (positions clamped into the box), so the loads are
  // in flight at once instead of one direction's after the other's: the
  // cell's own populations, the pulled one, the one of the cell behind, the
  // front of the column across a lateral link, the hot-wall temperature.
  const int col = col_of<MZ>(x, y, z, n);
  const double s_c = s[col], th_c = th[col];
  auto cl = [&](int v) { return v < 0 ? 0 : (v > n - 1 ? n - 1 : v); };
  double own[7], src[7], beh[7], sn[7];
#pragma unroll
  for (int q = 0; q < 7; ++q) {
    const int ex = ex7(q), ey = ey7(q), ez = ez7(q), p = opp7(q);
    own[q] = sv3<7>(g, P, q, x, y, z);
    src[q] = q == 0 ? 0.0 : sv3<7>(g, P, q, cl(x - ex), cl(y - ey), cl(z - ez));
    beh[q] = q == 0 ? 0.0 : sv3<7>(g, P, p, cl(x + ex), cl(y + ey), cl(z + ez));
    const bool along = MZ ? (ez != 0) : (ey != 0);
    sn[q] = (q == 0 || along) ? s_c : s[col_of<MZ>(cl(x - ex), cl(y - ey), cl(z - ez), n)];
  }
  const double a0 = melt_of<MZ>(y, z) + 0.5;
#pragma unroll
  for (int q = 0; q < 7; ++q) {
    const int ex = ex7(q), ey = ey7(q), ez = ez7(q), p = opp7(q);
    const int sx = x - ex, sy = y - ey, sz = z - ez;
    double v;
    if (q == 0) {
      v = own[0];  // the rest population stays in its cell
    } else if (!G.in(sx, sy, sz)) {
      const int sa = melt_of<MZ>(sy, sz);
      const double gp = own[p];
      if (sa < 0)
        v = -gp + 2.0 * w * (th_c - P.tref);
      else if (!MZ && sa >= n)
        v = -gp + 2.0 * w * (P.t_c - P.tref);
      else
        v = gp;
    } else if (liq(sx, sy, sz) == liquid) {
      v = src[q];
    } else {
      // link_delta, term for term
      const bool along = MZ ? (ez != 0) : (ey != 0);
      const double d = along ? fabs(s_c - a0) : (a0 - s_c) / (sn[q] - s_c);
      const double gp = own[p];
      if (d < 0.5) {
        const int bx = x + ex, by = y + ey, bz = z + ez;
        const bool behind = G.in(bx, by, bz) && liq(bx, by, bz) == liquid;
        v = behind ? -(2.0 * d * gp + (1.0 - 2.0 * d) * beh[q]) + 2.0 * wTm : -gp + 2.0 * wTm;
      } else {
        v = -gp / (2.0 * d) + (2.0 * d - 1.0) / (2.0 * d) * own[q] + wTm / d;
      }
    }
    M.add_g(v);
  }
  if (FLOW && liquid) {
#pragma unroll
    for (int q = 1; q < 19; ++q) {
      const int sx = x - ex19(q), sy = y - ey19(q), sz = z - ez19(q);
      const bool inb = G.in(sx, sy, sz);
      const bool ok = inb && liq(sx, sy, sz);
      // the pulled population or the bounce-back of the cell's own: one load
      // from the selected position, not a branch per direction
      double v = sv3<19>(f, P, ok ? q : opp19(q), ok ? sx : x, ok ? sy : y, ok ? sz : z);
      if (EXT && P.f_wall && inb && !ok) {  // interpolated no-slip at the front
        double num, den;
        const double d = frac19<MZ>(s, x, y, z, q, n, num, den);
        if (d < 0.5) {
          const int bx = x + ex19(q), by = y + ey19(q), bz = z + ez19(q);
          if (G.in(bx, by, bz) && liq(bx, by, bz))
            v = 2.0 * d * v + (1.0 - 2.0 * d) * sv<19>(f, P, opp19(q), G.cell(bx, by, bz));
        } else {
          v = v / (2.0 * d) + (2.0 * d - 1.0) / (2.0 * d) * sv<19>(f, P, q, i);
        }
      }
      M.add_f(q, v);
    }
  }
}

// Transposed collision Jacobian of one cell at the state (T, u) of its
// pulled populations: (lfo, lgo) -> (lfl, lgl)
template <bool FLOW>
__device__ void collide_adjoint(const Macro& M, bool liquid, const KParams& P,
                                const double (&lfo)[19], const double (&lgo)[7],
                                double (&lfl)[19], double (&lgl)[7]) {
  const bool fluid = FLOW && liquid;
  const double Tt = M.Tt;  // T - tref
  const double T = Tt + P.tref;
  double ux = 0.0, uy = 0.0, uz = 0.0, Fz = 0.0;
  if (fluid) {
    Fz = P.gbeta * (Tt + P.tref - P.t0);
    ux = M.jx;
    uy = M.jy;
    uz = M.jz + 0.5 * Fz;
  }
  // ---- energy distribution: g' = N^T D^-1 [(I - Q) N gl + Q n_eq(T, u)] ----
  const double qj = liquid ? P.q_j : P.q_js, qe = liquid ? P.q_e : P.q_es;
  const double Q[7] = {0.0, qj, qj, qj, qe, qe, qe};
  double lns[7], ln[7], lne[7];
  m7(lgo, lns);
  for (int k = 0; k < 7; ++k) {
    lns[k] *= kInvD7[k];
    ln[k] = (1.0 - Q[k]) * lns[k];
    lne[k] = Q[k] * lns[k];
  }
  double lT = ux * lne[1] + uy * lne[2] + uz * lne[3] + 0.75 * lne[4];
  double lux = T * lne[1], luy = T * lne[2], luz = T * lne[3];
  if (fluid) {
    // ---- flow: f' = M^T D^-1 [m - S (m - m_eq) + (I - S/2) F_m] ----
    const double sv_ = P.s_nu;
    const double S[19] = {0.0, 1.19, 1.4, 0.0, 1.2, 0.0, 1.2, 0.0, 1.2, sv_,
                          1.4, sv_,  1.4, sv_, sv_, sv_, 1.98, 1.98, 1.98};
    double lms[19], lm[19], le[19], lF[19];
    m19(lfo, lms);
    for (int k = 0; k < 19; ++k) {
      lms[k] *= kInvD19[k];
      lm[k] = (1.0 - S[k]) * lms[k];
      le[k] = S[k] * lms[k];
      lF[k] = (1.0 - 0.5 * S[k]) * lms[k];
    }
    // equilibria (deviation form, rho0 = 1): dependence on drho and u
    const double aq = 19.0 * le[1] - 5.5 * le[2];
    const double a9 = le[9] - 0.5 * le[10], a11 = le[11] - 0.5 * le[12];
    const double ldrho = -11.0 * le[1] + 3.0 * le[2];
    lux += 2.0 * ux * aq - 2.0 / 3.0 * le[4] + 4.0 * ux * a9 + uy * le[13] + uz * le[15];
    luy += 2.0 * uy * aq - 2.0 / 3.0 * le[6] - 2.0 * uy * a9 + 2.0 * uy * a11 + ux * le[13] +
           uz * le[14];
    luz += 2.0 * uz * aq - 2.0 / 3.0 * le[8] - 2.0 * uz * a9 - 2.0 * uz * a11 + uy * le[14] +
           ux * le[15];
    // forcing moments with F = (0, 0, Fz)
    const double cF = 38.0 * lF[1] - 11.0 * lF[2] - 2.0 * lF[9] + lF[10] - 2.0 * lF[11] + lF[12];
    luz += Fz * cF;
    luy += Fz * lF[14];
    lux += Fz * lF[15];
    double lFz = uz * cF + lF[7] - 2.0 / 3.0 * lF[8] + uy * lF[14] + ux * lF[15];
    // u = j + F/2, F_z = gbeta (T - t0)
    lFz += 0.5 * luz;
    lT += P.gbeta * lFz;
    lm[0] += ldrho;
    lm[3] += lux;
    lm[5] += luy;
    lm[7] += luz;
    m19t(lm, lfl);
  } else {
    for (int q = 0; q < 19; ++q) lfl[q] = 0.0;
  }
  m7t(ln, lgl);
  for (int q = 0; q < 7; ++q) lgl[q] += lT;
}

// ---- front velocity and its derivatives (node selection frozen) ----
// Every array below is indexed by constants once the loops are unrolled, so
// the whole record stays in registers.  Node slots 0 and 1 hold the liquid
// side, 2 and 3 the solid side; a slot taken by a wall point is not used.
struct VDer {
  double V;
  bool use[4];
  uint32_t node[4];
  double dT[4];
  double dth;
  int col[5];
  double ds[5];
};

// Slope at xi = 0 of the one-sided quadratic through (0, tm), (xi0, T0),
// (xi1, T1) (k = 2), or of the chord to (xi0, T0) (k = 1), with its
// derivatives with respect to the node temperatures and distances.
__device__ __forceinline__ double slope_der(int k, double xi0, double xi1, double T0, double T1,
                                            double tm, double& dT0, double& dT1, double& dxi0,
                                            double& dxi1) {
  dT0 = dT1 = dxi0 = dxi1 = 0.0;
  if (k >= 2) {
    const double A = T0 - tm, B = T1 - tm;
    const double D = xi0 * xi1 * (xi1 - xi0);
    const double num = A * xi1 * xi1 - B * xi0 * xi0;
    const double dD0 = xi1 * xi1 - 2.0 * xi0 * xi1;
    const double dD1 = 2.0 * xi0 * xi1 - xi0 * xi0;
    dT0 = xi1 * xi1 / D;
    dT1 = -xi0 * xi0 / D;
    dxi0 = (-2.0 * B * xi0 * D - num * dD0) / (D * D);
    dxi1 = (2.0 * A * xi1 * D - num * dD1) / (D * D);
    return num / D;
  }
  if (k == 1 && xi0 > 0.0) {
    dT0 = 1.0 / xi0;
    dxi0 = -(T0 - tm) / (xi0 * xi0);
    return (T0 - tm) / xi0;
  }
  return 0.0;
}

template <typename Ts, typename Lam, bool MZ>
__device__ __forceinline__ void front_der(const Ts* g1, const double* s, const double* th, int c,
                                          const KParams& P, VDer& d, const Lam* lg1,
                                          Lam (&old)[4][7]) {
  const int n = P.n;
  const double sc = s[c];
  // front slopes by central differences, mirrored at the walls, and the
  // hot-wall temperature: loads that depend on nothing else, issued first
  const int o = (int)div_n((uint32_t)c, P), x = c - o * n;
  const int cxp = o * n + (x + 1 < n ? x + 1 : x), cxm = o * n + (x > 0 ? x - 1 : x);
  const int cop = (o + 1 < n ? o + 1 : o) * n + x, com = (o > 0 ? o - 1 : o) * n + x;
  const double dsx = 0.5 * (s[cxp] - s[cxm]), dso = 0.5 * (s[cop] - s[com]);
  const double thc = th[c];
  const int cnt = count_liquid(sc, n);
  auto Tcell = [&](uint32_t i) {
    double acc = 0.0;
    for (int q = 0; q < 7; ++q) acc += sv<7>(g1, P, q, i);
    return acc + P.tref;
  };
  // The nodes: on each side the two nearest centres at distance >= 1/2 from
  // the front.  The nearest liquid one is at height cnt - 1 or, if that
  // centre is closer than 1/2, cnt - 2; the nearest solid one at cnt or
  // cnt + 1.  The four candidate cells are known from the front alone, so
  // their temperatures are loaded together (heights clamped into the box;
  // a candidate outside it is not used).
  int at = cnt - 1;
  if (at >= 0 && sc - (at + 0.5) < 0.5) --at;
  int ab = cnt;
  if (ab < n && (ab + 0.5) - sc < 0.5) ++ab;
  auto cell_at = [&](int a) {
    return cell_in_column<MZ>(c, a < 0 ? 0 : (a > n - 1 ? n - 1 : a), P);
  };
  const uint32_t cl0 = cell_at(at), cl1 = cell_at(at - 1), cs0 = cell_at(ab), cs1 = cell_at(ab + 1);
  // the adjoints at the same four cells, which the caller updates: a node
  // that is used is one of these candidates
  const uint32_t cand[4] = {cl0, cl1, cs0, cs1};
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int q = 0; q < 7; ++q) old[k][q] = lg1[(size_t)q * P.ncell + cand[k]];
  const double Tl0 = Tcell(cl0), Tl1 = Tcell(cl1), Ts0 = Tcell(cs0), Ts1 = Tcell(cs1);

  // liquid side: those nodes toward the heated wall, then the wall itself
  double xi0 = 0.0, xi1 = 0.0, T0 = 0.0, T1 = 0.0;
  uint32_t nd0 = 0, nd1 = 0;
  int k = 0, wall_l = -1;
  if (at >= 0) {
    xi0 = sc - (at + 0.5);
    nd0 = cl0;
    T0 = Tl0;
    k = 1;
    if (at - 1 >= 0) {
      xi1 = sc - ((at - 1) + 0.5);
      nd1 = cl1;
      T1 = Tl1;
      k = 2;
    }
  }
  if (k < 2) {
    if (k == 0) { xi0 = sc; T0 = thc; } else { xi1 = sc; T1 = thc; }
    wall_l = k;
    ++k;
  }
  const int kl = k;
  double dTl0, dTl1, dxil0, dxil1;
  const double sl = slope_der(kl, xi0, xi1, T0, T1, P.t_m, dTl0, dTl1, dxil0, dxil1);
  d.use[0] = kl > 0 && wall_l != 0;
  d.use[1] = kl > 1 && wall_l != 1;
  d.node[0] = nd0;
  d.node[1] = nd1;

  // solid side: the nodes beyond the front, then the cold wall (melt axis y)
  xi0 = xi1 = T0 = T1 = 0.0;
  nd0 = nd1 = 0;
  k = 0;
  int wall_s = -1;
  if (ab < n) {
    xi0 = (ab + 0.5) - sc;
    nd0 = cs0;
    T0 = Ts0;
    k = 1;
    if (ab + 1 < n) {
      xi1 = ((ab + 1) + 0.5) - sc;
      nd1 = cs1;
      T1 = Ts1;
      k = 2;
    }
  }
  if (k < 2 && !MZ) {
    if (k == 0) { xi0 = n - sc; T0 = P.t_c; } else { xi1 = n - sc; T1 = P.t_c; }
    wall_s = k;
    ++k;
  }
  const int ks = k;
  double dTs0, dTs1, dxis0, dxis1;
  const double ss = slope_der(ks, xi0, xi1, T0, T1, P.t_m, dTs0, dTs1, dxis0, dxis1);
  d.use[2] = ks > 0 && wall_s != 0;
  d.use[3] = ks > 1 && wall_s != 1;
  d.node[2] = nd0;
  d.node[3] = nd1;

  const double Pf = 1.0 + dsx * dsx + dso * dso;
  const double K = P.alpha * P.ste / P.dT, kap = P.kappa;  // Eq. (6): kappa on the solid side
  d.V = Pf * K * (kap * ss + sl);
  d.dT[0] = Pf * K * dTl0;
  d.dT[1] = Pf * K * dTl1;
  d.dT[2] = Pf * K * kap * dTs0;
  d.dT[3] = Pf * K * kap * dTs1;
  // the hot-wall temperature enters through the liquid side's wall point
  d.dth = wall_l == 0 ? Pf * K * dTl0 : (wall_l == 1 ? Pf * K * dTl1 : 0.0);
  // unused slopes and distances are zero, so every sum keeps its terms in order
  const double dself = dxil0 + dxil1 - kap * dxis0 - kap * dxis1;
  const double KG = K * (kap * ss + sl);
  d.col[0] = c;
  d.ds[0] = Pf * K * dself;
  d.col[1] = cxp;
  d.ds[1] = KG * dsx;
  d.col[2] = cxm;
  d.ds[2] = -KG * dsx;
  d.col[3] = cop;
  d.ds[3] = KG * dso;
  d.col[4] = com;
  d.ds[4] = -KG * dso;
}

// ---------------------------------------------------------------- kernels
// Adjoint buffers are dense FP64 arrays [q][n^3] (populations) and [n^2].

template <typename Ts, typename Lam, bool FLOW, bool MZ>
__global__ __launch_bounds__(64) void k_adj_front(const double* __restrict__ s0, const Ts* __restrict__ g1,
                            const double* __restrict__ th, const double* __restrict__ ls1, Lam* __restrict__ lg1,
                            double* __restrict__ out5, double* __restrict__ own,
                            double* __restrict__ lth, KParams P) {
  const int n = P.n;
  const int x = blockIdx.x * blockDim.x + threadIdx.x, o = blockIdx.y;
  if (x >= n) return;
  const int c = o * n + x;
  const size_t nc = P.ncell, nn = (size_t)n * n;
  VDer d;
  Lam old[4][7];
  front_der<Ts, Lam, MZ>(g1, s0, th, c, P, d, lg1, old);
  const double v = s0[c] + d.V;  // the unclamped update, recomputed as the step did
  const double l = ls1[c];
  if (v < 0.0 || v > (double)n) {  // clamped: no dependence
    own[c] = 0.0;
    for (int j = 0; j < 5; ++j) out5[j * nn + c] = 0.0;
    return;
  }
  own[c] = l;
  // The 28 updated values are distinct (other direction or other cell of this
  // column, and no other column touches these cells), so their loads were
  // issued with the node temperatures, before the first store.  An unused
  // slot stores nothing.
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (d.use[k])
#pragma unroll
      for (int q = 0; q < 7; ++q)
        lg1[(size_t)q * nc + d.node[k]] = (Lam)((double)old[k][q] + l * d.dT[k]);
  for (int j = 0; j < 5; ++j) out5[j * nn + c] = l * d.ds[j];
  lth[c] += l * d.dth;
}

// s contributions: own slot 0; slot 1 of the x-1 neighbour (its x+1 is this
// column), slot 2 of x+1, slot 3 of o-1, slot 4 of o+1; at the walls the
// mirrored slots of the column itself
// Reverse of the conservative front update s' = clamp(s + heat Ste / dT):
// the direct term of s, and the weight by which each column's interface heat
// enters J (zero where the front was clamped).  out5 is cleared so that the
// gather below adds nothing else.
__global__ __launch_bounds__(64) void k_adj_front_heat(const double* __restrict__ s0, const double* __restrict__ heat,
                                 const double* __restrict__ ls1, double* __restrict__ wq,
                                 double* __restrict__ own, double* __restrict__ out5, KParams P) {
  const int n = P.n;
  const int x = blockIdx.x * blockDim.x + threadIdx.x, o = blockIdx.y;
  if (x >= n) return;
  const int nn = n * n, c = o * n + x;
  const double v = s0[c] + heat[c] * P.ste / P.dT;
  const bool clamped = v < 0.0 || v > (double)n;
  wq[c] = clamped ? 0.0 : ls1[c] * P.ste / P.dT;
  own[c] = clamped ? 0.0 : ls1[c];
  for (int k = 0; k < 5; ++k) out5[(size_t)k * nn + c] = 0.0;
}

// the front part of the adjoint of s for column (x, o): its own term and the
// contributions its four neighbours left for it in out5
__device__ __forceinline__ double front_gather(const double* __restrict__ own,
                                               const double* __restrict__ out5, int x, int o,
                                               int n) {
  const size_t nn = (size_t)n * n;
  const int c = o * n + x;
  double acc = own[c] + out5[0 * nn + c];
  if (x > 0) acc += out5[1 * nn + c - 1]; else acc += out5[2 * nn + c];
  if (x < n - 1) acc += out5[2 * nn + c + 1]; else acc += out5[1 * nn + c];
  if (o > 0) acc += out5[3 * nn + c - n]; else acc += out5[4 * nn + c];
  if (o < n - 1) acc += out5[4 * nn + c + n]; else acc += out5[3 * nn + c];
  return acc;
}

// reverse collision of one cell (any row)
template <typename Ts, typename Lam, bool FLOW, bool MZ, bool EXT>
__device__ __forceinline__ void adj_collide_cell(
    const Ts* __restrict__ f0, const Ts* __restrict__ g0, const double* __restrict__ s0,
    const double* __restrict__ s1, const double* __restrict__ th, const int* __restrict__ cnt,
    const int* __restrict__ cmin2, const int* __restrict__ cmax2, const Lam* __restrict__ lf1,
    const Lam* __restrict__ lg1, Lam* __restrict__ lfh, Lam* __restrict__ lgh, const KParams& P,
    int x, int y, int z) {
  const int n = P.n;
  const size_t nc = P.ncell;
  const uint32_t i = ((uint32_t)z * n + y) * n + x;
  const bool liquid = liquid_at<MZ>(cnt, x, y, z, n);
  // f of a cell that is solid after the step is dead data (never read; a
  // melting cell is refilled), so its adjoint is zero and is not stored
  const bool live1 = liquid && melt_of<MZ>(y, z) < count_liquid(s1[col_of<MZ>(x, y, z, n)], n);
  // the adjoints after the step are loaded before the state pull, so the two
  // round trips overlap
  Lam lfr[19], lgr[7];
  for (int q = 0; q < 19; ++q) lfr[q] = (FLOW && live1) ? lf1[(size_t)q * nc + i] : Lam(0);
  for (int q = 0; q < 7; ++q) lgr[q] = lg1[(size_t)q * nc + i];
  Macro M;
  if (__all(adj_fast<MZ>(cmin2, cmax2, x, y, z, n)))
    pull_fast<Ts, FLOW>(f0, g0, x, y, z, liquid, P, M);
  else
    pull_cell<Ts, FLOW, MZ, EXT>(f0, g0, s0, th, cnt, x, y, z, liquid, P, M);
  double lfo[19], lgo[7], lfl[19], lgl[7];
  for (int q = 0; q < 19; ++q) lfo[q] = (double)lfr[q];
  for (int q = 0; q < 7; ++q) lgo[q] = (double)lgr[q];
  collide_adjoint<FLOW>(M, liquid, P, lfo, lgo, lfl, lgl);
  if (FLOW && liquid)  // read only at liquid cells
    for (int q = 0; q < 19; ++q) lfh[(size_t)q * nc + i] = (Lam)lfl[q];
  for (int q = 0; q < 7; ++q) lgh[(size_t)q * nc + i] = (Lam)lgl[q];
}

// The rows with a liquid cell, the m n rows at heights below the largest
// liquid count m, visited by a grid of gridDim.y row slots (this kernel
// needs many registers, so its waves are not spent on rows it would skip).
template <typename Ts, typename Lam, bool FLOW, bool MZ, bool EXT>
__device__ __forceinline__ void adj_collide_rows(
    int slot, int nslots, int x, const Ts* __restrict__ f0, const Ts* __restrict__ g0,
    const double* __restrict__ s0, const double* __restrict__ s1, const double* __restrict__ th,
    const int* __restrict__ cnt, const int* __restrict__ cmin2, const int* __restrict__ cmax2,
    const int* __restrict__ rowb, const Lam* __restrict__ lf1, const Lam* __restrict__ lg1,
    Lam* __restrict__ lfh, Lam* __restrict__ lgh, const KParams& P) {
  const int n = P.n;
  const int R = rowb[0] * n;
  for (int r = slot; r < R; r += nslots) {
    const int a = (int)div_n((uint32_t)r, P), o = r - a * n;
    if (x < n)
      adj_collide_cell<Ts, Lam, FLOW, MZ, EXT>(f0, g0, s0, s1, th, cnt, cmin2, cmax2, lf1, lg1,
                                               lfh, lgh, P, x, MZ ? o : a, MZ ? a : o);
  }
}

template <typename Ts, typename Lam, bool FLOW, bool MZ, bool EXT>
__global__ __launch_bounds__(256) void k_adj_collide(
    const Ts* __restrict__ f0, const Ts* __restrict__ g0, const double* __restrict__ s0,
    const double* __restrict__ s1, const double* __restrict__ th, const int* __restrict__ cnt,
    const int* __restrict__ cmin2, const int* __restrict__ cmax2, const int* __restrict__ rowb,
    const Lam* __restrict__ lf1, const Lam* __restrict__ lg1, Lam* __restrict__ lfh,
    Lam* __restrict__ lgh, KParams P) {
  adj_collide_rows<Ts, Lam, FLOW, MZ, EXT>(blockIdx.y, gridDim.y,
                                           blockIdx.x * blockDim.x + threadIdx.x, f0, g0, s0, s1,
                                           th, cnt, cmin2, cmax2, rowb, lf1, lg1, lfh, lgh, P);
}

// The all-solid rows k_adj_collide leaves out: only the energy distribution
// is reversed, with few registers, so these rows (most of a melting state)
// run at full occupancy.  A solid cell is at rest, and at u = 0 the heat
// collision is linear in g: its transpose needs no state, so the kernel reads
// the 7 adjoints and writes 7 (56 B per cell in FP32).
template <typename Lam, bool MZ>
__device__ __forceinline__ void adj_collide_solid_row(int x, int y, int z,
                                                      const int* __restrict__ rowb,
                                                      const int* __restrict__ rowb_prev,
                                                      const Lam* __restrict__ lg1,
                                                      const Lam* __restrict__ lgh_prev,
                                                      Lam* __restrict__ lgh, const KParams& P) {
  const int n = P.n, a = melt_of<MZ>(y, z);
  if (x >= n || !solid_collide_row(a, rowb[0])) return;
  const size_t nc = P.ncell;
  const uint32_t i = ((uint32_t)z * n + y) * n + x;
  const Macro M;  // T enters only the flow part, which a solid cell skips
  double lfo[19] = {}, lgo[7], lfl[19], lgl[7];
  if (rowb_prev && paired_row(a, MZ ? y : z, rowb_prev[0], rowb[0], n)) {
    // the transposed streaming of state t+1 (push_fast's gather), in place of
    // its stored result
    const Geo G{n, (uint32_t)n * (uint32_t)n};
    Lam v[7];
#pragma unroll
    for (int p = 0; p < 7; ++p) {
      const int ex = ex7(p), ey = ey7(p), ez = ez7(p);
      const bool in = (unsigned)(x + ex) < (unsigned)n;
      v[p] = lgh_prev[in ? (size_t)p * nc + G.cell(x + ex, y + ey, z + ez)
                         : (size_t)opp7(p) * nc + i];
    }
#pragma unroll
    for (int p = 0; p < 7; ++p) lgo[p] = (double)v[p];
  } else {
    for (int q = 0; q < 7; ++q) lgo[q] = (double)lg1[(size_t)q * nc + i];
  }
  collide_adjoint<false>(M, false, P, lfo, lgo, lfl, lgl);
  for (int q = 0; q < 7; ++q) lgh[(size_t)q * nc + i] = (Lam)lgl[q];
}

template <typename Lam, bool MZ>
__global__ __launch_bounds__(256) void k_adj_collide_solid(
    const int* __restrict__ rowb, const int* __restrict__ rowb_prev, const Lam* __restrict__ lg1,
    const Lam* __restrict__ lgh_prev, Lam* __restrict__ lgh, KParams P) {
  adj_collide_solid_row<Lam, MZ>(blockIdx.x * blockDim.x + threadIdx.x, blockIdx.y, blockIdx.z,
                                 rowb, rowb_prev, lg1, lgh_prev, lgh, P);
}

// Transposed streaming of one cell outside the bulk-solid rows.
template <typename Ts, typename Lam, bool FLOW, bool MZ, bool EXT>
__device__ __forceinline__ void adj_stream_cell(
    const double* __restrict__ s0, const int* __restrict__ cnt, const int* __restrict__ cmin2,
    const int* __restrict__ cmax2, const Lam* __restrict__ lfh, const Lam* __restrict__ lgh,
    Lam* __restrict__ lf0, Lam* __restrict__ lg0, const double* __restrict__ wq,
    const KParams& P, int x, int y, int z) {
  const int n = P.n;
  const Geo G{n, (uint32_t)n * (uint32_t)n};
  const size_t nc = P.ncell;
  const uint32_t i = G.cell(x, y, z);
  const bool L = liquid_at<MZ>(cnt, x, y, z, n);
  auto LG = [&](int q, uint32_t j) { return (double)lgh[(size_t)q * nc + j]; };

  if (__all(adj_fast<MZ>(cmin2, cmax2, x, y, z, n))) {
    push_fast<7>(lgh, lg0, G, nc, x, y, z, i);
    if (FLOW && L) push_fast<19>(lfh, lf0, G, nc, x, y, z, i);
    return;
  }

  // The liquid counts the phase tests below ask for, loaded together: the
  // 3x3 columns around this one and the four at distance two along the
  // lateral axes (indices clamped at the walls; only in-box columns are
  // asked for).  The offsets are constants of the unrolled loops, so each
  // test reads a register.
  const int o = MZ ? y : z;
  int nbc[13];
  {
    auto cl = [&](int v) { return v < 0 ? 0 : (v > n - 1 ? n - 1 : v); };
#pragma unroll
    for (int k = 0; k < 9; ++k) nbc[k] = cnt[cl(o + k / 3 - 1) * n + cl(x + k % 3 - 1)];
    nbc[9] = cnt[o * n + cl(x - 2)];
    nbc[10] = cnt[o * n + cl(x + 2)];
    nbc[11] = cnt[cl(o - 2) * n + x];
    nbc[12] = cnt[cl(o + 2) * n + x];
  }
  // phase of the in-box cell (X, Y, Z) within those columns
  auto liq = [&](int X, int Y, int Z) -> bool {
    const int dx = X - x, dob = (MZ ? Y : Z) - o;
    const int k = dx == -2 ? 9 : dx == 2 ? 10 : dob == -2 ? 11 : dob == 2 ? 12
                                                                      : (dob + 1) * 3 + dx + 1;
    return melt_of<MZ>(Y, Z) < nbc[k];
  };

  // Every value the terms below may read is loaded before the tests that
  // pick them (indices selected or clamped into the box), so the loads of a
  // direction are in flight together: the adjoints at this cell and at
  // x + e_p, and the fronts of this column and of the columns at x + e_p,
  // x - e_p and x + 2 e_p (this column itself for a link along the melt
  // axis).  The link fractions are those of link_delta, term for term.
  const double s_own = s0[col_of<MZ>(x, y, z, n)];
  auto s_at = [&](int X, int Y, int Z) {
    X = X < 0 ? 0 : (X > n - 1 ? n - 1 : X);
    Y = Y < 0 ? 0 : (Y > n - 1 ? n - 1 : Y);
    Z = Z < 0 ? 0 : (Z > n - 1 ? n - 1 : Z);
    return s0[col_of<MZ>(X, Y, Z, n)];
  };
  const double a0 = melt_of<MZ>(y, z) + 0.5;
#pragma unroll
  for (int p = 0; p < 7; ++p) {
    const int ex = ex7(p), ey = ey7(p), ez = ez7(p), q = opp7(p);
    const bool along = MZ ? (ez != 0) : (ey != 0);
    const int yx = x + ex, yy = y + ey, yz = z + ez;
    const bool yin = G.in(yx, yy, yz);
    const bool ysame = yin && liq(yx, yy, yz) == L;
    const uint32_t cy = yin ? G.cell(yx, yy, yz) : i;
    const double la = LG(p, cy), lq = LG(q, i), lp = LG(p, i), lqy = LG(q, cy);
    const double s_p1 = along ? s_own : s_at(x + ex, y + ey, z + ez);
    const double s_m1 = along ? s_own : s_at(x - ex, y - ey, z - ez);
    const double s_p2 = along ? s_own : s_at(x + 2 * ex, y + 2 * ey, z + 2 * ez);
    double acc = 0.0;
    // (a) regular pull of direction p by the neighbour x + e_p
    if (ysame) acc += la;
    // (b) this cell's direction q = opp(p), whose source x + e_p is a wall or
    //     across the front
    if (p != 0) {
      if (!yin) {
        const int sa = melt_of<MZ>(yy, yz);
        const bool dirichlet = sa < 0 || (!MZ && sa >= n);
        acc += (dirichlet ? -1.0 : 1.0) * lq;
      } else if (!ysame) {
        const double d = along ? fabs(s_own - a0) : (a0 - s_own) / (s_p1 - s_own);
        if (d < 0.5) {
          const int bx = x - ex, by = y - ey, bz = z - ez;
          const bool behind = G.in(bx, by, bz) && liq(bx, by, bz) == L;
          acc += (behind ? -2.0 * d : -1.0) * lq;
          // conservative front: the heat of this link, sent minus received
          if (EXT && wq)
            acc += (behind ? 1.0 + 2.0 * d : 2.0) * heat_weight<MZ>(wq, x, y, z, q, L, n);
        } else {
          acc += -lq / (2.0 * d);
          if (EXT && wq) acc += (1.0 + 1.0 / (2.0 * d)) * heat_weight<MZ>(wq, x, y, z, q, L, n);
        }
      }
      // (c) this cell's direction p itself, when its source x - e_p is across
      //     the front with a link fraction >= 1/2
      const int sx = x - ex, sy = y - ey, sz = z - ez;
      if (G.in(sx, sy, sz) && liq(sx, sy, sz) != L) {
        const double d = along ? fabs(s_own - a0) : (a0 - s_own) / (s_m1 - s_own);
        if (d >= 0.5) {
          acc += (2.0 * d - 1.0) / (2.0 * d) * lp;
          if (EXT && wq)
            acc -= (2.0 * d - 1.0) / (2.0 * d) * heat_weight<MZ>(wq, x, y, z, p, L, n);
        }
      }
      // (d) the neighbour x + e_p, direction q, when its source x + 2 e_p is
      //     across the front with a link fraction < 1/2 (this cell is then the
      //     cell behind it)
      if (ysame) {
        const int tx = yx + ex, ty = yy + ey, tz = yz + ez;
        if (G.in(tx, ty, tz) && liq(tx, ty, tz) != L) {
          const double ay = melt_of<MZ>(yy, yz) + 0.5;
          const double d = along ? fabs(s_own - ay) : (ay - s_p1) / (s_p2 - s_p1);
          if (d < 0.5) {
            acc += -(1.0 - 2.0 * d) * lqy;
            if (EXT && wq) acc += (1.0 - 2.0 * d) * heat_weight<MZ>(wq, yx, yy, yz, q, L, n);
          }
        }
      }
    }
    lg0[(size_t)p * nc + i] = (Lam)acc;
  }
  // adjoint of f before the step: only liquid cells read their f (solid
  // cells hold dead data, whose adjoint is zero and is not stored)
  if (FLOW && L && !(EXT && P.f_wall)) {
#pragma unroll
    for (int p = 0; p < 19; ++p) {
      const int yx = x + ex19(p), yy = y + ey19(p), yz = z + ez19(p);
      const bool pulled = G.in(yx, yy, yz) && liq(yx, yy, yz);
      lf0[(size_t)p * nc + i] =
          pulled ? lfh[(size_t)p * nc + G.cell(yx, yy, yz)] : lfh[(size_t)opp19(p) * nc + i];
    }
  } else if (FLOW && L) {  // interpolated no-slip of f
    auto LF = [&](int q, uint32_t j) { return (double)lfh[(size_t)q * nc + j]; };
    for (int p = 0; p < 19; ++p) {
      const int yx = x + ex19(p), yy = y + ey19(p), yz = z + ez19(p), q = opp19(p);
      const bool yin = G.in(yx, yy, yz);
      const bool pulled = yin && liquid_at<MZ>(cnt, yx, yy, yz, n);
      if (p == 0) {
        lf0[(size_t)p * nc + i] = lfh[(size_t)p * nc + i];
        continue;
      }
      // every reader of f*_p(x) under the interpolated no-slip
      double acc = 0.0, num, den;
      if (pulled) {  // (a) the regular pull of the neighbour x + e_p
        acc += LF(p, G.cell(yx, yy, yz));
      } else if (!yin) {  // (b) this cell's direction q: a box wall (halfway)
        acc += LF(q, i);
      } else {  // (b) ... or a solid source: the weight of f*_p(x)
        const double d = frac19<MZ>(s0, x, y, z, q, n, num, den);
        if (d < 0.5) {
          const int bx = x - ex19(p), by = y - ey19(p), bz = z - ez19(p);
          const bool behind = G.in(bx, by, bz) && liquid_at<MZ>(cnt, bx, by, bz, n);
          acc += (behind ? 2.0 * d : 1.0) * LF(q, i);
        } else {
          acc += LF(q, i) / (2.0 * d);
        }
      }
      // (c) this cell's direction p itself, when its source x - e_p is solid
      //     and cut at d >= 1/2
      {
        const int sx = x - ex19(p), sy = y - ey19(p), sz = z - ez19(p);
        if (G.in(sx, sy, sz) && !liquid_at<MZ>(cnt, sx, sy, sz, n)) {
          const double d = frac19<MZ>(s0, x, y, z, p, n, num, den);
          if (d >= 0.5) acc += (2.0 * d - 1.0) / (2.0 * d) * LF(p, i);
        }
      }
      // (d) the neighbour x + e_p, direction q, whose source x + 2 e_p is solid
      //     and cut at d < 1/2: this cell is the cell behind it
      if (pulled) {
        const int tx = yx + ex19(p), ty = yy + ey19(p), tz = yz + ez19(p);
        if (G.in(tx, ty, tz) && !liquid_at<MZ>(cnt, tx, ty, tz, n)) {
          const double d = frac19<MZ>(s0, yx, yy, yz, q, n, num, den);
          if (d < 0.5) acc += (1.0 - 2.0 * d) * LF(q, G.cell(yx, yy, yz));
        }
      }
      lf0[(size_t)p * nc + i] = (Lam)acc;
    }
  }
}

// The rows outside the bulk solid, visited by row slots as in k_adj_collide
// (its general path needs more registers than the bulk rows should pay for).
template <typename Ts, typename Lam, bool FLOW, bool MZ, bool EXT>
__device__ __forceinline__ void adj_stream_rows(
    int slot, int nslots, int x, const double* __restrict__ s0, const int* __restrict__ cnt,
    const int* __restrict__ cmin2, const int* __restrict__ cmax2, const int* __restrict__ rowb,
    const Lam* __restrict__ lfh, const Lam* __restrict__ lgh, Lam* __restrict__ lf0,
    Lam* __restrict__ lg0, const double* __restrict__ wq, const KParams& P) {
  const int n = P.n;
  const int A = row_bound(rowb[0], n), R = front_rows(A, n);
  for (int r = slot; r < R; r += nslots) {
    int a, o;
    front_row(r, A, P, a, o);
    if (x < n)
      adj_stream_cell<Ts, Lam, FLOW, MZ, EXT>(s0, cnt, cmin2, cmax2, lfh, lgh, lf0, lg0, wq, P, x,
                                              MZ ? o : a, MZ ? a : o);
  }
}

template <typename Ts, typename Lam, bool FLOW, bool MZ, bool EXT>
__global__ __launch_bounds__(256) void k_adj_stream(
    const double* __restrict__ s0, const int* __restrict__ cnt, const int* __restrict__ cmin2,
    const int* __restrict__ cmax2, const int* __restrict__ rowb, const Lam* __restrict__ lfh,
    const Lam* __restrict__ lgh, Lam* __restrict__ lf0, Lam* __restrict__ lg0,
    const double* __restrict__ wq, KParams P) {
  adj_stream_rows<Ts, Lam, FLOW, MZ, EXT>(blockIdx.y, gridDim.y,
                                          blockIdx.x * blockDim.x + threadIdx.x, s0, cnt, cmin2,
                                          cmax2, rowb, lfh, lgh, lf0, lg0, wq, P);
}

// The bulk-solid rows: g alone, gathered from the neighbours with no phase
// reads, at full occupancy.
template <typename Lam, bool MZ>
__device__ __forceinline__ void adj_stream_solid_row(int x, int y, int z,
                                                     const int* __restrict__ rowb,
                                                     const int* __restrict__ rowb_next,
                                                     const Lam* __restrict__ lgh,
                                                     Lam* __restrict__ lg0, const KParams& P) {
  const int n = P.n, a = melt_of<MZ>(y, z);
  if (x >= n || !bulk_solid_row(a, MZ ? y : z, row_bound(rowb[0], n), n)) return;
  if (rowb_next && a >= rowb_next[0] + 3) return;  // paired: see paired_row
  const Geo G{n, (uint32_t)n * (uint32_t)n};
  push_fast<7>(lgh, lg0, G, P.ncell, x, y, z, G.cell(x, y, z));
}

template <typename Lam, bool MZ>
__global__ __launch_bounds__(256) void k_adj_stream_solid(const int* __restrict__ rowb,
                                                          const int* __restrict__ rowb_next,
                                                          const Lam* __restrict__ lgh,
                                                          Lam* __restrict__ lg0, KParams P) {
  adj_stream_solid_row<Lam, MZ>(blockIdx.x * blockDim.x + threadIdx.x, blockIdx.y, blockIdx.z,
                                rowb, rowb_next, lgh, lg0, P);
}

// derivative of the pulled population of an interface link with respect to
// its link fraction, times its adjoint; reader cell (x,y,z), incoming
// direction q (its source across the front).  With the conservative front
// update (wq not NULL) the link's heat, sent minus received, enters J with
// the weight of its column as well.
template <typename Ts, typename Lam, bool MZ, bool EXT>
__device__ __forceinline__ double link_sens(const Ts* g0, const double* s0, const int* cnt,
                                            const Lam* lgh, const double* wq, int x, int y,
                                            int z, int q, bool L, double& dfrac,
                                            const KParams& P) {
  const int n = P.n;
  const Geo G{n, (uint32_t)n * (uint32_t)n};
  const size_t nc = P.ncell;
  const uint32_t i = G.cell(x, y, z);
  const int p = opp7(q);
  // every value either branch may read, loaded first (the cell behind
  // replaced by this one where it is outside the box)
  const int bx = x + ex7(q), by = y + ey7(q), bz = z + ez7(q);
  const bool bin = G.in(bx, by, bz);
  const uint32_t ib = bin ? G.cell(bx, by, bz) : i;
  const double gp = sv<7>(g0, P, p, i), gq = sv<7>(g0, P, q, i), gpb = sv<7>(g0, P, p, ib);
  const int cb = cnt[bin ? col_of<MZ>(bx, by, bz, n) : col_of<MZ>(x, y, z, n)];
  const double lg = (double)lgh[(size_t)q * nc + i];
  const double d = link_delta<MZ>(s0, x, y, z, -ex7(q), -ey7(q), -ez7(q), n);
  dfrac = d;
  const double l = lg - ((EXT && wq) ? heat_weight<MZ>(wq, x, y, z, q, L, n) : 0.0);
  if (d < 0.5) {
    if (bin && (melt_of<MZ>(by, bz) < cb) == L) return (-2.0 * gp + 2.0 * gpb) * l;
    return 0.0;
  }
  const double w = 0.125;
  return (gp / (2.0 * d * d) + gq / (2.0 * d * d) - w * (P.t_m - P.tref) / (d * d)) * l;
}

// Interpolated no-slip of f: derivative of the pulled population q of the
// liquid cell (x,y,z), whose source is solid, with respect to its link
// fraction d, times that population's adjoint.  num, den: d = num / den.
template <typename Ts, typename Lam, bool MZ>
__device__ double flink_sens(const Ts* f0, const double* s0, const int* cnt, const Lam* lfh,
                             int x, int y, int z, int q, double& num, double& den,
                             const KParams& P) {
  const int n = P.n;
  const Geo G{n, (uint32_t)n * (uint32_t)n};
  const uint32_t i = G.cell(x, y, z);
  const int p = opp19(q);
  const double d = frac19<MZ>(s0, x, y, z, q, n, num, den);
  const double l = (double)lfh[(size_t)q * P.ncell + i];
  if (d < 0.5) {
    const int bx = x + ex19(q), by = y + ey19(q), bz = z + ez19(q);
    if (!G.in(bx, by, bz) || !liquid_at<MZ>(cnt, bx, by, bz, n)) return 0.0;
    return 2.0 * (sv<19>(f0, P, p, i) - sv<19>(f0, P, p, G.cell(bx, by, bz))) * l;
  }
  return (sv<19>(f0, P, q, i) - sv<19>(f0, P, p, i)) / (2.0 * d * d) * l;
}

// Sum over the f links whose link fraction depends on the front of column
// (x, o): d = num / den with num = a + 1/2 - s_reader and den = s_source -
// s_reader + e_a, so dd/ds_reader = (num - den) / den^2 and dd/ds_source =
// -num / den^2.  (i) the links of this column's liquid cells, (ii) the links
// of the 8 neighbour columns' liquid cells whose source lies in this column.
// Every link is visited from both of its columns, so no atomics are needed.
template <typename Ts, typename Lam, bool MZ>
__device__ double flink_column(const Ts* f0, const double* s0, const int* cnt, const Lam* lfh,
                               int x, int o, const KParams& P) {
  const int n = P.n;
  const int c = o * n + x;
  int lo = cnt[c], hi = cnt[c];
  for (int dd = -1; dd <= 1; ++dd)
    for (int dx = -1; dx <= 1; ++dx) {
      const int xx = x + dx, oo = o + dd;
      if (xx < 0 || xx >= n || oo < 0 || oo >= n) continue;
      lo = cnt[oo * n + xx] < lo ? cnt[oo * n + xx] : lo;
      hi = cnt[oo * n + xx] > hi ? cnt[oo * n + xx] : hi;
    }
  lo = lo - 1 < 0 ? 0 : lo - 1;
  hi = hi - 1 > n - 1 ? n - 1 : hi - 1;
  double acc = 0.0, num, den;
  for (int a = lo; a <= hi; ++a) {
    for (int dd = -1; dd <= 1; ++dd)
      for (int dx = -1; dx <= 1; ++dx) {
        const int xx = x + dx, oo = o + dd;  // the reader's column
        if (xx < 0 || xx >= n || oo < 0 || oo >= n) continue;
        if (a >= cnt[oo * n + xx]) continue;  // the reader is liquid
        const int ry = MZ ? oo : a, rz = MZ ? a : oo;
        for (int q = 1; q < 19; ++q) {
          const int sx = xx - ex19(q), sy = ry - ey19(q), sz = rz - ez19(q);
          if ((unsigned)sx >= (unsigned)n || (unsigned)sy >= (unsigned)n ||
              (unsigned)sz >= (unsigned)n)
            continue;
          if (liquid_at<MZ>(cnt, sx, sy, sz, n)) continue;  // regular pull
          const int so = MZ ? sy : sz;
          const bool src_here = sx == x && so == o, reader_here = dx == 0 && dd == 0;
          if (!src_here && !reader_here) continue;
          const double ld = flink_sens<Ts, Lam, MZ>(f0, s0, cnt, lfh, xx, ry, rz, q, num, den, P);
          if (reader_here) acc += ld * (num - den) / (den * den);
          if (src_here) acc += ld * (-num) / (den * den);
        }
      }
  }
  return acc;
}

template <typename Ts, typename Lam, bool MZ, bool EXT>
__device__ __forceinline__ void adj_interface_column(
    int x, int o, const Ts* __restrict__ g0, const double* __restrict__ s0,
    const int* __restrict__ cnt, const Lam* __restrict__ lgh, const Ts* __restrict__ f0,
    const Lam* __restrict__ lfh, const double* __restrict__ wq, const double* __restrict__ own,
    const double* __restrict__ out5, double* __restrict__ ls0, double* __restrict__ lth,
    const KParams& P) {
  const int n = P.n;
  if (x >= n) return;
  const int c = o * n + x;
  const size_t nc = P.ncell;
  // hot-wall anti-bounce-back of the cell next to the heated wall:
  // g_in = -g_out + 2 w (T_h - tref)
  {
    const uint32_t i = cell_in_column<MZ>(c, 0, P);
    const int qin = MZ ? 5 : 3;  // +z or +y: pulled from the heated wall
    lth[c] += 2.0 * 0.125 * (double)lgh[(size_t)qin * nc + i];
  }
  // lateral neighbour columns, one fixed slot each (constant indices once the
  // loops are unrolled, so the slots live in registers); ok: in the box
  int nb[4], nbx[4], nbo[4], nbc[4];
  bool ok[4];
  const int dx[4] = {1, -1, 0, 0}, dob[4] = {0, 0, 1, -1};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int xx = x + dx[j], oo = o + dob[j];
    ok[j] = xx >= 0 && xx < n && oo >= 0 && oo < n;
    nbx[j] = xx;
    nbo[j] = oo;
    nb[j] = ok[j] ? oo * n + xx : c;
    nbc[j] = cnt[nb[j]];
  }
  int lo = cnt[c], hi = cnt[c];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (!ok[j]) continue;
    lo = nbc[j] < lo ? nbc[j] : lo;
    hi = nbc[j] > hi ? nbc[j] : hi;
  }
  lo = lo - 1 < 0 ? 0 : lo - 1;
  hi = hi > n - 1 ? n - 1 : hi;
  const double sc = s0[c];
  double acc = 0.0;
  for (int a = lo; a <= hi; ++a) {
    const double ya = a + 0.5;
    // (i) links of this column's cell at height a
    {
      const int cx = x, cy = MZ ? o : a, cz = MZ ? a : o;
      const bool L = a < cnt[c];
      for (int q = 1; q < 7; ++q) {
        const int sx = cx - ex7(q), sy = cy - ey7(q), sz = cz - ez7(q);
        if ((unsigned)sx >= (unsigned)n || (unsigned)sy >= (unsigned)n || (unsigned)sz >= (unsigned)n)
          continue;
        if (liquid_at<MZ>(cnt, sx, sy, sz, n) == L) continue;
        double d;
        const double ld =
            link_sens<Ts, Lam, MZ, EXT>(g0, s0, cnt, lgh, wq, cx, cy, cz, q, L, d, P);
        const bool along = MZ ? (ez7(q) != 0) : (ey7(q) != 0);
        if (along) {
          acc += (sc > ya ? 1.0 : -1.0) * ld;
        } else {
          const double sn = s0[col_of<MZ>(sx, sy, sz, n)];
          acc += ld * (ya - sn) / ((sn - sc) * (sn - sc));
        }
      }
    }
    // (ii) lateral links of the neighbours' cells at height a that point into
    //      this column
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (!ok[j]) continue;
      const int cx = nbx[j], cy = MZ ? nbo[j] : a, cz = MZ ? a : nbo[j];
      const bool L = a < nbc[j];
      if ((a < cnt[c]) == L) continue;
      // incoming direction of the neighbour whose source is this column
      const int ddx = x - nbx[j], ddo = o - nbo[j];
      int q = -1;
      for (int qq = 1; qq < 7; ++qq) {
        const int ox = -ex7(qq), oy = -ey7(qq), oz = -ez7(qq);  // source offset
        const int oo_ = MZ ? oy : oz, om = MZ ? oz : oy;
        if (ox == ddx && oo_ == ddo && om == 0) q = qq;
      }
      if (q < 1) continue;  // every lateral neighbour has one such direction
      double d;
      const double ld = link_sens<Ts, Lam, MZ, EXT>(g0, s0, cnt, lgh, wq, cx, cy, cz, q, L, d, P);
      const double sself = s0[nb[j]];
      acc += ld * (-(ya - sself)) / ((sc - sself) * (sc - sself));
    }
  }
  if (EXT && P.flow && P.f_wall) acc += flink_column<Ts, Lam, MZ>(f0, s0, cnt, lfh, x, o, P);
  ls0[c] = front_gather(own, out5, x, o, n) + acc;
}

template <typename Ts, typename Lam, bool MZ, bool EXT>
__global__ __launch_bounds__(64) void k_adj_interface(
    const Ts* __restrict__ g0, const double* __restrict__ s0, const int* __restrict__ cnt,
    const Lam* __restrict__ lgh, const Ts* __restrict__ f0, const Lam* __restrict__ lfh,
    const double* __restrict__ wq, const double* __restrict__ own,
    const double* __restrict__ out5, double* __restrict__ ls0, double* __restrict__ lth,
    KParams P) {
  adj_interface_column<Ts, Lam, MZ, EXT>(blockIdx.x * blockDim.x + threadIdx.x, blockIdx.y, g0,
                                         s0, cnt, lgh, f0, lfh, wq, own, out5, ls0, lth, P);
}

// Small lattices, where each kernel of the reverse step is latency bound
// (one row or one column of work per wave, fewer waves than SIMDs): the
// independent kernels share a launch, each workgroup taking one role by its
// index, so their latencies overlap instead of adding up.  The same cell and
// column functions as the separate kernels: the same results bit for bit.
// Collision: row slots of the rows with a liquid cell first (the longer
// chain), then the all-solid rows.
template <typename Ts, typename Lam, bool FLOW, bool MZ, bool EXT>
__global__ __launch_bounds__(256) void k_adj_collide_all(
    const Ts* __restrict__ f0, const Ts* __restrict__ g0, const double* __restrict__ s0,
    const double* __restrict__ s1, const double* __restrict__ th, const int* __restrict__ cnt,
    const int* __restrict__ cmin2, const int* __restrict__ cmax2, const int* __restrict__ rowb,
    const Lam* __restrict__ lf1, const Lam* __restrict__ lg1, Lam* __restrict__ lfh,
    Lam* __restrict__ lgh, int nslots, KParams P) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, b = blockIdx.y;
  if (b < nslots) {
    adj_collide_rows<Ts, Lam, FLOW, MZ, EXT>(b, nslots, x, f0, g0, s0, s1, th, cnt, cmin2, cmax2,
                                             rowb, lf1, lg1, lfh, lgh, P);
  } else {
    const int r = b - nslots;  // row (y, z) = (r mod n, r / n)
    const int rz = (int)div_n((uint32_t)r, P);
    adj_collide_solid_row<Lam, MZ>(x, r - rz * P.n, rz, rowb, nullptr, lg1, nullptr, lgh, P);
  }
}

// Streaming and interface: the interface columns first, then the row slots
// of the rows outside the bulk solid, then the bulk-solid rows.  64-lane
// workgroups (the interface needs the registers a 64-lane bound allows).
template <typename Ts, typename Lam, bool FLOW, bool MZ, bool EXT>
__global__ __launch_bounds__(64) void k_adj_stream_all(
    const Ts* __restrict__ g0, const Ts* __restrict__ f0, const double* __restrict__ s0,
    const int* __restrict__ cnt, const int* __restrict__ cmin2, const int* __restrict__ cmax2,
    const int* __restrict__ rowb, const Lam* __restrict__ lfh, const Lam* __restrict__ lgh,
    Lam* __restrict__ lf0, Lam* __restrict__ lg0, const double* __restrict__ wq,
    const double* __restrict__ own, const double* __restrict__ out5, double* __restrict__ ls0,
    double* __restrict__ lth, int nslots, KParams P) {
  const int n = P.n;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  int b = blockIdx.y;
  if (b < n) {
    adj_interface_column<Ts, Lam, MZ, EXT>(x, b, g0, s0, cnt, lgh, f0, lfh, wq, own, out5, ls0,
                                           lth, P);
  } else if ((b -= n) < nslots) {
    adj_stream_rows<Ts, Lam, FLOW, MZ, EXT>(b, nslots, x, s0, cnt, cmin2, cmax2, rowb, lfh, lgh,
                                            lf0, lg0, wq, P);
  } else {
    b -= nslots;
    const int bz = (int)div_n((uint32_t)b, P);
    adj_stream_solid_row<Lam, MZ>(x, b - bz * n, bz, rowb, nullptr, lgh, lg0, P);
  }
}

template <typename V>
__global__ void k_fill(V* __restrict__ v, size_t count, double value) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) v[i] = (V)value;
}

template <typename V>
hipError_t fill_t(V* v, size_t count, double value, hipStream_t st) {
  if (!v) return hipErrorInvalidValue;
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL((k_fill<V>), dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, v,
                     count, value);
  return hipGetLastError();
}

// EXT: the interpolated no-slip of f or the conservative front update is on
// (a separate instantiation, so that the default one compiles without them)
template <typename Ts, typename Lam, bool FLOW, bool MZ, bool EXT>
hipError_t adjoint_step_t(const KParams& P, const AdjointStep& A, hipStream_t st) {
  const int n = P.n;
  const dim3 bcol(64, 1, 1), gcol((n + 63) / 64, n, 1);
  // one lattice row per workgroup (up to 256 lanes)
  const int bx = n >= 256 ? 256 : ((n + 63) / 64) * 64;
  const dim3 bcell(bx, 1, 1), gcell((n + bx - 1) / bx, n, n);
  const Ts* f0 = static_cast<const Ts*>(A.f0);
  const Ts* g0 = static_cast<const Ts*>(A.g0);
  const Ts* g1 = static_cast<const Ts*>(A.g1);
  Lam* lf1 = static_cast<Lam*>(A.lf1);
  Lam* lg1 = static_cast<Lam*>(A.lg1);
  Lam* lf0 = static_cast<Lam*>(A.lf0);
  Lam* lg0 = static_cast<Lam*>(A.lg0);
  Lam* lfh = static_cast<Lam*>(A.lfh);
  Lam* lgh = static_cast<Lam*>(A.lgh);
  if (A.heat)  // conservative front update
    hipLaunchKernelGGL(k_adj_front_heat, gcol, bcol, 0, st, A.s0, A.heat, A.ls1, A.wq, A.own,
                       A.out5, P);
  else
    hipLaunchKernelGGL((k_adj_front<Ts, Lam, FLOW, MZ>), gcol, bcol, 0, st, A.s0, g1, A.th, A.ls1,
                       lg1, A.out5, A.own, A.lth, P);
  const double* wq = A.heat ? A.wq : nullptr;
  // row slots of the full reverse collision: at most one per row
  const int nslots = n * n < 2048 ? n * n : 2048;
  if (n <= kAdjFuseMaxN) {  // two launches, each over all its independent parts
    const int gx = (n + 63) / 64;
    hipLaunchKernelGGL((k_adj_collide_all<Ts, Lam, FLOW, MZ, EXT>),
                       dim3(gx, (unsigned)(nslots + n * n), 1), dim3(64, 1, 1), 0, st, f0, g0,
                       A.s0, A.s1, A.th, A.cnt, A.cmin2, A.cmax2, A.rowb, lf1, lg1, lfh, lgh,
                       nslots, P);
    hipLaunchKernelGGL((k_adj_stream_all<Ts, Lam, FLOW, MZ, EXT>),
                       dim3(gx, (unsigned)(n + nslots + n * n), 1), dim3(64, 1, 1), 0, st, g0, f0,
                       A.s0, A.cnt, A.cmin2, A.cmax2, A.rowb, lfh, lgh, lf0, lg0, wq, A.own,
                       A.out5, A.ls0, A.lth, nslots, P);
    return hipGetLastError();
  }
  const dim3 gfront((n + bx - 1) / bx, (unsigned)nslots, 1);
  hipLaunchKernelGGL((k_adj_collide<Ts, Lam, FLOW, MZ, EXT>), gfront, bcell, 0, st, f0, g0, A.s0,
                     A.s1, A.th, A.cnt, A.cmin2, A.cmax2, A.rowb, lf1, lg1, lfh, lgh, P);
  const Lam* lghp = static_cast<const Lam*>(A.lgh_prev);
  if (A.rowb_prev && (!lghp || lghp == lgh)) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_adj_collide_solid<Lam, MZ>), gcell, bcell, 0, st, A.rowb, A.rowb_prev,
                     lg1, lghp, lgh, P);
  hipLaunchKernelGGL((k_adj_stream<Ts, Lam, FLOW, MZ, EXT>), gfront, bcell, 0, st, A.s0, A.cnt,
                     A.cmin2, A.cmax2, A.rowb, lfh, lgh, lf0, lg0, wq, P);
  hipLaunchKernelGGL((k_adj_stream_solid<Lam, MZ>), gcell, bcell, 0, st, A.rowb, A.rowb_next,
                     lgh, lg0, P);
  hipLaunchKernelGGL((k_adj_interface<Ts, Lam, MZ, EXT>), gcol, bcol, 0, st, g0, A.s0, A.cnt, lgh, f0,
                     lfh, wq, A.own, A.out5, A.ls0, A.lth, P);
  return hipGetLastError();
}

template <typename Ts, typename Lam, bool FLOW, bool MZ>
hipError_t adjoint_step_e(const KParams& P, const AdjointStep& A, hipStream_t st) {
  if ((FLOW && P.f_wall) || A.heat) return adjoint_step_t<Ts, Lam, FLOW, MZ, true>(P, A, st);
  return adjoint_step_t<Ts, Lam, FLOW, MZ, false>(P, A, st);
}

template <typename Ts, typename Lam>
hipError_t adjoint_step_d(const KParams& P, const AdjointStep& A, hipStream_t st) {
  if (P.flow)
    return P.melt_z ? adjoint_step_e<Ts, Lam, true, true>(P, A, st)
                    : adjoint_step_e<Ts, Lam, true, false>(P, A, st);
  return P.melt_z ? adjoint_step_e<Ts, Lam, false, true>(P, A, st)
                  : adjoint_step_e<Ts, Lam, false, false>(P, A, st);
}

}  // namespace

hipError_t launch_adjoint_step(int kind, const KParams& P, const AdjointStep& A, hipStream_t st) {
  switch (kind) {
    case kF64: return adjoint_step_d<double, double>(P, A, st);
    case kF32: return adjoint_step_d<float, float>(P, A, st);
    case kF16S: return adjoint_step_d<_Float16, float>(P, A, st);
    case kBF16S: return adjoint_step_d<__bf16, float>(P, A, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_adj_partition(const KParams& P, const double* const* states, int count,
                                int* cnt, int* cmin2, int* cmax2, int* rmax, hipStream_t st) {
  const int n = P.n;
  const size_t nn = (size_t)n * n;
  constexpr int kMaxPlanes = 65535;  // grid z limit
  for (int t0 = 0; t0 < count; t0 += kMaxPlanes) {
    const int planes = count - t0 < kMaxPlanes ? count - t0 : kMaxPlanes;
    hipLaunchKernelGGL(k_adj_partition,
                       dim3((n + 63) / 64, (n + kPartRows - 1) / kPartRows, planes),
                       dim3(64, kPartRows, 1), 0, st, states + t0, cnt + t0 * nn,
                       cmin2 + t0 * nn, cmax2 + t0 * nn, rmax + t0, n);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_fill(double* v, size_t count, double value, hipStream_t st) {
  return fill_t(v, count, value, st);
}

size_t lambda_bytes(int kind) { return kind == kF64 ? sizeof(double) : sizeof(float); }

hipError_t launch_fill_lambda(int kind, void* v, size_t count, double value, hipStream_t st) {
  return kind == kF64 ? fill_t(static_cast<double*>(v), count, value, st)
                      : fill_t(static_cast<float*>(v), count, value, st);
}

}  // namespace lbmk
