// gfx950 kernels of the double-MRT lattice Boltzmann melting step.
//
// Method: Li, Yang & Zhang, arXiv:1604.03478, section 2.
//   f: D3Q19 (Eq. (3) velocity order), Eq. (1) with the MRT collision of
//      Eq. (2) and a Boussinesq body force (section 1, assumption 4).
//   g: D3Q7 (Eq. (5) velocity order), Eq. (4).
//   front: Eq. (6), one height per column along the melt axis.
//
// Design (MI355X):
//   * Row-interleaved storage (lbm_device.h): the 19 (f) or 7 (g) direction
//     rows of one lattice row (y, z) are contiguous, x fastest.  One
//     workgroup per lattice row, one thread per cell, so every population
//     load and store of a wave is one contiguous 256 B (FP32) segment and a
//     row update reads 9 neighbouring row blocks and writes its own.  Pull
//     streaming: each stored value is read once and written once per step
//     (208 B per FP32 cell update).
//   * Populations are stored shifted (f - w*rho0, g - w*tref) and the whole
//     collision works on deviations, which keeps FP32 and 16-bit storage
//     accurate; tref = (t_h + t_m)/2 centres the liquid temperature range.
//   * The 19x19 and 7x7 moment transforms use the integer structure of the
//     orthogonal bases (pairwise sums and differences), about 250 flops per
//     cell instead of 1444 for a dense product; no MFMA (the transform is a
//     tiny, sparse, per-cell integer matrix and the kernel is HBM bound).
//   * A wave takes the fast path when every lane is away from the y/z walls
//     and its 3x3x3 stencil lies in one phase; x walls are handled there by a
//     per-lane address select, so all 26 loads of a cell are issued before
//     the first wait.  Waves that touch the front or a y/z wall take the
//     general path with per-link boundary handling.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_internal.h"

#include "lbm_device.h"

namespace lbmk {
namespace {

// --------------------------------------------------------------- collision
template <typename C, typename G>
struct Rates {
  C sv, gb;  // shear rate and buoyancy coefficient of the flow
  G qj, qe;  // rates of the energy distribution (liquid cells)
  G qjs, qes;  // the same in solid cells
  G tref;    // storage shift of g: the stored value is g_q - w_q * tref
  G dbuoy;   // tref - t0, so that T - t0 = (T - tref) + dbuoy
};

// A parameter in the collision's type: the host's FP32 rounding of it for
// FP32 arithmetic (no conversion in every wave), else the FP64 value.
template <typename T>
__device__ __forceinline__ T param_as(double d, float f) {
  if constexpr (sizeof(T) == 4) return f;
  else return (T)d;
}

template <typename C, typename G>
__device__ __forceinline__ Rates<C, G> make_rates(const KParams& P) {
  Rates<C, G> r;
  r.sv = param_as<C>(P.s_nu, P.s_nu_f);
  r.gb = param_as<C>(P.gbeta, P.gbeta_f);
  r.qj = param_as<G>(P.q_j, P.q_j_f);
  r.qe = param_as<G>(P.q_e, P.q_e_f);
  r.qjs = param_as<G>(P.q_js, P.q_js_f);
  r.qes = param_as<G>(P.q_es, P.q_es_f);
  r.tref = param_as<G>(P.tref, P.tref_f);
  r.dbuoy = param_as<G>(P.tref - P.t0, P.dbuoy_f);
  return r;
}

// MRT collision of f (Eq. (2) with the force of Eq. (1)) and of g (Eq. (4))
// on shifted populations, in place (f is left untouched in solid cells).
// Gravity is along z, so the force has one component F_z = gbeta (T - t0).
// Returns true when a non-finite value appeared.
template <bool FLOW, typename C, typename G>
__device__ __forceinline__ bool collide(C (&f)[19], G (&g)[7], bool liquid, const Rates<C, G>& r) {
  const G Tt = ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + g[6]);  // T - tref
  C ux = C(0), uy = C(0), uz = C(0);
  bool bad = !(fabs(Tt) < G(1e30));

  if (FLOW && liquid) {
    // ---- forward transform m = M f (orthogonal D3Q19 basis) ----
    const C axp = f[1] + f[2], axm = f[1] - f[2];
    const C ayp = f[3] + f[4], aym = f[3] - f[4];
    const C azp = f[5] + f[6], azm = f[5] - f[6];
    const C a78 = f[7] + f[8], b78 = f[7] - f[8], a910 = f[9] + f[10], b910 = f[9] - f[10];
    const C Sxy = a78 + a910, Xxy = b78 + b910, Yxy = a78 - a910, Pxy = b78 - b910;
    const C a1112 = f[11] + f[12], b1112 = f[11] - f[12];
    const C a1314 = f[13] + f[14], b1314 = f[13] - f[14];
    const C Sxz = a1112 + a1314, Xxz = b1112 + b1314, Zxz = a1112 - a1314, Pxz = b1112 - b1314;
    const C a1516 = f[15] + f[16], b1516 = f[15] - f[16];
    const C a1718 = f[17] + f[18], b1718 = f[17] - f[18];
    const C Syz = a1516 + a1718, Yyz = b1516 + b1718, Zyz = a1516 - a1718, Pyz = b1516 - b1718;
    const C A = axp + ayp + azp;
    const C E = Sxy + Sxz + Syz;

    const C drho = f[0] + A + E;
    const C m1 = C(-30) * f[0] - C(11) * A + C(8) * E;
    const C m2 = C(12) * f[0] - C(4) * A + E;
    const C jx = axm + Xxy + Xxz;
    const C m4 = C(-4) * axm + Xxy + Xxz;
    const C jy = aym + Yxy + Yyz;
    const C m6 = C(-4) * aym + Yxy + Yyz;
    const C jz = azm + Zxz + Zyz;
    const C m8 = C(-4) * azm + Zxz + Zyz;
    const C Ed = Sxy + Sxz - C(2) * Syz;
    const C m9 = C(2) * axp - ayp - azp + Ed;
    const C m10 = C(-4) * axp + C(2) * ayp + C(2) * azp + Ed;
    const C m11 = ayp - azp + Sxy - Sxz;
    const C m12 = C(-2) * ayp + C(2) * azp + Sxy - Sxz;
    const C m16 = Xxy - Xxz, m17 = Yyz - Yxy, m18 = Zxz - Zyz;

    // ---- macroscopic, force, equilibria (incompressible, rho0 = 1) ----
    const C Fz = r.gb * (C)(Tt + r.dbuoy);
    ux = jx;
    uy = jy;
    uz = jz + C(0.5) * Fz;
    const C usq = ux * ux + uy * uy + uz * uz;
    const C uF = uz * Fz;
    const C p9 = C(3) * ux * ux - usq;
    const C p11 = uy * uy - uz * uz;

    // ---- relaxation S (reading: d'Humieres et al. 2002 rates) ----
    constexpr C s_e = C(1.19), s_eps = C(1.4), s_q = C(1.2), s_pi = C(1.4), s_m = C(1.98);
    const C sv = r.sv;
    const C hv = C(1) - C(0.5) * sv;
    const C m1s = m1 - s_e * (m1 - (C(-11) * drho + C(19) * usq)) + (C(1) - C(0.5) * s_e) * C(38) * uF;
    const C m2s = m2 - s_eps * (m2 - (C(3) * drho - C(5.5) * usq)) + (C(1) - C(0.5) * s_eps) * C(-11) * uF;
    const C m4s = m4 - s_q * (m4 + C(2.0 / 3.0) * ux);
    const C m6s = m6 - s_q * (m6 + C(2.0 / 3.0) * uy);
    const C m8s = m8 - s_q * (m8 + C(2.0 / 3.0) * uz) + (C(1) - C(0.5) * s_q) * C(-2.0 / 3.0) * Fz;
    const C m7s = jz + Fz;
    const C m9s = m9 - sv * (m9 - p9) + hv * C(-2) * uF;
    const C m10s = m10 - s_pi * (m10 + C(0.5) * p9) + (C(1) - C(0.5) * s_pi) * uF;
    const C m11s = m11 - sv * (m11 - p11) + hv * C(-2) * uF;
    const C m12s = m12 - s_pi * (m12 + C(0.5) * p11) + (C(1) - C(0.5) * s_pi) * uF;
    const C m13s = Pxy - sv * (Pxy - ux * uy);
    const C m14s = Pyz - sv * (Pyz - uy * uz) + hv * uy * Fz;
    const C m15s = Pxz - sv * (Pxz - ux * uz) + hv * ux * Fz;
    const C km = C(1) - s_m;

    // ---- inverse transform f = M^T D^-1 m* ----
    const C a0 = drho * C(1.0 / 19.0);
    const C a1 = m1s * C(1.0 / 2394.0);
    const C a2 = m2s * C(1.0 / 252.0);
    const C a3 = jx * C(0.1), a5 = jy * C(0.1), a7 = m7s * C(0.1);
    const C a4 = m4s * C(1.0 / 40.0), a6 = m6s * C(1.0 / 40.0), a8 = m8s * C(1.0 / 40.0);
    const C a9 = m9s * C(1.0 / 36.0), a10 = m10s * C(1.0 / 72.0);
    const C a11 = m11s * C(1.0 / 12.0), a12 = m12s * C(1.0 / 24.0);
    const C a13 = m13s * C(0.25), a14 = m14s * C(0.25), a15 = m15s * C(0.25);
    const C a16 = km * m16 * C(0.125), a17 = km * m17 * C(0.125), a18 = km * m18 * C(0.125);

    const C Aax = a0 - C(11) * a1 - C(4) * a2;
    const C Aed = a0 + C(8) * a1 + a2;
    C o[19];
    o[0] = a0 - C(30) * a1 + C(12) * a2;
    {
      const C c = Aax + C(2) * a9 - C(4) * a10, d = a3 - C(4) * a4;
      o[1] = c + d;
      o[2] = c - d;
    }
    {
      const C c = Aax - a9 + C(2) * a10 + a11 - C(2) * a12, d = a5 - C(4) * a6;
      o[3] = c + d;
      o[4] = c - d;
    }
    {
      const C c = Aax - a9 + C(2) * a10 - a11 + C(2) * a12, d = a7 - C(4) * a8;
      o[5] = c + d;
      o[6] = c - d;
    }
    {  // xy edges 7..10
      const C b = Aed + a9 + a10 + a11 + a12, X = a3 + a4 + a16, Y = a5 + a6 - a17;
      o[7] = b + X + Y + a13;
      o[8] = b - X + Y - a13;
      o[9] = b + X - Y - a13;
      o[10] = b - X - Y + a13;
    }
    {  // xz edges 11..14
      const C b = Aed + a9 + a10 - a11 - a12, X = a3 + a4 - a16, Z = a7 + a8 + a18;
      o[11] = b + X + Z + a15;
      o[12] = b - X + Z - a15;
      o[13] = b + X - Z - a15;
      o[14] = b - X - Z + a15;
    }
    {  // yz edges 15..18
      const C b = Aed - C(2) * a9 - C(2) * a10, Y = a5 + a6 + a17, Z = a7 + a8 - a18;
      o[15] = b + Y + Z + a14;
      o[16] = b - Y + Z - a14;
      o[17] = b + Y - Z - a14;
      o[18] = b - Y - Z + a14;
    }
#pragma unroll
    for (int q = 0; q < 19; ++q) f[q] = o[q];
    bad = bad || !(fabs(drho) < C(1e30));
  }

  // ---- D3Q7 MRT collision of g (Eq. (4)), c_sT^2 = 1/4 ----
  {
    const G T = Tt + r.tref;
    const G px = g[1] + g[2], py = g[3] + g[4], pz = g[5] + g[6];
    const G n1 = g[1] - g[2], n2 = g[3] - g[4], n3 = g[5] - g[6];
    const G n4 = G(6) * g[0] - (px + py + pz);
    const G n5 = G(2) * px - py - pz;
    const G n6 = py - pz;
    const G qj = liquid ? r.qj : r.qjs, qe = liquid ? r.qe : r.qes;
    const G n1s = n1 - qj * (n1 - G(ux) * T);
    const G n2s = n2 - qj * (n2 - G(uy) * T);
    const G n3s = n3 - qj * (n3 - G(uz) * T);
    const G n4s = n4 - qe * (n4 - G(0.75) * Tt);
    const G ke = G(1) - qe;
    const G b0 = Tt * G(1.0 / 7.0);
    const G b1 = G(0.5) * n1s, b2 = G(0.5) * n2s, b3 = G(0.5) * n3s;
    const G b4 = n4s * G(1.0 / 42.0), b5 = ke * n5 * G(1.0 / 12.0), b6 = ke * n6 * G(0.25);
    const G c1 = b0 - b4 + G(2) * b5;
    const G c3 = b0 - b4 - b5 + b6;
    const G c5 = b0 - b4 - b5 - b6;
    g[0] = b0 + G(6) * b4;
    g[1] = c1 + b1;
    g[2] = c1 - b1;
    g[3] = c3 + b2;
    g[4] = c3 - b2;
    g[5] = c5 + b3;
    g[6] = c5 - b3;
  }
  return bad;
}

// --------------------------------------------------------------- step kernel
// One cell of the fused step: pull-stream f and g, collide, store.  Addresses
// are a row pointer (64-bit, the same for a whole lattice row) plus a small
// per-lane offset q * pitch + x.  FWALL: no-slip of f at the front
// interpolated to the link fraction (a separate instantiation, so that the
// default halfway rule compiles to the same code as without the option).
template <typename Ts, bool FLOW, bool MZ, bool FWALL>
__device__ __forceinline__ void update_cell(
    int x, int y, int z, const Ts* __restrict__ fs, Ts* __restrict__ fd,
    const Ts* __restrict__ gs, Ts* __restrict__ gd, const int* __restrict__ cnt,
    const uint32_t* __restrict__ cext, const double* __restrict__ s,
    const double* __restrict__ th, int* __restrict__ flag, const KParams& P) {
  using C = typename Compute<Ts>::type;
  using G = typename Compute<Ts>::gtype;
  const int n = P.n;
  if (x >= n || y >= n) return;
  const uint32_t pitch = P.pitch;
  const uint32_t nn = (uint32_t)n * (uint32_t)n;
  const uint32_t self = (uint32_t)z * nn + (uint32_t)y * (uint32_t)n + (uint32_t)x;
  const int a = MZ ? z : y;  // coordinate along the melt axis
  const int o = MZ ? y : z;  // the other lateral coordinate
  const int col = o * n + x;
  const bool interior = (y > 0) & (y < n - 1) & (z > 0) & (z < n - 1);
  // min and max of the liquid counts over the 3x3 columns around this one:
  // with 16-bit storage one precomputed word per column (its kernel is held
  // to 64 registers), else taken from the counts here, which saves the
  // per-step neighbourhood kernel (clamped at the walls: a repeated column
  // leaves min and max unchanged).  The column's own count cc decides the
  // phase; with 16-bit storage it is loaded on the general path only (on the
  // fast path the extremes decide it), which saves one of the two column
  // loads per cell.
  int cc = 0, lo, hi;
  bool liquid = false;
  int nb[9];  // counts of the 3x3 columns, [(o offset + 1) * 3 + x offset + 1]
  if constexpr (sizeof(Ts) == 2) {
    const uint32_t w = cext[col];
    lo = (int)(w & 0xffffu);
    hi = (int)(w >> 16);
  } else {
    cc = cnt[col];
    liquid = a < cc;
    const int xm = x > 0 ? x - 1 : x, xp = x < n - 1 ? x + 1 : x;
    const int om = o > 0 ? o - 1 : o, op = o < n - 1 ? o + 1 : o;
    nb[0] = cnt[om * n + xm];
    nb[1] = cnt[om * n + x];
    nb[2] = cnt[om * n + xp];
    nb[3] = cnt[o * n + xm];
    nb[4] = cc;
    nb[5] = cnt[o * n + xp];
    nb[6] = cnt[op * n + xm];
    nb[7] = cnt[op * n + x];
    nb[8] = cnt[op * n + xp];
    lo = cc;
    hi = cc;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      lo = nb[k] < lo ? nb[k] : lo;
      hi = nb[k] > hi ? nb[k] : hi;
    }
  }
  // With 16-bit storage the general path packs the phases of the 3x3x3
  // stencil into one register instead (bit ((da + 1) * 3 + do + 1) * 3 + dx +
  // 1 for the cell at offsets dx, do and da along the melt axis); nine live
  // counts would spill under that kernel's register cap.  Against a load of
  // the count per link, measured at 256^3 (all-liquid / melting, us per step):
  // FP16 with the melt axis y 346 / 203 -> 322 / 167; BF16 with the melt axis
  // y 345 / 203 -> 323 / 162; either format with the melt axis z 341 / 154 ->
  // 323 / 146 (those three at 7 waves, where the mask does not spill).
  constexpr bool kMask = sizeof(Ts) == 2;
  uint32_t phase27 = 0;
  // phase of the in-box cell at offsets (dx, do) across and da along the melt
  // axis; the offsets are constants of the unrolled loops
  auto liquid_off = [&](int dx, int dob, int da) -> bool {
    if constexpr (kMask)
      return (phase27 >> (((da + 1) * 3 + dob + 1) * 3 + dx + 1)) & 1u;
    else if constexpr (sizeof(Ts) == 2)
      return a + da < cnt[(o + dob) * n + x + dx];
    else
      return a + da < nb[(dob + 1) * 3 + dx + 1];
  };
  const bool all_liq = (a + 1) < lo;
  const bool all_sol = (a - 1) >= hi;
  const bool fast = interior & (all_liq | all_sol);

  const Rates<C, G> r = make_rates<C, G>(P);

  C f[19];
  G g[7];

  if (__all(fast)) {
    // ---------- fast path: one phase, only x walls possible ----------
    if constexpr (sizeof(Ts) == 2) liquid = all_liq;  // a + 1 < lo <= cc, or a - 1 >= hi >= cc
    // Every source row lies in the 3x3 block of rows around (y, z).  Offsets
    // are counted from the block's first row (y - 1, z - 1), so all loads of
    // a distribution share one uniform base and differ by a 32-bit lane
    // offset; an x-wall bounce-back selects another offset, not another
    // pointer, and the loads of all directions stay in flight together.
    const Ts* gb = row_ptr<7>(gs, P, y - 1, z - 1);
    const Ts* fb = row_ptr<19>(fs, P, y - 1, z - 1);
    const uint32_t un = (uint32_t)n;
    auto row_ofs = [&](uint32_t Q, int dy, int dz) {  // row (y + dy, z + dz)
      return ((uint32_t)(1 + dz) * un + (uint32_t)(1 + dy)) * (Q * pitch);
    };
#pragma unroll
    for (int q = 0; q < 7; ++q) {
      const int ex = ex7(q);
      uint32_t i = row_ofs(7, -ey7(q), -ez7(q)) + q * pitch + (uint32_t)(x - ex);
      if (ex != 0) {  // adiabatic x wall: bounce-back
        const bool wall = ex > 0 ? (x == 0) : (x == n - 1);
        i = wall ? row_ofs(7, 0, 0) + opp7(q) * pitch + x : i;
      }
      g[q] = load_stream<G>(gb, i);
    }
    if (FLOW && liquid) {
#pragma unroll
      for (int q = 0; q < 19; ++q) {
        const int ex = ex19(q);
        uint32_t i = row_ofs(19, -ey19(q), -ez19(q)) + q * pitch + (uint32_t)(x - ex);
        if (ex != 0) {  // no-slip x wall: halfway bounce-back
          const bool wall = ex > 0 ? (x == 0) : (x == n - 1);
          i = wall ? row_ofs(19, 0, 0) + opp19(q) * pitch + x : i;
        }
        f[q] = load_stream<C>(fb, i);
      }
    }
    // FP32 storage: no instruction moves across this point, so the
    // collision is not scheduled among the loads.  The kernel then needs 64
    // instead of 76 VGPRs: 8 instead of 6 waves per SIMD, the loads of more
    // cells in flight (256^3 melting state 171.6 -> 163.3 us, all-liquid
    // 607.2 -> 599.4 us, 64^3 unchanged; the same results bit for bit).
    if constexpr (sizeof(Ts) == 4) __builtin_amdgcn_sched_barrier(0);
  } else {
    // ---------- general path: walls and the front, link by link ----------
    if constexpr (sizeof(Ts) == 2) {
      cc = cnt[col];
      liquid = a < cc;
    }
    if constexpr (kMask) {
      const int xm = x > 0 ? x - 1 : x, xp = x < n - 1 ? x + 1 : x;
      const int om = o > 0 ? o - 1 : o, op = o < n - 1 ? o + 1 : o;
      const int c9[9] = {cnt[om * n + xm], cnt[om * n + x], cnt[om * n + xp],
                         cnt[o * n + xm],  cc,               cnt[o * n + xp],
                         cnt[op * n + xm], cnt[op * n + x], cnt[op * n + xp]};
#pragma unroll
      for (int k = 0; k < 27; ++k)
        phase27 |= (uint32_t)(a + k / 9 - 1 < c9[k % 9]) << k;
    }
    // this row and the rows the directions pull from (valid rows only)
    const Ts* g_self = row_ptr<7>(gs, P, y, z);
    const Ts* f_self = row_ptr<19>(fs, P, y, z);
    auto g_src = [&](int q) { return row_ptr<7>(gs, P, y - ey7(q), z - ez7(q)); };
    auto f_src = [&](int q) { return row_ptr<19>(fs, P, y - ey19(q), z - ez19(q)); };
    const double s_self = s[col];
    const G wTm = G(kW7Axis) * (G)(P.t_m - P.tref);
#pragma unroll
    for (int q = 0; q < 7; ++q) {
      const int ex = ex7(q), ey = ey7(q), ez = ez7(q), p = opp7(q);
      const int sx = x - ex, sy = y - ey, sz = z - ez;
      G v;
      if ((unsigned)sx >= (unsigned)n || (unsigned)sy >= (unsigned)n || (unsigned)sz >= (unsigned)n) {
        // thermal wall: Dirichlet (anti-bounce-back) or adiabatic (bounce-back)
        const int sa = MZ ? sz : sy;
        const G gp = load_stream<G>(g_self, p * pitch + x);
        if (sa < 0) {
          v = -gp + G(2.0 * kW7Axis) * (G)(th[col] - P.tref);
        } else if (!MZ && sa >= n) {
          v = -gp + G(2.0 * kW7Axis) * (G)(P.t_c - P.tref);
        } else {
          v = gp;
        }
      } else {
        const int sa = MZ ? sz : sy, so = MZ ? sy : sz;
        const int scol = so * n + sx;
        const bool src_liq = liquid_off(-ex, MZ ? -ey : -ez, sa - a);
        if (src_liq == liquid) {
          v = load_stream<G>(g_src(q), q * pitch + sx);
        } else {
          // interpolated anti-bounce-back at the front (wall value t_m)
          const bool along = MZ ? (ez != 0) : (ey != 0);
          double d;
          if (along) {
            d = fabs(s_self - (a + 0.5));
          } else {
            d = ((a + 0.5) - s_self) / (s[scol] - s_self);
          }
          const G dl = (G)d;
          const G gp = load_stream<G>(g_self, p * pitch + x);
          if (d < 0.5) {
            const int bx = x + ex, by = y + ey, bz = z + ez;
            bool behind = (unsigned)bx < (unsigned)n && (unsigned)by < (unsigned)n &&
                          (unsigned)bz < (unsigned)n;
            if (behind) {
              const int ba = MZ ? bz : by;
              behind = liquid_off(ex, MZ ? ey : ez, ba - a) == liquid;
            }
            if (behind) {
              const G gb = load_stream<G>(row_ptr<7>(gs, P, by, bz), p * pitch + bx);
              v = -(G(2) * dl * gp + (G(1) - G(2) * dl) * gb) + G(2) * wTm;
            } else {
              v = -gp + G(2) * wTm;
            }
          } else {
            const G inv2d = G(1) / (G(2) * dl);
            v = -gp * inv2d + (G(2) * dl - G(1)) * inv2d * load_stream<G>(g_self, q * pitch + x) +
                wTm / dl;
          }
        }
      }
      g[q] = v;
    }
    if (FLOW && liquid) {
#pragma unroll
      for (int q = 0; q < 19; ++q) {
        const int ex = ex19(q), ey = ey19(q), ez = ez19(q), p = opp19(q);
        const int sx = x - ex, sy = y - ey, sz = z - ez;
        const bool inb = (unsigned)sx < (unsigned)n && (unsigned)sy < (unsigned)n &&
                         (unsigned)sz < (unsigned)n;
        bool ok = inb;
        int scol = 0;
        if (inb) {
          const int sa = MZ ? sz : sy, so = MZ ? sy : sz;
          scol = so * n + sx;
          ok = liquid_off(-ex, MZ ? -ey : -ez, sa - a);
        }
        // halfway bounce-back from walls and solid cells (address select: the
        // source row of an out-of-box link is never dereferenced)
        const Ts* src = ok ? f_src(q) + ((int)(q * pitch) + sx) : f_self + (p * pitch + x);
        C v = load_stream<C>(src, 0);
        if (FWALL && inb && !ok) {
          // Solid source: bounce back from where the front cuts the link.  The
          // height on the melt axis and the front (linear between the two
          // columns) meet at fraction d of the link; the weights sum to one,
          // so they apply to the shifted populations as stored.
          const int ea = MZ ? ez : ey;
          const double d = ((a + 0.5) - s_self) / ((s[scol] - s_self) + ea);
          const C dl = (C)d;
          if (d < 0.5) {
            const int bx = x + ex, by = y + ey, bz = z + ez;
            bool behind = (unsigned)bx < (unsigned)n && (unsigned)by < (unsigned)n &&
                          (unsigned)bz < (unsigned)n;
            if (behind) {
              const int ba = MZ ? bz : by;
              behind = liquid_off(ex, MZ ? ey : ez, ba - a);
            }
            if (behind)  // else halfway bounce-back, as the front condition of g does
              v = C(2) * dl * v +
                  (C(1) - C(2) * dl) * load_stream<C>(row_ptr<19>(fs, P, by, bz), p * pitch + bx);
          } else {
            const C inv2d = C(1) / (C(2) * dl);
            v = v * inv2d + (C(2) * dl - C(1)) * inv2d * load_stream<C>(f_self, q * pitch + x);
          }
        }
        f[q] = v;
      }
    }
  }
  if (collide<FLOW>(f, g, liquid, r)) *flag = 1;
  uint32_t rs = mix32(self * 0x9e3779b1u + step_of(P) * 0x85ebca77u);
  if (FLOW && liquid) {
    Ts* fr = row_ptr<19>(fd, P, y, z);
#pragma unroll
    for (int q = 0; q < 19; ++q) store_stream(fr, q * pitch + x, f[q], rs);
  }
  Ts* gr = row_ptr<7>(gd, P, y, z);
#pragma unroll
  for (int q = 0; q < 7; ++q) store_stream(gr, q * pitch + x, g[q], rs);
}

// A cell of a lattice row whose cells and 3x3x3 stencils are all solid, off
// the y and z walls (16-bit storage): only g moves.  The row is known to be
// such a row from one uniform load (the row maximum of the liquid counts), so
// the cell issues its 7 population loads at once, without first loading the
// liquid counts of its column and their neighbourhood extremes.  Those solid
// cells are latency-bound (14 bytes of loads per cell); the round trip saved
// is a quarter of their time.  The arithmetic, the x-wall bounce-back and
// the rounding stream are those of the fast path of update_cell, so the
// results are the same bit for bit.
template <typename Ts, bool FLOW, bool MZ>
__device__ __forceinline__ void solid_cell(int x, int y, int z, const Ts* __restrict__ gs,
                                           Ts* __restrict__ gd, int* __restrict__ flag,
                                           const KParams& P) {
  using C = typename Compute<Ts>::type;
  using G = typename Compute<Ts>::gtype;
  const int n = P.n;
  if (x >= n) return;
  const uint32_t pitch = P.pitch;
  const Ts* gb = row_ptr<7>(gs, P, y - 1, z - 1);  // y, z are interior rows
  const uint32_t un = (uint32_t)n;
  auto row_ofs = [&](uint32_t Q, int dy, int dz) {  // row (y + dy, z + dz)
    return ((uint32_t)(1 + dz) * un + (uint32_t)(1 + dy)) * (Q * pitch);
  };
  G g[7];
#pragma unroll
  for (int q = 0; q < 7; ++q) {
    const int ex = ex7(q);
    uint32_t i = row_ofs(7, -ey7(q), -ez7(q)) + q * pitch + (uint32_t)(x - ex);
    if (ex != 0) {  // adiabatic x wall: bounce-back
      const bool wall = ex > 0 ? (x == 0) : (x == n - 1);
      i = wall ? row_ofs(7, 0, 0) + opp7(q) * pitch + x : i;
    }
    g[q] = load_stream<G>(gb, i);
  }
  const Rates<C, G> r = make_rates<C, G>(P);
  C fdummy[19];  // not read: the cell is solid
  if (collide<FLOW>(fdummy, g, false, r)) *flag = 1;
  const uint32_t nn = (uint32_t)n * (uint32_t)n;
  const uint32_t self = (uint32_t)z * nn + (uint32_t)y * (uint32_t)n + (uint32_t)x;
  uint32_t rs = mix32(self * 0x9e3779b1u + step_of(P) * 0x85ebca77u);
  Ts* gr = row_ptr<7>(gd, P, y, z);
#pragma unroll
  for (int q = 0; q < 7; ++q) store_stream(gr, q * pitch + x, g[q], rs);
}

template <typename Ts, bool FLOW, bool MZ, bool FWALL>
__global__ __launch_bounds__(512) void k_stream_collide(
    const Ts* __restrict__ fs, Ts* __restrict__ fd, const Ts* __restrict__ gs,
    Ts* __restrict__ gd, const int* __restrict__ cnt, const double* __restrict__ s,
    const double* __restrict__ th, int* __restrict__ flag, KParams P) {
  int y, z, xb;
  step_row<row_run<Ts>()>(P, y, z, xb);
  const int x = xb * blockDim.x + threadIdx.x;
  update_cell<Ts, FLOW, MZ, FWALL>(x, y, z, fs, fd, gs, gd, cnt, nullptr, s, th, flag, P);
}

// The same for 16-bit storage, held to 7 or 8 resident waves per SIMD.  Its
// instruction stream is long for the bytes it moves (conversions and the
// rounding of 26 values), and more resident waves hide more of it.  The
// conduction-only step (g alone) fits 8 waves.  With flow the general path
// needs 65 VGPRs for its phase mask: at 8 waves it spills, at 7 nothing
// does.  FP16 with the melt axis y once ran at 8 with a 12-byte spill; with
// the solid-row path (solid_cell) that spill grew to 32 bytes and the
// all-liquid 256^3 step went from 305 to 404 us, while at 7 waves it takes
// 304 us.  (For FP32 an 8-wave limit spills 60 bytes and costs 24 %.)
template <typename Ts, bool FLOW, bool MZ, bool FWALL>
constexpr int kWaves16 = !FLOW ? 8 : 7;
// PAIR: the row order that keeps both halves of a row on one XCD (two
// workgroups per row; see step_row).
template <typename Ts, bool FLOW, bool MZ, bool FWALL, bool PAIR>
__global__ __launch_bounds__(512) __attribute__((
    amdgpu_waves_per_eu(kWaves16<Ts, FLOW, MZ, FWALL>, kWaves16<Ts, FLOW, MZ, FWALL>))) void
k_stream_collide_h(const Ts* __restrict__ fs, Ts* __restrict__ fd, const Ts* __restrict__ gs,
                   Ts* __restrict__ gd, const int* __restrict__ cnt,
                   const uint32_t* __restrict__ cext, const int* __restrict__ rowmax,
                   const double* __restrict__ s, const double* __restrict__ th,
                   int* __restrict__ flag, KParams P) {
  int y, z, xb;
  step_row<row_run<Ts>(), PAIR>(P, y, z, xb);
  const int x = xb * blockDim.x + threadIdx.x;
  if (rowmax) {
    // rowmax[o]: the largest liquid count over the 3x3 neighbourhoods of the
    // columns with this other-lateral index, so every stencil of the row is
    // solid when its height a satisfies a - 1 >= rowmax[o] (uniform)
    const int n = P.n, a = MZ ? z : y, o = MZ ? y : z;
    if (a - 1 >= rowmax[o] && a <= n - 2 && o >= 1 && o <= n - 2) {
      solid_cell<Ts, FLOW, MZ>(x, y, z, gs, gd, flag, P);
      return;
    }
  }
  update_cell<Ts, FLOW, MZ, FWALL>(x, y, z, fs, fd, gs, gd, cnt, cext, s, th, flag, P);
}

// --------------------------------------------------------------- front update
// Gradient of the one-sided quadratic through (0, tm), (xi0, T0v), (xi1, T1v)
// at xi = 0; with one node, the chord slope.
__device__ __forceinline__ double one_sided(int k, double xi0, double T0v, double xi1, double T1v,
                                            double tm) {
  if (k >= 2)
    return ((T0v - tm) * xi1 * xi1 - (T1v - tm) * xi0 * xi0) / (xi0 * xi1 * (xi1 - xi0));
  if (k == 1 && xi0 > 0.0) return (T0v - tm) / xi0;
  return 0.0;
}

template <typename Ts>
__device__ __forceinline__ double cell_T(const Ts* __restrict__ g, const KParams& P, int x, int y,
                                         int z) {
  const Ts* row = row_ptr<7>(g, P, y, z);
  double acc = 0.0;
#pragma unroll
  for (int q = 0; q < 7; ++q) acc += (double)load(row, q * P.pitch + x);
  return acc + P.tref;
}


template <typename Ts, bool FLOW, bool MZ>
__global__ __launch_bounds__(256) void k_front(const double* __restrict__ s_old,
                                               double* __restrict__ s_new, int* __restrict__ cnt,
                                               const Ts* __restrict__ g, Ts* __restrict__ f,
                                               const double* __restrict__ th,
                                               int* __restrict__ melted, int* __restrict__ frozen,
                                               int* __restrict__ flag,
                                               const int* __restrict__ replay,
                                               const int* __restrict__ replay_next,
                                               int* __restrict__ record,
                                               const double* __restrict__ heat,
                                               uint32_t* __restrict__ step_ctr, KParams P) {
  const int n = P.n;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int o = blockIdx.y;
  // the step counter of graph replays: no later kernel of this step reads it
  if (step_ctr && x == 0 && o == 0) *step_ctr += 1u;
  if (x >= n) return;
  const int col = o * n + x;
  const uint32_t nn = (uint32_t)n * (uint32_t)n;
  // temperature of the cell at height a of this column
  auto T_at = [&](int a) { return MZ ? cell_T(g, P, x, o, a) : cell_T(g, P, x, a, o); };
  const double sc = s_old[col];
  const int c0 = cnt[col];

  // node selection: the nearest liquid and solid centres at distance >= 1/2
  // from the front (only the very nearest can be closer); a recorded
  // schedule replaces it when replaying a run along fixed phases and nodes
  int a_top, a_bot;
  if (replay) {
    a_top = replay[nn + col];
    a_bot = replay[2 * nn + col];
  } else {
    a_top = c0 - 1;
    if (a_top >= 0 && sc - (a_top + 0.5) < 0.5) --a_top;
    a_bot = c0;
    if (a_bot < n && (a_bot + 0.5) - sc < 0.5) ++a_bot;
  }
  if (record) {
    record[col] = c0;
    record[nn + col] = a_top;
    record[2 * nn + col] = a_bot;
  }

  // front velocity: Eq. (6) from one-sided temperature gradients, or (heat
  // given) the heat the lattice carried into this column's front over L
  auto gradient_velocity = [&]() -> double {
    // The nodes are a_top, a_top - 1 (liquid side) and a_bot, a_bot + 1
    // (solid side) where they lie in the box.  Their temperatures, the
    // neighbouring fronts and the hot-wall temperature are loaded together
    // (heights clamped into the box; a candidate outside it is not used).
    auto in_box = [&](int a) { return a < 0 ? 0 : (a > n - 1 ? n - 1 : a); };
    const double Tl0 = T_at(in_box(a_top)), Tl1 = T_at(in_box(a_top - 1));
    const double Ts0 = T_at(in_box(a_bot)), Ts1 = T_at(in_box(a_bot + 1));
    const double thc = th[col];
    // front slopes by central differences, mirrored at the walls
    const double sxp = s_old[o * n + (x + 1 < n ? x + 1 : x)];
    const double sxm = s_old[o * n + (x > 0 ? x - 1 : x)];
    const double sop = s_old[(o + 1 < n ? o + 1 : o) * n + x];
    const double som = s_old[(o > 0 ? o - 1 : o) * n + x];

    // liquid side: the nodes toward the heated wall, then the wall
    double xi0 = 0, T0v = 0, xi1 = 0, T1v = 0;
    int k = 0;
    if (a_top >= 0) {
      xi0 = sc - (a_top + 0.5);
      T0v = Tl0;
      k = 1;
      if (a_top - 1 >= 0) {
        xi1 = sc - ((a_top - 1) + 0.5);
        T1v = Tl1;
        k = 2;
      }
    }
    if (k < 2) {
      if (k == 0) { xi0 = sc; T0v = thc; } else { xi1 = sc; T1v = thc; }
      ++k;
    }
    const double Gl = -one_sided(k, xi0, T0v, xi1, T1v, P.t_m);

    // solid side: nodes beyond the front, then the cold wall (melt axis y)
    k = 0;
    if (a_bot < n) {
      xi0 = (a_bot + 0.5) - sc;
      T0v = Ts0;
      k = 1;
      if (a_bot + 1 < n) {
        xi1 = ((a_bot + 1) + 0.5) - sc;
        T1v = Ts1;
        k = 2;
      }
    }
    if (k < 2 && !MZ) {
      if (k == 0) { xi0 = n - sc; T0v = P.t_c; } else { xi1 = n - sc; T1v = P.t_c; }
      ++k;
    }
    const double Gs = one_sided(k, xi0, T0v, xi1, T1v, P.t_m);

    const double dsx = 0.5 * (sxp - sxm), dso = 0.5 * (sop - som);
    // Eq. (6): k_s dT_s - k_l dT_l in units of k_l (kappa = k_s / k_l)
    return (1.0 + dsx * dsx + dso * dso) * P.alpha * P.ste * (P.kappa * Gs - Gl) / P.dT;
  };
  const double V = heat ? heat[col] * P.ste / P.dT : gradient_velocity();
  double sn = sc + V;
  if (!(sn == sn)) *flag = 1;
  sn = sn < 0.0 ? 0.0 : (sn > (double)n ? (double)n : sn);
  s_new[col] = sn;

  // phase switch: newly liquid cells start from the rest state of f
  const int c1 = replay_next ? replay_next[col] : count_liquid(sn, n);
  if (FLOW) {
    for (int a = c0; a < c1; ++a) {
      Ts* row = MZ ? row_ptr<19>(f, P, o, a) : row_ptr<19>(f, P, a, o);
#pragma unroll
      for (int q = 0; q < 19; ++q) store(row, q * P.pitch + x, 0.0f);
    }
  }
  if (c1 > c0) melted[col] += c1 - c0;
  if (c1 < c0) frozen[col] += c0 - c1;
  cnt[col] = c1;
}

__global__ void k_counts(const double* __restrict__ s, int* __restrict__ cnt, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n * n) cnt[i] = count_liquid(s[i], n);
}

// One workgroup per row of columns o: the min and max liquid count of every
// column's 3x3 neighbourhood, packed into one word (min in the low 16 bits,
// max in the high; counts are at most n <= 1024), and (rowmax != null) the
// largest max of the row, which bounds the liquid counts near every cell of
// the lattice rows with this o.
constexpr int kNbThreads = 256;
__global__ __launch_bounds__(kNbThreads) void k_neighbourhood(const int* __restrict__ cnt,
                                                              uint32_t* __restrict__ cext,
                                                              int* __restrict__ rowmax, int n) {
  __shared__ int sh[kNbThreads / 64];
  const int o = blockIdx.x;
  int rmax = -1;
  for (int x = threadIdx.x; x < n; x += kNbThreads) {
    int lo = 0x7fffffff, hi = -1;
    for (int d_o = -1; d_o <= 1; ++d_o) {
      const int oo = o + d_o;
      if (oo < 0 || oo >= n) continue;
      for (int dx = -1; dx <= 1; ++dx) {
        const int xx = x + dx;
        if (xx < 0 || xx >= n) continue;
        const int c = cnt[oo * n + xx];
        lo = c < lo ? c : lo;
        hi = c > hi ? c : hi;
      }
    }
    cext[o * n + x] = (uint32_t)lo | ((uint32_t)hi << 16);
    rmax = hi > rmax ? hi : rmax;
  }
  if (!rowmax) return;  // uniform
  for (int off = 32; off > 0; off >>= 1) {
    const int v = __shfl_down(rmax, off, 64);
    rmax = v > rmax ? v : rmax;
  }
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = rmax;
  __syncthreads();
  if (threadIdx.x == 0) {
    int m = sh[0];
    for (int w = 1; w < kNbThreads / 64; ++w) m = sh[w] > m ? sh[w] : m;
    rowmax[o] = m;
  }
}

// --------------------------------------------------------------- init, fields
template <typename Ts, bool MZ>
__global__ void k_init(const double* __restrict__ seedT, Ts* __restrict__ f, Ts* __restrict__ g,
                       KParams P) {
  const int n = P.n;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y, z = blockIdx.z;
  if (x >= n) return;
  const int a = MZ ? z : y;
  const double Tt = seedT[a] - P.tref;  // per height, solid heights included
  Ts* gr = row_ptr<7>(g, P, y, z);
  store(gr, x, kW7Rest * Tt);
  for (int q = 1; q < 7; ++q) store(gr, q * P.pitch + x, kW7Axis * Tt);
  if (P.flow) {
    Ts* fr = row_ptr<19>(f, P, y, z);
    for (int q = 0; q < 19; ++q) store(fr, q * P.pitch + x, 0.0);
  }
}

template <typename Ts, bool MZ>
__global__ void k_fields(const Ts* __restrict__ f, const Ts* __restrict__ g,
                         const int* __restrict__ cnt, double* __restrict__ T,
                         double* __restrict__ ux, double* __restrict__ uy,
                         double* __restrict__ uz, double* __restrict__ rho, KParams P) {
  const int n = P.n;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y, z = blockIdx.z;
  if (x >= n) return;
  const uint32_t i = ((uint32_t)z * n + y) * n + x;
  const int a = MZ ? z : y, o = MZ ? y : z;
  const bool liquid = a < cnt[o * n + x];
  double Tt = 0.0;
  const Ts* gr = row_ptr<7>(g, P, y, z);
  for (int q = 0; q < 7; ++q) Tt += (double)load(gr, q * P.pitch + x);
  double r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
  if (P.flow && liquid) {
    const Ts* fr = row_ptr<19>(f, P, y, z);
    double d = 0.0;
    for (int q = 0; q < 19; ++q) {
      const double v = (double)load(fr, q * P.pitch + x);
      d += v;
      jx += ex19(q) * v;
      jy += ey19(q) * v;
      jz += ez19(q) * v;
    }
    r = 1.0 + d;
    jz -= 0.5 * P.gbeta * (Tt + P.tref - P.t0);
  }
  if (T) T[i] = Tt + P.tref;
  if (rho) rho[i] = r;
  if (ux) ux[i] = jx;
  if (uy) uy[i] = jy;
  if (uz) uz[i] = jz;
}

// --------------------------------------------------------------- conversions
__device__ __forceinline__ double weight(int qcount, int q) {
  if (qcount == 7) return q == 0 ? kW7Rest : kW7Axis;
  const int e2 = ex19(q) * ex19(q) + ey19(q) * ey19(q) + ez19(q) * ez19(q);
  return e2 == 0 ? 1.0 / 3.0 : (e2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
}

template <typename Ts>
__global__ void k_to_storage(const double* __restrict__ src, Ts* __restrict__ dst, int qcount,
                             KParams P) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t total = (uint64_t)qcount * P.ncell;
  if (i >= total) return;
  const int q = (int)(i / P.ncell);
  const uint32_t cell = (uint32_t)(i - (uint64_t)q * P.ncell);
  const uint32_t n = (uint32_t)P.n, x = cell % n, y = (cell / n) % n, z = cell / (n * n);
  const double shift = weight(qcount, q) * (qcount == 7 ? P.tref : 1.0);
  dst[pop_index(P, qcount, q, x, y, z)] = static_cast<Ts>(src[i] - shift);
}

template <typename Ts>
__global__ void k_from_storage(const Ts* __restrict__ src, double* __restrict__ dst, int qcount,
                               KParams P) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t total = (uint64_t)qcount * P.ncell;
  if (i >= total) return;
  const int q = (int)(i / P.ncell);
  const uint32_t cell = (uint32_t)(i - (uint64_t)q * P.ncell);
  const uint32_t n = (uint32_t)P.n, x = cell % n, y = (cell / n) % n, z = cell / (n * n);
  const double shift = weight(qcount, q) * (qcount == 7 ? P.tref : 1.0);
  dst[i] = (double)static_cast<typename Compute<Ts>::type>(src[pop_index(P, qcount, q, x, y, z)]) +
           shift;
}

// --------------------------------------------------------------- reductions
constexpr int kSumThreads = 1024;

__device__ __forceinline__ double block_sum(double v, double* sh) {
  // deterministic: fixed shuffle tree inside the wave, fixed order across waves
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kSumThreads / 64; ++w) t += sh[w];
  __syncthreads();
  return t;
}

__global__ __launch_bounds__(kSumThreads) void k_sum(const double* __restrict__ v, int64_t count,
                                                     double* __restrict__ out) {
  __shared__ double sh[kSumThreads / 64];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < count; i += kSumThreads) acc += v[i];
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) out[0] = t;
}

// --------------------------------------------------------------- dispatch
template <typename Ts>
hipError_t sc_dispatch(const KParams& P, const void* fs, void* fd, const void* gs, void* gd,
                       const int* cnt, const uint32_t* cext, const int* rowmax,
                       const double* s, const double* th, int* flag, hipStream_t st,
                       hipEvent_t ev_start, hipEvent_t ev_stop) {
  auto F = static_cast<const Ts*>(fs);
  auto Fd = static_cast<Ts*>(fd);
  auto G = static_cast<const Ts*>(gs);
  auto Gd = static_cast<Ts*>(gd);
  // one whole x row per workgroup (up to 512 cells; 256 with 16-bit
  // storage): the +-1-shifted loads of a row hit cache lines the same
  // workgroup fetches, and the row pointers are uniform.  The 16-bit kernels
  // run 7 waves per SIMD, 28 per compute unit: workgroups of 8 waves leave 4
  // of those slots empty, workgroups of 4 fill all of them (512^3,
  // bottom-heated FP16: melting state 786 -> 713 us, all-liquid 2520 -> 2445
  // us per step, two runs each)
  const int bmax = step_block_max(sizeof(Ts));
  const int bx = P.n >= bmax ? bmax : ((P.n + 63) / 64) * 64;
  dim3 block(bx, 1, 1);
  dim3 grid((P.n + bx - 1) / bx, P.n, P.n);
  // the paired row order applies at two workgroups per row only
  const bool pair = P.pair_rows != 0 && grid.x == 2 && (P.n & 7) == 0;
#define LAUNCH_ONE(K, ...)                                                                      \
  do {                                                                                          \
    if (ev_start)  /* the dispatch itself records the kernel's start and end */                 \
      hipExtLaunchKernelGGL(K, grid, block, 0, st, ev_start, ev_stop, 0, __VA_ARGS__);          \
    else                                                                                        \
      hipLaunchKernelGGL(K, grid, block, 0, st, __VA_ARGS__);                                   \
  } while (0)
#define LAUNCH(FLOW, MZ, FWALL)                                                                \
  do {                                                                                          \
    if constexpr (sizeof(Ts) == 2) {                                                            \
      if (pair)                                                                                 \
        LAUNCH_ONE((k_stream_collide_h<Ts, FLOW, MZ, FWALL, true>), F, Fd, G, Gd, cnt, cext,     \
                   rowmax, s, th, flag, P);                                                     \
      else                                                                                      \
        LAUNCH_ONE((k_stream_collide_h<Ts, FLOW, MZ, FWALL, false>), F, Fd, G, Gd, cnt, cext,    \
                   rowmax, s, th, flag, P);                                                     \
    } else                                                                                      \
      LAUNCH_ONE((k_stream_collide<Ts, FLOW, MZ, FWALL>), F, Fd, G, Gd, cnt, s, th, flag, P);    \
  } while (0)
  if (P.flow && P.f_wall) {
    if (P.melt_z) LAUNCH(true, true, true); else LAUNCH(true, false, true);
  } else if (P.flow) {
    if (P.melt_z) LAUNCH(true, true, false); else LAUNCH(true, false, false);
  } else {
    if (P.melt_z) LAUNCH(false, true, false); else LAUNCH(false, false, false);
  }
#undef LAUNCH_ONE
#undef LAUNCH
  return hipGetLastError();
}

template <typename Ts>
hipError_t front_dispatch(const KParams& P, const double* s_old, double* s_new, int* cnt,
                          const void* g, void* f, const double* th, int* melted, int* frozen,
                          int* flag, const int* replay, const int* replay_next, int* record,
                          const double* heat, uint32_t* step_ctr, hipStream_t st) {
  dim3 block(64, 1, 1);
  dim3 grid((P.n + 63) / 64, P.n, 1);
  auto G = static_cast<const Ts*>(g);
  auto F = static_cast<Ts*>(f);
#define LAUNCH(FLOW, MZ)                                                                   \
  hipLaunchKernelGGL((k_front<Ts, FLOW, MZ>), grid, block, 0, st, s_old, s_new, cnt, G, F, th, \
                     melted, frozen, flag, replay, replay_next, record, heat, step_ctr, P)
  if (P.flow) {
    if (P.melt_z)
      LAUNCH(true, true);
    else
      LAUNCH(true, false);
  } else {
    if (P.melt_z)
      LAUNCH(false, true);
    else
      LAUNCH(false, false);
  }
#undef LAUNCH
  return hipGetLastError();
}

template <typename Ts>
hipError_t init_dispatch(const KParams& P, const double* seedT, void* f, void* g, hipStream_t st) {
  dim3 block(64, 1, 1);
  dim3 grid((P.n + 63) / 64, P.n, P.n);
  if (P.melt_z)
    hipLaunchKernelGGL((k_init<Ts, true>), grid, block, 0, st, seedT, static_cast<Ts*>(f),
                       static_cast<Ts*>(g), P);
  else
    hipLaunchKernelGGL((k_init<Ts, false>), grid, block, 0, st, seedT, static_cast<Ts*>(f),
                       static_cast<Ts*>(g), P);
  return hipGetLastError();
}

template <typename Ts>
hipError_t fields_dispatch(const KParams& P, const void* f, const void* g, const int* cnt,
                           double* T, double* ux, double* uy, double* uz, double* rho,
                           hipStream_t st) {
  dim3 block(64, 1, 1);
  dim3 grid((P.n + 63) / 64, P.n, P.n);
  if (P.melt_z)
    hipLaunchKernelGGL((k_fields<Ts, true>), grid, block, 0, st, static_cast<const Ts*>(f),
                       static_cast<const Ts*>(g), cnt, T, ux, uy, uz, rho, P);
  else
    hipLaunchKernelGGL((k_fields<Ts, false>), grid, block, 0, st, static_cast<const Ts*>(f),
                       static_cast<const Ts*>(g), cnt, T, ux, uy, uz, rho, P);
  return hipGetLastError();
}

template <typename Ts>
hipError_t conv_dispatch(bool to_storage, const KParams& P, int qcount, const void* src,
                         void* dst, hipStream_t st) {
  const uint64_t total = (uint64_t)qcount * P.ncell;
  dim3 block(256, 1, 1);
  dim3 grid((unsigned)((total + 255) / 256), 1, 1);
  if (to_storage)
    hipLaunchKernelGGL((k_to_storage<Ts>), grid, block, 0, st, static_cast<const double*>(src),
                       static_cast<Ts*>(dst), qcount, P);
  else
    hipLaunchKernelGGL((k_from_storage<Ts>), grid, block, 0, st, static_cast<const Ts*>(src),
                       static_cast<double*>(dst), qcount, P);
  return hipGetLastError();
}

}  // namespace

#define LBMK_DISPATCH(kind, call)            \
  switch (kind) {                            \
    case kF64: return call<double>;          \
    case kF32: return call<float>;           \
    case kF16S: return call<_Float16>;       \
    case kBF16S: return call<__bf16>;        \
    default: return hipErrorInvalidValue;    \
  }

uint32_t row_pitch(int n, int kind) {
  // rows start on 128-byte boundaries
  const uint32_t e = (uint32_t)store_bytes(kind);
  if (!e) return 0;
  const uint32_t bytes = ((uint32_t)n * e + 127u) / 128u * 128u;
  return bytes / e;
}

size_t store_bytes(int kind) {
  switch (kind) {
    case kF64: return 8;
    case kF32: return 4;
    case kF16S:
    case kBF16S: return 2;
    default: return 0;
  }
}

hipError_t launch_stream_collide(int kind, const KParams& P, const void* fs, void* fd,
                                 const void* gs, void* gd, const int* cnt, const uint32_t* cext,
                                 const int* rowmax, const double* s, const double* th, int* flag,
                                 hipStream_t st, hipEvent_t ev_start, hipEvent_t ev_stop) {
#define CALL(T) \
  sc_dispatch<T>(P, fs, fd, gs, gd, cnt, cext, rowmax, s, th, flag, st, ev_start, ev_stop)
  switch (kind) {
    case kF64: return CALL(double);
    case kF32: return CALL(float);
    case kF16S: return CALL(_Float16);
    case kBF16S: return CALL(__bf16);
    default: return hipErrorInvalidValue;
  }
#undef CALL
}

hipError_t launch_front(int kind, const KParams& P, const double* s_old, double* s_new, int* cnt,
                        const void* g, void* f, const double* th, int* melted, int* frozen,
                        int* flag, const int* replay, const int* replay_next, int* record,
                        const double* heat, uint32_t* step_ctr, hipStream_t st) {
#define CALL(T)                                                                                 \
  front_dispatch<T>(P, s_old, s_new, cnt, g, f, th, melted, frozen, flag, replay, replay_next, \
                    record, heat, step_ctr, st)
  switch (kind) {
    case kF64: return CALL(double);
    case kF32: return CALL(float);
    case kF16S: return CALL(_Float16);
    case kBF16S: return CALL(__bf16);
    default: return hipErrorInvalidValue;
  }
#undef CALL
}

hipError_t launch_neighbourhood(const KParams& P, const int* cnt, uint32_t* cext, int* rowmax,
                                hipStream_t st) {
  hipLaunchKernelGGL(k_neighbourhood, dim3(P.n), dim3(kNbThreads), 0, st, cnt, cext, rowmax,
                     P.n);
  return hipGetLastError();
}

__global__ void k_set_u32(uint32_t* p, uint32_t v) { *p = v; }

hipError_t launch_set_u32(uint32_t* p, uint32_t v, hipStream_t st) {
  hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(1), 0, st, p, v);
  return hipGetLastError();
}

hipError_t launch_counts(const KParams& P, const double* s, int* cnt, hipStream_t st) {
  const int total = P.n * P.n;
  hipLaunchKernelGGL(k_counts, dim3((total + 255) / 256), dim3(256), 0, st, s, cnt, P.n);
  return hipGetLastError();
}

hipError_t launch_init(int kind, const KParams& P, const double* seedT, void* f, void* g,
                       hipStream_t st) {
#define CALL(T) init_dispatch<T>(P, seedT, f, g, st)
  switch (kind) {
    case kF64: return CALL(double);
    case kF32: return CALL(float);
    case kF16S: return CALL(_Float16);
    case kBF16S: return CALL(__bf16);
    default: return hipErrorInvalidValue;
  }
#undef CALL
}

hipError_t launch_fields(int kind, const KParams& P, const void* f, const void* g, const int* cnt,
                         double* T, double* ux, double* uy, double* uz, double* rho,
                         hipStream_t st) {
#define CALL(T_) fields_dispatch<T_>(P, f, g, cnt, T, ux, uy, uz, rho, st)
  switch (kind) {
    case kF64: return CALL(double);
    case kF32: return CALL(float);
    case kF16S: return CALL(_Float16);
    case kBF16S: return CALL(__bf16);
    default: return hipErrorInvalidValue;
  }
#undef CALL
}

hipError_t launch_to_storage(int kind, const KParams& P, int q_count, const double* src, void* dst,
                             hipStream_t st) {
#define CALL(T) conv_dispatch<T>(true, P, q_count, src, dst, st)
  switch (kind) {
    case kF64: return CALL(double);
    case kF32: return CALL(float);
    case kF16S: return CALL(_Float16);
    case kBF16S: return CALL(__bf16);
    default: return hipErrorInvalidValue;
  }
#undef CALL
}

hipError_t launch_from_storage(int kind, const KParams& P, int q_count, const void* src,
                               double* dst, hipStream_t st) {
#define CALL(T) conv_dispatch<T>(false, P, q_count, src, dst, st)
  switch (kind) {
    case kF64: return CALL(double);
    case kF32: return CALL(float);
    case kF16S: return CALL(_Float16);
    case kBF16S: return CALL(__bf16);
    default: return hipErrorInvalidValue;
  }
#undef CALL
}

hipError_t launch_sum(const double* v, int64_t count, double* out, hipStream_t st) {
  if (!v || !out || count < 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(kSumThreads), 0, st, v, count, out);
  return hipGetLastError();
}


}  // namespace lbmk
