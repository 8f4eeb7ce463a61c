// Host side of liblbmmelt: the C ABI declared in include/lbmmelt.h.
//
// Owns the device memory of one simulation (double-buffered row-interleaved
// distributions in HBM, the front, per-column counters), maps the physical
// parameters of the problem statement (section 1 of Li, Yang & Zhang,
// arXiv:1604.03478) to lattice units, and enqueues the gfx950 kernels on one
// HIP stream.  Device work is asynchronous except where the header says a
// call synchronizes.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "lbm_adjoint.h"
#include "lbm_ceiling.h"
#include "lbm_diag.h"
#include "lbm_front_heat.h"
#include "lbm_internal.h"
#include "lbmmelt.h"

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(LBM_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));          \
  } while (0)

// Root of lam * exp(lam^2) * erf(lam) = Ste / sqrt(pi): the Neumann constant
// of one-dimensional melting without subcooling (section 3.1 verification
// case), by bisection.
double neumann_constant(double ste) {
  const double target = ste / std::sqrt(M_PI);
  auto h = [&](double l) { return l * std::exp(l * l) * std::erf(l) - target; };
  double lo = 0.0, hi = 1.0;
  while (h(hi) < 0.0) hi *= 2.0;
  for (int it = 0; it < 200 && hi - lo > 1e-16; ++it) {
    const double mid = 0.5 * (lo + hi);
    (h(mid) < 0.0 ? lo : hi) = mid;
  }
  return 0.5 * (lo + hi);
}

// Similarity constant of melting into a solid subcooled to T_c whose
// conductivity is kappa times the liquid's (same rho c, so its diffusivity
// is kappa alpha): the root of
//   lam sqrt(pi) = Ste_l exp(-lam^2)/erf(lam)
//                  - sqrt(kappa) Ste_s exp(-lam^2/kappa)/erfc(lam/sqrt(kappa))
// with Ste_s = Ste (t_m - t_c)/(t_h - t_m), by bisection.  Ste_s = 0 gives
// neumann_constant.
double two_phase_constant(double ste_l, double ste_s, double kappa) {
  const double rk = std::sqrt(kappa);
  auto h = [&](double l) {
    return l * std::sqrt(M_PI) - ste_l * std::exp(-l * l) / std::erf(l) +
           rk * ste_s * std::exp(-l * l / kappa) / std::erfc(l / rk);
  };
  double lo = 1e-12, hi = 1.0;
  while (h(hi) < 0.0) hi *= 2.0;
  for (int it = 0; it < 200 && hi - lo > 1e-16; ++it) {
    const double mid = 0.5 * (lo + hi);
    (h(mid) < 0.0 ? lo : hi) = mid;
  }
  return 0.5 * (lo + hi);
}

}  // namespace

// The recomputed states of one segment (0..K) and their phase bookkeeping
// (launch_adj_partition), for up to pcap states: counts, their 5x5 extremes
// (pcap n^2 each), the largest count of each state, and the device array of
// their fronts.  State 0 is the segment's checkpoint: its populations are
// read in place (sf[0] and sg[0] stay null), its front is copied into ss[0]
// so that the device array of fronts does not change from segment to
// segment.
struct SegSet {
  std::vector<void*> sf, sg;
  std::vector<double*> ss;
  int *cnt2 = nullptr, *cmin2 = nullptr, *cmax2 = nullptr, *rowb = nullptr;
  const double** sptr = nullptr;
  std::vector<const double*> sptr_host;  // source of the last upload of sptr
  int pcap = 0;
};

// Checkpoints of a forward run and the buffers of its reverse sweep.
struct AdjData {
  bool ready = false;
  int64_t start = 0, nsteps = 0, end = 0;
  int K = 0, nck = 0;
  std::vector<void*> ckf, ckg;
  std::vector<double*> cks;
  // one segment set, or two: then the recompute of the next segment (on the
  // side stream) overlaps the reverse sweep of the current one
  SegSet set[2];
  hipStream_t side = nullptr;
  hipEvent_t ev_start = nullptr, ev_rc[2] = {nullptr, nullptr}, ev_rv[2] = {nullptr, nullptr};
  // recompute scratch (only the recompute uses these)
  int *cnt = nullptr, *melted = nullptr, *frozen = nullptr, *flag = nullptr;
  uint32_t* cext = nullptr;  // 3x3 count extremes of the recompute (16-bit storage)
  double* heat_rc = nullptr;  // interface heat of a recomputed step (front scheme 1)
  double* wq = nullptr;  // per-column weight of the interface heat (front scheme 1)
  void *lf[2] = {nullptr, nullptr}, *lg[2] = {nullptr, nullptr};  // per-cell adjoints
  void *lfh = nullptr, *lgh = nullptr;
  // above the shared-launch size: the second buffer of the pulled adjoints,
  // alternating with lgh step by step (paired bulk-solid rows)
  void* lgh_b = nullptr;
  double *ls[2] = {nullptr, nullptr};
  double *out5 = nullptr, *own = nullptr, *lth = nullptr;
};

// A captured chunk of steps (lbm_set_graph): `steps` (even) steps that start
// and end at buffer parity (cur, scur).
struct StepGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int cur = -1, scur = -1;
  int pair_rows = -1;  // the row order the graph's kernels were captured with
};

struct lbm_ctx {
  lbm_params p{};
  lbm_lattice lat{};
  lbmk::KParams kp{};
  int kind = 0;
  size_t esz = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;
  void* f[2] = {nullptr, nullptr};
  void* g[2] = {nullptr, nullptr};
  int cur = 0;
  double* s[2] = {nullptr, nullptr};
  int scur = 0;
  int* cnt = nullptr;
  uint32_t* cext = nullptr;  // min | max << 16 of the counts over 3x3 columns (16-bit storage)
  int* rowmax = nullptr;     // largest such max per row of columns (16-bit storage)
  int* melted = nullptr;
  int* frozen = nullptr;
  int* flag = nullptr;
  double* th = nullptr;
  double* red = nullptr;
  double* dpart = nullptr;   // partial sums of the diagnostics reductions
  double* scratch = nullptr; // this device's address of the no-allocation scratch
  double* seedT = nullptr;
  double* fields = nullptr;  // 5 * n^3 FP64 scratch for the field output
  double* wall = nullptr;    // n^2 FP64 scratch of per-column wall diagnostics
  double* heat = nullptr;    // n^2 FP64 front heat of a step (front_scheme 1)
  int64_t step = 0;
  AdjData adj;
  // schedule (liquid counts and node indices per step) of the last recorded run
  int* sched = nullptr;
  size_t sched_cap = 0;   // ints
  int64_t sched_steps = 0;
  int64_t rec_start = -1;  // first step being recorded, -1 when not recording
  int* replay = nullptr;   // device copy of a schedule being replayed
  size_t replay_cap = 0;
  bool unstable = false;  // a query saw the device flag; steps refused until load
  bool timing = false;
  // the liquid fraction last known on the host (the seed front, then every
  // query): picks the row order of the 16-bit step kernel at two workgroups
  // per row (KParams::pair_rows), which changes no result
  double fl_hint = 0.0;
  std::vector<hipEvent_t> ev;  // pairs (start, stop) of timed kernels
  size_t ev_used = 0;
  // graph replays of the step loop (lbm_set_graph)
  int graph_steps = 0;           // steps per captured chunk, 0: launch every kernel
  StepGraph sgraph;
  hipStream_t cap = nullptr;     // capture stream (never runs work)
  uint32_t* step_dev = nullptr;  // the step counter that graph replays advance
};

namespace {

// bytes of one distribution with Q directions in the row-interleaved layout
size_t dist_bytes(const lbm_ctx* c, int Q) {
  return (size_t)Q * c->kp.pitch * ((size_t)c->p.n * c->p.n) * c->esz;
}

void free_all(std::vector<void*>& v) {
  for (void* p : v)
    if (p) (void)hipFree(p);
  v.clear();
}
void free_all(std::vector<double*>& v) {
  for (double* p : v)
    if (p) (void)hipFree(p);
  v.clear();
}

void release_states(SegSet& s) {
  free_all(s.sf);
  free_all(s.sg);
  free_all(s.ss);
}

void release_set(SegSet& s) {
  release_states(s);
  void* ptrs[] = {s.cnt2, s.cmin2, s.cmax2, s.rowb, s.sptr};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  s = SegSet();
}

void release_adjoint(AdjData& a) {
  if (a.side) (void)hipStreamSynchronize(a.side);  // its recompute may still use the buffers
  free_all(a.ckf);
  free_all(a.ckg);
  free_all(a.cks);
  release_set(a.set[0]);
  release_set(a.set[1]);
  void* ptrs[] = {a.cnt,   a.cext,  a.heat_rc, a.melted, a.frozen, a.flag, a.lf[0], a.lf[1],
                  a.lg[0], a.lg[1], a.ls[0],   a.ls[1],  a.lfh,    a.lgh,  a.out5,  a.own,
                  a.lth,   a.wq,    a.lgh_b};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  hipEvent_t evs[] = {a.ev_start, a.ev_rc[0], a.ev_rc[1], a.ev_rv[0], a.ev_rv[1]};
  for (hipEvent_t e : evs)
    if (e) (void)hipEventDestroy(e);
  if (a.side) (void)hipStreamDestroy(a.side);
  a = AdjData();
}

void release_graph(StepGraph& g) {
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (g.graph) (void)hipGraphDestroy(g.graph);
  g = StepGraph();
}

void release(lbm_ctx* c) {
  release_graph(c->sgraph);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  if (c->step_dev) (void)hipFree(c->step_dev);
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  c->ev.clear();
  release_adjoint(c->adj);
  void* ptrs[] = {c->f[0], c->f[1], c->g[0], c->g[1], c->s[0], c->s[1], c->cnt,  c->cext,
                  c->melted, c->frozen, c->flag, c->th,  c->red,  c->seedT, c->fields,
                  c->sched, c->replay, c->wall, c->heat, c->dpart, c->rowmax};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
}

int validate(const lbm_params* p) {
  if (!p) return fail(LBM_EINVAL, "params is NULL");
  if (p->n < 4 || p->n > 1024) return fail(LBM_EINVAL, "n = %d outside [4, 1024]", p->n);
  if (p->precision < LBM_F64 || p->precision > LBM_BF16S)
    return fail(LBM_EINVAL, "precision = %d is not an lbm_precision", p->precision);
  // two buffers of each distribution must leave room for the rest on one
  // 288 GB device
  const double bytes = 2.0 * ((p->flow ? 19 : 0) + 7) *
                       (double)lbmk::row_pitch(p->n, p->precision) * (double)p->n * p->n *
                       (double)lbmk::store_bytes(p->precision);
  if (bytes > 256.0 * 1073741824.0)
    return fail(LBM_EINVAL, "n = %d too large for this storage precision (%.0f GiB of "
                "distributions)", p->n, bytes / 1073741824.0);
  if (p->heating != LBM_HEAT_Y0 && p->heating != LBM_HEAT_Z0)
    return fail(LBM_EINVAL, "heating = %d is not an lbm_heating", p->heating);
  if (p->flow != 0 && p->flow != 1) return fail(LBM_EINVAL, "flow must be 0 or 1");
  if (p->seed_profile < 0 || p->seed_profile > 2)
    return fail(LBM_EINVAL, "seed_profile must be 0, 1 or 2");
  if (!(p->t_c <= p->t_m && p->t_m < p->t_h))
    return fail(LBM_EINVAL, "temperatures must satisfy t_c <= t_m < t_h");
  if (!(p->ste >= 0.0) || !std::isfinite(p->ste)) return fail(LBM_EINVAL, "ste must be >= 0");
  if (p->seed_profile >= 1 && !(p->ste > 0.0))
    return fail(LBM_EINVAL, "the Neumann seed profile needs ste > 0");
  if (!(p->ma > 0.0 && p->ma < 0.3)) return fail(LBM_EINVAL, "ma must lie in (0, 0.3)");
  if (!(p->s0 >= 0.0 && p->s0 <= p->n)) return fail(LBM_EINVAL, "s0 must lie in [0, n]");
  if (!(p->ks_kl >= 0.0) || !std::isfinite(p->ks_kl))
    return fail(LBM_EINVAL, "ks_kl must be >= 0 (0 or 1: equal phase properties)");
  if (p->front_scheme != 0 && p->front_scheme != 1)
    return fail(LBM_EINVAL, "front_scheme must be 0 (Eq. (6) gradients) or 1 (interface heat)");
  if (p->f_wall != 0 && p->f_wall != 1)
    return fail(LBM_EINVAL, "f_wall must be 0 (halfway bounce-back) or 1 (interpolated)");
  if (p->flow) {
    if (!(p->ra > 0.0) || !(p->pr > 0.0) || !std::isfinite(p->ra) || !std::isfinite(p->pr))
      return fail(LBM_EINVAL, "ra and pr must be positive");
  } else if (!(p->alpha > 0.0) || !std::isfinite(p->alpha)) {
    return fail(LBM_EINVAL, "alpha must be positive when flow == 0");
  }
  return LBM_OK;
}

// Lattice units: U0 = Ma c_s; nu = U0 H sqrt(Pr/Ra); alpha = U0 H / sqrt(Ra Pr);
// g beta = U0^2 / (H (t_h - t_m)), so that Ra = g beta dT H^3 / (nu alpha),
// and the Fourier number alpha t / H^2 equals Eq. (7).
int derive(const lbm_params* p, lbm_lattice* L) {
  const double n = p->n;
  L->u0 = p->ma / std::sqrt(3.0);
  if (p->flow) {
    L->nu = L->u0 * n * std::sqrt(p->pr / p->ra);
    L->alpha = L->u0 * n / std::sqrt(p->ra * p->pr);
    L->gbeta = L->u0 * L->u0 / (n * (p->t_h - p->t_m));
    L->s_nu = 1.0 / (3.0 * L->nu + 0.5);
    if (!(3.0 * L->nu + 0.5 > 0.5 + 1e-3))
      return fail(LBM_EINVAL, "viscous relaxation time %.6g too close to 1/2 (raise n or ma, "
                  "or lower ra)", 3.0 * L->nu + 0.5);
  } else {
    L->nu = 0.0;
    L->alpha = p->alpha;
    L->gbeta = 0.0;
    L->s_nu = 1.0;
  }
  L->t0 = 0.5 * (p->t_h + p->t_c);
  L->q_j = 1.0 / (4.0 * L->alpha + 0.5);
  L->q_e = 1.0 / (0.5 + 1.0 / (16.0 * L->alpha));
  return LBM_OK;
}

int refresh_masks(lbm_ctx* c) {
  HIP_TRY(lbmk::launch_counts(c->kp, c->s[c->scur], c->cnt, c->stream));
  HIP_TRY(lbmk::launch_neighbourhood(c->kp, c->cnt, c->cext, c->rowmax, c->stream));
  return LBM_OK;
}

int check_ctx(const lbm_ctx* c) {
  if (!c) return fail(LBM_EINVAL, "context is NULL");
  return LBM_OK;
}

int check_unstable(lbm_ctx* c) {
  int flag = 0;
  HIP_TRY(hipMemcpyAsync(&flag, c->flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (flag) {
    c->unstable = true;
    return fail(LBM_EUNSTABLE, "a non-finite value appeared (step <= %lld)", (long long)c->step);
  }
  return LBM_OK;
}

int ensure_fields(lbm_ctx* c) {
  if (!c->fields) {
    const size_t nc = c->kp.ncell;
    if (hipMalloc((void**)&c->fields, 5 * nc * sizeof(double)) != hipSuccess) {
      c->fields = nullptr;
      return fail(LBM_ENOMEM, "cannot allocate %zu bytes for field output",
                  5 * nc * sizeof(double));
    }
  }
  return LBM_OK;
}

template <typename T>
int dalloc(T** p, size_t count) {
  if (hipMalloc((void**)p, count * sizeof(T)) != hipSuccess) {
    *p = nullptr;
    return fail(LBM_ENOMEM, "hipMalloc of %zu bytes failed", count * sizeof(T));
  }
  return LBM_OK;
}

int dalloc_bytes(void** p, size_t bytes) {
  if (hipMalloc(p, bytes) != hipSuccess) {
    *p = nullptr;
    return fail(LBM_ENOMEM, "hipMalloc of %zu bytes failed", bytes);
  }
  return LBM_OK;
}

// Scratch of lbm_diagnostics_noalloc: the partial sums of its two-pass
// reduction, in a file-scope device array (one copy per GPU, held until the
// process ends), so that the call allocates nothing.  In host code the name
// `scratch` is only a stand-in for the symbol: its address on each device
// comes from hipGetSymbolAddress, taken once per device at lbm_init with that
// device current, and only that address is handed to kernels.
constexpr size_t kScratchDoubles = 5 * (size_t)lbmk::kDiagBlocks + 5;
static __device__ __align__(256) double scratch[kScratchDoubles];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// The scratch address of `device` (the current device), looked up once.
int scratch_address(int device, double** out) {
  if (device < 0 || device >= kMaxDevices)
    return fail(LBM_EDEVICE, "device %d beyond the %d the library tracks", device, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(LBM_EDEVICE, "hipGetSymbolAddress of the scratch array failed: %s",
                  hipGetErrorString(e));
    g_scratch_ptr[device] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[device];
  return LBM_OK;
}

struct StateHeader {
  char magic[8];
  int32_t n, precision, flow, heating;
  int64_t step;
  uint64_t ncell;
};

}  // namespace

extern "C" {

const char* lbm_last_error(void) { return g_err; }

int lbm_init(const lbm_params* params, void* hip_stream, lbm_ctx** out) {
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate(params);
  if (rc) return rc;
  lbm_lattice L{};
  rc = derive(params, &L);
  if (rc) return rc;

  lbm_ctx* c = new (std::nothrow) lbm_ctx();
  if (!c) return fail(LBM_ENOMEM, "host allocation failed");
  c->p = *params;
  c->lat = L;
  c->kind = params->precision;
  c->esz = lbmk::store_bytes(c->kind);
  const int n = params->n;
  const size_t nn = (size_t)n * n, nc = nn * n;
  lbmk::KParams& k = c->kp;
  k.n = n;
  k.ncell = (uint32_t)nc;
  k.pitch = lbmk::row_pitch(n, c->kind);
  k.inv_nm2 = lbmk::recip32((uint32_t)(n - 2));
  k.inv_n = lbmk::recip32((uint32_t)n);
  k.melt_z = params->heating == LBM_HEAT_Z0;
  k.flow = params->flow;
  k.t0 = L.t0;
  k.tref = 0.5 * (params->t_h + params->t_m);
  k.t_m = params->t_m;
  k.t_c = params->t_c;
  k.gbeta = L.gbeta;
  k.s_nu = L.s_nu;
  k.q_j = L.q_j;
  k.q_e = L.q_e;
  // solid: conductivity kappa k_l with the same rho c, diffusivity kappa alpha
  k.kappa = params->ks_kl > 0.0 ? params->ks_kl : 1.0;
  k.f_wall = params->f_wall;
  {
    const double alpha_s = k.kappa * L.alpha;
    k.q_js = 1.0 / (4.0 * alpha_s + 0.5);
    k.q_es = 1.0 / (0.5 + 1.0 / (16.0 * alpha_s));
  }
  k.alpha = L.alpha;
  k.ste = params->ste;
  k.dT = params->t_h - params->t_m;
  lbmk::set_f32_params(k);

  auto bail = [&](int code) {
    release(c);
    delete c;
    return code;
  };
  if (hipGetDevice(&c->device) != hipSuccess) return bail(fail(LBM_EDEVICE, "no HIP device"));
  if ((rc = scratch_address(c->device, &c->scratch))) return bail(rc);
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
  } else {
    // blocking stream: ordered with work on the legacy default stream
    if (hipStreamCreate(&c->stream) != hipSuccess)
      return bail(fail(LBM_EDEVICE, "hipStreamCreate failed"));
    c->own_stream = true;
  }
  const size_t fbytes = dist_bytes(c, 19), gbytes = dist_bytes(c, 7);
  if (params->flow) {
    for (int b = 0; b < 2; ++b)
      if (hipMalloc(&c->f[b], fbytes) != hipSuccess) {
        c->f[b] = nullptr;
        return bail(fail(LBM_ENOMEM, "cannot allocate f (%zu bytes)", fbytes));
      }
  }
  for (int b = 0; b < 2; ++b)
    if (hipMalloc(&c->g[b], gbytes) != hipSuccess) {
      c->g[b] = nullptr;
      return bail(fail(LBM_ENOMEM, "cannot allocate g (%zu bytes)", gbytes));
    }
  if ((rc = dalloc(&c->s[0], nn)) || (rc = dalloc(&c->s[1], nn)) || (rc = dalloc(&c->cnt, nn)) ||
      (rc = dalloc(&c->cext, nn)) ||
      (rc = dalloc(&c->rowmax, (size_t)n)) ||
      (rc = dalloc(&c->melted, nn)) || (rc = dalloc(&c->frozen, nn)) ||
      (rc = dalloc(&c->flag, 1)) || (rc = dalloc(&c->th, nn)) || (rc = dalloc(&c->red, 8)) ||
      (rc = dalloc(&c->seedT, (size_t)n)) ||
      (rc = dalloc(&c->dpart, lbmk::diag_scratch_doubles(n))) ||
      (params->front_scheme == 1 && (rc = dalloc(&c->heat, nn))))
    return bail(rc);

  // initial front, hot wall, seed temperature profile along the melt axis
  std::vector<double> hs(nn, params->s0), ht(nn, params->t_h), seed(n, params->t_c);
  double lam = 0.0, t_init = 0.0;
  if (params->seed_profile >= 1) {
    lam = params->seed_profile == 1
              ? neumann_constant(params->ste)
              : two_phase_constant(params->ste,
                                   params->ste * (params->t_m - params->t_c) /
                                       (params->t_h - params->t_m),
                                   k.kappa);
    t_init = (params->s0 / (2.0 * lam)) * (params->s0 / (2.0 * lam)) / L.alpha;
  }
  for (int a = 0; a < n; ++a) {
    const double y = a + 0.5;
    const double eta = params->seed_profile >= 1 ? y / (2.0 * std::sqrt(L.alpha * t_init)) : 0.0;
    if (!(y < params->s0)) {  // solid: t_c, or the subcooled two-phase profile
      if (params->seed_profile == 2)  // solid diffusivity kappa alpha
        seed[a] = params->t_c + (params->t_m - params->t_c) *
                                    std::erfc(eta / std::sqrt(k.kappa)) /
                                    std::erfc(lam / std::sqrt(k.kappa));
      continue;
    }
    if (params->seed_profile >= 1)
      seed[a] = params->t_h - (params->t_h - params->t_m) * std::erf(eta) / std::erf(lam);
    else
      seed[a] = params->t_h + (params->t_m - params->t_h) * y / params->s0;
  }
  auto dev = [&](int code) { return bail(code); };
  if (hipMemcpyAsync(c->s[0], hs.data(), nn * sizeof(double), hipMemcpyHostToDevice, c->stream) ||
      hipMemcpyAsync(c->th, ht.data(), nn * sizeof(double), hipMemcpyHostToDevice, c->stream) ||
      hipMemcpyAsync(c->seedT, seed.data(), n * sizeof(double), hipMemcpyHostToDevice,
                     c->stream) ||
      hipMemsetAsync(c->melted, 0, nn * sizeof(int), c->stream) ||
      hipMemsetAsync(c->frozen, 0, nn * sizeof(int), c->stream) ||
      hipMemsetAsync(c->flag, 0, sizeof(int), c->stream))
    return dev(fail(LBM_EDEVICE, "initial upload failed"));
  if ((rc = refresh_masks(c))) return bail(rc);
  if (lbmk::launch_init(c->kind, k, c->seedT, c->f[0], c->g[0], c->stream) != hipSuccess)
    return bail(fail(LBM_EDEVICE, "init kernel launch failed"));
  if (hipStreamSynchronize(c->stream) != hipSuccess)
    return bail(fail(LBM_EDEVICE, "initialisation failed on the device"));
  c->fl_hint = std::min(std::max(params->s0, 0.0), (double)n) / n;
  *out = c;
  return LBM_OK;
}

void lbm_destroy(lbm_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  release(c);
  delete c;
}

namespace {

// The kernels of one step from buffer parity (cur, scur) on stream st: the
// same launches whether they run at once or are captured into a graph.
// rec: schedule slot to record (or null).  step_ctr: the device step counter
// to advance (graph replays, else null).  ev0/ev1 (or null): events the
// stream-collide kernel's dispatch records at its start and end.
hipError_t enqueue_step(lbm_ctx* c, const lbmk::KParams& k, int cur, int scur, int* rec,
                        uint32_t* step_ctr, hipEvent_t ev0, hipEvent_t ev1, hipStream_t st) {
  const int nx = cur ^ 1, sx = scur ^ 1;
  hipError_t e;
  if ((e = lbmk::launch_stream_collide(c->kind, k, c->f[cur], c->f[nx], c->g[cur], c->g[nx],
                                       c->cnt, c->cext, c->rowmax, c->s[scur], c->th, c->flag,
                                       st, ev0, ev1)) != hipSuccess)
    return e;
  if (c->heat &&  // conservative front: heat of the streaming from the state g[cur]
      (e = lbmk::launch_front_heat(c->kind, k, c->g[cur], c->s[scur], c->cnt, c->heat, st)) !=
          hipSuccess)
    return e;
  if ((e = lbmk::launch_front(c->kind, k, c->s[scur], c->s[sx], c->cnt, c->g[nx], c->f[nx], c->th,
                              c->melted, c->frozen, c->flag, nullptr, nullptr, rec, c->heat,
                              step_ctr, st)) != hipSuccess)
    return e;
  if (lbmk::uses_neighbourhood(c->kind) &&
      (e = lbmk::launch_neighbourhood(k, c->cnt, c->cext, c->rowmax, st)) != hipSuccess)
    return e;
  return hipSuccess;
}

// Captures c->graph_steps steps from the current buffer parity.  Nothing
// runs during the capture.  The stream-collide kernels of the graph read the
// step (the seed of the stochastic rounding of FP32 and 16-bit storage) from
// c->step_dev, which each step's front kernel advances, so a replay rounds
// with the same per-step random streams as launches one by one.
int build_step_graph(lbm_ctx* c) {
  release_graph(c->sgraph);
  if (!c->cap) HIP_TRY(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
  lbmk::KParams k = c->kp;
  k.step_dev = c->step_dev;
  HIP_TRY(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  int cur = c->cur, scur = c->scur;
  for (int i = 0; i < c->graph_steps && e == hipSuccess; ++i) {
    e = enqueue_step(c, k, cur, scur, nullptr, c->step_dev, nullptr, nullptr, c->cap);
    cur ^= 1;
    scur ^= 1;
  }
  hipGraph_t g = nullptr;
  const hipError_t ee = hipStreamEndCapture(c->cap, &g);
  if (e != hipSuccess || ee != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return fail(LBM_EDEVICE, "capture of the step graph failed: %s",
                hipGetErrorString(e != hipSuccess ? e : ee));
  }
  hipGraphExec_t x = nullptr;
  const hipError_t ei = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (ei != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail(LBM_EDEVICE, "hipGraphInstantiate failed: %s", hipGetErrorString(ei));
  }
  c->sgraph.graph = g;
  c->sgraph.exec = x;
  c->sgraph.cur = c->cur;
  c->sgraph.scur = c->scur;
  c->sgraph.pair_rows = c->kp.pair_rows;
  return LBM_OK;
}

}  // namespace

int lbm_step(lbm_ctx* c, int64_t nsteps) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (nsteps < 0) return fail(LBM_EINVAL, "nsteps must be >= 0");
  if (c->unstable) return fail(LBM_ESTATE, "state is unstable; restore it with lbm_load_state");
  lbmk::KParams& k = c->kp;
  k.pair_rows = c->fl_hint > 0.5 ? 1 : 0;
  // whole chunks as graph replays (an even number of steps returns the
  // buffers to their parity, so one graph serves every chunk)
  if (c->graph_steps > 0 && !c->timing && c->rec_start < 0 && nsteps >= c->graph_steps) {
    if (!c->sgraph.exec || c->sgraph.cur != c->cur || c->sgraph.scur != c->scur ||
        c->sgraph.pair_rows != k.pair_rows)
      if ((rc = build_step_graph(c))) return rc;
    HIP_TRY(lbmk::launch_set_u32(c->step_dev, (uint32_t)c->step, c->stream));
    const int64_t reps = nsteps / c->graph_steps;
    for (int64_t r = 0; r < reps; ++r) HIP_TRY(hipGraphLaunch(c->sgraph.exec, c->stream));
    c->step += reps * c->graph_steps;
    nsteps -= reps * c->graph_steps;
  }
  for (int64_t i = 0; i < nsteps; ++i) {
    k.step = (uint32_t)c->step;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (c->timing) {
      if (c->ev_used + 2 > c->ev.size()) {
        for (int e = 0; e < 2; ++e) {
          hipEvent_t h;
          HIP_TRY(hipEventCreate(&h));
          c->ev.push_back(h);
        }
      }
      ev0 = c->ev[c->ev_used];
      ev1 = c->ev[c->ev_used + 1];
      c->ev_used += 2;
    }
    int* rec = c->rec_start >= 0
                   ? c->sched + (size_t)(c->step - c->rec_start) * 3 * ((size_t)c->p.n * c->p.n)
                   : nullptr;
    HIP_TRY(enqueue_step(c, k, c->cur, c->scur, rec, nullptr, ev0, ev1, c->stream));
    c->cur ^= 1;
    c->scur ^= 1;
    c->step++;
  }
  return LBM_OK;
}

int lbm_set_graph(lbm_ctx* c, int32_t steps) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (steps < 0 || steps > 4096 || (steps & 1))
    return fail(LBM_EINVAL, "graph chunk of %d steps: need 0 or an even number up to 4096",
                (int)steps);
  if (steps == c->graph_steps) return LBM_OK;
  if (steps && !c->step_dev && hipMalloc((void**)&c->step_dev, sizeof(uint32_t)) != hipSuccess) {
    c->step_dev = nullptr;
    return fail(LBM_ENOMEM, "cannot allocate the step counter");
  }
  HIP_TRY(hipStreamSynchronize(c->stream));  // no replay of the old graph is pending
  release_graph(c->sgraph);
  c->graph_steps = steps;
  return LBM_OK;
}

int lbm_liquid_fraction(lbm_ctx* c, double* fl) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!fl) return fail(LBM_EINVAL, "fl is NULL");
  const int64_t nn = (int64_t)c->p.n * c->p.n;
  HIP_TRY(lbmk::launch_sum(c->s[c->scur], nn, c->red, c->stream));
  double host[1];
  HIP_TRY(hipMemcpyAsync(host, c->red, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  if ((rc = check_unstable(c))) return rc;
  *fl = host[0] / ((double)nn * c->p.n);
  c->fl_hint = *fl;
  return LBM_OK;
}

int lbm_fields(lbm_ctx* c, double* T, double* u, double* rho, double* s) {
  int rc = check_ctx(c);
  if (rc) return rc;
  const size_t nc = c->kp.ncell, nn = (size_t)c->p.n * c->p.n;
  if (T || u || rho) {  // the cell fields are computed only when asked for
    if ((rc = ensure_fields(c))) return rc;
    double* d = c->fields;
    HIP_TRY(lbmk::launch_fields(c->kind, c->kp, c->f[c->cur], c->g[c->cur], c->cnt, d, d + nc,
                                d + 2 * nc, d + 3 * nc, d + 4 * nc, c->stream));
    if (T) HIP_TRY(hipMemcpyAsync(T, d, nc * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    if (u)
      HIP_TRY(hipMemcpyAsync(u, d + nc, 3 * nc * sizeof(double), hipMemcpyDeviceToHost,
                             c->stream));
    if (rho)
      HIP_TRY(hipMemcpyAsync(rho, d + 4 * nc, nc * sizeof(double), hipMemcpyDeviceToHost,
                             c->stream));
  }
  if (s)
    HIP_TRY(hipMemcpyAsync(s, c->s[c->scur], nn * sizeof(double), hipMemcpyDeviceToHost,
                           c->stream));
  return check_unstable(c);
}

int lbm_wall_nusselt(lbm_ctx* c, double* nu) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!nu) return fail(LBM_EINVAL, "nu is NULL");
  const size_t nn = (size_t)c->p.n * c->p.n;
  if (!c->wall && (rc = dalloc(&c->wall, nn))) return rc;
  HIP_TRY(lbmk::launch_wall_nusselt(c->kind, c->kp, c->g[c->cur], c->s[c->scur], c->th, c->wall,
                                    c->stream));
  HIP_TRY(hipMemcpyAsync(nu, c->wall, nn * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  return check_unstable(c);
}

int lbm_get_lattice(const lbm_ctx* c, lbm_lattice* out) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  *out = c->lat;
  return LBM_OK;
}

int lbm_get_step(const lbm_ctx* c, int64_t* step) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!step) return fail(LBM_EINVAL, "step is NULL");
  *step = c->step;
  return LBM_OK;
}

int lbm_set_hot_wall(lbm_ctx* c, const double* th, int on_device) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!th) return fail(LBM_EINVAL, "th is NULL");
  const size_t nn = (size_t)c->p.n * c->p.n;
  c->adj.ready = false;  // a recorded run no longer matches the wall it ran with
  HIP_TRY(hipMemcpyAsync(c->th, th, nn * sizeof(double),
                         on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream));
  if (!on_device) HIP_TRY(hipStreamSynchronize(c->stream));  // host buffer may be reused
  return LBM_OK;
}

int lbm_set_populations(lbm_ctx* c, const double* f, const double* g, const double* s) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (c->p.flow && !f) return fail(LBM_EINVAL, "f is required when flow == 1");
  if (!g || !s) return fail(LBM_EINVAL, "g and s are required");
  const size_t nc = c->kp.ncell, nn = (size_t)c->p.n * c->p.n;
  c->adj.ready = false;  // the state no longer ends a recorded run
  double* tmp = nullptr;
  if ((rc = dalloc(&tmp, (c->p.flow ? 19 : 7) * nc))) return rc;
  auto done = [&](int code) {
    (void)hipStreamSynchronize(c->stream);
    (void)hipFree(tmp);
    return code;
  };
  if (c->p.flow) {
    if (hipMemcpyAsync(tmp, f, 19 * nc * sizeof(double), hipMemcpyHostToDevice, c->stream) ||
        lbmk::launch_to_storage(c->kind, c->kp, 19, tmp, c->f[c->cur], c->stream))
      return done(fail(LBM_EDEVICE, "upload of f failed"));
    if (hipStreamSynchronize(c->stream)) return done(fail(LBM_EDEVICE, "upload of f failed"));
  }
  if (hipMemcpyAsync(tmp, g, 7 * nc * sizeof(double), hipMemcpyHostToDevice, c->stream) ||
      lbmk::launch_to_storage(c->kind, c->kp, 7, tmp, c->g[c->cur], c->stream) ||
      hipMemcpyAsync(c->s[c->scur], s, nn * sizeof(double), hipMemcpyHostToDevice, c->stream))
    return done(fail(LBM_EDEVICE, "upload of g or s failed"));
  if ((rc = refresh_masks(c))) return done(rc);
  double sum = 0.0;
  for (size_t i = 0; i < nn; ++i) sum += std::min(std::max(s[i], 0.0), (double)c->p.n);
  c->fl_hint = sum / ((double)nn * c->p.n);
  return done(LBM_OK);
}

int lbm_get_populations(lbm_ctx* c, double* f, double* g, double* s) {
  int rc = check_ctx(c);
  if (rc) return rc;
  const size_t nc = c->kp.ncell, nn = (size_t)c->p.n * c->p.n;
  double* tmp = nullptr;
  if ((f && c->p.flow) || g)
    if ((rc = dalloc(&tmp, ((f && c->p.flow) ? 19 : 7) * nc))) return rc;
  auto done = [&](int code) {
    (void)hipStreamSynchronize(c->stream);
    if (tmp) (void)hipFree(tmp);
    return code;
  };
  if (f && c->p.flow) {
    if (lbmk::launch_from_storage(c->kind, c->kp, 19, c->f[c->cur], tmp, c->stream) ||
        hipMemcpyAsync(f, tmp, 19 * nc * sizeof(double), hipMemcpyDeviceToHost, c->stream) ||
        hipStreamSynchronize(c->stream))
      return done(fail(LBM_EDEVICE, "download of f failed"));
  }
  if (g) {
    if (lbmk::launch_from_storage(c->kind, c->kp, 7, c->g[c->cur], tmp, c->stream) ||
        hipMemcpyAsync(g, tmp, 7 * nc * sizeof(double), hipMemcpyDeviceToHost, c->stream))
      return done(fail(LBM_EDEVICE, "download of g failed"));
  }
  if (s && hipMemcpyAsync(s, c->s[c->scur], nn * sizeof(double), hipMemcpyDeviceToHost, c->stream))
    return done(fail(LBM_EDEVICE, "download of s failed"));
  return done(LBM_OK);
}

int lbm_diagnostics(lbm_ctx* c, double out[5]) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  HIP_TRY(lbmk::launch_diag_sums(c->kind, c->kp, c->f[c->cur], c->g[c->cur], c->cnt,
                                 c->s[c->scur], c->melted, c->frozen, c->dpart, c->stream));
  HIP_TRY(hipMemcpyAsync(out, c->dpart + 5 * (size_t)lbmk::diag_blocks(c->p.n),
                         5 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->fl_hint = out[2] / ((double)c->p.n * c->p.n * c->p.n);  // the front sum over n^3
  return check_unstable(c);
}

int lbm_diagnostics_noalloc(lbm_ctx* c, double* out, int on_device) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  const size_t need = lbmk::diag_scratch_doubles(c->p.n);
  if (need > kScratchDoubles)
    return fail(LBM_EINVAL, "n = %d needs %zu scratch values, the array holds %zu", c->p.n, need,
                kScratchDoubles);
  HIP_TRY(lbmk::launch_diag_sums(c->kind, c->kp, c->f[c->cur], c->g[c->cur], c->cnt,
                                 c->s[c->scur], c->melted, c->frozen, c->scratch, c->stream));
  const double* res = c->scratch + 5 * (size_t)lbmk::diag_blocks(c->p.n);
  if (on_device) {
    HIP_TRY(hipMemcpyAsync(out, res, 5 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    return LBM_OK;
  }
  HIP_TRY(hipMemcpyAsync(out, res, 5 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return check_unstable(c);
}

int lbm_save_state(lbm_ctx* c, void* host_buf, size_t* bytes) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!bytes) return fail(LBM_EINVAL, "bytes is NULL");
  const size_t nc = c->kp.ncell, nn = (size_t)c->p.n * c->p.n;
  const size_t fb = c->p.flow ? dist_bytes(c, 19) : 0, gb = dist_bytes(c, 7);
  const size_t need = sizeof(StateHeader) + fb + gb + nn * (sizeof(double) + 2 * sizeof(int));
  if (!host_buf) {
    *bytes = need;
    return LBM_OK;
  }
  if (*bytes < need) return fail(LBM_EINVAL, "buffer holds %zu bytes, %zu needed", *bytes, need);
  StateHeader h{};
  memcpy(h.magic, "LBMMELT2", 8);
  h.n = c->p.n;
  h.precision = c->p.precision;
  h.flow = c->p.flow;
  h.heating = c->p.heating;
  h.step = c->step;
  h.ncell = nc;
  char* b = static_cast<char*>(host_buf);
  memcpy(b, &h, sizeof(h));
  b += sizeof(h);
  // distributions as stored (row-interleaved layout, storage precision)
  if (fb) HIP_TRY(hipMemcpyAsync(b, c->f[c->cur], fb, hipMemcpyDeviceToHost, c->stream));
  b += fb;
  HIP_TRY(hipMemcpyAsync(b, c->g[c->cur], gb, hipMemcpyDeviceToHost, c->stream));
  b += gb;
  HIP_TRY(hipMemcpyAsync(b, c->s[c->scur], nn * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  b += nn * sizeof(double);
  HIP_TRY(hipMemcpyAsync(b, c->melted, nn * sizeof(int), hipMemcpyDeviceToHost, c->stream));
  b += nn * sizeof(int);
  HIP_TRY(hipMemcpyAsync(b, c->frozen, nn * sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  *bytes = need;
  return LBM_OK;
}

int lbm_load_state(lbm_ctx* c, const void* host_buf, size_t bytes) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!host_buf) return fail(LBM_EINVAL, "host_buf is NULL");
  const size_t nc = c->kp.ncell, nn = (size_t)c->p.n * c->p.n;
  const size_t fb = c->p.flow ? dist_bytes(c, 19) : 0, gb = dist_bytes(c, 7);
  const size_t need = sizeof(StateHeader) + fb + gb + nn * (sizeof(double) + 2 * sizeof(int));
  if (bytes < need) return fail(LBM_EINVAL, "state blob has %zu bytes, %zu needed", bytes, need);
  StateHeader h;
  memcpy(&h, host_buf, sizeof(h));
  if (memcmp(h.magic, "LBMMELT2", 8) != 0) return fail(LBM_EINVAL, "not a state blob");
  if (h.n != c->p.n || h.precision != c->p.precision || h.flow != c->p.flow ||
      h.heating != c->p.heating || h.ncell != nc)
    return fail(LBM_EINVAL, "state blob was made by an incompatible context");
  c->adj.ready = false;  // the state no longer ends a recorded run
  const char* b = static_cast<const char*>(host_buf) + sizeof(h);
  if (fb) HIP_TRY(hipMemcpyAsync(c->f[c->cur], b, fb, hipMemcpyHostToDevice, c->stream));
  b += fb;
  HIP_TRY(hipMemcpyAsync(c->g[c->cur], b, gb, hipMemcpyHostToDevice, c->stream));
  b += gb;
  HIP_TRY(hipMemcpyAsync(c->s[c->scur], b, nn * sizeof(double), hipMemcpyHostToDevice, c->stream));
  {
    double sum = 0.0, v;
    for (size_t i = 0; i < nn; ++i) {
      memcpy(&v, b + i * sizeof(double), sizeof(double));
      sum += std::min(std::max(v, 0.0), (double)c->p.n);
    }
    c->fl_hint = sum / ((double)nn * c->p.n);
  }
  b += nn * sizeof(double);
  HIP_TRY(hipMemcpyAsync(c->melted, b, nn * sizeof(int), hipMemcpyHostToDevice, c->stream));
  b += nn * sizeof(int);
  HIP_TRY(hipMemcpyAsync(c->frozen, b, nn * sizeof(int), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemsetAsync(c->flag, 0, sizeof(int), c->stream));
  if ((rc = refresh_masks(c))) return rc;
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->step = h.step;
  c->unstable = false;
  return LBM_OK;
}

int lbm_forward_ckpt(lbm_ctx* c, int64_t nsteps, int32_t every_k, double* fl) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (nsteps < 1 || every_k < 1) return fail(LBM_EINVAL, "need nsteps >= 1 and every_k >= 1");
  if (c->unstable) return fail(LBM_ESTATE, "state is unstable; restore it with lbm_load_state");
  AdjData& a = c->adj;
  const size_t nn = (size_t)c->p.n * c->p.n;
  const size_t fb = c->p.flow ? dist_bytes(c, 19) : 0, gb = dist_bytes(c, 7);
  const int nck = (int)((nsteps + every_k - 1) / every_k);
  a.ready = false;
  // a reverse sweep that failed part way may have left recompute work on the
  // side stream; it uses the buffers resized below
  if (a.side) HIP_TRY(hipStreamSynchronize(a.side));
  if (a.K != every_k) {  // the segment buffers are sized by every_k
    release_states(a.set[0]);
    release_states(a.set[1]);
  }
  while ((int)a.ckg.size() > nck) {
    if (a.ckf.back()) (void)hipFree(a.ckf.back());
    (void)hipFree(a.ckg.back());
    (void)hipFree(a.cks.back());
    a.ckf.pop_back();
    a.ckg.pop_back();
    a.cks.pop_back();
  }
  while ((int)a.ckg.size() < nck) {
    void *f = nullptr, *g = nullptr;
    double* sp = nullptr;
    if ((fb && hipMalloc(&f, fb) != hipSuccess) || hipMalloc(&g, gb) != hipSuccess ||
        hipMalloc((void**)&sp, nn * sizeof(double)) != hipSuccess) {
      if (f) (void)hipFree(f);
      if (g) (void)hipFree(g);
      return fail(LBM_ENOMEM, "cannot allocate checkpoint %zu of %d", a.ckg.size(), nck);
    }
    a.ckf.push_back(f);
    a.ckg.push_back(g);
    a.cks.push_back(sp);
  }
  a.K = every_k;
  a.nck = nck;
  a.start = c->step;
  a.nsteps = nsteps;
  // schedule of the run: (nsteps + 1) entries of 3 n^2 ints
  const size_t need = (size_t)(nsteps + 1) * 3 * nn;
  if (need > c->sched_cap) {
    if (c->sched) (void)hipFree(c->sched);
    c->sched = nullptr;
    c->sched_cap = 0;
    if ((rc = dalloc(&c->sched, need))) return rc;
    c->sched_cap = need;
  }
  // The checkpoints take the population buffers themselves instead of copies:
  // at the start of segment i the buffers that hold the current populations
  // become checkpoint i, the segment's first step reads them there and writes
  // the other buffers as usual, and checkpoint i's previous buffers (same
  // sizes) then take their place in the context.  Only the fronts are
  // copied.  A captured step graph addresses the old buffers: it goes.
  if (c->sgraph.exec) {
    HIP_TRY(hipStreamSynchronize(c->stream));  // no replay of it is pending
    release_graph(c->sgraph);
  }
  c->rec_start = c->step;
  c->sched_steps = 0;
  for (int i = 0; i < nck; ++i) {
    const int cur = c->cur;
    void* spare_f = a.ckf[i];
    void* spare_g = a.ckg[i];
    a.ckf[i] = c->f[cur];
    a.ckg[i] = c->g[cur];
    HIP_TRY(hipMemcpyAsync(a.cks[i], c->s[c->scur], nn * sizeof(double), hipMemcpyDeviceToDevice,
                           c->stream));
    const int64_t len = std::min<int64_t>(every_k, nsteps - (int64_t)i * every_k);
    rc = lbm_step(c, 1);
    if (c->cur != cur) {  // the step was enqueued: the state lives on in the other buffers
      c->f[cur] = spare_f;
      c->g[cur] = spare_g;
    } else {  // it was not: the context keeps its buffers, the checkpoint its own
      a.ckf[i] = spare_f;
      a.ckg[i] = spare_g;
    }
    if (!rc && len > 1) rc = lbm_step(c, len - 1);
    if (rc) {
      c->rec_start = -1;
      return rc;
    }
  }
  c->rec_start = -1;
  // final entry: the liquid counts after the last step (its node slots are
  // not used and hold zeros)
  HIP_TRY(hipMemcpyAsync(c->sched + (size_t)nsteps * 3 * nn, c->cnt, nn * sizeof(int),
                         hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(hipMemsetAsync(c->sched + (size_t)nsteps * 3 * nn + nn, 0, 2 * nn * sizeof(int),
                         c->stream));
  c->sched_steps = nsteps;
  a.end = c->step;
  a.ready = true;
  if (fl) return lbm_liquid_fraction(c, fl);
  HIP_TRY(hipStreamSynchronize(c->stream));
  return LBM_OK;
}

namespace {

// Device bytes of one segment set: the populations of K states, the fronts
// of K + 1 and the bookkeeping of K.
size_t segset_bytes(const lbm_ctx* c, int K) {
  const size_t nn = (size_t)c->p.n * c->p.n;
  const size_t fb = c->p.flow ? dist_bytes(c, 19) : 0, gb = dist_bytes(c, 7);
  return (size_t)K * (fb + gb) + (size_t)(K + 1) * nn * sizeof(double) +
         (size_t)K * (3 * nn * sizeof(int) + sizeof(int) + sizeof(double*));
}

// Fill a segment set up to K + 1 states and K bookkeeping entries.
int alloc_segset(lbm_ctx* c, SegSet& S, int K) {
  const size_t nn = (size_t)c->p.n * c->p.n;
  const size_t fb = c->p.flow ? dist_bytes(c, 19) : 0, gb = dist_bytes(c, 7);
  while ((int)S.sg.size() < K + 1) {
    void *f = nullptr, *g = nullptr;
    double* sp = nullptr;
    const bool pops = !S.sg.empty();  // state 0: the checkpoint's populations
    if ((pops && fb && hipMalloc(&f, fb) != hipSuccess) ||
        (pops && hipMalloc(&g, gb) != hipSuccess) ||
        hipMalloc((void**)&sp, nn * sizeof(double)) != hipSuccess) {
      if (f) (void)hipFree(f);
      if (g) (void)hipFree(g);
      return fail(LBM_ENOMEM, "cannot allocate the recompute segment (%d states)", K + 1);
    }
    S.sf.push_back(f);
    S.sg.push_back(g);
    S.ss.push_back(sp);
  }
  if (S.pcap < K) {
    void* ptrs[] = {S.cnt2, S.cmin2, S.cmax2, S.rowb, S.sptr};
    for (void* p : ptrs)
      if (p) (void)hipFree(p);
    S.cnt2 = S.cmin2 = S.cmax2 = S.rowb = nullptr;
    S.sptr = nullptr;
    S.pcap = 0;
    const size_t np = (size_t)K * nn;
    int rc;
    if ((rc = dalloc(&S.cnt2, np)) || (rc = dalloc(&S.cmin2, np)) || (rc = dalloc(&S.cmax2, np)) ||
        (rc = dalloc(&S.rowb, (size_t)K)) ||
        (rc = dalloc_bytes((void**)&S.sptr, (size_t)K * sizeof(double*))))
      return rc;
    S.pcap = K;
  }
  return LBM_OK;
}

// Recompute segment i of the recorded run into set S on stream st, bit for
// bit as the forward run, then its phase bookkeeping (one launch).
int enqueue_recompute(lbm_ctx* c, int i, SegSet& S, hipStream_t st) {
  AdjData& a = c->adj;
  const size_t nn = (size_t)c->p.n * c->p.n;
  const int64_t len = std::min<int64_t>(a.K, a.nsteps - (int64_t)i * a.K);
  lbmk::KParams k = c->kp;
  HIP_TRY(hipMemcpyAsync(S.ss[0], a.cks[i], nn * sizeof(double), hipMemcpyDeviceToDevice, st));
  for (int64_t t = 0; t < len; ++t) {
    const void* fs = t == 0 ? a.ckf[i] : S.sf[t];  // state 0: the checkpoint, in place
    const void* gs = t == 0 ? a.ckg[i] : S.sg[t];
    k.step = (uint32_t)(a.start + (int64_t)i * a.K + t);
    // the front kernel leaves the counts of the next state behind
    if (t == 0) HIP_TRY(lbmk::launch_counts(k, S.ss[t], a.cnt, st));
    if (lbmk::uses_neighbourhood(c->kind))
      HIP_TRY(lbmk::launch_neighbourhood(k, a.cnt, a.cext, nullptr, st));
    // the one-cell path throughout (no row maxima): bit for bit the forward run
    HIP_TRY(lbmk::launch_stream_collide(c->kind, k, fs, S.sf[t + 1], gs, S.sg[t + 1], a.cnt,
                                        a.cext, nullptr, S.ss[t], c->th, a.flag, st));
    if (c->heat)  // conservative front: heat of the streaming from the state gs
      HIP_TRY(lbmk::launch_front_heat(c->kind, k, gs, S.ss[t], a.cnt, a.heat_rc, st));
    HIP_TRY(lbmk::launch_front(c->kind, k, S.ss[t], S.ss[t + 1], a.cnt, S.sg[t + 1],
                               S.sf[t + 1], c->th, a.melted, a.frozen, a.flag, nullptr, nullptr,
                               nullptr, c->heat ? a.heat_rc : nullptr, nullptr, st));
  }
  HIP_TRY(hipMemsetAsync(S.rowb, 0, (size_t)len * sizeof(int), st));
  HIP_TRY(lbmk::launch_adj_partition(k, S.sptr, (int)len, S.cnt2, S.cmin2, S.cmax2, S.rowb, st));
  return LBM_OK;
}

// The reverse steps of segment i from set S on stream st; cur: the slot of
// the per-cell adjoints of the newest state, updated.
int enqueue_reverse(lbm_ctx* c, int i, SegSet& S, int& cur, hipStream_t st) {
  AdjData& a = c->adj;
  const size_t nn = (size_t)c->p.n * c->p.n;
  const int64_t len = std::min<int64_t>(a.K, a.nsteps - (int64_t)i * a.K);
  for (int64_t t = len - 1; t >= 0; --t) {
    const int* cnt_t = S.cnt2 + (size_t)t * nn;
    const void* g0 = t == 0 ? a.ckg[i] : S.sg[t];  // state 0: the checkpoint, in place
    if (c->heat)  // the interface heat of state t, for the reverse of the front update
      HIP_TRY(lbmk::launch_front_heat(c->kind, c->kp, g0, S.ss[t], cnt_t, c->heat, st));
    lbmk::AdjointStep A;
    A.f0 = t == 0 ? a.ckf[i] : S.sf[t];
    A.g0 = g0;
    A.s0 = S.ss[t];
    A.g1 = S.sg[t + 1];
    A.s1 = S.ss[t + 1];
    A.th = c->th;
    A.cnt = cnt_t;
    A.cmin2 = S.cmin2 + (size_t)t * nn;
    A.cmax2 = S.cmax2 + (size_t)t * nn;
    A.rowb = S.rowb + t;
    A.lf1 = a.lf[cur];
    A.lg1 = a.lg[cur];
    A.ls1 = a.ls[cur];
    A.lf0 = a.lf[1 - cur];
    A.lg0 = a.lg[1 - cur];
    A.ls0 = a.ls[1 - cur];
    A.lfh = a.lfh;
    // paired bulk-solid rows: this step's pulled adjoints alternate between
    // two buffers, and the step reversed just before (state t+1, same
    // segment) left those rows' transposed streaming to this one
    const bool pair = c->p.n > lbmk::kAdjFuseMaxN;
    A.lgh = pair && cur ? a.lgh_b : a.lgh;
    A.lgh_prev = pair ? (cur ? a.lgh : a.lgh_b) : nullptr;
    A.rowb_prev = pair && t + 1 < len ? S.rowb + t + 1 : nullptr;
    A.rowb_next = pair && t >= 1 ? S.rowb + t - 1 : nullptr;
    A.out5 = a.out5;
    A.own = a.own;
    A.lth = a.lth;
    A.heat = c->heat;
    A.wq = a.wq;
    HIP_TRY(lbmk::launch_adjoint_step(c->kind, c->kp, A, st));
    cur = 1 - cur;
  }
  return LBM_OK;
}

}  // namespace

int lbm_adjoint(lbm_ctx* c, double dJ_dfl, double* grad_th, int on_device) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!grad_th) return fail(LBM_EINVAL, "grad_th is NULL");
  AdjData& a = c->adj;
  if (!a.ready || c->step != a.end)
    return fail(LBM_ESTATE, "lbm_adjoint needs lbm_forward_ckpt with no step, state change "
                "or hot-wall change since");
  if (a.side) HIP_TRY(hipStreamSynchronize(a.side));  // left over from a failed sweep
  const size_t nn = (size_t)c->p.n * c->p.n, nc = c->kp.ncell;
  const bool flow = c->p.flow != 0;
  // segment sets: a second one when the run has several segments and the set
  // fits with room to spare, so that the recompute of each segment overlaps
  // the reverse sweep of the one after it
  if ((rc = alloc_segset(c, a.set[0], a.K))) return rc;
  if (a.nck > 1) {
    if (a.set[1].sg.empty()) {
      size_t free_b = 0, total_b = 0;
      const size_t need = segset_bytes(c, a.K);
      if (hipMemGetInfo(&free_b, &total_b) == hipSuccess &&
          free_b > need + need / 4 + ((size_t)4 << 30) &&
          alloc_segset(c, a.set[1], a.K) != LBM_OK) {
        release_set(a.set[1]);  // not enough after all: one set
        (void)hipGetLastError();
      }
    } else if ((rc = alloc_segset(c, a.set[1], a.K))) {
      return rc;
    }
  }
  const int nsets = a.nck > 1 && !a.set[1].sg.empty() ? 2 : 1;
  const size_t lb = lbmk::lambda_bytes(c->kind);  // bytes of one per-cell adjoint value
  if (!a.lg[0]) {
    // all or nothing (lg[0] marks the set as allocated): after a failure
    // here the next call allocates afresh
    if ((rc = dalloc(&a.cnt, nn)) || (rc = dalloc(&a.cext, nn)) ||
        (rc = dalloc(&a.melted, nn)) || (rc = dalloc(&a.frozen, nn)) || (rc = dalloc(&a.flag, 1)) ||
        (rc = dalloc_bytes(&a.lg[0], 7 * nc * lb)) || (rc = dalloc_bytes(&a.lg[1], 7 * nc * lb)) ||
        (rc = dalloc(&a.ls[0], nn)) || (rc = dalloc(&a.ls[1], nn)) ||
        (rc = dalloc_bytes(&a.lgh, 7 * nc * lb)) || (rc = dalloc(&a.out5, 5 * nn)) ||
        (rc = dalloc(&a.own, nn)) || (rc = dalloc(&a.lth, nn)) || (rc = dalloc(&a.wq, nn)) ||
        (c->heat && (rc = dalloc(&a.heat_rc, nn))) ||
        (c->p.n > lbmk::kAdjFuseMaxN && (rc = dalloc_bytes(&a.lgh_b, 7 * nc * lb))) ||
        (flow && ((rc = dalloc_bytes(&a.lf[0], 19 * nc * lb)) ||
                  (rc = dalloc_bytes(&a.lf[1], 19 * nc * lb)) ||
                  (rc = dalloc_bytes(&a.lfh, 19 * nc * lb))))) {
      auto drop = [](auto*& p) {
        if (p) (void)hipFree(p);
        p = nullptr;
      };
      drop(a.cnt), drop(a.cext), drop(a.melted), drop(a.frozen), drop(a.flag);
      drop(a.lg[0]), drop(a.lg[1]), drop(a.ls[0]), drop(a.ls[1]), drop(a.lgh), drop(a.out5);
      drop(a.own), drop(a.lth), drop(a.wq), drop(a.heat_rc), drop(a.lgh_b);
      drop(a.lf[0]), drop(a.lf[1]), drop(a.lfh);
      return rc;
    }
  }
  const bool two = nsets == 2;
  if (two && !a.side) {
    HIP_TRY(hipStreamCreateWithFlags(&a.side, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&a.ev_start, hipEventDisableTiming));
    for (int b = 0; b < 2; ++b) {
      HIP_TRY(hipEventCreateWithFlags(&a.ev_rc[b], hipEventDisableTiming));
      HIP_TRY(hipEventCreateWithFlags(&a.ev_rv[b], hipEventDisableTiming));
    }
  }
  // the recompute runs on the side stream (after everything enqueued so far)
  const hipStream_t rs = two ? a.side : c->stream;
  if (two) {
    HIP_TRY(hipEventRecord(a.ev_start, c->stream));
    HIP_TRY(hipStreamWaitEvent(rs, a.ev_start, 0));
  }
  HIP_TRY(hipMemsetAsync(a.melted, 0, nn * sizeof(int), rs));
  HIP_TRY(hipMemsetAsync(a.frozen, 0, nn * sizeof(int), rs));
  HIP_TRY(hipMemsetAsync(a.flag, 0, sizeof(int), rs));
  // the fronts of the segment states 0..K-1, for the batched partition
  for (int b = 0; b < nsets; ++b) {
    SegSet& S = a.set[b];
    S.sptr_host.assign(S.ss.begin(), S.ss.begin() + a.K);
    HIP_TRY(hipMemcpyAsync(S.sptr, S.sptr_host.data(), (size_t)a.K * sizeof(double*),
                           hipMemcpyHostToDevice, rs));
  }
  // adjoint of the final state: J = dJ_dfl * sum(s) / n^3
  int cur = 1;
  HIP_TRY(lbmk::launch_fill(a.ls[cur], nn, dJ_dfl / ((double)nn * c->p.n), c->stream));
  HIP_TRY(lbmk::launch_fill_lambda(c->kind, a.lg[cur], 7 * nc, 0.0, c->stream));
  if (flow) HIP_TRY(lbmk::launch_fill_lambda(c->kind, a.lf[cur], 19 * nc, 0.0, c->stream));
  HIP_TRY(lbmk::launch_fill(a.lth, nn, 0.0, c->stream));
  if (!two) {
    for (int i = a.nck - 1; i >= 0; --i) {
      if ((rc = enqueue_recompute(c, i, a.set[0], c->stream))) return rc;
      if ((rc = enqueue_reverse(c, i, a.set[0], cur, c->stream))) return rc;
    }
  } else {
    // segment i uses set (nck - 1 - i) mod 2.  The side stream recomputes
    // segment i - 1 into the other set as soon as the reverse sweep of
    // segment i + 1 has released it; the main stream reverses segment i once
    // its recompute is done.
    const int last = a.nck - 1;
    if ((rc = enqueue_recompute(c, last, a.set[0], rs))) return rc;
    HIP_TRY(hipEventRecord(a.ev_rc[0], rs));
    for (int i = last; i >= 0; --i) {
      const int b = (last - i) & 1;
      if (i > 0) {
        if (i < last) HIP_TRY(hipStreamWaitEvent(rs, a.ev_rv[1 - b], 0));
        if ((rc = enqueue_recompute(c, i - 1, a.set[1 - b], rs))) return rc;
        HIP_TRY(hipEventRecord(a.ev_rc[1 - b], rs));
      }
      HIP_TRY(hipStreamWaitEvent(c->stream, a.ev_rc[b], 0));
      if ((rc = enqueue_reverse(c, i, a.set[b], cur, c->stream))) return rc;
      HIP_TRY(hipEventRecord(a.ev_rv[b], c->stream));
    }
  }
  HIP_TRY(hipMemcpyAsync(grad_th, a.lth, nn * sizeof(double),
                         on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (two) HIP_TRY(hipStreamSynchronize(rs));
  return LBM_OK;
}

int lbm_get_schedule(lbm_ctx* c, int32_t* out, size_t count) {
  int rc = check_ctx(c);
  if (rc) return rc;
  const size_t nn = (size_t)c->p.n * c->p.n;
  const size_t need = c->sched_steps > 0 ? (size_t)(c->sched_steps + 1) * 3 * nn : 0;
  if (!need) return fail(LBM_ESTATE, "no recorded run (call lbm_forward_ckpt first)");
  if (!out || count < need)
    return fail(LBM_EINVAL, "schedule needs %zu ints (%zu given)", need, out ? count : 0);
  HIP_TRY(hipMemcpyAsync(out, c->sched, need * sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return LBM_OK;
}

int lbm_step_replay(lbm_ctx* c, const int32_t* schedule, int64_t nsteps) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!schedule || nsteps < 1) return fail(LBM_EINVAL, "need a schedule and nsteps >= 1");
  if (c->unstable) return fail(LBM_ESTATE, "state is unstable; restore it with lbm_load_state");
  const int n = c->p.n;
  const size_t nn = (size_t)n * n;
  const size_t need = (size_t)(nsteps + 1) * 3 * nn;
  // the front kernel walks the given node indices: every one must lie in the column
  // (the node slots of the final entry are not used)
  for (size_t e = 0; e <= (size_t)nsteps; ++e) {
    const int32_t* en = schedule + e * 3 * nn;
    const bool nodes = e < (size_t)nsteps;
    for (size_t i = 0; i < nn; ++i) {
      if (en[i] < 0 || en[i] > n ||
          (nodes && (en[nn + i] < -1 || en[nn + i] > n - 1 || en[2 * nn + i] < 0 ||
                     en[2 * nn + i] > n)))
        return fail(LBM_EINVAL, "schedule entry %zu, column %zu is outside the lattice", e, i);
    }
  }
  if (need > c->replay_cap) {
    if (c->replay) (void)hipFree(c->replay);
    c->replay = nullptr;
    c->replay_cap = 0;
    if ((rc = dalloc(&c->replay, need))) return rc;
    c->replay_cap = need;
  }
  HIP_TRY(hipMemcpyAsync(c->replay, schedule, need * sizeof(int), hipMemcpyHostToDevice,
                         c->stream));
  // phases of entry 0, then the ordinary step with the recorded nodes and switches
  HIP_TRY(hipMemcpyAsync(c->cnt, c->replay, nn * sizeof(int), hipMemcpyDeviceToDevice,
                         c->stream));
  lbmk::KParams& k = c->kp;
  HIP_TRY(lbmk::launch_neighbourhood(k, c->cnt, c->cext, c->rowmax, c->stream));
  for (int64_t t = 0; t < nsteps; ++t) {
    const int nx = c->cur ^ 1, sx = c->scur ^ 1;
    const int* e = c->replay + (size_t)t * 3 * nn;
    k.step = (uint32_t)c->step;
    // the one-cell path throughout (no row maxima): bit for bit the recorded run
    HIP_TRY(lbmk::launch_stream_collide(c->kind, k, c->f[c->cur], c->f[nx], c->g[c->cur], c->g[nx],
                                        c->cnt, c->cext, nullptr, c->s[c->scur], c->th,
                                        c->flag, c->stream));
    if (c->heat)  // conservative front: heat of the streaming from the state g[cur]
      HIP_TRY(lbmk::launch_front_heat(c->kind, k, c->g[c->cur], c->s[c->scur], c->cnt, c->heat,
                                      c->stream));
    HIP_TRY(lbmk::launch_front(c->kind, k, c->s[c->scur], c->s[sx], c->cnt, c->g[nx], c->f[nx],
                               c->th, c->melted, c->frozen, c->flag, e, e + 3 * nn, nullptr,
                               c->heat, nullptr, c->stream));
    if (lbmk::uses_neighbourhood(c->kind))
      HIP_TRY(lbmk::launch_neighbourhood(k, c->cnt, c->cext, c->rowmax, c->stream));
    c->cur = nx;
    c->scur = sx;
    c->step++;
  }
  HIP_TRY(hipStreamSynchronize(c->stream));
  return LBM_OK;
}

int lbm_kernel_timing(lbm_ctx* c, int enable) {
  int rc = check_ctx(c);
  if (rc) return rc;
  c->timing = enable != 0;
  return LBM_OK;
}

int lbm_kernel_time(lbm_ctx* c, double* ms, int64_t* launches) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!ms || !launches) return fail(LBM_EINVAL, "ms and launches are required");
  HIP_TRY(hipStreamSynchronize(c->stream));
  double total = 0.0;
  for (size_t i = 0; i + 1 < c->ev_used; i += 2) {
    float t = 0.0f;
    HIP_TRY(hipEventElapsedTime(&t, c->ev[i], c->ev[i + 1]));
    total += t;
  }
  *ms = total;
  *launches = (int64_t)(c->ev_used / 2);
  c->ev_used = 0;
  return LBM_OK;
}

int lbm_bandwidth_ceiling(int32_t which, int32_t n, int32_t precision, int32_t flow,
                          int32_t reps, void* hip_stream, double* ms_per_launch,
                          double* bytes_per_launch) {
  if (which != LBM_CEIL_COPY && which != LBM_CEIL_PATTERN)
    return fail(LBM_EINVAL, "which = %d is not an lbm_ceiling", which);
  if (n < 4 || n > 1024) return fail(LBM_EINVAL, "n = %d outside [4, 1024]", n);
  if (precision < LBM_F64 || precision > LBM_BF16S)
    return fail(LBM_EINVAL, "precision = %d is not an lbm_precision", precision);
  if (flow != 0 && flow != 1) return fail(LBM_EINVAL, "flow must be 0 or 1");
  if (reps < 1) return fail(LBM_EINVAL, "reps must be >= 1");
  if (!ms_per_launch || !bytes_per_launch)
    return fail(LBM_EINVAL, "ms_per_launch and bytes_per_launch are required");
  lbmk::KParams k{};
  k.n = n;
  k.ncell = (uint32_t)((size_t)n * n * n);
  k.pitch = lbmk::row_pitch(n, precision);
  k.inv_nm2 = lbmk::recip32((uint32_t)(n - 2));
  k.inv_n = lbmk::recip32((uint32_t)n);
  k.flow = flow;
  const size_t esz = lbmk::store_bytes(precision), nn = (size_t)n * n;
  const size_t fb = flow ? 19 * (size_t)k.pitch * nn * esz : 0, gb = 7 * (size_t)k.pitch * nn * esz;
  hipStream_t st = (hipStream_t)hip_stream;
  void* buf[4] = {nullptr, nullptr, nullptr, nullptr};  // fs, fd, gs, gd
  hipEvent_t ev[2] = {nullptr, nullptr};
  auto done = [&](int code) {
    (void)hipStreamSynchronize(st);
    for (void* p : buf)
      if (p) (void)hipFree(p);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
    return code;
  };
  const size_t sizes[4] = {fb, fb, gb, gb};
  for (int b = 0; b < 4; ++b) {
    if (!sizes[b]) continue;
    if (hipMalloc(&buf[b], sizes[b]) != hipSuccess) {
      buf[b] = nullptr;
      return done(fail(LBM_ENOMEM, "cannot allocate %zu bytes", sizes[b]));
    }
    if (hipMemsetAsync(buf[b], 0, sizes[b], st) != hipSuccess)
      return done(fail(LBM_EDEVICE, "hipMemsetAsync failed"));
  }
  auto launch = [&]() -> hipError_t {
    if (which == LBM_CEIL_PATTERN)
      return lbmk::launch_pull_pattern(precision, k, buf[0], buf[1], buf[2], buf[3], st);
    hipError_t e = lbmk::launch_copy4(buf[2], buf[3], gb, st);  // g rows, then f rows
    if (e == hipSuccess && fb) e = lbmk::launch_copy4(buf[0], buf[1], fb, st);
    return e;
  };
  for (int w = 0; w < 2; ++w)
    if (launch() != hipSuccess) return done(fail(LBM_EDEVICE, "ceiling kernel launch failed"));
  if (hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess)
    return done(fail(LBM_EDEVICE, "hipEventCreate failed"));
  if (hipEventRecord(ev[0], st) != hipSuccess) return done(fail(LBM_EDEVICE, "event record"));
  for (int r = 0; r < reps; ++r)
    if (launch() != hipSuccess) return done(fail(LBM_EDEVICE, "ceiling kernel launch failed"));
  if (hipEventRecord(ev[1], st) != hipSuccess || hipEventSynchronize(ev[1]) != hipSuccess)
    return done(fail(LBM_EDEVICE, "ceiling kernels failed on the device"));
  float ms = 0.0f;
  if (hipEventElapsedTime(&ms, ev[0], ev[1]) != hipSuccess)
    return done(fail(LBM_EDEVICE, "hipEventElapsedTime failed"));
  *ms_per_launch = (double)ms / reps;
  *bytes_per_launch = which == LBM_CEIL_PATTERN
                          ? 2.0 * ((flow ? 19.0 : 0.0) + 7.0) * (double)k.ncell * (double)esz
                          : 2.0 * (double)(fb + gb);
  return done(LBM_OK);
}

}  // extern "C"
