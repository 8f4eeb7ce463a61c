/*
 * lbmmelt — double-MRT lattice Boltzmann melting step on one MI355X (gfx950).
 *
 * C ABI of the library liblbmmelt.so.  Plain C99 types only; no exceptions
 * cross this boundary.  Every function returns an lbm_status (0 = success);
 * on failure lbm_last_error() returns a thread-local message.
 *
 * Method: Li, Yang & Zhang, "Lattice Boltzmann method simulation of 3-D
 * melting using double MRT model with interfacial tracking method"
 * (arXiv:1604.03478).  One time step is
 *   1. pull-streaming of f (D3Q19, section 2 Eq. (1) and Eq. (3)) and of g
 *      (D3Q7, Eq. (4) and Eq. (5)) with no-slip, thermal wall and front
 *      boundary conditions,
 *   2. the MRT collision of f (Eq. (2)) with a Boussinesq buoyancy force
 *      (section 1, assumption 4) and the MRT collision of g (Eq. (4)),
 *   3. the interfacial-tracking update of the solid-liquid front from the
 *      interface energy balance, Eq. (6), which masks solid cells out of the
 *      flow.
 * Geometry (section 1): a cube of edge H = n lattice units; the hot wall at
 * t_h, the opposite wall at t_c <= t_m, the other walls adiabatic, no slip
 * on every wall, the solid initially at t_c.
 *
 * Layouts.  Cell (x, y, z) has linear index (z*n + y)*n + x (x fastest).
 * The front s is one value per column along the melt axis: with
 * LBM_HEAT_Y0 the melt axis is y and s is stored [z][x]; with LBM_HEAT_Z0
 * the melt axis is z and s is stored [y][x].  A cell is liquid iff its
 * centre coordinate along the melt axis (index + 1/2) is strictly below the
 * front of its column.
 *
 * Threads and streams.  One context per host thread.  All device work of a
 * context is enqueued on its stream (the caller's, or one the library owns);
 * lbm_step only enqueues.  The functions that return host data
 * (lbm_liquid_fraction, lbm_fields, lbm_get_populations, lbm_save_state,
 * lbm_diagnostics) synchronize that stream.
 */
#ifndef LBMMELT_H
#define LBMMELT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx; /* opaque; owns all of its device memory */

typedef enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,    /* invalid argument or parameter                      */
  LBM_ENOMEM = -2,    /* device or host allocation failed                   */
  LBM_EDEVICE = -3,   /* HIP runtime or kernel launch error                 */
  LBM_EUNSTABLE = -4, /* a non-finite value appeared; state is unusable      */
  LBM_ESTATE = -5     /* call not valid in the context's current state       */
} lbm_status;

/* Storage precision of the distributions.  Every format stores the shifted
 * populations f_q - w_q*rho0 and g_q - w_q*(t_h + t_m)/2.  LBM_F64 and LBM_F32 collide
 * in the storage type; the two 16-bit formats collide in FP32.  The front
 * and all reductions are FP64 in every mode. */
typedef enum { LBM_F64 = 0, LBM_F32 = 1, LBM_F16S = 2, LBM_BF16S = 3 } lbm_precision;

typedef enum {
  LBM_HEAT_Y0 = 0, /* hot wall y = 0, cold wall y = n (paper, section 1) */
  LBM_HEAT_Z0 = 1  /* hot wall z = 0 (bottom heating), all others adiabatic */
} lbm_heating;

typedef struct {
  int32_t n;        /* cells per edge, 4 <= n <= 1024                         */
  double ra;        /* Rayleigh number (flow = 1), > 0                        */
  double pr;        /* Prandtl number (flow = 1), > 0                         */
  double ste;       /* Stefan number c_p (t_h - t_m)/h_sl >= 0; 0 = front fixed*/
  double t_h;       /* hot-wall temperature                                   */
  double t_c;       /* cold-wall and initial solid temperature, t_c <= t_m    */
  double t_m;       /* melting temperature, t_m < t_h                         */
  double ma;        /* Mach number, 0 < ma < 0.3 (section 3.2)                */
  double alpha;     /* lattice thermal diffusivity, used only when flow == 0 */
  double s0;        /* initial front position in lattice units, 0 <= s0 <= n  */
  int32_t heating;  /* lbm_heating                                            */
  int32_t flow;     /* 0: flow frozen (energy distribution only), 1: full    */
  int32_t precision;/* lbm_precision                                          */
  int32_t seed_profile; /* initial temperature: 0 linear from t_h to t_m
                           across the seed layer, solid at t_c; 1 the
                           Neumann profile whose front is at s0, solid at
                           t_c; 2 the two-phase Neumann solution of a solid
                           subcooled to t_c (equal properties) whose front
                           is at s0, in both phases (ste > 0 for 1 and 2)  */
  double ks_kl;     /* solid / liquid thermal conductivity ratio of Eq. (6),
                       >= 0; 0 or 1: equal properties.  rho c is the same in
                       both phases, so the solid diffusivity is ks_kl * alpha */
  int32_t front_scheme; /* interface update: 0 Eq. (6) with one-sided
                           temperature gradients; 1 the same energy balance
                           taken from the heat the lattice carries across
                           the interface links in each step (conserves
                           sum(T) + L sum(s) up to the wall heat)          */
  int32_t f_wall;       /* no-slip of f at the front: 0 halfway bounce-back;
                           1 bounce-back interpolated linearly to the point
                           where the front cuts each link (the link
                           fraction of the front condition of g, extended
                           to the diagonal links).
                           The walls of the box keep halfway bounce-back  */
} lbm_params;

/* Lattice units derived from the parameters (Eq. (7) time scale: the
 * Fourier number is alpha * t / n^2). */
typedef struct {
  double u0;      /* buoyancy velocity scale Ma * c_s                       */
  double nu;      /* kinematic viscosity                                    */
  double alpha;   /* thermal diffusivity                                    */
  double gbeta;   /* buoyancy coefficient g*beta (force = gbeta*(T - t0))   */
  double t0;      /* reference temperature (t_h + t_c)/2                    */
  double s_nu;    /* shear relaxation rate of f                            */
  double q_j;     /* heat-flux relaxation rate of g                        */
  double q_e;     /* remaining relaxation rate of g                        */
} lbm_lattice;

/* Create a context: validates *params (the problem statement of section 1:
 * cube of edge n, hot wall t_h, cold wall t_c <= t_m, adiabatic top and
 * bottom, no slip everywhere, and Ra, Pr, Ste; Mach number below 0.3 as
 * section 3.2 allows), maps them to lattice units (the time scale of
 * Eq. (7)), allocates the double-buffered distributions in HBM and writes
 * the initial state (f at rest, g at equilibrium of the seed temperature
 * profile, front at s0).  hip_stream is a hipStream_t, or NULL for a stream the library
 * creates and owns.  On success *out receives the context.
 * Errors: LBM_EINVAL (bad parameter; e.g. n out of range, t_c > t_m,
 * ma >= 0.3, derived viscous relaxation time <= 0.5 + 1e-3),
 * LBM_ENOMEM, LBM_EDEVICE. */
int lbm_init(const lbm_params *params, void *hip_stream, lbm_ctx **out);

/* Release every device and host resource of ctx (NULL is accepted). */
void lbm_destroy(lbm_ctx *ctx);

/* Enqueue nsteps >= 0 time steps (stream, collide, front update and phase
 * switch; section 2, Eq. (1), (2), (4), (6)).  Asynchronous: the device
 * instability flag is only read by the synchronizing queries.
 * Errors: LBM_EINVAL (nsteps < 0), LBM_ESTATE (a query has reported
 * LBM_EUNSTABLE and no lbm_load_state followed), LBM_EDEVICE. */
int lbm_step(lbm_ctx *ctx, int64_t nsteps);

/* Graph replays of the step loop (a launch-overhead option, not part of the
 * method).  steps = 0 (the default): lbm_step launches every kernel of every
 * step.  steps = an even number in [2, 4096]: lbm_step runs whole chunks of
 * that many steps as replays of one captured HIP graph (the same kernels in
 * the same order, captured on first use and again after the buffer parity
 * changed, e.g. by an odd remainder) and the remaining steps one by one; the
 * step counter that seeds the stochastic rounding lives in device memory
 * while a chunk runs, so the results are the same bit for bit either way.
 * Replays are not used while kernel timing is on or inside lbm_forward_ckpt,
 * lbm_step_replay and lbm_adjoint.  The graph holds pointers into the
 * context only; it lives until the next lbm_set_graph, lbm_forward_ckpt
 * (which moves the populations to other buffers, see there) or lbm_destroy.
 * Costs 4 bytes of device memory and one capture stream.  Synchronizes the
 * context's stream when the setting changes.  Callers that capture the
 * context's stream into a graph of their own leave the setting at 0 (lbm_step
 * then only launches kernels, with no memory operations, and can be
 * captured) and capture again after an lbm_forward_ckpt.
 * Errors: LBM_EINVAL (steps odd, negative or above 4096), LBM_ENOMEM,
 * LBM_EDEVICE (capture failures are reported by the lbm_step that captures). */
int lbm_set_graph(lbm_ctx *ctx, int32_t steps);

/* Liquid fraction: sum of the column fronts over n^3, in FP64 (the quantity
 * plotted against the Fourier number in the paper's Fig. 2 and Fig. 4(d)).
 * Synchronizes.  Returns LBM_EUNSTABLE if a non-finite value was detected in
 * any step so far. */
int lbm_liquid_fraction(lbm_ctx *ctx, double *fl);

/* Copy the macroscopic fields of the current state to host memory, in FP64
 * (section 2: T is the sum of the D3Q7 populations of Eq. (4), rho the sum of
 * the D3Q19 populations of Eq. (1), u the first moment of f).
 * T and rho: n^3 values each; u: 3*n^3 values (u_x, u_y, u_z planes);
 * s: n^2 values.  Any pointer may be NULL.  Solid cells report rho = 0 and
 * u = 0.  u is the velocity the collision used (momentum plus half the
 * force).  Synchronizes; LBM_EUNSTABLE as for lbm_liquid_fraction. */
int lbm_fields(lbm_ctx *ctx, double *T, double *u, double *rho, double *s);

/* Local Nusselt number on the heated wall, per column (n^2 FP64 values to
 * host memory, column layout of s): the distribution the paper shows for its
 * convection cases (section 3.2, Fig. 4(b) and Fig. 5(b)), which it does not
 * define.  Here Nu = -n (dT/da)(a = 0) / (t_h - t_m), a the melt-axis
 * coordinate, dT/da from the quadratic through the wall point (0, T_w) and
 * the first two cell centres (1/2, 3/2) when both are liquid, else from the
 * chord to the front point (s, t_m); 0 in a column with no liquid.
 * Synchronizes; LBM_EUNSTABLE as for lbm_liquid_fraction. */
int lbm_wall_nusselt(lbm_ctx *ctx, double *nu);

/* Derived lattice parameters of the context. */
int lbm_get_lattice(const lbm_ctx *ctx, lbm_lattice *out);

/* Number of time steps taken since lbm_init (or restored by
 * lbm_load_state). */
int lbm_get_step(const lbm_ctx *ctx, int64_t *step);

/* Set the hot-wall temperature of every column (n^2 FP64 values, column
 * layout of s).  th points to device memory if on_device != 0, else to host
 * memory.  Takes effect from the next step; the initial seed profile always
 * uses params->t_h.  Enqueued on the context stream. */
int lbm_set_hot_wall(lbm_ctx *ctx, const double *th, int on_device);

/* Overwrite the state with unshifted FP64 populations from host memory:
 * f is 19*n^3 values in the velocity order of Eq. (3) ([q][z][y][x]; NULL
 * when flow == 0), g is 7*n^3 values in the order of Eq. (5), s is n^2 front
 * positions.  Values are rounded to the storage precision.  Synchronizes. */
int lbm_set_populations(lbm_ctx *ctx, const double *f, const double *g,
                        const double *s);

/* Copy the current state out as unshifted FP64 populations (same layout as
 * lbm_set_populations; any pointer may be NULL).  Synchronizes. */
int lbm_get_populations(lbm_ctx *ctx, double *f, double *g, double *s);

/* FP64 reductions of the current state.  out[0] liquid mass (sum of rho over
 * liquid cells), out[1] thermal energy sum of (T - t_m) over all cells,
 * out[2] sum of the fronts, out[3] cells melted since init, out[4] cells
 * that changed from liquid to solid since init.  Synchronizes. */
int lbm_diagnostics(lbm_ctx *ctx, double out[5]);

/* The same reductions as lbm_diagnostics, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): this call allocates nothing.  The partial
 * sums of its reduction live in a fixed device array of the library
 * (5 * 1024 + 5 FP64 values, 41 KB on every GPU the library runs on, held
 * until the process ends), enough for every lattice lbm_init accepts; a
 * larger need would be rejected with LBM_EINVAL.  out: 5 values as for
 * lbm_diagnostics.  on_device != 0: out is device memory and the call only
 * enqueues on the context stream (no synchronization; the instability flag
 * is not read).  on_device == 0: out is host memory, the call synchronizes
 * and reports LBM_EUNSTABLE as lbm_diagnostics does.  Every call on one GPU
 * uses that GPU's one array, whose contents each call overwrites: calls that
 * overlap on one GPU (unordered streams or threads) race and give wrong
 * sums.  Errors: LBM_EINVAL, LBM_EDEVICE, LBM_EUNSTABLE. */
int lbm_diagnostics_noalloc(lbm_ctx *ctx, double *out, int on_device);

/* Checkpoint.  With host_buf == NULL, *bytes receives the size needed.
 * Otherwise the state (distributions in storage precision, front, counters,
 * step) is copied into host_buf, which must hold *bytes bytes.
 * lbm_load_state restores a blob made by a context with the same n,
 * precision, flow and heating (else LBM_EINVAL), and clears the unstable
 * flag.  Both synchronize. */
int lbm_save_state(lbm_ctx *ctx, void *host_buf, size_t *bytes);
int lbm_load_state(lbm_ctx *ctx, const void *host_buf, size_t bytes);

/* Gradient of the liquid fraction with respect to the hot-wall temperatures
 * (reverse mode; not part of the paper, which runs the forward method only).
 * lbm_forward_ckpt runs nsteps >= 1 steps from the current state exactly as
 * lbm_step does and keeps the state every every_k >= 1 steps
 * (ceil(nsteps/every_k) states; the checkpoints take over the context's
 * population buffers of those states instead of copying them, and the
 * context continues in buffers of the same size, so a step graph captured
 * before is captured again at the next replay); *fl (may be NULL) receives
 * the liquid fraction at the end.  lbm_adjoint then writes grad_th[c] = dJ/dT_h(c) for
 * J = dJ_dfl * f_l at the end of that run: it recomputes each segment of
 * every_k steps from its checkpoint (holding the populations of every_k
 * states in device memory, the first state of a segment being its
 * checkpoint, read in place) and applies the transposed step in reverse
 * order.  When the run has several segments and free device memory holds a
 * second set of every_k states with a quarter and 4 GB to spare,
 * lbm_adjoint allocates it (kept
 * with the context, like the first) and recomputes each segment on a stream
 * of its own while the context's stream reverses the segment after it; the
 * gradient is the same bit for bit either way, and for every every_k.  The phase
 * masks and the node selection of Eq. (6) are those of the forward run (the
 * gradient of the piecewise-smooth map along that schedule).  grad_th has
 * n^2 values in the column layout of s and points to device memory if
 * on_device != 0.  lbm_adjoint needs a preceding lbm_forward_ckpt with no
 * lbm_step, lbm_step_replay, lbm_set_hot_wall, lbm_set_populations or
 * lbm_load_state since (else LBM_ESTATE): the recompute between checkpoints
 * uses the current hot wall; it does not change the state.  Both
 * synchronize.  Every front_scheme and f_wall is covered.  Errors:
 * LBM_EINVAL, LBM_ENOMEM, LBM_ESTATE, LBM_EDEVICE. */
int lbm_forward_ckpt(lbm_ctx *ctx, int64_t nsteps, int32_t every_k, double *fl);
int lbm_adjoint(lbm_ctx *ctx, double dJ_dfl, double *grad_th, int on_device);

/* The schedule of the run recorded by the last lbm_forward_ckpt: for every
 * step and the state after the last one, 3*n^2 ints (liquid count of every
 * column, index of its first liquid node and of its first solid node used
 * by Eq. (6)); (nsteps + 1) * 3 * n^2 ints in all (the node slots of the
 * final entry are unused: zeros).  lbm_step_replay takes
 * nsteps steps along such a schedule (phases and node selection fixed, every
 * other quantity recomputed): the map whose derivative lbm_adjoint gives,
 * for finite-difference checks.  The schedule is host memory; both
 * synchronize.  lbm_step_replay returns LBM_EINVAL for a schedule whose
 * counts or node indices lie outside the lattice. */
int lbm_get_schedule(lbm_ctx *ctx, int32_t *out, size_t count);
int lbm_step_replay(lbm_ctx *ctx, const int32_t *schedule, int64_t nsteps);

/* Kernel timing for measurement.  While enabled (enable != 0), the dispatch
 * of every step's fused stream-collide kernel records a pair of HIP events
 * at the kernel's start and end (hipExtLaunchKernel, on the context stream).
 * lbm_kernel_time synchronizes, returns the summed duration of those kernels
 * in milliseconds and their count, and clears the record.  Steps are then
 * launched one by one (no graph replays); leave it off when timing whole
 * steps. */
int lbm_kernel_timing(lbm_ctx *ctx, int enable);
int lbm_kernel_time(lbm_ctx *ctx, double *ms, int64_t *launches);

/* Bandwidth ceilings for the measurement of the step kernel (a measurement
 * aid, not part of the method; no context needed).  Kernels:
 *   LBM_CEIL_COPY     a float4 copy of buffers the size of one step's
 *                     distributions at (n, precision, flow), each byte read
 *                     once and written once (non-temporal stores);
 *   LBM_CEIL_PATTERN  the bare access pattern of the all-liquid step in the
 *                     step kernel's row-interleaved layout, launch shape and
 *                     row order: every population pulled from its source
 *                     (bounce-back addresses at the walls) and stored, with
 *                     no arithmetic.
 * The buffers (four distribution-sized device allocations) are allocated,
 * zero-filled and freed here.  Two untimed launches, then reps >= 1 launches
 * timed with HIP events on hip_stream (a hipStream_t; NULL is the default
 * stream): *ms_per_launch their average duration, *bytes_per_launch the bytes
 * one launch moves (for the pattern the algorithmic 2 (19 + 7) n^3 element
 * bytes; without flow 2 * 7 n^3).  Synchronizes.  Errors: LBM_EINVAL,
 * LBM_ENOMEM, LBM_EDEVICE. */
typedef enum { LBM_CEIL_COPY = 0, LBM_CEIL_PATTERN = 1 } lbm_ceiling;
int lbm_bandwidth_ceiling(int32_t which, int32_t n, int32_t precision, int32_t flow,
                          int32_t reps, void *hip_stream, double *ms_per_launch,
                          double *bytes_per_launch);

/* Thread-local message describing the last error of this thread. */
const char *lbm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LBMMELT_H */
