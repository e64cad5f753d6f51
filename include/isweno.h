/*
 * isweno.h - C ABI of the MI355X (gfx950) library for the incremental-stencil
 * WENO finite-volume right-hand side of compressible two-phase flow
 * (B. Wang, G. Xiang, W. Zhang, X. Y. Hu, "An incremental-stencil WENO
 * reconstruction for simulation of compressible two-phase flows",
 * arXiv:1707.00592).
 *
 * The library evaluates the semi-discrete operator dU/dt = L(U) of the
 * quasi-conservative stiffened-gas model (Sec. 2, eqs. (1)-(4); Sec. 3.1,
 * eqs. (5)-(7)) on a uniform Cartesian grid, dimension by dimension, with
 *   - characteristic primitive-variable projection (Sec. 3.2, eqs. (9)-(13)),
 *   - WENO-IS reconstruction (Sec. 3.3, eqs. (19)-(29)),
 *   - the MOOD-type positivity cascade (Sec. 3.4, eq. (32)),
 *   - the HLLC flux and interface velocity (Sec. 3.2.1, eqs. (14)-(18)),
 * and advances it with the third-order TVD Runge-Kutta scheme cited in
 * Sec. 3.1 (Shu-Osher form).
 *
 * Conventions for every entry point:
 *   - Array arguments are DEVICE pointers (HIP device memory of the device
 *     the context was created on), owned by the caller.  The library never
 *     frees or keeps them beyond the call.
 *   - Conservative state U: float64, component-major (SoA), x fastest,
 *     interior cells only (ghost cells are synthesised from the boundary
 *     conditions inside the library).  Components, nc = 4 + ndim:
 *       (rho, rho*u[, rho*v[, rho*w]], E, Gamma, Pi)
 *     with Gamma = 1/(gamma-1) and Pi = gamma*Pinf/(gamma-1) (eqs. (2),
 *     (7), (9)).  Element (c, i, j, k) is at U[c*N + i + nx*(j + ny*k)],
 *     N = nx*ny*nz.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Every call is
 *     asynchronous on that stream and does no host synchronisation, so it
 *     can be captured into a HIP graph (the first call for a new grid size
 *     may allocate workspace; make one uncaptured call first).
 *   - Return value: ISWENO_OK, or a negative code for errors detected on the
 *     host (bad argument, unsupported option, HIP error), in which case
 *     nothing is enqueued.  Non-physical states found on the device are
 *     latched into stats->status (see isweno_stats).
 *   - Not thread-safe per context: calls on one context must not overlap
 *     from several host threads.
 */
#ifndef ISWENO_H
#define ISWENO_H

#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define ISWENO_API __attribute__((visibility("default")))
#else
#define ISWENO_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef struct isweno_ctx isweno_ctx;
typedef struct isweno_batch_plan isweno_batch_plan;

enum {
  ISWENO_OK = 0,
  ISWENO_ERR_ARG = -1,          /* invalid argument (host-detected) */
  ISWENO_ERR_UNSUPPORTED = -2,  /* option combination not available */
  ISWENO_ERR_DEVICE = -3,       /* a HIP runtime call failed */
  ISWENO_ERR_NONPHYSICAL = -4   /* latched on the device, see isweno_stats */
};

/* Boundary conditions per axis side (ghost cells, 3 per side). */
enum {
  ISWENO_BC_TRANSMISSIVE = 0, /* zero gradient: copy of the boundary cell
                                 (the "non-reflection"/"constant
                                 extrapolation" conditions of Sec. 6) */
  ISWENO_BC_PERIODIC = 1,     /* periodic (Sec. 4) */
  ISWENO_BC_REFLECTIVE = 2    /* mirror with the normal velocity negated
                                 (the reflecting walls of Sec. 6.1) */
};

/* Arithmetic of the reconstruction and flux; the state stays float64. */
enum {
  ISWENO_FP64 = 0,  /* everything in float64 */
  ISWENO_FP32 = 1   /* projection, WENO-IS and HLLC in float32; primitive
                       recovery, the positivity check of the MOOD cascade,
                       the flux difference and the Runge-Kutta update in
                       float64 */
};

/* Nonlinear weights of the reconstruction. */
enum {
  ISWENO_W_MODIFIED = 0, /* eq. (28), Sec. 3.3.2 (the paper's final form) */
  ISWENO_W_BASIC = 1,    /* eq. (21) with q = 1 */
  ISWENO_W_MLP = 2,      /* learned weights (isweno_mlp_*) for the
                            acoustic, entropy and shear fields, with the
                            eq. (28) weights as fallback (confidence below
                            the threshold, a face value outside the range
                            of the two cells next to the face, or a face
                            state that fails the positivity check, which
                            is redone with them before the MOOD cascade)
                            and for the material fields Gamma, Pi
                            throughout */
  ISWENO_W_CUTOFF = 3    /* not in the paper: the targeted-ENO cut-off that
                            its conclusions (Sec. 7) propose for lower
                            dissipation in smooth regions, on the eq. (28)
                            quantities.  Stencil k has the measure
                            gamma_k = (alpha_k/d_k)^6; stencils whose share
                            gamma_k / sum gamma is below C_T = 1e-5 get
                            weight 0, the others d_k renormalised over the
                            kept ones (exactly d_k when none is cut, i.e.
                            the linear 5th-order scheme on resolved smooth
                            data).  Order 3 of the MOOD cascade cuts among
                            the two 2-point stencils. */
};

typedef struct {
  int32_t ndim;     /* 1, 2 or 3 */
  int32_t reserved; /* must be 0 */
  int64_t n[3];     /* interior cells per axis (x, y, z); unused axes = 1 */
  double dx[3];     /* cell size per axis, > 0 */
  int32_t bc_lo[3]; /* ISWENO_BC_* at the low end of each axis */
  int32_t bc_hi[3]; /* ISWENO_BC_* at the high end of each axis */
} isweno_grid;

typedef struct {
  int32_t precision; /* ISWENO_FP64 or ISWENO_FP32 */
  int32_t weights;   /* ISWENO_W_* */
  int32_t mood;      /* 1: MOOD-type positivity cascade of Sec. 3.4, each
                        failing face side redone inside its wave;
                        2: the same cascade with the failing faces of a
                        tile gathered and redone by full waves after the
                        tile's faces (the fused 2D stage; elsewhere as 1):
                        the same results, faster only where fallbacks are
                        dense; 0: off */
  int32_t reserved;  /* must be 0 */
  double eps;        /* epsilon in eqs. (21)/(28); the paper leaves it open,
                        1e-40 is the default reading */
  double cfl;        /* > 0: isweno_rk3_step computes
                        dt = cfl / max_cells sum_d (|u_d| + c)/dx_d from U^n
                        and writes it to *dt; <= 0: *dt is used as given */
  double dt_max;     /* > 0: upper bound on the computed dt (e.g. the time
                        left to a final time); <= 0: none */
  const uint16_t *mlp_params; /* ISWENO_W_MLP only: device pointer to the
                        network in the bf16 layout of isweno_mlp_pack */
  float mlp_conf_threshold;   /* ISWENO_W_MLP only: fall back to the
                        eq. (28) weights when sigmoid(confidence) is below */
  int32_t reserved2;          /* must be 0 */
} isweno_opts;

/* Device-resident counters, accumulated over calls; the caller allocates
 * and zeroes it (sizeof(isweno_stats) bytes of device memory). */
typedef struct {
  uint64_t o3[3];           /* face sides per axis that fell back to the
                               3rd-order reconstruction (Sec. 3.4) */
  uint64_t o1[3];           /* face sides per axis that fell back to the
                               1st-order state, eq. (32) */
  uint64_t mlp_fallback[3]; /* ISWENO_W_MLP: per axis, face-fields below
                               the confidence threshold plus face sides
                               outside their cell range, whose learned
                               weights were replaced by those of eq. (28),
                               plus face sides whose learned state failed
                               the positivity check of Sec. 3.4 and was
                               redone with the eq. (28) weights (before the
                               order-3 / order-1 cascade, which o3 and o1
                               count) */
  int32_t status;           /* ISWENO_OK, or ISWENO_ERR_NONPHYSICAL once an
                               input cell of any evaluation had rho <= 0,
                               Gamma <= 0, c^2 <= 0 or a non-finite value;
                               while it is set, later calls write nothing */
  int32_t reserved;
} isweno_stats;

/* Context: workspace (two state-sized buffers, grown on demand), a device
 * scalar for the time-step reduction and the batch plans' graphs.  Makes
 * `device` current on the calling thread. */
ISWENO_API int isweno_create(isweno_ctx **out, int device);
ISWENO_API void isweno_destroy(isweno_ctx *ctx);

/* dUdt = L(U): eq. (5) for rho, momenta and E and eq. (6) for Gamma and Pi,
 * summed over axes x, then y, then z (Sec. 3, dimension by dimension), with
 * face states from eqs. (12)-(13) and (19) and the flux of eqs. (14)-(18).
 * U and dUdt are nc*N float64 each and must not overlap.  stats may be NULL
 * (no counters, no status latch). */
ISWENO_API int isweno_rhs(isweno_ctx *ctx, const isweno_grid *grid,
               const isweno_opts *opts, const double *U, double *dUdt,
               isweno_stats *stats, void *stream);

/* Device time step: dt[0] = cfl / max_cells sum_d (|u_d| + c)/dx_d,
 * clipped to opts->dt_max when that is > 0 (the CFL condition behind the
 * Courant number 0.5 of Secs. 5 and 6).  Requires opts->cfl > 0. */
ISWENO_API int isweno_cfl_dt(isweno_ctx *ctx, const isweno_grid *grid,
                  const isweno_opts *opts, const double *U, double *dt,
                  void *stream);

/* One third-order TVD Runge-Kutta step in place (U: U^n in, U^{n+1} out):
 *   U1 = U + dt L(U); U2 = 3/4 U + 1/4 (U1 + dt L(U1));
 *   U^{n+1} = 1/3 U + 2/3 (U2 + dt L(U2)).
 * dt is a device scalar: computed from U^n and written when opts->cfl > 0
 * (the value of isweno_cfl_dt on U^n; in the FP32 form of a 2D or 3D grid
 * within a few ulp of it, its primitive recovery dividing through
 * reciprocals), read otherwise.  The step's launches are captured once into a HIP graph
 * per (U, dt, stats, grid, opts) and replayed on the given stream; with
 * kernel timing enabled, or with opts->dt_max > 0, they are launched
 * directly instead.  Same results either way. */
ISWENO_API int isweno_rk3_step(isweno_ctx *ctx, const isweno_grid *grid,
                    const isweno_opts *opts, double *U, double *dt,
                    isweno_stats *stats, void *stream);

/* isweno_rk3_step for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same step with the same results, but its intermediate states and
 * time-step words live in a fixed scratch array of the library (a device
 * global of 128 MiB plus 256 bytes that every GPU the library runs on holds
 * until the process ends) instead of the context's workspace, and it
 * launches its kernels directly (no graph, no timing events).  It calls no
 * hipMalloc, hipFree or other allocating routine.
 *   - Limit: (2 * nc * N + T) * 8 bytes <= 128 MiB, T the number of tiles
 *     whose wave speeds a step with cfl > 0 keeps (2D: 15 x 16 cells; 3D:
 *     31 x 8 cells of x lines; else 0) (2D, nc = 6: N up to about 1,397,600
 *     cells; 3D, nc = 7: N up to about 1,197,900); larger grids return
 *     ISWENO_ERR_ARG and enqueue nothing.  Other errors as isweno_rk3_step.
 *   - The scratch is shared by every call on one GPU and keeps the last
 *     call's contents; the step clears what must start at zero.  Calls that
 *     overlap on one GPU (other streams, other contexts, other host threads)
 *     race on it: order them. */
ISWENO_API int isweno_rk3_step_noalloc(isweno_ctx *ctx, const isweno_grid *grid,
                            const isweno_opts *opts, double *U, double *dt,
                            isweno_stats *stats, void *stream);

/* ---- many independent 1D problems (uneven lengths) ----
 * Problem p owns cells offsets[p] .. offsets[p+1]-1 of a state laid out as
 * U[c*offsets[nprob] + cell], c = 0..4 (1D components), with its own cell
 * size dx[p] and time step dt[p]; every problem uses the boundary
 * conditions bc_lo / bc_hi.  A plan copies offsets and dx (HOST arrays,
 * offsets[0] = 0, increasing, every length >= 1, >= 3 with a reflective
 * end) to the device, cuts the problems into tiles and keeps the launch
 * configuration (tile length and persistent grid size). */
ISWENO_API int isweno_batch_plan_create(isweno_ctx *ctx, int32_t nprob,
                             const int64_t *offsets, const double *dx,
                             int32_t bc_lo, int32_t bc_hi,
                             isweno_batch_plan **out);
ISWENO_API void isweno_batch_plan_destroy(isweno_batch_plan *plan);

/* Times every tile configuration on a scratch copy of U (device) and keeps
 * the fastest for this plan; *chosen_tile (may be NULL) receives the tile
 * length picked.  Synchronises the stream. */
ISWENO_API int isweno_batch_autotune(isweno_ctx *ctx, isweno_batch_plan *plan,
                          const isweno_opts *opts, const double *U,
                          int32_t *chosen_tile, void *stream);

/* nsteps RK3 steps of every problem, in place.  dt: device [nprob]; with
 * opts->cfl > 0 each problem's dt is recomputed from its own cells at the
 * start of every step and written there, otherwise it is read.
 * status: device int32 [nprob], required, sticky per problem: a problem is
 * advanced only while its entry is ISWENO_OK (0).  A problem whose stage
 * input has a non-finite or non-physical interior cell gets
 * ISWENO_ERR_NONPHYSICAL; the step in which that is found is completed (its
 * values are then unspecified) and the problem is not advanced afterwards,
 * while the other problems go on.  stats (may be NULL) gets the MOOD
 * counters and, when any problem failed, ISWENO_ERR_NONPHYSICAL.  Each step
 * is one HIP graph launch (per-problem start-of-step kernel plus three
 * persistent stage kernels), instantiated on first use for this (plan, U,
 * dt, stats, status, opts) and replayed afterwards. */
ISWENO_API int isweno_batch_step(isweno_ctx *ctx, isweno_batch_plan *plan,
                      const isweno_opts *opts, double *U, double *dt,
                      int32_t nsteps, isweno_stats *stats, int32_t *status,
                      void *stream);

/* ---- learned weights (not in the paper) ----
 * A network 8 -> 32 -> 32 -> 9 (ReLU) replaces the nonlinear weights of
 * eq. (19): per face and characteristic field its input is the six
 * characteristic values of the stencil scaled to [0, 1] by their range
 * (all zero when the range is at most 1e-30) plus two material features, its output two softmax heads of four
 * weights (left and right face states) and a confidence logit.
 * Parameters are float32 masters, layout W1[32][8], b1[32], W2[32][32],
 * b2[32], W3[9][32], b3[9] (ISWENO_MLP_NPARAM floats). */
#define ISWENO_MLP_NI 8
#define ISWENO_MLP_H 32
#define ISWENO_MLP_NO 9
#define ISWENO_MLP_NPARAM (32 * 8 + 32 + 32 * 32 + 32 + 9 * 32 + 9)

/* Face samples for training: for every face of every axis and every
 * characteristic field, the 8 network inputs X[n][8] and the eq. (28)
 * weights of both sides Y[n][8] (float32), computed from U.  Face-field g
 * (axis-major, then face, then field) is written at row g/stride when
 * g % stride == 0 and g/stride < max_samples; *count (device int64)
 * receives the number of rows written.  Synchronises the stream. */
ISWENO_API int isweno_mlp_samples(isweno_ctx *ctx, const isweno_grid *grid,
                       const isweno_opts *opts, const double *U, float *X,
                       float *Y, int64_t max_samples, int64_t stride,
                       int64_t *count, void *stream);

/* Forward pass in bf16 matrix-core arithmetic with float32 accumulation:
 * out[n][9] = logits.  params: float32 masters (converted on the fly). */
ISWENO_API int isweno_mlp_forward(isweno_ctx *ctx, const float *params, const float *X,
                       int64_t n, float *out, void *stream);

/* Inference exactly as the stage kernel runs it (isweno_opts.weights =
 * ISWENO_W_MLP): packed bf16 parameters (isweno_mlp_pack), activations kept
 * in registers, bf16 matrix-core layers with float32 accumulation, 64
 * samples per wavefront.  X: device float [n][8]; out: device float [n][9]
 * logits.  For users who cannot run the whole solver and for checking the
 * solver's network against the float32 one. */
ISWENO_API int isweno_mlp_infer(isweno_ctx *ctx, const uint16_t *packed, const float *X,
                     int64_t n, float *out, void *stream);

/* Loss, averaged over the n samples, and its gradient w.r.t. the float32
 * parameters, from bf16 forward/backward matrix-core kernels.  Per side
 * (left, right) the value the predicted weights give, applied to the
 * candidates of eq. (20) on the sample's normalised stencil X[0..5] (left
 * from X[0..4], right from the mirror X[5..1]), is compared with the value
 * the target weights Y give: ((qhat - q) / 0.01)^2.  Plus binary
 * cross-entropy of the confidence logit against C in {0,1}; C may be NULL:
 * the label is then 1 when both |qhat - q| < 0.005 (units of the stencil's
 * range) and 0 otherwise.  loss: device float[1]; grad: device
 * float[ISWENO_MLP_NPARAM] (overwritten).  Deterministic: the per-workgroup
 * partial sums are reduced in a fixed order. */
ISWENO_API int isweno_mlp_loss_grad(isweno_ctx *ctx, const float *params, const float *X,
                         const float *Y, const float *C, int64_t n,
                         float *loss, float *grad, void *stream);

/* One Adam step (float32) on params with moment buffers m, v (device,
 * ISWENO_MLP_NPARAM floats each, zero before step 1); step is 1-based. */
ISWENO_API int isweno_mlp_adam(isweno_ctx *ctx, float *params, const float *grad,
                    float *m, float *v, int32_t step, float lr, float beta1,
                    float beta2, float eps, void *stream);

/* Packs float32 parameters into the bf16 device layout opts->mlp_params
 * points to (ISWENO_MLP_NPARAM uint16 values). */
ISWENO_API int isweno_mlp_pack(isweno_ctx *ctx, const float *params, uint16_t *packed,
                    void *stream);

/* ---- kernel timing (measurement support) ----
 * While enabled, every stage and time-step launch the library makes outside
 * a graph records a pair of HIP events through the dispatch itself (start
 * and end of its kernels, on its launch stream, without the launch latency
 * around them); durations are accumulated per kernel kind.  isweno_timing_read synchronises on the
 * recorded events and returns the total milliseconds and launch count of
 * one kind since the last enable. */
enum {
  ISWENO_K_SWEEP_X = 0,  /* stage sweep along x (also the whole 1D stage) */
  ISWENO_K_SWEEP_Y = 1,  /* stage sweep along y */
  ISWENO_K_SWEEP_Z = 2,  /* stage sweep along z */
  ISWENO_K_CFL = 3,      /* time-step reduction */
  ISWENO_K_STAGE2D = 4,  /* whole stage of a 2D grid, x and y faces fused
                            (plain and float32 forms) */
  ISWENO_K_COUNT = 8
};
ISWENO_API int isweno_timing_enable(isweno_ctx *ctx, int enable);
ISWENO_API int isweno_timing_read(isweno_ctx *ctx, int kind, double *total_ms,
                                  int64_t *launches);

/* Field-sides per axis (counts[0..2], host memory) whose reconstruction
 * took its shortcut since timing was last enabled.  FP64: the global
 * indicator tau5 of eq. (25) is exactly zero, so every weight of eqs. (21)
 * and (28) is exactly d_k and the value is the linear combination of the
 * candidates of eq. (20) (bit-identical; no other indicator or division is
 * formed).  FP32 form: the stencil's spread is below 1e-30 and its centre
 * value is returned.  Counted by the stage sweeps of isweno_rhs and
 * isweno_rk3_step while timing is enabled (never inside a captured step).
 * Synchronises the device.  Errors: ISWENO_ERR_ARG for a null pointer,
 * ISWENO_ERR_DEVICE. */
ISWENO_API int isweno_shortcut_read(isweno_ctx *ctx, int64_t *counts);

/* Library version string. */
ISWENO_API const char *isweno_version(void);

#ifdef __cplusplus
}
#endif
#endif /* ISWENO_H */
