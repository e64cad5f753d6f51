/*
 * Oracle for the incremental-stencil WENO (WENO-IS) finite-volume method of
 * Wang, Xiang, Zhang & Hu, "An incremental-stencil WENO reconstruction for
 * simulation of compressible two-phase flows" (arXiv:1707.00592).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, FP64 CPU implementation
 * written from the paper.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header
 * or constant with the HIP library and must never be used as a fallback
 * for it.
 *
 * Conventions (shared by all functions below):
 *   - Conservative state per cell, component-major (SoA), x fastest:
 *       ndim=1: (rho, rho*u, E, Gamma, Pi)                 nc = 5
 *       ndim=2: (rho, rho*u, rho*v, E, Gamma, Pi)          nc = 6
 *       ndim=3: (rho, rho*u, rho*v, rho*w, E, Gamma, Pi)   nc = 7
 *     with Gamma = 1/(gamma-1) and Pi = gamma*Pinf/(gamma-1), the two
 *     advected material properties (Sec. 2 eq. (4) and Sec. 3.1 eq. (7);
 *     the reading Gamma = 1/(gamma-1) follows eqs. (7) and (9)).
 *   - Primitive state at a face of direction d ("face order"):
 *       (rho, u_n, u_t..., p, Gamma, Pi), u_n the velocity along d and the
 *       transverse velocities in ascending axis order (Sec. 3.2 eq. (9),
 *       dimension by dimension as stated at the start of Sec. 3).
 *   - Characteristic fields in the row order of L in eq. (11):
 *       (u-c wave, entropy, transverse..., Gamma, Pi, u+c wave).
 */
#ifndef ISWENO_ORACLE_H
#define ISWENO_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define OR_OK 0
#define OR_ERR_ARG (-1)
#define OR_ERR_NONPHYSICAL (-4)
#define OR_ERR_VACUUM (-5)

#define OR_BC_TRANSMISSIVE 0
#define OR_BC_PERIODIC 1
#define OR_BC_REFLECTIVE 2

#define OR_W_MODIFIED 0 /* Sec. 3.3.2, eq. (28) */
#define OR_W_BASIC 1    /* Sec. 3.3.1, eq. (21) with q = 1 */
/* Cut-off of the eq. (28) weights in the manner of the targeted ENO schemes
 * that the conclusions (Sec. 7) name as the next step: stencils whose share
 * of the smoothness measure is below OR_CUTOFF_CT are dropped, the others
 * take the optimal weights.  Not part of the paper's scheme. */
#define OR_W_CUTOFF 3
#define OR_CUTOFF_CT 1e-5 /* C_T of the 5th-order targeted ENO scheme */
#define OR_CUTOFF_Q 6     /* exponent q of its smoothness measure */

#define OR_MAXNC 7

typedef struct {
  int ndim;
  long n[3];
  double dx[3];
  int bc_lo[3], bc_hi[3];
} or_grid;

typedef struct {
  int weights; /* OR_W_MODIFIED, OR_W_BASIC or OR_W_CUTOFF */
  int mood;    /* 1: MOOD-type positivity cascade of Sec. 3.4 */
  double eps;  /* epsilon of the weights, eqs. (21), (28) */
  double cfl;  /* Courant number for the time step */
} or_opts;

typedef struct {
  long o3[3]; /* face sides that fell back to the 3rd-order reconstruction */
  long o1[3]; /* face sides that fell back to the 1st-order state */
  int status; /* OR_OK or OR_ERR_NONPHYSICAL */
} or_stats;

/* ---- building blocks (exposed for the pins) ---- */

/* Candidate values q^(1..4) at x_{i+1/2} of eq. (20) from v = q_{i-2..i+2}. */
void or_weno_candidates(const double v[5], double cand[4]);
/* Indicators (beta1..beta4, beta12, tau5) of eqs. (24), (25), (29). */
void or_weno_indicators(const double v[5], double ind[6]);
/* Nonlinear weights omega_1..4; order 5 uses all four candidate stencils,
 * order 3 drops the two 3-point stencils (d3 = d4 = 0, end of Sec. 3.3.1). */
void or_weno_weights(const double v[5], int weights, double eps, int order,
                     double omega[4]);
/* Reconstructed left value at x_{i+1/2}, eq. (19). */
double or_weno_is(const double v[5], int weights, double eps, int order);

/* L and R of eq. (11) (nc x nc, row-major) at the averaged face state
 * qbar (face order).  nt = number of transverse velocities (ndim - 1). */
void or_eigen(int nt, const double qbar[], double *L, double *R);

/* HLLC flux of Sec. 3.2.1 (eqs. (14)-(18)) in face order, plus u^HLLC. */
void or_hllc(int nt, const double ql[], const double qr[], double F[],
             double *ustar);

/* One face: q6 = six cells i-2..i+3 (face order, 6 x nc row-major).
 * Returns the face states after the MOOD cascade, the order used on each
 * side (5, 3 or 1) and the HLLC flux. */
void or_face(int nt, const double q6[], const or_opts *o, double ql[],
             double qr[], int order_lr[2], double F[], double *ustar);

/* Positivity test used by the MOOD cascade on a face-order state. */
int or_pos(int nt, const double q[]);

/* Threads of the oracle's OpenMP loops: sets them when n > 0 and returns
 * the number in force (1 without OpenMP). */
int or_threads(int n);

/* ---- the semi-discrete operator and time stepping ---- */

/* dU/dt = L(U), Sec. 3.1 eqs. (5)-(6), dimension by dimension. */
int or_rhs(const or_grid *g, const or_opts *o, const double *U, double *dUdt,
           or_stats *st);
/* dt = cfl / max_cells sum_d (|u_d| + c) / dx_d. */
int or_cfl_dt(const or_grid *g, const or_opts *o, const double *U, double *dt);
/* One third-order TVD Runge-Kutta step (Shu & Osher form), in place. */
int or_rk3_step(const or_grid *g, const or_opts *o, double *U, double dt,
                or_stats *st);
/* nsteps RK3 steps on each of nprob independent 1D problems stored back to
 * back: U is [5][offsets[nprob]], problem p owns cells
 * offsets[p]..offsets[p+1]-1 with cell size dx[p].  If o->cfl > 0 each
 * problem's dt is recomputed every step and written to dt[p]; otherwise
 * dt[p] is used as given.  A problem stops after the step in which its
 * status became non-OK; pstatus (may be NULL) holds the per-problem status
 * on entry (problems not OK are skipped) and on exit. */
int or_batch_step(int nprob, const long *offsets, const double *dx, int bc_lo,
                  int bc_hi, const or_opts *o, double *U, double *dt,
                  int nsteps, or_stats *st, int *pstatus);

/* ---- exact stiffened-gas Riemann problem (verification only) ----
 * W = (rho, u, p, gamma, Pinf). */
int or_exact_star(const double WL[5], const double WR[5], double *pstar,
                  double *ustar);
void or_exact_sample(const double WL[5], const double WR[5], double pstar,
                     double ustar, double xi, double W[5]);
/* or_exact_sample at n coordinates xi[0..n-1]; W is n x 5, row-major. */
void or_exact_sample_n(const double WL[5], const double WR[5], double pstar,
                       double ustar, const double *xi, long n, double *W);

/* ---- reference MLP for the learned-weights form (FP64) ----
 * Layout of params (float64): W1[H][NI], b1[H], W2[H][H], b2[H],
 * W3[NO][H], b3[NO] with NI = 8, H = 32, NO = 9.  Outputs: two softmax
 * heads over 4 weights (left, right) and one confidence logit. */
#define OR_MLP_NI 8
#define OR_MLP_H 32
#define OR_MLP_NO 9
#define OR_MLP_NPARAM \
  (OR_MLP_H * OR_MLP_NI + OR_MLP_H + OR_MLP_H * OR_MLP_H + OR_MLP_H + \
   OR_MLP_NO * OR_MLP_H + OR_MLP_NO)
void or_mlp_forward(const double *params, const double *X, long n,
                    double *logits);
/* Loss = mean over samples of, per side h (left, right), the squared error
 * ((qhat_h - q_h) / OR_MLP_VALUE_SCALE)^2 of the reconstructed value, where
 * qhat_h = sum_k softmax(z_h)_k c_hk and q_h = sum_k Y_hk c_hk with c_hk the
 * candidates of eq. (20) on the sample's normalised stencil X[0..5] (left
 * side from X[0..4], right side from the mirror X[5..1]), plus binary
 * cross-entropy of the confidence logit against its label: C[s], or when C
 * is NULL, 1 where both |qhat_h - q_h| < OR_MLP_CONF_TOL, else 0.  Writes
 * the loss and its gradient w.r.t. params. */
#define OR_MLP_VALUE_SCALE 0.01
#define OR_MLP_CONF_TOL 0.005
double or_mlp_loss_grad(const double *params, const double *X, const double *Y,
                        const double *C, long n, double *grad);

#ifdef __cplusplus
}
#endif
#endif
