/*
 * Oracle for the WENO-IS finite-volume right-hand side of arXiv:1707.00592.
 *
 * TEST INFRASTRUCTURE ONLY: plain, slow, FP64, written from the paper for
 * checking the HIP library.  Nothing in the product may call it.
 *
 * Every function follows the paper's statement step by step; readings of
 * passages that are silent or garbled are stated where they are used.
 * Build with -ffp-contract=off so that no multiply-add is fused.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads of the OpenMP loops: set them when n > 0; returns the count in
 * force (1 in a build without OpenMP). */
int or_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Incremental-stencil WENO reconstruction, Sec. 3.3                          */
/* ------------------------------------------------------------------------ */

/* Candidate values at x_{i+1/2}, eq. (20), on v = (q_{i-2},...,q_{i+2}),
 * with the printed coefficients.  Stencils follow Fig. 1: S1 = {i,i+1},
 * S2 = {i-1,i}, S3 = {i,i+1,i+2}, S4 = {i-2,i-1,i}.  The first candidate is
 * printed with a minus sign; the sign that makes it a consistent 2-point
 * reconstruction (coefficients summing to one, and the linear combination
 * with d_k equal to the 5th-order upwind scheme) is a plus. */
void or_weno_candidates(const double v[5], double cand[4]) {
  const double a = v[0], b = v[1], c = v[2], d = v[3], e = v[4];
  cand[0] = (1.0 / 2.0) * c + (1.0 / 2.0) * d;
  cand[1] = -(1.0 / 2.0) * b + (3.0 / 2.0) * c;
  cand[2] = (1.0 / 3.0) * c + (5.0 / 6.0) * d - (1.0 / 6.0) * e;
  cand[3] = (1.0 / 3.0) * a - (7.0 / 6.0) * b + (11.0 / 6.0) * c;
}

/* Smoothness indicators beta_1..beta_4 (eq. (24)), beta_12 of the central
 * 3-point stencil {i-1,i,i+1} (Sec. 3.3.2; its printed stencil name
 * "{i-1,i,i+2}" disagrees with its formula, the formula is used) and the
 * global reference indicator tau_5 (eq. (25)).  Eq. (25) fixes tau_5's value,
 * not an order of its sums; its two bracketed sums are formed with the
 * stencil's mirror-image points paired, (e - a) - 2 (d - b) and
 * ((e + a) - 4 (d + b)) + 6 c, which keeps tau_5 exactly zero on a stencil
 * of equal values (as the exact formula is) and identical for a stencil and
 * its mirror image. */
void or_weno_indicators(const double v[5], double ind[6]) {
  const double a = v[0], b = v[1], c = v[2], d = v[3], e = v[4];
  const double k13 = 13.0 / 12.0;
  double t1, t2;
  ind[0] = (d - c) * (d - c);
  ind[1] = (c - b) * (c - b);
  t1 = c - 2.0 * d + e;
  t2 = 3.0 * c - 4.0 * d + e;
  ind[2] = k13 * t1 * t1 + 0.25 * t2 * t2;
  t1 = a - 2.0 * b + c;
  t2 = a - 4.0 * b + 3.0 * c;
  ind[3] = k13 * t1 * t1 + 0.25 * t2 * t2;
  t1 = b - 2.0 * c + d;
  t2 = b - d;
  ind[4] = k13 * t1 * t1 + 0.25 * t2 * t2;
  t1 = (e - a) - 2.0 * (d - b);
  t2 = ((e + a) - 4.0 * (d + b)) + 6.0 * c;
  ind[5] = 0.25 * t1 * t1 + k13 * t2 * t2;
}

/* Optimal weights d_k of Sec. 3.3.1. */
static const double OR_D[4] = {0.4, 0.2, 0.3, 0.1};

/* Cut-off weights (OR_W_CUTOFF), the targeted-ENO optimisation that Sec. 7
 * proposes for lower dissipation in smooth regions, applied to the
 * weights of eq. (28).  Stencil k gets the targeted-ENO smoothness measure
 *   gamma_k = (1 + r_k)^q,  q = OR_CUTOFF_Q,
 * with r_k the ratio term of eq. (28) for that stencil (the product
 * tau_5/(beta_k + eps) * tau_5/(beta_12 + eps) for the 2-point stencils,
 * tau_5/(beta_k + eps) for the 3-point ones), so that 1 + r_k =
 * alpha_k / d_k.  Its share chi_k = gamma_k / sum_s gamma_s is compared
 * with C_T = OR_CUTOFF_CT: delta_k = 1 if chi_k >= C_T, else 0, and
 *   omega_k = d_k delta_k / sum_s d_s delta_s.
 * On data smooth enough that no stencil is cut this is exactly the linear
 * 5th-order scheme; a stencil crossing a discontinuity gets weight zero.
 * (On the single ratios of eq. (21) the cut-off would inherit that form's
 * loss of order at critical points, where a 2-point indicator vanishes.)
 * Order 3 of the MOOD cascade keeps the two 2-point stencils only (as
 * d3 = d4 = 0 does for the other forms) and cuts among them.  Evaluation:
 * gamma_k overflows for the pressure-like fields, so each 1 + r_k is first
 * divided by the largest of them, t_k = g_k / g_max, and chi_k >= C_T is
 * tested as t_k^6 >= C_T sum_s t_s^6 (the same inequality multiplied by
 * g_max^-6), with t^6 formed as (t^2 t^2) t^2 and the sum in stencil order.
 * The optimal weights are taken as 4, 2, 3, 1 over their kept sum (exact
 * integers), so that an uncut stencil set gives omega_k = d_k to the last
 * bit. */
static void cutoff_weights(const double ind[6], double eps, int order,
                           double omega[4]) {
  static const double dint[4] = {4.0, 2.0, 3.0, 1.0};
  const int ns = order == 3 ? 2 : 4;
  const double tau5 = ind[5];
  double g[4], p[4], gmax, psum, dsum;
  int k, keep[4];
  const double r12 = tau5 / (ind[4] + eps);
  g[0] = 1.0 + (tau5 / (ind[0] + eps)) * r12;
  g[1] = 1.0 + (tau5 / (ind[1] + eps)) * r12;
  g[2] = 1.0 + tau5 / (ind[2] + eps);
  g[3] = 1.0 + tau5 / (ind[3] + eps);
  gmax = g[0];
  for (k = 1; k < ns; k++)
    if (g[k] > gmax) gmax = g[k];
  psum = 0.0;
  for (k = 0; k < ns; k++) {
    const double t = g[k] / gmax;
    const double t2 = t * t;
    p[k] = (t2 * t2) * t2;
    psum += p[k];
  }
  dsum = 0.0;
  for (k = 0; k < 4; k++) {
    keep[k] = k < ns && p[k] >= OR_CUTOFF_CT * psum;
    if (keep[k]) dsum += dint[k];
  }
  for (k = 0; k < 4; k++) omega[k] = keep[k] ? dint[k] / dsum : 0.0;
}

/* Nonlinear weights.  Basic form: eq. (21) with q = 1.  Modified form:
 * eq. (28), where each alpha line carries its own d_k (the printed "d_k"
 * on every line is read as d_1..d_4 in turn).  Cut-off form: above.  Order 3 sets d3 = d4 = 0
 * (end of Sec. 3.3.1), i.e. only the two 2-point stencils remain. */
void or_weno_weights(const double v[5], int weights, double eps, int order,
                     double omega[4]) {
  double ind[6], alpha[4], sum;
  int k;
  or_weno_indicators(v, ind);
  const double tau5 = ind[5];
  if (weights == OR_W_CUTOFF) {
    cutoff_weights(ind, eps, order, omega);
    return;
  }
  if (weights == OR_W_BASIC) {
    for (k = 0; k < 4; k++) alpha[k] = OR_D[k] * (1.0 + tau5 / (ind[k] + eps));
  } else {
    const double r12 = tau5 / (ind[4] + eps);
    alpha[0] = OR_D[0] * (1.0 + (tau5 / (ind[0] + eps)) * r12);
    alpha[1] = OR_D[1] * (1.0 + (tau5 / (ind[1] + eps)) * r12);
    alpha[2] = OR_D[2] * (1.0 + tau5 / (ind[2] + eps));
    alpha[3] = OR_D[3] * (1.0 + tau5 / (ind[3] + eps));
  }
  if (order == 3) {
    alpha[2] = 0.0;
    alpha[3] = 0.0;
  }
  sum = 0.0;
  for (k = 0; k < 4; k++) sum += alpha[k];
  for (k = 0; k < 4; k++) omega[k] = alpha[k] / sum;
}

/* Eq. (19): weighted average of the candidate values. */
double or_weno_is(const double v[5], int weights, double eps, int order) {
  double cand[4], omega[4], q = 0.0;
  int k;
  or_weno_candidates(v, cand);
  or_weno_weights(v, weights, eps, order, omega);
  for (k = 0; k < 4; k++) q += omega[k] * cand[k];
  return q;
}

/* ------------------------------------------------------------------------ */
/* Equation of state and characteristic decomposition, Secs. 2 and 3.2       */
/* ------------------------------------------------------------------------ */

/* Index helpers for a face-order primitive vector with nt transverse
 * velocities: rho, u_n, u_t[nt], p, Gamma, Pi. */
#define IP(nt) (2 + (nt))
#define IG(nt) (3 + (nt))
#define IPI(nt) (4 + (nt))

/* Squared sound speed of the stiffened gas, c^2 = gamma (p + Pinf) / rho,
 * rewritten with Gamma = 1/(gamma-1) and Pi = gamma Pinf/(gamma-1) (eq. (2)):
 * c^2 = ((Gamma + 1) p + Pi) / (Gamma rho).  It is the entry rho c^2 of A
 * in eq. (9) divided by rho. */
static double sound2(double rho, double p, double G, double P) {
  return ((G + 1.0) * p + P) / (G * rho);
}

/* L and R of eq. (11) at the face state qbar.  The eigenvalue symbol "a"
 * of eq. (10) is the sound speed c of eq. (11).  Extended to nt transverse
 * velocities, each an identity row/column like v in eq. (11). */
void or_eigen(int nt, const double qbar[], double *L, double *R) {
  const int nc = 5 + nt;
  const double rho = qbar[0];
  const double c2 = sound2(rho, qbar[IP(nt)], qbar[IG(nt)], qbar[IPI(nt)]);
  const double c = sqrt(c2);
  int i, t;
  for (i = 0; i < nc * nc; i++) {
    L[i] = 0.0;
    R[i] = 0.0;
  }
  /* rows of L */
  L[0 * nc + 1] = -rho * c / 2.0;
  L[0 * nc + IP(nt)] = 1.0 / 2.0;
  L[1 * nc + 0] = 1.0;
  L[1 * nc + IP(nt)] = -1.0 / c2;
  for (t = 0; t < nt; t++) L[(2 + t) * nc + 2 + t] = 1.0;
  L[(2 + nt) * nc + IG(nt)] = 1.0;
  L[(3 + nt) * nc + IPI(nt)] = 1.0;
  L[(4 + nt) * nc + 1] = rho * c / 2.0;
  L[(4 + nt) * nc + IP(nt)] = 1.0 / 2.0;
  /* columns of R */
  R[0 * nc + 0] = 1.0 / c2;
  R[0 * nc + 1] = 1.0;
  R[0 * nc + (4 + nt)] = 1.0 / c2;
  R[1 * nc + 0] = -1.0 / (rho * c);
  R[1 * nc + (4 + nt)] = 1.0 / (rho * c);
  for (t = 0; t < nt; t++) R[(2 + t) * nc + 2 + t] = 1.0;
  R[IP(nt) * nc + 0] = 1.0;
  R[IP(nt) * nc + (4 + nt)] = 1.0;
  R[IG(nt) * nc + (2 + nt)] = 1.0;
  R[IPI(nt) * nc + (3 + nt)] = 1.0;
}

/* y = M x for an nc x nc row-major matrix, summed in column order. */
static void matvec(int nc, const double *M, const double *x, double *y) {
  int i, k;
  for (i = 0; i < nc; i++) {
    double s = 0.0;
    for (k = 0; k < nc; k++) s += M[i * nc + k] * x[k];
    y[i] = s;
  }
}

/* MOOD positivity test, Sec. 3.4.  The text asks for rho > 0 and
 * p + gamma Pinf >= 0 and, for the HLLC wave speeds, non-negative
 * quantities under the square roots.  Read as: rho > 0, Gamma > 0 (material
 * property in range) and c^2 > 0, i.e. (Gamma+1) p + Pi > 0, which implies
 * p + gamma Pinf > 0 and keeps every square root of Sec. 3.2.1 real. */
int or_pos(int nt, const double q[]) {
  const double rho = q[0], p = q[IP(nt)], G = q[IG(nt)], P = q[IPI(nt)];
  return (rho > 0.0) && (G > 0.0) && ((G + 1.0) * p + P > 0.0);
}

/* ------------------------------------------------------------------------ */
/* HLLC Riemann solver, Sec. 3.2.1                                            */
/* ------------------------------------------------------------------------ */

static double sgn(double x) { return x > 0.0 ? 1.0 : (x < 0.0 ? -1.0 : 0.0); }
static double mn(double a, double b) { return a < b ? a : b; }
static double mx(double a, double b) { return a > b ? a : b; }

/* Conservative vector U_k and physical flux F_k of one face state (face
 * order: rho, rho u_n, rho u_t..., E, Gamma, Pi).  The material rows carry
 * Gamma u_n and Pi u_n, the flux part of eq. (3). */
static void cons_flux(int nt, const double q[], double U[], double F[]) {
  const double rho = q[0], un = q[1], p = q[IP(nt)], G = q[IG(nt)],
               P = q[IPI(nt)];
  double ke = un * un;
  int t;
  for (t = 0; t < nt; t++) ke += q[2 + t] * q[2 + t];
  const double E = G * p + P + 0.5 * rho * ke;
  U[0] = rho;
  U[1] = rho * un;
  for (t = 0; t < nt; t++) U[2 + t] = rho * q[2 + t];
  U[2 + nt] = E;
  U[3 + nt] = G;
  U[4 + nt] = P;
  F[0] = rho * un;
  F[1] = rho * un * un + p;
  for (t = 0; t < nt; t++) F[2 + t] = rho * un * q[2 + t];
  F[2 + nt] = (E + p) * un;
  F[3 + nt] = G * un;
  F[4 + nt] = P * un;
}

/* Eqs. (14)-(18).  Readings: the averaged velocity and sound speed of
 * eq. (17) carry two index typos; they are read as the Roe-type average
 * (sqrt(rho_l) u_l + sqrt(rho_r) u_r)/(sqrt(rho_l)+sqrt(rho_r)) and the
 * Einfeldt-type average with sqrt(rho_r) c_r^2 in the second term.
 * sign(0) = 0.  When S_k equals S* (possible only once S_k has been clipped
 * to zero) the star flux of that side is taken as its limit F_k and the
 * star velocity as u_k. */
void or_hllc(int nt, const double ql[], const double qr[], double F[],
             double *ustar) {
  const int nc = 5 + nt;
  double Ul[OR_MAXNC], Ur[OR_MAXNC], Fl[OR_MAXNC], Fr[OR_MAXNC];
  double Fsl[OR_MAXNC], Fsr[OR_MAXNC], D[OR_MAXNC];
  const double rl = ql[0], ul = ql[1], pl = ql[IP(nt)];
  const double rr = qr[0], ur = qr[1], pr = qr[IP(nt)];
  const double cl2 = sound2(rl, pl, ql[IG(nt)], ql[IPI(nt)]);
  const double cr2 = sound2(rr, pr, qr[IG(nt)], qr[IPI(nt)]);
  const double cl = sqrt(cl2), cr = sqrt(cr2);
  const double sl = sqrt(rl), sr = sqrt(rr);
  const double ubar = (sl * ul + sr * ur) / (sl + sr);
  const double cbar2 = (sl * cl2 + sr * cr2) / (sl + sr) +
                       0.5 * sl * sr / ((sl + sr) * (sl + sr)) * (ur - ul) *
                           (ur - ul);
  const double cbar = sqrt(cbar2);
  const double Sls = mn(ubar - cbar, ul - cl);
  const double Srs = mx(ubar + cbar, ur + cr);
  const double Sl = mn(Sls, 0.0);
  const double Sr = mx(Srs, 0.0);
  const double Ss = (pr - pl + rl * ul * (Sl - ul) - rr * ur * (Sr - ur)) /
                    (rl * (Sl - ul) - rr * (Sr - ur));
  double usl, usr;
  int k;
  cons_flux(nt, ql, Ul, Fl);
  cons_flux(nt, qr, Ur, Fr);
  for (k = 0; k < nc; k++) D[k] = 0.0;
  D[1] = 1.0;
  D[2 + nt] = Ss;
  if (Sl - Ss == 0.0) {
    for (k = 0; k < nc; k++) Fsl[k] = Fl[k];
    usl = ul;
  } else {
    const double pk = pl + rl * (Sl - ul) * (Ss - ul);
    for (k = 0; k < nc; k++)
      Fsl[k] = (Ss * (Sl * Ul[k] - Fl[k]) + Sl * pk * D[k]) / (Sl - Ss);
    usl = Ss * (Sl - ul) / (Sl - Ss);
  }
  if (Sr - Ss == 0.0) {
    for (k = 0; k < nc; k++) Fsr[k] = Fr[k];
    usr = ur;
  } else {
    const double pk = pr + rr * (Sr - ur) * (Ss - ur);
    for (k = 0; k < nc; k++)
      Fsr[k] = (Ss * (Sr * Ur[k] - Fr[k]) + Sr * pk * D[k]) / (Sr - Ss);
    usr = Ss * (Sr - ur) / (Sr - Ss);
  }
  const double s = sgn(Ss);
  const double wl = (1.0 + s) / 2.0, wr = (1.0 - s) / 2.0;
  for (k = 0; k < nc; k++) F[k] = wl * Fsl[k] + wr * Fsr[k];
  *ustar = wl * usl + wr * usr;
}

/* ------------------------------------------------------------------------ */
/* One face: projection, reconstruction, MOOD cascade, flux (Secs. 3.2-3.4)  */
/* ------------------------------------------------------------------------ */

/* Reconstruct both face states at a given order from the characteristic
 * values w (6 cells x nc).  Left uses q~_{i-2..i+2}; the right state is the
 * mirror image about the face, q~_{i+3..i-1} in the roles of i-2..i+2
 * (the paper writes out the left state only). */
static void recon_side(int nc, const double *w, const or_opts *o, int order,
                       int side, double *wt) {
  int m, j;
  for (m = 0; m < nc; m++) {
    double v[5];
    for (j = 0; j < 5; j++)
      v[j] = (side == 0) ? w[j * nc + m] : w[(5 - j) * nc + m];
    wt[m] = or_weno_is(v, o->weights, o->eps, order);
  }
}

void or_face(int nt, const double q6[], const or_opts *o, double ql[],
             double qr[], int order_lr[2], double F[], double *ustar) {
  const int nc = 5 + nt;
  double qbar[OR_MAXNC], L[OR_MAXNC * OR_MAXNC], R[OR_MAXNC * OR_MAXNC];
  double w[6 * OR_MAXNC], wt[OR_MAXNC];
  int k, j, side;
  /* The face matrices: L_{i+1/2} "an average between L_i and L_{i+1}"
   * (Sec. 3.2) is read as L evaluated at the arithmetic mean of the two
   * primitive states; R is its exact inverse at the same state. */
  for (k = 0; k < nc; k++) qbar[k] = 0.5 * (q6[2 * nc + k] + q6[3 * nc + k]);
  or_eigen(nt, qbar, L, R);
  /* Eq. (12) on the six cells i-2..i+3 (the printed range
   * i+r > j > i+1-r with r = 3 is read with non-strict bounds). */
  for (j = 0; j < 6; j++) matvec(nc, L, q6 + j * nc, w + j * nc);
  for (side = 0; side < 2; side++) {
    double *q = (side == 0) ? ql : qr;
    /* 5th order, back-projected by eq. (13). */
    recon_side(nc, w, o, 5, side, wt);
    matvec(nc, R, wt, q);
    order_lr[side] = 5;
    if (o->mood && !or_pos(nt, q)) {
      /* Sec. 3.4: redo without the two 3-point stencils. */
      recon_side(nc, w, o, 3, side, wt);
      matvec(nc, R, wt, q);
      order_lr[side] = 3;
      if (!or_pos(nt, q)) {
        /* Eq. (32): first-order upwind, q~ = q~_i (left) or q~_{i+1}
         * (right).  R L q_i = q_i, so the cell's primitive state is used
         * directly. */
        const double *qc = q6 + (side == 0 ? 2 : 3) * nc;
        for (k = 0; k < nc; k++) q[k] = qc[k];
        order_lr[side] = 1;
      }
    }
  }
  or_hllc(nt, ql, qr, F, ustar);
}

/* ------------------------------------------------------------------------ */
/* Semi-discrete operator, Sec. 3.1                                          */
/* ------------------------------------------------------------------------ */

static long ncells(const or_grid *g) {
  long n = 1;
  int d;
  for (d = 0; d < g->ndim; d++) n *= g->n[d];
  return n;
}

static int check_grid(const or_grid *g) {
  int d;
  if (!g || g->ndim < 1 || g->ndim > 3) return 0;
  for (d = 0; d < g->ndim; d++) {
    if (g->n[d] < 1 || !(g->dx[d] > 0.0)) return 0;
    if (g->bc_lo[d] < 0 || g->bc_lo[d] > 2 || g->bc_hi[d] < 0 ||
        g->bc_hi[d] > 2)
      return 0;
    if ((g->bc_lo[d] == OR_BC_REFLECTIVE || g->bc_hi[d] == OR_BC_REFLECTIVE) &&
        g->n[d] < 3)
      return 0;
  }
  return 1;
}

/* Primitive state of cell `cell` in face order for direction d.  Recovery
 * of p from E through eq. (2): E = Gamma p + Pi + rho |u|^2 / 2. */
static void cell_prim(int ndim, long ncell, const double *U, long cell, int d,
                      double *q) {
  const int nt = ndim - 1;
  const double rho = U[cell];
  double vel[3], ke = 0.0;
  int a, t;
  for (a = 0; a < ndim; a++) vel[a] = U[(1 + a) * ncell + cell] / rho;
  for (a = 0; a < ndim; a++) ke += vel[a] * vel[a];
  const double E = U[(1 + ndim) * ncell + cell];
  const double G = U[(2 + ndim) * ncell + cell];
  const double P = U[(3 + ndim) * ncell + cell];
  q[0] = rho;
  q[1] = vel[d];
  t = 0;
  for (a = 0; a < ndim; a++)
    if (a != d) q[2 + t++] = vel[a];
  q[IP(nt)] = (E - 0.5 * rho * ke - P) / G;
  q[IG(nt)] = G;
  q[IPI(nt)] = P;
}

/* Index of the interior cell that ghost/interior position l (-3..n+2) of a
 * line maps to, and whether its normal velocity is mirrored. */
static long bc_map(long l, long n, int bclo, int bchi, int *flip) {
  *flip = 0;
  if (l < 0) {
    if (bclo == OR_BC_PERIODIC) return ((l % n) + n) % n;
    if (bclo == OR_BC_REFLECTIVE) {
      *flip = 1;
      return -l - 1;
    }
    return 0;
  }
  if (l >= n) {
    if (bchi == OR_BC_PERIODIC) return l % n;
    if (bchi == OR_BC_REFLECTIVE) {
      *flip = 1;
      return 2 * n - 1 - l;
    }
    return n - 1;
  }
  return l;
}

/* Physical-state test on a cell (used on the input of every evaluation). */
static int cell_ok(int ndim, long ncell, const double *U, long cell) {
  const int nc = 4 + ndim;
  double q[OR_MAXNC];
  int k;
  for (k = 0; k < nc; k++)
    if (!isfinite(U[k * ncell + cell])) return 0;
  cell_prim(ndim, ncell, U, cell, 0, q);
  return or_pos(ndim - 1, q);
}

/* Map from face-order component k (direction d) to the conservative
 * component index. */
static int face_to_cons(int ndim, int d, int k) {
  const int nt = ndim - 1;
  if (k == 0) return 0;
  if (k == 1) return 1 + d;
  if (k < 2 + nt) {
    int t = k - 2, a, c = 0;
    for (a = 0; a < ndim; a++) {
      if (a == d) continue;
      if (c == t) return 1 + a;
      c++;
    }
  }
  return k; /* E, Gamma, Pi keep their slots */
}

/* One direction's contribution to dU/dt along one grid line.
 * Eq. (5): -(F_{i+1/2} - F_{i-1/2}) / dx for rho, momenta, E.
 * Eq. (6): -(H_{i+1/2} - H_{i-1/2}) / dx + phi_i (u_{i+1/2} - u_{i-1/2}) / dx
 * for Gamma and Pi, with H the material rows of the HLLC flux and
 * u_{i+1/2} = u^HLLC of eq. (18). */
static void line_rhs(const or_grid *g, const or_opts *o, const double *U,
                     double *dUdt, int d, long base, long stride,
                     long *o3, long *o1) {
  const int ndim = g->ndim, nt = ndim - 1, nc = 5 + nt;
  const long n = g->n[d], ncell = ncells(g);
  const double dx = g->dx[d];
  double *ext = (double *)malloc(sizeof(double) * (size_t)(n + 6) * nc);
  double *F = (double *)malloc(sizeof(double) * (size_t)(n + 1) * nc);
  double *us = (double *)malloc(sizeof(double) * (size_t)(n + 1));
  long l, i, f;
  int k;
  for (l = -3; l < n + 3; l++) {
    int flip;
    const long c = bc_map(l, n, g->bc_lo[d], g->bc_hi[d], &flip);
    double *q = ext + (l + 3) * nc;
    cell_prim(ndim, ncell, U, base + c * stride, d, q);
    if (flip) q[1] = -q[1];
  }
  for (f = 0; f <= n; f++) {
    double ql[OR_MAXNC], qr[OR_MAXNC];
    int ord[2];
    or_face(nt, ext + f * nc, o, ql, qr, ord, F + f * nc, us + f);
    if (ord[0] == 3) (*o3)++;
    if (ord[0] == 1) (*o1)++;
    if (ord[1] == 3) (*o3)++;
    if (ord[1] == 1) (*o1)++;
  }
  for (i = 0; i < n; i++) {
    const long cell = base + i * stride;
    for (k = 0; k < nc; k++) {
      const int kc = face_to_cons(ndim, d, k);
      double r = -(F[(i + 1) * nc + k] - F[i * nc + k]) / dx;
      if (k >= 3 + nt) {
        const double phi = U[kc * ncell + cell];
        r = r + phi * (us[i + 1] - us[i]) / dx;
      }
      if (d == 0)
        dUdt[kc * ncell + cell] = r;
      else
        dUdt[kc * ncell + cell] = dUdt[kc * ncell + cell] + r;
    }
  }
  free(ext);
  free(F);
  free(us);
}

int or_rhs(const or_grid *g, const or_opts *o, const double *U, double *dUdt,
           or_stats *st) {
  if (!check_grid(g) || !o || !U || !dUdt) return OR_ERR_ARG;
  const long ncell = ncells(g);
  int status = OR_OK, d;
  long c;
  for (c = 0; c < ncell; c++)
    if (!cell_ok(g->ndim, ncell, U, c)) status = OR_ERR_NONPHYSICAL;
  /* Dimension by dimension: x, then y, then z contributions are summed in
   * that order. */
  for (d = 0; d < g->ndim; d++) {
    long stride = 1, nlines, line;
    int a;
    for (a = 0; a < d; a++) stride *= g->n[a];
    nlines = ncell / g->n[d];
    long o3 = 0, o1 = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : o3, o1)
    for (line = 0; line < nlines; line++) {
      /* line enumerates all cells whose index along d is 0 */
      const long lo = line % stride, hi = line / stride;
      const long base = lo + hi * stride * g->n[d];
      line_rhs(g, o, U, dUdt, d, base, stride, &o3, &o1);
    }
    if (st) {
      st->o3[d] += o3;
      st->o1[d] += o1;
    }
  }
  if (st && status != OR_OK) st->status = status;
  return status;
}

int or_cfl_dt(const or_grid *g, const or_opts *o, const double *U,
              double *dt) {
  if (!check_grid(g) || !o || !U || !dt || !(o->cfl > 0.0)) return OR_ERR_ARG;
  const long ncell = ncells(g);
  const int ndim = g->ndim, nt = ndim - 1;
  double m = 0.0;
  long c;
  for (c = 0; c < ncell; c++) {
    double q[OR_MAXNC], vel[3], s = 0.0;
    int a;
    cell_prim(ndim, ncell, U, c, 0, q);
    const double cs = sqrt(sound2(q[0], q[IP(nt)], q[IG(nt)], q[IPI(nt)]));
    for (a = 0; a < ndim; a++) vel[a] = U[(1 + a) * ncell + c] / q[0];
    for (a = 0; a < ndim; a++) s += (fabs(vel[a]) + cs) / g->dx[a];
    if (s > m) m = s;
  }
  *dt = o->cfl / m;
  return OR_OK;
}

/* Third-order TVD Runge-Kutta (cited in Sec. 3.1), Shu-Osher form:
 *   U1 = U0 + dt L(U0)
 *   U2 = 3/4 U0 + 1/4 (U1 + dt L(U1))
 *   U3 = 1/3 U0 + 2/3 (U2 + dt L(U2)) */
int or_rk3_step(const or_grid *g, const or_opts *o, double *U, double dt,
                or_stats *st) {
  if (!check_grid(g) || !o || !U) return OR_ERR_ARG;
  const long n = ncells(g) * (4 + g->ndim);
  double *U0 = (double *)malloc(sizeof(double) * (size_t)n);
  double *U1 = (double *)malloc(sizeof(double) * (size_t)n);
  double *U2 = (double *)malloc(sizeof(double) * (size_t)n);
  double *Lu = (double *)malloc(sizeof(double) * (size_t)n);
  int status = OR_OK, s;
  long i;
  memcpy(U0, U, sizeof(double) * (size_t)n);
  s = or_rhs(g, o, U0, Lu, st);
  if (s != OR_OK) status = s;
  for (i = 0; i < n; i++) U1[i] = U0[i] + dt * Lu[i];
  s = or_rhs(g, o, U1, Lu, st);
  if (s != OR_OK) status = s;
  for (i = 0; i < n; i++) U2[i] = 0.75 * U0[i] + 0.25 * (U1[i] + dt * Lu[i]);
  s = or_rhs(g, o, U2, Lu, st);
  if (s != OR_OK) status = s;
  for (i = 0; i < n; i++)
    U[i] = (1.0 / 3.0) * U0[i] + (2.0 / 3.0) * (U2[i] + dt * Lu[i]);
  free(U0);
  free(U1);
  free(U2);
  free(Lu);
  return status;
}

/* Independent 1D problems stored back to back (each run with its own grid
 * spacing and time step).  A problem stops after the step in which its
 * status became non-OK; pstatus (may be NULL) holds the per-problem status
 * on entry (problems not OK are skipped) and on exit. */
int or_batch_step(int nprob, const long *offsets, const double *dx, int bc_lo,
                  int bc_hi, const or_opts *o, double *U, double *dt,
                  int nsteps, or_stats *st, int *pstatus) {
  if (nprob < 1 || !offsets || !dx || !o || !U || !dt || nsteps < 0)
    return OR_ERR_ARG;
  const long total = offsets[nprob];
  int status = OR_OK, p;
  long o3 = 0, o1 = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : o3, o1)
  for (p = 0; p < nprob; p++) {
    const long n = offsets[p + 1] - offsets[p];
    or_grid g;
    or_stats ls;
    double *Up = (double *)malloc(sizeof(double) * (size_t)(5 * n));
    int c, step, s = pstatus ? pstatus[p] : OR_OK;
    long i;
    memset(&g, 0, sizeof(g));
    memset(&ls, 0, sizeof(ls));
    g.ndim = 1;
    g.n[0] = n;
    g.n[1] = g.n[2] = 1;
    g.dx[0] = dx[p];
    g.dx[1] = g.dx[2] = 1.0;
    g.bc_lo[0] = bc_lo;
    g.bc_hi[0] = bc_hi;
    for (c = 0; c < 5; c++)
      for (i = 0; i < n; i++) Up[c * n + i] = U[c * total + offsets[p] + i];
    for (step = 0; step < nsteps && s == OR_OK; step++) {
      if (o->cfl > 0.0) s = or_cfl_dt(&g, o, Up, &dt[p]);
      if (s == OR_OK) s = or_rk3_step(&g, o, Up, dt[p], &ls);
    }
    for (c = 0; c < 5; c++)
      for (i = 0; i < n; i++) U[c * total + offsets[p] + i] = Up[c * n + i];
    o3 += ls.o3[0];
    o1 += ls.o1[0];
    if (pstatus) pstatus[p] = s;
    if (s != OR_OK) {
#pragma omp critical
      status = s;
    }
    free(Up);
  }
  if (st) {
    st->o3[0] += o3;
    st->o1[0] += o1;
    if (status != OR_OK) st->status = status;
  }
  return status;
}
