/*
 * Exact solution of the 1D Riemann problem for two stiffened gases.
 *
 * TEST INFRASTRUCTURE ONLY (verification of the finite-volume solution of
 * the gas-liquid shock tube of Sec. 5.2 and of the batched shock tubes).
 *
 * Method: the textbook exact Riemann solver for the ideal gas (Toro,
 * "Riemann Solvers and Numerical Methods for Fluid Dynamics", ch. 4) applied
 * to the shifted pressure pbar = p + Pinf of each material.  With
 * rho e = (p + gamma Pinf)/(gamma-1) (eq. (2)) the Hugoniot and isentrope of
 * a stiffened gas are those of an ideal gas in pbar, so each side's wave
 * curve is the ideal-gas one in its own pbar.  The star pressure is found by
 * bisection on the monotone pressure function, which is slow and robust.
 */
#include <math.h>

#include "oracle.h"

typedef struct {
  double rho, u, p, g, pinf;
} sg_state;

static sg_state unpack(const double W[5]) {
  sg_state s;
  s.rho = W[0];
  s.u = W[1];
  s.p = W[2];
  s.g = W[3];
  s.pinf = W[4];
  return s;
}

static double sound(const sg_state *K) {
  return sqrt(K->g * (K->p + K->pinf) / K->rho);
}

/* Velocity change across the left- or right-facing wave connecting state K
 * to pressure ps (Toro eqs. 4.6-4.7 in pbar). */
static double wave_f(double ps, const sg_state *K) {
  const double pb = K->p + K->pinf, psb = ps + K->pinf;
  if (ps > K->p) {
    const double A = 2.0 / ((K->g + 1.0) * K->rho);
    const double B = (K->g - 1.0) / (K->g + 1.0) * pb;
    return (ps - K->p) * sqrt(A / (psb + B));
  }
  return 2.0 * sound(K) / (K->g - 1.0) *
         (pow(psb / pb, (K->g - 1.0) / (2.0 * K->g)) - 1.0);
}

int or_exact_star(const double WL[5], const double WR[5], double *pstar,
                  double *ustar) {
  const sg_state L = unpack(WL), R = unpack(WR);
  const double du = R.u - L.u;
  /* Admissible pressures keep pbar >= 0 on both sides. */
  const double plo = -(L.pinf < R.pinf ? L.pinf : R.pinf);
  double lo = plo, hi, flo, fhi;
  int it;
  flo = wave_f(lo, &L) + wave_f(lo, &R) + du;
  if (flo > 0.0) return OR_ERR_VACUUM; /* the two rarefactions open a cavity */
  hi = (L.p > R.p ? L.p : R.p) + (L.pinf > R.pinf ? L.pinf : R.pinf) + 1.0;
  fhi = wave_f(hi, &L) + wave_f(hi, &R) + du;
  while (fhi < 0.0) {
    hi = 2.0 * hi + 1.0;
    fhi = wave_f(hi, &L) + wave_f(hi, &R) + du;
  }
  for (it = 0; it < 400; it++) {
    const double mid = 0.5 * (lo + hi);
    if (mid == lo || mid == hi) break;
    const double fm = wave_f(mid, &L) + wave_f(mid, &R) + du;
    if (fm > 0.0)
      hi = mid;
    else
      lo = mid;
  }
  *pstar = 0.5 * (lo + hi);
  *ustar = 0.5 * (L.u + R.u) + 0.5 * (wave_f(*pstar, &R) - wave_f(*pstar, &L));
  return OR_OK;
}

/* State at similarity coordinate xi = x/t (Toro sec. 4.5), returned as
 * (rho, u, p, gamma, Pinf). */
void or_exact_sample(const double WL[5], const double WR[5], double pstar,
                     double ustar, double xi, double W[5]) {
  const sg_state L = unpack(WL), R = unpack(WR);
  if (xi <= ustar) {
    const sg_state *K = &L;
    const double g = K->g, pb = K->p + K->pinf, psb = pstar + K->pinf;
    const double c = sound(K);
    W[3] = g;
    W[4] = K->pinf;
    if (pstar > K->p) {
      const double S =
          K->u - c * sqrt((g + 1.0) / (2.0 * g) * psb / pb + (g - 1.0) / (2.0 * g));
      if (xi <= S) {
        W[0] = K->rho;
        W[1] = K->u;
        W[2] = K->p;
      } else {
        const double gr = (g - 1.0) / (g + 1.0);
        W[0] = K->rho * (psb / pb + gr) / (gr * psb / pb + 1.0);
        W[1] = ustar;
        W[2] = pstar;
      }
    } else {
      const double sh = K->u - c;
      const double cs = c * pow(psb / pb, (g - 1.0) / (2.0 * g));
      const double st = ustar - cs;
      if (xi <= sh) {
        W[0] = K->rho;
        W[1] = K->u;
        W[2] = K->p;
      } else if (xi > st) {
        W[0] = K->rho * pow(psb / pb, 1.0 / g);
        W[1] = ustar;
        W[2] = pstar;
      } else {
        const double cf = 2.0 / (g + 1.0) * (c + (g - 1.0) / 2.0 * (K->u - xi));
        W[0] = K->rho * pow(cf / c, 2.0 / (g - 1.0));
        W[1] = 2.0 / (g + 1.0) * (c + (g - 1.0) / 2.0 * K->u + xi);
        W[2] = pb * pow(cf / c, 2.0 * g / (g - 1.0)) - K->pinf;
      }
    }
  } else {
    const sg_state *K = &R;
    const double g = K->g, pb = K->p + K->pinf, psb = pstar + K->pinf;
    const double c = sound(K);
    W[3] = g;
    W[4] = K->pinf;
    if (pstar > K->p) {
      const double S =
          K->u + c * sqrt((g + 1.0) / (2.0 * g) * psb / pb + (g - 1.0) / (2.0 * g));
      if (xi >= S) {
        W[0] = K->rho;
        W[1] = K->u;
        W[2] = K->p;
      } else {
        const double gr = (g - 1.0) / (g + 1.0);
        W[0] = K->rho * (psb / pb + gr) / (gr * psb / pb + 1.0);
        W[1] = ustar;
        W[2] = pstar;
      }
    } else {
      const double sh = K->u + c;
      const double cs = c * pow(psb / pb, (g - 1.0) / (2.0 * g));
      const double st = ustar + cs;
      if (xi >= sh) {
        W[0] = K->rho;
        W[1] = K->u;
        W[2] = K->p;
      } else if (xi < st) {
        W[0] = K->rho * pow(psb / pb, 1.0 / g);
        W[1] = ustar;
        W[2] = pstar;
      } else {
        const double cf = 2.0 / (g + 1.0) * (c - (g - 1.0) / 2.0 * (K->u - xi));
        W[0] = K->rho * pow(cf / c, 2.0 / (g - 1.0));
        W[1] = 2.0 / (g + 1.0) * (-c + (g - 1.0) / 2.0 * K->u + xi);
        W[2] = pb * pow(cf / c, 2.0 * g / (g - 1.0)) - K->pinf;
      }
    }
  }
}

/* The same at n similarity coordinates xi[i]; W is n x 5, row-major. */
void or_exact_sample_n(const double WL[5], const double WR[5], double pstar,
                       double ustar, const double *xi, long n, double *W) {
  long i;
  for (i = 0; i < n; i++) or_exact_sample(WL, WR, pstar, ustar, xi[i], W + 5 * i);
}
