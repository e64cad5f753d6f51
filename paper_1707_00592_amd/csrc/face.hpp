// Face-level device arithmetic of the WENO-IS finite-volume method
// (arXiv:1707.00592): characteristic projection (Sec. 3.2, eqs. (11)-(13)),
// WENO-IS reconstruction (Sec. 3.3, eqs. (19)-(29)), MOOD-type positivity
// cascade (Sec. 3.4, eq. (32)) and the HLLC flux (Sec. 3.2.1,
// eqs. (14)-(18)).
//
// Precision: the template type T is the arithmetic of the projection,
// reconstruction and flux (double, or float for the mixed form).  The
// back-projected face states and their positivity test are always double.
// With T = double every operation is written in one fixed order (no fused
// multiply-add; the library is compiled with -ffp-contract=off), so results
// are reproducible bit for bit between launches and tile shapes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace isw {

// Optimal weights d_k of Sec. 3.3.1 and the 13/12 of the indicators.
#define ISW_D1 0.4
#define ISW_D2 0.2
#define ISW_D3 0.3
#define ISW_D4 0.1
#define ISW_K13 (13.0 / 12.0)

enum { W_MODIFIED = 0, W_BASIC = 1, W_MLP = 2, W_CUTOFF = 3 };

// Cut-off weights: the targeted-ENO threshold C_T of the 5th-order scheme.
#define ISW_CT 1e-5

template <typename T>
__device__ __forceinline__ T dmin(T a, T b) { return a < b ? a : b; }
template <typename T>
__device__ __forceinline__ T dmax(T a, T b) { return a > b ? a : b; }

// c^2 = gamma (p + Pinf) / rho of the stiffened gas (eq. (2)) in terms of
// Gamma = 1/(gamma-1) and Pi = gamma Pinf/(gamma-1).
// Quotient in the arithmetic of T: the IEEE division for double (the FP64
// path reproduces the oracle's rounding); for the float form, x times the
// hardware reciprocal (within about 1 ulp), whose results are bounded, not
// exact.  Zero and infinite divisors give the same infinities and NaNs.
template <typename T>
__device__ __forceinline__ T qdiv(T x, T y);
template <>
__device__ __forceinline__ double qdiv<double>(double x, double y) {
  return x / y;
}
template <>
__device__ __forceinline__ float qdiv<float>(float x, float y) {
  return x * __builtin_amdgcn_rcpf(y);
}

template <typename T>
__device__ __forceinline__ T sound2(T rho, T p, T G, T P) {
  return qdiv<T>((G + T(1)) * p + P, G * rho);
}

// Admissibility used by the MOOD cascade: rho > 0, Gamma > 0 and
// (Gamma+1) p + Pi > 0 (c^2 > 0, so every square root of the HLLC solver is
// real and p + gamma Pinf > 0).
__device__ __forceinline__ bool admissible(double rho, double p, double G,
                                           double P) {
  return (rho > 0.0) && (G > 0.0) && ((G + 1.0) * p + P > 0.0);
}

// ---------------------------------------------------------------------------
// WENO-IS on the left-biased stencil (a, b, c, d, e) = q~_{i-2..i+2}.
// ---------------------------------------------------------------------------

// Indicators of eqs. (24), (25) and the central beta_12 of Sec. 3.3.2.
template <typename T>
struct Ind {
  T b1, b2, b3, b4, b12, tau;
};

// The global reference indicator tau5 of eq. (25), its bracketed sums
// formed with the mirror-image points paired: exactly zero on a stencil of
// equal values and the same for a stencil and its mirror image.
template <typename T>
__device__ __forceinline__ T tau5(T a, T b, T c, T d, T e) {
  const T k13 = T(ISW_K13);
  const T t1 = (e - a) - T(2) * (d - b);
  const T t2 = ((e + a) - T(4) * (d + b)) + T(6) * c;
  return T(0.25) * t1 * t1 + k13 * t2 * t2;
}

template <typename T>
__device__ __forceinline__ Ind<T> indicators(T a, T b, T c, T d, T e) {
  const T k13 = T(ISW_K13);
  Ind<T> r;
  T t1, t2;
  r.b1 = (d - c) * (d - c);
  r.b2 = (c - b) * (c - b);
  t1 = c - T(2) * d + e;
  t2 = T(3) * c - T(4) * d + e;
  r.b3 = k13 * t1 * t1 + T(0.25) * t2 * t2;
  t1 = a - T(2) * b + c;
  t2 = a - T(4) * b + T(3) * c;
  r.b4 = k13 * t1 * t1 + T(0.25) * t2 * t2;
  t1 = b - T(2) * c + d;
  t2 = b - d;
  r.b12 = k13 * t1 * t1 + T(0.25) * t2 * t2;
  r.tau = tau5<T>(a, b, c, d, e);
  return r;
}

// Unnormalised weights alpha_k: eq. (28) (modified) or eq. (21) with q = 1.
// Order 3 drops the 3-point stencils (d3 = d4 = 0).
struct Alpha {
  double a1, a2, a3, a4;
};

__device__ __forceinline__ Alpha alphas_f64(const Ind<double>& s, int weights,
                                            double eps, bool order3) {
  Alpha al;
  if (weights == W_BASIC) {
    al.a1 = ISW_D1 * (1.0 + s.tau / (s.b1 + eps));
    al.a2 = ISW_D2 * (1.0 + s.tau / (s.b2 + eps));
    al.a3 = ISW_D3 * (1.0 + s.tau / (s.b3 + eps));
    al.a4 = ISW_D4 * (1.0 + s.tau / (s.b4 + eps));
  } else {
    const double r12 = s.tau / (s.b12 + eps);
    al.a1 = ISW_D1 * (1.0 + (s.tau / (s.b1 + eps)) * r12);
    al.a2 = ISW_D2 * (1.0 + (s.tau / (s.b2 + eps)) * r12);
    al.a3 = order3 ? 0.0 : ISW_D3 * (1.0 + s.tau / (s.b3 + eps));
    al.a4 = order3 ? 0.0 : ISW_D4 * (1.0 + s.tau / (s.b4 + eps));
  }
  if (order3) {
    al.a3 = 0.0;
    al.a4 = 0.0;
  }
  return al;
}

// Eq. (19) in FP64: omega_k = alpha_k / sum(alpha), q = sum omega_k q^(k),
// with the candidates of eq. (20) in their printed coefficients (the first
// one read with a plus sign: (q_i + q_{i+1})/2).
__device__ __forceinline__ double weno_f64(double a, double b, double c,
                                           double d, double e, int weights,
                                           double eps, bool order3) {
  const Ind<double> s = indicators<double>(a, b, c, d, e);
  const Alpha al = alphas_f64(s, weights, eps, order3);
  const double sum = ((al.a1 + al.a2) + al.a3) + al.a4;
  const double c1 = (1.0 / 2.0) * c + (1.0 / 2.0) * d;
  const double c2 = -(1.0 / 2.0) * b + (3.0 / 2.0) * c;
  if (order3) {
    return (al.a1 / sum) * c1 + (al.a2 / sum) * c2;
  }
  const double c3 = (1.0 / 3.0) * c + (5.0 / 6.0) * d - (1.0 / 6.0) * e;
  const double c4 = (1.0 / 3.0) * a - (7.0 / 6.0) * b + (11.0 / 6.0) * c;
  return (((al.a1 / sum) * c1 + (al.a2 / sum) * c2) + (al.a3 / sum) * c3) +
         (al.a4 / sum) * c4;
}

// ---------------------------------------------------------------------------
// The same FP64 reconstruction with cheaper divisions and identical bits.
//
// An IEEE double division x / y is computed on this hardware as: operand
// scaling (only for extreme exponents), an approximate reciprocal r of y,
// two Newton steps r += r (1 - y r), q = x r, one residual correction
// q += r (x - y q) (Markstein's method, all steps fused multiply-adds), and a
// special-value fix-up.  When no scaling can occur and no operand is special
// the scaling and fix-up steps return their inputs, so the five fused steps
// alone give the correctly rounded quotient, bit for bit.  Divisions by the
// same y then also share r: the four omega_k = alpha_k / sum(alpha) need one
// reciprocal instead of four.
//
// Range that guarantees it here: epsilon in [2^-200, 2^100], every indicator
// finite with their sum at most 2^200, and tau either 0 or at least 2^-700.
// Then every denominator lies in [2^-200, 2^201], every nonzero quotient and
// every alpha in [2^-901, 2^801], no residual is subnormal, and sum(alpha)
// is at least 0.1.  Lanes outside the range redo the reconstruction with the
// plain divisions (weno_f64).
// ---------------------------------------------------------------------------
struct Recip {
  double y, r;
};

__device__ __forceinline__ Recip recip(double y) {
  double r = __builtin_amdgcn_rcp(y);
  double e = __builtin_fma(-y, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-y, r, 1.0);
  r = __builtin_fma(r, e, r);
  return {y, r};
}

__device__ __forceinline__ double divide(double x, const Recip& d) {
  const double q = x * d.r;
  const double rem = __builtin_fma(-d.y, q, x);
  return __builtin_fma(rem, d.r, q);
}

__device__ __forceinline__ bool fast_division_range(const Ind<double>& s) {
  const double sum = ((((s.tau + s.b1) + s.b2) + s.b3) + s.b4) + s.b12;
  return sum <= 0x1p200 && (s.tau == 0.0 || s.tau >= 0x1p-700);
}

__device__ __forceinline__ double weno_f64_shared_recip(const Ind<double>& s, double a, double b,
                                                       double c, double d, double e,
                                                       int weights, double eps, bool order3) {
  Alpha al;
  if (weights == W_BASIC) {
    al.a1 = ISW_D1 * (1.0 + divide(s.tau, recip(s.b1 + eps)));
    al.a2 = ISW_D2 * (1.0 + divide(s.tau, recip(s.b2 + eps)));
    al.a3 = ISW_D3 * (1.0 + divide(s.tau, recip(s.b3 + eps)));
    al.a4 = ISW_D4 * (1.0 + divide(s.tau, recip(s.b4 + eps)));
  } else {
    const double r12 = divide(s.tau, recip(s.b12 + eps));
    al.a1 = ISW_D1 * (1.0 + divide(s.tau, recip(s.b1 + eps)) * r12);
    al.a2 = ISW_D2 * (1.0 + divide(s.tau, recip(s.b2 + eps)) * r12);
    al.a3 = order3 ? 0.0 : ISW_D3 * (1.0 + divide(s.tau, recip(s.b3 + eps)));
    al.a4 = order3 ? 0.0 : ISW_D4 * (1.0 + divide(s.tau, recip(s.b4 + eps)));
  }
  if (order3) {
    al.a3 = 0.0;
    al.a4 = 0.0;
  }
  const double sum = ((al.a1 + al.a2) + al.a3) + al.a4;
  const Recip rs = recip(sum);
  const double c1 = (1.0 / 2.0) * c + (1.0 / 2.0) * d;
  const double c2 = -(1.0 / 2.0) * b + (3.0 / 2.0) * c;
  if (order3) {
    return divide(al.a1, rs) * c1 + divide(al.a2, rs) * c2;
  }
  const double c3 = (1.0 / 3.0) * c + (5.0 / 6.0) * d - (1.0 / 6.0) * e;
  const double c4 = (1.0 / 3.0) * a - (7.0 / 6.0) * b + (11.0 / 6.0) * c;
  return ((divide(al.a1, rs) * c1 + divide(al.a2, rs) * c2) + divide(al.a3, rs) * c3) +
         divide(al.a4, rs) * c4;
}

// Eq. (19) when the global indicator tau5 of eq. (25) is exactly zero
// (epsilon > 0): every ratio tau5/(beta + epsilon) of eqs. (21) and (28) is
// then exactly zero, every weight exactly d_k, and the normalisation
// divides by the same sum on every such stencil -- the linear scheme, which
// the indicators select on data with vanishing third and fourth
// differences -- every stencil of equal values, among others.
// The candidates of eq. (20) are formed as in the general path and
// combined in its order with d_k / sum_j d_j (divided at compile time,
// correctly rounded as the general path divides): the same bits without
// the divisions of the weights.
__device__ __forceinline__ double weno_f64_linear(double a, double b, double c, double d,
                                                  double e, bool order3) {
  constexpr double s3 = ISW_D1 + ISW_D2;
  constexpr double s5 = ((ISW_D1 + ISW_D2) + ISW_D3) + ISW_D4;
  const double c1 = (1.0 / 2.0) * c + (1.0 / 2.0) * d;
  const double c2 = -(1.0 / 2.0) * b + (3.0 / 2.0) * c;
  if (order3) return (ISW_D1 / s3) * c1 + (ISW_D2 / s3) * c2;
  const double c3 = (1.0 / 3.0) * c + (5.0 / 6.0) * d - (1.0 / 6.0) * e;
  const double c4 = (1.0 / 3.0) * a - (7.0 / 6.0) * b + (11.0 / 6.0) * c;
  return (((ISW_D1 / s5) * c1 + (ISW_D2 / s5) * c2) + (ISW_D3 / s5) * c3) +
         (ISW_D4 / s5) * c4;
}

// FP64 reconstruction as used by the stage kernels: stencils with tau5 = 0
// take the linear form (no other indicator is needed); the others the
// shared-reciprocal form, recomputed with the plain divisions (weno_f64) on
// the lanes outside its range.  The branches diverge per lane; a wave skips
// a branch no lane needs.  nlin counts the stencils of the linear form.
__device__ __forceinline__ double weno_f64_fast(double a, double b, double c, double d,
                                                double e, int weights, double eps,
                                                bool order3, int& nlin) {
  if (eps > 0.0 && tau5<double>(a, b, c, d, e) == 0.0) {
    nlin++;
    return weno_f64_linear(a, b, c, d, e, order3);
  }
  const Ind<double> s = indicators<double>(a, b, c, d, e);
  double q = weno_f64_shared_recip(s, a, b, c, d, e, weights, eps, order3);
  if (!(eps >= 0x1p-200 && eps <= 0x1p100 && fast_division_range(s)))
    q = weno_f64(a, b, c, d, e, weights, eps, order3);
  return q;
}

// Eq. (19) in FP32.  The indicators grow with the square of the data and
// the modified weights multiply two ratios, which overflows float for the
// pressure-like fields (|q| up to 1e9).  The stencil is therefore shifted by
// its centre value and scaled by s = max |q_j - q_i| (both ratios of
// eq. (28) are invariant under that map when epsilon is scaled by 1/s^2),
// the scaled epsilon is kept >= 1e-30 and each product of ratios is clamped
// at 1e30.  A stencil whose spread is below 1e-30 (flat, or denormal-level
// noise such as a material property diffused into the other phase) returns
// the centre value: its reciprocal would overflow float.
__device__ __forceinline__ float weno_f32(float a, float b, float c, float d,
                                          float e, int weights, float eps,
                                          bool order3, int& nshort) {
  const float s = fmaxf(fmaxf(fmaxf(fabsf(a - c), fabsf(b - c)), fabsf(d - c)),
                        fabsf(e - c));
  if (!(s > 1e-30f)) {
    nshort++;
    return c;
  }
  const float is = __builtin_amdgcn_rcpf(s);
  const float A = (a - c) * is, B = (b - c) * is, D = (d - c) * is,
              E = (e - c) * is;
  const Ind<float> r = indicators<float>(A, B, 0.0f, D, E);
  const float es = fmaxf(eps * is * is, 1e-30f);
  float a1, a2, a3, a4;
  if (weights == W_BASIC) {
    a1 = 0.4f * (1.0f + r.tau * __builtin_amdgcn_rcpf(r.b1 + es));
    a2 = 0.2f * (1.0f + r.tau * __builtin_amdgcn_rcpf(r.b2 + es));
    a3 = 0.3f * (1.0f + r.tau * __builtin_amdgcn_rcpf(r.b3 + es));
    a4 = 0.1f * (1.0f + r.tau * __builtin_amdgcn_rcpf(r.b4 + es));
  } else {
    const float r12 = r.tau * __builtin_amdgcn_rcpf(r.b12 + es);
    a1 = 0.4f * (1.0f + fminf(r.tau * __builtin_amdgcn_rcpf(r.b1 + es) * r12, 1e30f));
    a2 = 0.2f * (1.0f + fminf(r.tau * __builtin_amdgcn_rcpf(r.b2 + es) * r12, 1e30f));
    a3 = 0.3f * (1.0f + fminf(r.tau * __builtin_amdgcn_rcpf(r.b3 + es), 1e30f));
    a4 = 0.1f * (1.0f + fminf(r.tau * __builtin_amdgcn_rcpf(r.b4 + es), 1e30f));
  }
  const float C1 = 0.5f * D;
  const float C2 = -0.5f * B;
  if (order3) {
    const float inv = __builtin_amdgcn_rcpf(a1 + a2);
    return c + s * ((a1 * C1 + a2 * C2) * inv);
  }
  const float C3 = (5.0f * D - E) * (1.0f / 6.0f);
  const float C4 = (2.0f * A - 7.0f * B) * (1.0f / 6.0f);
  const float inv = __builtin_amdgcn_rcpf(((a1 + a2) + a3) + a4);
  return c + s * ((a1 * C1 + a2 * C2 + a3 * C3 + a4 * C4) * inv);
}

// ---------------------------------------------------------------------------
// Cut-off weights (W_CUTOFF): the targeted-ENO optimisation that the
// conclusions (Sec. 7) propose for lower dissipation in smooth regions,
// applied to the eq. (28) weights.  Each stencil's measure is
// gamma_k = (alpha_k / d_k)^6 (alpha_k of eq. (28)); a stencil whose share
// gamma_k / sum(gamma) is below C_T gets weight zero and the others the
// optimal weights renormalised, d_k / sum(kept d).  The share test is taken
// on t_k = (alpha_k/d_k) / max_s(alpha_s/d_s), as t_k^6 >= C_T sum t_s^6
// (no overflow), and the renormalised weights as 4, 2, 3, 1 over their kept
// sum, so that a stencil set with nothing cut gives d_k exactly.  Order 3
// cuts among the two 2-point stencils.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double cut_pow6(double t) {
  const double t2 = t * t;
  return (t2 * t2) * t2;
}

// omega of every set of kept stencils (bit k-1 of the index: stencil k):
// 4, 2, 3, 1 over the kept sum, divided (correctly rounded) at compile time.
struct CutWeights {
  double w[16][4];
};
constexpr CutWeights make_cut_weights() {
  CutWeights t{};
  const double dk[4] = {4.0, 2.0, 3.0, 1.0};
  for (int m = 0; m < 16; m++) {
    double ds = 0.0;
    for (int k = 0; k < 4; k++)
      if (m >> k & 1) ds += dk[k];
    for (int k = 0; k < 4; k++) t.w[m][k] = (m >> k & 1) ? dk[k] / ds : 0.0;
  }
  return t;
}
__constant__ CutWeights kCutWeights = make_cut_weights();

// Eq. (19) with the weights of a kept-stencil mask.
__device__ __forceinline__ double cut_combine(int mask, double a, double b, double c, double d,
                                              double e, bool order3) {
  if (order3) mask &= 3;
  const double* w = kCutWeights.w[mask];
  const double c1 = (1.0 / 2.0) * c + (1.0 / 2.0) * d;
  const double c2 = -(1.0 / 2.0) * b + (3.0 / 2.0) * c;
  if (order3) return w[0] * c1 + w[1] * c2;
  const double c3 = (1.0 / 3.0) * c + (5.0 / 6.0) * d - (1.0 / 6.0) * e;
  const double c4 = (1.0 / 3.0) * a - (7.0 / 6.0) * b + (11.0 / 6.0) * c;
  return ((w[0] * c1 + w[1] * c2) + w[2] * c3) + w[3] * c4;
}

// The kept-stencil mask of the share test.  FAST: every quotient through the
// unscaled division sequence (divide, recip), the shares t_k = g_k / g_max
// through one reciprocal of g_max.  Inside the range of fast_division_range
// with epsilon in [2^-200, 2^100], each ratio tau/(beta + eps) is one of the
// WENO-IS weights' quotients, g_k = 1 + ratios lies in [1, 2^801] and
// t_k = g_k / g_max in [2^-801, 1]: no operand scaling, no special value,
// the bits of the plain divisions.  Otherwise: the plain divisions.
template <bool FAST>
__device__ __forceinline__ double cut_quot(double x, double y) {
  if constexpr (FAST) return divide(x, recip(y));
  else return x / y;
}

template <bool FAST>
__device__ __forceinline__ int cut_mask_f64(const Ind<double>& s, double eps, bool order3) {
  const double r12 = cut_quot<FAST>(s.tau, s.b12 + eps);
  const double g1 = 1.0 + cut_quot<FAST>(s.tau, s.b1 + eps) * r12;
  const double g2 = 1.0 + cut_quot<FAST>(s.tau, s.b2 + eps) * r12;
  double gm = g1;
  if (g2 > gm) gm = g2;
  if (order3) {
    const Recip rg = recip(gm);
    const double p1 = cut_pow6(FAST ? divide(g1, rg) : g1 / gm);
    const double p2 = cut_pow6(FAST ? divide(g2, rg) : g2 / gm);
    const double th = ISW_CT * (p1 + p2);
    return (p1 >= th ? 1 : 0) | (p2 >= th ? 2 : 0);
  }
  const double g3 = 1.0 + cut_quot<FAST>(s.tau, s.b3 + eps);
  const double g4 = 1.0 + cut_quot<FAST>(s.tau, s.b4 + eps);
  if (g3 > gm) gm = g3;
  if (g4 > gm) gm = g4;
  const Recip rg = recip(gm);
  const double p1 = cut_pow6(FAST ? divide(g1, rg) : g1 / gm);
  const double p2 = cut_pow6(FAST ? divide(g2, rg) : g2 / gm);
  const double p3 = cut_pow6(FAST ? divide(g3, rg) : g3 / gm);
  const double p4 = cut_pow6(FAST ? divide(g4, rg) : g4 / gm);
  const double th = ISW_CT * (((p1 + p2) + p3) + p4);
  return (p1 >= th ? 1 : 0) | (p2 >= th ? 2 : 0) | (p3 >= th ? 4 : 0) | (p4 >= th ? 8 : 0);
}

// FP64 cut-off reconstruction as used by the kernels.  Stencils with
// tau5 = 0 keep every stencil (every ratio is zero) and take the weights of
// the full set as compile-time constants.  The others take the FAST mask;
// lanes outside its range redo the whole reconstruction with the plain
// divisions (a separate path, as in weno_f64_fast, keeps the common path's
// registers low).
__device__ __forceinline__ double weno_f64_cutoff(double a, double b, double c, double d,
                                                  double e, double eps, bool order3,
                                                  int& nlin) {
  if (eps > 0.0 && tau5<double>(a, b, c, d, e) == 0.0) {
    nlin++;
    constexpr CutWeights W = make_cut_weights();
    const double c1 = (1.0 / 2.0) * c + (1.0 / 2.0) * d;
    const double c2 = -(1.0 / 2.0) * b + (3.0 / 2.0) * c;
    if (order3) return W.w[3][0] * c1 + W.w[3][1] * c2;
    const double c3 = (1.0 / 3.0) * c + (5.0 / 6.0) * d - (1.0 / 6.0) * e;
    const double c4 = (1.0 / 3.0) * a - (7.0 / 6.0) * b + (11.0 / 6.0) * c;
    return ((W.w[15][0] * c1 + W.w[15][1] * c2) + W.w[15][2] * c3) + W.w[15][3] * c4;
  }
  const Ind<double> s = indicators<double>(a, b, c, d, e);
  double q = cut_combine(cut_mask_f64<true>(s, eps, order3), a, b, c, d, e, order3);
  if (!(eps >= 0x1p-200 && eps <= 0x1p100 && fast_division_range(s)))
    q = cut_combine(cut_mask_f64<false>(s, eps, order3), a, b, c, d, e, order3);
  return q;
}

// The same cut-off in the float form: the stencil shifted and scaled as in
// weno_f32, ratios clamped at 1e30, hardware reciprocals.
__device__ __forceinline__ float weno_f32_cutoff(float a, float b, float c, float d, float e,
                                                 float eps, bool order3, int& nshort) {
  const float s = fmaxf(fmaxf(fmaxf(fabsf(a - c), fabsf(b - c)), fabsf(d - c)),
                        fabsf(e - c));
  if (!(s > 1e-30f)) {
    nshort++;
    return c;
  }
  const float is = __builtin_amdgcn_rcpf(s);
  const float A = (a - c) * is, B = (b - c) * is, D = (d - c) * is,
              E = (e - c) * is;
  const Ind<float> r = indicators<float>(A, B, 0.0f, D, E);
  const float es = fmaxf(eps * is * is, 1e-30f);
  const float r12 = r.tau * __builtin_amdgcn_rcpf(r.b12 + es);
  const float g1 = 1.0f + fminf(r.tau * __builtin_amdgcn_rcpf(r.b1 + es) * r12, 1e30f);
  const float g2 = 1.0f + fminf(r.tau * __builtin_amdgcn_rcpf(r.b2 + es) * r12, 1e30f);
  const float C1 = 0.5f * D;
  const float C2 = -0.5f * B;
  auto share = [](float g, float rg) {
    const float t = g * rg;
    const float t2 = t * t;
    return (t2 * t2) * t2;
  };
  if (order3) {
    const float rg = __builtin_amdgcn_rcpf(fmaxf(g1, g2));
    const float p1 = share(g1, rg), p2 = share(g2, rg);
    const float th = float(ISW_CT) * (p1 + p2);
    const float k1 = p1 >= th ? 4.0f : 0.0f, k2 = p2 >= th ? 2.0f : 0.0f;
    return c + s * ((k1 * C1 + k2 * C2) * __builtin_amdgcn_rcpf(k1 + k2));
  }
  const float g3 = 1.0f + fminf(r.tau * __builtin_amdgcn_rcpf(r.b3 + es), 1e30f);
  const float g4 = 1.0f + fminf(r.tau * __builtin_amdgcn_rcpf(r.b4 + es), 1e30f);
  const float rg = __builtin_amdgcn_rcpf(fmaxf(fmaxf(g1, g2), fmaxf(g3, g4)));
  const float p1 = share(g1, rg), p2 = share(g2, rg), p3 = share(g3, rg), p4 = share(g4, rg);
  const float th = float(ISW_CT) * (((p1 + p2) + p3) + p4);
  const float k1 = p1 >= th ? 4.0f : 0.0f, k2 = p2 >= th ? 2.0f : 0.0f,
              k3 = p3 >= th ? 3.0f : 0.0f, k4 = p4 >= th ? 1.0f : 0.0f;
  const float C3 = (5.0f * D - E) * (1.0f / 6.0f);
  const float C4 = (2.0f * A - 7.0f * B) * (1.0f / 6.0f);
  return c + s * ((k1 * C1 + k2 * C2 + k3 * C3 + k4 * C4) *
                  __builtin_amdgcn_rcpf(((k1 + k2) + k3) + k4));
}

template <typename T>
__device__ __forceinline__ T weno(T a, T b, T c, T d, T e, int weights,
                                  T eps, bool order3, int& nshort);
template <>
__device__ __forceinline__ double weno<double>(double a, double b, double c,
                                               double d, double e, int w,
                                               double eps, bool o3, int& nshort) {
  return weno_f64_fast(a, b, c, d, e, w, eps, o3, nshort);
}
template <>
__device__ __forceinline__ float weno<float>(float a, float b, float c,
                                             float d, float e, int w,
                                             float eps, bool o3, int& nshort) {
  return weno_f32(a, b, c, d, e, w, eps, o3, nshort);
}

// ---------------------------------------------------------------------------
// Face state container (face order: rho, u_n, u_t..., p, Gamma, Pi).
// ---------------------------------------------------------------------------
template <int NT>
struct FState {
  static constexpr int NC = 5 + NT;
  double v[NC];
};

// ---------------------------------------------------------------------------
// HLLC, eqs. (14)-(18).  Averages of eq. (17) read as the Roe-type
// (sqrt(rho_l) u_l + sqrt(rho_r) u_r)/(sqrt(rho_l) + sqrt(rho_r)) and the
// Einfeldt-type c^2 with sqrt(rho_r) c_r^2; sign(0) = 0; when S_k equals S*
// the star flux of that side is its limit F_k (star velocity u_k).
// Only the star state selected by sign(S*) is formed (both at S* = 0).
// ---------------------------------------------------------------------------
template <typename T, int NT>
__device__ __forceinline__ void star_flux(const T* q, T Sk, T Ss, T* F,
                                          T& us) {
  constexpr int NC = 5 + NT;
  const T rho = q[0], un = q[1], p = q[2 + NT], G = q[3 + NT], P = q[4 + NT];
  T ke = un * un;
#pragma unroll
  for (int t = 0; t < NT; t++) ke = ke + q[2 + t] * q[2 + t];
  const T E = G * p + P + T(0.5) * rho * ke;
  T Uk[NC], Fk[NC];
  Uk[0] = rho;
  Uk[1] = rho * un;
#pragma unroll
  for (int t = 0; t < NT; t++) Uk[2 + t] = rho * q[2 + t];
  Uk[2 + NT] = E;
  Uk[3 + NT] = G;
  Uk[4 + NT] = P;
  Fk[0] = rho * un;
  Fk[1] = rho * un * un + p;
#pragma unroll
  for (int t = 0; t < NT; t++) Fk[2 + t] = rho * un * q[2 + t];
  Fk[2 + NT] = (E + p) * un;
  Fk[3 + NT] = G * un;
  Fk[4 + NT] = P * un;
  const T den = Sk - Ss;
  if (den == T(0)) {
#pragma unroll
    for (int k = 0; k < NC; k++) F[k] = Fk[k];
    us = un;
    return;
  }
  const T pk = p + rho * (Sk - un) * (Ss - un);
  const T sp = Sk * pk;
#pragma unroll
  for (int k = 0; k < NC; k++) {
    const T Dk = (k == 1) ? T(1) : ((k == 2 + NT) ? Ss : T(0));
    F[k] = qdiv<T>(Ss * (Sk * Uk[k] - Fk[k]) + sp * Dk, den);
  }
  us = qdiv<T>(Ss * (Sk - un), den);
}

// The products 0 * F*_k and 0 * u*_k of eq. (14) for a star state whose
// weight is zero: signed zeros (or NaN for a non-finite state).  Formed
// with star_flux's operations up to its division; a quotient's sign is the
// sign of numerator times denominator, so (0 * num) * den is 0 * (num / den)
// for every finite num and den != 0 (and den == 0 takes the physical flux,
// as star_flux does).  FP64 only.
template <int NT>
__device__ __forceinline__ void star_zeros(const double* q, double Sk, double Ss, double* Z,
                                           double& zus) {
  constexpr int NC = 5 + NT;
  const double rho = q[0], un = q[1], p = q[2 + NT], G = q[3 + NT], P = q[4 + NT];
  double ke = un * un;
#pragma unroll
  for (int t = 0; t < NT; t++) ke = ke + q[2 + t] * q[2 + t];
  const double E = G * p + P + 0.5 * rho * ke;
  double Uk[NC], Fk[NC];
  Uk[0] = rho;
  Uk[1] = rho * un;
#pragma unroll
  for (int t = 0; t < NT; t++) Uk[2 + t] = rho * q[2 + t];
  Uk[2 + NT] = E;
  Uk[3 + NT] = G;
  Uk[4 + NT] = P;
  Fk[0] = rho * un;
  Fk[1] = rho * un * un + p;
#pragma unroll
  for (int t = 0; t < NT; t++) Fk[2 + t] = rho * un * q[2 + t];
  Fk[2 + NT] = (E + p) * un;
  Fk[3 + NT] = G * un;
  Fk[4 + NT] = P * un;
  const double den = Sk - Ss;
  if (den == 0.0) {
#pragma unroll
    for (int k = 0; k < NC; k++) Z[k] = 0.0 * Fk[k];
    zus = 0.0 * un;
    return;
  }
  const double pk = p + rho * (Sk - un) * (Ss - un);
  const double sp = Sk * pk;
#pragma unroll
  for (int k = 0; k < NC; k++) {
    const double Dk = (k == 1) ? 1.0 : ((k == 2 + NT) ? Ss : 0.0);
    Z[k] = (0.0 * (Ss * (Sk * Uk[k] - Fk[k]) + sp * Dk)) * den;
  }
  zus = (0.0 * (Ss * (Sk - un))) * den;
}

template <typename T, int NT>
__device__ __forceinline__ void hllc(const T* ql, const T* qr, T* F, T& us) {
  constexpr int NC = 5 + NT;
  const T rl = ql[0], ul = ql[1], pl = ql[2 + NT];
  const T rr = qr[0], ur = qr[1], pr = qr[2 + NT];
  const T cl2 = sound2<T>(rl, pl, ql[3 + NT], ql[4 + NT]);
  const T cr2 = sound2<T>(rr, pr, qr[3 + NT], qr[4 + NT]);
  const T cl = sqrt(cl2), cr = sqrt(cr2);
  const T sl = sqrt(rl), sr = sqrt(rr);
  const T ubar = qdiv<T>(sl * ul + sr * ur, sl + sr);
  const T cbar2 = qdiv<T>(sl * cl2 + sr * cr2, sl + sr) +
                  qdiv<T>(T(0.5) * sl * sr, (sl + sr) * (sl + sr)) * (ur - ul) *
                      (ur - ul);
  const T cbar = sqrt(cbar2);
  const T Sl = dmin<T>(dmin<T>(ubar - cbar, ul - cl), T(0));
  const T Sr = dmax<T>(dmax<T>(ubar + cbar, ur + cr), T(0));
  const T Ss = qdiv<T>(pr - pl + rl * ul * (Sl - ul) - rr * ur * (Sr - ur),
                      rl * (Sl - ul) - rr * (Sr - ur));
  if (Ss != T(0)) {
    const bool left = Ss > T(0);
    T qs[NC];
#pragma unroll
    for (int k = 0; k < NC; k++) qs[k] = left ? ql[k] : qr[k];
    star_flux<T, NT>(qs, left ? Sl : Sr, Ss, F, us);
    if constexpr (sizeof(T) == 8) {
      // Eq. (14) as written adds the other star state times zero.  That
      // changes no value, only the sign of a flux component that is exactly
      // zero (a transverse momentum flux where u_t = 0, say), so the FP64
      // path adds it where the selected state has such a component.
      bool z = us == T(0);
#pragma unroll
      for (int k = 0; k < NC; k++) z = z || F[k] == T(0);
      if (z) {
        T qo[NC], Z[NC], zus;
#pragma unroll
        for (int k = 0; k < NC; k++) qo[k] = left ? qr[k] : ql[k];
        star_zeros<NT>(qo, left ? Sr : Sl, Ss, Z, zus);
#pragma unroll
        for (int k = 0; k < NC; k++) F[k] = F[k] + Z[k];
        us = us + zus;
      }
    }
  } else {
    T Fl[NC], Fr[NC], usl, usr;
    star_flux<T, NT>(ql, Sl, Ss, Fl, usl);
    star_flux<T, NT>(qr, Sr, Ss, Fr, usr);
#pragma unroll
    for (int k = 0; k < NC; k++) F[k] = T(0.5) * Fl[k] + T(0.5) * Fr[k];
    us = T(0.5) * usl + T(0.5) * usr;
  }
}

// The reconstruction a stage kernel evaluates: the cut-off form (a
// compile-time choice: its kernels are instantiated apart), or weno<T> with
// the eq. (21)/(28) weights.
template <typename T, bool CUT>
__device__ __forceinline__ T weno_sel(T a, T b, T c, T d, T e, int weights, T eps, bool order3,
                                      int& nshort) {
  if constexpr (CUT) {
    if constexpr (sizeof(T) == 8) return weno_f64_cutoff(a, b, c, d, e, eps, order3, nshort);
    else return weno_f32_cutoff(a, b, c, d, e, eps, order3, nshort);
  } else {
    return weno<T>(a, b, c, d, e, weights, eps, order3, nshort);
  }
}

}  // namespace isw
