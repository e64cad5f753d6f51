// Direction-sweep stage kernel of the WENO-IS finite-volume operator.
//
// One launch handles one axis D of an RK stage (Sec. 3, dimension by
// dimension).  A workgroup owns a tile of TL cells along D by TW cells
// across it:
//   1. load U for the tile plus 3 ghost cells per side along D (boundary
//      conditions applied while loading), recover the primitive state in
//      FP64 (eq. (2)) and stage it in LDS, latching non-physical cells;
//   2. one lane per face: project the six stencil cells onto the
//      characteristic fields (eqs. (11)-(12)), reconstruct both face states
//      with WENO-IS (eqs. (19)-(28)), back-project (eq. (13)), apply the
//      MOOD cascade (Sec. 3.4) and evaluate HLLC (eqs. (14)-(18)); the
//      flux and u^HLLC go to LDS;
//   3. one lane per cell: the D-contribution to dU/dt, eqs. (5)-(6), added to
//      the partial sum of the previous axes, and either stored as a partial
//      sum, stored as dU/dt, or combined into the Runge-Kutta stage.
// Coalescing: along x the tile rows are contiguous; for y and z sweeps the
// tile is TW consecutive x cells wide.
#pragma once

#include "face.hpp"
#include "mlp.hpp"

namespace isw {

enum OutMode {
  OUT_PARTIAL = 0,  // R = (R +) r_D
  OUT_RHS = 1,      // dUdt = (R +) r_D
  OUT_RK1 = 2,      // Uout = U0 + dt L
  OUT_RK2 = 3,      // Uout = 3/4 U0 + 1/4 (Uin + dt L)
  OUT_RK3 = 4,      // Uout = 1/3 U0 + 2/3 (Uin + dt L)
  // the time step inside the first two stages (fused 2D stage only):
  OUT_RK1L = 5,     // Rout = L(Uin), and each workgroup's max wave speed of Uin
  OUT_RK2L = 6,     // as OUT_RK2 with the stage input U0 + dt R, R = L(U0) of OUT_RK1L
  // the time step inside the first sweep of a 3D stage:
  OUT_PARTIAL_S = 7 // as OUT_PARTIAL (x sweep), and each workgroup's max wave speed of Uin
};

enum { ST_OK = 0, ST_NONPHYSICAL = -4 };

struct StatsDev {  // layout of isweno_stats
  unsigned long long o3[3], o1[3], mlp_fallback[3];
  int status;
  int reserved;
};

struct SweepArgs {
  const double* Uin;   // stage input (stencil source), nc x N
  const double* R;     // partial sum of previous axes (when read)
  double* Rout;        // partial-sum / dUdt output
  const double* U0;    // U^n for the RK combine
  double* Uout;        // RK stage output
  const double* dt;    // device scalar
  StatsDev* stats;     // may be null
  int64_t n[3];
  double dx[3];
  int bc_lo, bc_hi;    // of axis D
  int bcl[3], bch[3];  // of every axis (fused multi-axis stage kernels)
  int weights, mood;
  double eps;
  const uint16_t* mlp; // packed bf16 network (learned weights only)
  float mlp_thr;
  unsigned long long* shortcut;  // 256 x 3 counters of shortcut field-sides, or null
  // OUT_RK1L, OUT_PARTIAL_S: one max wave speed per workgroup (the bits of
  // the double)
  unsigned long long* cflp;
};

// Sum of an int over the 64 lanes of a wave (every lane active).
__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Boundary map of a ghost/interior position l (-3..n+2) on a line of n
// cells: interior index and whether the normal velocity is mirrored.
__device__ __forceinline__ int64_t bc_index(int64_t l, int64_t n, int bclo,
                                            int bchi, bool& flip) {
  flip = false;
  if (l < 0) {
    if (bclo == 1) return ((l % n) + n) % n;
    if (bclo == 2) {
      flip = true;
      return -l - 1;
    }
    return 0;
  }
  if (l >= n) {
    if (bchi == 1) return l % n;
    if (bchi == 2) {
      flip = true;
      return 2 * n - 1 - l;
    }
    return n - 1;
  }
  return l;
}

// FP64 quotients in the kernels: exact (IEEE) in the FP64 form, which
// reproduces the oracle bit for bit; in the float form, whose reconstruction
// and flux are float, x times the refined reciprocal of the divisor (within
// 2 ulp of the quotient for a normal divisor), a third of the instructions.
template <typename T>
__device__ __forceinline__ double div64(double x, double y) {
  if constexpr (sizeof(T) == 8) return x / y;
  else return x * recip(y).r;
}

// The same for many quotients by one divisor (the reciprocal formed once).
template <typename T>
struct Div64 {
  double y, r;
  __device__ __forceinline__ explicit Div64(double d) : y(d), r(0.0) {
    if constexpr (sizeof(T) == 4) r = recip(d).r;
  }
  __device__ __forceinline__ double operator()(double x) const {
    if constexpr (sizeof(T) == 8) return x / y;
    else return x * r;
  }
};

// Primitive recovery of one cell, axis order (rho, u_x.., p, Gamma, Pi),
// eq. (2): p = (E - rho |u|^2 / 2 - Pi) / Gamma; the quotients as div64<T>.
template <int NDIM, typename T = double>
__device__ __forceinline__ void cons_prim(const double* u, double* q) {
  const double rho = u[0];
  const Div64<T> by_rho(rho);
  double vel[NDIM];
#pragma unroll
  for (int a = 0; a < NDIM; a++) vel[a] = by_rho(u[1 + a]);
  double ke = vel[0] * vel[0];
#pragma unroll
  for (int a = 1; a < NDIM; a++) ke = ke + vel[a] * vel[a];
  const double E = u[1 + NDIM];
  const double G = u[2 + NDIM];
  const double P = u[3 + NDIM];
  q[0] = rho;
#pragma unroll
  for (int a = 0; a < NDIM; a++) q[1 + a] = vel[a];
  q[1 + NDIM] = div64<T>(E - 0.5 * rho * ke - P, G);
  q[2 + NDIM] = G;
  q[3 + NDIM] = P;
}

template <int NDIM, typename T = double>
__device__ __forceinline__ void cell_prim(const double* U, int64_t N,
                                          int64_t cell, double* q) {
  double u[4 + NDIM];
#pragma unroll
  for (int k = 0; k < 4 + NDIM; k++) u[k] = U[k * N + cell];
  cons_prim<NDIM, T>(u, q);
}

// Time step (the CFL condition of Secs. 5 and 6): one cell's
// sum_d (|u_d| + c)/dx_d from its axis-order primitives q, the quotients as
// div64<T>.
template <int NDIM, typename T = double>
__device__ __forceinline__ double cell_speed(const double* q, const double* dx) {
  const double cs = sqrt(sound2<double>(q[0], q[1 + NDIM], q[2 + NDIM], q[3 + NDIM]));
  double sp = div64<T>(fabs(q[1]) + cs, dx[0]);
#pragma unroll
  for (int a = 1; a < NDIM; a++) sp = sp + div64<T>(fabs(q[1 + a]) + cs, dx[a]);
  return sp;
}

// Each wave's max of m over its lanes, as the bits of the double (positive
// doubles order as their bits do; a NaN orders above every number), into
// red[wave]; the caller combines red after a barrier.
__device__ __forceinline__ void wave_max_bits(double m, unsigned long long* red) {
  unsigned long long b = (unsigned long long)__double_as_longlong(m);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long x = __shfl_xor(b, o);
    b = x > b ? x : b;
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = b;
}

template <int NDIM>
__device__ __forceinline__ bool cell_ok(const double* U, int64_t N,
                                        int64_t cell, const double* q) {
  bool fin = true;
#pragma unroll
  for (int k = 0; k < 4 + NDIM; k++) fin = fin && isfinite(U[k * N + cell]);
  return fin && admissible(q[0], q[1 + NDIM], q[2 + NDIM], q[3 + NDIM]);
}

// The same check on a cell's conservative values u (already loaded).
template <int NDIM>
__device__ __forceinline__ bool cell_ok_u(const double* u, const double* q) {
  bool fin = true;
#pragma unroll
  for (int k = 0; k < 4 + NDIM; k++) fin = fin && isfinite(u[k]);
  return fin && admissible(q[0], q[1 + NDIM], q[2 + NDIM], q[3 + NDIM]);
}

// Face-order component k -> axis-order (LDS / conservative) component.
template <int NDIM, int D>
__device__ __host__ constexpr int axis_comp(int k) {
  return k == 0 ? 0
         : k == 1 ? 1 + D
         : (k < 1 + NDIM) ? 1 + ((k - 2) < D ? (k - 2) : (k - 1))
                          : k;
}

// Reconstruct the face states at the given order and back-project them to
// face-order primitives in FP64.  One characteristic field per iteration
// (the loop is kept rolled to bound register use; the branches on the field
// index are wave-uniform): project the six stencil cells with the field's
// row of L (eq. (11)), reconstruct the left state from positions 0..4
// (i-2..i+2) and the right state from the mirror image 5..1, and add the
// field's column of R (eq. (13)) into the face states in field order.
// sides: bit 0 = left, bit 1 = right.  S(c, j) reads LDS component c (axis
// order) at stencil position j.
// Learned weights for one field: the network on the 64 faces of the wave
// (two 32-sample tiles, all lanes take part), its weights applied to the
// candidates of eq. (20) as in eq. (19); below the confidence threshold, or
// for a side whose value leaves the range of the two cells next to the
// face, the eq. (28) weights are used instead (each counted as a fallback).
template <typename T>
__device__ __forceinline__ void mlp_field(const T* w, MlpRun& mr, T eps, T& rl, T& rr) {
  // Flat on both sides (spread below 1e-30, as the plain float form tests
  // it): every candidate is the centre value, so both the learned weights
  // and their fallback give it exactly.  A wave whose every lane is flat
  // skips the network (which needs the whole wave).
  const T sl = fmaxf(fmaxf(fmaxf(fabsf(w[0] - w[2]), fabsf(w[1] - w[2])), fabsf(w[3] - w[2])),
                     fabsf(w[4] - w[2]));
  const T sr = fmaxf(fmaxf(fmaxf(fabsf(w[5] - w[3]), fabsf(w[4] - w[3])), fabsf(w[2] - w[3])),
                     fabsf(w[1] - w[3]));
  if (__all(!(sl > T(1e-30)) && !(sr > T(1e-30)))) {
    rl = w[2];
    rr = w[3];
    return;
  }
  float x[8], z[9];
  mlp_features<T>(w, mr.f6, mr.f7, x);
  mlp_logits_wave(x, *mr.R, *mr.B, z);
  const float conf = 1.0f / (1.0f + __expf(-z[8]));
  if (!(conf >= mr.thr)) {
    int nf = 0;
    rl = weno<T>(w[0], w[1], w[2], w[3], w[4], W_MODIFIED, eps, false, nf);
    rr = weno<T>(w[5], w[4], w[3], w[2], w[1], W_MODIFIED, eps, false, nf);
    mr.fallbacks++;
    return;
  }
#pragma unroll
  for (int side = 0; side < 2; side++) {
    const float* zs = z + 4 * side;
    const float m = fmaxf(fmaxf(zs[0], zs[1]), fmaxf(zs[2], zs[3]));
    float e[4], sum = 0.0f;
#pragma unroll
    for (int k = 0; k < 4; k++) {
      e[k] = __expf(zs[k] - m);
      sum += e[k];
    }
    const float A = float(side ? w[5] : w[0]), B = float(side ? w[4] : w[1]),
                C = float(side ? w[3] : w[2]), D_ = float(side ? w[2] : w[3]),
                E = float(side ? w[1] : w[4]);
    // candidates of eq. (20) written as the centre value plus differences,
    // so that a constant stencil is reproduced exactly; weighted and
    // normalised by one reciprocal
    const float d1 = 0.5f * (D_ - C), d2 = 0.5f * (C - B);
    const float d3 = (5.0f / 6.0f) * (D_ - C) - (1.0f / 6.0f) * (E - C);
    const float d4 = (1.0f / 3.0f) * (A - C) - (7.0f / 6.0f) * (B - C);
    const float q =
        C + (e[0] * d1 + e[1] * d2 + e[2] * d3 + e[3] * d4) * __builtin_amdgcn_rcpf(sum);
    // A face value outside the range of the two cells next to the face (a
    // confident but wrong prediction: an overshoot, or a material property
    // mixed into a pure fluid) takes the eq. (28) weights instead.
    if (q >= fminf(C, D_) && q <= fmaxf(C, D_)) {
      if (side) rr = T(q); else rl = T(q);
    } else {
      int nf = 0;
      if (side)
        rr = weno<T>(w[5], w[4], w[3], w[2], w[1], W_MODIFIED, eps, false, nf);
      else
        rl = weno<T>(w[0], w[1], w[2], w[3], w[4], W_MODIFIED, eps, false, nf);
      mr.fallbacks++;
    }
  }
}

template <typename T, int NDIM, int D, bool CUT = false, class S>
__device__ __forceinline__ void recon(const S& st, int sides, bool order3, int weights, T eps,
                                      T a, T b, double bd, double gd, double* ql, double* qr,
                                      int& nshort, MlpRun* mr = nullptr) {
  constexpr int NT = NDIM - 1, NC = 5 + NT;
  constexpr int CR = 0, CU = 1 + D, CP = 1 + NDIM, CG = 2 + NDIM, CPI = 3 + NDIM;
  // Fully unrolled over the fields (static register indices for the face
  // states, no loop-carried copies); the scheduling barrier keeps the
  // compiler from interleaving fields, which bounds register pressure.
#pragma unroll
  for (int m = 0; m < NC; m++) {
    __builtin_amdgcn_sched_barrier(0);
    // row of L: 0 = acoustic (sign sa), 1 = entropy, 2 = copy of component cx
    int kind = 2, cx = CG;
    T sa = a;
    if (m == 0) {
      kind = 0;
      sa = -a;
    } else if (m == NC - 1) {
      kind = 0;
    } else if (m == 1) {
      kind = 1;
    } else if (m < 2 + NT) {
      cx = 1 + ((m - 2) < D ? (m - 2) : (m - 1));
    } else if (m == 3 + NT) {
      cx = CPI;
    }
    T w[6];
#pragma unroll
    for (int j = 0; j < 6; j++) {
      if (kind == 0) {
        w[j] = sa * T(st(CU, j)) + T(0.5) * T(st(CP, j));
      } else if (kind == 1) {
        w[j] = T(st(CR, j)) - b * T(st(CP, j));
      } else {
        w[j] = T(st(cx, j));
      }
    }
    T rlm = T(0), rrm = T(0);
    // the material fields (Gamma, Pi) keep the eq. (28) weights: their
    // reconstruction decides the mixture at an interface
    const bool learned = mr != nullptr && !order3 && m != 2 + NT && m != 3 + NT;
    if (learned) mlp_field<T>(w, *mr, eps, rlm, rrm);
    const int wk = weights == W_MLP ? W_MODIFIED : weights;
#pragma unroll
    for (int side = 0; side < 2; side++) {
      if (!(sides & (1 << side))) continue;
      __builtin_amdgcn_sched_barrier(0);
      double* q = side ? qr : ql;
      const double r =
          learned ? double(side ? rrm : rlm)
          : side ? double(weno_sel<T, CUT>(w[5], w[4], w[3], w[2], w[1], wk, eps, order3, nshort))
                 : double(weno_sel<T, CUT>(w[0], w[1], w[2], w[3], w[4], wk, eps, order3, nshort));
      if (m == 0) {
        q[0] = bd * r;
        q[1] = (-gd) * r;
        q[2 + NT] = r;
      } else if (m == 1) {
        q[0] = q[0] + r;
      } else if (m == NC - 1) {
        q[0] = q[0] + bd * r;
        q[1] = q[1] + gd * r;
        q[2 + NT] = q[2 + NT] + r;
      } else {
#pragma unroll
        for (int t = 0; t < NT; t++)
          if (m == 2 + t) q[2 + t] = r;
        if (m == 2 + NT) q[3 + NT] = r;
        if (m == 3 + NT) q[4 + NT] = r;
      }
    }
  }
}

// Full face: average state, eigen-parameters, both reconstructions, MOOD
// cascade, HLLC.  F (face order) and us are written; o3/o1 report the
// orders used (per side), nshort the field-sides of the first pass whose
// reconstruction took its shortcut (weno<T>).
// The weights a stage kernel evaluates: the cut-off form in the kernels
// instantiated for it, else eq. (21) or eq. (28) as asked (those kernels
// never see W_CUTOFF, and the compiler knows it).
template <bool CUT>
__device__ __forceinline__ int kernel_weights(int w) {
  return CUT ? W_CUTOFF : (w == W_BASIC ? W_BASIC : W_MODIFIED);
}

template <typename T, int NDIM, int D, bool CUT = false, class S>
__device__ __forceinline__ void face_flux(const S& st, int weights, int mood,
                                          double eps, double* F, double& us,
                                          int& n3, int& n1, int& nshort,
                                          MlpRun* mr = nullptr) {
  constexpr int NT = NDIM - 1, NC = 5 + NT;
  constexpr int CR = 0, CP = 1 + NDIM, CG = 2 + NDIM, CPI = 3 + NDIM;
  // L_{i+1/2}: L of eq. (11) at the mean of the two primitive states.
  const double rb = 0.5 * (st(CR, 2) + st(CR, 3));
  const double pb = 0.5 * (st(CP, 2) + st(CP, 3));
  const double Gb = 0.5 * (st(CG, 2) + st(CG, 3));
  const double Pb = 0.5 * (st(CPI, 2) + st(CPI, 3));
  T a, b;
  double bd, gd;
  {
    const T c2 = sound2<T>(T(rb), T(pb), T(Gb), T(Pb));
    const T c = sqrt(c2);
    a = T(rb) * c / T(2);
    b = qdiv<T>(T(1), c2);
    bd = double(b);
    gd = div64<T>(1.0, double(T(rb) * c));
    if (sizeof(T) == 8) {
      bd = 1.0 / double(c2);
    }
  }
  double ql[NC], qr[NC];
  if (mr) mlp_material(Gb, Pb, mr->f6, mr->f7);
  nshort = 0;
  recon<T, NDIM, D, CUT>(st, 3, false, weights, T(eps), a, b, bd, gd, ql, qr, nshort, mr);
  n3 = 0;
  n1 = 0;
  if (mood) {
    // Sec. 3.4: redo a failing side without the 3-point stencils, then fall
    // back to the first-order state of eq. (32) (the cell's own primitive
    // state, since R L q_i = q_i).
    int fail = (admissible(ql[0], ql[2 + NT], ql[3 + NT], ql[4 + NT]) ? 0 : 1) |
               (admissible(qr[0], qr[2 + NT], qr[3 + NT], qr[4 + NT]) ? 0 : 2);
    if (mr && fail) {
      // learned weights: a failing side is first redone with the plain
      // 5th-order WENO-IS weights of eq. (28) (counted as a fallback of the
      // network); the cascade below then starts from that state
      int nfl = 0;
      recon<T, NDIM, D>(st, fail, false, W_MODIFIED, T(eps), a, b, bd, gd, ql, qr, nfl);
      mr->fallbacks += (fail & 1) + (fail >> 1);
      fail = (admissible(ql[0], ql[2 + NT], ql[3 + NT], ql[4 + NT]) ? 0 : 1) |
             (admissible(qr[0], qr[2 + NT], qr[3 + NT], qr[4 + NT]) ? 0 : 2);
    }
    if (fail) {
      int nf3 = 0;
      recon<T, NDIM, D, CUT>(st, fail, true, weights, T(eps), a, b, bd, gd, ql, qr, nf3);
#pragma unroll
      for (int side = 0; side < 2; side++) {
        if (!(fail & (1 << side))) continue;
        double* q = side ? qr : ql;
        // counted without a branch: a counter picked by a branch ends up
        // in private (scratch) memory on every face
        const int ok = admissible(q[0], q[2 + NT], q[3 + NT], q[4 + NT]) ? 1 : 0;
        if (!ok) {
          const int j = side ? 3 : 2;
#pragma unroll
          for (int k = 0; k < NC; k++) q[k] = st(axis_comp<NDIM, D>(k), j);
        }
        n3 += ok;
        n1 += 1 - ok;
      }
    }
  }
  T tl[NC], tr[NC], tF[NC], tus;
#pragma unroll
  for (int k = 0; k < NC; k++) {
    tl[k] = T(ql[k]);
    tr[k] = T(qr[k]);
  }
  hllc<T, NT>(tl, tr, tF, tus);
#pragma unroll
  for (int k = 0; k < NC; k++) F[k] = double(tF[k]);
  us = double(tus);
}

// The same face in two passes, for a kernel that gathers the faces the
// MOOD cascade needs and redoes them by full waves.  First pass: the
// 5th-order states and their check; a face with a failing side returns its
// fail bits (non-zero) and no flux.  Second pass (face_flux_redo, on the
// gathered faces): the 5th-order states are formed again (the same bits),
// the failing sides go through the cascade, then HLLC -- the flux that
// face_flux gives, bit for bit.
template <typename T, int NDIM, class S>
__device__ __forceinline__ void face_params(const S& st, T& a, T& b, double& bd, double& gd) {
  constexpr int CR = 0, CP = 1 + NDIM, CG = 2 + NDIM, CPI = 3 + NDIM;
  const double rb = 0.5 * (st(CR, 2) + st(CR, 3));
  const double pb = 0.5 * (st(CP, 2) + st(CP, 3));
  const double Gb = 0.5 * (st(CG, 2) + st(CG, 3));
  const double Pb = 0.5 * (st(CPI, 2) + st(CPI, 3));
  const T c2 = sound2<T>(T(rb), T(pb), T(Gb), T(Pb));
  const T c = sqrt(c2);
  a = T(rb) * c / T(2);
  b = qdiv<T>(T(1), c2);
  bd = double(b);
  gd = div64<T>(1.0, double(T(rb) * c));
  if (sizeof(T) == 8) {
    bd = 1.0 / double(c2);
  }
}

template <typename T, int NDIM, int D, bool CUT = false, class S>
__device__ __forceinline__ int face_flux_first(const S& st, int weights, double eps, double* F,
                                               double& us, int& nshort) {
  constexpr int NT = NDIM - 1, NC = 5 + NT;
  T a, b;
  double bd, gd;
  face_params<T, NDIM>(st, a, b, bd, gd);
  double ql[NC], qr[NC];
  nshort = 0;
  recon<T, NDIM, D, CUT>(st, 3, false, weights, T(eps), a, b, bd, gd, ql, qr, nshort);
  const int fail = (admissible(ql[0], ql[2 + NT], ql[3 + NT], ql[4 + NT]) ? 0 : 1) |
                   (admissible(qr[0], qr[2 + NT], qr[3 + NT], qr[4 + NT]) ? 0 : 2);
  if (fail) return fail;
  T tl[NC], tr[NC], tF[NC], tus;
#pragma unroll
  for (int k = 0; k < NC; k++) {
    tl[k] = T(ql[k]);
    tr[k] = T(qr[k]);
  }
  hllc<T, NT>(tl, tr, tF, tus);
#pragma unroll
  for (int k = 0; k < NC; k++) F[k] = double(tF[k]);
  us = double(tus);
  return 0;
}

template <typename T, int NDIM, int D, bool CUT = false, class S>
__device__ __forceinline__ void face_flux_redo(const S& st, int fail, int weights, double eps,
                                               double* F, double& us, int& n3, int& n1) {
  constexpr int NT = NDIM - 1, NC = 5 + NT;
  T a, b;
  double bd, gd;
  face_params<T, NDIM>(st, a, b, bd, gd);
  double ql[NC], qr[NC];
  int nsc = 0, nf3 = 0;
  recon<T, NDIM, D, CUT>(st, 3, false, weights, T(eps), a, b, bd, gd, ql, qr, nsc);
  recon<T, NDIM, D, CUT>(st, fail, true, weights, T(eps), a, b, bd, gd, ql, qr, nf3);
  n3 = 0;
  n1 = 0;
#pragma unroll
  for (int side = 0; side < 2; side++) {
    if (!(fail & (1 << side))) continue;
    double* q = side ? qr : ql;
    const int ok = admissible(q[0], q[2 + NT], q[3 + NT], q[4 + NT]) ? 1 : 0;
    if (!ok) {
      const int j = side ? 3 : 2;
#pragma unroll
      for (int k = 0; k < NC; k++) q[k] = st(axis_comp<NDIM, D>(k), j);
    }
    n3 += ok;
    n1 += 1 - ok;
  }
  T tl[NC], tr[NC], tF[NC], tus;
#pragma unroll
  for (int k = 0; k < NC; k++) {
    tl[k] = T(ql[k]);
    tr[k] = T(qr[k]);
  }
  hllc<T, NT>(tl, tr, tF, tus);
#pragma unroll
  for (int k = 0; k < NC; k++) F[k] = double(tF[k]);
  us = double(tus);
}

}  // namespace isw
