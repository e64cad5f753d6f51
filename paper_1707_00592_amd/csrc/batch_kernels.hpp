// Kernels of the batched 1D path (isweno_batch_*): the stage kernel and its
// launch templates, instantiated by batch.hip (FP64) and batch_f32.hip (the
// float form, built with multiply-add contraction).
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <new>
#include <tuple>
#include <vector>

#include "isweno.h"
#include "sweep.hpp"

namespace isw {

struct BatchArgs {
  const double* Uin;
  const double* U0;
  double* Uout;
  const double* dt;        // per problem
  const double* dx;        // per problem
  const int64_t* offsets;  // nprob + 1
  const int64_t* tstart;   // first cell of each tile
  const int32_t* tprob;    // problem of each tile
  int64_t ntiles, total;
  const int32_t* active;   // per problem: advanced in this step (set by the dt kernel)
  int32_t* pstatus;        // per problem: sticky status
  StatsDev* stats;
  int bc_lo, bc_hi, weights, mood;
  double eps;
};

template <typename E>
struct Lds1 {
  const E* base;
  int cstride;
  __device__ __forceinline__ E operator()(int c, int j) const {
    return base[c * cstride + j];
  }
};

template <typename T, int TL, int MODE, bool CUT>
__global__ __launch_bounds__(TL + 1) void batch_stage_kernel(BatchArgs g) {
  constexpr int NC = 5, NP = TL + 6, NF = TL + 1, NTHR = TL + 1;
  // FP64 primitives and the face values, both in the arithmetic's type (the
  // float form reconstructs from float values and its fluxes are float)
  __shared__ T sq[NC * NP];
  __shared__ T sf[(NC + 1) * NF];
  __shared__ int s_status;
  const int tid = threadIdx.x;
  if (tid == 0) s_status = ST_OK;
  __syncthreads();
  const int64_t total = g.total;
  int my3 = 0, my1 = 0;
  for (int64_t t = blockIdx.x; t < g.ntiles; t += gridDim.x) {
    const int prob = g.tprob[t];
    // problems that were non-physical when this step began are frozen (the
    // flag is written before the step's stages and not during them, so the
    // branch is the same for every lane and every stage of the step)
    if (!g.active[prob]) continue;
    const int64_t lo = g.offsets[prob], n = g.offsets[prob + 1] - lo;
    const int64_t l0 = g.tstart[t] - lo;
    const int len = (int)((n - l0) < TL ? (n - l0) : TL);
    bool bad = false;
    // FP64: raised instruction priority while the tile is staged (its loads
    // go out ahead of the other workgroups' arithmetic), normal afterwards
    if constexpr (sizeof(T) == 8) __builtin_amdgcn_s_setprio(1);
    for (int p = tid; p < NP; p += NTHR) {
      const int64_t l = l0 + p - 3;
      if (l >= n + 3) continue;
      bool flip;
      const int64_t li = bc_index(l, n, g.bc_lo, g.bc_hi, flip);
      double q[NC];
      cell_prim<1, T>(g.Uin, total, lo + li, q);
      if (p >= 3 && p < 3 + len) bad = bad || !cell_ok<1>(g.Uin, total, lo + li, q);
      if (flip) q[1] = -q[1];
#pragma unroll
      for (int c = 0; c < NC; c++) sq[c * NP + p] = T(q[c]);
    }
    if (bad) {
      s_status = ST_NONPHYSICAL;
      atomicExch(&g.pstatus[prob], (int32_t)ST_NONPHYSICAL);
    }
    __syncthreads();
    if constexpr (sizeof(T) == 8) __builtin_amdgcn_s_setprio(0);
    for (int j = tid; j <= len; j += NTHR) {
      Lds1<T> st;
      st.base = &sq[j];
      st.cstride = NP;
      double F[NC], us;
      int n3, n1, nf;
      face_flux<T, 1, 0, CUT>(st, kernel_weights<CUT>(g.weights), g.mood, g.eps, F, us, n3, n1,
                              nf);
      if (j < len || l0 + j == n) {  // count each face of a problem once
        my3 += n3;
        my1 += n1;
      }
#pragma unroll
      for (int k = 0; k < NC; k++) sf[k * NF + j] = T(F[k]);
      sf[NC * NF + j] = T(us);
    }
    __syncthreads();
    const Div64<T> bydx(g.dx[prob]);
    const double h = g.dt[prob];
    for (int j = tid; j < len; j += NTHR) {
      const int64_t cell = lo + l0 + j;
#pragma unroll
      for (int k = 0; k < NC; k++) {
        double r = bydx(-(double(sf[k * NF + j + 1]) - double(sf[k * NF + j])));
        if (k >= 3)
          r = r + bydx(double(sq[k * NP + j + 3]) *
                       (double(sf[NC * NF + j + 1]) - double(sf[NC * NF + j])));
        const int64_t o = k * total + cell;
        if (MODE == OUT_RK1) {
          g.Uout[o] = g.U0[o] + h * r;
        } else if (MODE == OUT_RK2) {
          g.Uout[o] = 0.75 * g.U0[o] + 0.25 * (g.Uin[o] + h * r);
        } else {
          g.Uout[o] = (1.0 / 3.0) * g.U0[o] + (2.0 / 3.0) * (g.Uin[o] + h * r);
        }
      }
    }
    __syncthreads();  // LDS is reused by the next tile
  }
  if (g.stats) {
    if (my3) atomicAdd(&g.stats->o3[0], (unsigned long long)my3);
    if (my1) atomicAdd(&g.stats->o1[0], (unsigned long long)my1);
    if (tid == 0 && s_status != ST_OK) atomicExch(&g.stats->status, s_status);
  }
}

// Start of a step, one workgroup per problem: a problem is advanced in this
// step when its status is still OK (active[p]); then, when cfl > 0,
// dt[p] = cfl / max_cells (|u| + c)/dx_p (clipped to dt_max).  Frozen
// problems keep their last dt.

template <typename T, int TL, bool CUT>
static hipError_t launch_stage_c(const BatchArgs& a, int mode, int blocks, hipStream_t s) {
  if (mode == OUT_RK1)
    hipLaunchKernelGGL((batch_stage_kernel<T, TL, OUT_RK1, CUT>), dim3(blocks), dim3(TL + 1), 0,
                       s, a);
  else if (mode == OUT_RK2)
    hipLaunchKernelGGL((batch_stage_kernel<T, TL, OUT_RK2, CUT>), dim3(blocks), dim3(TL + 1), 0,
                       s, a);
  else
    hipLaunchKernelGGL((batch_stage_kernel<T, TL, OUT_RK3, CUT>), dim3(blocks), dim3(TL + 1), 0,
                       s, a);
  return hipGetLastError();
}

// the cut-off weights in kernels of their own (register allocation of the
// other forms unchanged)
template <typename T, int TL>
static hipError_t launch_stage_tl(const BatchArgs& a, int mode, int blocks, hipStream_t s) {
  return a.weights == W_CUTOFF ? launch_stage_c<T, TL, true>(a, mode, blocks, s)
                               : launch_stage_c<T, TL, false>(a, mode, blocks, s);
}

template <typename T>
static hipError_t launch_stage_t(int tl, const BatchArgs& a, int mode, int blocks,
                                 hipStream_t s) {
  // the tile list was cut for exactly this tile length (a kernel for a
  // shorter one would overrun its LDS on the list's longer tiles)
  if (blocks < 1) return hipErrorInvalidValue;
  switch (tl) {
    case 63: return launch_stage_tl<T, 63>(a, mode, blocks, s);
    case 127: return launch_stage_tl<T, 127>(a, mode, blocks, s);
    case 255: return launch_stage_tl<T, 255>(a, mode, blocks, s);
    default: return hipErrorInvalidValue;
  }
}

// The float form's instantiations (batch_f32.hip).
hipError_t launch_batch_stage_f32(int tl, const BatchArgs& a, int mode, int blocks, hipStream_t s);

}  // namespace isw
