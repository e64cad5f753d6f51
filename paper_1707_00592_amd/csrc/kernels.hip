// Time-step reduction and the sweep launch entry point of the WENO-IS
// operator for gfx950.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "launch.hpp"
#include "sweep_kernels.hpp"

namespace isw {

// ---------------------------------------------------------------------------
// Time step in one launch: per-cell sum_d (|u_d| + c)/dx_d, the workgroup's
// max, a device-wide max through an integer atomic on the bits of the
// (positive) doubles, which order as the doubles do (a NaN above every
// number), and dt formed by the workgroup that finishes last, found by a
// ticket counter.  words[kCflMax] and words[kCflTicket] start zero and are
// left zero.
// ---------------------------------------------------------------------------
constexpr int kCflThreads = 1024;
constexpr int kCflCells = 2;  // cells per lane and pass, loaded before any arithmetic

template <int NDIM>
__global__ __launch_bounds__(kCflThreads) void cfl_kernel(
    const double* U, int64_t n0, int64_t n1, int64_t n2, double dx0, double dx1, double dx2,
    double cfl, double dt_max, unsigned long long* words, double* dt) {
  constexpr int NC = 4 + NDIM;
  const int64_t N = n0 * n1 * n2;
  const double dxs[3] = {dx0, dx1, dx2};
  double m = 0.0;
  const int64_t span = (int64_t)kCflThreads * kCflCells;
  for (int64_t c0 = blockIdx.x * span + threadIdx.x; c0 < N; c0 += (int64_t)gridDim.x * span) {
    double u[kCflCells][NC];
#pragma unroll
    for (int r = 0; r < kCflCells; r++) {
      const int64_t c = c0 + (int64_t)r * kCflThreads;
#pragma unroll
      for (int k = 0; k < NC; k++) u[r][k] = c < N ? U[k * N + c] : 1.0;
    }
#pragma unroll
    for (int r = 0; r < kCflCells; r++) {
      if (c0 + (int64_t)r * kCflThreads >= N) continue;
      double q[NC];
      cons_prim<NDIM>(u[r], q);
      const double cs = sqrt(sound2<double>(q[0], q[1 + NDIM], q[2 + NDIM], q[3 + NDIM]));
      double sp = (fabs(q[1]) + cs) / dxs[0];
#pragma unroll
      for (int a = 1; a < NDIM; a++) sp = sp + (fabs(q[1 + a]) + cs) / dxs[a];
      m = (sp > m || sp != sp) ? sp : m;
    }
  }
  unsigned long long b = (unsigned long long)__double_as_longlong(m);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long x = __shfl_xor(b, o);
    b = x > b ? x : b;
  }
  __shared__ unsigned long long red[kCflThreads / 64];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = b;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kCflThreads / 64; w++) b = red[w] > b ? red[w] : b;
    atomicMax(&words[kCflMax], b);
    __threadfence();
    if (atomicAdd(&words[kCflTicket], 1ull) == gridDim.x - 1) {
      // every other workgroup's max precedes its ticket
      __threadfence();
      const double mx = __longlong_as_double((long long)atomicMax(&words[kCflMax], 0ull));
      double h = cfl / mx;
      if (dt_max > 0.0 && h > dt_max) h = dt_max;
      *dt = h;
      atomicExch(&words[kCflMax], 0ull);
      atomicExch(&words[kCflTicket], 0ull);
    }
  }
}

hipError_t launch_sweep(int precision, int ndim, int D, const SweepArgs& a, int mode,
                        bool readR, hipStream_t s, LaunchEvents ev) {
  if (a.weights == W_MLP) {
    // learned weights: float32 reconstruction with a packed network only
    if (precision != 1 || !a.mlp) return hipErrorInvalidValue;
    return launch_sweep_p<float, true, false>(ndim, D, a, mode, readR, s, ev);
  }
  // the cut-off weights run in kernels of their own (another translation
  // unit), so that the other forms keep their register allocation
  if (a.weights == W_CUTOFF) return launch_sweep_cut(precision, ndim, D, a, mode, readR, s, ev);
  return precision == 1 ? launch_sweep_p<float, false, false>(ndim, D, a, mode, readR, s, ev)
                        : launch_sweep_p<double, false, false>(ndim, D, a, mode, readR, s, ev);
}

__global__ void zero_cfl_kernel(unsigned long long* w) {
  w[kCflMax] = 0ull;
  w[kCflTicket] = 0ull;
}

hipError_t launch_zero_cfl(unsigned long long* w, hipStream_t s) {
  hipLaunchKernelGGL(zero_cfl_kernel, dim3(1), dim3(1), 0, s, w);
  return hipGetLastError();
}

hipError_t launch_cfl(int ndim, const double* U, const int64_t* n, const double* dx,
                      double cfl, double dt_max, unsigned long long* words, double* dt,
                      int ncu, hipStream_t s, LaunchEvents ev) {
  if (n[0] < 1 || n[1] < 1 || n[2] < 1 || ncu < 1) return hipErrorInvalidValue;
  const int64_t N = n[0] * n[1] * n[2];
  int64_t blocks = (N + kCflThreads * kCflCells - 1) / (kCflThreads * kCflCells);
  // one workgroup per CU at most: every workgroup ends in atomics on the
  // same two words
  if (blocks > (int64_t)ncu) blocks = ncu;
  if (blocks < 1) blocks = 1;
  const dim3 grid((unsigned)blocks), block(kCflThreads);
  auto go = [&](auto kern) {
    if (ev.start)
      hipExtLaunchKernelGGL(kern, grid, block, 0, s, ev.start, ev.stop, 0, U, n[0], n[1], n[2],
                            dx[0], dx[1], dx[2], cfl, dt_max, words, dt);
    else
      hipLaunchKernelGGL(kern, grid, block, 0, s, U, n[0], n[1], n[2], dx[0], dx[1], dx[2], cfl,
                         dt_max, words, dt);
  };
  if (ndim == 1)
    go(cfl_kernel<1>);
  else if (ndim == 2)
    go(cfl_kernel<2>);
  else
    go(cfl_kernel<3>);
  return hipGetLastError();
}

}  // namespace isw
