// Time-step reduction and the sweep launch entry point of the WENO-IS
// operator for gfx950.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "launch.hpp"
#include "sweep_kernels.hpp"

namespace isw {

// ---------------------------------------------------------------------------
// Time step in one launch: per-cell sum_d (|u_d| + c)/dx_d (cell_speed), the
// workgroup's max, then cfl_ticket: a device-wide max through an integer
// atomic on the doubles' bits and dt formed by the workgroup that finishes
// last.  The words start zero and are left zero.
// ---------------------------------------------------------------------------
constexpr int kCflThreads = 1024;
constexpr int kCflCells = 2;  // cells per lane and pass, loaded before any arithmetic
constexpr int kCflMax = 0, kCflTicket = 1;  // the time-step words

// One workgroup's end of the reduction (one lane): its max (bits) into the
// max word by an integer atomic, then a ticket; the workgroup holding the
// last of nblocks tickets forms dt = cfl / max (clipped to dt_max > 0),
// writes it and clears both words.
__device__ __forceinline__ void cfl_ticket(unsigned long long* w, unsigned long long bits,
                                           unsigned nblocks, double cfl, double dt_max,
                                           double* dt) {
  atomicMax(&w[kCflMax], bits);
  __threadfence();
  if (atomicAdd(&w[kCflTicket], 1ull) == nblocks - 1) {
    // every other workgroup's max precedes its ticket
    __threadfence();
    const double mx = __longlong_as_double((long long)atomicMax(&w[kCflMax], 0ull));
    double h = cfl / mx;
    if (dt_max > 0.0 && h > dt_max) h = dt_max;
    *dt = h;
    atomicExch(&w[kCflMax], 0ull);
    atomicExch(&w[kCflTicket], 0ull);
  }
}

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
      const double sp = cell_speed<NDIM>(q, dxs);
      m = (sp > m || sp != sp) ? sp : m;
    }
  }
  __shared__ unsigned long long red[kCflThreads / 64];
  wave_max_bits(m, red);
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long b = red[0];
    for (int w = 1; w < kCflThreads / 64; w++) b = red[w] > b ? red[w] : b;
    cfl_ticket(words, b, gridDim.x, cfl, dt_max, dt);
  }
}

// dt from the per-workgroup maxima the first fused 2D stage stored (one
// workgroup): the max over them, dt = cfl / max, clipped to dt_max > 0.
__global__ __launch_bounds__(kCflThreads) void cfl_final_kernel(const unsigned long long* part,
                                                                 int64_t n, double cfl,
                                                                 double dt_max, double* dt) {
  // eight loads in flight per lane (a 3D x sweep leaves tens of thousands)
  constexpr int UNR = 8;
  unsigned long long b = 0;
  for (int64_t i0 = threadIdx.x; i0 < n; i0 += (int64_t)kCflThreads * UNR) {
    unsigned long long v[UNR];
#pragma unroll
    for (int r = 0; r < UNR; r++) {
      const int64_t i = i0 + (int64_t)r * kCflThreads;
      v[r] = i < n ? part[i] : 0ull;
    }
#pragma unroll
    for (int r = 0; r < UNR; r++) b = v[r] > b ? v[r] : b;
  }
  __shared__ unsigned long long red[kCflThreads / 64];
  wave_max_bits(__longlong_as_double((long long)b), red);
  __syncthreads();
  if (threadIdx.x == 0) {
    b = red[0];
    for (int w = 1; w < kCflThreads / 64; w++) b = red[w] > b ? red[w] : b;
    double h = cfl / __longlong_as_double((long long)b);
    if (dt_max > 0.0 && h > dt_max) h = dt_max;
    *dt = h;
  }
}

int64_t sweep3d_x_tiles(const int64_t* n) {
  using TS = TileShape<3, 0>;
  return ((n[0] + TS::TL - 1) / TS::TL) * ((n[1] * n[2] + TS::TW - 1) / TS::TW);
}

hipError_t launch_cfl_final(const unsigned long long* part, int64_t n, double cfl,
                            double dt_max, double* dt, hipStream_t s, LaunchEvents ev) {
  if (n < 1) return hipErrorInvalidValue;
  if (ev.start)
    hipExtLaunchKernelGGL(cfl_final_kernel, dim3(1), dim3(kCflThreads), 0, s, ev.start, ev.stop, 0,
                          part, n, cfl, dt_max, dt);
  else
    hipLaunchKernelGGL(cfl_final_kernel, dim3(1), dim3(kCflThreads), 0, s, part, n, cfl, dt_max, dt);
  return hipGetLastError();
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
  return precision == 1 ? launch_sweep_f32(ndim, D, a, mode, readR, s, ev)
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
