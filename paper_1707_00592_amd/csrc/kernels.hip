// Time-step reduction and the sweep launch entry point of the WENO-IS
// operator for gfx950.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "launch.hpp"
#include "sweep_kernels.hpp"

namespace isw {

// ---------------------------------------------------------------------------
// Time step: per-cell sum_d (|u_d| + c)/dx_d, block max, then a device-wide
// max through an integer atomic on the (positive) double's bits.
// ---------------------------------------------------------------------------
template <int NDIM>
__global__ __launch_bounds__(256) void cfl_reduce_kernel(
    const double* U, int64_t n0, int64_t n1, int64_t n2, double dx0,
    double dx1, double dx2, unsigned long long* maxbits) {
  constexpr int NC = 4 + NDIM;
  constexpr int UNR = 4;  // cells per lane and pass, loaded before any arithmetic
  const int64_t N = n0 * n1 * n2;
  const double dxs[3] = {dx0, dx1, dx2};
  double m = 0.0;
  const int64_t span = (int64_t)blockDim.x * UNR;
  for (int64_t c0 = blockIdx.x * span + threadIdx.x; c0 < N; c0 += (int64_t)gridDim.x * span) {
    double u[UNR][NC];
#pragma unroll
    for (int r = 0; r < UNR; r++) {
      const int64_t c = c0 + (int64_t)r * blockDim.x;
#pragma unroll
      for (int k = 0; k < NC; k++) u[r][k] = c < N ? U[k * N + c] : 1.0;
    }
#pragma unroll
    for (int r = 0; r < UNR; r++) {
      if (c0 + (int64_t)r * blockDim.x >= N) continue;
      double q[NC];
      cons_prim<NDIM>(u[r], q);
      const double cs = sqrt(sound2<double>(q[0], q[1 + NDIM], q[2 + NDIM], q[3 + NDIM]));
      double s = (fabs(q[1]) + cs) / dxs[0];
#pragma unroll
      for (int a = 1; a < NDIM; a++) s = s + (fabs(q[1 + a]) + cs) / dxs[a];
      m = (s > m || s != s) ? s : m;
    }
  }
  __shared__ double red[256];
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      const double x = red[threadIdx.x + o];
      if (x > red[threadIdx.x] || x != x) red[threadIdx.x] = x;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(maxbits, (unsigned long long)__double_as_longlong(red[0]));
}

__global__ void cfl_finalize_kernel(unsigned long long* maxbits, double cfl,
                                    double dt_max, double* dt) {
  const double m = __longlong_as_double((long long)*maxbits);
  double h = cfl / m;
  if (dt_max > 0.0 && h > dt_max) h = dt_max;
  *dt = h;
  *maxbits = 0ull;
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

__global__ void zero_u64_kernel(unsigned long long* w) { *w = 0ull; }

hipError_t launch_zero_u64(unsigned long long* w, hipStream_t s) {
  hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(1), 0, s, w);
  return hipGetLastError();
}

hipError_t launch_cfl(int ndim, const double* U, const int64_t* n, const double* dx,
                      double cfl, double dt_max, unsigned long long* maxbits, double* dt,
                      int ncu, hipStream_t s, LaunchEvents ev) {
  if (n[0] < 1 || n[1] < 1 || n[2] < 1 || ncu < 1) return hipErrorInvalidValue;
  const int64_t N = n[0] * n[1] * n[2];
  int64_t blocks = (N + 1023) / 1024;
  // one workgroup per CU: every workgroup ends in one atomic on the same
  // word, and those serialise (measured: the kernel time grows by about
  // 10 ns per workgroup)
  const int64_t cap = (int64_t)ncu;
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  // events (timing only, never captured): start of the reduction, end of
  // the finalisation
  const dim3 grid((unsigned)blocks), block(256);
  auto reduce = [&](auto kern) {
    if (ev.start)
      hipExtLaunchKernelGGL(kern, grid, block, 0, s, ev.start, nullptr, 0, U, n[0], n[1], n[2],
                            dx[0], dx[1], dx[2], maxbits);
    else
      hipLaunchKernelGGL(kern, grid, block, 0, s, U, n[0], n[1], n[2], dx[0], dx[1], dx[2],
                         maxbits);
  };
  if (ndim == 1)
    reduce(cfl_reduce_kernel<1>);
  else if (ndim == 2)
    reduce(cfl_reduce_kernel<2>);
  else
    reduce(cfl_reduce_kernel<3>);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (ev.stop)
    hipExtLaunchKernelGGL(cfl_finalize_kernel, dim3(1), dim3(1), 0, s, nullptr, ev.stop, 0,
                          maxbits, cfl, dt_max, dt);
  else
    hipLaunchKernelGGL(cfl_finalize_kernel, dim3(1), dim3(1), 0, s, maxbits, cfl, dt_max, dt);
  return hipGetLastError();
}

}  // namespace isw
