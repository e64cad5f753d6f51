// Learned nonlinear weights: training data, bf16 MFMA forward/backward,
// Adam, and packing for the stage kernel (isweno_mlp_*).
#include <hip/hip_runtime.h>

#include "ctx.hpp"
#include "isweno.h"
#include "mlp.hpp"
#include "sweep.hpp"

namespace isw {

constexpr int MLP_WAVES = 4;  // waves per workgroup in the training kernels

// Scale of the value error in the loss and tolerance of the confidence
// label, in units of the stencil's range (the inputs are normalised to it).
constexpr float kValueScale = 0.01f;
constexpr float kConfTol = 0.005f;

// Candidates of eq. (20) on a normalised stencil a..e = v_{i-2}..v_{i+2}.
__device__ __forceinline__ void candidates(float a, float b, float c, float d, float e,
                                           float* q) {
  q[0] = 0.5f * c + 0.5f * d;
  q[1] = -0.5f * b + 1.5f * c;
  q[2] = (1.0f / 3.0f) * c + (5.0f / 6.0f) * d - (1.0f / 6.0f) * e;
  q[3] = (1.0f / 3.0f) * a - (7.0f / 6.0f) * b + (11.0f / 6.0f) * c;
}

// Per-sample loss (unscaled) and logit gradient (scaled by 1/n).  Per side
// h: qhat_h = sum_k softmax(z_h)_k c_hk, q_h = sum_k y_hk c_hk with c_hk the
// candidates on the normalised stencil x (left from x0..x4, right from the
// mirror x5..x1); loss ((qhat_h - q_h) / kValueScale)^2.  Plus binary
// cross-entropy of the confidence logit against c; c < 0 asks for the
// label to be formed here: 1 when both |qhat_h - q_h| < kConfTol, else 0.
__device__ __forceinline__ float sample_loss(const float* z, const float* y, const float* x,
                                             float c, float inv_n, float* dz) {
  float loss = 0.0f, err = 0.0f;
#pragma unroll
  for (int h = 0; h < 2; h++) {
    const float* zh = z + 4 * h;
    float cand[4];
    if (h == 0)
      candidates(x[0], x[1], x[2], x[3], x[4], cand);
    else
      candidates(x[5], x[4], x[3], x[2], x[1], cand);
    float m = zh[0];
#pragma unroll
    for (int k = 1; k < 4; k++) m = fmaxf(m, zh[k]);
    float e[4], s = 0.0f;
#pragma unroll
    for (int k = 0; k < 4; k++) {
      e[k] = __expf(zh[k] - m);
      s += e[k];
    }
    float qh = 0.0f, qt = 0.0f;
#pragma unroll
    for (int k = 0; k < 4; k++) {
      e[k] = e[k] / s;
      qh += e[k] * cand[k];
      qt += y[4 * h + k] * cand[k];
    }
    const float r = (qh - qt) * (1.0f / kValueScale);
    loss += r * r;
    err = fmaxf(err, fabsf(qh - qt));
    const float g = 2.0f * r * (1.0f / kValueScale) * inv_n;
#pragma unroll
    for (int k = 0; k < 4; k++) dz[4 * h + k] = g * e[k] * (cand[k] - qh);
  }
  if (c < 0.0f) c = err < kConfTol ? 1.0f : 0.0f;
  const float zc = z[8];
  const float sig = 1.0f / (1.0f + __expf(-zc));
  loss += fmaxf(zc, 0.0f) - zc * c + log1pf(__expf(-fabsf(zc)));
  dz[8] = (sig - c) * inv_n;
  return loss;
}

// Forward + backward over n samples; each workgroup writes its partial
// gradient (and loss) to part[blockIdx.x][MLP_NPARAM + 1].
__global__ __launch_bounds__(64 * MLP_WAVES) void mlp_grad_kernel(
    const float* __restrict__ P, const float* __restrict__ X, const float* __restrict__ Y,
    const float* __restrict__ Cc, int64_t n, float* __restrict__ part) {
  __shared__ MlpLds W;
  __shared__ MlpTile tiles[MLP_WAVES];
  __shared__ uint16_t dzb[MLP_WAVES][32 * 16];   // dz (bf16), 16 columns (9 used)
  __shared__ uint16_t dh2[MLP_WAVES][32 * MLP_H];
  __shared__ uint16_t dh1[MLP_WAVES][32 * MLP_H];
  __shared__ float red[MLP_WAVES][MLP_NPARAM + 1];
  const int tid = threadIdx.x, wave = tid >> 6, l = tid & 63;
  mlp_stage_f32(W, P, tid, blockDim.x);
  __syncthreads();
  MlpTile& T = tiles[wave];
  const float inv_n = 1.0f / (float)n;
  f32x16 g1 = zero16(), g2 = zero16(), g3 = zero16();
  float gb1 = 0.0f, gb2 = 0.0f, gb3 = 0.0f, loss = 0.0f;
  const int64_t ntile = (n + 31) / 32;
  for (int64_t t = (int64_t)blockIdx.x * MLP_WAVES + wave; t < ntile;
       t += (int64_t)gridDim.x * MLP_WAVES) {
    const int64_t s0 = t * 32;
    for (int e = l; e < 32 * MLP_NI; e += 64) {
      const int64_t s = s0 + e / MLP_NI;
      T.x[e] = f2bf(s < n ? X[s * MLP_NI + e % MLP_NI] : 0.0f);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    mlp_tile_forward(W, T);
    // loss and dz: lanes 0..31 own one sample each
    if (l < 32) {
      const int64_t s = s0 + l;
      float dz[9];
      if (s < n) {
        float z[9], y[8], xs[MLP_NI];
#pragma unroll
        for (int k = 0; k < 9; k++) z[k] = T.z[l * 16 + k];
#pragma unroll
        for (int k = 0; k < 8; k++) y[k] = Y[s * 8 + k];
#pragma unroll
        for (int k = 0; k < MLP_NI; k++) xs[k] = X[s * MLP_NI + k];
        loss += sample_loss(z, y, xs, Cc ? Cc[s] : -1.0f, inv_n, dz) * inv_n;
      } else {
#pragma unroll
        for (int k = 0; k < 9; k++) dz[k] = 0.0f;
      }
#pragma unroll
      for (int k = 0; k < 16; k++) {
        const float v = k < 9 ? dz[k] : 0.0f;
        dzb[wave][l * 16 + k] = f2bf(v);
        T.z[l * 16 + k] = v;  // float dz for the bias gradient
      }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    // gb3[j] = sum_s dz[s][j]
    if (l < 9) {
      float s = 0.0f;
      for (int i = 0; i < 32; i++) s += T.z[i * 16 + l];
      gb3 += s;
    }
    // gW3[j][k] += sum_s dz[s][j] h2[s][k]
    g3 = mma32<32>(g3, [&](int i, int s) { return i < 16 ? dzb[wave][s * 16 + i] : (uint16_t)0; },
                   [&](int s, int k) { return T.h2[s * MLP_H + k]; });
    // dh2[s][k] = (sum_j dz[s][j] W3[j][k]) * relu'(h2)
    f32x16 acc = mma32<16>(zero16(), [&](int s, int j) { return dzb[wave][s * 16 + j]; },
                           [&](int j, int k) { return W.w3[j * MLP_H + k]; });
    float cs = 0.0f;
#pragma unroll
    for (int r = 0; r < 16; r++) {
      const int s = mrow(l, r), k = mcol(l);
      const float v = bf2f(T.h2[s * MLP_H + k]) > 0.0f ? acc[r] : 0.0f;
      cs += v;
      dh2[wave][s * MLP_H + k] = f2bf(v);
    }
    cs += __shfl_xor(cs, 32);
    if (l < 32) gb2 += cs;
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    // gW2[j][k] += sum_s dh2[s][j] h1[s][k]
    g2 = mma32<32>(g2, [&](int j, int s) { return dh2[wave][s * MLP_H + j]; },
                   [&](int s, int k) { return T.h1[s * MLP_H + k]; });
    // dh1[s][k] = (sum_j dh2[s][j] W2[j][k]) * relu'(h1)
    acc = mma32<32>(zero16(), [&](int s, int j) { return dh2[wave][s * MLP_H + j]; },
                    [&](int j, int k) { return W.w2[j * MLP_H + k]; });
    cs = 0.0f;
#pragma unroll
    for (int r = 0; r < 16; r++) {
      const int s = mrow(l, r), k = mcol(l);
      const float v = bf2f(T.h1[s * MLP_H + k]) > 0.0f ? acc[r] : 0.0f;
      cs += v;
      dh1[wave][s * MLP_H + k] = f2bf(v);
    }
    cs += __shfl_xor(cs, 32);
    if (l < 32) gb1 += cs;
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    // gW1[j][k] += sum_s dh1[s][j] x[s][k]
    g1 = mma32<32>(g1, [&](int j, int s) { return dh1[wave][s * MLP_H + j]; },
                   [&](int s, int k) { return k < MLP_NI ? T.x[s * MLP_NI + k] : (uint16_t)0; });
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
  }
  // per-wave results -> red[wave][...]
  float* R = red[wave];
#pragma unroll
  for (int r = 0; r < 16; r++) {
    const int i = mrow(l, r), k = mcol(l);
    if (k < MLP_NI) R[P_W1 + i * MLP_NI + k] = g1[r];
    R[P_W2 + i * MLP_H + k] = g2[r];
    if (i < MLP_NO) R[P_W3 + i * MLP_H + k] = g3[r];
  }
  if (l < 32) {
    R[P_B1 + l] = gb1;
    R[P_B2 + l] = gb2;
  }
  if (l < MLP_NO) R[P_B3 + l] = gb3;
  // wave loss: sum over lanes
  float ls = loss;
  for (int o = 32; o > 0; o >>= 1) ls += __shfl_xor(ls, o);
  if (l == 0) R[MLP_NPARAM] = ls;
  __syncthreads();
  for (int e = tid; e < MLP_NPARAM + 1; e += blockDim.x) {
    float s = 0.0f;
#pragma unroll
    for (int w = 0; w < MLP_WAVES; w++) s += red[w][e];
    part[(int64_t)blockIdx.x * (MLP_NPARAM + 1) + e] = s;
  }
}

// Fixed-order sum of the workgroup partials.
__global__ void mlp_reduce_kernel(const float* part, int nblk, float* grad, float* loss) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e > MLP_NPARAM) return;
  float s = 0.0f;
  for (int b = 0; b < nblk; b++) s += part[(int64_t)b * (MLP_NPARAM + 1) + e];
  if (e < MLP_NPARAM)
    grad[e] = s;
  else
    *loss = s;
}

// The network as the stage kernel evaluates it (packed bf16 parameters,
// activations in registers, 64 samples per wave): one sample per lane,
// lanes past n evaluate zeros and store nothing.
__global__ __launch_bounds__(256) void mlp_infer_kernel(const uint16_t* packed, const float* X,
                                                       int64_t n, float* out) {
  __shared__ MlpLds W;
  __shared__ MlpBiasLds B;
  const int tid = threadIdx.x;
  mlp_stage_bf16(W, packed, tid, 256);
  __syncthreads();
  mlp_bias_stage(B, W, tid, 256);
  MlpRegs R;
  mlp_regs_load(W, R);
  __syncthreads();
  const int64_t s = (int64_t)blockIdx.x * 256 + tid;
  float x[MLP_NI], z[MLP_NO];
#pragma unroll
  for (int k = 0; k < MLP_NI; k++) x[k] = s < n ? X[s * MLP_NI + k] : 0.0f;
  mlp_logits_wave(x, R, B, z);
  if (s < n) {
#pragma unroll
    for (int k = 0; k < MLP_NO; k++) out[s * MLP_NO + k] = z[k];
  }
}

__global__ __launch_bounds__(64 * MLP_WAVES) void mlp_forward_kernel(const float* P,
                                                                     const float* X, int64_t n,
                                                                     float* out) {
  __shared__ MlpLds W;
  __shared__ MlpTile tiles[MLP_WAVES];
  const int tid = threadIdx.x, wave = tid >> 6, l = tid & 63;
  mlp_stage_f32(W, P, tid, blockDim.x);
  __syncthreads();
  MlpTile& T = tiles[wave];
  const int64_t ntile = (n + 31) / 32;
  for (int64_t t = (int64_t)blockIdx.x * MLP_WAVES + wave; t < ntile;
       t += (int64_t)gridDim.x * MLP_WAVES) {
    const int64_t s0 = t * 32;
    for (int e = l; e < 32 * MLP_NI; e += 64) {
      const int64_t s = s0 + e / MLP_NI;
      T.x[e] = f2bf(s < n ? X[s * MLP_NI + e % MLP_NI] : 0.0f);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    mlp_tile_forward(W, T);
    for (int e = l; e < 32 * MLP_NO; e += 64) {
      const int64_t s = s0 + e / MLP_NO;
      if (s < n) out[s * MLP_NO + e % MLP_NO] = T.z[(e / MLP_NO) * 16 + e % MLP_NO];
    }
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
  }
}

__global__ void mlp_adam_kernel(float* P, const float* G, float* M, float* V, float lr, float b1,
                                float b2, float eps, float c1, float c2) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= MLP_NPARAM) return;
  const float g = G[e];
  const float m = b1 * M[e] + (1.0f - b1) * g;
  const float v = b2 * V[e] + (1.0f - b2) * g * g;
  M[e] = m;
  V[e] = v;
  P[e] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

__global__ void mlp_pack_kernel(const float* P, uint16_t* out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < MLP_NPARAM) out[e] = f2bf(P[e]);
}

// Training samples: for every face of every axis and every characteristic
// field, the network inputs and the eq. (28) weights of both sides (FP64,
// read straight from global memory; this is data preparation, not the hot
// path).  Face-field g (axis-major, then face, then field) is taken when
// g % stride == 0 and written at row g / stride < max.
template <int NDIM>
__global__ void mlp_samples_kernel(const double* U, int64_t n0, int64_t n1, int64_t n2, int bclo0,
                                   int bchi0, int bclo1, int bchi1, int bclo2, int bchi2,
                                   double eps, int64_t stride, int64_t maxs, float* X, float* Y) {
  constexpr int NC = 4 + NDIM, NT = NDIM - 1;
  const int64_t n[3] = {n0, n1, n2};
  const int bl[3] = {bclo0, bclo1, bclo2}, bh[3] = {bchi0, bchi1, bchi2};
  const int64_t N = n0 * n1 * n2;
  int64_t base = 0;
  for (int D = 0; D < NDIM; D++) {
    const int64_t nf = N / n[D] * (n[D] + 1);
    for (int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; f < nf;
         f += (int64_t)gridDim.x * blockDim.x) {
      const int64_t g0 = (base + f) * NC;
      // any of this face's fields selected?
      const int64_t first = ((g0 + stride - 1) / stride) * stride;
      if (first >= g0 + NC || first / stride >= maxs) continue;
      // face f: index along D and the line it sits on
      const int64_t fl = f % (n[D] + 1), line = f / (n[D] + 1);
      int64_t sL = 1, sA = 0, sT = 0, a = 0, tt = 0;
      if (D == 0) {
        sL = 1; a = line; sA = n0;
      } else if (D == 1) {
        sL = n0; a = line % n0; sA = 1; tt = line / n0; sT = n0 * n1;
      } else {
        sL = n0 * n1; a = line % n0; sA = 1; tt = line / n0; sT = n0;
      }
      double q[6][NC];
      for (int j = 0; j < 6; j++) {
        bool flip;
        const int64_t li = bc_index(fl - 3 + j, n[D], bl[D], bh[D], flip);
        cell_prim<NDIM>(U, N, a * sA + li * sL + tt * sT, q[j]);
        if (flip) q[j][1 + D] = -q[j][1 + D];
      }
      const double rb = 0.5 * (q[2][0] + q[3][0]), pb = 0.5 * (q[2][1 + NDIM] + q[3][1 + NDIM]);
      const double Gb = 0.5 * (q[2][2 + NDIM] + q[3][2 + NDIM]);
      const double Pb = 0.5 * (q[2][3 + NDIM] + q[3][3 + NDIM]);
      const double c2 = sound2<double>(rb, pb, Gb, Pb), c = sqrt(c2);
      const double aa = rb * c / 2.0, b = 1.0 / c2;
      for (int m = 0; m < NC; m++) {
        const int64_t g = g0 + m;
        if (g % stride || g / stride >= maxs) continue;
        double w[6];
        for (int j = 0; j < 6; j++) {
          if (m == 0) w[j] = (-aa) * q[j][1 + D] + 0.5 * q[j][1 + NDIM];
          else if (m == NC - 1) w[j] = aa * q[j][1 + D] + 0.5 * q[j][1 + NDIM];
          else if (m == 1) w[j] = q[j][0] - b * q[j][1 + NDIM];
          else if (m < 2 + NT) w[j] = q[j][1 + ((m - 2) < D ? (m - 2) : (m - 1))];
          else if (m == 2 + NT) w[j] = q[j][2 + NDIM];
          else w[j] = q[j][3 + NDIM];
        }
        const int64_t row = g / stride;
        float x[8], f6, f7;
        mlp_material(Gb, Pb, f6, f7);
        mlp_features<double>(w, f6, f7, x);
        for (int k = 0; k < 8; k++) X[row * 8 + k] = x[k];
        for (int side = 0; side < 2; side++) {
          double v[5];
          for (int k = 0; k < 5; k++) v[k] = side ? w[5 - k] : w[k];
          const Ind<double> s = indicators<double>(v[0], v[1], v[2], v[3], v[4]);
          const Alpha al = alphas_f64(s, W_MODIFIED, eps, false);
          const double sum = ((al.a1 + al.a2) + al.a3) + al.a4;
          Y[row * 8 + 4 * side + 0] = float(al.a1 / sum);
          Y[row * 8 + 4 * side + 1] = float(al.a2 / sum);
          Y[row * 8 + 4 * side + 2] = float(al.a3 / sum);
          Y[row * 8 + 4 * side + 3] = float(al.a4 / sum);
        }
      }
    }
    base += nf;
  }
}

}  // namespace isw

namespace {
int grad_blocks(int64_t n) {
  int64_t b = (n + 32 * isw::MLP_WAVES - 1) / (32 * isw::MLP_WAVES);
  if (b > 1024) b = 1024;
  if (b < 1) b = 1;
  return (int)b;
}
}  // namespace

extern "C" {

int isweno_mlp_samples(isweno_ctx* ctx, const isweno_grid* g, const isweno_opts* o, const double* U,
                       float* X, float* Y, int64_t max_samples, int64_t stride, int64_t* count,
                       void* stream) {
  if (!ctx || !g || !o || !U || !X || !Y || !count || max_samples < 1 || stride < 1)
    return ISWENO_ERR_ARG;
  int r;
  // the same grid and option checks as the solver: the sampler stages the
  // same ghost cells (a reflective end needs at least 3 cells)
  if ((r = isw::check_grid(g)) != ISWENO_OK) return r;
  if ((r = isw::check_opts(o)) != ISWENO_OK) return r;
  if (hipSetDevice(ctx->device) != hipSuccess) return ISWENO_ERR_DEVICE;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int64_t N = g->n[0] * g->n[1] * g->n[2];
  int64_t total = 0;
  for (int d = 0; d < g->ndim; d++) total += N / g->n[d] * (g->n[d] + 1) * (4 + g->ndim);
  const int64_t rows = (total + stride - 1) / stride;
  const int64_t written = rows < max_samples ? rows : max_samples;
  const dim3 grid(1024), block(256);
  if (g->ndim == 1)
    hipLaunchKernelGGL(isw::mlp_samples_kernel<1>, grid, block, 0, s, U, g->n[0], g->n[1], g->n[2],
                       g->bc_lo[0], g->bc_hi[0], g->bc_lo[1], g->bc_hi[1], g->bc_lo[2],
                       g->bc_hi[2], o->eps, stride, max_samples, X, Y);
  else if (g->ndim == 2)
    hipLaunchKernelGGL(isw::mlp_samples_kernel<2>, grid, block, 0, s, U, g->n[0], g->n[1], g->n[2],
                       g->bc_lo[0], g->bc_hi[0], g->bc_lo[1], g->bc_hi[1], g->bc_lo[2],
                       g->bc_hi[2], o->eps, stride, max_samples, X, Y);
  else
    hipLaunchKernelGGL(isw::mlp_samples_kernel<3>, grid, block, 0, s, U, g->n[0], g->n[1], g->n[2],
                       g->bc_lo[0], g->bc_hi[0], g->bc_lo[1], g->bc_hi[1], g->bc_lo[2],
                       g->bc_hi[2], o->eps, stride, max_samples, X, Y);
  if (hipGetLastError() != hipSuccess) return ISWENO_ERR_DEVICE;
  if (hipMemcpyAsync(count, &written, sizeof(int64_t), hipMemcpyHostToDevice, s) != hipSuccess)
    return ISWENO_ERR_DEVICE;
  return hipStreamSynchronize(s) == hipSuccess ? ISWENO_OK : ISWENO_ERR_DEVICE;
}

int isweno_mlp_infer(isweno_ctx* ctx, const uint16_t* packed, const float* X, int64_t n,
                     float* out, void* stream) {
  if (!ctx || !packed || !X || !out || n < 0) return ISWENO_ERR_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return ISWENO_ERR_DEVICE;
  if (n == 0) return ISWENO_OK;
  const int64_t blocks = (n + 255) / 256;
  if (blocks > 0x7fffffffLL) return ISWENO_ERR_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(isw::mlp_infer_kernel, dim3((unsigned)blocks), dim3(256), 0, s, packed, X, n,
                     out);
  return hipGetLastError() == hipSuccess ? ISWENO_OK : ISWENO_ERR_DEVICE;
}

int isweno_mlp_forward(isweno_ctx* ctx, const float* P, const float* X, int64_t n, float* out,
                       void* stream) {
  if (!ctx || !P || !X || !out || n < 0) return ISWENO_ERR_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return ISWENO_ERR_DEVICE;
  if (n == 0) return ISWENO_OK;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(isw::mlp_forward_kernel, dim3(grad_blocks(n)), dim3(64 * isw::MLP_WAVES), 0,
                     s, P, X, n, out);
  return hipGetLastError() == hipSuccess ? ISWENO_OK : ISWENO_ERR_DEVICE;
}

int isweno_mlp_loss_grad(isweno_ctx* ctx, const float* P, const float* X, const float* Y,
                         const float* Cc, int64_t n, float* loss, float* grad, void* stream) {
  if (!ctx || !P || !X || !Y || !loss || !grad || n < 1) return ISWENO_ERR_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return ISWENO_ERR_DEVICE;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int nb = grad_blocks(n);
  // partial gradients in the context's own buffer (grown on demand; calls
  // on one context do not overlap, see isweno.h)
  if (nb > ctx->mlp_part_blocks) {
    if (ctx->mlp_part) {
      if (hipDeviceSynchronize() != hipSuccess) return ISWENO_ERR_DEVICE;
      (void)hipFree(ctx->mlp_part);
      ctx->mlp_part = nullptr;
      ctx->mlp_part_blocks = 0;
    }
    if (hipMalloc(&ctx->mlp_part, sizeof(float) * (size_t)nb * (isw::MLP_NPARAM + 1)) !=
        hipSuccess)
      return ISWENO_ERR_DEVICE;
    ctx->mlp_part_blocks = nb;
  }
  hipLaunchKernelGGL(isw::mlp_grad_kernel, dim3(nb), dim3(64 * isw::MLP_WAVES), 0, s, P, X, Y, Cc,
                     n, ctx->mlp_part);
  if (hipGetLastError() != hipSuccess) return ISWENO_ERR_DEVICE;
  hipLaunchKernelGGL(isw::mlp_reduce_kernel, dim3((isw::MLP_NPARAM + 1 + 255) / 256), dim3(256), 0,
                     s, ctx->mlp_part, nb, grad, loss);
  return hipGetLastError() == hipSuccess ? ISWENO_OK : ISWENO_ERR_DEVICE;
}

int isweno_mlp_adam(isweno_ctx* ctx, float* P, const float* G, float* M, float* V, int32_t step,
                    float lr, float beta1, float beta2, float eps, void* stream) {
  if (!ctx || !P || !G || !M || !V || step < 1) return ISWENO_ERR_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return ISWENO_ERR_DEVICE;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const float c1 = 1.0f - powf(beta1, (float)step), c2 = 1.0f - powf(beta2, (float)step);
  hipLaunchKernelGGL(isw::mlp_adam_kernel, dim3((isw::MLP_NPARAM + 255) / 256), dim3(256), 0, s, P,
                     G, M, V, lr, beta1, beta2, eps, c1, c2);
  return hipGetLastError() == hipSuccess ? ISWENO_OK : ISWENO_ERR_DEVICE;
}

int isweno_mlp_pack(isweno_ctx* ctx, const float* P, uint16_t* packed, void* stream) {
  if (!ctx || !P || !packed) return ISWENO_ERR_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return ISWENO_ERR_DEVICE;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(isw::mlp_pack_kernel, dim3((isw::MLP_NPARAM + 255) / 256), dim3(256), 0, s, P,
                     packed);
  return hipGetLastError() == hipSuccess ? ISWENO_OK : ISWENO_ERR_DEVICE;
}

}  // extern "C"
