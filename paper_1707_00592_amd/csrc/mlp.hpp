// Small dense network (8 -> 32 -> 32 -> 9, ReLU) on bf16 matrix cores.
//
// Shared by the training kernels and by the learned-weights stage kernel.
// Tiles of 32 samples: y[32 x N] += x[32 x K] * W^T[K x N] with
// v_mfma_f32_32x32x8bf16_1k (wave64): lane l supplies A[l%32][4*(l/32)+t]
// and B[4*(l/32)+t][l%32], t = 0..3, per 8-wide K slice, and holds
// D[8*(r/4) + 4*(l/32) + r%4][l%32] in accumulator r = 0..15.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace isw {

constexpr int MLP_NI = 8, MLP_H = 32, MLP_NO = 9;
// parameter offsets (float32 master layout of isweno.h)
constexpr int P_W1 = 0, P_B1 = P_W1 + MLP_H * MLP_NI, P_W2 = P_B1 + MLP_H,
              P_B2 = P_W2 + MLP_H * MLP_H, P_W3 = P_B2 + MLP_H, P_B3 = P_W3 + MLP_NO * MLP_H,
              MLP_NPARAM = P_B3 + MLP_NO;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// float -> bf16 bits, round to nearest even (finite inputs).
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

__device__ __forceinline__ int mrow(int lane, int r) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }
__device__ __forceinline__ int mcol(int lane) { return lane & 31; }

// acc += A(32 x K) B(K x 32); fa(i, k), fb(k, j) return bf16 bits.
template <int K, class FA, class FB>
__device__ __forceinline__ f32x16 mma32(f32x16 acc, FA fa, FB fb) {
  const int l = threadIdx.x & 63, i = l & 31, kh = (l >> 5) * 4;
#pragma unroll
  for (int kb = 0; kb < K; kb += 8) {
    bf16x4 a, b;
#pragma unroll
    for (int t = 0; t < 4; t++) {
      a[t] = (short)fa(i, kb + kh + t);
      b[t] = (short)fb(kb + kh + t, i);
    }
    acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
  }
  return acc;
}

__device__ __forceinline__ f32x16 zero16() {
  f32x16 z;
#pragma unroll
  for (int r = 0; r < 16; r++) z[r] = 0.0f;
  return z;
}

// Weights staged in LDS as bf16 (W3 padded to 32 rows with zeros) plus
// float biases.
struct MlpLds {
  uint16_t w1[MLP_H * MLP_NI];
  uint16_t w2[MLP_H * MLP_H];
  uint16_t w3[32 * MLP_H];
  float b1[MLP_H], b2[MLP_H], b3[32];
};

// Per-wave activations of one 32-sample tile.
struct MlpTile {
  uint16_t x[32 * MLP_NI];
  uint16_t h1[32 * MLP_H];
  uint16_t h2[32 * MLP_H];
  float z[32 * 16];  // logits (9 used); reused for dz in training
};

// Forward pass of one tile (all 64 lanes of the wave take part): x (bf16,
// 32 x 8) -> h1, h2 (bf16 after ReLU, 32 x 32) -> z (float logits, 32 x 16,
// 9 used).  z may alias h1 (h1 is dead once h2 is formed).
__device__ __forceinline__ void mlp_forward32(const MlpLds& W, const uint16_t* x, uint16_t* h1,
                                              uint16_t* h2, float* z) {
  const int l = threadIdx.x & 63;
  f32x16 acc = mma32<MLP_NI>(zero16(), [&](int i, int k) { return x[i * MLP_NI + k]; },
                             [&](int k, int j) { return W.w1[j * MLP_NI + k]; });
#pragma unroll
  for (int r = 0; r < 16; r++) {
    const float v = acc[r] + W.b1[mcol(l)];
    h1[mrow(l, r) * MLP_H + mcol(l)] = f2bf(v > 0.0f ? v : 0.0f);
  }
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_wave_barrier();
  acc = mma32<MLP_H>(zero16(), [&](int i, int k) { return h1[i * MLP_H + k]; },
                     [&](int k, int j) { return W.w2[j * MLP_H + k]; });
#pragma unroll
  for (int r = 0; r < 16; r++) {
    const float v = acc[r] + W.b2[mcol(l)];
    h2[mrow(l, r) * MLP_H + mcol(l)] = f2bf(v > 0.0f ? v : 0.0f);
  }
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_wave_barrier();
  acc = mma32<MLP_H>(zero16(), [&](int i, int k) { return h2[i * MLP_H + k]; },
                     [&](int k, int j) { return W.w3[j * MLP_H + k]; });
#pragma unroll
  for (int r = 0; r < 16; r++) {
    const int j = mcol(l);
    if (j < 16) z[mrow(l, r) * 16 + j] = acc[r] + W.b3[j];
  }
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ void mlp_tile_forward(const MlpLds& W, MlpTile& T) {
  mlp_forward32(W, T.x, T.h1, T.h2, T.z);
}

// Per-wave scratch for inference inside the stage kernel (z over h1).
struct MlpInfTile {
  uint16_t x[32 * MLP_NI];
  uint16_t h2[32 * MLP_H];
  union {
    uint16_t h1[32 * MLP_H];
    float z[32 * 16];
  };
};

// Stage float32 master parameters into LDS (whole workgroup; caller syncs).
__device__ __forceinline__ void mlp_stage_f32(MlpLds& W, const float* P, int tid, int nthr) {
  for (int e = tid; e < MLP_H * MLP_NI; e += nthr) W.w1[e] = f2bf(P[P_W1 + e]);
  for (int e = tid; e < MLP_H * MLP_H; e += nthr) W.w2[e] = f2bf(P[P_W2 + e]);
  for (int e = tid; e < 32 * MLP_H; e += nthr)
    W.w3[e] = e < MLP_NO * MLP_H ? f2bf(P[P_W3 + e]) : (uint16_t)0;
  for (int e = tid; e < MLP_H; e += nthr) {
    W.b1[e] = P[P_B1 + e];
    W.b2[e] = P[P_B2 + e];
  }
  for (int e = tid; e < 32; e += nthr) W.b3[e] = e < MLP_NO ? P[P_B3 + e] : 0.0f;
}

// Same from the packed bf16 layout (biases converted back to float).
__device__ __forceinline__ void mlp_stage_bf16(MlpLds& W, const uint16_t* P, int tid, int nthr) {
  for (int e = tid; e < MLP_H * MLP_NI; e += nthr) W.w1[e] = P[P_W1 + e];
  for (int e = tid; e < MLP_H * MLP_H; e += nthr) W.w2[e] = P[P_W2 + e];
  for (int e = tid; e < 32 * MLP_H; e += nthr)
    W.w3[e] = e < MLP_NO * MLP_H ? P[P_W3 + e] : (uint16_t)0;
  for (int e = tid; e < MLP_H; e += nthr) {
    W.b1[e] = bf2f(P[P_B1 + e]);
    W.b2[e] = bf2f(P[P_B2 + e]);
  }
  for (int e = tid; e < 32; e += nthr) W.b3[e] = e < MLP_NO ? bf2f(P[P_B3 + e]) : 0.0f;
}

// Material inputs of a face: its gamma as (gamma - 1)/4 and its Pinf as
// log10(1 + Pinf/1e5)/4, from the averaged Gamma and Pi.
__device__ __forceinline__ void mlp_material(double Gb, double Pb, float& f6, float& f7) {
  const double gamma = 1.0 + 1.0 / Gb;
  const double pinf = Pb / (Gb + 1.0);
  f6 = float((gamma - 1.0) * 0.25);
  f7 = float(log10(1.0 + (pinf > 0.0 ? pinf : 0.0) / 1e5) * 0.25);
}

// Network inputs for one characteristic field at one face: the six stencil
// values scaled to [0, 1] by their range (all zero for a flat stencil, i.e.
// a range of at most 1e-30) and the two material inputs.
template <typename T>
__device__ __forceinline__ void mlp_features(const T* w, float f6, float f7, float* x) {
  T lo = w[0], hi = w[0];
#pragma unroll
  for (int j = 1; j < 6; j++) {
    lo = w[j] < lo ? w[j] : lo;
    hi = w[j] > hi ? w[j] : hi;
  }
  const T rng = hi - lo;
  // ranges below 1e-30 count as flat: their reciprocal would overflow the
  // float features (and 0 * inf gives NaN)
  const float inv = rng > T(1e-30) ? float(T(1) / rng) : 0.0f;
#pragma unroll
  for (int j = 0; j < 6; j++) x[j] = float(w[j] - lo) * inv;
  x[6] = f6;
  x[7] = f7;
}

// Learned-weights state of one wave inside the stage kernel.
struct MlpRun {
  const MlpLds* W;
  MlpInfTile* T;
  float thr;       // confidence threshold (sigmoid of the last logit)
  float f6, f7;    // material inputs of the current face
  int fallbacks;   // face-fields that used the eq. (28) weights instead
};

}  // namespace isw
