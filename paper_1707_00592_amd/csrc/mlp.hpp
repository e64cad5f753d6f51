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

// ---------------------------------------------------------------------------
// Inference inside the stage kernel, activations in registers.
//
// Layers are computed transposed, h^T = W x^T, so that the 32 samples of a
// tile are the columns: lane l then holds, for sample l % 32, the output
// rows 8 (r / 4) + 4 (l / 32) + r % 4 in accumulator r, which are exactly the
// K entries 8 q + 4 (l / 32) + t (q = r / 4, t = r % 4) that it has to supply
// as the B operand of the next layer's q-th 8-wide slice.  Only the network
// inputs (and the logits) cross between the two halves of the wave.
// ---------------------------------------------------------------------------

// A operands of the three layers as lane l supplies them: row l % 32,
// K entries 4 (l / 32) + t of every 8-wide slice (W3 rows 9..31 are zero).
struct MlpRegs {
  bf16x4 w1, w2[4], w3[4];
};

// Biases in LDS, arranged as the accumulator registers of each wave half.
struct alignas(16) MlpBiasLds {
  float b[3][2][16];
};

__device__ __forceinline__ void mlp_regs_load(const MlpLds& W, MlpRegs& R) {
  const int l = threadIdx.x & 63, i = l & 31, kh = (l >> 5) * 4;
#pragma unroll
  for (int t = 0; t < 4; t++) R.w1[t] = (short)W.w1[i * MLP_NI + kh + t];
#pragma unroll
  for (int q = 0; q < 4; q++) {
#pragma unroll
    for (int t = 0; t < 4; t++) {
      R.w2[q][t] = (short)W.w2[i * MLP_H + 8 * q + kh + t];
      R.w3[q][t] = (short)W.w3[i * MLP_H + 8 * q + kh + t];
    }
  }
}

// Whole workgroup, after W is staged; the caller synchronises.
__device__ __forceinline__ void mlp_bias_stage(MlpBiasLds& B, const MlpLds& W, int tid, int nthr) {
  for (int e = tid; e < 3 * 2 * 16; e += nthr) {
    const int layer = e / 32, half = (e / 16) & 1, r = e & 15;
    const int row = 8 * (r >> 2) + 4 * half + (r & 3);
    B.b[layer][half][r] = layer == 0 ? W.b1[row] : (layer == 1 ? W.b2[row] : W.b3[row]);
  }
}

__device__ __forceinline__ f32x16 mlp_bias_acc(const MlpBiasLds& B, int layer) {
  const int half = (threadIdx.x & 63) >> 5;
  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; r++) acc[r] = B.b[layer][half][r];
  return acc;
}

typedef int i32x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));

// Four floats to bf16 (round to nearest even, the hardware conversion).
__device__ __forceinline__ bf16x4 pack_bf16x4(float a, float b, float c, float d) {
  const bf16x2v lo = __builtin_convertvector((f32x2){a, b}, bf16x2v);
  const bf16x2v hi = __builtin_convertvector((f32x2){c, d}, bf16x2v);
  i32x2 u;
  u[0] = __builtin_bit_cast(int, lo);
  u[1] = __builtin_bit_cast(int, hi);
  return __builtin_bit_cast(bf16x4, u);
}

// max(x, 0) in one integer instruction: negative floats (sign bit set) are
// negative as integers, non-negative ones keep their order.
__device__ __forceinline__ float relu(float x) {
  const int i = __builtin_bit_cast(int, x);
  return __builtin_bit_cast(float, i > 0 ? i : 0);
}

// One 32-sample tile: xb is this lane's layer-1 B operand (inputs
// 4 (l / 32) + t of sample l % 32).  Returns the layer-3 accumulators:
// lanes 0..31 hold logits 0..3 (r = 0..3) and 8 (r = 4) of sample l, lanes
// 32..63 logits 4..7 (r = 0..3) of sample l - 32.
__device__ __forceinline__ f32x16 mlp_tile_regs(const MlpRegs& R, const MlpBiasLds& B,
                                                bf16x4 xb) {
  __builtin_amdgcn_sched_barrier(0);
  f32x16 acc = mlp_bias_acc(B, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(R.w1, xb, acc, 0, 0, 0);
  bf16x4 h[4];
#pragma unroll
  for (int q = 0; q < 4; q++)
    h[q] = pack_bf16x4(relu(acc[4 * q]), relu(acc[4 * q + 1]), relu(acc[4 * q + 2]),
                       relu(acc[4 * q + 3]));
  acc = mlp_bias_acc(B, 1);
#pragma unroll
  for (int q = 0; q < 4; q++) acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(R.w2[q], h[q], acc, 0, 0, 0);
#pragma unroll
  for (int q = 0; q < 4; q++)
    h[q] = pack_bf16x4(relu(acc[4 * q]), relu(acc[4 * q + 1]), relu(acc[4 * q + 2]),
                       relu(acc[4 * q + 3]));
  acc = mlp_bias_acc(B, 2);
#pragma unroll
  for (int q = 0; q < 4; q++) acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(R.w3[q], h[q], acc, 0, 0, 0);
  return acc;
}


// Exchange with the lane 32 apart (the other half of the wave).
__device__ __forceinline__ bf16x4 shfl_xor32(bf16x4 v);

// Logits z[9] of this lane's sample x[8]: the 64 samples of the wave run as
// two 32-sample tiles (every lane must call; tile 0 holds the samples of
// lanes 0..31, tile 1 those of lanes 32..63).
__device__ __forceinline__ void mlp_logits_wave(const float* x, const MlpRegs& R,
                                                const MlpBiasLds& B, float* z);

__device__ __forceinline__ bf16x4 shfl_xor32(bf16x4 v) {
  i32x2 u = __builtin_bit_cast(i32x2, v);
  u[0] = __shfl_xor(u[0], 32);
  u[1] = __shfl_xor(u[1], 32);
  return __builtin_bit_cast(bf16x4, u);
}

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

__device__ __forceinline__ void mlp_logits_wave(const float* x, const MlpRegs& R,
                                                const MlpBiasLds& B, float* z) {
  const bool upper = (threadIdx.x & 32) != 0;
  const bf16x4 lo = pack_bf16x4(x[0], x[1], x[2], x[3]);
  const bf16x4 hi = pack_bf16x4(x[4], x[5], x[6], x[7]);
  // tile 0 needs inputs 4..7 of the lower lanes' samples from the upper
  // lanes, tile 1 inputs 0..3 of the upper lanes' samples from the lower ones
  const bf16x4 recv = shfl_xor32(upper ? lo : hi);
  // only accumulators 0..4 of each tile are used (the rest die at once)
  float t0[5], t1[5];
  {
    const f32x16 a = mlp_tile_regs(R, B, upper ? recv : lo);
#pragma unroll
    for (int k = 0; k < 5; k++) t0[k] = a[k];
  }
  {
    const f32x16 a = mlp_tile_regs(R, B, upper ? hi : recv);
#pragma unroll
    for (int k = 0; k < 5; k++) t1[k] = a[k];
  }
  // lower lanes own logits 0..3 and 8 of tile 0 and hold those of tile 1's
  // samples; upper lanes own logits 4..7 of tile 1 and hold those of tile 0's
  float sendv[5], got[5];
#pragma unroll
  for (int k = 0; k < 5; k++) sendv[k] = upper ? (k < 4 ? t0[k] : 0.0f) : t1[k];
#pragma unroll
  for (int k = 0; k < 5; k++) got[k] = __shfl_xor(sendv[k], 32);
#pragma unroll
  for (int k = 0; k < 4; k++) {
    z[k] = upper ? got[k] : t0[k];
    z[4 + k] = upper ? t1[k] : got[k];
  }
  z[8] = upper ? got[4] : t0[4];
}

// Learned-weights state of one wave inside the stage kernel.
struct MlpRun {
  const MlpRegs* R;
  const MlpBiasLds* B;
  float thr;       // confidence threshold (sigmoid of the last logit)
  float f6, f7;    // material inputs of the current face
  int fallbacks;   // face-fields that used the eq. (28) weights instead
};

}  // namespace isw
