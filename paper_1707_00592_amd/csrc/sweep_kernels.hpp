// Sweep kernels of the WENO-IS operator (one axis of a stage per launch) and
// their launch templates, shared by the translation units that instantiate
// them: the eq. (21)/(28) and learned-weight forms, and the cut-off form.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <type_traits>

#include "launch.hpp"
#include "sweep.hpp"

namespace isw {

// LDS accessor for a stencil: component c at stencil position j (0..5).
template <typename E>
struct LdsStencil {
  const E* base;  // component 0, position 0
  int cstride, pstride;
  __device__ __forceinline__ E operator()(int c, int j) const {
    return base[c * cstride + j * pstride];
  }
};

// The same with the two material rows (Gamma, Pi) stored before the others:
// base points at component 0, which is row 2; Gamma and Pi sit NC rows
// before their component number.
template <int NC, typename E>
struct LdsStencilMatFirst {
  const E* base;  // component 0 (row 2), position 0
  int cstride, pstride;
  __device__ __forceinline__ E operator()(int c, int j) const {
    const int r = c >= NC - 2 ? c - NC : c;
    return base[r * cstride + j * pstride];
  }
};

// Tile geometry of a sweep along axis D.  Cells are addressed as
// a*sA + l*sL + t*sT with l along D, a across (x for D > 0, the combined
// (y,z) line index for D = 0) and t the remaining axis.
template <int NDIM, int D>
struct Geo {
  int64_t nL, nA, nT, sL, sA, sT;
  __device__ __forceinline__ Geo(const int64_t* n) {
    if (D == 0) {
      nL = n[0]; sL = 1;
      nA = n[1] * n[2]; sA = n[0];
      nT = 1; sT = 0;
    } else if (D == 1) {
      nL = n[1]; sL = n[0];
      nA = n[0]; sA = 1;
      nT = n[2]; sT = n[0] * n[1];
    } else {
      nL = n[2]; sL = n[0] * n[1];
      nA = n[0]; sA = 1;
      nT = n[1]; sT = n[0];
    }
  }
};

// Tile of workgroup b among ntiles.  Workgroups go to the 8 XCDs in turn
// (b mod 8), each XCD with its own L2; tiles are numbered with the sweep
// axis fastest, so consecutive tiles share halo lines.  Each XCD takes runs
// of kSweepRun consecutive tiles, the runs of the 8 XCDs interleaved (the
// work of a front stays spread over the XCDs); tiles past the last whole
// group of 8 runs keep their own number.  A bijection of [0, ntiles).
constexpr int64_t kSweepRun = 64;
__device__ __forceinline__ int64_t sweep_tile(int64_t b, int64_t ntiles) {
  const int64_t whole = ntiles / (8 * kSweepRun) * (8 * kSweepRun);
  if (b >= whole) return b;
  const int64_t xcd = b & 7, k = b >> 3;
  return ((k / kSweepRun) * 8 + xcd) * kSweepRun + k % kSweepRun;
}

template <typename T, int NDIM, int D, int TL, int TW, int NTHR, int MODE,
          bool READ_R, bool CUT>
__global__ __launch_bounds__(NTHR, MODE == OUT_PARTIAL_S ? 5 : 1) void sweep_kernel(SweepArgs g) {
  constexpr int NC = 4 + NDIM;
  constexpr int NP = TL + 6;     // staged positions along D
  constexpr int NF = TL + 1;     // faces along D per tile row
  static_assert(TW * NF == NTHR, "one face per thread");
  // One LDS buffer, two phases.  Faces read the staged primitives sq
  // (recovered in FP64, staged in the arithmetic's type: the float form
  // reconstructs from float values anyway); the cells read the face values
  // sf (fluxes and u*, in the arithmetic's type: the float form's fluxes are
  // float values, so float storage is exact) and only the Gamma and Pi rows
  // of sq.  In 3D (ALIAS) the rows are stored
  // in the order (Gamma, Pi, rho, u..., p), sf starts after the first two
  // and overwrites the others once every face is evaluated (33 -> 21 KB per
  // FP64 workgroup, 4 -> 5 waves per SIMD); in 1D and 2D registers bound the
  // occupancy anyway, the rows keep the component order and sf follows sq.
  // Layouts: D = 0 -> [row][w][p]; D > 0 -> [row][p][w].
  constexpr bool ALIAS = NDIM == 3;
  constexpr int QROW = TW * NP;
  constexpr int SQ_BYTES = NC * QROW * (int)sizeof(T);
  constexpr int SF_OFF = ALIAS ? 2 * QROW * (int)sizeof(T) : SQ_BYTES;
  constexpr int SF_BYTES = (NC + 1) * TW * NF * (int)sizeof(T);
  constexpr int LDS_BYTES = SQ_BYTES > SF_OFF + SF_BYTES ? SQ_BYTES : SF_OFF + SF_BYTES;
  __shared__ __attribute__((aligned(16))) unsigned char lds[LDS_BYTES];
  T* const sq = reinterpret_cast<T*>(lds);
  T* const sf = reinterpret_cast<T*>(lds + SF_OFF);
  __shared__ int s_status;
  __shared__ int s_skip;
  // OUT_PARTIAL_S: this x sweep also finds its tile's max wave speed (the
  // step's time step; the tiles of an x sweep hold every cell once)
  constexpr bool SPEEDS = MODE == OUT_PARTIAL_S;
  __shared__ unsigned long long s_red[SPEEDS ? NTHR / 64 : 1];

  const Geo<NDIM, D> geo(g.n);
  const int64_t ntl = (geo.nL + TL - 1) / TL;
  const int64_t nta = (geo.nA + TW - 1) / TW;
  const int64_t bid = sweep_tile(blockIdx.x, ntl * nta * geo.nT);
  const int64_t tl = bid % ntl;
  const int64_t rest = bid / ntl;
  const int64_t ta = rest % nta;
  const int64_t tt = rest / nta;
  const int64_t l0 = tl * TL, a0 = ta * TW;
  const int64_t N = g.n[0] * g.n[1] * g.n[2];
  const int tid = threadIdx.x;
  if (tid == 0) {
    s_status = ST_OK;
    // sticky failure: one read per workgroup so that all lanes agree
    s_skip = g.stats ? (__atomic_load_n(&g.stats->status, __ATOMIC_RELAXED) != ST_OK) : 0;
  }
  __syncthreads();
  if (s_skip) {
    if (SPEEDS && tid == 0) g.cflp[blockIdx.x] = 0ull;
    return;
  }

  auto lidx = [](int c, int w, int p) {
    const int r = !ALIAS ? c : c >= NC - 2 ? c - (NC - 2) : c + 2;
    return D == 0 ? (r * TW + w) * NP + p : (r * NP + p) * TW + w;
  };
  auto fidx = [](int k, int w, int j) {
    return D == 0 ? (k * TW + w) * NF + j : (k * NF + j) * TW + w;
  };

  // FP64: raised instruction priority while the tile is staged (its loads
  // go out ahead of the resident workgroups' arithmetic), normal afterwards
  // (the float sweeps ran slower with it)
  if constexpr (sizeof(T) == 8) __builtin_amdgcn_s_setprio(1);
  // 1. stage primitives (FP64) with ghost cells
  bool bad = false;
  double m = 0.0;  // SPEEDS: the lane's max wave speed
  const double dxs[3] = {g.dx[0], g.dx[1], g.dx[2]};
  for (int e = tid; e < TW * NP; e += NTHR) {
    const int w = D == 0 ? e / NP : e % TW;
    const int p = D == 0 ? e % NP : e / TW;
    const int64_t a = a0 + w;
    const int64_t l = l0 + p - 3;
    if (a >= geo.nA || l >= geo.nL + 3) continue;
    bool flip;
    const int64_t li = bc_index(l, geo.nL, g.bc_lo, g.bc_hi, flip);
    const int64_t cell = a * geo.sA + li * geo.sL + tt * geo.sT;
    double q[NC];
    cell_prim<NDIM, T>(g.Uin, N, cell, q);
    if (p >= 3 && p < 3 + TL && l < geo.nL) {
      bad = bad || !cell_ok<NDIM>(g.Uin, N, cell, q);
      if constexpr (SPEEDS) {
        const double sp = cell_speed<NDIM, T>(q, dxs);
        m = (sp > m || sp != sp) ? sp : m;
      }
    }
    if (flip) q[1 + D] = -q[1 + D];
#pragma unroll
    for (int c = 0; c < NC; c++) sq[lidx(c, w, p)] = T(q[c]);
  }
  if constexpr (SPEEDS) wave_max_bits(m, s_red);
  if (bad) s_status = ST_NONPHYSICAL;
  __syncthreads();
  if constexpr (sizeof(T) == 8) __builtin_amdgcn_s_setprio(0);
  if constexpr (SPEEDS) {
    if (tid == 0) {
      unsigned long long b = s_red[0];
      for (int w = 1; w < NTHR / 64; w++) b = s_red[w] > b ? s_red[w] : b;
      g.cflp[blockIdx.x] = b;
    }
  }

  // 2. faces: thread tid owns face (w, j); with ALIAS the values wait in
  // registers until every face has read sq
  int my3 = 0, my1 = 0, mys = 0;
  // FP64 x tiles of 8 rows x 32 faces: each wave takes an 8 x 8 block, so a
  // front across x splits fewer waves between the linear-weight form and
  // the general one (x sweep -2% in 2D, -4% in 3D; the float form, whose
  // flat-stencil return saves less, measured slower with it)
  constexpr bool BLOCKED = D == 0 && TW == 8 && NF == 32 && sizeof(T) == 8;
  const int fw = BLOCKED ? (tid & 63) >> 3 : D == 0 ? tid / NF : tid % TW;
  const int fj = BLOCKED ? ((tid >> 6) << 3) | (tid & 7) : D == 0 ? tid % NF : tid / TW;
  const bool fvalid = a0 + fw < geo.nA && l0 + fj <= geo.nL;
  double F[NC], us;
  if (fvalid) {
    const int64_t gl = l0 + fj;  // face index along D (between gl-1 and gl)
    std::conditional_t<ALIAS, LdsStencilMatFirst<NC, T>, LdsStencil<T>> st;
    st.base = &sq[lidx(0, fw, fj)];
    st.cstride = D == 0 ? TW * NP : NP * TW;
    st.pstride = D == 0 ? 1 : TW;
    int n3, n1, nf;
    face_flux<T, NDIM, D, CUT>(st, kernel_weights<CUT>(g.weights), g.mood, g.eps, F, us, n3, n1,
                          nf);
    // the face on a tile boundary is evaluated by both tiles; count it once
    // (in the tile to its right, or the last tile for the domain's last face)
    if (fj < TL || gl == geo.nL) {
      my3 += n3;
      my1 += n1;
      mys += nf;
    }
    if constexpr (!ALIAS) {
#pragma unroll
      for (int k = 0; k < NC; k++) sf[fidx(k, fw, fj)] = T(F[k]);
      sf[fidx(NC, fw, fj)] = T(us);
    }
  }
  if constexpr (ALIAS) {
    __syncthreads();
    if (fvalid) {
#pragma unroll
      for (int k = 0; k < NC; k++) sf[fidx(k, fw, fj)] = T(F[k]);
      sf[fidx(NC, fw, fj)] = T(us);
    }
  }
  if (g.stats && g.mood) {
    const unsigned long long b3 = __ballot(my3 != 0);
    const unsigned long long b1 = __ballot(my1 != 0);
    if (b3 | b1) {
      if (my3) atomicAdd(&g.stats->o3[D], (unsigned long long)my3);
      if (my1) atomicAdd(&g.stats->o1[D], (unsigned long long)my1);
    }
  }
  if (g.shortcut) {
    // measurement only: one atomic per wave, spread over 256 slots
    const int ws = wave_sum(mys);
    const unsigned blk = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    if ((threadIdx.x & 63) == 0 && ws)
      atomicAdd(&g.shortcut[(blk & 255) * 3 + D], (unsigned long long)ws);
  }
  __syncthreads();
  if (g.stats && tid == 0 && s_status != ST_OK) atomicExch(&g.stats->status, s_status);

  // 3. cells
  const Div64<T> bydx(g.dx[D]);
  for (int e = tid; e < TW * TL; e += NTHR) {
    const int w = D == 0 ? e / TL : e % TW;
    const int j = D == 0 ? e % TL : e / TW;
    const int64_t a = a0 + w;
    const int64_t l = l0 + j;
    if (a >= geo.nA || l >= geo.nL) continue;
    const int64_t cell = a * geo.sA + l * geo.sL + tt * geo.sT;
#pragma unroll
    for (int k = 0; k < NC; k++) {
      const int kc = axis_comp<NDIM, D>(k);
      double r = bydx(-(double(sf[fidx(k, w, j + 1)]) - double(sf[fidx(k, w, j)])));
      if (k >= 3 + (NDIM - 1)) {
        const double phi = sq[lidx(kc, w, j + 3)];
        r = r + bydx(phi * (double(sf[fidx(NC, w, j + 1)]) - double(sf[fidx(NC, w, j)])));
      }
      double L = READ_R ? g.R[kc * N + cell] + r : r;
      const int64_t o = kc * N + cell;
      if (MODE == OUT_PARTIAL || MODE == OUT_PARTIAL_S || MODE == OUT_RHS) {
        g.Rout[o] = L;
      } else {
        const double h = *g.dt;
        if (MODE == OUT_RK1) {
          g.Uout[o] = g.U0[o] + h * L;
        } else if (MODE == OUT_RK2) {
          g.Uout[o] = 0.75 * g.U0[o] + 0.25 * (g.Uin[o] + h * L);
        } else {
          g.Uout[o] = (1.0 / 3.0) * g.U0[o] + (2.0 / 3.0) * (g.Uin[o] + h * L);
        }
      }
    }
  }
}

// Learned-weights stage kernel (float32 reconstruction only): the same three
// phases, but the face loop runs with every lane of the wave so that the
// network's matrix instructions see the whole wave; lanes without a face
// of their own evaluate face (0, 0) and store nothing.
template <typename T, int NDIM, int D, int TL, int TW, int NTHR, int MODE, bool READ_R>
__global__ __launch_bounds__(NTHR) void sweep_mlp_kernel(SweepArgs g) {
  constexpr int NC = 4 + NDIM;
  constexpr int NP = TL + 6;     // staged positions along D
  constexpr int NF = TL + 1;     // faces along D per tile row
  // LDS layouts: D = 0 -> [c][w][p]; D > 0 -> [c][p][w]
  __shared__ T sq[NC * TW * NP];  // FP64 primitives staged as T
  // face fluxes in the arithmetic's type: the float form's fluxes are
  // float values, so float storage is exact and frees LDS for occupancy
  __shared__ T sf[(NC + 1) * TW * NF];
  __shared__ int s_status;
  __shared__ int s_skip;
  // learned weights: network + one inference tile per wave
  __shared__ MlpLds mW[1];
  __shared__ MlpBiasLds mB[1];

  const Geo<NDIM, D> geo(g.n);
  const int64_t ntl = (geo.nL + TL - 1) / TL;
  const int64_t bid = blockIdx.x;
  const int64_t tl = bid % ntl;
  const int64_t rest = bid / ntl;
  const int64_t nta = (geo.nA + TW - 1) / TW;
  const int64_t ta = rest % nta;
  const int64_t tt = rest / nta;
  const int64_t l0 = tl * TL, a0 = ta * TW;
  const int64_t N = g.n[0] * g.n[1] * g.n[2];
  const int tid = threadIdx.x;
  if (tid == 0) {
    s_status = ST_OK;
    // sticky failure: one read per workgroup so that all lanes agree
    s_skip = g.stats ? (__atomic_load_n(&g.stats->status, __ATOMIC_RELAXED) != ST_OK) : 0;
  }
  mlp_stage_bf16(*mW, g.mlp, tid, NTHR);
  __syncthreads();
  mlp_bias_stage(*mB, *mW, tid, NTHR);
  MlpRegs regs;
  mlp_regs_load(*mW, regs);
  __syncthreads();
  if (s_skip) return;

  auto lidx = [](int c, int w, int p) {
    return D == 0 ? (c * TW + w) * NP + p : (c * NP + p) * TW + w;
  };
  auto fidx = [](int k, int w, int j) {
    return D == 0 ? (k * TW + w) * NF + j : (k * NF + j) * TW + w;
  };

  // 1. stage primitives (FP64) with ghost cells
  bool bad = false;
  for (int e = tid; e < TW * NP; e += NTHR) {
    const int w = D == 0 ? e / NP : e % TW;
    const int p = D == 0 ? e % NP : e / TW;
    const int64_t a = a0 + w;
    const int64_t l = l0 + p - 3;
    if (a >= geo.nA || l >= geo.nL + 3) continue;
    bool flip;
    const int64_t li = bc_index(l, geo.nL, g.bc_lo, g.bc_hi, flip);
    const int64_t cell = a * geo.sA + li * geo.sL + tt * geo.sT;
    double q[NC];
    cell_prim<NDIM, T>(g.Uin, N, cell, q);
    if (p >= 3 && p < 3 + TL && l < geo.nL) bad = bad || !cell_ok<NDIM>(g.Uin, N, cell, q);
    if (flip) q[1 + D] = -q[1 + D];
#pragma unroll
    for (int c = 0; c < NC; c++) sq[lidx(c, w, p)] = T(q[c]);
  }
  if (bad) s_status = ST_NONPHYSICAL;
  __syncthreads();

  // 2. faces: the trip count is the same for every lane (see above)
  int my3 = 0, my1 = 0;
  MlpRun mr;
  mr.R = &regs;
  mr.B = mB;
  mr.thr = g.mlp_thr;
  mr.fallbacks = 0;
  for (int f0 = 0; f0 < TW * NF; f0 += NTHR) {
    const int f = f0 + tid;
    // x tiles of 8 rows x 32 faces: each wave takes an 8 x 8 block, so more
    // waves find every stencil flat and skip the network (x sweep -7%)
    constexpr bool BLOCKED = D == 0 && TW == 8 && NF == 32 && TW * NF == NTHR;
    int w = BLOCKED ? (f & 63) >> 3 : D == 0 ? f / NF : f % TW;
    int j = BLOCKED ? ((f >> 6) << 3) | (f & 7) : D == 0 ? f % NF : f / TW;
    bool valid = f < TW * NF && a0 + w < geo.nA && l0 + j <= geo.nL;
    if (!valid) {
      w = 0;
      j = 0;
    }
    LdsStencil<T> st;
    st.base = &sq[lidx(0, w, j)];
    st.cstride = D == 0 ? TW * NP : NP * TW;
    st.pstride = D == 0 ? 1 : TW;
    double F[NC], us;
    int n3, n1, nf;
    face_flux<T, NDIM, D>(st, g.weights, g.mood, g.eps, F, us, n3, n1, nf, &mr);
    if (!valid) continue;
    // the face on a tile boundary is evaluated by both tiles; count it once
    // (in the tile to its right, or the last tile for the domain's last face)
    if (j < TL || l0 + j == geo.nL) {
      my3 += n3;
      my1 += n1;
    }
#pragma unroll
    for (int k = 0; k < NC; k++) sf[fidx(k, w, j)] = T(F[k]);
    sf[fidx(NC, w, j)] = T(us);
  }
  if (g.stats) {
    if (g.mood) {
      if (my3) atomicAdd(&g.stats->o3[D], (unsigned long long)my3);
      if (my1) atomicAdd(&g.stats->o1[D], (unsigned long long)my1);
    }
    if (mr.fallbacks) atomicAdd(&g.stats->mlp_fallback[D], (unsigned long long)mr.fallbacks);
  }
  __syncthreads();
  if (g.stats && tid == 0 && s_status != ST_OK) atomicExch(&g.stats->status, s_status);

  // 3. cells
  const Div64<T> bydx(g.dx[D]);
  for (int e = tid; e < TW * TL; e += NTHR) {
    const int w = D == 0 ? e / TL : e % TW;
    const int j = D == 0 ? e % TL : e / TW;
    const int64_t a = a0 + w;
    const int64_t l = l0 + j;
    if (a >= geo.nA || l >= geo.nL) continue;
    const int64_t cell = a * geo.sA + l * geo.sL + tt * geo.sT;
#pragma unroll
    for (int k = 0; k < NC; k++) {
      const int kc = axis_comp<NDIM, D>(k);
      double r = bydx(-(double(sf[fidx(k, w, j + 1)]) - double(sf[fidx(k, w, j)])));
      if (k >= 3 + (NDIM - 1)) {
        const double phi = sq[lidx(kc, w, j + 3)];
        r = r + bydx(phi * (double(sf[fidx(NC, w, j + 1)]) - double(sf[fidx(NC, w, j)])));
      }
      double L = READ_R ? g.R[kc * N + cell] + r : r;
      const int64_t o = kc * N + cell;
      if (MODE == OUT_PARTIAL || MODE == OUT_RHS) {
        g.Rout[o] = L;
      } else {
        const double h = *g.dt;
        if (MODE == OUT_RK1) {
          g.Uout[o] = g.U0[o] + h * L;
        } else if (MODE == OUT_RK2) {
          g.Uout[o] = 0.75 * g.U0[o] + 0.25 * (g.Uin[o] + h * L);
        } else {
          g.Uout[o] = (1.0 / 3.0) * g.U0[o] + (2.0 / 3.0) * (g.Uin[o] + h * L);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <int NDIM, int D>
struct TileShape;
// x sweeps: 31 cells x 8 rows -> 32 faces per row, two rows per wave (a
// shorter halo per row than 63 x 4 costs less than the extra rows; 15 x 16
// was slower again)
template <int NDIM>
struct TileShape<NDIM, 0> {
  static constexpr int TL = NDIM == 1 ? 255 : 31;
  static constexpr int TW = NDIM == 1 ? 1 : 8;
};
// y / z sweeps: 16 x-consecutive columns x 15 cells -> 256 faces
template <int NDIM>
struct TileShape<NDIM, 1> {
  static constexpr int TL = 15, TW = 16;
};
template <int NDIM>
struct TileShape<NDIM, 2> {
  static constexpr int TL = 15, TW = 16;
};

template <typename T, int NDIM, int D, int MODE, bool READ_R, bool LEARNED, bool CUT>
static hipError_t launch_sweep_t(const SweepArgs& a, hipStream_t s, LaunchEvents ev) {
  using TS = TileShape<NDIM, D>;
  constexpr int NTHR = 256;
  // the tile decomposition below covers [0, n) on every axis and the kernel
  // bounds each access by n; axes beyond NDIM must be 1
  if (a.n[0] < 1 || a.n[1] < 1 || a.n[2] < 1 || (NDIM < 2 && a.n[1] != 1) ||
      (NDIM < 3 && a.n[2] != 1))
    return hipErrorInvalidValue;
  const int64_t nL = a.n[D];
  int64_t nA, nT;
  if (D == 0) { nA = a.n[1] * a.n[2]; nT = 1; }
  else if (D == 1) { nA = a.n[0]; nT = a.n[2]; }
  else { nA = a.n[0]; nT = a.n[1]; }
  const int64_t blocks = ((nL + TS::TL - 1) / TS::TL) * ((nA + TS::TW - 1) / TS::TW) * nT;
  if (blocks <= 0) return hipSuccess;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  // with events (timing only, never captured), the dispatch records its own
  // start and end: the kernel's duration without the launch latency
  const dim3 grid((unsigned)blocks), block(NTHR);
  if constexpr (LEARNED) {
    if (ev.start)
      hipExtLaunchKernelGGL((sweep_mlp_kernel<T, NDIM, D, TS::TL, TS::TW, NTHR, MODE, READ_R>),
                            grid, block, 0, s, ev.start, ev.stop, 0, a);
    else
      hipLaunchKernelGGL((sweep_mlp_kernel<T, NDIM, D, TS::TL, TS::TW, NTHR, MODE, READ_R>),
                         grid, block, 0, s, a);
  } else {
    if (ev.start)
      hipExtLaunchKernelGGL((sweep_kernel<T, NDIM, D, TS::TL, TS::TW, NTHR, MODE, READ_R, CUT>),
                            grid, block, 0, s, ev.start, ev.stop, 0, a);
    else
      hipLaunchKernelGGL((sweep_kernel<T, NDIM, D, TS::TL, TS::TW, NTHR, MODE, READ_R, CUT>),
                         grid, block, 0, s, a);
  }
  return hipGetLastError();
}

template <typename T, int NDIM, int D, bool LEARNED, bool CUT>
static hipError_t launch_sweep_d(const SweepArgs& a, int mode, bool readR, hipStream_t s,
                                 LaunchEvents ev) {
  switch (mode) {
    case OUT_PARTIAL:
      return readR ? launch_sweep_t<T, NDIM, D, OUT_PARTIAL, true, LEARNED, CUT>(a, s, ev)
                   : launch_sweep_t<T, NDIM, D, OUT_PARTIAL, false, LEARNED, CUT>(a, s, ev);
    case OUT_PARTIAL_S:
      // the first sweep of a 3D stage, also storing its tiles' max wave speeds
      if constexpr (NDIM == 3 && D == 0 && !LEARNED) {
        if (readR || !a.cflp) return hipErrorInvalidValue;
        return launch_sweep_t<T, NDIM, D, OUT_PARTIAL_S, false, LEARNED, CUT>(a, s, ev);
      } else {
        return hipErrorInvalidValue;
      }
    case OUT_RHS:
      return readR ? launch_sweep_t<T, NDIM, D, OUT_RHS, true, LEARNED, CUT>(a, s, ev)
                   : launch_sweep_t<T, NDIM, D, OUT_RHS, false, LEARNED, CUT>(a, s, ev);
    case OUT_RK1:
      return readR ? launch_sweep_t<T, NDIM, D, OUT_RK1, true, LEARNED, CUT>(a, s, ev)
                   : launch_sweep_t<T, NDIM, D, OUT_RK1, false, LEARNED, CUT>(a, s, ev);
    case OUT_RK2:
      return readR ? launch_sweep_t<T, NDIM, D, OUT_RK2, true, LEARNED, CUT>(a, s, ev)
                   : launch_sweep_t<T, NDIM, D, OUT_RK2, false, LEARNED, CUT>(a, s, ev);
    default:
      return readR ? launch_sweep_t<T, NDIM, D, OUT_RK3, true, LEARNED, CUT>(a, s, ev)
                   : launch_sweep_t<T, NDIM, D, OUT_RK3, false, LEARNED, CUT>(a, s, ev);
  }
}

template <typename T, bool LEARNED, bool CUT>
static hipError_t launch_sweep_p(int ndim, int D, const SweepArgs& a, int mode, bool readR,
                                 hipStream_t s, LaunchEvents ev) {
  if (ndim == 1) return launch_sweep_d<T, 1, 0, LEARNED, CUT>(a, mode, readR, s, ev);
  if (ndim == 2) {
    return D == 0 ? launch_sweep_d<T, 2, 0, LEARNED, CUT>(a, mode, readR, s, ev)
                  : launch_sweep_d<T, 2, 1, LEARNED, CUT>(a, mode, readR, s, ev);
  }
  if (D == 0) return launch_sweep_d<T, 3, 0, LEARNED, CUT>(a, mode, readR, s, ev);
  if (D == 1) return launch_sweep_d<T, 3, 1, LEARNED, CUT>(a, mode, readR, s, ev);
  return launch_sweep_d<T, 3, 2, LEARNED, CUT>(a, mode, readR, s, ev);
}

}  // namespace isw
