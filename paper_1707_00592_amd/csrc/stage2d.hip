// Fused two-dimensional stage kernel of the WENO-IS finite-volume operator.
//
// One launch evaluates a whole Runge-Kutta stage of a 2D grid: a workgroup
// owns a TX x TY tile of cells and
//   1. loads U for the tile plus a cross-shaped halo of 3 cells on each side
//      along x (for the tile's rows) and along y (for its columns) -- the
//      method is dimension by dimension (Sec. 3), so no corner cell is
//      needed -- applying each axis' boundary condition to its own halo,
//      recovers the primitive state in FP64 (eq. (2)) and stages it in LDS;
//   2. evaluates every x face of the tile (one lane per face: projection,
//      WENO-IS, MOOD cascade, HLLC), then forms each cell's x terms of
//      eqs. (5)-(6) in registers;
//   3. evaluates every y face into the same LDS buffer, adds each cell's y
//      terms to its x terms (the order of the dimension-by-dimension sum,
//      L = r_x + r_y) and writes dU/dt or the Runge-Kutta stage.
// Compared with one sweep per axis, the x terms never travel through memory
// and the state is read once per stage.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "launch.hpp"
#include "sweep.hpp"

namespace isw {

namespace {

struct LdsStencil2 {
  const double* base;  // component 0, stencil position 0
  int cstride, pstride;
  __device__ __forceinline__ double operator()(int c, int j) const {
    return base[c * cstride + j * pstride];
  }
};

}  // namespace

template <typename T, int TX, int TY, int NTHR, int MODE, bool CUT, bool GATHER>
__global__ __launch_bounds__(NTHR, GATHER && !CUT ? 4 : 1) void stage2d_kernel(SweepArgs g) {
  constexpr int NDIM = 2, NC = 6;
  constexpr int SX = TX + 6, SY = TY + 6;  // staged rectangle; its corners stay unused
  constexpr int QROW = SX * SY;
  constexpr int NFX = (TX + 1) * TY;       // x faces of the tile, row-major
  constexpr int NFY = TX * (TY + 1);       // y faces of the tile, row-major
  constexpr int NFMAX = NFX > NFY ? NFX : NFY;
  constexpr int NCELL = TX * TY;
  constexpr int CPL = (NCELL + NTHR - 1) / NTHR;  // cells per lane
  __shared__ double sq[NC * QROW];               // primitives [c][yy][xx]
  // face fluxes and u* in the arithmetic's type (the float form's fluxes
  // are float values, so float storage is exact); x faces, then y faces
  __shared__ T sf[(NC + 1) * NFMAX];
  __shared__ int s_status;
  __shared__ int s_skip;
  // GATHER: faces whose MOOD check failed, per phase (face index | fail
  // bits << 16), redone by full waves after the phase's faces
  __shared__ int s_queue[GATHER ? NFMAX : 1];
  __shared__ int s_nq[GATHER ? 2 : 1];

  const int64_t nx = g.n[0], ny = g.n[1], N = nx * ny;
  // Tile order.  The hardware deals workgroups to its 8 XCDs in turn
  // (workgroup b to XCD b mod 8), each XCD with its own L2.  XCD x's
  // workgroups take one contiguous run of tiles, in an order that walks
  // along tile rows (x-neighbours, whose halo lines overlap, share an L2)
  // and visits the rows as 0, 8, 16, ..., 1, 9, ... (every XCD gets rows
  // spread over the whole height, so fronts stay evenly shared).
  const int64_t ntx = (nx + TX - 1) / TX, nty = (ny + TY - 1) / TY;
  const int64_t ntiles = ntx * nty;
  const int64_t xcd = blockIdx.x & 7, k = blockIdx.x >> 3;
  const int64_t per = ntiles >> 3, extra = ntiles & 7;
  const int64_t pos = xcd * per + (xcd < extra ? xcd : extra) + k;
  const int64_t prow = pos / ntx;
  int64_t cls = 0, first = 0;  // rows cls, cls + 8, ... hold positions first ...
  while (prow >= first + ((nty - cls + 7) >> 3)) {
    first += (nty - cls + 7) >> 3;
    cls++;
  }
  const int64_t gx0 = (pos % ntx) * TX;
  const int64_t gy0 = (cls + 8 * (prow - first)) * TY;
  const int tid = threadIdx.x;
  if (tid == 0) {
    if constexpr (GATHER) {
      s_nq[0] = 0;
      s_nq[1] = 0;
    }
    s_status = ST_OK;
    // sticky failure: one read per workgroup so that all lanes agree
    s_skip = g.stats ? (__atomic_load_n(&g.stats->status, __ATOMIC_RELAXED) != ST_OK) : 0;
  }
  __syncthreads();
  if (s_skip) return;

  // 1. stage primitives: the tile's interior cells, its rows extended by 3
  // cells each way along x and its columns by 3 each way along y
  bool bad = false;
  for (int e = tid; e < QROW; e += NTHR) {
    const int yy = e / SX, xx = e % SX;
    const int64_t gxl = gx0 + xx - 3, gyl = gy0 + yy - 3;
    const bool colin = xx >= 3 && xx < TX + 3 && gxl < nx;  // a column of the tile
    const bool rowin = yy >= 3 && yy < TY + 3 && gyl < ny;  // a row of the tile
    const bool xhalo = rowin && !colin && gxl < nx + 3;
    const bool yhalo = colin && !rowin && gyl < ny + 3;
    if (!(colin && rowin) && !xhalo && !yhalo) continue;
    bool flip = false;
    int64_t ix = gxl, iy = gyl;
    if (xhalo) ix = bc_index(gxl, nx, g.bcl[0], g.bch[0], flip);
    if (yhalo) iy = bc_index(gyl, ny, g.bcl[1], g.bch[1], flip);
    const int64_t cell = iy * nx + ix;
    double q[NC];
    cell_prim<NDIM>(g.Uin, N, cell, q);
    if (colin && rowin) bad = bad || !cell_ok<NDIM>(g.Uin, N, cell, q);
    if (flip) {
      if (xhalo) q[1] = -q[1];
      else q[2] = -q[2];
    }
#pragma unroll
    for (int c = 0; c < NC; c++) sq[c * QROW + e] = q[c];
  }
  if (bad) s_status = ST_NONPHYSICAL;
  __syncthreads();
  if (g.stats && tid == 0 && s_status != ST_OK) atomicExch(&g.stats->status, s_status);

  int my3[2] = {0, 0}, my1[2] = {0, 0}, mys[2] = {0, 0};

  const int wts = kernel_weights<CUT>(g.weights);
  // a face whose check failed joins the phase's queue: one LDS atomic per
  // wave, slots in lane order (GATHER only)
  auto enqueue = [&](int d, int f, int fail) {
    const unsigned long long bal = __ballot(fail != 0);
    if (bal == 0) return;
    const int lane = tid & 63, lead = __builtin_ctzll(bal);
    int base = 0;
    if (lane == lead) base = atomicAdd(&s_nq[d], __popcll(bal));
    base = __shfl(base, lead);
    if (fail) s_queue[base + __popcll(bal & ((1ull << lane) - 1))] = f | (fail << 16);
  };
  auto store = [&](int f, const double* F, double us) {
#pragma unroll
    for (int k = 0; k < NC; k++) sf[k * NFMAX + f] = T(F[k]);
    sf[NC * NFMAX + f] = T(us);
  };
  auto xstencil = [&](int f) {
    LdsStencil2 st;
    st.base = &sq[(f / (TX + 1) + 3) * SX + f % (TX + 1)];
    st.cstride = QROW;
    st.pstride = 1;
    return st;
  };
  auto ystencil = [&](int f) {
    LdsStencil2 st;
    st.base = &sq[(f / TX) * SX + f % TX + 3];
    st.cstride = QROW;
    st.pstride = SX;
    return st;
  };
  // a face on a tile boundary is evaluated by both tiles: it is counted in
  // the tile after it (the last tile for the domain's last face)
  auto xcounted = [&](int f) {
    const int fx = f % (TX + 1);
    return fx < TX || gx0 + fx == nx;
  };
  auto ycounted = [&](int f) {
    const int fy = f / TX;
    return fy < TY || gy0 + fy == ny;
  };

  // 2. x faces: face (fx, y) lies between cells fx-1 and fx of row y
  if constexpr (GATHER) {
    for (int f0 = 0; f0 < NFX; f0 += NTHR) {
      const int f = f0 + tid;
      int fail = 0;
      if (f < NFX && gy0 + f / (TX + 1) < ny && gx0 + f % (TX + 1) <= nx) {
        double F[NC], us;
        int nsc;
        fail = face_flux_first<T, NDIM, 0, CUT>(xstencil(f), wts, g.eps, F, us, nsc);
        if (xcounted(f)) mys[0] += nsc;
        if (!fail) store(f, F, us);
      }
      enqueue(0, f, fail);
    }
    __syncthreads();
    const int nq = s_nq[0];
    if (nq) {
      for (int q = tid; q < nq; q += NTHR) {
        const int f = s_queue[q] & 0xffff, fail = s_queue[q] >> 16;
        double F[NC], us;
        int n3, n1;
        face_flux_redo<T, NDIM, 0, CUT>(xstencil(f), fail, wts, g.eps, F, us, n3, n1);
        if (xcounted(f)) {
          my3[0] += n3;
          my1[0] += n1;
        }
        store(f, F, us);
      }
      __syncthreads();
    }
  } else {
    for (int f = tid; f < NFX; f += NTHR) {
      if (!(gy0 + f / (TX + 1) < ny && gx0 + f % (TX + 1) <= nx)) continue;
      double F[NC], us;
      int n3, n1, nsc;
      face_flux<T, NDIM, 0, CUT>(xstencil(f), wts, g.mood, g.eps, F, us, n3, n1, nsc);
      if (xcounted(f)) {
        my3[0] += n3;
        my1[0] += n1;
        mys[0] += nsc;
      }
      store(f, F, us);
    }
    __syncthreads();
  }

  // x terms of eqs. (5)-(6) per cell, kept in registers (axis order; for
  // the x axis face order and axis order coincide)
  const double dx = g.dx[0], dy = g.dx[1];
  double rx[CPL][NC];
#pragma unroll
  for (int i = 0; i < CPL; i++) {
    const int e = tid + i * NTHR;
    const int x = e % TX, y = e / TX;
    if (e >= NCELL) continue;
#pragma unroll
    for (int k = 0; k < NC; k++) {
      const int f = y * (TX + 1) + x;
      double r = -(double(sf[k * NFMAX + f + 1]) - double(sf[k * NFMAX + f])) / dx;
      if (k >= 4) {
        const double phi = sq[k * QROW + (y + 3) * SX + x + 3];
        r = r + phi * (double(sf[NC * NFMAX + f + 1]) - double(sf[NC * NFMAX + f])) / dx;
      }
      rx[i][k] = r;
    }
  }
  __syncthreads();

  // 3. y faces: face (x, fy) lies between cells fy-1 and fy of column x
  if constexpr (GATHER) {
    for (int f0 = 0; f0 < NFY; f0 += NTHR) {
      const int f = f0 + tid;
      int fail = 0;
      if (f < NFY && gx0 + f % TX < nx && gy0 + f / TX <= ny) {
        double F[NC], us;
        int nsc;
        fail = face_flux_first<T, NDIM, 1, CUT>(ystencil(f), wts, g.eps, F, us, nsc);
        if (ycounted(f)) mys[1] += nsc;
        if (!fail) store(f, F, us);
      }
      enqueue(1, f, fail);
    }
    __syncthreads();
    const int nq = s_nq[1];
    for (int q = tid; q < nq; q += NTHR) {
      const int f = s_queue[q] & 0xffff, fail = s_queue[q] >> 16;
      double F[NC], us;
      int n3, n1;
      face_flux_redo<T, NDIM, 1, CUT>(ystencil(f), fail, wts, g.eps, F, us, n3, n1);
      if (ycounted(f)) {
        my3[1] += n3;
        my1[1] += n1;
      }
      store(f, F, us);
    }
  } else {
    for (int f = tid; f < NFY; f += NTHR) {
      if (!(gx0 + f % TX < nx && gy0 + f / TX <= ny)) continue;
      double F[NC], us;
      int n3, n1, nsc;
      face_flux<T, NDIM, 1, CUT>(ystencil(f), wts, g.mood, g.eps, F, us, n3, n1, nsc);
      if (ycounted(f)) {
        my3[1] += n3;
        my1[1] += n1;
        mys[1] += nsc;
      }
      store(f, F, us);
    }
  }
  if (g.stats && g.mood) {
    const unsigned long long b = __ballot((my3[0] | my1[0] | my3[1] | my1[1]) != 0);
    if (b) {
#pragma unroll
      for (int d = 0; d < 2; d++) {
        if (my3[d]) atomicAdd(&g.stats->o3[d], (unsigned long long)my3[d]);
        if (my1[d]) atomicAdd(&g.stats->o1[d], (unsigned long long)my1[d]);
      }
    }
  }
  if (g.shortcut) {
    // measurement only: one atomic per wave and axis, spread over 256 slots
    const unsigned blk = blockIdx.x;
#pragma unroll
    for (int d = 0; d < 2; d++) {
      const int ws = wave_sum(mys[d]);
      if ((threadIdx.x & 63) == 0 && ws)
        atomicAdd(&g.shortcut[(blk & 255) * 3 + d], (unsigned long long)ws);
    }
  }
  __syncthreads();

  // y terms added to the x terms (face order -> axis order: u_n = v is
  // component 2, u_t = u component 1), then the output step
#pragma unroll
  for (int i = 0; i < CPL; i++) {
    const int e = tid + i * NTHR;
    const int x = e % TX, y = e / TX;
    if (e >= NCELL || gx0 + x >= nx || gy0 + y >= ny) continue;
    const int64_t cell = (gy0 + y) * nx + gx0 + x;
#pragma unroll
    for (int k = 0; k < NC; k++) {
      const int kc = axis_comp<NDIM, 1>(k);
      const int f = y * TX + x;
      double r = -(double(sf[k * NFMAX + f + TX]) - double(sf[k * NFMAX + f])) / dy;
      if (k >= 4) {
        const double phi = sq[kc * QROW + (y + 3) * SX + x + 3];
        r = r + phi * (double(sf[NC * NFMAX + f + TX]) - double(sf[NC * NFMAX + f])) / dy;
      }
      const double L = rx[i][kc] + r;
      const int64_t o = kc * N + cell;
      if (MODE == OUT_RHS) {
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

// 16 x 15 tiles: 255 x faces and 256 y faces, one per lane in each phase.
constexpr int kTX = 16, kTY = 15, kThreads = 256;

template <typename T, int MODE, bool CUT, bool GATHER>
static hipError_t launch_t(const SweepArgs& a, hipStream_t s, LaunchEvents ev) {
  // one workgroup per tile: the kernel maps block b to tile (b & 7, b >> 3)
  // of the XCD-ordered list of exactly this many tiles
  if (a.n[0] < 1 || a.n[1] < 1 || a.n[2] != 1) return hipErrorInvalidValue;
  const int64_t blocks = ((a.n[0] + kTX - 1) / kTX) * ((a.n[1] + kTY - 1) / kTY);
  if (blocks <= 0) return hipSuccess;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 grid((unsigned)blocks), block(kThreads);
  if (ev.start)
    hipExtLaunchKernelGGL((stage2d_kernel<T, kTX, kTY, kThreads, MODE, CUT, GATHER>), grid, block, 0, s,
                          ev.start, ev.stop, 0, a);
  else
    hipLaunchKernelGGL((stage2d_kernel<T, kTX, kTY, kThreads, MODE, CUT, GATHER>), grid, block, 0, s, a);
  return hipGetLastError();
}

template <typename T, bool CUT, bool GATHER>
static hipError_t launch_g(const SweepArgs& a, int mode, hipStream_t s, LaunchEvents ev) {
  switch (mode) {
    case OUT_RHS: return launch_t<T, OUT_RHS, CUT, GATHER>(a, s, ev);
    case OUT_RK1: return launch_t<T, OUT_RK1, CUT, GATHER>(a, s, ev);
    case OUT_RK2: return launch_t<T, OUT_RK2, CUT, GATHER>(a, s, ev);
    case OUT_RK3: return launch_t<T, OUT_RK3, CUT, GATHER>(a, s, ev);
    default: return hipErrorInvalidValue;
  }
}

// mood 2: the gathered cascade, in kernels of its own
template <typename T, bool CUT>
static hipError_t launch_m(const SweepArgs& a, int mode, hipStream_t s, LaunchEvents ev) {
  return a.mood == 2 ? launch_g<T, CUT, true>(a, mode, s, ev)
                     : launch_g<T, CUT, false>(a, mode, s, ev);
}

// The cut-off weights run in kernels of their own, so that the other forms
// keep their register allocation.
template <typename T>
static hipError_t launch_p(const SweepArgs& a, int mode, hipStream_t s, LaunchEvents ev) {
  return a.weights == W_CUTOFF ? launch_m<T, true>(a, mode, s, ev)
                               : launch_m<T, false>(a, mode, s, ev);
}

hipError_t launch_stage2d(int precision, const SweepArgs& a, int mode, hipStream_t s,
                          LaunchEvents ev) {
  if (a.weights == W_MLP) return hipErrorInvalidValue;
  return precision == 1 ? launch_p<float>(a, mode, s, ev) : launch_p<double>(a, mode, s, ev);
}

}  // namespace isw
