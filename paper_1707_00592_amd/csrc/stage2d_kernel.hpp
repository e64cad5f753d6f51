// Fused two-dimensional stage kernel of the WENO-IS finite-volume operator.
//
// One launch evaluates a whole Runge-Kutta stage of a 2D grid: a workgroup
// of 256 lanes owns a 15 x 16 tile of cells and
//   1. loads U for the tile plus a cross-shaped halo of 3 cells on each side
//      along x (for the tile's rows) and along y (for its columns) -- the
//      method is dimension by dimension (Sec. 3), so no corner cell is
//      needed -- applying each axis' boundary condition to its own halo,
//      recovers the primitive state in FP64 (eq. (2)) and stages it in LDS;
//   2. evaluates the 255 y faces (projection, WENO-IS, MOOD cascade, HLLC),
//      one per lane, into an LDS face buffer;
//   3. evaluates the 16 x faces of each of the 16 rows, one per lane,
//      lane = 16 row + face, so that a cell's right face sits in the next
//      lane of the same 16-lane group: each lane forms its cell's x terms of
//      eqs. (5)-(6) from its own face and the neighbour lane's, adds the y
//      terms from the face buffer (the order of the dimension-by-dimension
//      sum, L = r_x + r_y) and writes dU/dt or the Runge-Kutta stage.
// Compared with one sweep per axis, neither axis' terms travel through
// memory and the state is read once per stage; no face evaluation runs with
// another face's results held in registers.  A CFL step forms its time step
// in its first stage (OUT_RK1L: L(U^n) and each tile's max wave speed,
// reduced by one workgroup between the stages) and stages U^n + dt L in the
// second (OUT_RK2L), so that U^n is not read by a reduction of its own.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "launch.hpp"
#include "sweep.hpp"

namespace isw {

namespace {

constexpr int kTX = 15, kTY = 16, kThreads = 256;
constexpr int kSX = kTX + 6, kSY = kTY + 6;  // staged rectangle; its corners stay unused
constexpr int kQROW = kSX * kSY;

template <typename E>
struct LdsStencil2 {
  const E* base;  // LDS row of component 0, stencil position 0
  int pstride;
  __device__ __forceinline__ E operator()(int c, int j) const {
    return base[c * kQROW + j * pstride];
  }
};

}  // namespace

// At least 4 resident waves per SIMD (registers capped at 128).  The
// cut-off weights with the gathered cascade need more (about 250 in FP64)
// and get 2.
template <typename T, int MODE, bool CUT, bool GATHER>
__global__ __launch_bounds__(kThreads, CUT && GATHER ? 2 : 4) void stage2d_kernel(SweepArgs g) {
  constexpr int NDIM = 2, NC = 6, TX = kTX, TY = kTY, NTHR = kThreads;
  constexpr int SX = kSX, QROW = kQROW;
  constexpr int NFX = (TX + 1) * TY;  // 256 x faces: lane = 16 row + face
  constexpr int NFY = TX * (TY + 1);  // 255 y faces: face (x, fy) at fy * TX + x
  static_assert(NFX == NTHR && NFY <= NTHR, "one face per lane in each phase");
  // primitives [c][yy][xx], recovered in FP64 and staged in the arithmetic's
  // type (the float form reconstructs from float values anyway)
  __shared__ T sq[NC * QROW];
  // y-face fluxes and v* in the arithmetic's type (the float form's fluxes
  // are float values, so float storage is exact)
  __shared__ T sfy[(NC + 1) * NFY];
  __shared__ int s_status;
  __shared__ int s_skip;
  // GATHER: faces whose MOOD check failed, per phase (face index | fail
  // bits << 16), redone by full waves after the phase's faces; the x faces
  // redone hand their values back through sfx
  __shared__ int s_queue[GATHER ? NTHR : 1];
  __shared__ int s_nq[GATHER ? 2 : 1];
  __shared__ T sfx[GATHER ? (NC + 1) * NFX : 1];
  // OUT_RK1L: this stage also finds its tile's max wave speed (the step's
  // time step); OUT_RK2L: its input is U0 + dt R
  constexpr bool SPEEDS = MODE == OUT_RK1L, FROM_L = MODE == OUT_RK2L;
  __shared__ unsigned long long s_red[SPEEDS ? NTHR / 64 : 1];

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
  if (s_skip) {
    if (SPEEDS && tid == 0) g.cflp[blockIdx.x] = 0ull;
    return;
  }

  // The waves of a workgroup that is staging its tile run at a raised
  // instruction priority (s_setprio), so that its loads are issued ahead of
  // the arithmetic of the resident workgroups and arrive while they compute;
  // back to normal once the tile is staged.
  __builtin_amdgcn_s_setprio(1);
  // 1. stage primitives: the tile's interior cells, its rows extended by 3
  // cells each way along x and its columns by 3 each way along y
  bool bad = false;
  double m = 0.0, h1 = 0.0;  // SPEEDS: the lane's max wave speed; FROM_L: dt
  if constexpr (FROM_L) h1 = *g.dt;
  const double dxs[2] = {g.dx[0], g.dx[1]};
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
    double u[NC], q[NC];
#pragma unroll
    for (int c = 0; c < NC; c++) {
      if constexpr (FROM_L) u[c] = g.U0[c * N + cell] + h1 * g.R[c * N + cell];
      else u[c] = g.Uin[c * N + cell];
    }
    cons_prim<NDIM, T>(u, q);
    if (colin && rowin) {
      bad = bad || !cell_ok_u<NDIM>(u, q);
      if constexpr (SPEEDS) {
        const double sp = cell_speed<NDIM, T>(q, dxs);
        m = (sp > m || sp != sp) ? sp : m;
      }
    }
    if (flip) {
      if (xhalo) q[1] = -q[1];
      else q[2] = -q[2];
    }
#pragma unroll
    for (int c = 0; c < NC; c++) sq[c * QROW + e] = T(q[c]);
  }
  if constexpr (SPEEDS) wave_max_bits(m, s_red);
  if (bad) s_status = ST_NONPHYSICAL;
  __syncthreads();
  __builtin_amdgcn_s_setprio(0);
  if (g.stats && tid == 0 && s_status != ST_OK) atomicExch(&g.stats->status, s_status);
  if constexpr (SPEEDS) {
    if (tid == 0) {
      unsigned long long b = s_red[0];
      for (int w = 1; w < NTHR / 64; w++) b = s_red[w] > b ? s_red[w] : b;
      g.cflp[blockIdx.x] = b;
    }
  }

  int my3[2] = {0, 0}, my1[2] = {0, 0}, mys[2] = {0, 0};
  const int wts = kernel_weights<CUT>(g.weights);
  const Div64<T> bydx(g.dx[0]), bydy(g.dx[1]);
  auto xstencil = [&](int f) {  // x face (f % 16, f / 16)
    LdsStencil2<T> st;
    st.base = &sq[(f / 16 + 3) * SX + f % 16];
    st.pstride = 1;
    return st;
  };
  auto ystencil = [&](int f) {  // y face (f % TX, f / TX)
    LdsStencil2<T> st;
    st.base = &sq[(f / TX) * SX + f % TX + 3];
    st.pstride = SX;
    return st;
  };
  auto storey = [&](int f, const double* G, double vs) {
#pragma unroll
    for (int kk = 0; kk < NC; kk++) sfy[kk * NFY + f] = T(G[kk]);
    sfy[NC * NFY + f] = T(vs);
  };
  // a face on a tile boundary is evaluated by both tiles: it is counted in
  // the tile after it (the last tile for the domain's last face)
  auto xcounted = [&](int f) {
    const int fx = f % 16;
    return fx < TX || gx0 + fx == nx;
  };
  auto ycounted = [&](int f) {
    const int fy = f / TX;
    return fy < TY || gy0 + fy == ny;
  };
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

  // 2. y faces: lane tid < 255 holds face (tid % 15, tid / 15), between
  // cells fy-1 and fy of its column
  {
    const bool yvalid = tid < NFY && gx0 + tid % TX < nx && gy0 + tid / TX <= ny;
    if constexpr (GATHER) {
      int fail = 0;
      if (yvalid) {
        double G[NC], vs;
        int nsc;
        fail = face_flux_first<T, NDIM, 1, CUT>(ystencil(tid), wts, g.eps, G, vs, nsc);
        if (ycounted(tid)) mys[1] += nsc;
        if (!fail) storey(tid, G, vs);
      }
      enqueue(1, tid, fail);
      __syncthreads();
      // the gathered faces, by full waves
      const int nq = s_nq[1];
      if (tid < nq) {
        const int f = s_queue[tid] & 0xffff, fl = s_queue[tid] >> 16;
        double G[NC], vs;
        int n3, n1;
        face_flux_redo<T, NDIM, 1, CUT>(ystencil(f), fl, wts, g.eps, G, vs, n3, n1);
        if (ycounted(f)) {
          my3[1] += n3;
          my1[1] += n1;
        }
        storey(f, G, vs);
      }
    } else if (yvalid) {
      double G[NC], vs;
      int n3, n1, nsc;
      face_flux<T, NDIM, 1, CUT>(ystencil(tid), wts, g.mood, g.eps, G, vs, n3, n1, nsc);
      if (ycounted(tid)) {
        my3[1] += n3;
        my1[1] += n1;
        mys[1] += nsc;
      }
      storey(tid, G, vs);
    }
  }
  // The x faces read only the staged primitives; the y faces' values are
  // read by the cells, after the barrier below.  The gathered cascade
  // reuses its queue in the x phase, so it waits here.
  if constexpr (GATHER) __syncthreads();

  // 3. x faces: lane tid holds face (cx, cy), between cells cx-1 and cx of
  // row cy, and, for cx < 15, cell (cx, cy)
  const int cy = tid >> 4, cx = tid & 15;
  double F[NC], us = 0.0;
#pragma unroll
  for (int kk = 0; kk < NC; kk++) F[kk] = 0.0;
  const bool xvalid = gy0 + cy < ny && gx0 + cx <= nx;
  if constexpr (GATHER) {
    int fail = 0;
    if (xvalid) {
      int nsc;
      fail = face_flux_first<T, NDIM, 0, CUT>(xstencil(tid), wts, g.eps, F, us, nsc);
      if (xcounted(tid)) mys[0] += nsc;
    }
    enqueue(0, tid, fail);
    __syncthreads();
    const int nq = s_nq[0];
    if (nq) {
      if (tid < nq) {
        const int f = s_queue[tid] & 0xffff, fl = s_queue[tid] >> 16;
        double Fq[NC], uq;
        int n3, n1;
        face_flux_redo<T, NDIM, 0, CUT>(xstencil(f), fl, wts, g.eps, Fq, uq, n3, n1);
        if (xcounted(f)) {
          my3[0] += n3;
          my1[0] += n1;
        }
#pragma unroll
        for (int kk = 0; kk < NC; kk++) sfx[kk * NFX + f] = T(Fq[kk]);
        sfx[NC * NFX + f] = T(uq);
      }
      __syncthreads();
      if (fail) {
#pragma unroll
        for (int kk = 0; kk < NC; kk++) F[kk] = double(sfx[kk * NFX + tid]);
        us = double(sfx[NC * NFX + tid]);
      }
    }
  } else if (xvalid) {
    int n3, n1, nsc;
    face_flux<T, NDIM, 0, CUT>(xstencil(tid), wts, g.mood, g.eps, F, us, n3, n1, nsc);
    if (xcounted(tid)) {
      my3[0] += n3;
      my1[0] += n1;
      mys[0] += nsc;
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
  // every y face is in sfy from here on (a wave that finished its y faces
  // early went on to its x face first)
  if constexpr (!GATHER) __syncthreads();
  // the face to the right of cell cx is the next lane's (same 16-lane
  // group); for cx = 15 there is no cell and the value goes unused
  double Fr[NC];
#pragma unroll
  for (int kk = 0; kk < NC; kk++) Fr[kk] = __shfl_down(F[kk], 1, 16);
  const double usr = __shfl_down(us, 1, 16);

  // x terms of eqs. (5)-(6) (for the x axis face order and axis order
  // coincide), plus the y terms (face order -> axis order: u_n = v is
  // component 2, u_t = u component 1), then the output step
  if (cx < TX && gx0 + cx < nx && gy0 + cy < ny) {
    const int64_t cell = (gy0 + cy) * nx + gx0 + cx;
    const int fb = cy * TX + cx, fa = fb + TX;  // the cell's lower and upper y faces
    double rx[NC];
#pragma unroll
    for (int kk = 0; kk < NC; kk++) {
      double r = bydx(-(Fr[kk] - F[kk]));
      if (kk >= 4) {
        const double phi = sq[kk * QROW + (cy + 3) * SX + cx + 3];
        r = r + bydx(phi * (usr - us));
      }
      rx[kk] = r;
    }
#pragma unroll
    for (int kk = 0; kk < NC; kk++) {
      const int kc = axis_comp<NDIM, 1>(kk);
      double r = bydy(-(double(sfy[kk * NFY + fa]) - double(sfy[kk * NFY + fb])));
      if (kk >= 4) {
        const double phi = sq[kc * QROW + (cy + 3) * SX + cx + 3];
        r = r + bydy(phi * (double(sfy[NC * NFY + fa]) - double(sfy[NC * NFY + fb])));
      }
      const double L = rx[kc] + r;
      const int64_t o = kc * N + cell;
      if (MODE == OUT_RHS || MODE == OUT_RK1L) {
        g.Rout[o] = L;
      } else {
        const double h = *g.dt;
        if (MODE == OUT_RK1) {
          g.Uout[o] = g.U0[o] + h * L;
        } else if (MODE == OUT_RK2) {
          g.Uout[o] = 0.75 * g.U0[o] + 0.25 * (g.Uin[o] + h * L);
        } else if (MODE == OUT_RK2L) {
          // the stage input U0 + dt R, formed as stage 1 would have written it
          const double u0 = g.U0[o];
          g.Uout[o] = 0.75 * u0 + 0.25 * ((u0 + h * g.R[o]) + h * L);
        } else {
          g.Uout[o] = (1.0 / 3.0) * g.U0[o] + (2.0 / 3.0) * (g.Uin[o] + h * L);
        }
      }
    }
  }
}

template <typename T, int MODE, bool CUT, bool GATHER>
static hipError_t launch_t(const SweepArgs& a, hipStream_t s, LaunchEvents ev) {
  // one workgroup per tile: the kernel maps block b to tile (b & 7, b >> 3)
  // of the XCD-ordered list of exactly this many tiles (OUT_RK1L: and
  // stores one max per tile into cflp)
  if (a.n[0] < 1 || a.n[1] < 1 || a.n[2] != 1) return hipErrorInvalidValue;
  if ((MODE == OUT_RK1L && !a.cflp) || (MODE == OUT_RK2L && !a.R)) return hipErrorInvalidValue;
  const int64_t blocks = stage2d_tiles(a.n[0], a.n[1]);
  if (blocks <= 0) return hipSuccess;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 grid((unsigned)blocks), block(kThreads);
  if (ev.start)
    hipExtLaunchKernelGGL((stage2d_kernel<T, MODE, CUT, GATHER>), grid, block, 0, s, ev.start,
                          ev.stop, 0, a);
  else
    hipLaunchKernelGGL((stage2d_kernel<T, MODE, CUT, GATHER>), grid, block, 0, s, a);
  return hipGetLastError();
}

template <typename T, bool CUT, bool GATHER>
static hipError_t launch_g(const SweepArgs& a, int mode, hipStream_t s, LaunchEvents ev) {
  switch (mode) {
    case OUT_RHS: return launch_t<T, OUT_RHS, CUT, GATHER>(a, s, ev);
    case OUT_RK1: return launch_t<T, OUT_RK1, CUT, GATHER>(a, s, ev);
    case OUT_RK2: return launch_t<T, OUT_RK2, CUT, GATHER>(a, s, ev);
    case OUT_RK3: return launch_t<T, OUT_RK3, CUT, GATHER>(a, s, ev);
    case OUT_RK1L: return launch_t<T, OUT_RK1L, CUT, GATHER>(a, s, ev);
    case OUT_RK2L: return launch_t<T, OUT_RK2L, CUT, GATHER>(a, s, ev);
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

}  // namespace isw
