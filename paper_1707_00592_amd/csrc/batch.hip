// Many independent 1D problems of uneven length (isweno_batch_*).
//
// Layout: U[c * total + cell], problem p owns cells offsets[p] ..
// offsets[p+1]-1.  Each RK stage is ONE persistent launch: a grid of
// (compute units x blocks per CU) workgroups walks a static list of tiles
// (a tile = up to TL consecutive cells of one problem) in round-robin order,
// so the assignment is deterministic and the launch count does not grow
// with the number of problems.  Ghost cells come from each problem's own
// boundary conditions while loading, so tiles never straddle problems.
// One RK3 step (per-problem time step + three stages) is captured once into
// a HIP graph and replayed.  The tile length TL and the grid size are chosen
// by timing every candidate on the caller's data (isweno_batch_autotune).
#include "batch_kernels.hpp"

#include <algorithm>
#include <map>
#include <new>
#include <tuple>
#include <vector>

namespace isw {

__global__ __launch_bounds__(256) void batch_dt_kernel(const double* U, int64_t total,
                                                       const int64_t* offsets,
                                                       const double* dx, double cfl,
                                                       double dt_max, double* dt,
                                                       const int32_t* pstatus,
                                                       int32_t* active) {
  const int p = blockIdx.x;
  const int act = pstatus[p] == ST_OK;
  if (threadIdx.x == 0) active[p] = act;
  if (!act || !(cfl > 0.0)) return;
  const int64_t lo = offsets[p], hi = offsets[p + 1];
  double m = 0.0;
  for (int64_t c = lo + threadIdx.x; c < hi; c += blockDim.x) {
    double q[5];
    cell_prim<1>(U, total, c, q);
    const double cs = sqrt(sound2<double>(q[0], q[2], q[3], q[4]));
    const double s = (fabs(q[1]) + cs) / dx[p];
    m = (s > m || s != s) ? s : m;
  }
  __shared__ double red[256];
  red[threadIdx.x] = m;
  __syncthreads();
  for (unsigned o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      const double x = red[threadIdx.x + o];
      if (x > red[threadIdx.x] || x != x) red[threadIdx.x] = x;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double h = cfl / red[0];
    if (dt_max > 0.0 && h > dt_max) h = dt_max;
    dt[p] = h;
  }
}

static hipError_t launch_batch_stage(int precision, int tl, const BatchArgs& a, int mode,
                                     int blocks, hipStream_t s) {
  return precision == ISWENO_FP32 ? launch_batch_stage_f32(tl, a, mode, blocks, s)
                                  : launch_stage_t<double>(tl, a, mode, blocks, s);
}

}  // namespace isw

// ---------------------------------------------------------------------------
// Plan
// ---------------------------------------------------------------------------
static const int kTiles[] = {63, 127, 255};
static const int kBlocksPerCU[] = {2, 4, 8, 16};

struct TileTable {
  int64_t* start = nullptr;
  int32_t* prob = nullptr;
  int64_t ntiles = 0;
};

struct isweno_batch_plan {
  int device = 0;
  int ncu = 256;
  int32_t nprob = 0;
  int64_t total = 0;
  int32_t bc_lo = 0, bc_hi = 0;
  int64_t* offsets = nullptr;  // device
  double* dx = nullptr;        // device
  double* ws = nullptr;        // U1, U2 (device, 2 x 5 x total)
  int32_t* active = nullptr;   // per problem, written at the start of each step
  int32_t* tune_status = nullptr;  // per problem, for the autotuner's scratch runs
  std::map<int, TileTable> tables;  // by tile length
  int tl = 255;
  int blocks_per_cu = 4;
  hipStream_t cap = nullptr;   // capture stream
  // graph cache keyed by everything a captured step depends on
  using Key = std::tuple<const void*, const void*, const void*, const void*, int, int, int,
                         double, double, double, int, int>;
  std::map<Key, hipGraphExec_t> graphs;
  std::vector<int64_t> host_offsets;
};

static void free_graphs(isweno_batch_plan* p) {
  for (auto& kv : p->graphs) (void)hipGraphExecDestroy(kv.second);
  p->graphs.clear();
}

static int build_table(isweno_batch_plan* p, int tl) {
  if (p->tables.count(tl)) return ISWENO_OK;
  std::vector<int64_t> st;
  std::vector<int32_t> pr;
  for (int32_t q = 0; q < p->nprob; q++) {
    for (int64_t c = p->host_offsets[q]; c < p->host_offsets[q + 1]; c += tl) {
      st.push_back(c);
      pr.push_back(q);
    }
  }
  TileTable t;
  t.ntiles = (int64_t)st.size();
  if (hipMalloc(&t.start, st.size() * sizeof(int64_t)) != hipSuccess) return ISWENO_ERR_DEVICE;
  if (hipMalloc(&t.prob, pr.size() * sizeof(int32_t)) != hipSuccess) {
    (void)hipFree(t.start);
    return ISWENO_ERR_DEVICE;
  }
  if (hipMemcpy(t.start, st.data(), st.size() * sizeof(int64_t), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(t.prob, pr.data(), pr.size() * sizeof(int32_t), hipMemcpyHostToDevice) !=
          hipSuccess)
    return ISWENO_ERR_DEVICE;
  p->tables[tl] = t;
  return ISWENO_OK;
}

static int check_batch_opts(const isweno_opts* o) {
  if (!o || o->reserved != 0 || o->reserved2 != 0) return ISWENO_ERR_ARG;
  if (o->precision != ISWENO_FP64 && o->precision != ISWENO_FP32) return ISWENO_ERR_ARG;
  if (o->weights < 0 || o->weights > 3 || o->mood < 0 || o->mood > 2) return ISWENO_ERR_ARG;
  if (!(o->eps >= 0.0)) return ISWENO_ERR_ARG;
  if (o->weights == ISWENO_W_MLP) return ISWENO_ERR_UNSUPPORTED;
  return ISWENO_OK;
}

// Enqueue one RK3 step (dt kernel + three persistent stages) on s.
static hipError_t enqueue_step(isweno_batch_plan* p, const isweno_opts* o, double* U, double* dt,
                               isweno_stats* stats, int32_t* pstatus, int tl, int bpc,
                               hipStream_t s) {
  const TileTable& t = p->tables[tl];
  const int64_t sz = 5 * p->total;
  double* U1 = p->ws;
  double* U2 = p->ws + sz;
  {
    hipLaunchKernelGGL(isw::batch_dt_kernel, dim3(p->nprob), dim3(256), 0, s, U, p->total,
                       p->offsets, p->dx, o->cfl, o->dt_max, dt, pstatus, p->active);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  isw::BatchArgs a{};
  a.active = p->active;
  a.pstatus = pstatus;
  a.dt = dt;
  a.dx = p->dx;
  a.offsets = p->offsets;
  a.tstart = t.start;
  a.tprob = t.prob;
  a.ntiles = t.ntiles;
  a.total = p->total;
  a.stats = reinterpret_cast<isw::StatsDev*>(stats);
  a.bc_lo = p->bc_lo;
  a.bc_hi = p->bc_hi;
  a.weights = o->weights;
  a.mood = o->mood;
  a.eps = o->eps;
  a.U0 = U;
  int64_t blocks64 = (int64_t)p->ncu * bpc;
  if (blocks64 > t.ntiles) blocks64 = t.ntiles;
  if (blocks64 < 1) blocks64 = 1;
  const int blocks = (int)blocks64;
  hipError_t e;
  a.Uin = U;
  a.Uout = U1;
  if ((e = isw::launch_batch_stage(o->precision, tl, a, isw::OUT_RK1, blocks, s)) != hipSuccess)
    return e;
  a.Uin = U1;
  a.Uout = U2;
  if ((e = isw::launch_batch_stage(o->precision, tl, a, isw::OUT_RK2, blocks, s)) != hipSuccess)
    return e;
  a.Uin = U2;
  a.Uout = U;
  return isw::launch_batch_stage(o->precision, tl, a, isw::OUT_RK3, blocks, s);
}

extern "C" {

int isweno_batch_plan_create(isweno_ctx* ctx, int32_t nprob, const int64_t* offsets,
                             const double* dx, int32_t bc_lo, int32_t bc_hi,
                             isweno_batch_plan** out) {
  if (!out) return ISWENO_ERR_ARG;
  *out = nullptr;
  if (!ctx || nprob < 1 || !offsets || !dx) return ISWENO_ERR_ARG;
  if (bc_lo < 0 || bc_lo > 2 || bc_hi < 0 || bc_hi > 2) return ISWENO_ERR_ARG;
  if (offsets[0] != 0) return ISWENO_ERR_ARG;
  const int minlen = (bc_lo == ISWENO_BC_REFLECTIVE || bc_hi == ISWENO_BC_REFLECTIVE) ? 3 : 1;
  for (int32_t q = 0; q < nprob; q++) {
    if (offsets[q + 1] - offsets[q] < minlen || !(dx[q] > 0.0)) return ISWENO_ERR_ARG;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return ISWENO_ERR_DEVICE;
  isweno_batch_plan* p = new (std::nothrow) isweno_batch_plan();
  if (!p) return ISWENO_ERR_DEVICE;
  p->device = dev;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
    p->ncu = prop.multiProcessorCount;
  p->nprob = nprob;
  p->total = offsets[nprob];
  p->bc_lo = bc_lo;
  p->bc_hi = bc_hi;
  p->host_offsets.assign(offsets, offsets + nprob + 1);
  bool ok = hipMalloc(&p->offsets, sizeof(int64_t) * (nprob + 1)) == hipSuccess &&
            hipMalloc(&p->dx, sizeof(double) * nprob) == hipSuccess &&
            hipMalloc(&p->ws, sizeof(double) * 10 * p->total) == hipSuccess &&
            hipMalloc(&p->active, sizeof(int32_t) * nprob) == hipSuccess &&
            hipMalloc(&p->tune_status, sizeof(int32_t) * nprob) == hipSuccess &&
            hipMemcpy(p->offsets, offsets, sizeof(int64_t) * (nprob + 1),
                      hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(p->dx, dx, sizeof(double) * nprob, hipMemcpyHostToDevice) == hipSuccess &&
            hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking) == hipSuccess;
  if (ok) ok = build_table(p, p->tl) == ISWENO_OK;
  if (!ok) {
    isweno_batch_plan_destroy(p);
    return ISWENO_ERR_DEVICE;
  }
  *out = p;
  return ISWENO_OK;
}

void isweno_batch_plan_destroy(isweno_batch_plan* p) {
  if (!p) return;
  (void)hipSetDevice(p->device);
  (void)hipDeviceSynchronize();
  free_graphs(p);
  for (auto& kv : p->tables) {
    (void)hipFree(kv.second.start);
    (void)hipFree(kv.second.prob);
  }
  if (p->offsets) (void)hipFree(p->offsets);
  if (p->dx) (void)hipFree(p->dx);
  if (p->ws) (void)hipFree(p->ws);
  if (p->active) (void)hipFree(p->active);
  if (p->tune_status) (void)hipFree(p->tune_status);
  if (p->cap) (void)hipStreamDestroy(p->cap);
  delete p;
}

int isweno_batch_autotune(isweno_ctx* ctx, isweno_batch_plan* p, const isweno_opts* o,
                          const double* U, int32_t* chosen_tile, void* stream) {
  int r;
  if (!ctx || !p || !U) return ISWENO_ERR_ARG;
  if ((r = check_batch_opts(o)) != ISWENO_OK) return r;
  if (hipSetDevice(p->device) != hipSuccess) return ISWENO_ERR_DEVICE;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const size_t bytes = sizeof(double) * 5 * p->total;
  double* S = nullptr;
  double* dt = nullptr;
  if (hipMalloc(&S, bytes) != hipSuccess) return ISWENO_ERR_DEVICE;
  if (hipMalloc(&dt, sizeof(double) * p->nprob) != hipSuccess) {
    (void)hipFree(S);
    return ISWENO_ERR_DEVICE;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  isweno_opts to = *o;
  if (!(to.cfl > 0.0)) to.cfl = 0.5;  // keep the scratch run physical
  float best = 1e30f;
  int best_tl = p->tl, best_bpc = p->blocks_per_cu;
  r = ISWENO_OK;
  for (int tl : kTiles) {
    if ((r = build_table(p, tl)) != ISWENO_OK) break;
    for (int bpc : kBlocksPerCU) {
      float ms_min = 1e30f;
      for (int rep = 0; rep < 3 && r == ISWENO_OK; rep++) {
        if (hipMemcpyAsync(S, U, bytes, hipMemcpyDeviceToDevice, s) != hipSuccess ||
            hipMemsetAsync(p->tune_status, 0, sizeof(int32_t) * p->nprob, s) != hipSuccess ||
            hipEventRecord(e0, s) != hipSuccess ||
            enqueue_step(p, &to, S, dt, nullptr, p->tune_status, tl, bpc, s) != hipSuccess ||
            hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
          r = ISWENO_ERR_DEVICE;
          break;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        ms_min = std::min(ms_min, ms);
      }
      if (r != ISWENO_OK) break;
      if (ms_min < best) {
        best = ms_min;
        best_tl = tl;
        best_bpc = bpc;
      }
    }
    if (r != ISWENO_OK) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(S);
  (void)hipFree(dt);
  if (r != ISWENO_OK) return r;
  if (best_tl != p->tl || best_bpc != p->blocks_per_cu) free_graphs(p);
  p->tl = best_tl;
  p->blocks_per_cu = best_bpc;
  if (chosen_tile) *chosen_tile = best_tl;
  return ISWENO_OK;
}

int isweno_batch_step(isweno_ctx* ctx, isweno_batch_plan* p, const isweno_opts* o, double* U,
                      double* dt, int32_t nsteps, isweno_stats* stats, int32_t* status,
                      void* stream) {
  int r;
  if (!ctx || !p || !U || !dt || !status || nsteps < 0) return ISWENO_ERR_ARG;
  if ((r = check_batch_opts(o)) != ISWENO_OK) return r;
  if (nsteps == 0) return ISWENO_OK;
  if (hipSetDevice(p->device) != hipSuccess) return ISWENO_ERR_DEVICE;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  isweno_batch_plan::Key key{U, dt, stats, status, o->precision, o->weights, o->mood, o->eps,
                             o->cfl, o->dt_max, p->tl, p->blocks_per_cu};
  auto it = p->graphs.find(key);
  hipGraphExec_t exec = nullptr;
  if (it == p->graphs.end()) {
    // capture one step on the plan's own stream (the caller's may be the
    // legacy default stream, which cannot be captured)
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return ISWENO_ERR_DEVICE;
    const hipError_t e =
        enqueue_step(p, o, U, dt, stats, status, p->tl, p->blocks_per_cu, p->cap);
    const hipError_t e2 = hipStreamEndCapture(p->cap, &graph);
    if (e != hipSuccess || e2 != hipSuccess || !graph) {
      if (graph) (void)hipGraphDestroy(graph);
      return ISWENO_ERR_DEVICE;
    }
    const hipError_t e3 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e3 != hipSuccess) return ISWENO_ERR_DEVICE;
    p->graphs[key] = exec;
  } else {
    exec = it->second;
  }
  for (int32_t k = 0; k < nsteps; k++) {
    if (hipGraphLaunch(exec, s) != hipSuccess) return ISWENO_ERR_DEVICE;
  }
  return ISWENO_OK;
}

}  // extern "C"
