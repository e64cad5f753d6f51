// C ABI of the WENO-IS library (declarations and contracts in isweno.h).
#include <hip/hip_runtime.h>

#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "ctx.hpp"
#include "isweno.h"
#include "launch.hpp"
#include "sweep.hpp"

namespace {

constexpr size_t kShortcutBytes = 256 * 3 * sizeof(unsigned long long);

hipEvent_t take_event(isweno_ctx* c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Timing of one launch when enabled: a pair of events the launch itself
// records at the start and end of its kernels (on the launch stream),
// collected into the context's records after the launch.
struct KTimer {
  isweno_ctx* c;
  int kind;
  isw::LaunchEvents ev;
  KTimer(isweno_ctx* c_, int kind_) : c(c_), kind(kind_) {
    if (c && c->timing) {
      ev.start = take_event(c);
      ev.stop = ev.start ? take_event(c) : nullptr;
      if (!ev.stop && ev.start) {
        c->pool.push_back(ev.start);
        ev.start = nullptr;
      }
    }
  }
  ~KTimer() {
    if (ev.start) c->recs.push_back({kind, ev.start, ev.stop});
  }
};

void drain_timing(isweno_ctx* c) {
  for (auto& r : c->recs) {
    float ms = 0.0f;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      c->total_ms[r.kind] += ms;
      c->launches[r.kind] += 1;
    }
    c->pool.push_back(r.a);
    c->pool.push_back(r.b);
  }
  c->recs.clear();
}

}  // namespace

namespace isw {

int check_grid(const isweno_grid* g) {
  if (!g || g->ndim < 1 || g->ndim > 3 || g->reserved != 0) return ISWENO_ERR_ARG;
  for (int d = 0; d < 3; d++) {
    if (d < g->ndim) {
      if (g->n[d] < 1 || !(g->dx[d] > 0.0)) return ISWENO_ERR_ARG;
      if (g->bc_lo[d] < 0 || g->bc_lo[d] > 2 || g->bc_hi[d] < 0 || g->bc_hi[d] > 2)
        return ISWENO_ERR_ARG;
      if ((g->bc_lo[d] == ISWENO_BC_REFLECTIVE || g->bc_hi[d] == ISWENO_BC_REFLECTIVE) &&
          g->n[d] < 3)
        return ISWENO_ERR_ARG;
    } else if (g->n[d] != 1) {
      return ISWENO_ERR_ARG;
    }
  }
  const int64_t N = g->n[0] * g->n[1] * g->n[2];
  if (N / g->n[0] / g->n[1] != g->n[2]) return ISWENO_ERR_ARG;  // overflow
  return ISWENO_OK;
}

int check_opts(const isweno_opts* o) {
  if (!o || o->reserved != 0 || o->reserved2 != 0) return ISWENO_ERR_ARG;
  if (o->precision != ISWENO_FP64 && o->precision != ISWENO_FP32) return ISWENO_ERR_ARG;
  if (o->weights < 0 || o->weights > 3) return ISWENO_ERR_ARG;
  if (o->mood < 0 || o->mood > 2) return ISWENO_ERR_ARG;
  if (!(o->eps >= 0.0)) return ISWENO_ERR_ARG;
  if (o->weights == ISWENO_W_MLP) {
    // the learned weights run with the float32 reconstruction only
    if (!o->mlp_params) return ISWENO_ERR_ARG;
    if (o->precision != ISWENO_FP32) return ISWENO_ERR_UNSUPPORTED;
  }
  return ISWENO_OK;
}

}  // namespace isw

namespace {

using isw::check_grid;
using isw::check_opts;

int64_t ncells(const isweno_grid* g) { return g->n[0] * g->n[1] * g->n[2]; }

void free_graphs(isweno_ctx* c) {
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  c->graphs.clear();
}

int ensure_ws(isweno_ctx* c, size_t bytes) {
  if (c->ws_bytes >= bytes) return ISWENO_OK;
  if (c->ws) {
    // the old buffers may still be in use by queued work on any stream,
    // and captured steps refer to them
    if (hipDeviceSynchronize() != hipSuccess) return ISWENO_ERR_DEVICE;
    free_graphs(c);
    (void)hipFree(c->ws);
    c->ws = nullptr;
    c->ws_bytes = 0;
  }
  if (hipMalloc(&c->ws, bytes) != hipSuccess) return ISWENO_ERR_DEVICE;
  c->ws_bytes = bytes;
  return ISWENO_OK;
}

isw::SweepArgs base_args(const isweno_grid* g, const isweno_opts* o, isweno_stats* st) {
  isw::SweepArgs a{};
  for (int d = 0; d < 3; d++) {
    a.n[d] = g->n[d];
    a.dx[d] = g->dx[d];
    a.bcl[d] = g->bc_lo[d];
    a.bch[d] = g->bc_hi[d];
  }
  a.weights = o->weights;
  a.mood = o->mood;
  a.eps = o->eps;
  a.stats = reinterpret_cast<isw::StatsDev*>(st);
  a.mlp = o->mlp_params;
  a.mlp_thr = o->mlp_conf_threshold;
  return a;
}

// The time step formed inside a 3D stage: the x sweep stores one max wave
// speed per tile into part, and one workgroup turns the n maxima into dt
// before the y sweep.
struct DtInStage {
  unsigned long long* part;
  int64_t n;
  double cfl, dt_max;
  double* dt;
};

// One evaluation of L on Uin followed by the output step `mode`; the partial
// sums of the first ndim-1 axes go to `partial` (which may alias the final
// output buffer, cell by cell).  timed = false: no timing events or
// shortcut counts even while timing is enabled (the allocation-free step).
// fin (3D only): form the step's dt after the x sweep.
hipError_t stage(isweno_ctx* c, const isweno_grid* g, const isweno_opts* o, isw::SweepArgs a,
                 double* partial, int mode, bool timed, hipStream_t s,
                 const DtInStage* fin = nullptr) {
  const int nd = g->ndim;
  isweno_ctx* tc = timed ? c : nullptr;
  unsigned long long* shortcut = timed && c->timing ? c->shortcut : nullptr;
  if (nd == 2 && o->weights != ISWENO_W_MLP) {
    // one fused launch: the x terms stay in registers
    isw::SweepArgs b = a;
    b.shortcut = shortcut;  // never inside a captured graph
    KTimer t(tc, ISWENO_K_STAGE2D);
    return isw::launch_stage2d(o->precision, b, mode, s, t.ev);
  }
  for (int D = 0; D < nd; D++) {
    isw::SweepArgs b = a;
    b.bc_lo = g->bc_lo[D];
    b.bc_hi = g->bc_hi[D];
    const bool last = D == nd - 1;
    b.R = partial;
    if (!last) b.Rout = partial;
    b.shortcut = shortcut;  // never inside a captured graph
    int m = last ? mode : isw::OUT_PARTIAL;
    const bool speeds = fin && D == 0 && nd == 3;
    if (speeds) {
      b.cflp = fin->part;
      m = isw::OUT_PARTIAL_S;
    }
    {
      KTimer t(tc, ISWENO_K_SWEEP_X + D);
      const hipError_t e = isw::launch_sweep(o->precision, nd, D, b, m, D > 0, s, t.ev);
      if (e != hipSuccess) return e;
    }
    if (speeds) {
      KTimer t(tc, ISWENO_K_CFL);
      const hipError_t e =
          isw::launch_cfl_final(fin->part, fin->n, fin->cfl, fin->dt_max, fin->dt, s, t.ev);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

// Whether a step forms its time step inside its first stage: CFL steps of
// 2D and 3D grids (not 1D, whose only sweep needs dt, nor the learned
// weights).
bool fused_dt(const isweno_grid* g, const isweno_opts* o) {
  return o->cfl > 0.0 && g->ndim >= 2 && o->weights != ISWENO_W_MLP;
}

// Per-tile maxima a step with fused_dt stores: one per tile of the fused 2D
// stage or of the 3D x sweep (else none).
int64_t dt_slots(const isweno_grid* g, const isweno_opts* o) {
  if (!fused_dt(g, o)) return 0;
  return g->ndim == 2 ? isw::stage2d_tiles(g->n[0], g->n[1]) : isw::sweep3d_x_tiles(g->n);
}

// One RK3 step on stream s: the time step (when cfl > 0), then the three
// stages, with the intermediate states in U1 and U2 (nc*N each), the
// time-step words maxbits (two, zero on entry, left zero) and, for
// fused_dt, the per-tile maxima in part (dt_slots).  With fused_dt in 2D
// the first stage writes L(U) into U1 and its tiles' max wave speeds, one
// workgroup turns those into dt, and the second stage reads U + dt L; in
// 3D the first stage's x sweep stores the maxima and dt is formed before
// its y sweep.  The same states, bit for bit, without a pass of its own
// over U.
hipError_t enqueue_rk3(isweno_ctx* c, const isweno_grid* g, const isweno_opts* o, double* U,
                       double* dt, isweno_stats* stats, double* U1, double* U2,
                       unsigned long long* maxbits, unsigned long long* part, bool timed,
                       hipStream_t s) {
  hipError_t e;
  const bool fused = fused_dt(g, o);
  const bool fused2d = fused && g->ndim == 2;
  if (o->cfl > 0.0 && !fused) {
    KTimer t(timed ? c : nullptr, ISWENO_K_CFL);
    if ((e = isw::launch_cfl(g->ndim, U, g->n, g->dx, o->cfl, o->dt_max, maxbits, dt, c->ncu,
                             s, t.ev)) != hipSuccess)
      return e;
  }
  isw::SweepArgs a = base_args(g, o, stats);
  a.dt = dt;
  a.U0 = U;
  if (fused2d) {
    // stage 1: L(U) into U1, the tiles' max wave speeds into part; dt
    a.Uin = U;
    a.Rout = U1;
    a.cflp = part;
    if ((e = stage(c, g, o, a, U1, isw::OUT_RK1L, timed, s)) != hipSuccess) return e;
    {
      KTimer t(timed ? c : nullptr, ISWENO_K_CFL);
      if ((e = isw::launch_cfl_final(part, dt_slots(g, o), o->cfl, o->dt_max, dt, s, t.ev)) !=
          hipSuccess)
        return e;
    }
    // stage 2: U2 = 3/4 U + 1/4 (U1 + dt L(U1)), U1 = U + dt L(U) formed on the fly
    a.cflp = nullptr;
    a.R = U1;
    a.Uout = U2;
    if ((e = stage(c, g, o, a, U2, isw::OUT_RK2L, timed, s)) != hipSuccess) return e;
  } else {
    // stage 1: U1 = U + dt L(U) (3D with fused_dt: dt formed after its x sweep)
    a.Uin = U;
    a.Uout = U1;
    const DtInStage fin{part, dt_slots(g, o), o->cfl, o->dt_max, dt};
    if ((e = stage(c, g, o, a, U1, isw::OUT_RK1, timed, s, fused ? &fin : nullptr)) !=
        hipSuccess)
      return e;
    // stage 2: U2 = 3/4 U + 1/4 (U1 + dt L(U1))
    a.Uin = U1;
    a.Uout = U2;
    if ((e = stage(c, g, o, a, U2, isw::OUT_RK2, timed, s)) != hipSuccess) return e;
  }
  // stage 3: U = 1/3 U + 2/3 (U2 + dt L(U2)); partial sums in U1
  a.R = nullptr;
  a.Uin = U2;
  a.Uout = U;
  return stage(c, g, o, a, U1, isw::OUT_RK3, timed, s);
}

// Workspace of the context: U1 = ws, U2 = ws + nc*N, then the per-tile
// maxima of a fused_dt step.
size_t ws_bytes(const isweno_grid* g, const isweno_opts* o) {
  const size_t sz = (size_t)(4 + g->ndim) * (size_t)ncells(g);
  return 2 * sz * sizeof(double) + (size_t)dt_slots(g, o) * sizeof(unsigned long long);
}

hipError_t enqueue_rk3_ws(isweno_ctx* c, const isweno_grid* g, const isweno_opts* o, double* U,
                          double* dt, isweno_stats* stats, hipStream_t s) {
  const size_t sz = (size_t)(4 + g->ndim) * (size_t)ncells(g);
  auto* part = reinterpret_cast<unsigned long long*>(c->ws + 2 * sz);
  return enqueue_rk3(c, g, o, U, dt, stats, c->ws, c->ws + sz, c->maxbits, part, true, s);
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free step (isweno_rk3_step_noalloc): the
// time-step reduction words in its first kCflWordsBytes, then U1, U2 and
// the per-tile maxima of a step that forms dt in its first stage.  A device
// global: every GPU the library runs on holds its own copy from the load of
// the library's code object until the process ends.  Host code never uses
// the array's name as an address: scratch_addr() returns this device's copy,
// looked up once per device with hipGetSymbolAddress.
// ---------------------------------------------------------------------------
constexpr size_t kScratchStates = (size_t)128 << 20;  // bytes for U1, U2 (and the maxima)
static __device__ __align__(256) unsigned char scratch[isw::kCflWordsBytes + kScratchStates];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};

// This device's scratch (the caller has made `device` current), or null
// when the runtime cannot resolve the symbol.
unsigned char* scratch_addr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    g_scratch_ptr[device] = static_cast<unsigned char*>(p);
  }
  return g_scratch_ptr[device];
}

// Everything a captured RK3 step depends on (compared bytewise).
struct StepKey {
  const void* U;
  const void* dt;
  const void* stats;
  const void* ws;
  isweno_grid grid;
  isweno_opts opts;
};
constexpr size_t kMaxGraphs = 64;

}  // namespace

extern "C" {

const char* isweno_version(void) { return "isweno 0.1 (gfx950)"; }

int isweno_create(isweno_ctx** out, int device) {
  if (!out) return ISWENO_ERR_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return ISWENO_ERR_ARG;
  if (hipSetDevice(device) != hipSuccess) return ISWENO_ERR_DEVICE;
  isweno_ctx* c = new (std::nothrow) isweno_ctx();
  if (!c) return ISWENO_ERR_DEVICE;
  c->device = device;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
    c->ncu = prop.multiProcessorCount;
  // this device's scratch of the allocation-free step, resolved once here
  // (with the device current) so that the step itself makes no runtime
  // lookups
  if (!scratch_addr(device)) {
    delete c;
    return ISWENO_ERR_DEVICE;
  }
  if (hipMalloc(&c->maxbits, isw::kCflWordsBytes) != hipSuccess ||
      hipMemset(c->maxbits, 0, isw::kCflWordsBytes) != hipSuccess ||
      hipMalloc(&c->shortcut, kShortcutBytes) != hipSuccess ||
      hipMemset(c->shortcut, 0, kShortcutBytes) != hipSuccess) {
    if (c->maxbits) (void)hipFree(c->maxbits);
    if (c->shortcut) (void)hipFree(c->shortcut);
    delete c;
    return ISWENO_ERR_DEVICE;
  }
  *out = c;
  return ISWENO_OK;
}

void isweno_destroy(isweno_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  free_graphs(c);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  if (c->ws) (void)hipFree(c->ws);
  if (c->maxbits) (void)hipFree(c->maxbits);
  if (c->shortcut) (void)hipFree(c->shortcut);
  if (c->mlp_part) (void)hipFree(c->mlp_part);
  drain_timing(c);
  for (hipEvent_t e : c->pool) (void)hipEventDestroy(e);
  delete c;
}

int isweno_rhs(isweno_ctx* c, const isweno_grid* g, const isweno_opts* o, const double* U,
               double* dUdt, isweno_stats* stats, void* stream) {
  int r;
  if (!c || !U || !dUdt) return ISWENO_ERR_ARG;
  if ((r = check_grid(g)) != ISWENO_OK) return r;
  if ((r = check_opts(o)) != ISWENO_OK) return r;
  const int64_t N = ncells(g);
  const int nc = 4 + g->ndim;
  if ((U < dUdt + (size_t)nc * N) && (dUdt < U + (size_t)nc * N)) return ISWENO_ERR_ARG;
  if (hipSetDevice(c->device) != hipSuccess) return ISWENO_ERR_DEVICE;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  isw::SweepArgs a = base_args(g, o, stats);
  a.Uin = U;
  a.Rout = dUdt;
  return stage(c, g, o, a, dUdt, isw::OUT_RHS, true, s) == hipSuccess ? ISWENO_OK
                                                                       : ISWENO_ERR_DEVICE;
}

int isweno_cfl_dt(isweno_ctx* c, const isweno_grid* g, const isweno_opts* o, const double* U,
                  double* dt, void* stream) {
  int r;
  if (!c || !U || !dt) return ISWENO_ERR_ARG;
  if ((r = check_grid(g)) != ISWENO_OK) return r;
  if (!o || !(o->cfl > 0.0)) return ISWENO_ERR_ARG;
  if (hipSetDevice(c->device) != hipSuccess) return ISWENO_ERR_DEVICE;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  KTimer t(c, ISWENO_K_CFL);
  return isw::launch_cfl(g->ndim, U, g->n, g->dx, o->cfl, o->dt_max, c->maxbits, dt, c->ncu,
                         s, t.ev) == hipSuccess
             ? ISWENO_OK
             : ISWENO_ERR_DEVICE;
}

int isweno_rk3_step(isweno_ctx* c, const isweno_grid* g, const isweno_opts* o, double* U,
                    double* dt, isweno_stats* stats, void* stream) {
  int r;
  if (!c || !U || !dt) return ISWENO_ERR_ARG;
  if ((r = check_grid(g)) != ISWENO_OK) return r;
  if ((r = check_opts(o)) != ISWENO_OK) return r;
  if (hipSetDevice(c->device) != hipSuccess) return ISWENO_ERR_DEVICE;
  if ((r = ensure_ws(c, ws_bytes(g, o))) != ISWENO_OK) return r;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  // Launch directly with kernel timing on (events bracket each kernel) and
  // when dt is clipped (dt_max > 0: a value that usually changes from call
  // to call, and a graph per value would only be captured to be dropped);
  // otherwise replay the step's graph (captured on first use).
  if (c->timing || o->dt_max > 0.0)
    return enqueue_rk3_ws(c, g, o, U, dt, stats, s) == hipSuccess ? ISWENO_OK
                                                                  : ISWENO_ERR_DEVICE;
  StepKey k;
  std::memset(&k, 0, sizeof(k));
  k.U = U;
  k.dt = dt;
  k.stats = stats;
  k.ws = c->ws;
  k.grid = *g;
  k.opts = *o;
  std::string key(reinterpret_cast<const char*>(&k), sizeof(k));
  auto it = c->graphs.find(key);
  hipGraphExec_t exec = nullptr;
  if (it != c->graphs.end()) {
    exec = it->second;
  } else {
    if (!c->cap && hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking) != hipSuccess) {
      c->cap = nullptr;
      return ISWENO_ERR_DEVICE;
    }
    if (c->graphs.size() >= kMaxGraphs) {
      // bounded cache: the caller's streams may still run old graphs
      if (hipDeviceSynchronize() != hipSuccess) return ISWENO_ERR_DEVICE;
      free_graphs(c);
    }
    // capture on the context's own stream (the caller's may be the legacy
    // default stream, which cannot be captured)
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return ISWENO_ERR_DEVICE;
    const hipError_t e = enqueue_rk3_ws(c, g, o, U, dt, stats, c->cap);
    const hipError_t e2 = hipStreamEndCapture(c->cap, &graph);
    if (e != hipSuccess || e2 != hipSuccess || !graph) {
      if (graph) (void)hipGraphDestroy(graph);
      return ISWENO_ERR_DEVICE;
    }
    const hipError_t e3 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e3 != hipSuccess) return ISWENO_ERR_DEVICE;
    c->graphs.emplace(std::move(key), exec);
  }
  return hipGraphLaunch(exec, s) == hipSuccess ? ISWENO_OK : ISWENO_ERR_DEVICE;
}

int isweno_rk3_step_noalloc(isweno_ctx* c, const isweno_grid* g, const isweno_opts* o,
                            double* U, double* dt, isweno_stats* stats, void* stream) {
  int r;
  if (!c || !U || !dt) return ISWENO_ERR_ARG;
  if ((r = check_grid(g)) != ISWENO_OK) return r;
  if ((r = check_opts(o)) != ISWENO_OK) return r;
  const int64_t N = ncells(g);
  const int nc = 4 + g->ndim;
  if ((uint64_t)N > kScratchStates / (2 * sizeof(double) * (size_t)nc) ||
      ws_bytes(g, o) > kScratchStates)
    return ISWENO_ERR_ARG;
  if (hipSetDevice(c->device) != hipSuccess) return ISWENO_ERR_DEVICE;
  unsigned char* base = scratch_addr(c->device);  // resolved by isweno_create
  if (!base) return ISWENO_ERR_DEVICE;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  auto* maxbits = reinterpret_cast<unsigned long long*>(base);
  double* U1 = reinterpret_cast<double*>(base + isw::kCflWordsBytes);
  double* U2 = U1 + (size_t)nc * (size_t)N;
  auto* part = reinterpret_cast<unsigned long long*>(U2 + (size_t)nc * (size_t)N);
  // the reduction words keep whatever the previous call on this GPU left:
  // clear them with a kernel (no memset node, should a caller capture this)
  if (o->cfl > 0.0 && isw::launch_zero_cfl(maxbits, s) != hipSuccess) return ISWENO_ERR_DEVICE;
  return enqueue_rk3(c, g, o, U, dt, stats, U1, U2, maxbits, part, false, s) == hipSuccess
             ? ISWENO_OK
             : ISWENO_ERR_DEVICE;
}

int isweno_timing_enable(isweno_ctx* c, int enable) {
  if (!c) return ISWENO_ERR_ARG;
  drain_timing(c);
  for (int k = 0; k < ISWENO_K_COUNT; k++) {
    c->total_ms[k] = 0.0;
    c->launches[k] = 0;
  }
  if (hipDeviceSynchronize() != hipSuccess || hipMemset(c->shortcut, 0, kShortcutBytes) != hipSuccess)
    return ISWENO_ERR_DEVICE;
  c->timing = enable != 0;
  return ISWENO_OK;
}

int isweno_shortcut_read(isweno_ctx* c, int64_t* counts) {
  if (!c || !counts) return ISWENO_ERR_ARG;
  unsigned long long h[256 * 3];
  if (hipDeviceSynchronize() != hipSuccess ||
      hipMemcpy(h, c->shortcut, kShortcutBytes, hipMemcpyDeviceToHost) != hipSuccess)
    return ISWENO_ERR_DEVICE;
  for (int d = 0; d < 3; d++) {
    unsigned long long t = 0;
    for (int k = 0; k < 256; k++) t += h[k * 3 + d];
    counts[d] = (int64_t)t;
  }
  return ISWENO_OK;
}

int isweno_timing_read(isweno_ctx* c, int kind, double* total_ms, int64_t* launches) {
  if (!c || kind < 0 || kind >= ISWENO_K_COUNT) return ISWENO_ERR_ARG;
  drain_timing(c);
  if (total_ms) *total_ms = c->total_ms[kind];
  if (launches) *launches = c->launches[kind];
  return ISWENO_OK;
}

// Batch and learned-weight entry points are provided in batch.hip / mlp.hip.

}  // extern "C"
