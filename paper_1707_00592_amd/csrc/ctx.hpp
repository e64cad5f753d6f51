// Library context (the opaque isweno_ctx of isweno.h) and the host-side
// argument checks shared by the entry points (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <vector>

#include "isweno.h"

struct isweno_ctx {
  int device = 0;
  int ncu = 256;
  double* ws = nullptr;          // two state-sized buffers (U1, U2)
  size_t ws_bytes = 0;
  unsigned long long* maxbits = nullptr;  // time-step reduction words (max, ticket)
  unsigned long long* shortcut = nullptr;  // 256 x 3 reconstruction-shortcut counters (timing only)
  float* mlp_part = nullptr;     // per-workgroup partial gradients of isweno_mlp_loss_grad
  int mlp_part_blocks = 0;
  // kernel timing
  struct Rec {
    int kind;
    hipEvent_t a, b;
  };
  bool timing = false;
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  double total_ms[ISWENO_K_COUNT] = {};
  int64_t launches[ISWENO_K_COUNT] = {};
  // RK3 steps captured as HIP graphs, keyed by everything a captured step
  // bakes in (pointers, grid, options, workspace)
  hipStream_t cap = nullptr;
  std::map<std::string, hipGraphExec_t> graphs;
};

namespace isw {

// ISWENO_OK, or ISWENO_ERR_ARG for a grid the stage kernels cannot take
// (ndim outside 1..3, an axis with no cells or dx <= 0, an unknown boundary
// condition, a reflective end on an axis of fewer than 3 cells, unused axes
// not of one cell, a cell count that overflows).
int check_grid(const isweno_grid* g);

// ISWENO_OK, ISWENO_ERR_ARG (unknown precision, weights or MOOD flag, a
// negative epsilon, nonzero reserved fields, learned weights without a
// network) or ISWENO_ERR_UNSUPPORTED (learned weights in FP64).
int check_opts(const isweno_opts* o);

}  // namespace isw
