// The fused 2D stage, FP64 instantiations and the dispatcher (the kernel
// and its launch templates are in stage2d_kernel.hpp).  This file is built
// without contraction of multiplies and adds: the FP64 path evaluates every
// expression in the order written, which the oracle follows too.  The float
// form's instantiations are built from stage2d_f32.hip.
#include "stage2d_kernel.hpp"

namespace isw {

int64_t stage2d_tiles(int64_t nx, int64_t ny) {
  return ((nx + kTX - 1) / kTX) * ((ny + kTY - 1) / kTY);
}

hipError_t launch_stage2d(int precision, const SweepArgs& a, int mode, hipStream_t s,
                          LaunchEvents ev) {
  if (a.weights == W_MLP) return hipErrorInvalidValue;
  return precision == 1 ? launch_stage2d_f32(a, mode, s, ev) : launch_p<double>(a, mode, s, ev);
}

}  // namespace isw
