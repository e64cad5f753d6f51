// The fused 2D stage, float-form instantiations.  The float form is held to
// an error bound, not to the oracle's bits, so this file is built with
// multiplies and adds contracted into fused multiply-adds (one rounding
// instead of two, fewer instructions); its FP64 parts (primitive recovery,
// the admissibility check, the update) are contracted as well.
#include "stage2d_kernel.hpp"

namespace isw {

hipError_t launch_stage2d_f32(const SweepArgs& a, int mode, hipStream_t s, LaunchEvents ev) {
  if (a.weights == W_MLP) return hipErrorInvalidValue;
  return launch_p<float>(a, mode, s, ev);
}

}  // namespace isw
