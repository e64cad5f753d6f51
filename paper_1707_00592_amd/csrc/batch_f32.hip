// The batched 1D stage kernels of the float form.  That form is held to an
// error bound, not to the oracle's bits, so this file is built with
// multiplies and adds contracted into fused multiply-adds, its FP64 parts
// included; the FP64 kernels (batch.hip) keep every operation as written.
#include "batch_kernels.hpp"

namespace isw {

hipError_t launch_batch_stage_f32(int tl, const BatchArgs& a, int mode, int blocks,
                                  hipStream_t s) {
  return launch_stage_t<float>(tl, a, mode, blocks, s);
}

}  // namespace isw
