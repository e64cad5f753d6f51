// Sweep kernels of the float form (eq. (21), eq. (28) and cut-off weights).
// The float form is held to an error bound, not to the oracle's bits, so
// this file is built with multiplies and adds contracted into fused
// multiply-adds, its FP64 parts included; the FP64 sweeps (kernels.hip,
// sweep_cut.hip) keep every operation as written.  The learned weights'
// sweeps stay in kernels.hip: contracted, they ran slower.
#include "sweep_kernels.hpp"

namespace isw {

hipError_t launch_sweep_f32(int ndim, int D, const SweepArgs& a, int mode, bool readR,
                            hipStream_t s, LaunchEvents ev) {
  return launch_sweep_p<float, false, false>(ndim, D, a, mode, readR, s, ev);
}

hipError_t launch_sweep_cut_f32(int ndim, int D, const SweepArgs& a, int mode, bool readR,
                                hipStream_t s, LaunchEvents ev) {
  return launch_sweep_p<float, false, true>(ndim, D, a, mode, readR, s, ev);
}

}  // namespace isw
