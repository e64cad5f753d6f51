// FP64 sweep kernels of the cut-off weights (W_CUTOFF), instantiated apart
// from the other forms: the extra branch of the reconstruction would
// otherwise raise the register count of every stage kernel.  The float
// form's are in sweep_f32.hip.
#include "sweep_kernels.hpp"

namespace isw {

hipError_t launch_sweep_cut(int precision, int ndim, int D, const SweepArgs& a, int mode,
                            bool readR, hipStream_t s, LaunchEvents ev) {
  return precision == 1 ? launch_sweep_cut_f32(ndim, D, a, mode, readR, s, ev)
                        : launch_sweep_p<double, false, true>(ndim, D, a, mode, readR, s, ev);
}

}  // namespace isw
