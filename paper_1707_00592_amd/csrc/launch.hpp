// Host-side launch entry points of the device kernels (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace isw {

struct SweepArgs;
struct BatchArgs;

// Optional timing events: when set, the launch itself records the start of
// its (first) kernel into start and the end of its (last) kernel into stop.
struct LaunchEvents {
  hipEvent_t start = nullptr, stop = nullptr;
};

// One axis D of a stage: mode is an OutMode, readR adds the partial sum of
// the previous axes.  precision: 0 = FP64, 1 = FP32 reconstruction/flux.
hipError_t launch_sweep(int precision, int ndim, int D, const SweepArgs& a, int mode,
                        bool readR, hipStream_t s, LaunchEvents ev = {});

// launch_sweep for the cut-off weights (W_CUTOFF).
hipError_t launch_sweep_cut(int precision, int ndim, int D, const SweepArgs& a, int mode,
                            bool readR, hipStream_t s, LaunchEvents ev = {});

// One whole RK stage of a 2D grid (x and y faces of each tile in one
// launch); mode is OUT_RHS or one of the OUT_RK* modes (OUT_RK1L and
// OUT_RK2L: the step's time step formed inside the first stage).  Not for
// the learned weights.
hipError_t launch_stage2d(int precision, const SweepArgs& a, int mode, hipStream_t s,
                          LaunchEvents ev = {});
// The float form's instantiations (built apart, with contraction).
hipError_t launch_stage2d_f32(const SweepArgs& a, int mode, hipStream_t s, LaunchEvents ev);
hipError_t launch_sweep_f32(int ndim, int D, const SweepArgs& a, int mode, bool readR,
                            hipStream_t s, LaunchEvents ev);
hipError_t launch_sweep_cut_f32(int ndim, int D, const SweepArgs& a, int mode, bool readR,
                                hipStream_t s, LaunchEvents ev);

// Bytes of the time-step words (the max and the ticket).
constexpr size_t kCflWordsBytes = 256;

// dt = cfl / max sum_d (|u_d| + c)/dx_d (clipped to dt_max > 0), one launch;
// the words (kCflWordsBytes) are zero on entry and left zero.
hipError_t launch_cfl(int ndim, const double* U, const int64_t* n, const double* dx,
                      double cfl, double dt_max, unsigned long long* words, double* dt,
                      int ncu, hipStream_t s, LaunchEvents ev = {});

// dt = cfl / max over n per-workgroup maxima (bits of positive doubles, as
// the first fused 2D stage or the first 3D sweep stores them), clipped to
// dt_max > 0; one workgroup.
hipError_t launch_cfl_final(const unsigned long long* part, int64_t n, double cfl,
                            double dt_max, double* dt, hipStream_t s, LaunchEvents ev = {});

// The number of workgroups (tiles) of the fused 2D stage on an nx x ny grid.
int64_t stage2d_tiles(int64_t nx, int64_t ny);

// The number of workgroups (tiles) of a 3D x sweep on an n[0] x n[1] x n[2]
// grid (one OUT_PARTIAL_S maximum each).
int64_t sweep3d_x_tiles(const int64_t* n);

// Zeroes the time-step words by a kernel (used instead of a
// memset, which a captured graph should not contain).
hipError_t launch_zero_cfl(unsigned long long* w, hipStream_t s);

}  // namespace isw
