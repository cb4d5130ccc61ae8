// sweep_launch.hpp -- host interface of the block-sweep kernels. The kernels are instantiated per sweep
// length (1..6 steps) in separate translation units (sweep_kernel.hip compiled with BBP_KT = 1..6).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "geom.hpp"
#include "plan.hpp"

namespace bbp {

#ifndef BBP_SWEEP_WAVES
#define BBP_SWEEP_WAVES 1
#endif
// independent sweeps (wavefronts) per workgroup: one, so that the wavefront of a converged job, or one
// that finishes early, frees its slot at once
constexpr int SWEEP_WAVES = BBP_SWEEP_WAVES;
constexpr int MSTRIDE = 64;      // floats per stored message (2^6)

struct SweepArgs {
  const SweepDesc* sweeps;   // this launch's sweeps (all of one class: length, caps present)
  int d;
  const uint8_t* labels;     // [job][L*L] coset labels
  float* msgs;               // [job][M][MSTRIDE] dense messages, position 0 most significant
  int M;
  double* terms;             // [job][M] distance terms of the last update
  const int32_t* conv;       // [job] converged flags
  float p00, pe;             // depolarizing noise entries: 1 - p and p / 3
  float eta;                 // damping
  int mode;                  // 0: message update, 1: closing sweep (W_v)
  double* lnW;               // [job][nblocks] (mode 1)
  int nblocks;
  int64_t jobs;
};

// Class of a sweep: the kernel instantiation that runs it -- length, caps present, one position across,
// first site a qubit: code (((kt - 1) * 4 + top * 2 + bottom) * 2 + single) * 2 + q00.
inline int sweep_class(const SweepDesc& s) {
  return (((s.kt - 1) * 4 + (s.msg_top >= 0 ? 2 : 0) + (s.msg_bot >= 0 ? 1 : 0)) * 2 + (s.kp == 1 ? 1 : 0)) * 2 +
         ((s.geo & GEO_Q00) ? 1 : 0);
}

// Launch the sweeps a.sweeps[0 .. count) of class `cls` for a.jobs jobs on stream st.
hipError_t launch_sweeps(int cls, unsigned count, hipStream_t st, const SweepArgs& a);

// per-length launchers (one translation unit each); variant = class code modulo 16
hipError_t launch_sweeps_k1(int variant, dim3 grid, hipStream_t st, const SweepArgs& a);
hipError_t launch_sweeps_k2(int variant, dim3 grid, hipStream_t st, const SweepArgs& a);
hipError_t launch_sweeps_k3(int variant, dim3 grid, hipStream_t st, const SweepArgs& a);
hipError_t launch_sweeps_k4(int variant, dim3 grid, hipStream_t st, const SweepArgs& a);
hipError_t launch_sweeps_k5(int variant, dim3 grid, hipStream_t st, const SweepArgs& a);
hipError_t launch_sweeps_k6(int variant, dim3 grid, hipStream_t st, const SweepArgs& a);

}  // namespace bbp
