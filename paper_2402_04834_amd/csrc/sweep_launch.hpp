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
constexpr int MSTRIDE = 64;      // floats per stored message (2^6) for plans whose blocks are at most 6 wide

constexpr int MAX_GROUPS = 8;   // (d, p) groups of one mixed batch

// One (d, p) group of a sweep launch: its sweeps of the launch's class and its job state.
struct SweepGroup {
  const SweepDesc* sweeps;   // the group's sweeps of this class (count of them)
  const uint8_t* labels;     // [job][L*L] coset labels
  float* msgs;               // [job][M][MSTRIDE] dense messages, position 0 most significant
  double* terms;             // [job][M] distance terms of the last update
  const int32_t* conv;       // [job] converged flags
  double* lnW;               // [job][nblocks] (closing sweeps)
  int64_t jobs;
  int64_t item0;             // first item of the group in the launch
  int32_t count;             // sweeps of this class in the group
  int32_t d, M, nblocks;
  float p00, pe;             // depolarizing noise entries: 1 - p and p / 3
  const double* pdev;        // optional [job / 4] per-syndrome p (overrides p00, pe)
  int32_t biased;            // 1: the qubit entries are pi (Pauli probabilities by code x + 2z)
  float pi[4];
  double pq[4];              // the four Pauli probabilities by code x + 2z in FP64 (truncating kernel)
  int32_t mstride;           // floats per stored message (MSTRIDE unless a block is wider than 6)
  int32_t chi;               // bond dimension (truncating kernel)
};

struct SweepArgs {
  SweepGroup g[MAX_GROUPS];
  int64_t items;             // sum over groups of jobs * count: one wavefront each
  int32_t ngroups;
  int32_t mode;              // 0: message update, 1: closing sweep (W_v)
  int32_t order;             // item order inside a group: 0 sweep-major (item = sweep * jobs + job), 1 job-major
  int32_t bf16;              // 1: products of BF16-rounded inputs (precision mode 1); 0: FP32 products
  float eta;                 // damping
  int32_t small;             // 1: every block is at most 2x2 tensors: one lane per item (small_sweep.hip)
  double gate;               // > 0: skip an update whose message and input messages all changed by less (terms)
  double* tws;               // truncating kernel: workspace of tws_slots slots of trunc_slot_bytes()
  int64_t tws_slots;         // items per launch of the truncating kernel (larger classes run in chunks)
  int64_t item_base;         // first item of the current chunk
};

// Sweep classes of the truncating kernel (any length; sweeps with SweepDesc::trunc set): TRUNC_CLASS, and
// TRUNC_CLASS | 1 for the narrow form (trunc_shape.hpp).
constexpr int TRUNC_CLASS = 1 << 12;
inline bool trunc_class(int cls) { return (cls & ~1) == TRUNC_CLASS; }

// workspace bytes of one truncating-kernel item
size_t trunc_slot_bytes();
// launch the a.items truncating sweeps (in chunks of a.tws_slots items), all of the narrow form or none
hipError_t launch_trunc_sweeps(hipStream_t st, const SweepArgs& a, bool narrow);

// Class of a sweep: the kernel instantiation that runs it -- length, caps present, one position across,
// first site a qubit: code (((kt - 1) * 4 + top * 2 + bottom) * 2 + single) * 2 + q00.
inline int sweep_class(const SweepDesc& s) {
  if (s.trunc) return TRUNC_CLASS | (s.trunc == 2 ? 1 : 0);
  return (((s.kt - 1) * 4 + (s.msg_top >= 0 ? 2 : 0) + (s.msg_bot >= 0 ? 1 : 0)) * 2 + (s.kp == 1 ? 1 : 0)) * 2 +
         ((s.geo & GEO_Q00) ? 1 : 0);
}

// Launch the a.items (job, sweep) items of class `cls` on stream st.
hipError_t launch_sweeps(int cls, hipStream_t st, const SweepArgs& a);

// blocks of at most 2x2 tensors, any class, FP32 (small_sweep.hip)
hipError_t launch_small_sweeps(hipStream_t st, const SweepArgs& a);

// per-length launchers (one translation unit each); variant = class code modulo 16, plus 16 for the
// BF16-input kernels or 32 for the biased-noise kernels
hipError_t launch_sweeps_k1(int variant, dim3 grid, hipStream_t st, const SweepArgs& a);
hipError_t launch_sweeps_k2(int variant, dim3 grid, hipStream_t st, const SweepArgs& a);
hipError_t launch_sweeps_k3(int variant, dim3 grid, hipStream_t st, const SweepArgs& a);
hipError_t launch_sweeps_k4(int variant, dim3 grid, hipStream_t st, const SweepArgs& a);
hipError_t launch_sweeps_k5(int variant, dim3 grid, hipStream_t st, const SweepArgs& a);
hipError_t launch_sweeps_k6(int variant, dim3 grid, hipStream_t st, const SweepArgs& a);

}  // namespace bbp
