// bmps_launch.hpp -- host interface of the boundary-MPS kernels (bmps.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace bbp {

constexpr int BMPS_CHI_MAX = 16;   // bond dimension of the compressed boundary MPS (padded to 2 chi_max = 32)

struct BmpsArgs {
  const uint8_t* labels;   // [job][L*L] coset labels (code x + 2z)
  double* A;               // [job][L][16 * 2 * 16] compressed rows (workspace)
  double* Q;               // [job][L][64 * 32] pass-1 factors (workspace)
  double* loglik;          // [job] ln Z estimates
  const double* pdev;      // optional [job / 4] per-syndrome p
  int32_t d, chi;
  int64_t jobs;            // syndromes * 4
  double p00, pe;          // depolarizing entries 1 - p, p / 3
  int32_t biased;          // 1: pi holds the Pauli probabilities by code
  double pi[4];
};

// device bytes of the per-job MPS state (A and Q) for `jobs` coset networks of distance d
size_t bmps_state_bytes(int d, int64_t jobs);

// contract every job (one wavefront each)
hipError_t launch_bmps_contract(hipStream_t st, const BmpsArgs& a);
// decide every syndrome and write its correction (correction may be NULL)
hipError_t launch_bmps_decide(hipStream_t st, const BmpsArgs& a, uint8_t* coset, uint8_t* correction);

// coset labels of every syndrome (bbp.hip)
hipError_t launch_labels(hipStream_t st, const uint8_t* syn, int d, int64_t batch, uint8_t* labels);

}  // namespace bbp
