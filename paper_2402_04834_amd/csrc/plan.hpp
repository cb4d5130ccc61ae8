// plan.hpp -- host-side plan of the blockBP decoder: block partition, directed message table, the two
// colour rounds of updates, the Bethe closing sweeps, and the plan-time rank analysis.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

namespace bbp {

constexpr int TRUNC_KMAX = 8;      // widest block and longest sweep of the truncating kernel
constexpr int TRUNC_CHI_MAX = 16;  // largest chi of the truncating kernel

// One block sweep as the device consumes it (plain 64-byte record).
struct SweepDesc {
  int32_t r0, c0, kr, kc;       // block origin and size on the grid
  int32_t frame, kt, kp;        // receiver side; sweep steps; positions across the sweep
  int32_t msg_out;              // outgoing message id, -1 for a Bethe closing sweep
  int32_t msg_init;             // message entering on the side opposite the receiver, -1 if none
  int32_t msg_top, msg_bot;     // side messages entering as end caps, -1 if none
  int32_t msg_close;            // Bethe: message from the receiver side, -1 if none
  int32_t block;                // block index (row-major)
  float flops;                  // algorithmic flops of this sweep
  int32_t geo;                  // GEO_* flags (geom.hpp)
  int32_t trunc;                // 1: the boundary state of this sweep can exceed chi (truncating kernel); 2: the
                                // same in the narrow form (every bond within 8, trunc_shape.hpp)
};
static_assert(sizeof(SweepDesc) == 64, "SweepDesc layout");

struct Plan {
  int d = 0, L = 0, kr = 0, kc = 0, chi = 0;
  int nI = 0, nJ = 0, nblocks = 0, M = 0;
  std::vector<int> row0, rowsz, col0, colsz;
  std::vector<int> edge_src, edge_dst, edge_dir, edge_len;   // directed messages, id = index
  std::vector<SweepDesc> round[2];                            // colour (I+J)%2 == 0 sends first
  std::vector<SweepDesc> bethe;                               // one closing sweep per block
  std::vector<int32_t> pair_ids;                              // undirected edges: (u->v, v->u) ids
  int max_msg_len = 0;
  bool exact = false;        // no boundary state can exceed chi: truncation is the identity
  int mstride = 64;          // floats per stored dense message: 2^max(6, widest block)
  int trunc_sweeps = 0;      // sweeps (rounds and closing) that run in the truncating kernel
  int max_kp = 0;            // widest sweep (positions across)
  int max_rank = 0;          // largest generic Schmidt rank among cuts whose dimensions exceed chi on both sides
  bool gpu_ok = false;
  std::string why;           // reason when !gpu_ok
  double flops_iter = 0.0, flops_bethe = 0.0;
};

// Build the plan (and run the rank analysis) for distance d, blocks kr x kc, bond chi.
Plan make_plan(int d, int kr, int kc, int chi);

// make_plan, cached per (d, kr, kc, chi) for the life of the process (thread-safe).
const Plan& cached_plan(int d, int kr, int kc, int chi);

// Host-side reference of one block sweep in float64 with the GPU's index arithmetic (used only by the
// self-check entry point). labels: L*L grid bytes; msgs: dense messages (stride 64) indexed by id.
int host_sweep(const Plan& plan, const SweepDesc& s, const uint8_t* labels, const float* pi,
               const double* msgs, double* out, double* logscale);

}  // namespace bbp
