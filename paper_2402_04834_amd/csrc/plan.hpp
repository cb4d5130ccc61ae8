// plan.hpp -- host-side plan of the blockBP decoder: block partition, directed message table, the two
// colour rounds of updates, the Bethe closing sweeps, and the plan-time rank analysis.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

namespace bbp {

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
  int32_t col_off;              // index of this sweep's first column descriptor
  int32_t pad;
};
static_assert(sizeof(SweepDesc) == 64, "SweepDesc layout");

// Per-column constants of a sweep (the uniform part of sweep.hpp's Column), precomputed on the host.
struct ColumnDesc {
  int32_t top_kind, top_Pold, top_Pnew, top_R2;
  int32_t bot_kind, bot_Pold, bot_Pnew, bot_R2;
  int32_t flags;       // bit 0: site 0 qubit; 1: site 0 up-leg absent; 2: last site qubit;
                       // 3: last site down-leg absent; 4: single position (kp == 1)
  int32_t nmid;        // middle qubits
  int32_t mids;        // their positions, 4 bits each
  int32_t in_absent, out_absent;
  int32_t pad[3];
  // per position i: block-local row r - r0 in bits 0..3 and column c - c0 in bits 4..7, qubit flag bit 8,
  // orientation swap bit 9, absent legs (up, in, down, out) bits 10..13
  int32_t site[6];
  int32_t pad2[10];
};
static_assert(sizeof(ColumnDesc) == 128, "ColumnDesc layout");

struct Plan {
  int d = 0, L = 0, kr = 0, kc = 0, chi = 0;
  int nI = 0, nJ = 0, nblocks = 0, M = 0;
  std::vector<int> row0, rowsz, col0, colsz;
  std::vector<int> edge_src, edge_dst, edge_dir, edge_len;   // directed messages, id = index
  std::vector<SweepDesc> round[2];                            // colour (I+J)%2 == 0 sends first
  std::vector<SweepDesc> bethe;                               // one closing sweep per block
  std::vector<int32_t> pair_ids;                              // undirected edges: (u->v, v->u) ids
  std::vector<ColumnDesc> columns;                            // all sweeps' column descriptors
  int max_msg_len = 0;
  bool exact = false;        // no boundary state can exceed chi: truncation is the identity
  int max_rank = 0;          // largest generic Schmidt rank found across cuts that could bind
  bool gpu_ok = false;
  std::string why;           // reason when !gpu_ok
  double flops_iter = 0.0, flops_bethe = 0.0;
};

// Build the plan (and run the rank analysis) for distance d, blocks kr x kc, bond chi.
Plan make_plan(int d, int kr, int kc, int chi);

// Host-side reference of one block sweep in float64 with the GPU's index arithmetic (used only by the
// self-check entry point). labels: L*L grid bytes; msgs: dense messages (stride 64) indexed by id.
int host_sweep(const Plan& plan, const SweepDesc& s, const uint8_t* labels, const float* pi,
               const double* msgs, double* out, double* logscale);

}  // namespace bbp
