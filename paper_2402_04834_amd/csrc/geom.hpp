// geom.hpp -- geometry of the coset tensor networks and of the in-block sweeps, shared by the host plan
// and the device kernels.
//
// Grid (2d-1) x (2d-1); qubits at (r+c) even, Z-checks at (even r, odd c), X-checks at (odd r, even c)
// (Sec. II.B). Every check is a COPY tensor over its legs; a qubit tensor is the noise probability of its
// label flipped by the adjacent checks: a horizontal edge (even r) is flipped in x by the checks above /
// below and in z by those left / right, a vertical edge (odd r) the other way round (Sec. III.A reading).
//
// A block update toward side F ("frame") sweeps the block in the direction of F: step t walks the block
// columns (F = E, W) or rows (F = S, N) starting on the side opposite to F; position i runs across the
// sweep (rows for E/W, columns for S/N), always in absolute top->bottom / left->right order. In the frame
// every tensor has legs (up, in, down, out): "in" faces the side the sweep came from, "out" the receiver,
// "up"/"down" the two side messages, which enter as the top and bottom end caps of the boundary state.
#pragma once
#include <stdint.h>

#if defined(__HIP__)
#include <hip/hip_runtime.h>
#define BBP_HD __host__ __device__ __forceinline__
#else
#define BBP_HD inline
#endif

namespace bbp {

enum : int { FRAME_E = 0, FRAME_W = 1, FRAME_S = 2, FRAME_N = 3 };

// Geometry flags of a block sweep, uniform over its steps (qubits and checks alternate along both axes,
// and the orientation of the qubits of a step alternates with the step).
enum : int {
  GEO_Q00 = 1,        // the first site of the first step is a qubit
  GEO_SWAP0 = 2,      // orientation flag (qubit_coef's `swap`) of the qubits of the first step
  GEO_TOP_EDGE = 4,   // the up-leg of the first position leaves the grid
  GEO_BOT_EDGE = 8,   // the down-leg of the last position leaves the grid
  GEO_IN_EDGE = 16,   // the in-legs of the first step leave the grid
  GEO_OUT_EDGE = 32,  // the out-legs of the last step leave the grid
};

// Grid site visited at sweep step t, position i of a block with origin (r0, c0) and size kr x kc.
BBP_HD void frame_site(int frame, int r0, int c0, int kr, int kc, int t, int i, int& r, int& c) {
  switch (frame) {
    case FRAME_E: r = r0 + i; c = c0 + t; break;
    case FRAME_W: r = r0 + i; c = c0 + kc - 1 - t; break;
    case FRAME_S: r = r0 + t; c = c0 + i; break;
    default:      r = r0 + kr - 1 - t; c = c0 + i; break;
  }
}

// Dimension of bond j (0..K) of a K-site side message in the open-leg reading: bonds up to K/2 carry the
// first j legs, later bonds the remaining K-j legs.
BBP_HD int cap_dim(int K, int j) { return (j <= K / 2) ? (1 << j) : (1 << (K - j)); }

// Coefficient T(vi, hi, vo, ho) of a qubit tensor in a sweep frame: the noise probability of its label
// flipped by the parities of its vertical (vi ^ vo) and crossing (hi ^ ho) legs -- which of x / z each parity
// flips depends on the edge orientation and the frame (`swap`). absent = bits (up, in, down, out) of legs
// that leave the grid; such a leg only takes the value 0.
BBP_HD float qubit_coef(int label, int swap, int absent, float p00, float p01, float p10, float p11, int vi, int hi,
                        int vo, int ho) {
  if (((absent & 1) && vi) || ((absent & 2) && hi) || ((absent & 4) && vo) || ((absent & 8) && ho)) return 0.0f;
  const int pv = vi ^ vo, ph = hi ^ ho;
  const int ex = (label & 1) ^ (swap ? ph : pv);
  const int ez = ((label >> 1) & 1) ^ (swap ? pv : ph);
  const int k = ex * 2 + ez;
  return (k == 0) ? p00 : (k == 1) ? p01 : (k == 2) ? p10 : p11;
}

// Entry e = vi*8 + hi*4 + vo*2 + ho of a COPY tensor in a sweep frame: 1 when all present legs agree.
BBP_HD float copy_coef(int absent, int e) {
  const int vi = (e >> 3) & 1, hi = (e >> 2) & 1, vo = (e >> 1) & 1, ho = e & 1;
  if (((absent & 1) && vi) || ((absent & 2) && hi) || ((absent & 4) && vo) || ((absent & 8) && ho)) return 0.0f;
  int ref = -1;
  bool ok = true;
  if (!(absent & 1)) ref = vi;
  if (!(absent & 2)) { if (ref < 0) ref = hi; else if (hi != ref) ok = false; }
  if (!(absent & 4)) { if (ref < 0) ref = vo; else if (vo != ref) ok = false; }
  if (!(absent & 8)) { if (ref < 0) ref = ho; else if (ho != ref) ok = false; }
  return ok ? 1.0f : 0.0f;
}

// Entry e = vi*8 + hi*4 + vo*2 + ho of the frame table T[vi][hi][vo][ho] of the tensor at grid site (r, c)
// for a sweep toward `frame`. label bit 0 = x, bit 1 = z of f_s L at the site; pi = noise table
// {p(I), p(Z), p(X), p(Y)} indexed x*2 + z. Legs that leave the grid have dimension 1 and are padded with
// zeros at value 1.
BBP_HD float site_entry(int frame, int L, int r, int c, int label, float p00, float p01, float p10, float p11,
                        int e) {
  const bool au = (r == 0), al = (c == 0), ad = (r == L - 1), ar = (c == L - 1);
  bool a_up, a_in, a_dn, a_out;
  switch (frame) {
    case FRAME_E: a_up = au; a_in = al; a_dn = ad; a_out = ar; break;
    case FRAME_W: a_up = au; a_in = ar; a_dn = ad; a_out = al; break;
    case FRAME_S: a_up = al; a_in = au; a_dn = ar; a_out = ad; break;
    default:      a_up = al; a_in = ad; a_dn = ar; a_out = au; break;
  }
  const int vi = (e >> 3) & 1, hi = (e >> 2) & 1, vo = (e >> 1) & 1, ho = e & 1;
  if (((r + c) & 1) == 0) {
    const int swap = ((r & 1) != 0) != (frame >= FRAME_S);
    const int absent = (a_up ? 1 : 0) | (a_in ? 2 : 0) | (a_dn ? 4 : 0) | (a_out ? 8 : 0);
    return qubit_coef(label, swap, absent, p00, p01, p10, p11, vi, hi, vo, ho);
  }
  // COPY: all present legs equal (absent legs are pinned to 0 and take no part)
  return copy_coef((a_up ? 1 : 0) | (a_in ? 2 : 0) | (a_dn ? 4 : 0) | (a_out ? 8 : 0), e);
}

// All 16 entries of the frame table (see site_entry).
BBP_HD void site_table(int frame, int L, int r, int c, int label, const float* pi, float* T) {
  for (int e = 0; e < 16; ++e) T[e] = site_entry(frame, L, r, c, label, pi[0], pi[1], pi[2], pi[3], e);
}

}  // namespace bbp
