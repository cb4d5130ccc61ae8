// small_sweep.hip -- block updates for blocks of at most 2x2 tensors (block size 1 is plain BP between single
// tensors, the paper's naive limit of blockBP): one lane per (job, sweep) instead of one wavefront, since a
// sweep of such a block has at most four crossing configurations and a wavefront would leave 60 of its 64
// lanes idle.
//
// A lane contracts its block directly. Every bond joins a qubit and a check and carries the check's
// variable (checks are COPY tensors), so the block's variables are its own checks and the outside checks
// that its qubits touch across the boundary; a boundary leg carries the variable of whichever of its two
// sites is a check. The lane sums, over all variables not fixed by the output legs, the product of the
// block's qubit entries pi(label flipped by the adjacent variables) and the entries of the incoming messages
// at their legs' values (Sec. III.D update; a leg that leaves the grid has the value 0). Mode 0 produces
// the outgoing message, then normalises (remark 3), damps (remark 7) and stores the distance term
// (remark 4) as the wavefront kernel does; mode 1 the closing contraction W_v of the Bethe estimate
// (Lemma 3.1), all four incoming messages included, summed in FP64.
#include <hip/hip_runtime.h>

#include "geom.hpp"
#include "sweep_launch.hpp"

namespace bbp {
namespace {

constexpr int SIDE_E = 0, SIDE_W = 1, SIDE_S = 2, SIDE_N = 3;

struct Var {          // a check variable of the contraction
  int r, c;
};

// variable index of the check at (r, c), adding it when new; -1 for a site outside the grid
__device__ __forceinline__ int var_of(Var* v, int& nv, int r, int c, int L) {
  if (r < 0 || r >= L || c < 0 || c >= L) return -1;
  for (int k = 0; k < nv; ++k)
    if (v[k].r == r && v[k].c == c) return k;
  v[nv].r = r;
  v[nv].c = c;
  return nv++;
}

// sites (inside, outside) of leg i of the block's side
__device__ __forceinline__ void leg_sites(int side, int r0, int c0, int kr, int kc, int i, int& ra, int& ca, int& rb,
                                         int& cb) {
  switch (side) {
    case SIDE_E: ra = r0 + i; ca = c0 + kc - 1; rb = ra; cb = ca + 1; break;
    case SIDE_W: ra = r0 + i; ca = c0; rb = ra; cb = ca - 1; break;
    case SIDE_S: ra = r0 + kr - 1; ca = c0 + i; rb = ra + 1; cb = ca; break;
    default:     ra = r0; ca = c0 + i; rb = ra - 1; cb = ca; break;
  }
}

__global__ __launch_bounds__(256) void small_sweep_kernel(SweepArgs a) {
  const int64_t item = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (item >= a.items) return;
  int gi = 0;
  for (int k = 1; k < a.ngroups; ++k)
    if (item >= a.g[k].item0) gi = k;
  const SweepGroup& G = a.g[gi];
  const int64_t local = item - G.item0;
  int64_t job, sw;
  if (a.order == 0) {
    sw = local / G.jobs;
    job = local - sw * G.jobs;
  } else {
    job = local / G.count;
    sw = local - job * G.count;
  }
  if (a.mode == 0 && G.conv[job]) return;
  const SweepDesc s = G.sweeps[sw];
  const int L = 2 * G.d - 1;
  const uint8_t* lab = G.labels + job * L * L;
  const float* mbase = G.msgs + job * G.M * MSTRIDE;

  // Pauli probabilities by code x + 2z
  float pi[4];
  if (G.biased) {
    for (int k = 0; k < 4; ++k) pi[k] = G.pi[k];
  } else {
    float p00 = G.p00, pe = G.pe;
    if (G.pdev) {
      const float pj = (float)G.pdev[job >> 2];
      p00 = 1.0f - pj;
      pe = pj / 3.0f;
    }
    pi[0] = p00;
    pi[1] = pi[2] = pi[3] = pe;
  }

  // incoming messages by side; the receiver side carries the output (mode 0) or msg_close (mode 1)
  const int out_side = s.frame;
  const int opp[4] = {SIDE_W, SIDE_E, SIDE_N, SIDE_S};
  int mid[4] = {-1, -1, -1, -1};
  mid[opp[out_side]] = s.msg_init;
  if (out_side <= SIDE_W) {
    mid[SIDE_N] = s.msg_top;
    mid[SIDE_S] = s.msg_bot;
  } else {
    mid[SIDE_W] = s.msg_top;
    mid[SIDE_E] = s.msg_bot;
  }
  if (a.mode == 1) mid[out_side] = s.msg_close;

  // variables: the block's checks, then the outside checks across its boundary
  Var v[12];
  int nv = 0;
  int qr[2], qlab[2], qnb[2][4];   // the block's qubits: row, label, variables (up, left, down, right)
  int nq = 0;
  for (int r = s.r0; r < s.r0 + s.kr; ++r)
    for (int c = s.c0; c < s.c0 + s.kc; ++c)
      if (((r + c) & 1) != 0) var_of(v, nv, r, c, L);
  for (int r = s.r0; r < s.r0 + s.kr; ++r)
    for (int c = s.c0; c < s.c0 + s.kc; ++c)
      if (((r + c) & 1) == 0) {
        qr[nq] = r;
        qlab[nq] = lab[r * L + c] & 3;
        qnb[nq][0] = var_of(v, nv, r - 1, c, L);
        qnb[nq][1] = var_of(v, nv, r, c - 1, L);
        qnb[nq][2] = var_of(v, nv, r + 1, c, L);
        qnb[nq][3] = var_of(v, nv, r, c + 1, L);
        ++nq;
      }
  // legs of each side: the variable each carries (-1 where the leg leaves the grid)
  int legv[4][2], K[4];
  for (int side = 0; side < 4; ++side) {
    K[side] = (side <= SIDE_W) ? s.kr : s.kc;
    for (int i = 0; i < K[side]; ++i) {
      int ra, ca, rb, cb;
      leg_sites(side, s.r0, s.c0, s.kr, s.kc, i, ra, ca, rb, cb);
      const bool a_check = ((ra + ca) & 1) != 0;
      legv[side][i] = a_check ? var_of(v, nv, ra, ca, L)
                              : ((rb < 0 || rb >= L || cb < 0 || cb >= L) ? -1 : var_of(v, nv, rb, cb, L));
    }
  }
  // message entries, read once
  float m[4][4];
  for (int side = 0; side < 4; ++side)
    for (int e = 0; e < 4; ++e)
      m[side][e] = (mid[side] >= 0 && e < (1 << K[side])) ? mbase[mid[side] * MSTRIDE + e] : 0.0f;

  // weight of one assignment x of all variables (bit k = variable k), without the output side's message
  auto weight = [&](int x, bool with_out) -> float {
    float w = 1.0f;
    for (int q = 0; q < nq; ++q) {
      auto val = [&](int k) { return k < 0 ? 0 : (x >> k) & 1; };
      const int u = val(qnb[q][0]), l = val(qnb[q][1]), dn = val(qnb[q][2]), rt = val(qnb[q][3]);
      // horizontal edge (even row): checks above / below flip x, left / right flip z; vertical edge: swapped
      const int px = (qr[q] & 1) ? (l ^ rt) : (u ^ dn);
      const int pz = (qr[q] & 1) ? (u ^ dn) : (l ^ rt);
      w *= pi[(qlab[q] ^ px ^ (pz << 1)) & 3];
    }
    for (int side = 0; side < 4; ++side) {
      if (mid[side] < 0 || (side == out_side && !with_out)) continue;
      int e = 0;
      for (int i = 0; i < K[side]; ++i) {
        const int k = legv[side][i];
        e = (e << 1) | (k < 0 ? 0 : (x >> k) & 1);
      }
      w *= m[side][e];
    }
    return w;
  };

  if (a.mode == 1) {
    double W = 0.0;
    for (int x = 0; x < (1 << nv); ++x) W += (double)weight(x, true);
    G.lnW[job * G.nblocks + s.block] = (W > 0.0) ? log(W) : NAN;
    return;
  }
  // outgoing message: entries over the receiver side's legs (leg 0 most significant)
  const int Ko = K[out_side], H = 1 << Ko;
  int fixed = 0;   // variables the output legs fix
  for (int i = 0; i < Ko; ++i)
    if (legv[out_side][i] >= 0) fixed |= 1 << legv[out_side][i];
  float fin[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int h = 0; h < H; ++h) {
    // the output legs fix their (distinct) variables; a leg leaving the grid only takes 0
    int base = 0;
    bool ok = true;
    for (int i = 0; i < Ko; ++i) {
      const int b = (h >> (Ko - 1 - i)) & 1, k = legv[out_side][i];
      if (k < 0) ok = ok && b == 0;
      else base |= b << k;
    }
    if (!ok) continue;
    float acc = 0.0f;
    const int free_mask = ((1 << nv) - 1) & ~fixed;
    // enumerate the free variables as subsets of free_mask
    for (int sub = free_mask;; sub = (sub - 1) & free_mask) {
      acc += weight(base | sub, false);
      if (sub == 0) break;
    }
    fin[h] = acc;
  }
  // normalised new message, damping against the old one, distance term
  float* mo = G.msgs + job * G.M * MSTRIDE + s.msg_out * MSTRIDE;
  float ss = 0.0f;
  for (int h = 0; h < 4; ++h) ss += fin[h] * fin[h];
  const float rn = ss > 0.0f ? __builtin_amdgcn_rsqf(ss) : 0.0f;
  float dm[4], old[4], t2 = 0.0f;
  for (int h = 0; h < 4; ++h) {
    old[h] = h < H ? mo[h] : 0.0f;
    dm[h] = (1.0f - a.eta) * (fin[h] * rn) + a.eta * old[h];
    t2 += dm[h] * dm[h];
  }
  const float rd = t2 > 0.0f ? __builtin_amdgcn_rsqf(t2) : 0.0f;
  float dd = 0.0f, su = 0.0f;
  for (int h = 0; h < 4; ++h) {
    const float fm = dm[h] * rd;
    dd += (fm - old[h]) * (fm - old[h]);
    su += (fm + old[h]) * (fm + old[h]);
    if (h < H) mo[h] = fm;
  }
  G.terms[job * G.M + s.msg_out] = 0.5 * (double)dd * (double)su;
}

}  // namespace

hipError_t launch_small_sweeps(hipStream_t st, const SweepArgs& a) {
  const dim3 grid((unsigned)((a.items + 255) / 256));
  small_sweep_kernel<<<grid, dim3(256), 0, st>>>(a);
  return hipGetLastError();
}

}  // namespace bbp
