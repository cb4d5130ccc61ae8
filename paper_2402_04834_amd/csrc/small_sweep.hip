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

// entry e (0..3) of four values, without indexing a private array
__device__ __forceinline__ float sel4(float a0, float a1, float a2, float a3, int e) {
  const float lo = (e & 1) ? a1 : a0, hi = (e & 1) ? a3 : a2;
  return (e & 2) ? hi : lo;
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
  if (a.mode == 0 && a.gate > 0.0) {
    // residual-gated schedule: skip the update when the message and every input message have settled
    const double* tj = G.terms + job * G.M;
    const double ti = s.msg_init >= 0 ? tj[s.msg_init] : 0.0, tt = s.msg_top >= 0 ? tj[s.msg_top] : 0.0,
                 tb = s.msg_bot >= 0 ? tj[s.msg_bot] : 0.0;
    if (tj[s.msg_out] < a.gate && ti < a.gate && tt < a.gate && tb < a.gate) {
      G.terms[job * G.M + s.msg_out] = 0.0;
      return;
    }
  }
  const int L = 2 * G.d - 1;
  const uint8_t* lab = G.labels + job * L * L;
  const float* mbase = G.msgs + job * G.M * MSTRIDE;

  // Pauli probabilities by code x + 2z
  float pi0, pi1, pi2, pi3;
  if (G.biased) {
    pi0 = G.pi[0];
    pi1 = G.pi[1];
    pi2 = G.pi[2];
    pi3 = G.pi[3];
  } else {
    float p00 = G.p00, pe = G.pe;
    if (G.pdev) {
      const float pj = (float)G.pdev[job >> 2];
      p00 = 1.0f - pj;
      pe = pj / 3.0f;
    }
    pi0 = p00;
    pi1 = pi2 = pi3 = pe;
  }

  // incoming messages by side; the receiver side carries the output (mode 0) or msg_close (mode 1)
  const int out_side = s.frame;
  int mid[4];
  const int init_side = (out_side == SIDE_E) ? SIDE_W : (out_side == SIDE_W) ? SIDE_E : (out_side == SIDE_S) ? SIDE_N
                                                                                                           : SIDE_S;
#pragma unroll
  for (int side = 0; side < 4; ++side) {
    int id = -1;
    if (side == init_side) id = s.msg_init;
    else if (side == out_side) id = (a.mode == 1) ? s.msg_close : -1;
    else if (out_side <= SIDE_W) id = (side == SIDE_N) ? s.msg_top : s.msg_bot;
    else id = (side == SIDE_W) ? s.msg_top : s.msg_bot;
    mid[side] = id;
  }

  // A variable is a check site of the block or of its one-site halo, numbered by its position
  // (r - r0 + 1) * 4 + (c - c0 + 1) < 16; an assignment of all variables is a 16-bit mask.
  auto pos = [&](int r, int c) -> int {
    return (r < 0 || r >= L || c < 0 || c >= L) ? -1 : (r - s.r0 + 1) * 4 + (c - s.c0 + 1);
  };
  int used = 0;
  int qx[2] = {0, 0}, qnb[2][4] = {{-1, -1, -1, -1}, {-1, -1, -1, -1}}, nq = 0;   // qx: label | vertical-edge flag << 2
#pragma unroll
  for (int dr = 0; dr < 2; ++dr)
#pragma unroll
    for (int dc = 0; dc < 2; ++dc) {
      const int r = s.r0 + dr, c = s.c0 + dc;
      if (dr >= s.kr || dc >= s.kc) continue;
      if (((r + c) & 1) != 0) {
        used |= 1 << pos(r, c);
      } else {
        const int nb[4] = {pos(r - 1, c), pos(r, c - 1), pos(r + 1, c), pos(r, c + 1)};
#pragma unroll
        for (int q = 0; q < 2; ++q)
          if (q == nq) {
            qx[q] = (lab[r * L + c] & 3) | ((r & 1) << 2);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              qnb[q][k] = nb[k];
              if (nb[k] >= 0) used |= 1 << nb[k];
            }
          }
        ++nq;
      }
    }
  // legs: the variable (position) each carries, -1 where the leg leaves the grid; message entries
  int legp[4][2] = {{-1, -1}, {-1, -1}, {-1, -1}, {-1, -1}}, K[4];
  float m[4][4];
#pragma unroll
  for (int side = 0; side < 4; ++side) {
    K[side] = (side <= SIDE_W) ? s.kr : s.kc;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      if (i >= K[side]) continue;
      int ra, ca, rb, cb;
      leg_sites(side, s.r0, s.c0, s.kr, s.kc, i, ra, ca, rb, cb);
      legp[side][i] = (((ra + ca) & 1) != 0) ? pos(ra, ca) : pos(rb, cb);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e)
      m[side][e] = (mid[side] >= 0 && e < (1 << K[side])) ? mbase[mid[side] * MSTRIDE + e] : 0.0f;
  }

  auto bitof = [](int x, int p) { return p < 0 ? 0 : (x >> p) & 1; };
  // weight of one assignment x, the receiver side's message included or not
  auto weight = [&](int x, bool with_out) -> float {
    float w = 1.0f;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      if (q >= nq) continue;
      const int u = bitof(x, qnb[q][0]), l = bitof(x, qnb[q][1]), dn = bitof(x, qnb[q][2]), rt = bitof(x, qnb[q][3]);
      // horizontal edge (even row): checks above / below flip x, left / right flip z; vertical edge: swapped
      const bool vert = (qx[q] >> 2) & 1;
      const int px = vert ? (l ^ rt) : (u ^ dn), pz = vert ? (u ^ dn) : (l ^ rt);
      w *= sel4(pi0, pi1, pi2, pi3, (qx[q] ^ px ^ (pz << 1)) & 3);
    }
#pragma unroll
    for (int side = 0; side < 4; ++side) {
      if (mid[side] < 0 || (side == out_side && !with_out)) continue;
      int e = 0;
#pragma unroll
      for (int i = 0; i < 2; ++i)
        if (i < K[side]) e = (e << 1) | bitof(x, legp[side][i]);
      w *= sel4(m[side][0], m[side][1], m[side][2], m[side][3], e);
    }
    return w;
  };

  if (a.mode == 1) {
    double W = 0.0;
    for (int sub = used;; sub = (sub - 1) & used) {
      W += (double)weight(sub, true);
      if (sub == 0) break;
    }
    G.lnW[job * G.nblocks + s.block] = (W > 0.0) ? log(W) : NAN;
    return;
  }
  // outgoing message: entries over the receiver side's legs (leg 0 most significant); the legs fix their
  // (distinct) variables, and a leg leaving the grid only takes 0
  const int Ko = K[out_side], H = 1 << Ko;
  int fixed = 0;
#pragma unroll
  for (int i = 0; i < 2; ++i)
    if (i < Ko && legp[out_side][i] >= 0) fixed |= 1 << legp[out_side][i];
  const int free_mask = used & ~fixed;
  float fin[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    if (h >= H) continue;
    int base = 0;
    bool ok = true;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      if (i >= Ko) continue;
      const int b = (h >> (Ko - 1 - i)) & 1, p = legp[out_side][i];
      if (p < 0) ok = ok && b == 0;
      else base |= b << p;
    }
    float acc = 0.0f;
    if (ok)
      for (int sub = free_mask;; sub = (sub - 1) & free_mask) {
        acc += weight(base | sub, false);
        if (sub == 0) break;
      }
    fin[h] = acc;
  }
  // normalised new message, damping against the old one, distance term
  float* mo = G.msgs + job * G.M * MSTRIDE + s.msg_out * MSTRIDE;
  float ss = 0.0f;
#pragma unroll
  for (int h = 0; h < 4; ++h) ss += fin[h] * fin[h];
  const float rn = ss > 0.0f ? __builtin_amdgcn_rsqf(ss) : 0.0f;
  float dm[4], old[4], t2 = 0.0f;
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    old[h] = h < H ? mo[h] : 0.0f;
    dm[h] = (1.0f - a.eta) * (fin[h] * rn) + a.eta * old[h];
    t2 += dm[h] * dm[h];
  }
  const float rd = t2 > 0.0f ? __builtin_amdgcn_rsqf(t2) : 0.0f;
  float dd = 0.0f, su = 0.0f;
#pragma unroll
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
