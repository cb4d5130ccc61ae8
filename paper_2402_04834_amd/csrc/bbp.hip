// bbp.hip -- gfx950 kernels and C ABI of the blockBP surface-code decoder.
//
// Data path for a batch of syndromes (one "job" = one syndrome x one coset, job = 4*syndrome + coset):
//   labels_kernel     syndrome -> f_s (left/up check chains) -> coset labels f_s L on the grid (Alg. 1)
//   init_kernel       uniform unit messages (remark 2), convergence flags cleared
//   update_kernel     one block message update per workgroup (eq. of the BP update evaluated as in
//                     Sec. III.D), normalisation (remark 3), damping (remark 7), distance term (remark 4)
//   delta_kernel      convergence distance per job and early exit (Alg. 1 BP loop)
//   update_kernel     (closing mode) W_v of every block for the Bethe estimate (Lemma 3.1)
//   finalize_kernel   ln Z = sum ln W_v - sum ln <m_uv, m_vu>, decision rule, correction f_s L*
//
// Block update. The boundary state of the sweep is a dense FP32 array psi[top cap][h_0..h_{kp-1}][bottom
// cap] in LDS (<= 4096 entries for 6x6 blocks). A column is absorbed in kp+2 passes: the top side-message
// site (cap pass), the kp tensors of the column as in-place 4x4 transforms on the pair (vertical bond,
// crossing bond), and the bottom side-message site. The side messages enter in the open-leg reading: bond
// j of a K-site message carries its first j legs up to the middle site and its last K-j legs after it, the
// dense message sitting on the middle site. After every column the state is normalised and the norm is
// accumulated as a log-scale. The plan proves (exact rank analysis) that no boundary state can exceed
// bond chi for the options accepted here, so the compression to chi is the identity and is not executed.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/bbp.h"
#include "geom.hpp"
#include "plan.hpp"
#include "sweep.hpp"

using bbp::SweepDesc;

namespace {

constexpr int NT = 256;          // threads per update workgroup (4 waves)
constexpr int SMAX = 4096;       // max dense boundary-state entries (6x6 blocks, caps of dimension 8)
constexpr int BMAX = 2048;       // max pass-1 intermediate (top cap advanced, bottom cap not yet)
constexpr int MSTRIDE = 64;      // floats per stored message (2^6)

thread_local std::string g_err = "no error";

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIP_TRY(expr)                                                                           \
  do {                                                                                          \
    hipError_t _e = (expr);                                                                     \
    if (_e != hipSuccess) return fail(BBP_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

// --------------------------------------------------------------------------------------------------
// a1/a2: syndrome -> coset labels
__global__ __launch_bounds__(256) void labels_kernel(const uint8_t* __restrict__ syn, int d, int64_t batch,
                                                     uint8_t* __restrict__ labels) {
  const int b = blockIdx.x;
  const int L = 2 * d - 1, m = 2 * d * (d - 1), nz = d * (d - 1);
  __shared__ uint8_t s[2 * 32 * 31];
  for (int i = threadIdx.x; i < m; i += blockDim.x) s[i] = syn[(int64_t)b * m + i] & 1;
  __syncthreads();
  for (int site = threadIdx.x; site < L * L; site += blockDim.x) {
    const int r = site / L, c = site % L;
    int x = 0, z = 0;
    if ((r & 1) == 0 && (c & 1) == 0) {
      for (int cc = c + 1; cc < L; cc += 2) x ^= s[(r / 2) * (d - 1) + (cc - 1) / 2];      // Z-checks right of it
      for (int rr = r + 1; rr < L; rr += 2) z ^= s[nz + ((rr - 1) / 2) * d + c / 2];        // X-checks below it
    }
    const int lx = (r == 0 && (c & 1) == 0) ? 1 : 0;   // logical X: row 0 of horizontal edges
    const int lz = (c == 0 && (r & 1) == 0) ? 1 : 0;   // logical Z: column 0 of horizontal edges
    const int bx[4] = {0, 1, 1, 0}, bz[4] = {0, 0, 1, 1};
    for (int k = 0; k < 4; ++k) {
      const int xx = x ^ (bx[k] & lx), zz = z ^ (bz[k] & lz);
      labels[((int64_t)b * 4 + k) * L * L + site] = (uint8_t)(xx | (zz << 1));
    }
  }
}

__global__ void init_kernel(float* __restrict__ msgs, const int32_t* __restrict__ edge_len, int M, int64_t jobs,
                            int32_t* __restrict__ conv, int32_t* __restrict__ iters) {
  const int64_t job = blockIdx.x;
  for (int e = threadIdx.x; e < M * MSTRIDE; e += blockDim.x) {
    const int id = e / MSTRIDE, h = e % MSTRIDE;
    const int K = edge_len[id];
    msgs[job * M * MSTRIDE + e] = (h < (1 << K)) ? exp2f(-0.5f * K) : 0.0f;
  }
  if (threadIdx.x == 0) {
    conv[job] = 0;
    iters[job] = 0;
  }
}

__device__ __forceinline__ float block_sum(float v, float* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  float t = 0.0f;
  for (int w = 0; w < NT / 64; ++w) t += red[w];
  return t;
}

__device__ __forceinline__ double wave_sum_d(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
  return __shfl(v, 0);
}

// --------------------------------------------------------------------------------------------------
// Block sweeps. Lane h of a wavefront holds the crossing-bond configuration h (position 0 in the most
// significant of kp bits). The boundary state is a set of rows (top cap index n, bottom cap index s), one
// float per lane, stored in LDS as rows of 64 floats (row = n * Ps + s); the four waves of a workgroup take
// the rows round-robin. A qubit's 2x2 transform pairs lane h with lane h ^ bit: a cross-lane shuffle and two
// multiply-adds with coefficients chosen per lane from the check bits above and below. Only the cap sites
// mix rows (through LDS). The column structure is described in sweep.hpp.

// phi[np][v] of a cap site of kind KIND, reading psi[n] = sc * base[n * stride].
template <int KIND>
__device__ __forceinline__ float capv(const float* __restrict__ m, int Pold, int lPold, int Pnew, int R2, int np,
                                      int v, const float* base, int stride, float sc) {
  if constexpr (KIND == bbp::CAP_NONE) {
    return v == 0 ? sc * base[0] : 0.0f;
  } else if constexpr (KIND == bbp::CAP_F_LT) {
    return v == (np & 1) ? sc * base[(np >> 1) * stride] : 0.0f;
  } else if constexpr (KIND == bbp::CAP_F_EQ) {
    float acc = 0.0f;
    for (int a = 0; a < Pold; ++a) acc = fmaf(m[(a * 2 + v) * R2 + np], base[a * stride], acc);
    return sc * acc;
  } else if constexpr (KIND == bbp::CAP_F_GT) {
    return sc * base[(v * Pnew + np) * stride];
  } else if constexpr (KIND == bbp::CAP_B_GT) {
    return (v == (np >> lPold)) ? sc * base[(np & (Pold - 1)) * stride] : 0.0f;
  } else if constexpr (KIND == bbp::CAP_B_EQ) {
    float acc = 0.0f;
    for (int b = 0; b < Pold; ++b) acc = fmaf(m[(np * 2 + v) * R2 + b], base[b * stride], acc);
    return sc * acc;
  } else {   // CAP_B_LT
    return sc * base[(2 * np + v) * stride];
  }
}

struct LaneCoef {
  // site 0 (qubit): coefficients for (emitted leg v, own / partner input bit), scaled by the column scale;
  // middle qubits: own / partner
  float q00, q01, q10, q11;
  float cm_own[3], cm_par[3];
  int am[3];      // byte addresses of the partner lanes of the middle qubits (ds_bpermute)
};

constexpr int NW = NT / 64;

// cross-lane read of `x` from the lane whose byte address is `addr` (= 4 * lane)
__device__ __forceinline__ float lane_read(int addr, float x) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(x)));
}

// Kinds whose emitted leg is fixed by the new cap index (one of the two values of v is zero).
template <int KIND>
__device__ __forceinline__ constexpr bool single_v() {
  return KIND == bbp::CAP_NONE || KIND == bbp::CAP_F_LT || KIND == bbp::CAP_B_GT;
}
template <int KIND>
__device__ __forceinline__ int the_v(int np, int lPold) {
  if constexpr (KIND == bbp::CAP_NONE) return 0;
  else if constexpr (KIND == bbp::CAP_F_LT) return np & 1;
  else return np >> lPold;
}

// pass 1 (A -> B): top cap of kind KIND, site 0 and the middle qubits, for this wave's rows
template <int KIND>
__device__ __forceinline__ void pass1_rows(const bbp::ColumnDesc& cd, const LaneCoef& lc, const float* A, float* B,
                                           const float* mt, int h, int hr, int a0, int vchk, int Ptn, int Pso,
                                           int lso, float sc, int wid) {
  const bool q0 = cd.flags & 1;
  const int lPold = __builtin_ctz(cd.top_Pold);
  const int stride = Pso * 64;
  const int nmid = cd.nmid;
#pragma unroll 4
  for (int row = wid; row < Ptn * Pso; row += NW) {
    const int np = row >> lso, sb = row & (Pso - 1);
    const float* base = A + sb * 64 + hr;
    float out;
    if (q0) {
      if constexpr (single_v<KIND>()) {
        const int v = the_v<KIND>(np, lPold);
        const float f = capv<KIND>(mt, cd.top_Pold, lPold, cd.top_Pnew, cd.top_R2, np, v, base, stride, 1.0f);
        const float g = lane_read(a0, f);
        out = v ? (lc.q10 * f + lc.q11 * g) : (lc.q00 * f + lc.q01 * g);
      } else {
        const float f0 = capv<KIND>(mt, cd.top_Pold, lPold, cd.top_Pnew, cd.top_R2, np, 0, base, stride, 1.0f);
        const float f1 = capv<KIND>(mt, cd.top_Pold, lPold, cd.top_Pnew, cd.top_R2, np, 1, base, stride, 1.0f);
        const float g0 = lane_read(a0, f0);
        const float g1 = lane_read(a0, f1);
        out = lc.q00 * f0 + lc.q01 * g0 + lc.q10 * f1 + lc.q11 * g1;
      }
    } else {
      out = sc * capv<KIND>(mt, cd.top_Pold, lPold, cd.top_Pnew, cd.top_R2, np, vchk, base, stride, 1.0f);
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      if (j < nmid) {
        const float par = lane_read(lc.am[j], out);
        out = lc.cm_own[j] * out + lc.cm_par[j] * par;
      }
    }
    B[(np * Pso + sb) * 64 + h] = out;
  }
}

// pass 2 (B -> A): bottom cap of kind KIND and the last site, then the out-leg projections; returns the
// wave-local sum of squares
template <int KIND>
__device__ __forceinline__ float pass2_rows(const bbp::ColumnDesc& cd, const float* B, float* A, const float* mb,
                                            int h, int kp, int al, int vchk, float l00, float l01, float l10,
                                            float l11, int Ptn, int Pso, int Psn, int lsn, int wid) {
  const bool ql = cd.flags & 4;
  const int lPold = __builtin_ctz(cd.bot_Pold);
  float ss = 0.0f;
#pragma unroll 4
  for (int row = wid; row < Ptn * Psn; row += NW) {
    const int n = row >> lsn, sp = row & (Psn - 1);
    const float* base = B + n * Pso * 64 + h;
    float out;
    if (ql) {
      if constexpr (single_v<KIND>()) {
        const int v = the_v<KIND>(sp, lPold);
        const float f = capv<KIND>(mb, cd.bot_Pold, lPold, cd.bot_Pnew, cd.bot_R2, sp, v, base, 64, 1.0f);
        const float g = lane_read(al, f);
        out = v ? (l10 * f + l11 * g) : (l00 * f + l01 * g);
      } else {
        const float f0 = capv<KIND>(mb, cd.bot_Pold, lPold, cd.bot_Pnew, cd.bot_R2, sp, 0, base, 64, 1.0f);
        const float f1 = capv<KIND>(mb, cd.bot_Pold, lPold, cd.bot_Pnew, cd.bot_R2, sp, 1, base, 64, 1.0f);
        const float g0 = lane_read(al, f0);
        const float g1 = lane_read(al, f1);
        out = l00 * f0 + l01 * g0 + l10 * f1 + l11 * g1;
      }
    } else {
      out = capv<KIND>(mb, cd.bot_Pold, lPold, cd.bot_Pnew, cd.bot_R2, sp, vchk, base, 64, 1.0f);
    }
    if (cd.out_absent) {
      for (int b = 0; b < kp; ++b)
        if (cd.out_absent & (1 << b)) {
          const float o2 = __shfl_xor(out, 1 << b);
          out = (h & (1 << b)) ? 0.0f : out + o2;
        }
    }
    A[(n * Psn + sp) * 64 + h] = out;
    ss = fmaf(out, out, ss);
  }
  return ss;
}

// mode 0: BP update of message s.msg_out; mode 1: closing sweep W_v of block s.block.
__global__ __launch_bounds__(NT) void update_kernel(const SweepDesc* __restrict__ sweeps,
                                                    const bbp::ColumnDesc* __restrict__ cols, int d,
                                                    const uint8_t* __restrict__ labels, float* __restrict__ msgs,
                                                    int M, double* __restrict__ terms,
                                                    const int32_t* __restrict__ conv, float p0, float p1, float p2,
                                                    float p3, float eta, int mode, double* __restrict__ lnW,
                                                    int nblocks) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave index, uniform within the wave
  const int L = 2 * d - 1;

  __shared__ float A[SMAX];
  __shared__ float B[BMAX];
  __shared__ float T[36 * 16];
  __shared__ float mt[MSTRIDE], mb[MSTRIDE];
  __shared__ float red[NW];

  const int64_t job = blockIdx.x;
  if (mode == 0 && conv[job]) return;
  const SweepDesc s = sweeps[blockIdx.y];
  const int kt = s.kt, kp = s.kp, H = 1 << kp;

  const uint8_t* lab = labels + job * L * L;
  for (int q = tid; q < kt * kp * 16; q += NT) {
    int r, c;
    const int site = q >> 4;
    bbp::frame_site(s.frame, s.r0, s.c0, s.kr, s.kc, site / kp, site % kp, r, c);
    T[q] = bbp::site_entry(s.frame, L, r, c, lab[r * L + c], p0, p1, p2, p3, q & 15);
  }
  const float* mbase = msgs + job * M * MSTRIDE;
  const bool has_top = s.msg_top >= 0, has_bot = s.msg_bot >= 0;
  if (wid == 0) {
    mt[lane] = has_top ? mbase[s.msg_top * MSTRIDE + lane] : 0.0f;
    mb[lane] = has_bot ? mbase[s.msg_bot * MSTRIDE + lane] : 0.0f;
    A[lane] = (s.msg_init >= 0) ? mbase[s.msg_init * MSTRIDE + lane] : (lane == 0 ? 1.0f : 0.0f);
  }
  __syncthreads();

  const int h = lane;
  double logscale = 0.0;
  float scale = 1.0f;
  int Ps = 1;
  for (int t = 0; t < kt; ++t) {
    const bbp::ColumnDesc cd = cols[s.col_off + t];
    const float* Tt = &T[t * kp * 16];
    // frame-table entry T(vi, hi, vo, ho) of the site at position i of this column
    auto coef = [&](int i, int vi, int hi, int vo, int ho) { return Tt[i * 16 + vi * 8 + hi * 4 + vo * 2 + ho]; };
    const int Ptn = cd.top_Pnew, Psn = cd.bot_Pnew, Pso = Ps;
    const int lso = __builtin_ctz(Pso), lsn = __builtin_ctz(Psn);
    const float sc = scale;
    const int hr = h & ~cd.in_absent;      // checks entering from outside the grid: free variable
    if (cd.flags & 16) {
      // ---- one position (kp == 1): generic path --------------------------------------------------------
      bbp::CapInfo top{cd.top_kind, cd.top_Pold, cd.top_Pnew, cd.top_R2};
      bbp::CapInfo bot{cd.bot_kind, cd.bot_Pold, cd.bot_Pnew, cd.bot_R2};
      for (int row = wid; row < Ptn * Pso; row += NW) {
        const int np = row >> lso, sb = row & (Pso - 1);
        auto get = [&](int n) { return sc * A[(n * Pso + sb) * 64 + hr]; };
        for (int vt = 0; vt < 2; ++vt)
          B[((np * 2 + vt) * Pso + sb) * 64 + h] = bbp::cap_phi<float>(top, mt, np, vt, get);
      }
      __syncthreads();
      const int hol = h & 1;
      float ss = 0.0f;
      for (int row = wid; row < Ptn * Psn; row += NW) {
        const int n = row >> lsn, sp = row & (Psn - 1);
        float out = 0.0f;
        if (cd.flags & 4) {
          for (int vt = 0; vt < 2; ++vt)
            for (int vb = 0; vb < 2; ++vb) {
              auto get = [&](int sb) { return B[((n * 2 + vt) * Pso + sb) * 64 + h]; };
              const float f = bbp::cap_phi<float>(bot, mb, sp, vb, get);
              const float g = __shfl_xor(f, 1);
              out += coef(0, vt, hol, vb, hol) * f + coef(0, vt, 1 - hol, vb, hol) * g;
            }
        } else {
          const int vt = (cd.flags & 2) ? 0 : hol;
          const int vb = (cd.flags & 8) ? 0 : hol;
          auto get = [&](int sb) { return B[((n * 2 + vt) * Pso + sb) * 64 + h]; };
          out = bbp::cap_phi<float>(bot, mb, sp, vb, get);
        }
        if (cd.out_absent & 1) {
          const float o2 = __shfl_xor(out, 1);
          out = hol ? 0.0f : out + o2;
        }
        A[(n * Psn + sp) * 64 + h] = out;
        ss = fmaf(out, out, ss);
      }
      for (int o = 32; o > 0; o >>= 1) ss += __shfl_xor(ss, o);
      if (lane == 0) red[wid] = ss;
    } else {
      // ---- pass 1 -----------------------------------------------------------------------------------
      LaneCoef lc;
      const int b0 = bbp::pos_bit(kp, 0);
      const int ho0 = (h & b0) ? 1 : 0;
      const int vo0 = (h & bbp::pos_bit(kp, 1)) ? 1 : 0;
      lc.q00 = sc * coef(0, 0, ho0, vo0, ho0);
      lc.q01 = sc * coef(0, 0, 1 - ho0, vo0, ho0);
      lc.q10 = sc * coef(0, 1, ho0, vo0, ho0);
      lc.q11 = sc * coef(0, 1, 1 - ho0, vo0, ho0);
      const int a0 = (h ^ b0) << 2;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        lc.cm_own[j] = 0.0f;
        lc.cm_par[j] = 0.0f;
        lc.am[j] = h << 2;
        if (j < cd.nmid) {
          const int i = (cd.mids >> (4 * j)) & 15;
          const int bi = bbp::pos_bit(kp, i);
          const int vi = (h & bbp::pos_bit(kp, i - 1)) ? 1 : 0;
          const int vo = (h & bbp::pos_bit(kp, i + 1)) ? 1 : 0;
          const int ho = (h & bi) ? 1 : 0;
          lc.cm_own[j] = coef(i, vi, ho, vo, ho);
          lc.cm_par[j] = coef(i, vi, 1 - ho, vo, ho);
          lc.am[j] = (h ^ bi) << 2;
        }
      }
      const int vchk0 = (cd.flags & 2) ? 0 : ho0;
      switch (cd.top_kind) {
        case bbp::CAP_NONE: pass1_rows<bbp::CAP_NONE>(cd, lc, A, B, mt, h, hr, a0, vchk0, Ptn, Pso, lso, sc, wid); break;
        case bbp::CAP_F_LT: pass1_rows<bbp::CAP_F_LT>(cd, lc, A, B, mt, h, hr, a0, vchk0, Ptn, Pso, lso, sc, wid); break;
        case bbp::CAP_F_EQ: pass1_rows<bbp::CAP_F_EQ>(cd, lc, A, B, mt, h, hr, a0, vchk0, Ptn, Pso, lso, sc, wid); break;
        case bbp::CAP_F_GT: pass1_rows<bbp::CAP_F_GT>(cd, lc, A, B, mt, h, hr, a0, vchk0, Ptn, Pso, lso, sc, wid); break;
        case bbp::CAP_B_GT: pass1_rows<bbp::CAP_B_GT>(cd, lc, A, B, mt, h, hr, a0, vchk0, Ptn, Pso, lso, sc, wid); break;
        case bbp::CAP_B_EQ: pass1_rows<bbp::CAP_B_EQ>(cd, lc, A, B, mt, h, hr, a0, vchk0, Ptn, Pso, lso, sc, wid); break;
        default:            pass1_rows<bbp::CAP_B_LT>(cd, lc, A, B, mt, h, hr, a0, vchk0, Ptn, Pso, lso, sc, wid); break;
      }
      __syncthreads();
      // ---- pass 2 -----------------------------------------------------------------------------------
      const int bl = bbp::pos_bit(kp, kp - 1);
      const int hol = (h & bl) ? 1 : 0;
      const int vil = (h & bbp::pos_bit(kp, kp - 2)) ? 1 : 0;
      const float l00 = coef(kp - 1, vil, hol, 0, hol), l01 = coef(kp - 1, vil, 1 - hol, 0, hol);
      const float l10 = coef(kp - 1, vil, hol, 1, hol), l11 = coef(kp - 1, vil, 1 - hol, 1, hol);
      const int vchkl = (cd.flags & 8) ? 0 : hol;
      const int al = (h ^ bl) << 2;
      float ss;
      switch (cd.bot_kind) {
        case bbp::CAP_NONE: ss = pass2_rows<bbp::CAP_NONE>(cd, B, A, mb, h, kp, al, vchkl, l00, l01, l10, l11, Ptn, Pso, Psn, lsn, wid); break;
        case bbp::CAP_F_LT: ss = pass2_rows<bbp::CAP_F_LT>(cd, B, A, mb, h, kp, al, vchkl, l00, l01, l10, l11, Ptn, Pso, Psn, lsn, wid); break;
        case bbp::CAP_F_EQ: ss = pass2_rows<bbp::CAP_F_EQ>(cd, B, A, mb, h, kp, al, vchkl, l00, l01, l10, l11, Ptn, Pso, Psn, lsn, wid); break;
        case bbp::CAP_F_GT: ss = pass2_rows<bbp::CAP_F_GT>(cd, B, A, mb, h, kp, al, vchkl, l00, l01, l10, l11, Ptn, Pso, Psn, lsn, wid); break;
        case bbp::CAP_B_GT: ss = pass2_rows<bbp::CAP_B_GT>(cd, B, A, mb, h, kp, al, vchkl, l00, l01, l10, l11, Ptn, Pso, Psn, lsn, wid); break;
        case bbp::CAP_B_EQ: ss = pass2_rows<bbp::CAP_B_EQ>(cd, B, A, mb, h, kp, al, vchkl, l00, l01, l10, l11, Ptn, Pso, Psn, lsn, wid); break;
        default:            ss = pass2_rows<bbp::CAP_B_LT>(cd, B, A, mb, h, kp, al, vchkl, l00, l01, l10, l11, Ptn, Pso, Psn, lsn, wid); break;
      }
      for (int o = 32; o > 0; o >>= 1) ss += __shfl_xor(ss, o);
      if (lane == 0) red[wid] = ss;
    }
    __syncthreads();
    float tot = 0.0f;
#pragma unroll
    for (int w = 0; w < NW; ++w) tot += red[w];
    const float nrm = sqrtf(tot);
    scale = (nrm > 0.0f) ? 1.0f / nrm : 0.0f;
    logscale += (double)logf(nrm);
    Ps = Psn;
  }
  if (wid == 0) {
    const float fin = (lane < H) ? A[lane] * scale : 0.0f;
    if (mode == 1) {
      // closing contraction with the message from the receiver side (or the grid edge)
      double w = 0.0;
      if (s.msg_close >= 0) w = (double)mbase[s.msg_close * MSTRIDE + lane] * (double)fin;
      else if (lane == 0) w = fin;
      w = wave_sum_d(w);
      if (lane == 0) lnW[job * nblocks + s.block] = (w > 0.0) ? logscale + log(w) : NAN;
    } else {
      // normalised new message, damping against the old one, distance term
      float* mo = msgs + job * M * MSTRIDE + s.msg_out * MSTRIDE;
      const float old = (lane < H) ? mo[lane] : 0.0f;
      const double n2 = wave_sum_d((double)fin * fin);
      const float inv = (float)(1.0 / sqrt(n2));
      const float dm = (1.0f - eta) * (fin * inv) + eta * old;
      const double dd = wave_sum_d((double)dm * dm);
      const double od = wave_sum_d((double)old * old);
      const double c = wave_sum_d((double)dm * old);
      const float fm = dm * (float)(1.0 / sqrt(dd));
      if (lane < H) mo[lane] = fm;
      if (lane == 0) terms[job * M + s.msg_out] = 2.0 - 2.0 * (c * c) / (dd * od);
    }
  }
}

__global__ void delta_kernel(const double* __restrict__ terms, int M, int64_t jobs, int32_t* __restrict__ conv,
                             int32_t* __restrict__ iters, double* __restrict__ delta, double delta0, int fixed) {
  const int64_t job = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (job >= jobs || conv[job]) return;
  double acc = 0.0;
  for (int e = 0; e < M; ++e) acc += terms[job * M + e];
  const double dl = sqrt(fmax(acc, 0.0)) / (M > 0 ? M : 1);
  delta[job] = dl;
  iters[job] += 1;
  if (!fixed && dl < delta0) conv[job] = 1;
}

__global__ __launch_bounds__(256) void finalize_kernel(const double* __restrict__ lnW, int nblocks,
                                                       const float* __restrict__ msgs, int M,
                                                       const int32_t* __restrict__ pairs, int npairs,
                                                       const uint8_t* __restrict__ labels, int d,
                                                       const double* __restrict__ delta_ws,
                                                       const int32_t* __restrict__ iters_ws, double delta1,
                                                       int rule, double* __restrict__ loglik,
                                                       double* __restrict__ delta_out,
                                                       int32_t* __restrict__ iters_out, uint8_t* __restrict__ coset,
                                                       uint8_t* __restrict__ correction) {
  const int64_t b = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  __shared__ double part[4][4];
  __shared__ int badp[4][4];
  __shared__ int chosen;
  // wave k handles coset k
  {
    const int k = wid;
    const int64_t job = b * 4 + k;
    double acc = 0.0;
    int bad = 0;
    for (int blk = lane; blk < nblocks; blk += 64) {
      const double w = lnW[job * nblocks + blk];
      if (isnan(w)) bad = 1; else acc += w;
    }
    const float* mb = msgs + job * M * MSTRIDE;
    for (int q = 0; q < npairs; ++q) {
      const float* u = mb + pairs[2 * q] * MSTRIDE;
      const float* v = mb + pairs[2 * q + 1] * MSTRIDE;
      const double o = wave_sum_d((double)u[lane] * (double)v[lane]);
      if (o > 0.0) acc -= (lane == 0) ? log(o) : 0.0;
      else bad = 1;
    }
    acc = wave_sum_d(acc);
    for (int o = 32; o > 0; o >>= 1) bad |= __shfl_down(bad, o);
    bad = __shfl(bad, 0);
    if (lane == 0) {
      part[0][k] = acc;
      badp[0][k] = bad;
    }
  }
  __syncthreads();
  if (tid == 0) {
    double ll[4], dl[4];
    for (int k = 0; k < 4; ++k) {
      const int64_t job = b * 4 + k;
      ll[k] = badp[0][k] ? NAN : part[0][k];
      dl[k] = badp[0][k] ? INFINITY : delta_ws[job];
      loglik[job] = ll[k];
      delta_out[job] = dl[k];
      iters_out[job] = iters_ws[job];
    }
    int best = 0;
    if (rule == 1) {
      double bv = -INFINITY;
      best = 0;
      for (int k = 0; k < 4; ++k) if (!isnan(ll[k]) && ll[k] > bv) { bv = ll[k]; best = k; }
    } else {
      int any = 0;
      double bv = -INFINITY;
      for (int k = 0; k < 4; ++k)
        if (dl[k] < delta1) {
          const double v = isnan(ll[k]) ? -INFINITY : ll[k];
          if (!any || v > bv) { bv = v; best = k; }
          any = 1;
        }
      if (!any) {
        double dm = INFINITY;
        best = 0;
        for (int k = 0; k < 4; ++k) if (dl[k] < dm) { dm = dl[k]; best = k; }
      }
    }
    coset[b] = (uint8_t)best;
    chosen = best;
  }
  __syncthreads();
  const int L = 2 * d - 1, n = d * d + (d - 1) * (d - 1);
  const uint8_t* lab = labels + (b * 4 + chosen) * L * L;
  for (int site = tid; site < L * L; site += blockDim.x) {
    const int r = site / L, c = site % L;
    if ((r + c) & 1) continue;
    // qubit index: row-major over (r+c) even; rows alternate d and d-1 qubits
    const int q = (r / 2) * (2 * d - 1) + ((r & 1) ? d + (c - 1) / 2 : c / 2);
    const uint8_t lb = lab[site];
    correction[b * n + q] = (uint8_t)((lb & 1) + 2 * ((lb >> 1) & 1));
  }
}

// --------------------------------------------------------------------------------------------------
struct DevPlan {
  bbp::Plan plan;
  bbp::ColumnDesc* cols = nullptr;
  SweepDesc* round[2] = {nullptr, nullptr};
  SweepDesc* bethe = nullptr;
  int32_t* edge_len = nullptr;
  int32_t* pairs = nullptr;
  int device = -1;
};

std::mutex g_mu;
std::map<std::tuple<int, int, int, int, int>, std::unique_ptr<DevPlan>> g_plans;

int validate(int32_t d, const bbp_opts* o) {
  if (!o) return fail(BBP_EINVAL, "opts is NULL");
  if (d < 2 || d > 32) return fail(BBP_EINVAL, "d must be in [2, 32]");
  if (o->block_rows < 1 || o->block_cols < 1) return fail(BBP_EINVAL, "block sizes must be >= 1");
  if (o->chi < 1) return fail(BBP_EINVAL, "chi must be >= 1");
  if (o->max_iter < 1) return fail(BBP_EINVAL, "max_iter must be >= 1");
  if (!(o->delta0 <= o->delta1)) return fail(BBP_EINVAL, "delta0 must not exceed delta1");
  if (!(o->damping >= 0.0 && o->damping < 1.0)) return fail(BBP_EINVAL, "damping must be in [0, 1)");
  if (o->rule != 0 && o->rule != 1) return fail(BBP_EINVAL, "rule must be 0 or 1");
  if (o->precision != 0) return fail(BBP_EUNSUPPORTED, "only precision 0 (FP32) is implemented");
  return BBP_OK;
}

const bbp::Plan& host_plan(int d, const bbp_opts* o) {
  static std::map<std::tuple<int, int, int, int>, bbp::Plan> cache;
  static std::mutex mu;
  std::lock_guard<std::mutex> lk(mu);
  auto key = std::make_tuple(d, o->block_rows, o->block_cols, o->chi);
  auto it = cache.find(key);
  if (it == cache.end()) it = cache.emplace(key, bbp::make_plan(d, o->block_rows, o->block_cols, o->chi)).first;
  return it->second;
}

int device_plan(int d, const bbp_opts* o, DevPlan** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  auto key = std::make_tuple(d, o->block_rows, o->block_cols, o->chi, dev);
  auto it = g_plans.find(key);
  if (it != g_plans.end()) { *out = it->second.get(); return BBP_OK; }
  auto dp = std::make_unique<DevPlan>();
  dp->plan = host_plan(d, o);
  dp->device = dev;
  const bbp::Plan& p = dp->plan;
  for (int c = 0; c < 2; ++c) {
    HIP_TRY(hipMalloc(&dp->round[c], sizeof(SweepDesc) * std::max<size_t>(1, p.round[c].size())));
    if (!p.round[c].empty())
      HIP_TRY(hipMemcpy(dp->round[c], p.round[c].data(), sizeof(SweepDesc) * p.round[c].size(), hipMemcpyHostToDevice));
  }
  HIP_TRY(hipMalloc(&dp->cols, sizeof(bbp::ColumnDesc) * p.columns.size()));
  HIP_TRY(hipMemcpy(dp->cols, p.columns.data(), sizeof(bbp::ColumnDesc) * p.columns.size(), hipMemcpyHostToDevice));
  HIP_TRY(hipMalloc(&dp->bethe, sizeof(SweepDesc) * p.bethe.size()));
  HIP_TRY(hipMemcpy(dp->bethe, p.bethe.data(), sizeof(SweepDesc) * p.bethe.size(), hipMemcpyHostToDevice));
  std::vector<int32_t> el(p.edge_len.begin(), p.edge_len.end());
  if (el.empty()) el.push_back(0);
  HIP_TRY(hipMalloc(&dp->edge_len, sizeof(int32_t) * el.size()));
  HIP_TRY(hipMemcpy(dp->edge_len, el.data(), sizeof(int32_t) * el.size(), hipMemcpyHostToDevice));
  std::vector<int32_t> pr(p.pair_ids.begin(), p.pair_ids.end());
  if (pr.empty()) pr.push_back(0);
  HIP_TRY(hipMalloc(&dp->pairs, sizeof(int32_t) * pr.size()));
  HIP_TRY(hipMemcpy(dp->pairs, pr.data(), sizeof(int32_t) * pr.size(), hipMemcpyHostToDevice));
  *out = dp.get();
  g_plans.emplace(key, std::move(dp));
  return BBP_OK;
}

struct Layout {
  size_t labels, msgs, terms, lnw, conv, iters, delta, total;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

Layout layout(const bbp::Plan& p, int64_t batch) {
  const size_t jobs = (size_t)batch * 4;
  Layout l;
  size_t off = 0;
  l.labels = off; off = align256(off + jobs * p.L * p.L);
  l.msgs = off; off = align256(off + jobs * std::max(p.M, 1) * MSTRIDE * sizeof(float));
  l.terms = off; off = align256(off + jobs * std::max(p.M, 1) * sizeof(double));
  l.lnw = off; off = align256(off + jobs * p.nblocks * sizeof(double));
  l.conv = off; off = align256(off + jobs * sizeof(int32_t));
  l.iters = off; off = align256(off + jobs * sizeof(int32_t));
  l.delta = off; off = align256(off + jobs * sizeof(double));
  l.total = off;
  return l;
}

struct Bbp_net_impl {
  int d;
  double p;
  std::vector<uint8_t> syndrome;
  std::vector<uint8_t> labels;   // [4][L*L]
};

}  // namespace

struct bbp_net {
  Bbp_net_impl impl;
};

extern "C" {

void bbp_default_opts(bbp_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->block_rows = 6;
  o->block_cols = 6;
  o->chi = 16;
  o->max_iter = 20;
  o->delta0 = 1e-4;
  o->delta1 = 1e-2;
  o->damping = 0.1;
  o->rule = 0;
  o->fixed_iters = 0;
  o->precision = 0;
}

const char* bbp_last_error(void) { return g_err.c_str(); }

int bbp_build_network(int32_t d, double p, const uint8_t* syndrome, int64_t m, bbp_net** out) {
  if (!out) return fail(BBP_EINVAL, "out is NULL");
  *out = nullptr;
  if (d < 2 || d > 32) return fail(BBP_EINVAL, "d must be in [2, 32]");
  if (m != 2LL * d * (d - 1)) return fail(BBP_EINVAL, "syndrome length must be 2d(d-1)");
  if (!(p > 0.0 && p < 1.0)) return fail(BBP_EINVAL, "p must be in (0, 1)");
  if (!syndrome) return fail(BBP_EINVAL, "syndrome is NULL");
  for (int64_t i = 0; i < m; ++i)
    if (syndrome[i] > 1) return fail(BBP_EINVAL, "syndrome bytes must be 0 or 1");
  bbp_net* net = new (std::nothrow) bbp_net;
  if (!net) return fail(BBP_ENOMEM, "out of host memory");
  const int L = 2 * d - 1, nz = d * (d - 1);
  net->impl.d = d;
  net->impl.p = p;
  net->impl.syndrome.assign(syndrome, syndrome + m);
  net->impl.labels.assign((size_t)4 * L * L, 0);
  for (int r = 0; r < L; ++r)
    for (int c = 0; c < L; ++c) {
      int x = 0, z = 0;
      if ((r & 1) == 0 && (c & 1) == 0) {
        for (int cc = c + 1; cc < L; cc += 2) x ^= syndrome[(r / 2) * (d - 1) + (cc - 1) / 2];
        for (int rr = r + 1; rr < L; rr += 2) z ^= syndrome[nz + ((rr - 1) / 2) * d + c / 2];
      }
      const int lx = (r == 0 && (c & 1) == 0), lz = (c == 0 && (r & 1) == 0);
      const int bx[4] = {0, 1, 1, 0}, bz[4] = {0, 0, 1, 1};
      for (int k = 0; k < 4; ++k)
        net->impl.labels[(size_t)k * L * L + r * L + c] = (uint8_t)((x ^ (bx[k] & lx)) | ((z ^ (bz[k] & lz)) << 1));
    }
  *out = net;
  return BBP_OK;
}

int bbp_net_dims(const bbp_net* net, int32_t* d, int32_t* n, int32_t* m) {
  if (!net) return fail(BBP_EINVAL, "net is NULL");
  const int dd = net->impl.d;
  if (d) *d = dd;
  if (n) *n = dd * dd + (dd - 1) * (dd - 1);
  if (m) *m = 2 * dd * (dd - 1);
  return BBP_OK;
}

int bbp_net_labels(const bbp_net* net, uint8_t* labels) {
  if (!net || !labels) return fail(BBP_EINVAL, "NULL argument");
  std::memcpy(labels, net->impl.labels.data(), net->impl.labels.size());
  return BBP_OK;
}

void bbp_free_network(bbp_net* net) { delete net; }

int bbp_plan_query(int32_t d, const bbp_opts* opts, bbp_plan_info* info) {
  if (opts && opts->precision != 0) { /* precision does not change the plan */ }
  if (!opts) return fail(BBP_EINVAL, "opts is NULL");
  if (!info) return fail(BBP_EINVAL, "info is NULL");
  if (d < 2 || d > 32 || opts->block_rows < 1 || opts->block_cols < 1 || opts->chi < 1)
    return fail(BBP_EINVAL, "invalid d or options");
  const bbp::Plan& p = host_plan(d, opts);
  info->L = p.L;
  info->n = d * d + (d - 1) * (d - 1);
  info->m = 2 * d * (d - 1);
  info->block_grid_rows = p.nI;
  info->block_grid_cols = p.nJ;
  info->num_messages = p.M;
  info->updates_per_iter = p.M;
  info->exact_sweeps = p.exact ? 1 : 0;
  info->max_boundary_rank = p.max_rank;
  info->gpu_supported = p.gpu_ok ? 1 : 0;
  info->flops_per_iter = p.flops_iter;
  info->flops_bethe = p.flops_bethe;
  if (!p.gpu_ok) g_err = p.why;
  return BBP_OK;
}

int bbp_workspace_size(int32_t d, int64_t batch, const bbp_opts* opts, size_t* bytes) {
  const int rc = validate(d, opts);
  if (rc) return rc;
  if (!bytes) return fail(BBP_EINVAL, "bytes is NULL");
  if (batch < 0) return fail(BBP_EINVAL, "batch must be >= 0");
  *bytes = layout(host_plan(d, opts), batch).total;
  return BBP_OK;
}

int bbp_decode_device(int32_t d, double p, const uint8_t* syndromes_dev, int64_t batch, const bbp_opts* opts,
                      void* workspace, size_t workspace_bytes, double* loglik_dev, double* delta_dev,
                      int32_t* iters_dev, uint8_t* coset_dev, uint8_t* correction_dev, float* messages_dev,
                      void* stream, bbp_timing* timing) {
  int rc = validate(d, opts);
  if (rc) return rc;
  if (!(p > 0.0 && p < 1.0)) return fail(BBP_EINVAL, "p must be in (0, 1)");
  if (batch < 0) return fail(BBP_EINVAL, "batch must be >= 0");
  if (batch == 0) return BBP_OK;
  if (batch > (int64_t)1 << 24) return fail(BBP_EINVAL, "batch too large");
  if (!syndromes_dev || !workspace || !loglik_dev || !delta_dev || !iters_dev || !coset_dev || !correction_dev)
    return fail(BBP_EINVAL, "a required pointer is NULL");
  DevPlan* dp = nullptr;
  rc = device_plan(d, opts, &dp);
  if (rc) return rc;
  const bbp::Plan& P = dp->plan;
  if (!P.gpu_ok) return fail(BBP_EUNSUPPORTED, P.why);
  const Layout lay = layout(P, batch);
  if (workspace_bytes < lay.total) return fail(BBP_EINVAL, "workspace too small");
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)workspace;
  uint8_t* labels = (uint8_t*)(ws + lay.labels);
  float* msgs = (float*)(ws + lay.msgs);
  double* terms = (double*)(ws + lay.terms);
  double* lnw = (double*)(ws + lay.lnw);
  int32_t* conv = (int32_t*)(ws + lay.conv);
  int32_t* iters = (int32_t*)(ws + lay.iters);
  double* delta = (double*)(ws + lay.delta);
  const int64_t jobs = batch * 4;
  const float eps = (float)p;
  const float pi0 = 1.0f - eps, pe = eps / 3.0f;

  std::vector<hipEvent_t> evs;
  auto mark = [&]() -> int {
    if (!timing) return BBP_OK;
    hipEvent_t e;
    HIP_TRY(hipEventCreate(&e));
    HIP_TRY(hipEventRecord(e, st));
    evs.push_back(e);
    return BBP_OK;
  };
  std::vector<int> kinds;   // kind of the interval ending at each mark: 0 other, 1 update, 2 bethe
  std::vector<double> iv_flops;

  if ((rc = mark())) return rc;
  labels_kernel<<<dim3((unsigned)batch), dim3(256), 0, st>>>(syndromes_dev, d, batch, labels);
  init_kernel<<<dim3((unsigned)jobs), dim3(256), 0, st>>>(msgs, dp->edge_len, P.M, jobs, conv, iters);
  HIP_TRY(hipGetLastError());
  if ((rc = mark())) return rc;
  kinds.push_back(0);
  iv_flops.push_back(0.0);
  for (int it = 0; it < opts->max_iter; ++it) {
    for (int c = 0; c < 2; ++c) {
      if (P.round[c].empty()) continue;
      update_kernel<<<dim3((unsigned)jobs, (unsigned)P.round[c].size()), dim3(NT), 0, st>>>(
          dp->round[c], dp->cols, d, labels, msgs, P.M, terms, conv, pi0, pe, pe, pe, (float)opts->damping, 0, lnw,
          P.nblocks);
      HIP_TRY(hipGetLastError());
      if ((rc = mark())) return rc;
      kinds.push_back(1);
      double f = 0.0;
      for (auto& s : P.round[c]) f += s.flops;
      iv_flops.push_back(f);
    }
    delta_kernel<<<dim3((unsigned)((jobs + 255) / 256)), dim3(256), 0, st>>>(terms, P.M, jobs, conv, iters, delta,
                                                                            opts->delta0, opts->fixed_iters);
    HIP_TRY(hipGetLastError());
    if ((rc = mark())) return rc;
    kinds.push_back(0);
    iv_flops.push_back(0.0);
  }
  update_kernel<<<dim3((unsigned)jobs, (unsigned)P.bethe.size()), dim3(NT), 0, st>>>(
      dp->bethe, dp->cols, d, labels, msgs, P.M, terms, conv, pi0, pe, pe, pe, (float)opts->damping, 1, lnw, P.nblocks);
  HIP_TRY(hipGetLastError());
  if ((rc = mark())) return rc;
  kinds.push_back(2);
  iv_flops.push_back(0.0);
  finalize_kernel<<<dim3((unsigned)batch), dim3(256), 0, st>>>(
      lnw, P.nblocks, msgs, P.M, dp->pairs, (int)(P.pair_ids.size() / 2), labels, d, delta, iters, opts->delta1,
      opts->rule, loglik_dev, delta_dev, iters_dev, coset_dev, correction_dev);
  HIP_TRY(hipGetLastError());
  if (messages_dev)
    HIP_TRY(hipMemcpyAsync(messages_dev, msgs, (size_t)jobs * P.M * MSTRIDE * sizeof(float),
                           hipMemcpyDeviceToDevice, st));
  if ((rc = mark())) return rc;
  kinds.push_back(0);
  iv_flops.push_back(0.0);

  if (timing) {
    HIP_TRY(hipStreamSynchronize(st));
    std::memset(timing, 0, sizeof(*timing));
    // flops actually executed: per-job active iterations
    std::vector<int32_t> it_host((size_t)jobs);
    HIP_TRY(hipMemcpy(it_host.data(), iters, sizeof(int32_t) * jobs, hipMemcpyDeviceToHost));
    double job_iters = 0.0;
    for (auto v : it_host) job_iters += v;
    for (size_t k = 1; k < evs.size(); ++k) {
      float ms = 0.0f;
      HIP_TRY(hipEventElapsedTime(&ms, evs[k - 1], evs[k]));
      const int kind = kinds[k - 1];
      if (kind == 1) { timing->update_ms += ms; timing->update_launches += 1; }
      else if (kind == 2) timing->bethe_ms += ms;
      else timing->other_ms += ms;
    }
    timing->update_flops = job_iters * P.flops_iter;
    for (auto e : evs) (void)hipEventDestroy(e);
  }
  return BBP_OK;
}

int bbp_blockbp_decode(bbp_net* const* nets, int64_t batch, const bbp_opts* opts, double* loglik, double* delta,
                       int32_t* iters, uint8_t* coset, uint8_t* correction) {
  if (batch <= 0) return batch == 0 ? BBP_OK : fail(BBP_EINVAL, "batch must be >= 0");
  if (!nets || !nets[0]) return fail(BBP_EINVAL, "nets is NULL");
  if (!loglik || !delta || !iters || !coset || !correction) return fail(BBP_EINVAL, "a required pointer is NULL");
  const int d = nets[0]->impl.d;
  const double p = nets[0]->impl.p;
  for (int64_t i = 0; i < batch; ++i)
    if (!nets[i] || nets[i]->impl.d != d || nets[i]->impl.p != p)
      return fail(BBP_EINVAL, "all networks of one call must share d and p");
  const int m = 2 * d * (d - 1), n = d * d + (d - 1) * (d - 1);
  size_t wsb = 0;
  int rc = bbp_workspace_size(d, batch, opts, &wsb);
  if (rc) return rc;
  std::vector<uint8_t> syn((size_t)batch * m);
  for (int64_t i = 0; i < batch; ++i) std::memcpy(&syn[(size_t)i * m], nets[i]->impl.syndrome.data(), m);
  void *ws = nullptr, *dsyn = nullptr, *dout = nullptr;
  const size_t outb = (size_t)batch * (4 * 8 + 4 * 8 + 4 * 4 + 1 + n);
  auto cleanup = [&]() { if (ws) (void)hipFree(ws); if (dsyn) (void)hipFree(dsyn); if (dout) (void)hipFree(dout); };
  if (hipMalloc(&ws, wsb) != hipSuccess || hipMalloc(&dsyn, syn.size()) != hipSuccess ||
      hipMalloc(&dout, outb) != hipSuccess) {
    cleanup();
    return fail(BBP_ENOMEM, "device allocation failed");
  }
  char* o = (char*)dout;
  double* dl = (double*)o;
  double* dd = dl + batch * 4;
  int32_t* di = (int32_t*)(dd + batch * 4);
  uint8_t* dc = (uint8_t*)(di + batch * 4);
  uint8_t* dcorr = dc + batch;
  if (hipMemcpy(dsyn, syn.data(), syn.size(), hipMemcpyHostToDevice) != hipSuccess) {
    cleanup();
    return fail(BBP_EHIP, "copy of syndromes failed");
  }
  rc = bbp_decode_device(d, p, (const uint8_t*)dsyn, batch, opts, ws, wsb, dl, dd, di, dc, dcorr, nullptr, nullptr,
                         nullptr);
  if (rc == BBP_OK) {
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(loglik, dl, batch * 4 * 8, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(delta, dd, batch * 4 * 8, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(iters, di, batch * 4 * 4, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(coset, dc, batch, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(correction, dcorr, (size_t)batch * n, hipMemcpyDeviceToHost) != hipSuccess)
      rc = fail(BBP_EHIP, "decode or copy back failed");
  }
  cleanup();
  return rc;
}

int bbp_reference_update_host(int32_t d, double p, const bbp_opts* opts, const uint8_t* labels, int32_t msg_id,
                              const double* msgs, double* out, double* logscale) {
  if (!opts || !labels || !msgs || !out || !logscale) return fail(BBP_EINVAL, "NULL argument");
  if (d < 2 || d > 32 || opts->block_rows < 1 || opts->block_cols < 1 || opts->chi < 1)
    return fail(BBP_EINVAL, "invalid d or options");
  const bbp::Plan& P = host_plan(d, opts);
  const SweepDesc* found = nullptr;
  if (msg_id >= 0) {
    for (int c = 0; c < 2; ++c)
      for (auto& s : P.round[c]) if (s.msg_out == msg_id) found = &s;
  } else if (-1 - msg_id < (int)P.bethe.size()) {
    found = &P.bethe[-1 - msg_id];
  }
  if (!found) return fail(BBP_EINVAL, "unknown message or block id");
  const float eps = (float)p;
  const float pi[4] = {1.0f - eps, eps / 3.0f, eps / 3.0f, eps / 3.0f};
  return bbp::host_sweep(P, *found, labels, pi, msgs, out, logscale);
}

}  // extern "C"
