// trunc_sweep.hip -- block sweeps with a binding chi (Sec. III.D, Fig. 3): the boundary MPS of the in-block
// sweep compressed back to chi after every column by a Householder QR sweep and a truncated one-sided Jacobi
// SVD sweep, in FP64. The dense kernels (sweep_kernel.hip) serve every sweep whose boundary state provably
// stays within chi (the plan's rank analysis); this kernel serves the others, and every sweep of a plan whose
// blocks are wider than 6 (their state does not fit a wavefront's registers).
//
// One wavefront runs one (job, sweep):
//   caps     every side message enters with the part still to be absorbed an isometry: the left-canonical
//            chain (successive Householder QR) of the message -- of its leg-reversed form when the sweep walks
//            it from its first site -- is consumed from its weighted end. Cap operator t is CT_t[P][v][Q]
//            (old cap bond P, emitted vertical bond v, new cap bond Q), bonds min(2^j, 2^(K-j)) <= 16.
//   state    the boundary MPS: top cap site [q][d], the kp crossing sites [a][h][b], bottom cap site [d][q],
//            bonds padded to 16 (chi <= 16), to 32 once a column is absorbed.
//   column   pass 1, top to bottom: each site absorbs its column tensor (the caps their cap operator), is
//            multiplied by the carry R of the site above and factored M = Q R by Householder reflections whose
//            vectors stay in the wavefront while it factors (the owning lanes' registers, broadcast through
//            LDS); the vectors (Q in compact form) go to the item's workspace slot, R (unit Frobenius norm, the
//            norm into the log-scale) down to the next site. The bottom cap keeps M. Pass 2, bottom to top:
//            N = Q C (the reflections applied to the carry C from below; Q is never formed) as a (left bond) x
//            (leg, right bond) matrix, one-sided Jacobi SVD, the chi largest singular values kept: their right
//            singular vectors are the new site, N V (unit norm) the carry; the top cap takes Q C.
//   end      the chain contracted to the dense 2^kp message; normalisation (remark 3), damping (remark 7) and
//            distance term (remark 4) as in the dense kernels, or the closing overlap of Lemma 3.1.
//   narrow   with every bond within 8 (trunc_shape.hpp) the factorisations, reflections and SVDs run on the
//            blocks that can be nonzero, in layouts that keep all 64 lanes busy (trunc_sweep_kernel<true>).
// Keeping the chi largest values at every bond is the textbook QR + truncated-SVD compression: the part left
// of a bond is an isometry when it is truncated, so each cut keeps the chi largest Schmidt values of the
// current state. Where a bond carries at most chi values the SVD keeps them all (the state is unchanged).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>

#include "geom.hpp"
#include "sweep_launch.hpp"
#include "trunc_shape.hpp"
#include "wave_mps.hpp"

namespace bbp {
namespace {

using namespace wmps;

constexpr int KM = TRUNC_KMAX;
constexpr int TS = 16 * 2 * 16;   // one compressed site [a][h][b] (a, b < 16), or one cap operator [P][v][Q]
// workspace slot of one item, in doubles
constexpr int W_A = 0;                      // sites 0 .. kp+1
constexpr int W_Q = W_A + (KM + 2) * TS;    // pass-1 factors of sites 0 .. kp; site kp+1 keeps its matrix M
constexpr int W_CT = W_Q + (KM + 2) * TQ;   // cap operators: top t = 0 .. kt-1, then bottom
constexpr int W_SLOT = W_CT + 2 * KM * TS;

// LDS pool in doubles (the phases never overlap)
constexpr int P1 = 32 * 32 + 2 * 64 + 32 + 2 * TS;            // R carry, vector buffers, betas, site, CT (or Bb)
constexpr int P2 = 64 * XS + 32 * 16 + 32;                    // exchange (then V), carry C, singular values
constexpr int PC = 256 + 32 * 32 + 32;                        // chain: matrix, vectors, betas
constexpr int PE = 4 * 256;                                   // end: left / right chains (ping-pong)
constexpr int POOL = std::max(std::max(P1, P2), std::max(PC, PE));

__device__ __forceinline__ int bitrev(int w, int K) { return (int)(__brev((unsigned)w) >> (32 - K)); }

// Entry e = up*8 + in*4 + down*2 + out of the frame table at sweep step t, position i, in FP64: checks are
// COPY tensors (0 / 1), qubits one of the four Pauli probabilities pq (by code x + 2z).
__device__ __forceinline__ double tab(const SweepDesc& s, int L, const uint8_t* lab, const double* pq, int t, int i,
                                      int e) {
  int r, c;
  frame_site(s.frame, s.r0, s.c0, s.kr, s.kc, t, i, r, c);
  const float m = site_entry(s.frame, L, r, c, lab[r * L + c], 1.0f, 2.0f, 3.0f, 4.0f, e);
  if ((r + c) & 1) return (double)m;
  const int k = (int)m;
  return k == 0 ? 0.0 : pq[k - 1];
}

// Left-canonical chain of the K-leg vector in W[0 .. 2^K) (leg 0 most significant; W is overwritten): site
// j = A_j[a][v][q] with natural bonds. transposed: written as the cap operator CT_{K-1-j}[q][v][a] (the chain
// absorbed from its weighted end); else as site j itself, [a][v][q]. out must be zero beyond the bonds.
__device__ __forceinline__ void chain(double* W, double* Hv, double* Hb, int K, double* out, bool transposed) {
  const int ln = threadIdx.x;
  int b = 1;
  for (int j = 0; j < K - 1; ++j) {
    const int m = 2 * b, n = 1 << (K - j - 1), k = std::min(m, n);
    // Householder QR of W as an m x n row-major matrix
    for (int c = 0; c < k; ++c) {
      const double xr = (ln < m && ln >= c) ? W[ln * n + c] : 0.0;
      const double alpha = W[c * n + c];
      const double nrm = sqrt(wsum(xr * xr));
      double beta = 0.0, vj = alpha, diag = alpha;
      if (nrm > 0.0) {
        const double sg = (alpha >= 0.0) ? 1.0 : -1.0;
        vj = alpha + sg * nrm;
        beta = 1.0 / (nrm * (nrm + fabs(alpha)));
        diag = -sg * nrm;
      }
      if (ln < 32) Hv[c * 32 + ln] = (ln == c) ? vj : ((ln > c && ln < m) ? xr : 0.0);
      if (ln == 0) Hb[c] = beta;
      __syncthreads();
      for (int col = c + 1 + ln; col < n; col += 64) {
        double w = 0.0;
        for (int r = c; r < m; ++r) w += Hv[c * 32 + r] * W[r * n + col];
        w *= beta;
        for (int r = c; r < m; ++r) W[r * n + col] -= w * Hv[c * 32 + r];
      }
      __syncthreads();
      if (ln == 0) W[c * n + c] = diag;
      if (ln > c && ln < m) W[ln * n + c] = 0.0;
      __syncthreads();
    }
    // Q (m x k): lane q forms column q by applying the reflections to the unit vector e_q
    if (ln < k) {
      double qv[32];
#pragma unroll
      for (int r = 0; r < 32; ++r) qv[r] = (r == ln) ? 1.0 : 0.0;
      for (int c = k - 1; c >= 0; --c) {
        double w = 0.0;
#pragma unroll
        for (int r = 0; r < 32; ++r) w += (r >= c && r < m) ? Hv[c * 32 + r] * qv[r] : 0.0;
        w *= Hb[c];
#pragma unroll
        for (int r = 0; r < 32; ++r)
          if (r >= c && r < m) qv[r] -= w * Hv[c * 32 + r];
      }
#pragma unroll
      for (int r = 0; r < 32; ++r) {
        if (r >= m) break;
        const int a = r >> 1, v = r & 1;
        if (transposed) out[(K - 1 - j) * TS + ln * 32 + v * 16 + a] = qv[r];
        else out[j * TS + a * 32 + v * 16 + ln] = qv[r];
      }
    }
    __syncthreads();   // W now holds R (k x n): rows 0 .. k-1, the next step's (2k) x (n/2) matrix
    b = k;
  }
  // last site: A_{K-1}[a][v][0] = rest[a][v]
  for (int e = ln; e < 2 * b; e += 64) {
    const int a = e >> 1, v = e & 1;
    if (transposed) out[0 * TS + v * 16 + a] = W[e];
    else out[(K - 1) * TS + a * 32 + v * 16] = W[e];
  }
  __syncthreads();
}

// A crossing site's factorisation in the narrow form: M (rows (k, h) < 32 with R row k < 16, columns (b, dn)
// < 16) held as x[k] = M[4 k + q][c] by lane (c, q) = (ln >> 2, ln & 3), k < 8 -- the block of the padded
// 64 x 32 site matrix that can be nonzero, spread so that every lane holds 8 of its rows (the 64 x 32 layout
// of qr64u would leave half the lanes on zero columns). Householder QR with 16 reflections
// (vectors broadcast through LDS as in qr64u, sums over a column's four lanes by two exchanges), then R (unit
// Frobenius norm, zero in the columns >= 16) into Rsh [row][col] and the vectors and coefficients into the
// factor slot in store_v's format (rows < 32). Returns ln |R|_F.
__device__ __forceinline__ double factor_narrow(double (&x)[8], double* vb, double* Hb, double* Rsh, double* Vg) {
  const int ln = threadIdx.x, c = ln >> 2, q = ln & 3;
  double rd = 0.0;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int kj = j >> 2, qj = j & 3;   // pivot row j = 4 kj + qj
    double* v = vb + (j & 1) * 64;
    if (c == j) {
#pragma unroll
      for (int k = kj; k < 8; ++k) v[4 * k + q] = x[k];
    }
    __syncthreads();
    double hv[8], pn = 0.0;
#pragma unroll
    for (int k = kj; k < 8; ++k) {
      hv[k] = v[4 * k + q];
      if (k == kj) hv[k] = q < qj ? 0.0 : hv[k];   // rows above the pivot are not part of the vector
      pn += hv[k] * hv[k];
    }
    pn += __shfl_xor(pn, 1);
    pn += __shfl_xor(pn, 2);
    const double nrm = sqrt(pn);
    const double alpha = v[j];
    double beta = 0.0, vj = alpha, diag = alpha;
    if (nrm > 0.0) {
      const double sg = (alpha >= 0.0) ? 1.0 : -1.0;
      vj = alpha + sg * nrm;
      beta = 1.0 / (nrm * (nrm + fabs(alpha)));
      diag = -sg * nrm;
    }
    hv[kj] = (q == qj) ? vj : hv[kj];   // the pivot entry of the vector is v_j, not alpha
    double pw = 0.0;
#pragma unroll
    for (int k = kj; k < 8; ++k) pw += hv[k] * x[k];
    pw += __shfl_xor(pw, 1);
    pw += __shfl_xor(pw, 2);
    const double w = pw * beta;
    if (c > j) {
#pragma unroll
      for (int k = kj; k < 8; ++k) x[k] -= w * hv[k];
    } else if (c == j) {
      rd = diag;
      if (q == qj) x[kj] = vj;
    }
    if (ln == 0) Hb[j] = beta;
  }
  __syncthreads();
  double f = 0.0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int row = 4 * k + q;
    const double r = row < c ? x[k] : (row == c ? rd : 0.0);
    f += r * r;
  }
  const double fro = sqrt(wsum(f));
  const double inv = (fro > 0.0) ? 1.0 / fro : 0.0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int row = 4 * k + q;
    Rsh[row * 32 + c] = (row < c ? x[k] : (row == c ? rd : 0.0)) * inv;
    Rsh[row * 32 + 16 + c] = 0.0;
    Vg[c * 64 + row] = (row >= c) ? x[k] : 0.0;
  }
  if (ln < 16) Vg[2048 + ln] = Hb[ln];
  __syncthreads();
  return log(fro);
}

// apply_q and cols_to_rows (wave_mps.hpp) in the narrow form: X = Q C with 16 reflections for the rows < 32
// and the columns k < 8 that can be nonzero. Lane (kc, g) = (ln & 7, ln >> 3) holds rows 4 g + r (r < 4) of
// column kc; a reflection is a 4-term partial product, a sum over the eight row groups (three exchanges) and
// a 4-term update, with the next reflection's entries loaded meanwhile. Then, in svd_narrow's layout, lane
// (l, u) takes y[e] = X[2 l + u / 2][4 (u % 2) + e].
__device__ __forceinline__ void apply_q_narrow(const double* Vg, const double* Csh, double* Xsh, double (&y)[4]) {
  const int ln = threadIdx.x, kc = ln & 7, g = ln >> 3;
  double X[4], vn[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    X[r] = Csh[(4 * g + r) * 16 + kc];
    vn[r] = Vg[15 * 64 + 4 * g + r];
  }
  double bn = Vg[2048 + 15];
  for (int j = 15; j >= 0; --j) {
    double v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = vn[r];
    const double beta = bn;
    if (j > 0) {
#pragma unroll
      for (int r = 0; r < 4; ++r) vn[r] = Vg[(j - 1) * 64 + 4 * g + r];
      bn = Vg[2048 + j - 1];
    }
    double p = 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) p += v[r] * X[r];
    p += __shfl_xor(p, 8);
    p += __shfl_xor(p, 16);
    p += __shfl_xor(p, 32);
    const double w = p * beta;
#pragma unroll
    for (int r = 0; r < 4; ++r) X[r] -= w * v[r];
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) Xsh[(4 * g + r) * XS + kc] = X[r];
  __syncthreads();
  const int l = ln >> 2, u = ln & 3;
#pragma unroll
  for (int e = 0; e < 4; ++e) y[e] = Xsh[(2 * l + (u >> 1)) * XS + 4 * (u & 1) + e];
  __syncthreads();
}

// svd_step (wave_mps.hpp) in the narrow form: N has at most 16 nonzero rows, each with 2 x 8 nonzero entries
// (t, k), held as y[e] = N[l][(t, k)] with t = u / 2, k = 4 (u % 2) + e by lane (l, u) = (ln >> 2, ln & 3).
// The same one-sided Jacobi rotations, stopping test and outputs (kept right singular vectors as site rows,
// zero beyond chi and beyond k = 8; the carry C = N V / |.|_F into Csh [l][j], rows 16..31 cleared); the
// round-robin pairs 16 rows (15 rounds per sweep), and a round exchanges 4 entries and a norm per lane and
// sums a pair's product over the row's four lanes by two exchanges.
__device__ __forceinline__ double svd_narrow(double (&y)[4], int chi, double* Xsh, double* Csh, double* sig,
                                             double* site, bool bottom) {
  constexpr int XN = 5;   // exchange row stride: 4 entries and the row norm
  const int ln = threadIdx.x, l = ln >> 2, u = ln & 3, t = u >> 1, k0 = 4 * (u & 1);
  double y0[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) y0[e] = y[e];
  double nf2 = 0.0;
#pragma unroll
  for (int e = 0; e < 4; ++e) nf2 += y[e] * y[e];
  const double thr2 = wsum(nf2) * (RANKTOL * RANKTOL);
  auto rowsum = [](double v) {
    v += __shfl_xor(v, 1);
    return v + __shfl_xor(v, 2);
  };
  for (int sw = 0; sw < SWEEPS; ++sw) {
    int rotated = 0;
    double c2max = 0.0;
    double own = 0.0;
#pragma unroll
    for (int e = 0; e < 4; ++e) own += y[e] * y[e];
    own = rowsum(own);
    // round rd pairs rows l and pl: 15 and rd, the others (2 rd - l) mod 15, stepped by 2 each round
    int cyc = (30 - l) % 15;
    for (int rd = 0; rd < 15; ++rd, cyc = (cyc + 2 >= 15) ? cyc + 2 - 15 : cyc + 2) {
      const int pl = (l == 15) ? rd : (l == rd) ? 15 : cyc;
#pragma unroll
      for (int e = 0; e < 4; ++e) Xsh[ln * XN + e] = y[e];
      Xsh[ln * XN + 4] = own;
      __syncthreads();
      double z[4], gg = 0.0;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        z[e] = Xsh[(4 * pl + u) * XN + e];
        gg += y[e] * z[e];
      }
      const double other = Xsh[(4 * pl + u) * XN + 4];
      __syncthreads();
      gg = rowsum(gg);
      const bool lower = l < pl;
      const double al = lower ? own : other, be = lower ? other : own;
      const double c2 = (al > thr2 && be > thr2) ? gg * gg * __builtin_amdgcn_rcp(al * be) : 0.0;
      c2max = c2 > c2max ? c2 : c2max;
      if (c2 > JAC * JAC) {
        // the angle as in svd_step: tan in FP32, cos and sin in FP64 from it
        const float zf = (float)(be - al) * __builtin_amdgcn_rcpf(2.0f * (float)gg), azf = fabsf(zf);
        const float denf = azf + (azf < 1e18f ? __builtin_amdgcn_sqrtf(fmaf(zf, zf, 1.0f)) : azf);
        const double tt = (double)copysignf(__builtin_amdgcn_rcpf(denf), zf);
        const double xx = tt * tt + 1.0;
        double cs = __builtin_amdgcn_rsq(xx);
        cs = cs * (1.5 - 0.5 * xx * cs * cs);
        cs = cs * (1.5 - 0.5 * xx * cs * cs);
        const double sn = cs * tt;
        const double sz = lower ? -sn : sn;
#pragma unroll
        for (int e = 0; e < 4; ++e) y[e] = fma(sz, z[e], cs * y[e]);
        const double cc = cs * cs;
        own = lower ? cc * (al - 2.0 * tt * gg + tt * tt * be) : cc * (be + 2.0 * tt * gg + tt * tt * al);
        rotated = 1;
      }
    }
    if (!__any(rotated) || wmax(c2max) < 1e-12) break;
  }
  double s2 = 0.0;
#pragma unroll
  for (int e = 0; e < 4; ++e) s2 += y[e] * y[e];
  const double s2r = rowsum(s2);
  const double sv = (s2r > thr2) ? sqrt(s2r) : 0.0;
  const double key = (sv == sv) ? sv : -1.0;
  if (u == 0) sig[l] = key;
  __syncthreads();
  int rank = 0;
  for (int i = 0; i < 16; ++i) {
    const double o = sig[i];
    rank += (o > key || (o == key && i < l)) ? 1 : 0;
  }
  const bool kept = rank < chi && sv > 0.0;
  const double inv = kept ? 1.0 / sv : 0.0;
  double* Vsh = Xsh;   // the exchange buffer is free now
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    if (bottom) {
      if (t == 0) {
        site[rank * 16 + k0 + e] = y[e] * inv;
        site[rank * 16 + 8 + k0 + e] = 0.0;
      }
    } else {
      site[(rank * 2 + t) * 16 + k0 + e] = y[e] * inv;
      site[(rank * 2 + t) * 16 + 8 + k0 + e] = 0.0;
    }
    Vsh[rank * 32 + t * 16 + k0 + e] = y[e] * inv;
  }
  const double fro = sqrt(wsum((u == 0 && kept) ? sv * sv : 0.0));
  __syncthreads();
  const double finv = (fro > 0.0) ? 1.0 / fro : 0.0;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    double acc = 0.0;
#pragma unroll
    for (int e = 0; e < 4; ++e) acc += y0[e] * Vsh[j * 32 + t * 16 + k0 + e];
    acc = rowsum(acc);
    if ((j >> 2) == u) Csh[l * 16 + j] = acc * finv;
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) Csh[(16 + l) * 16 + 4 * u + e] = 0.0;
  __syncthreads();
  return log(fro);
}

// NARROW: the sweeps of the narrow form (trunc_shape.hpp), factored and decomposed at half size; each form has
// its own instantiation so that neither pays the other's registers.
template <bool NARROW>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void trunc_sweep_kernel(SweepArgs a) {
  const int ln = threadIdx.x, hi = ln >> 1, par = ln & 1;
  const int64_t item = a.item_base + (int64_t)blockIdx.x;
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
    const double* tj = G.terms + job * G.M;
    const double ti = s.msg_init >= 0 ? tj[s.msg_init] : 0.0, tt = s.msg_top >= 0 ? tj[s.msg_top] : 0.0,
                 tb = s.msg_bot >= 0 ? tj[s.msg_bot] : 0.0;
    if (tj[s.msg_out] < a.gate && ti < a.gate && tt < a.gate && tb < a.gate) {
      if (ln == 0) G.terms[job * G.M + s.msg_out] = 0.0;
      return;
    }
  }
  const int L = 2 * G.d - 1, kt = s.kt, kp = s.kp, chi = G.chi, ms = G.mstride;
  const uint8_t* lab = G.labels + job * (int64_t)L * L;
  double pq[4];
  if (G.pdev) {
    const double pj = G.pdev[job >> 2];
    pq[0] = 1.0 - pj;
    pq[1] = pq[2] = pq[3] = pj / 3.0;
  } else {
    for (int k = 0; k < 4; ++k) pq[k] = G.pq[k];
  }
  const float* mbase = G.msgs + job * G.M * (int64_t)ms;
  double* ws = a.tws + (int64_t)blockIdx.x * W_SLOT;
  double* A = ws + W_A;
  double* Q = ws + W_Q;
  double* CT = ws + W_CT;

  __shared__ double pool[POOL];
  const bool top = s.msg_top >= 0, bot = s.msg_bot >= 0, fwd = (s.frame == FRAME_E || s.frame == FRAME_S);

  // ---- caps and the initial state ----
  // the chains fill the natural bonds only: clear the padded operators and sites they are read as
  if (top)
    for (int e = ln; e < kt * TS; e += 64) CT[e] = 0.0;
  if (bot)
    for (int e = ln; e < kt * TS; e += 64) CT[KM * TS + e] = 0.0;
  for (int e = ln; e < (kp + 2) * TS; e += 64) A[e] = 0.0;
  __syncthreads();
  {
    double* W = pool;
    double* Hv = pool + 256;
    double* Hb = Hv + 32 * 32;
    for (int side = 0; side < 2; ++side) {
      const int id = side == 0 ? s.msg_top : s.msg_bot;
      if (id < 0) continue;
      for (int w = ln; w < (1 << kt); w += 64) W[w] = (double)mbase[id * (int64_t)ms + (fwd ? bitrev(w, kt) : w)];
      __syncthreads();
      chain(W, Hv, Hb, kt, CT + side * KM * TS, true);
    }
    if (s.msg_init >= 0) {
      for (int w = ln; w < (1 << kp); w += 64) W[w] = (double)mbase[s.msg_init * (int64_t)ms + w];
      __syncthreads();
      chain(W, Hv, Hb, kp, A + TS, false);
    } else {
      for (int i = 1; i <= kp; ++i)
        if (ln == 0) A[i * TS] = 1.0;   // every in-leg at its only value 0
    }
    if (ln == 0) {
      A[0] = 1.0;                  // top cap [q = 0][d = 0]
      A[(kp + 1) * TS] = 1.0;      // bottom cap [d = 0][q = 0]
    }
  }
  __syncthreads();

  double logs = 0.0;
  for (int t = 0; t < kt; ++t) {
    // ---------------- pass 1: absorb and factor, top to bottom ----------------
    double* Rsh = pool;
    double* vb = Rsh + 32 * 32;
    double* Hb = vb + 2 * 64;
    double* Ash = Hb + 32;
    double* CTs = Ash + TS;
    double* Bb = CTs;   // the bottom cap's product replaces the cap operator it is formed from
    double x[32], rd;
    // top cap: M_0[q'][(d, v)] = sum_P S_0[P][d] CT[P][v][q'], rows q' < 16
    for (int e = ln; e < 256; e += 64) Ash[e] = A[e];
    if (top)
      for (int e = ln; e < TS; e += 64) CTs[e] = CT[t * TS + e];
    __syncthreads();
    {
      const int d = hi >> 1, v = hi & 1;
#pragma unroll
      for (int k = 0; k < 32; ++k) x[k] = 0.0;
      if (top) {
        for (int P = 0; P < 16; ++P) {
          const double sp = Ash[P * 16 + d];
#pragma unroll
          for (int k = 0; k < 8; ++k) x[k] += sp * CTs[P * 32 + v * 16 + 2 * k + par];
        }
      } else if (v == 0 && par == 0) {
        x[0] = Ash[d];
      }
    }
    qr64u<16, 8>(x, rd, vb, Hb);   // rows q' < 16: registers k < 8
    logs += store_r(x, rd, Rsh);
    store_v(x, 16, Hb, Q);
    // crossing sites: M [(k, h)][(b, dn)] = sum_(a, u) R[k][(a, u)] (A_i T)[(a, u)][(h, b, dn)], factored; in the
    // narrow form R has at most 16 rows and the site's bonds at most 8, so M is 32 x 16 (factor_narrow)
    for (int i = 1; i <= kp; ++i) {
      for (int e = ln; e < TS; e += 64) Ash[e] = A[i * TS + e];
      __syncthreads();
      if constexpr (NARROW) {
        // lane (c, q): column c = (b, dn), rows 4 k + q = (R row 2 k + q / 2, leg q % 2)
        const int c = ln >> 2, q = ln & 3, b = c >> 1, dn = c & 1, h = q & 1, k0 = q >> 1;
        const double t00 = tab(s, L, lab, pq, t, i - 1, 0 * 8 + 0 * 4 + dn * 2 + h);
        const double t01 = tab(s, L, lab, pq, t, i - 1, 0 * 8 + 1 * 4 + dn * 2 + h);
        const double t10 = tab(s, L, lab, pq, t, i - 1, 1 * 8 + 0 * 4 + dn * 2 + h);
        const double t11 = tab(s, L, lab, pq, t, i - 1, 1 * 8 + 1 * 4 + dn * 2 + h);
        double xn[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) xn[k] = 0.0;
        for (int aa = 0; aa < 8; ++aa) {
          const double a0 = Ash[(aa * 2 + 0) * 16 + b], a1 = Ash[(aa * 2 + 1) * 16 + b];
          const double b0 = a0 * t00 + a1 * t01, b1 = a0 * t10 + a1 * t11;
#pragma unroll
          for (int k = 0; k < 8; ++k)
            xn[k] += Rsh[(2 * k + k0) * 32 + aa * 2] * b0 + Rsh[(2 * k + k0) * 32 + aa * 2 + 1] * b1;
        }
        __syncthreads();   // every lane has read R
        logs += factor_narrow(xn, vb, Hb, Rsh, Q + i * TQ);
      } else {
        {
          const int b = hi >> 1, dn = hi & 1;
          const double t00 = tab(s, L, lab, pq, t, i - 1, 0 * 8 + 0 * 4 + dn * 2 + par);
          const double t01 = tab(s, L, lab, pq, t, i - 1, 0 * 8 + 1 * 4 + dn * 2 + par);
          const double t10 = tab(s, L, lab, pq, t, i - 1, 1 * 8 + 0 * 4 + dn * 2 + par);
          const double t11 = tab(s, L, lab, pq, t, i - 1, 1 * 8 + 1 * 4 + dn * 2 + par);
#pragma unroll
          for (int k = 0; k < 32; ++k) x[k] = 0.0;
          for (int aa = 0; aa < 16; ++aa) {
            const double a0 = Ash[(aa * 2 + 0) * 16 + b], a1 = Ash[(aa * 2 + 1) * 16 + b];
            const double b0 = a0 * t00 + a1 * t01, b1 = a0 * t10 + a1 * t11;
#pragma unroll
            for (int k = 0; k < 32; ++k) x[k] += Rsh[k * 32 + aa * 2] * b0 + Rsh[k * 32 + aa * 2 + 1] * b1;
          }
        }
        __syncthreads();   // every lane has read R
        qr64u<32>(x, rd, vb, Hb);
        logs += store_r(x, rd, Rsh);
        store_v(x, 32, Hb, Q + i * TQ);
      }
    }
    // bottom cap: Bb[(d, v)][q'] = sum_P S[d][P] CT[P][v][q'], then M[l][q'] = sum R[l][(d, v)] Bb[(d, v)][q']
    for (int e = ln; e < 256; e += 64) Ash[e] = A[(kp + 1) * TS + e];
    if (bot)
      for (int e = ln; e < TS; e += 64) CTs[e] = CT[(KM + t) * TS + e];
    __syncthreads();
    {
      double bv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = ln + 64 * u, dv = e >> 4, q = e & 15, d = dv >> 1, v = dv & 1;
        double acc = 0.0;
        if (bot) {
          for (int P = 0; P < 16; ++P) acc += Ash[d * 16 + P] * CTs[P * 32 + v * 16 + q];
        } else if (v == 0 && q == 0) {
          acc = Ash[d * 16];
        }
        bv[u] = acc;
      }
      __syncthreads();   // every lane has read the operator before Bb overwrites it
#pragma unroll
      for (int u = 0; u < 8; ++u) Bb[ln + 64 * u] = bv[u];
    }
    __syncthreads();
    {
      double* Mg = Q + (kp + 1) * TQ;
#pragma unroll 1
      for (int qq = 0; qq < 8; ++qq) {
        const int q = 8 * par + qq;
        double acc = 0.0;
#pragma unroll 8
        for (int dv = 0; dv < 32; ++dv) acc += Rsh[hi * 32 + dv] * Bb[dv * 16 + q];
        Mg[hi * 16 + q] = acc;
      }
    }
    __syncthreads();

    // ---------------- pass 2: truncating SVD sweep, bottom to top ----------------
    double* Xsh = pool;
    double* Csh = Xsh + 64 * XS;
    double* sig = Csh + 32 * 16;
    for (int i = kp + 1; i >= 1; --i) {
      const double* Mg = Q + (kp + 1) * TQ;   // the bottom cap's M [l][q']
      if constexpr (NARROW) {
        double y[4];
        if (i == kp + 1) {
          const int l = ln >> 2, u = ln & 3;
#pragma unroll
          for (int e = 0; e < 4; ++e) y[e] = (u < 2) ? Mg[l * 16 + 4 * u + e] : 0.0;
        } else {
          apply_q_narrow(Q + i * TQ, Csh, Xsh, y);   // N = Q_i C
        }
        logs += svd_narrow(y, chi, Xsh, Csh, sig, A + i * TS, i == kp + 1);
      } else {
        double y[16];
        if (i == kp + 1) {
#pragma unroll
          for (int k = 0; k < 16; ++k) y[k] = par == 0 ? Mg[hi * 16 + k] : 0.0;
        } else {
          // N = Q_i C, then from the column layout to rows: lane (l, t) takes N[l][(t, k)] = X[2l + t][k]
          double X[16];
          apply_q(X, 32, Q + i * TQ, Csh);
          cols_to_rows(X, Xsh, y);
        }
        logs += svd_step(y, chi, Xsh, Csh, sig, A + i * TS, i == kp + 1);
      }
    }
    // top cap: S_0[q'][j] = sum_m Q_0[q'][m] C[m][j], unit Frobenius norm
    {
      // rows q' < 16 of Q_0 C sit in the lanes of quarter 0: S_0[q'][kc] = X[q']
      double X[16];
      apply_q(X, 16, Q, Csh);
      double f = 0.0;
#pragma unroll
      for (int r = 0; r < 16; ++r) f += (ln < 16) ? X[r] * X[r] : 0.0;
      const double fro = sqrt(wsum(f));
      const double inv = (fro > 0.0) ? 1.0 / fro : 0.0;
      if (ln < 16) {
#pragma unroll
        for (int r = 0; r < 16; ++r) A[r * 16 + ln] = X[r] * inv;
      }
      logs += log(fro);
    }
    __syncthreads();
  }

  // ---------------- the dense message: left chain x right chain ----------------
  const int hl = kp / 2, hr = kp - hl;
  // left chain in pool[0 .. 512) and right chain in pool[512 .. 1024), each ping-ponging between halves
  for (int e = ln; e < 16; e += 64) {
    pool[e] = A[e];                              // top cap row q' = 0
    pool[512 + e] = A[(kp + 1) * TS + e * 16];   // bottom cap column q' = 0
  }
  __syncthreads();
  int lc = 0, rc = 0;
  for (int i = 1; i <= hl; ++i) {   // L_i[(pre, h)][b] = sum_a L_{i-1}[pre][a] S_i[a][h][b]
    const int n = (1 << i) * 16;
    for (int e = ln; e < n; e += 64) {
      const int b = e & 15, ph = e >> 4, pre = ph >> 1, h = ph & 1;
      double acc = 0.0;
      for (int aa = 0; aa < 16; ++aa) acc += pool[lc * 256 + pre * 16 + aa] * A[i * TS + aa * 32 + h * 16 + b];
      pool[(lc ^ 1) * 256 + e] = acc;
    }
    __syncthreads();
    lc ^= 1;
  }
  for (int i = kp; i > hl; --i) {   // R_i[(h, suf)][a] = sum_b S_i[a][h][b] R_{i+1}[suf][b]
    const int nsuf = 1 << (kp - i), n = 2 * nsuf * 16;
    for (int e = ln; e < n; e += 64) {
      const int aa = e & 15, hs = e >> 4, h = hs / nsuf, suf = hs - h * nsuf;
      double acc = 0.0;
      for (int b = 0; b < 16; ++b) acc += A[i * TS + aa * 32 + h * 16 + b] * pool[512 + rc * 256 + suf * 16 + b];
      pool[512 + (rc ^ 1) * 256 + e] = acc;
    }
    __syncthreads();
    rc ^= 1;
  }
  double out[4];
  const int H = 1 << kp;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int e = ln + 64 * r;
    double acc = 0.0;
    if (e < H) {
      const int hL = e >> hr, hR = e & ((1 << hr) - 1);
      for (int b = 0; b < 16; ++b) acc += pool[lc * 256 + hL * 16 + b] * pool[512 + rc * 256 + hR * 16 + b];
    }
    out[r] = acc;
  }

  if (a.mode == 1) {
    double w = 0.0;
    if (s.msg_close >= 0) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int e = ln + 64 * r;
        if (e < H) w += out[r] * (double)mbase[s.msg_close * (int64_t)ms + e];
      }
    } else if (ln == 0) {
      w = out[0];
    }
    w = wsum(w);
    if (ln == 0) G.lnW[job * G.nblocks + s.block] = (w > 0.0) ? logs + log(w) : NAN;
    return;
  }
  // normalised new message, damping against the old one (unit norm), distance term
  float* mo = G.msgs + (job * G.M + s.msg_out) * (int64_t)ms;
  double f2 = 0.0;
#pragma unroll
  for (int r = 0; r < 4; ++r) f2 += out[r] * out[r];
  const double inv = 1.0 / sqrt(wsum(f2));
  double old[4], dm[4], g2 = 0.0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int e = ln + 64 * r;
    old[r] = (e < H) ? (double)mo[e] : 0.0;
    dm[r] = (1.0 - (double)a.eta) * out[r] * inv + (double)a.eta * old[r];
    g2 += dm[r] * dm[r];
  }
  const double ginv = 1.0 / sqrt(wsum(g2));
  double dd = 0.0, ss = 0.0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const double fm = dm[r] * ginv;
    dd += (fm - old[r]) * (fm - old[r]);
    ss += (fm + old[r]) * (fm + old[r]);
    dm[r] = fm;
  }
  dd = wsum(dd);
  ss = wsum(ss);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int e = ln + 64 * r;
    if (e < H) mo[e] = (float)dm[r];
  }
  if (ln == 0) G.terms[job * G.M + s.msg_out] = 0.5 * dd * ss;
}

}  // namespace

size_t trunc_slot_bytes() { return (size_t)W_SLOT * sizeof(double); }

hipError_t launch_trunc_sweeps(hipStream_t st, const SweepArgs& a, bool narrow) {
  if (a.items <= 0) return hipSuccess;
  if (!a.tws || a.tws_slots <= 0) return hipErrorInvalidValue;
  SweepArgs b = a;
  for (int64_t base = 0; base < a.items; base += a.tws_slots) {
    b.item_base = base;
    const int64_t n = std::min<int64_t>(a.tws_slots, a.items - base);
    if (narrow)
      trunc_sweep_kernel<true><<<dim3((unsigned)n), dim3(64), 0, st>>>(b);
    else
      trunc_sweep_kernel<false><<<dim3((unsigned)n), dim3(64), 0, st>>>(b);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace bbp
