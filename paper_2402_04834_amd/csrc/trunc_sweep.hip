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
// Keeping the chi largest values at every bond is the textbook QR + truncated-SVD compression: the part left
// of a bond is an isometry when it is truncated, so each cut keeps the chi largest Schmidt values of the
// current state. Where a bond carries at most chi values the SVD keeps them all (the state is unchanged).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>

#include "geom.hpp"
#include "sweep_launch.hpp"

namespace bbp {
namespace {

constexpr int KM = TRUNC_KMAX;
constexpr int TS = 16 * 2 * 16;   // one compressed site [a][h][b] (a, b < 16), or one cap operator [P][v][Q]
constexpr int TQ = 32 * 64 + 32;  // one pass-1 factor: reflection vectors [j][row] (rows 2l + h, l < 32), betas
// workspace slot of one item, in doubles
constexpr int W_A = 0;                      // sites 0 .. kp+1
constexpr int W_Q = W_A + (KM + 2) * TS;    // pass-1 factors of sites 0 .. kp; site kp+1 keeps its matrix M
constexpr int W_CT = W_Q + (KM + 2) * TQ;   // cap operators: top t = 0 .. kt-1, then bottom
constexpr int W_SLOT = W_CT + 2 * KM * TS;

// LDS pool in doubles (the phases never overlap)
constexpr int XS = 17;                                        // Jacobi exchange row stride (LDS banks)
constexpr int P1 = 32 * 32 + 2 * 64 + 32 + 3 * TS;            // R carry, vector buffers, betas, site, CT, Bb
constexpr int P2 = 64 * XS + 32 * 16 + 32;                    // exchange (then V), carry C, singular values
constexpr int PC = 256 + 32 * 32 + 32;                        // chain: matrix, vectors, betas
constexpr int PE = 4 * 256;                                   // end: left / right chains (ping-pong)
constexpr int POOL = std::max(std::max(P1, P2), std::max(PC, PE));

// Jacobi: rotate while |<c_p, c_q>| > JAC |c_p| |c_q|; a row of norm at most RANKTOL |N|_F is rounding noise
constexpr double JAC = 1e-13, RANKTOL = 1e-13;
constexpr int SWEEPS = 16;

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ __forceinline__ double wmax(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

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

// Householder QR of the 64 x 32 matrix held as x[k] = M[2k + par][hi] by lane (hi, par), reflections j < jmax.
// On return x holds R above the diagonal and reflection vector j (pivot entry v_j) from the diagonal down in
// lanes hi = j, rd the diagonal entry of R of the lane's column, Hb[j] the coefficients.
__device__ __forceinline__ void qr64(double (&x)[32], double& rd, int jmax, double* vb, double* Hb) {
  const int ln = threadIdx.x, hi = ln >> 1, par = ln & 1;
  rd = 0.0;
  for (int j = 0; j < jmax; ++j) {
    double* v = vb + (j & 1) * 64;
    if (hi == j) {
#pragma unroll
      for (int k = 0; k < 32; ++k) v[2 * k + par] = (2 * k + par >= j) ? x[k] : 0.0;
    }
    __syncthreads();
    double hv[32], pn = 0.0, pw = 0.0, xp = 0.0;
#pragma unroll
    for (int k = 0; k < 32; ++k) {
      hv[k] = v[2 * k + par];
      pn += hv[k] * hv[k];
      pw += hv[k] * x[k];
      xp += (2 * k + par == j) ? x[k] : 0.0;
    }
    const double nrm = sqrt(pn + __shfl_xor(pn, 1));
    const double alpha = v[j];
    double beta = 0.0, vj = alpha, diag = alpha;
    if (nrm > 0.0) {
      const double sg = (alpha >= 0.0) ? 1.0 : -1.0;
      vj = alpha + sg * nrm;
      beta = 1.0 / (nrm * (nrm + fabs(alpha)));
      diag = -sg * nrm;
    }
    pw += (vj - alpha) * xp;   // the pivot entry of the vector is v_j, not alpha
    const double w = (pw + __shfl_xor(pw, 1)) * beta;
    if (hi > j) {
#pragma unroll
      for (int k = 0; k < 32; ++k) x[k] -= w * ((2 * k + par == j) ? vj : hv[k]);
    } else if (hi == j) {
      rd = diag;
#pragma unroll
      for (int k = 0; k < 32; ++k)
        if (2 * k + par == j) x[k] = vj;
    }
    if (ln == 0) Hb[j] = beta;
  }
  __syncthreads();
}

// The reflection vectors left in x by qr64 (rows >= j of column j, zero above) and their coefficients into a
// pass-1 factor slot: Vg[j * 64 + row], Vg[2048 + j].
__device__ __forceinline__ void store_v(const double (&x)[32], int jmax, const double* Hb, double* Vg) {
  const int ln = threadIdx.x, hi = ln >> 1, par = ln & 1;
  if (hi < jmax) {
#pragma unroll
    for (int k = 0; k < 32; ++k) {
      const int row = 2 * k + par;
      Vg[hi * 64 + row] = (row >= hi) ? x[k] : 0.0;
    }
  }
  if (ln < jmax) Vg[2048 + ln] = Hb[ln];
}

// X = Q C for the carry C (Csh [m][k], m < 32, k < 16) and the factor stored by store_v, Q = H_0 ... H_{jmax-1}
// on the first 32 unit columns: X = H_0 (H_1 (... [C; 0])). Lane (kc, qt) = (ln & 15, ln >> 4) holds rows
// 16 qt + r of column kc in X[r]; a reflection is a 16-term partial product, two cross-quarter additions and
// a 16-term update. The vectors are read once, from the slot pass 1 wrote.
__device__ __forceinline__ void apply_q(double (&X)[16], int jmax, const double* Vg, const double* Csh) {
  const int ln = threadIdx.x, kc = ln & 15, qt = ln >> 4;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = qt * 16 + r;
    X[r] = (row < 32) ? Csh[row * 16 + kc] : 0.0;
  }
  for (int j = jmax - 1; j >= 0; --j) {
    const double* v = Vg + j * 64 + qt * 16;
    double p = 0.0;
#pragma unroll
    for (int r = 0; r < 16; ++r) p += v[r] * X[r];
    p += __shfl_xor(p, 16);
    p += __shfl_xor(p, 32);
    const double w = p * Vg[2048 + j];
#pragma unroll
    for (int r = 0; r < 16; ++r) X[r] -= w * v[r];
  }
}

// The carry R (rows 0..31 of the factored matrix) into Rsh [row][col], unit Frobenius norm; returns ln |R|_F.
__device__ __forceinline__ double store_r(const double (&x)[32], double rd, double* Rsh) {
  const int ln = threadIdx.x, hi = ln >> 1, par = ln & 1;
  double f = 0.0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int row = 2 * k + par;
    const double r = row < hi ? x[k] : (row == hi ? rd : 0.0);
    f += r * r;
  }
  const double fro = sqrt(wsum(f));
  const double inv = (fro > 0.0) ? 1.0 / fro : 0.0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int row = 2 * k + par;
    Rsh[row * 32 + hi] = (row < hi ? x[k] : (row == hi ? rd : 0.0)) * inv;
  }
  __syncthreads();
  return log(fro);
}

// One-sided Jacobi SVD of the 32 x 32 matrix N held as y[k] = N[l][(par, k)] by lane (l = hi, par), the chi
// largest singular values kept. Writes the kept right singular vectors (rows j < 16 of V, zero beyond chi) as
// site [j][par][k] (or, bottom cap, [j][k] from the par = 0 half) and the carry C = N V / |.|_F into Csh
// [l][j]; returns the log of that norm.
__device__ __forceinline__ double svd_step(double (&y)[16], int chi, double* Xsh, double* Csh, double* sig,
                                           double* site, bool bottom) {
  const int ln = threadIdx.x, hi = ln >> 1, par = ln & 1;
  double y0[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) y0[k] = y[k];
  double nf2 = 0.0;
#pragma unroll
  for (int k = 0; k < 16; ++k) nf2 += y[k] * y[k];
  const double thr2 = wsum(nf2) * (RANKTOL * RANKTOL);
  for (int sw = 0; sw < SWEEPS; ++sw) {
    int rotated = 0;
    double c2max = 0.0;
    double own = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) own += y[k] * y[k];
    own += __shfl_xor(own, 1);
    for (int rd = 0; rd < 31; ++rd) {
      const int pl = (hi == 31) ? rd : (hi == rd) ? 31 : (2 * rd - hi + 62) % 31;
#pragma unroll
      for (int k = 0; k < 16; ++k) Xsh[ln * XS + k] = y[k];
      Xsh[ln * XS + 16] = own;
      __syncthreads();
      double z[16], gg = 0.0;
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        z[k] = Xsh[(2 * pl + par) * XS + k];
        gg += y[k] * z[k];
      }
      const double other = Xsh[(2 * pl + par) * XS + 16];
      __syncthreads();
      gg += __shfl_xor(gg, 1);
      const bool lower = hi < pl;
      const double al = lower ? own : other, be = lower ? other : own;
      const double c2 = (al > thr2 && be > thr2) ? gg * gg / (al * be) : 0.0;
      c2max = c2 > c2max ? c2 : c2max;
      if (c2 > JAC * JAC) {
        // tan(theta) of the rotation that orthogonalises the pair (the smaller root), then cos and sin
        const double zeta = (be - al) / (2.0 * gg), az = fabs(zeta);
        const double tt = copysign(1.0 / (az + (az < 1e150 ? sqrt(zeta * zeta + 1.0) : az)), zeta);
        const double cs = 1.0 / sqrt(tt * tt + 1.0), sn = cs * tt;
#pragma unroll
        for (int k = 0; k < 16; ++k) y[k] = lower ? (cs * y[k] - sn * z[k]) : (sn * z[k] + cs * y[k]);
        const double cc = cs * cs;
        own = lower ? cc * (al - 2.0 * tt * gg + tt * tt * be) : cc * (be + 2.0 * tt * gg + tt * tt * al);
        rotated = 1;
      }
    }
    if (!__any(rotated) || wmax(c2max) < 1e-16) break;
  }
  double s2 = 0.0;
#pragma unroll
  for (int k = 0; k < 16; ++k) s2 += y[k] * y[k];
  const double s2r = s2 + __shfl_xor(s2, 1);
  const double sv = (s2r > thr2) ? sqrt(s2r) : 0.0;
  const double key = (sv == sv) ? sv : -1.0;
  if (par == 0) sig[hi] = key;
  __syncthreads();
  int rank = 0;
  for (int i = 0; i < 32; ++i) {
    const double o = sig[i];
    rank += (o > key || (o == key && i < hi)) ? 1 : 0;
  }
  const bool kept = rank < chi && sv > 0.0;
  const double inv = kept ? 1.0 / sv : 0.0;
  double* Vsh = Xsh;   // the exchange buffer is free now
  if (rank < 16) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      if (bottom) {
        if (par == 0) site[rank * 16 + k] = y[k] * inv;
      } else {
        site[(rank * 2 + par) * 16 + k] = y[k] * inv;
      }
      Vsh[rank * 32 + par * 16 + k] = y[k] * inv;
    }
  }
  const double fro = sqrt(wsum((par == 0 && kept) ? sv * sv : 0.0));
  __syncthreads();
  const double finv = (fro > 0.0) ? 1.0 / fro : 0.0;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) acc += y0[k] * Vsh[j * 32 + par * 16 + k];
    acc += __shfl_xor(acc, 1);
    if ((j >> 3) == par) Csh[hi * 16 + j] = acc * finv;
  }
  __syncthreads();
  return log(fro);
}

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
    double* Bb = CTs + TS;
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
    qr64(x, rd, 16, vb, Hb);
    logs += store_r(x, rd, Rsh);
    store_v(x, 16, Hb, Q);
    // crossing sites
    for (int i = 1; i <= kp; ++i) {
      for (int e = ln; e < TS; e += 64) Ash[e] = A[i * TS + e];
      __syncthreads();
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
      qr64(x, rd, 32, vb, Hb);
      logs += store_r(x, rd, Rsh);
      store_v(x, 32, Hb, Q + i * TQ);
    }
    // bottom cap: Bb[(d, v)][q'] = sum_P S[d][P] CT[P][v][q'], then M[l][q'] = sum R[l][(d, v)] Bb[(d, v)][q']
    for (int e = ln; e < 256; e += 64) Ash[e] = A[(kp + 1) * TS + e];
    if (bot)
      for (int e = ln; e < TS; e += 64) CTs[e] = CT[(KM + t) * TS + e];
    __syncthreads();
    for (int e = ln; e < 512; e += 64) {
      const int dv = e >> 4, q = e & 15, d = dv >> 1, v = dv & 1;
      double acc = 0.0;
      if (bot) {
        for (int P = 0; P < 16; ++P) acc += Ash[d * 16 + P] * CTs[P * 32 + v * 16 + q];
      } else if (v == 0 && q == 0) {
        acc = Ash[d * 16];
      }
      Bb[e] = acc;
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
      double y[16];
      if (i == kp + 1) {
        const double* Mg = Q + (kp + 1) * TQ;
#pragma unroll
        for (int k = 0; k < 16; ++k) y[k] = par == 0 ? Mg[hi * 16 + k] : 0.0;
      } else {
        // N = Q_i C, then from the column layout to rows: lane (l, t) takes N[l][(t, k)] = X[2l + t][k]
        double X[16];
        apply_q(X, 32, Q + i * TQ, Csh);
#pragma unroll
        for (int r = 0; r < 16; ++r) Xsh[((ln >> 4) * 16 + r) * XS + (ln & 15)] = X[r];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 16; ++k) y[k] = Xsh[ln * XS + k];
      }
      __syncthreads();   // the exchange buffer and Csh are rewritten by the step
      logs += svd_step(y, chi, Xsh, Csh, sig, A + i * TS, i == kp + 1);
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

hipError_t launch_trunc_sweeps(hipStream_t st, const SweepArgs& a) {
  if (a.items <= 0) return hipSuccess;
  if (!a.tws || a.tws_slots <= 0) return hipErrorInvalidValue;
  SweepArgs b = a;
  for (int64_t base = 0; base < a.items; base += a.tws_slots) {
    b.item_base = base;
    const int64_t n = std::min<int64_t>(a.tws_slots, a.items - base);
    trunc_sweep_kernel<<<dim3((unsigned)n), dim3(64), 0, st>>>(b);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace bbp
