// wave_mps.hpp -- one-wavefront FP64 building blocks of the boundary-MPS compression (Sec. III.A, III.D): the
// QR sweep's Householder factorisation of a site and the truncating sweep's SVD of a bond, shared by the
// truncating block sweeps (trunc_sweep.hip) and the single-block boundary-MPS decoder (bmps.hip).
//
// Shapes (bond dimensions padded to 2 chi_max = 32, chi <= 16):
//   factor   the 64 x 32 matrix M of a site after absorbing a column, rows 2l + h (left bond l, leg h), held
//            as x[k] = M[2k + par][hi] by lane (hi, par); M = Q R by Householder reflections j < jmax whose
//            vectors are broadcast through LDS from the lanes that own them (no memory round trip while
//            factoring) and then stored once in compact form with their coefficients (a factor slot);
//   carry    R (32 x 32, unit Frobenius norm) down the QR sweep, C (32 x 16, unit norm) up the SVD sweep;
//   bond     N = Q C as a 32 x 32 (left bond) x (leg, right bond) matrix, formed by applying the stored
//            reflections to [C; 0] (Q itself is never formed), then one-sided Jacobi on its rows: the chi
//            largest singular values are kept, their right singular vectors become the site and N V (unit
//            norm) the carry to the site above.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

namespace bbp {
namespace wmps {

constexpr int XS = 17;                                        // Jacobi exchange row stride (LDS banks)
constexpr int TQ = 32 * 64 + 32;  // one factor slot: reflection vectors [j][row] (rows 2l + h, l < 32), betas

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
    double hv[32], pn = 0.0;
#pragma unroll
    for (int k = 0; k < 32; ++k) {
      hv[k] = v[2 * k + par];
      pn += hv[k] * hv[k];
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
    // the pivot entry of the vector is v_j, not alpha: one select per entry, then plain products
    double pw = 0.0;
#pragma unroll
    for (int k = 0; k < 32; ++k) {
      hv[k] = (2 * k + par == j) ? vj : hv[k];
      pw += hv[k] * x[k];
    }
    const double w = (pw + __shfl_xor(pw, 1)) * beta;
    if (hi > j) {
#pragma unroll
      for (int k = 0; k < 32; ++k) x[k] -= w * hv[k];
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

// qr64 with the reflections unrolled (JMAX = jmax): reflection j touches rows >= j only, i.e. registers
// k >= j / 2, and its pivot row is a compile-time register, so the vector's rows above the pivot are neither
// stored, read nor multiplied, and the pivot takes one select instead of one per register. KR: only rows
// below 2 KR can be nonzero (x[k] = 0 for k >= KR, left untouched), as in a cap's 16-row matrix; the
// rolled form with 64 rows kept x in scratch memory there. (An unrolled instance with 16 reflections over
// all 32 registers beside the 32-reflection one took the compiler beyond 40 minutes.)
template <int JMAX, int KR = 32>
__device__ __forceinline__ void qr64u(double (&x)[32], double& rd, double* vb, double* Hb) {
  static_assert(KR <= 32 && JMAX <= 2 * KR, "reflections within the nonzero rows");
  const int ln = threadIdx.x, hi = ln >> 1, par = ln & 1;
  rd = 0.0;
#pragma unroll
  for (int j = 0; j < JMAX; ++j) {
    const int k0 = j >> 1, jp = j & 1;   // pivot row j = 2 k0 + jp
    double* v = vb + (j & 1) * 64;
    if (hi == j) {
#pragma unroll
      for (int k = k0; k < KR; ++k) v[2 * k + par] = x[k];
    }
    __syncthreads();
    double hv[32], pn = 0.0;
#pragma unroll
    for (int k = k0; k < KR; ++k) {
      hv[k] = v[2 * k + par];
      if (k == k0 && jp == 1) hv[k] = par ? hv[k] : 0.0;   // row 2 k0 < j is not part of the vector
      pn += hv[k] * hv[k];
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
    // the pivot entry of the vector is v_j, not alpha
    hv[k0] = (par == jp) ? vj : hv[k0];
    double pw = 0.0;
#pragma unroll
    for (int k = k0; k < KR; ++k) pw += hv[k] * x[k];
    const double w = (pw + __shfl_xor(pw, 1)) * beta;
    if (hi > j) {
#pragma unroll
      for (int k = k0; k < KR; ++k) x[k] -= w * hv[k];
    } else if (hi == j) {
      rd = diag;
      if (par == jp) x[k0] = vj;
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
  // the next reflection's vector quarter and coefficient are loaded while this one is applied (the loads
  // come from the workspace, through L2: one reflection's latency each, otherwise)
  double vn[16], bn = 0.0;
  if (jmax > 0) {
#pragma unroll
    for (int r = 0; r < 16; ++r) vn[r] = Vg[(jmax - 1) * 64 + qt * 16 + r];
    bn = Vg[2048 + jmax - 1];
  }
  for (int j = jmax - 1; j >= 0; --j) {
    double v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = vn[r];
    const double beta = bn;
    if (j > 0) {
#pragma unroll
      for (int r = 0; r < 16; ++r) vn[r] = Vg[(j - 1) * 64 + qt * 16 + r];
      bn = Vg[2048 + j - 1];
    }
    double p = 0.0;
#pragma unroll
    for (int r = 0; r < 16; ++r) p += v[r] * X[r];
    p += __shfl_xor(p, 16);
    p += __shfl_xor(p, 32);
    const double w = p * beta;
#pragma unroll
    for (int r = 0; r < 16; ++r) X[r] -= w * v[r];
  }
}

// From apply_q's column layout to the row layout of svd_step: y[k] = X[ln][k] (N[l][(t, k)] for ln = 2l + t).
__device__ __forceinline__ void cols_to_rows(const double (&X)[16], double* Xsh, double (&y)[16]) {
  const int ln = threadIdx.x;
#pragma unroll
  for (int r = 0; r < 16; ++r) Xsh[((ln >> 4) * 16 + r) * XS + (ln & 15)] = X[r];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 16; ++k) y[k] = Xsh[ln * XS + k];
  __syncthreads();
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
    // round rd pairs rows hi and pl: 31 and rd, the others (2 rd - hi) mod 31, stepped by 2 each round
    int cyc = (62 - hi) % 31;
    for (int rd = 0; rd < 31; ++rd, cyc = (cyc + 2 >= 31) ? cyc + 2 - 31 : cyc + 2) {
      const int pl = (hi == 31) ? rd : (hi == rd) ? 31 : cyc;
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
      // squared cosine of the pair (approximate reciprocal: it only decides whether to rotate)
      const double c2 = (al > thr2 && be > thr2) ? gg * gg * __builtin_amdgcn_rcp(al * be) : 0.0;
      c2max = c2 > c2max ? c2 : c2max;
      if (c2 > JAC * JAC) {
        // The angle only has to bring the pair closer to orthogonal, so t = tan(theta) (the smaller root) is
        // formed in FP32 (the hardware's approximate reciprocal and square root, one instruction each; above the
        // noise threshold zeta stays within 1e30);
        // cos and sin are then formed in FP64 from that t, so that the rotation is orthogonal to FP64
        // rounding.
        const float zf = (float)(be - al) * __builtin_amdgcn_rcpf(2.0f * (float)gg), azf = fabsf(zf);
        const float denf = azf + (azf < 1e18f ? __builtin_amdgcn_sqrtf(fmaf(zf, zf, 1.0f)) : azf);
        const double tt = (double)copysignf(__builtin_amdgcn_rcpf(denf), zf);
        const double xx = tt * tt + 1.0;
        double cs = __builtin_amdgcn_rsq(xx);
        cs = cs * (1.5 - 0.5 * xx * cs * cs);
        cs = cs * (1.5 - 0.5 * xx * cs * cs);
        const double sn = cs * tt;
        // lower row p: c p - s q; higher row q: c q + s p -- one multiply and one fused multiply-add each
        const double sz = lower ? -sn : sn;
#pragma unroll
        for (int k = 0; k < 16; ++k) y[k] = fma(sz, z[k], cs * y[k]);
        const double cc = cs * cs;
        own = lower ? cc * (al - 2.0 * tt * gg + tt * tt * be) : cc * (be + 2.0 * tt * gg + tt * tt * al);
        rotated = 1;
      }
    }
    // a sweep whose pairs all started within cos 1e-6 of orthogonal leaves them within about 1e-12
    // (quadratic convergence): far below the FP32 messages the singular vectors end up in
    if (!__any(rotated) || wmax(c2max) < 1e-12) break;
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

}  // namespace wmps
}  // namespace bbp
