// bmps.hip -- boundary-MPS contraction of whole coset networks: the single-block limit of blockBP.
//
// Sec. III.A describes the bMPS decoder: the network is contracted column by column from left to right; the
// contraction up to column c is an MPS over the L rows whose physical legs are the right legs of column c;
// the next column, an MPO with vertical bonds of dimension 2, doubles its bonds, and the product is
// compressed back to bond dimension chi. Sec. III.D notes that blockBP with one block covering the network
// is this algorithm; Sec. IV uses it with chi = 16 as the accuracy reference.
//
// One wavefront contracts one coset network (job). The compression after every column but the last:
//   pass 1, top row to bottom row: M_r = R_{r-1} B_r with B_r = A_r (x) T_r the MPO-applied row, as a
//     (2 chi * 2) x 2 chi matrix (rows: left bond and physical leg; columns: right bond); Householder QR
//     M_r = Q_r R_r; Q_r goes to the workspace, R_r (unit Frobenius norm, the norm into the log-scale) is
//     carried into the next row. The last row keeps M_r itself.
//   pass 2, bottom row to top row: N_r = Q_r C_{r+1} as a 2 chi x (2 * chi) matrix (rows: left bond;
//     columns: physical leg and right bond); one-sided Jacobi SVD; the chi largest singular values are kept:
//     their right singular vectors are the new row A_r, and C_r = N_r V (unit Frobenius norm, the norm into
//     the log-scale) is carried into the row above.
// This is the textbook QR + truncated-SVD compression: the left part is an isometry at every cut of
// pass 2, so every truncation keeps the chi largest Schmidt values of the state. The last column has no
// right legs; its MPO is applied and the chain of matrices multiplied out, with a running log-scale:
// ln Z = log-scale + ln(value), NaN when the value is not positive.
//
// Precision: FP64 throughout. The estimate of a coset is resolved only down to about the unit roundoff
// times the state's norm, and the state's norm is set by the likeliest configurations of the partial
// network, not by the coset's own value. An FP32 build of this kernel was off by up to 4 nats on cosets
// 15-30 nats below the best and returned non-positive values within 8 nats of the best (d=5, chi 16), so
// every matrix is FP64; only rotation angles (below) are formed in FP32.
//
// Layout: every lane owns matrix columns in registers. Pass 1: lane (col, par) holds the 32 entries of
// column col of M_r in the rows of parity par; a Householder vector is broadcast through the row's workspace
// slot (L1-resident). Pass 2: lane (l, t) holds the 16 entries (t, k) of row l of N_r; a Jacobi round pairs
// rows by the circle method and exchanges them through LDS. Bond dimensions are padded to 2 chi_max = 32
// with zeros.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "bmps_launch.hpp"

namespace bbp {
namespace {

constexpr int SITE_A = 16 * 2 * 16;   // entries per compressed row: [j][t][k], j, k < chi_max
constexpr int SITE_Q = 64 * 32;       // entries per pass-1 factor: [(l, t)][k]

template <typename T> struct Tol;
// Jacobi: rotate while |<c_p, c_q>| > jac |c_p| |c_q|. A row whose norm is at most rank |N|_F is rounding
// noise: it takes part in no rotation (two exactly parallel rows would otherwise be rotated over and over,
// the smaller one only shrinking) and its singular value counts as zero.
template <> struct Tol<double> { static constexpr double jac = 1e-13, rank = 1e-13; static constexpr int sweeps = 16; };

__device__ __forceinline__ float msqrt(float v) { return sqrtf(v); }
__device__ __forceinline__ double msqrt(double v) { return sqrt(v); }
__device__ __forceinline__ float mabs(float v) { return fabsf(v); }
__device__ __forceinline__ double mabs(double v) { return fabs(v); }

template <typename T>
__device__ __forceinline__ T sel4(T a0, T a1, T a2, T a3, int e) {
  const T lo = (e & 1) ? a1 : a0, hi = (e & 1) ? a3 : a2;
  return (e & 2) ? hi : lo;
}

// entry T[u][s][dn][t] of the tensor at (r, c) (legs up, left, down, right); a leg that leaves the grid
// only takes the value 0. Checks are COPY tensors, qubits pi(label flipped by the adjacent checks).
template <typename T>
__device__ __forceinline__ T tentry(int r, int c, int L, int lb, int u, int s, int dn, int t, T p0, T p1, T p2,
                                    T p3) {
  if ((u && r == 0) || (s && c == 0) || (dn && r == L - 1) || (t && c == L - 1)) return T(0);
  if ((r + c) & 1) {
    // COPY over the present legs: all equal
    int v = -1, ok = 1;
    if (r > 0) { v = u; }
    if (c > 0) { ok &= (v < 0 || v == s); v = s; }
    if (r < L - 1) { ok &= (v < 0 || v == dn); v = dn; }
    if (c < L - 1) { ok &= (v < 0 || v == t); }
    return ok ? T(1) : T(0);
  }
  // horizontal edge (even r): checks above / below flip x, left / right flip z; vertical edge: swapped
  const int px = (r & 1) ? (s ^ t) : (u ^ dn), pz = (r & 1) ? (u ^ dn) : (s ^ t);
  return sel4(p0, p1, p2, p3, (lb ^ px ^ (pz << 1)) & 3);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return __shfl(v, 0);
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return __shfl(v, 0);
}

// LDS: pass 1 and pass 2 never overlap in time, so their buffers share one pool (13 KB in FP64, so that three
// wavefronts fit per SIMD; the register file then holds 168 VGPRs per lane and the rest of the working set
// spills to scratch, which measures faster than one resident wavefront per SIMD); the Householder vectors of
// pass 1 live in the row's workspace slot until Q replaces them
constexpr int POOL_P1 = 32 * 32 + 32 + SITE_A;              // R, Householder betas, row
constexpr int XSTRIDE = 17;                                 // exchange row stride: 16 entries + 1 (LDS banks)
constexpr int POOL_P2 = 64 * XSTRIDE + 32 * 16 + 32;   // exchange (then V), C, singular values
constexpr int POOL = POOL_P1 > POOL_P2 ? POOL_P1 : POOL_P2;

template <typename T>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3, 3))) void bmps_kernel(BmpsArgs a) {
  const int64_t job = blockIdx.x;
  const int ln = threadIdx.x, hi = ln >> 1, par = ln & 1;
  const int L = 2 * a.d - 1, chi = a.chi;
  __shared__ T pool[POOL];
  __shared__ T vch[32];                 // last-column chain vector
  // pass 1
  T* Rsh = pool;                        // carry R [k][li]
  T* Hb = Rsh + 32 * 32;                // Householder coefficients
  T* Ash = Hb + 32;                     // the row being absorbed [a][s][b]
  // pass 2
  T* Xsh = pool;                        // Jacobi exchange [(l, t)][k], row stride XSTRIDE
  T* Vsh = pool;                        // after the rotations: kept right singular vectors [j][t][k]
  T* Csh = Xsh + 64 * XSTRIDE;          // carry C [k][j]
  T* sig = Csh + 32 * 16;               // singular values by row

  T* Aj = a.A + job * (int64_t)L * SITE_A;
  T* Qj = a.Q + job * (int64_t)L * SITE_Q;
  const uint8_t* lab = a.labels + job * (int64_t)L * L;
  // single-qubit Pauli probabilities by code x + 2z, formed in double and rounded once to T
  T p0, p1, p2, p3;
  if (a.biased) {
    p0 = (T)a.pi[0]; p1 = (T)a.pi[1]; p2 = (T)a.pi[2]; p3 = (T)a.pi[3];
  } else {
    double pe = a.pe, pp = a.p00;
    if (a.pdev) {
      const double pj = a.pdev[job >> 2];
      pp = 1.0 - pj;
      pe = pj / 3.0;
    }
    p0 = (T)pp; p1 = (T)pe; p2 = (T)pe; p3 = (T)pe;
  }
  double logs = 0.0;

  for (int c = 0; c < L; ++c) {
    const bool last = (c == L - 1);
    for (int i = ln; i < 32 * 32; i += 64) Rsh[i] = (i == 0) ? T(1) : T(0);
    if (ln < 32) vch[ln] = (ln == 0) ? T(1) : T(0);
    __syncthreads();

    // ---------------- pass 1 (or the chain of the last column) ----------------
    for (int r = 0; r < L; ++r) {
      for (int i = ln; i < SITE_A; i += 64) Ash[i] = (c == 0) ? (i == 0 ? T(1) : T(0)) : Aj[(int64_t)r * SITE_A + i];
      __syncthreads();
      const int lb = lab[r * L + c];
      if (last) {
        // v'[ri] = sum_li v[li] B[li][0][ri], li = (a, u), ri = (b, dn)
        T nv = T(0);
        if (ln < 32) {
          const int b = ln >> 1, dn = ln & 1;
          const T t00 = tentry(r, c, L, lb, 0, 0, dn, 0, p0, p1, p2, p3), t01 = tentry(r, c, L, lb, 0, 1, dn, 0, p0, p1, p2, p3);
          const T t10 = tentry(r, c, L, lb, 1, 0, dn, 0, p0, p1, p2, p3), t11 = tentry(r, c, L, lb, 1, 1, dn, 0, p0, p1, p2, p3);
#pragma unroll
          for (int aa = 0; aa < 16; ++aa) {
            const T a0 = Ash[(aa * 2 + 0) * 16 + b], a1 = Ash[(aa * 2 + 1) * 16 + b];
            nv += vch[aa * 2 + 0] * (a0 * t00 + a1 * t01) + vch[aa * 2 + 1] * (a0 * t10 + a1 * t11);
          }
        }
        const T mx = wave_max(mabs(nv));
        __syncthreads();
        if (ln < 32) vch[ln] = (mx > T(0)) ? nv / mx : nv;
        logs += log((double)mx);
        __syncthreads();
        continue;
      }
      // lane (col, par): column col = (b, dn) of M_r = R B_r in the rows (k, t = par)
      T x[32];
      {
        const int b = hi >> 1, dn = hi & 1;
        const T t00 = tentry(r, c, L, lb, 0, 0, dn, par, p0, p1, p2, p3), t01 = tentry(r, c, L, lb, 0, 1, dn, par, p0, p1, p2, p3);
        const T t10 = tentry(r, c, L, lb, 1, 0, dn, par, p0, p1, p2, p3), t11 = tentry(r, c, L, lb, 1, 1, dn, par, p0, p1, p2, p3);
#pragma unroll
        for (int k = 0; k < 32; ++k) x[k] = T(0);
        // B[li][par][col] for li = (aa, u), formed as it is used
#pragma unroll
        for (int aa = 0; aa < 16; ++aa) {
          const T a0 = Ash[(aa * 2 + 0) * 16 + b], a1 = Ash[(aa * 2 + 1) * 16 + b];
          const T b0 = a0 * t00 + a1 * t01, b1 = a0 * t10 + a1 * t11;
#pragma unroll
          for (int k = 0; k < 32; ++k) x[k] += Rsh[k * 32 + aa * 2] * b0 + Rsh[k * 32 + aa * 2 + 1] * b1;
        }
      }
      __syncthreads();   // every lane has read R
      T* Qr = Qj + (int64_t)r * SITE_Q;
      if (r == L - 1) {
#pragma unroll
        for (int k = 0; k < 32; ++k) Qr[(2 * k + par) * 32 + hi] = x[k];
        continue;
      }
      // Householder QR of M_r (64 x 32): reflection j zeroes rows j+1.. of column j. Vector j is kept in the
      // row's workspace slot as Hg[j][par][k] (row 2k + par), each lane's half contiguous.
      T* Hg = Qr;
      for (int j = 0; j < 32; ++j) {
        if (hi == j) {
#pragma unroll
          for (int k = 0; k < 32; ++k) Hg[(j * 2 + par) * 32 + k] = (2 * k + par >= j) ? x[k] : T(0);
        }
        __syncthreads();
        // one read of the (raw) vector for its norm and its product with this column; the pivot entry
        // changes from alpha to vj, which the product corrects with this lane's pivot-row entry xp
        const T* hv = Hg + (j * 2 + par) * 32;
        T pn = T(0), pw = T(0), xp = T(0);
#pragma unroll
        for (int k = 0; k < 32; ++k) {
          const T v = hv[k];
          pn += v * v;
          pw += v * x[k];
          xp += (2 * k + par == j) ? x[k] : T(0);
        }
        const T nrm = msqrt(pn + __shfl_xor(pn, 1));
        const T alpha = Hg[(j * 2 + (j & 1)) * 32 + (j >> 1)];
        T beta = T(0), vj = alpha, diag = alpha;
        if (nrm > T(0)) {
          const T sg = (alpha >= T(0)) ? T(1) : T(-1);
          vj = alpha + sg * nrm;
          beta = T(1) / (nrm * (nrm + mabs(alpha)));
          diag = -sg * nrm;
        }
        pw += (vj - alpha) * xp;
        const T w = (pw + __shfl_xor(pw, 1)) * beta;
        if (hi > j) {
#pragma unroll
          for (int k = 0; k < 32; ++k) x[k] -= w * ((2 * k + par == j) ? vj : hv[k]);
        } else if (hi == j && nrm > T(0)) {
#pragma unroll
          for (int k = 0; k < 32; ++k) {
            const int row = 2 * k + par;
            x[k] = (row == j) ? diag : (row > j ? T(0) : x[k]);
          }
        }
        __syncthreads();   // every lane has read vector j as it was
        if (ln == 0) {
          Hg[(j * 2 + (j & 1)) * 32 + (j >> 1)] = vj;
          Hb[j] = beta;
        }
      }
      __syncthreads();
      // carry R (rows 0..31 of the reduced matrix), unit Frobenius norm
      {
        T f = T(0);
#pragma unroll
        for (int k = 0; k < 16; ++k) f += x[k] * x[k];
        const T fro = msqrt(wave_sum(f));
        const T inv = (fro > T(0)) ? T(1) / fro : T(0);
#pragma unroll
        for (int k = 0; k < 16; ++k) Rsh[(2 * k + par) * 32 + hi] = x[k] * inv;
        logs += log((double)fro);
      }
      // Q = H_0 H_1 ... H_31 applied to the first 32 unit columns
      {
        T q[32];
#pragma unroll
        for (int k = 0; k < 32; ++k) q[k] = (2 * k + par == hi) ? T(1) : T(0);
        for (int j = 31; j >= 0; --j) {
          const T* hv = Hg + (j * 2 + par) * 32;
          T pw = T(0);
#pragma unroll
          for (int k = 0; k < 32; ++k) pw += hv[k] * q[k];
          const T w = (pw + __shfl_xor(pw, 1)) * Hb[j];
#pragma unroll
          for (int k = 0; k < 32; ++k) q[k] -= w * hv[k];
        }
        __syncthreads();   // every lane has read the vectors before Q replaces them
#pragma unroll
        for (int k = 0; k < 32; ++k) Qr[(2 * k + par) * 32 + hi] = q[k];
      }
      __syncthreads();
    }
    __syncthreads();
    if (last) break;

    // ---------------- pass 2: truncating SVD sweep, bottom row to top row ----------------
    for (int i = ln; i < 32 * 16; i += 64) Csh[i] = (i == 0) ? T(1) : T(0);
    __syncthreads();
    for (int r = L - 1; r >= 0; --r) {
      // lane (l, t) = ln: y[k] = N[l][(t, k)] = sum_m Q_r[(l, t)][m] C[m][k]
      T y[16];
      {
        const T* qrow = Qj + (int64_t)r * SITE_Q + ln * 32;
        T qv[32];
#pragma unroll
        for (int m = 0; m < 32; ++m) qv[m] = qrow[m];
#pragma unroll
        for (int k = 0; k < 16; ++k) y[k] = T(0);
#pragma unroll
        for (int m = 0; m < 32; ++m) {
#pragma unroll
          for (int k = 0; k < 16; ++k) y[k] += qv[m] * Csh[m * 16 + k];
        }
      }
      T y0[16];   // N before the rotations
#pragma unroll
      for (int k = 0; k < 16; ++k) y0[k] = y[k];
      // one-sided Jacobi on the rows of N (columns of N^T), paired by the circle method over 32
      T nf2 = T(0);
#pragma unroll
      for (int k = 0; k < 16; ++k) nf2 += y[k] * y[k];
      const T thr2 = wave_sum(nf2) * (Tol<T>::rank * Tol<T>::rank);
      for (int sw = 0; sw < Tol<T>::sweeps; ++sw) {
        int rotated = 0;
        T c2max = T(0);   // largest squared cosine of a pair above the noise threshold in this sweep
        // squared norm of this lane's row, exact at the start of the sweep and then carried through the
        // rotations (both lanes of a row hold the same value); it travels with the row in slot 16
        T own = T(0);
#pragma unroll
        for (int k = 0; k < 16; ++k) own += y[k] * y[k];
        own += __shfl_xor(own, 1);
        for (int rd = 0; rd < 31; ++rd) {
          const int pl = (hi == 31) ? rd : (hi == rd) ? 31 : (2 * rd - hi + 62) % 31;
#pragma unroll
          for (int k = 0; k < 16; ++k) Xsh[ln * XSTRIDE + k] = y[k];
          Xsh[ln * XSTRIDE + 16] = own;
          __syncthreads();
          T z[16], gg = T(0);
#pragma unroll
          for (int k = 0; k < 16; ++k) {
            z[k] = Xsh[(2 * pl + par) * XSTRIDE + k];
            gg += y[k] * z[k];
          }
          const T other = Xsh[(2 * pl + par) * XSTRIDE + 16];
          __syncthreads();   // every lane has read its partner before the next round's writes
          gg += __shfl_xor(gg, 1);
          // (alpha, beta) = squared norms of the lower- and higher-numbered row of the pair
          const bool lower = hi < pl;
          const T al = lower ? own : other, be = lower ? other : own;
          // squared cosine of the pair (approximate reciprocal: it only decides whether to rotate)
          const T c2 = (al > thr2 && be > thr2) ? gg * gg * __builtin_amdgcn_rcp(al * be) : T(0);
          c2max = c2 > c2max ? c2 : c2max;
          if (c2 > Tol<T>::jac * Tol<T>::jac) {
            // The angle only has to bring the pair closer to orthogonal, so t = tan(theta) is formed in FP32
            // (fast reciprocal and square root; above the noise threshold zeta stays within 1e30); cos and
            // sin are then formed in FP64 from that t, so that the rotation is orthogonal to FP64 rounding.
            const float zf = (float)(be - al) * __builtin_amdgcn_rcpf(2.0f * (float)gg), azf = fabsf(zf);
            const float denf = azf + (azf < 1e18f ? __builtin_sqrtf(fmaf(zf, zf, 1.0f)) : azf);
            const T tt = (T)copysignf(__builtin_amdgcn_rcpf(denf), zf);
            const T xx = tt * tt + T(1);
            T cs = __builtin_amdgcn_rsq(xx);
            cs = cs * (T(1.5) - T(0.5) * xx * cs * cs);
            cs = cs * (T(1.5) - T(0.5) * xx * cs * cs);
            const T sn = cs * tt;
            // lower row p: c p - s q; higher row q: s p + c q
#pragma unroll
            for (int k = 0; k < 16; ++k) y[k] = lower ? (cs * y[k] - sn * z[k]) : (sn * z[k] + cs * y[k]);
            // squared norms after this rotation: c^2 (alpha -+ 2 t gamma + t^2 beta) for the lower row and
            // c^2 (beta +- ...) for the higher one, exact for the c and s applied
            const T cc = cs * cs;
            own = lower ? cc * (al - T(2) * tt * gg + tt * tt * be) : cc * (be + T(2) * tt * gg + tt * tt * al);
            rotated = 1;
          }
        }
        // Jacobi converges quadratically: after a sweep whose pairs all started within cos 1e-8 of
        // orthogonal, they are within ~1e-16 and a confirming sweep would rotate nothing
        if (!__any(rotated) || wave_max(c2max) < T(1e-16)) break;
      }
      // singular values, ranks (largest first, ties to the lower row), kept rows
      T s2 = T(0);
#pragma unroll
      for (int k = 0; k < 16; ++k) s2 += y[k] * y[k];
      const T s2r = s2 + __shfl_xor(s2, 1);
      const T sv = (s2r > thr2) ? msqrt(s2r) : T(0);
      const T key = (sv == sv) ? sv : T(-1);
      if (par == 0) sig[hi] = key;
      __syncthreads();
      int rank = 0;
      for (int i = 0; i < 32; ++i) {
        const T o = sig[i];
        rank += (o > key || (o == key && i < hi)) ? 1 : 0;
      }
      const bool kept = rank < chi && sv > T(0);
      const T inv = kept ? T(1) / sv : T(0);
      if (rank < 16) {
        T* Ar = Aj + (int64_t)r * SITE_A + (rank * 2 + par) * 16;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          Ar[k] = y[k] * inv;
          Vsh[rank * 32 + par * 16 + k] = y[k] * inv;
        }
      }
      const T fro = msqrt(wave_sum((par == 0 && kept) ? sv * sv : T(0)));
      __syncthreads();
      // C[l][j] = sum_(t, k) N[l][(t, k)] V[j][(t, k)]: lane (l, t) sums its half t, the pair adds halves;
      // lane t = 0 stores j < 8, lane t = 1 stores j >= 8
      {
        const T finv = (fro > T(0)) ? T(1) / fro : T(0);
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          T acc = T(0);
#pragma unroll
          for (int k = 0; k < 16; ++k) acc += y0[k] * Vsh[j * 32 + par * 16 + k];
          acc += __shfl_xor(acc, 1);
          if ((j >> 3) == par) Csh[hi * 16 + j] = acc * finv;
        }
        logs += log((double)fro);
      }
      __syncthreads();
    }
  }
  if (ln == 0) {
    const T v = vch[0];
    a.loglik[job] = (v > T(0)) ? logs + log((double)v) : (double)NAN;
  }
}

// decision (largest estimate, NaN as -inf, ties to the lowest index) and correction f_s L*
__global__ __launch_bounds__(256) void bmps_decide_kernel(const double* __restrict__ loglik,
                                                          const uint8_t* __restrict__ labels, int d,
                                                          uint8_t* __restrict__ coset,
                                                          uint8_t* __restrict__ correction) {
  const int64_t b = blockIdx.x;
  int best = 0;
  double bv = -INFINITY;
  for (int k = 0; k < 4; ++k) {
    const double v = loglik[b * 4 + k];
    if (!isnan(v) && v > bv) { bv = v; best = k; }
  }
  if (threadIdx.x == 0) coset[b] = (uint8_t)best;
  if (!correction) return;
  const int L = 2 * d - 1, n = d * d + (d - 1) * (d - 1);
  const uint8_t* lab = labels + (b * 4 + best) * (int64_t)L * L;
  for (int site = threadIdx.x; site < L * L; site += blockDim.x) {
    const int r = site / L, c = site % L;
    if ((r + c) & 1) continue;
    const int q = (r / 2) * (2 * d - 1) + ((r & 1) ? d + (c - 1) / 2 : c / 2);
    correction[b * n + q] = (uint8_t)(lab[site] & 3);
  }
}

}  // namespace

size_t bmps_state_bytes(int d, int64_t jobs) {
  const int64_t L = 2 * d - 1;
  return (size_t)(jobs * L * (SITE_A + SITE_Q) * (int64_t)sizeof(double));
}

hipError_t launch_bmps_contract(hipStream_t st, const BmpsArgs& a) {
  if (a.jobs <= 0) return hipSuccess;
  bmps_kernel<double><<<dim3((unsigned)a.jobs), dim3(64), 0, st>>>(a);
  return hipGetLastError();
}

hipError_t launch_bmps_decide(hipStream_t st, const BmpsArgs& a, uint8_t* coset, uint8_t* correction) {
  if (a.jobs >= 4)
    bmps_decide_kernel<<<dim3((unsigned)(a.jobs / 4)), dim3(256), 0, st>>>(a.loglik, a.labels, a.d, coset, correction);
  return hipGetLastError();
}

}  // namespace bbp
