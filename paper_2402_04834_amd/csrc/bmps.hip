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
//     M_r = Q_r R_r; Q_r goes to the workspace in compact form (its reflection vectors), R_r (unit Frobenius
//     norm, the norm into the log-scale) is carried into the next row. The last row keeps M_r itself.
//   pass 2, bottom row to top row: N_r = Q_r C_{r+1} (the reflections applied to the carry; Q_r is never
//     formed) as a 2 chi x (2 * chi) matrix (rows: left bond;
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
// Layout (wave_mps.hpp): every lane owns matrix columns in registers. Pass 1: lane (col, par) holds the 32
// entries of column col of M_r in the rows of parity par; a Householder vector is broadcast through LDS from
// the two lanes that own it, and the vectors reach the workspace once, when the row is factored. Pass 2:
// the reflections are applied column-wise to the carry, and lane (l, t) then holds the 16 entries (t, k) of
// row l of N_r; a Jacobi round pairs rows by the circle method and exchanges them through LDS. Bond
// dimensions are padded to 2 chi_max = 32 with zeros.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "bmps_launch.hpp"
#include "wave_mps.hpp"

namespace bbp {
namespace {

using namespace wmps;

constexpr int SITE_A = 16 * 2 * 16;   // entries per compressed row: [j][t][k], j, k < chi_max
constexpr int SITE_Q = TQ;            // entries per pass-1 factor: compact reflections and coefficients


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


// LDS: pass 1 and pass 2 never overlap in time, so their buffers share one pool (13.6 KB). Pass 1: the carry
// R, the two Householder vector buffers and the coefficients, the row being absorbed; pass 2: the Jacobi
// exchange (then V), the carry C, the singular values. Two wavefronts per SIMD (256 registers per lane):
// measured faster than three, where the QR step's column, vector and row masks spill.
constexpr int POOL_P1 = 32 * 32 + 2 * 64 + 32 + SITE_A;
constexpr int POOL_P2 = 64 * XS + 32 * 16 + 32;
constexpr int POOL = POOL_P1 > POOL_P2 ? POOL_P1 : POOL_P2;

__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 2))) void bmps_kernel(BmpsArgs a) {
  using T = double;
  const int64_t job = blockIdx.x;
  const int ln = threadIdx.x, hi = ln >> 1, par = ln & 1;
  const int L = 2 * a.d - 1, chi = a.chi;
  __shared__ T pool[POOL];
  __shared__ T vch[32];                 // last-column chain vector
  // pass 1
  T* Rsh = pool;                        // carry R [k][li]
  T* vb = Rsh + 32 * 32;                // Householder vector buffers
  T* Hb = vb + 2 * 64;                  // Householder coefficients
  T* Ash = Hb + 32;                     // the row being absorbed [a][s][b]
  // pass 2
  T* Xsh = pool;                        // Jacobi exchange, row stride XS (then V)
  T* Csh = Xsh + 64 * XS;               // carry C [k][j]
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
        const T mx = wmax(fabs(nv));
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
#pragma unroll 1
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
        // the bottom row's right bond has one value: M has the single column (0, 0), kept as is
        if (hi == 0) {
#pragma unroll
          for (int k = 0; k < 32; ++k) Qr[2 * k + par] = x[k];
        }
        continue;
      }
      T rd;
      qr64u<32>(x, rd, vb, Hb);
      logs += store_r(x, rd, Rsh);
      store_v(x, 32, Hb, Qr);
    }
    __syncthreads();
    if (last) break;

    // ---------------- pass 2: truncating SVD sweep, bottom row to top row ----------------
    for (int r = L - 1; r >= 0; --r) {
      // lane (l, t) = ln: y[k] = N[l][(t, k)], N = Q_r C_{r+1} (the bottom row: its own matrix)
      T y[16];
      const T* Qr = Qj + (int64_t)r * SITE_Q;
      if (r == L - 1) {
#pragma unroll
        for (int k = 0; k < 16; ++k) y[k] = (k == 0) ? Qr[ln] : T(0);
      } else {
        T X[16];
        apply_q(X, 32, Qr, Csh);
        cols_to_rows(X, Xsh, y);
      }
      logs += svd_step(y, chi, Xsh, Csh, sig, Aj + (int64_t)r * SITE_A, false);
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
  bmps_kernel<<<dim3((unsigned)a.jobs), dim3(64), 0, st>>>(a);
  return hipGetLastError();
}

hipError_t launch_bmps_decide(hipStream_t st, const BmpsArgs& a, uint8_t* coset, uint8_t* correction) {
  if (a.jobs >= 4)
    bmps_decide_kernel<<<dim3((unsigned)(a.jobs / 4)), dim3(256), 0, st>>>(a.loglik, a.labels, a.d, coset, correction);
  return hipGetLastError();
}

}  // namespace bbp
