// warm.hip -- learned warm start of blockBP: a convolutional network that predicts the initial block
// messages (replacing the uniform start of Alg. 1, remark 2) from the local syndrome; inference and
// training (forward, backward, Adam) for gfx950.
//
// Network (per coset job, on the (2d-1) x (2d-1) grid):
//   input  11 channels per site: label x / z bits at qubits, syndrome bit at checks, qubit / Z-check /
//          X-check indicators, the noise rate p, 1 (inside the grid), the coset's X and Z bits, and the
//          generator bit G at checks (features_kernel); no absolute position, so that the network applies
//          unchanged to distances it was not trained on;
//   trunk  three 3x3 convolutions with zero padding (11 -> 64 -> 128 -> 96 channels), ReLU after the first
//          two; each is an implicit GEMM on the matrix cores: FP32 (v_mfma_f32_16x16x4f32) for training and
//          for parity, or BF16 weights and activations with FP32 sums (v_mfma_f32_16x16x32_bf16) for inference;
//          activations are row-major [site][channel];
//   head   per directed message with K legs (leg i joins site a_i of the sender to site b_i across the
//          boundary), with f_i = [F(a_i), F(b_i)] and the weights of the message's direction:
//          u_i = Wu^T f_i + bu (2 values), P_i = Wp^T [f_i, f_{i+1}] + bp (4 values),
//          s(b) = sum_i u_i[b_i] + sum_i P_i[2 b_i + b_{i+1}], message = exp(s) normalised to unit 2-norm,
//          one wavefront per (job, message), lane = leg configuration b (leg 0 most significant);
//   loss   KL(q || p) of the distributions q = t / sum(t) of the converged message t and p = softmax(s),
//          averaged over the trained messages (its gradient in s, p - q, does not vanish when the
//          prediction is peaked at the wrong configuration, unlike overlap losses of unit vectors).
// Parameters (FP32, in this order): conv1 W [99][64], b [64]; conv2 W [576][128], b [128]; conv3 W
// [1152][96], b [96]; then per direction E, W, S, N: Wu [192][2], bu [2], Wp [384][4], bp [4].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/bbp.h"
#include "plan.hpp"

namespace {

constexpr int C0 = 11, C1 = 64, C2 = 128, C3 = 96;
constexpr int MAXK = 6;                                   // legs of a message (block size <= 6)
constexpr int HEAD = 2 * C3 * 2 + 2 + 4 * C3 * 4 + 4;     // parameters of one direction's head
constexpr int NOUT = 2 * MAXK + 4 * (MAXK - 1);           // head outputs of one message (<= 32)

struct Offsets {
  size_t w1, b1, w2, b2, w3, b3, head, total;
};
constexpr Offsets offsets() {
  Offsets o{};
  size_t x = 0;
  o.w1 = x; x += 9 * C0 * C1;
  o.b1 = x; x += C1;
  o.w2 = x; x += 9 * C1 * C2;
  o.b2 = x; x += C2;
  o.w3 = x; x += 9 * C2 * C3;
  o.b3 = x; x += C3;
  o.head = x; x += 4 * HEAD;
  o.total = x;
  return o;
}
constexpr Offsets OFF = offsets();

thread_local std::string w_err = "no error";
int wfail(int code, const std::string& m) {
  w_err = m;
  return code;
}
#define W_TRY(expr)                                                                                    \
  do {                                                                                                 \
    hipError_t _e = (expr);                                                                            \
    if (_e != hipSuccess) return wfail(BBP_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e));    \
  } while (0)

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float wsum(float v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ float wmax(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}

// ------------------------------------------------------------------------------------------ kernels
// Input channels of every (job, site); job = 4 * syndrome + coset; one workgroup per syndrome. Generator
// bits G: the generators whose product clears f_s L from the horizontal edges (but for the last row of its
// x part and the last column of its z part), i.e. prefix parities of f_s L on the horizontal edges:
// plaquette (r, c): parity of (f_s L)^x on the horizontal edges above it in column c; vertex (r, c): parity
// of (f_s L)^z on the horizontal edges left of it in row r. They are quadrant parities of the syndrome: the
// non-local part of where the coset network's generator variables concentrate, out of reach of 3x3
// convolutions.
// BF16 storage (round to nearest even on the bit pattern) and widening
__device__ __forceinline__ unsigned short f2bf(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ void store_el(float* p, float v) { *p = v; }
__device__ __forceinline__ void store_el(unsigned short* p, float v) { *p = f2bf(v); }

// CS: channels stored per site (C0, or 16 for the BF16 convolutions, whose K steps need 8-channel groups;
// channels C0 .. CS-1 are zero)
template <class T, int CS>
__global__ __launch_bounds__(256) void features_kernel(const uint8_t* __restrict__ syn, const double* __restrict__ pdev,
                                                       float p, int d, T* __restrict__ X) {
  __shared__ uint8_t s[2 * 32 * 31];
  __shared__ uint8_t Q[64][64];   // bit 0: (f_s)^x, bit 1: (f_s)^z on horizontal edges
  __shared__ uint8_t G[64][64];   // generator bits of coset I at check sites
  const int64_t b = blockIdx.x;
  const int L = 2 * d - 1, m = 2 * d * (d - 1), nz = d * (d - 1);
  const int tid = threadIdx.x;
  for (int i = tid; i < m; i += blockDim.x) s[i] = syn[b * m + i] & 1;
  __syncthreads();
  auto zchk = [&](int r, int c) -> int { return s[(r / 2) * (d - 1) + (c - 1) / 2]; };
  auto xchk = [&](int r, int c) -> int { return s[nz + ((r - 1) / 2) * d + c / 2]; };
  // f_s: chains of the horizontal-edge qubits to the checks right of / below them
  auto fs = [&](int r, int c, int& x, int& z) {
    x = 0;
    z = 0;
    if ((r & 1) == 0 && (c & 1) == 0) {
      for (int cc = c + 1; cc < L; cc += 2) x ^= zchk(r, cc);
      for (int rr = r + 1; rr < L; rr += 2) z ^= xchk(rr, c);
    }
  };
  for (int site = tid; site < L * L; site += blockDim.x) {
    const int r = site / L, c = site % L;
    if ((r & 1) == 0 && (c & 1) == 0) {
      int x, z;
      fs(r, c, x, z);
      Q[r][c] = (uint8_t)(x | (z << 1));
    }
  }
  __syncthreads();
  // prefix parities: one thread per column (plaquettes) and one per row (vertices)
  for (int i = tid; i < 2 * L; i += blockDim.x) {
    int acc = 0;
    if (i < L) {
      const int c = i;
      if ((c & 1) == 0)
        for (int r = 0; r < L; ++r) {
          if ((r & 1) == 0) acc ^= Q[r][c] & 1;
          else G[r][c] = (uint8_t)acc;
        }
    } else {
      const int r = i - L;
      if ((r & 1) == 0)
        for (int c = 0; c < L; ++c) {
          if ((c & 1) == 0) acc ^= (Q[r][c] >> 1) & 1;
          else G[r][c] = (uint8_t)acc;
        }
    }
  }
  __syncthreads();
  const float pj = pdev ? (float)pdev[b] : p;
  for (int e = tid; e < 4 * L * L; e += blockDim.x) {
    const int coset = e / (L * L), site = e % (L * L), r = site / L, c = site % L;
    float v[C0];
    for (int k = 0; k < C0; ++k) v[k] = 0.0f;
    const int bx = (coset == 1 || coset == 2) ? 1 : 0, bz = (coset == 2 || coset == 3) ? 1 : 0;
    if (((r + c) & 1) == 0) {
      int x = 0, z = 0;
      if ((r & 1) == 0) {   // horizontal-edge qubit: f_s from the table above (vertical ones carry none)
        x = Q[r][c] & 1;
        z = Q[r][c] >> 1;
      }
      const int lx = (r == 0) ? 1 : 0, lz = (c == 0) ? 1 : 0;   // logical X on row 0, Z on column 0
      v[0] = (float)(x ^ (bx & lx));
      v[1] = (float)(z ^ (bz & lz));
      v[3] = 1.0f;
    } else if ((r & 1) == 0) {
      v[2] = (float)zchk(r, c);
      v[4] = 1.0f;
      v[10] = (float)(G[r][c] ^ bz);   // the coset's logical Z lies on column 0, left of every vertex
    } else {
      v[2] = (float)xchk(r, c);
      v[5] = 1.0f;
      v[10] = (float)(G[r][c] ^ bx);   // the coset's logical X lies on row 0, above every plaquette
    }
    v[6] = pj;
    v[7] = 1.0f;
    v[8] = (float)bx;
    v[9] = (float)bz;
    T* o = X + ((b * 4 + coset) * (int64_t)L * L + site) * CS;
    if constexpr (sizeof(T) == 2 && CS == 16) {
      // the site's 16 BF16 channels as two 16-byte stores
      unsigned w[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const float lo = 2 * k < C0 ? v[2 * k] : 0.0f, hi = 2 * k + 1 < C0 ? v[2 * k + 1] : 0.0f;
        w[k] = (unsigned)f2bf(lo) | ((unsigned)f2bf(hi) << 16);
      }
      ((uint4*)o)[0] = uint4{w[0], w[1], w[2], w[3]};
      ((uint4*)o)[1] = uint4{w[4], w[5], w[6], w[7]};
    } else {
      for (int k = 0; k < CS; ++k) store_el(o + k, k < C0 ? v[k] : 0.0f);
    }
  }
}

// Implicit-GEMM 3x3 convolution (zero padding) on the matrix cores, FP32 products and sums. The operand
// gathered from an activation is never materialised: a 64 x 16 tile is read straight from the shifted
// sites into LDS. Activations are [row = job * L^2 + r * L + c][channel]; tap t = 3 dy + dx reads site
// (r + dy - 1, c + dx - 1). Three uses:
//   G_FWD  Y[row][co] = act(sum_{t,ci} X[row + t][ci] W[t cin + ci][co] + b[co])      (M rows, N cout, K 9 cin)
//   G_DX   dX[row][ci] = mask * sum_{t,co} dY[row - t][co] W[t cin + ci][co]           (M rows, N cin, K 9 cout)
//          (the adjoint of the gather; mask = ReLU'(the layer's input activation) when EPI = 1)
//   G_DW   dW[t cin + ci][co] += sum_rows X[row + t][ci] dY[row][co]                  (M 9 cin, N cout, K rows)
//          (K split over grid.z, atomically accumulated into dW, which the caller has zeroed)
// 64 x 64 output tile per workgroup of four waves (each 32 x 32 = 2 x 2 MFMA 16x16x4 blocks), K in
// chunks of 16. grid.x = M tiles, grid.y = N tiles.
enum { G_FWD = 0, G_DX = 1, G_DW = 2 };

struct Site {
  int64_t base;
  int r, c;
};
__device__ __forceinline__ Site site_of(int64_t row, int L) {
  const int64_t LL = (int64_t)L * L, job = row / LL;
  const int s = (int)(row - job * LL);
  return Site{job * LL, s / L, s - (s / L) * L};
}
// row of the site shifted by tap (sign +1) or against it (sign -1); -1 outside the grid
__device__ __forceinline__ int64_t shifted(const Site& s, int tap, int sign, int L) {
  const int r = s.r + sign * (tap / 3 - 1), c = s.c + sign * (tap % 3 - 1);
  return (r >= 0 && r < L && c >= 0 && c < L) ? s.base + (int64_t)r * L + c : -1;
}

template <int MODE, int EPI>
__global__ __launch_bounds__(256) void conv_gemm(int L, int64_t rows, int cin, int cout, int64_t kchunk,
                                                 const float* __restrict__ X, const float* __restrict__ Bm,
                                                 float* __restrict__ C, const float* __restrict__ aux) {
  __shared__ float As[64][17];
  __shared__ float Bs[16][65];
  const int64_t Mdim = (MODE == G_DW) ? 9 * cin : rows;
  const int Ndim = (MODE == G_DX) ? cin : cout;
  const int64_t Kdim = (MODE == G_FWD) ? 9 * cin : (MODE == G_DX) ? 9 * cout : rows;
  const int Cs = (MODE == G_DX) ? cout : cin;     // channels of the gathered activation
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t m0 = (int64_t)blockIdx.x * 64;
  const int n0 = blockIdx.y * 64;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  const int64_t kb = (int64_t)blockIdx.z * kchunk, ke = std::min(Kdim, kb + kchunk);
  f4 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.0f, 0.0f, 0.0f, 0.0f};
  // the row this thread gathers for (fixed across K for G_FWD / G_DX)
  Site arow{0, 0, 0};
  const int amm = tid >> 2, akq = (tid & 3) * 4;
  if (MODE != G_DW && m0 + amm < Mdim) arow = site_of(m0 + amm, L);
  for (int64_t k0 = kb; k0 < ke; k0 += 16) {
    if (MODE != G_DW) {
      float v[4] = {0.0f, 0.0f, 0.0f, 0.0f};
      if (m0 + amm < Mdim)
        for (int j = 0; j < 4; ++j) {
          const int64_t k = k0 + akq + j;
          if (k < ke) {
            const int tap = (int)(k / Cs), ch = (int)(k - (int64_t)tap * Cs);
            const int64_t src = shifted(arow, tap, MODE == G_FWD ? 1 : -1, L);
            if (src >= 0) v[j] = X[src * Cs + ch];
          }
        }
      for (int j = 0; j < 4; ++j) As[amm][akq + j] = v[j];
    } else {
      const int kk = tid >> 4, mq = (tid & 15) * 4;
      const int64_t k = k0 + kk;
      float v[4] = {0.0f, 0.0f, 0.0f, 0.0f};
      if (k < ke) {
        const Site s = site_of(k, L);
        for (int j = 0; j < 4; ++j) {
          const int64_t m = m0 + mq + j;
          if (m < Mdim) {
            const int tap = (int)(m / cin), ch = (int)(m - (int64_t)tap * cin);
            const int64_t src = shifted(s, tap, 1, L);
            if (src >= 0) v[j] = X[src * cin + ch];
          }
        }
      }
      for (int j = 0; j < 4; ++j) As[mq + j][kk] = v[j];
    }
    if (MODE == G_DX) {
      const int nn = tid >> 2, kq = (tid & 3) * 4;
      const int n = n0 + nn;
      for (int j = 0; j < 4; ++j) {
        const int64_t k = k0 + kq + j;
        float v = 0.0f;
        if (n < Ndim && k < ke) {
          const int tap = (int)(k / cout), co = (int)(k - (int64_t)tap * cout);
          v = Bm[((int64_t)tap * cin + n) * cout + co];
        }
        Bs[kq + j][nn] = v;
      }
    } else {
      const int kk = tid >> 4, nq = (tid & 15) * 4;
      const int64_t k = k0 + kk;
      for (int j = 0; j < 4; ++j) {
        const int n = n0 + nq + j;
        Bs[kk][nq + j] = (k < ke && n < Ndim) ? Bm[k * Ndim + n] : 0.0f;
      }
    }
    __syncthreads();
    for (int ks = 0; ks < 4; ++ks) {
      const int kk = ks * 4 + (lane >> 4);
      float a[2], b[2];
      for (int i = 0; i < 2; ++i) a[i] = As[wm + i * 16 + (lane & 15)][kk];
      for (int j = 0; j < 2; ++j) b[j] = Bs[kk][wn + j * 16 + (lane & 15)];
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int r = 0; r < 4; ++r) {
        const int64_t row = m0 + wm + i * 16 + 4 * (lane >> 4) + r;
        const int col = n0 + wn + j * 16 + (lane & 15);
        if (row >= Mdim || col >= Ndim) continue;
        float v = acc[i][j][r];
        float* dst = &C[row * Ndim + col];
        if (MODE == G_FWD) {
          v += aux[col];
          *dst = EPI ? fmaxf(v, 0.0f) : v;
        } else if (MODE == G_DX) {
          *dst = (EPI && !(aux[row * Ndim + col] > 0.0f)) ? 0.0f : v;
        } else {
          atomicAdd(dst, v);
        }
      }
}

// Forward convolution in BF16 (inference): activations and weights stored as BF16, products and sums in FP32
// on v_mfma_f32_16x16x32_bf16 (lane l supplies row l%16 of A and column l%16 of B with k = 8 (l/16) .. +7 of
// a 32-step, and holds D rows 4 (l/16) .. +3 of column l%16). Implicit GEMM with the gather of conv_gemm<G_FWD>:
// Y[row][co] = act(sum_{t, ci} X[row + t][ci] Wt[co][t CIN + ci] + b[co]). One workgroup of four waves computes
// 128 rows x all NT output channels (2 x 2 waves of 64 x NT/2, i.e. 4 x NT/32 MFMA blocks each), so every
// gathered activation tile is read once; K advances in steps of 32 through double-buffered, swizzled LDS tiles
// (one barrier per step), the global loads two steps ahead in flight (two register sets). A 16-byte load is 8
// channels of one tap (CIN is a multiple of 16) at an offset computed once per row and tap; the weights come
// transposed, Wt[co][k], k padded to a multiple of the stage with zeros, so both LDS tiles are k-contiguous.
// BF16 outputs leave through an LDS tile in 16-byte rows. This gather kernel serves grids too large for the
// haloed tile of conv_halo_bf16 below (L > 49).
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));   // 16 bytes staged through registers

// Wt[co][kp] (kp < kpad) = W[t cin + ci][co] for kp = t cs + ci with ci < cin, else 0 (BF16)
__global__ void weights_t_kernel(const float* __restrict__ W, int cin, int cs, int cout, int kpad,
                                 unsigned short* __restrict__ Wt) {
  const int64_t n = (int64_t)cout * kpad;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int co = (int)(i / kpad), kp = (int)(i - (int64_t)co * kpad), t = kp / cs, ci = kp - t * cs;
    Wt[i] = (t < 9 && ci < cin) ? f2bf(W[((int64_t)t * cin + ci) * cout + co]) : (unsigned short)0;
  }
}

constexpr int CONV_KS = 32;   // k per LDS stage of the BF16 convolutions (one MFMA step)
// k of a BF16 weight row: 9 cs padded to a multiple of the stage
constexpr int kpad(int cs) { return (9 * cs + CONV_KS - 1) / CONV_KS * CONV_KS; }

typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
typedef float fl2 __attribute__((ext_vector_type(2)));

// LDS tiles hold rows of 32 BF16 (64 bytes, four 16-byte chunks); chunk g of row r sits at chunk g ^ ((r / 2) % 4).
// A thread quad writes the four chunks of one row, so eight consecutive lanes write two whole rows; the 16
// lanes of a fragment read one chunk of 16 consecutive rows, which the swizzle spreads over all banks.
__device__ __forceinline__ int swz(int r, int g) { return r * 32 + 8 * (g ^ ((r >> 1) & 3)); }

// WM: waves along M (wave tiles of 64 x NT/2, two waves along N: workgroups of 128 WM threads computing
// 64 WM x NT). Compiled for three wavefronts per SIMD (at most 168 registers): the unconstrained build takes
// 110 VGPRs and 96 accumulation registers, two wavefronts per SIMD, and ran the forward 13 % slower.
template <int CIN, int NT, int WM, int RELU, bool OUT_BF>
__global__ __launch_bounds__(128 * WM) __attribute__((amdgpu_waves_per_eu(3))) void conv_fwd_bf16(int L, int64_t rows, const unsigned short* __restrict__ X,
                                                     const unsigned short* __restrict__ Wt,
                                                     const float* __restrict__ bias, void* __restrict__ Y) {
  constexpr int KS = CONV_KS, KP = kpad(CIN), NS = KP / KS;   // stages
  constexpr int TH = 128 * WM;                                 // threads
  constexpr int MT = 64 * WM, WN = NT / 2, NJ = WN / 16;       // workgroup rows, wave columns, 16-blocks
  constexpr int UA = MT * 4 / TH, UB = (NT * 4 + TH - 1) / TH;  // 16-byte chunks per thread and stage
  constexpr int STAGE = (MT + NT) * KS;                        // one A and one B buffer
  constexpr int TILE = OUT_BF ? MT * NT : 0;                   // BF16 output tile, written out through LDS
  static_assert(CIN % 16 == 0 && NT % 32 == 0 && NT <= 128 && (WM == 2 || WM == 4) && KS == 32, "tile shape");
  __shared__ __align__(16) unsigned short lds[(2 * STAGE > TILE) ? 2 * STAGE : TILE];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t m0 = (int64_t)blockIdx.x * MT;
  const int wm = (w >> 1) * 64, wn = (w & 1) * WN;
  const int ag = tid & 3;   // the 8-k group of every chunk this thread stages
  // The gather is a raw buffer load: an offset at or past the buffer's size reads zeros without touching
  // memory, so the padding taps need no branch and every stage issues the same loads (the wait before a
  // stage's LDS store then covers only the older stage's loads, not the ones just issued).
  const unsigned xbytes = (unsigned)(rows * CIN * 2);   // the host keeps this + 256 below 2^32
  const __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc((void*)X, (short)0, (int)xbytes, 0x00020000);
  // per staged row: its byte offset and where it sits on the grid (bit 0: first grid row, 1: last grid row,
  // 2: first column, 3: last column, 4: past the rows); tap t is out of the grid where the row has a bit of
  // tapmask(t), and reads at the sentinel xbytes
  unsigned base[UA], edge[UA];
#pragma unroll
  for (int u = 0; u < UA; ++u) {
    const int64_t row = m0 + ((tid + TH * u) >> 2);
    const Site st = site_of(row < rows ? row : 0, L);
    base[u] = (unsigned)((row < rows ? row : 0) * CIN * 2);
    edge[u] = (st.r == 0 ? 1u : 0u) | (st.r == L - 1 ? 2u : 0u) | (st.c == 0 ? 4u : 0u) | (st.c == L - 1 ? 8u : 0u) |
              (row < rows ? 0u : 16u);
  }
  const int lrow = L * CIN * 2;   // bytes of one grid row
  auto tap_at = [&](const int u, const int t) -> unsigned {
    const unsigned mask = 16u | (t / 3 == 0 ? 1u : 0u) | (t / 3 == 2 ? 2u : 0u) | (t % 3 == 0 ? 4u : 0u) |
                          (t % 3 == 2 ? 8u : 0u);
    const int delta = (t / 3 - 1) * lrow + (t % 3 - 1) * CIN * 2;
    return (edge[u] & mask) ? xbytes : base[u] + (unsigned)delta;
  };
  auto loadA = [&](const int s, u32x4 (&ra)[UA]) {
#pragma unroll
    for (int u = 0; u < UA; ++u) {
      unsigned o;
      int ch;
      if constexpr (CIN >= KS) {   // a stage lies inside one tap
        o = tap_at(u, (KS * s) / CIN);
        ch = (KS * s) % CIN + 8 * ag;
      } else {                     // CIN = 16: a stage spans taps t0 and t0 + 1 (t0 + 1 may be the padding)
        const int t0 = (KS * s) / CIN;
        o = (ag >> 1) ? (t0 + 1 < 9 ? tap_at(u, t0 + 1) : xbytes) : (t0 < 9 ? tap_at(u, t0) : xbytes);
        ch = 8 * (ag & 1);
      }
      ra[u] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(xr, (int)(o + 2 * ch), 0, 0));
    }
  };
  auto loadB = [&](const int s, u32x4 (&rb)[UB]) {
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      // past the NT x 4 chunks the load repeats the last one (not stored): no branch around the load
      const int q = min(tid + TH * u, NT * 4 - 1);
      rb[u] = *(const u32x4*)(Wt + (int64_t)(q >> 2) * KP + KS * s + 8 * (q & 3));
    }
  };
  auto store = [&](const int buf, const u32x4 (&ra)[UA], const u32x4 (&rb)[UB]) {
    unsigned short* As = lds + buf * STAGE;
    unsigned short* Bs = As + MT * KS;
#pragma unroll
    for (int u = 0; u < UA; ++u) *(u32x4*)&As[swz((tid + TH * u) >> 2, ag)] = ra[u];
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      const int q = tid + TH * u;
      if ((NT * 4) % TH == 0 || q < NT * 4) *(u32x4*)&Bs[swz(q >> 2, q & 3)] = rb[u];
    }
  };
  f4 acc[4][NJ];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) acc[i][j] = f4{0.0f, 0.0f, 0.0f, 0.0f};
  // two register sets: the loads of stage s + 2 are issued while stage s is multiplied, and stored to LDS
  // at the end of stage s + 1
  u32x4 ra0[UA], rb0[UB], ra1[UA], rb1[UB];
  loadA(0, ra0);
  loadB(0, rb0);
  store(0, ra0, rb0);
  if (NS > 1) {
    loadA(1, ra1);
    loadB(1, rb1);
  }
  __syncthreads();
  const int fr = lane & 15, fc = lane >> 4;
  // one stage: multiply the LDS buffer s % 2 while the loads of stage s + 2 go into the register set that
  // stage s + 1 no longer needs; the register sets are named, not indexed, so they stay in registers
  auto stage = [&](const int s, u32x4 (&ra_next)[UA], u32x4 (&rb_next)[UB], const u32x4 (&ra_due)[UA],
                   const u32x4 (&rb_due)[UB]) {
    if (s + 2 < NS) {
      loadA(s + 2, ra_next);
      loadB(s + 2, rb_next);
    }
    const unsigned short* As = lds + (s & 1) * STAGE;
    const unsigned short* Bs = As + MT * KS;
    bf8 a[4], b[NJ];
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = *(const bf8*)&As[swz(wm + 16 * i + fr, fc)];
#pragma unroll
    for (int j = 0; j < NJ; ++j) b[j] = *(const bf8*)&Bs[swz(wn + 16 * j + fr, fc)];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    if (s + 1 < NS) store((s + 1) & 1, ra_due, rb_due);
    __syncthreads();
  };
  // stage s (even) refills set 0 and stores set 1; stage s + 1 the reverse
#pragma unroll
  for (int s = 0; s < NS; s += 2) {
    stage(s, ra0, rb0, ra1, rb1);
    if (s + 1 < NS) stage(s + 1, ra1, rb1, ra0, rb0);
  }
  // epilogue: bias, activation; lane l holds rows 4 (l / 16) .. +3 of column l % 16 of every block
  const bool full = m0 + MT <= rows;
  if constexpr (OUT_BF) {
    // BF16 tile [MT][NT] in LDS (the stage buffers are free), then 16-byte rows out
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int col = wn + 16 * j + fr;
      const float bc = bias[col];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float v[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          v[r] = acc[i][j][r] + bc;
          if (RELU) v[r] = fmaxf(v[r], 0.0f);
        }
        // two values per v_cvt_pk_bf16_f32 (round to nearest even), the pair taken as one 32-bit word: single
        // elements of a BF16 vector are not extracted (the compiler mishandles that form)
        const unsigned p01 = __builtin_bit_cast(unsigned, __builtin_convertvector((fl2){v[0], v[1]}, bf2));
        const unsigned p23 = __builtin_bit_cast(unsigned, __builtin_convertvector((fl2){v[2], v[3]}, bf2));
        const int row = wm + 16 * i + 4 * fc;
        lds[(row + 0) * NT + col] = (unsigned short)(p01 & 0xFFFFu);
        lds[(row + 1) * NT + col] = (unsigned short)(p01 >> 16);
        lds[(row + 2) * NT + col] = (unsigned short)(p23 & 0xFFFFu);
        lds[(row + 3) * NT + col] = (unsigned short)(p23 >> 16);
      }
    }
    __syncthreads();
    constexpr int CPR = NT / 8;   // 16-byte chunks per row
#pragma unroll
    for (int q = tid; q < MT * CPR; q += TH) {
      const int row = q / CPR, c8 = q - row * CPR;
      if (full || m0 + row < rows)
        *(uint4*)((unsigned short*)Y + (m0 + row) * NT + 8 * c8) = *(const uint4*)&lds[row * NT + 8 * c8];
    }
  } else {
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int col = wn + 16 * j + fr;
      const float bc = bias[col];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t row = m0 + wm + 16 * i + 4 * fc + r;
          float v = acc[i][j][r] + bc;
          if (RELU) v = fmaxf(v, 0.0f);
          if (full || row < rows) ((float*)Y)[row * NT + col] = v;
        }
    }
  }
}

// The same convolution from a haloed input tile: the MT output rows of a workgroup read their 3 x 3
// neighbourhoods from the contiguous input rows m0 - L - 1 .. m0 + MT + L, which are staged in LDS once per
// chunk of up to 32 channels (HALO_ROWS rows, each padded by 16 bytes so that 16 consecutive rows fall on
// distinct banks) instead of being gathered nine times. With CIN >= 32, K runs chunk by chunk and, inside a
// chunk, tap by tap (one 32-deep step each); with CIN = 16 a step holds two taps (lanes 0-31 the first, 32-63
// the second; the tenth tap is the weights' zero padding). A tap's activation fragments are the halo rows
// shifted by dr L + dc, and a row whose tap leaves the grid reads a zero row instead. The weight stages and
// their register sets are those of the gather kernel; here the weights are the MFMA's first operand, so each
// lane ends with four consecutive output channels of one site. Four waves, each 64 rows x NT; 256 rows per
// workgroup, so that every weight stage and halo row loaded serves twice the outputs of a 128-row tile (the
// composed layer 8.8 % faster, the first layer 7 %, the second unchanged: its 256 registers then spill a few).
// Needs 2 L + 2 <= HALO_ROWS - HALO_MT (L <= 49, d <= 25); larger grids take the gather kernel.
constexpr int HALO_MT = 256, HALO_ROWS = HALO_MT + 100;   // rows per tile, halo rows

template <int CIN, int NT, int RELU, bool OUT_BF, int PN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void conv_halo_bf16(int L, int64_t rows, const unsigned short* __restrict__ X,
                                                       const unsigned short* __restrict__ Wt,
                                                       const float* __restrict__ bias, void* __restrict__ Y) {
  constexpr int KS = CONV_KS, KP = kpad(CIN);                // k per step, weight row
  constexpr int CH = CIN < KS ? CIN : KS, NC = CIN / CH;     // channels per chunk, chunks
  constexpr int NS = CIN < KS ? KP / KS : 9 * NC;            // steps
  constexpr int RE = CH + 8, RP = CH / 8;                    // elements and 16-byte pieces per halo row
  constexpr int TH = 256, MT = HALO_MT, MI = MT / 64, NJ = NT / 16;   // 16-row and 16-channel blocks per wave
  constexpr int UB = (NT * 4 + TH - 1) / TH;                 // 16-byte weight chunks per thread and step
  constexpr int UH = (HALO_ROWS * RP + TH - 1) / TH;         // 16-byte halo pieces per thread and chunk
  constexpr int NH = NC > 1 ? 2 : 1, HALO = HALO_ROWS * RE;  // halo buffers, elements of one
  constexpr int BST = NT * KS;                               // elements of one weight stage
  constexpr int TILE = OUT_BF ? MT * (NT + 16) : 0;          // BF16 output tile (padded rows)
  constexpr int MAIN = NH * HALO + 2 * BST + 32;             // halo buffers, two weight stages, a zero row
  static_assert((CIN == 16 || CIN % 32 == 0) && NT % 16 == 0 && NT <= 128, "tile shape");
  __shared__ __align__(16) unsigned short lds[MAIN > TILE ? MAIN : TILE];
  unsigned short* const Bsm = lds + NH * HALO;
  unsigned short* const zrow = Bsm + 2 * BST;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  // workgroups are dealt to the eight XCDs in turn; tile b / 8 of XCD b % 8 is made consecutive with the
  // XCD's previous tile, so the halo rows that neighbouring tiles share are found in that XCD's L2
  const unsigned nb = gridDim.x, per = nb / 8, bid = blockIdx.x;
  const unsigned tile = bid < 8 * per ? (bid % 8) * per + bid / 8 : bid;
  const int64_t m0 = (int64_t)tile * MT;
  const int wm = w * (MT / 4);   // the wave's first row
  const int fr = lane & 15, fc = lane >> 4;
  const unsigned xbytes = (unsigned)(rows * CIN * 2);   // the host keeps this + 512 below 2^32
  const __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc((void*)X, (short)0, (int)xbytes, 0x00020000);
  const int hr = MT + 2 * L + 2;                         // halo rows in use
  // (rows < 2^31: 32-bit row arithmetic)
  const int g0 = (int)m0 - L - 1;                        // input row of halo row 0
  // halo pieces of this thread: row h = p / RP, 16-byte group p % RP; byte offset of channel 0 of the group
  // (chunk c adds 2 CH c), xbytes for rows outside the input or the halo
  unsigned hoff[UH];
#pragma unroll
  for (int u = 0; u < UH; ++u) {
    const int p = tid + TH * u, h = p / RP, g = g0 + h;
    hoff[u] = (h < hr && g >= 0 && (int64_t)g < rows) ? (unsigned)g * (2u * CIN) + 16u * (p % RP) : xbytes;
  }
  // A fragment rows of this lane (i = 0..3): halo element offset of the unshifted row and its 8 channels, and
  // where the row sits on the grid (bit 0: first grid row, 1: last grid row, 2: first column, 3: last column;
  // bit 4 always set: the padding tap reads the zero row for every row). The row's place in its job's grid
  // comes from the tile's (uniform) and small quotients by L^2 and by L per lane: x < L^2 + MT, so the FP32
  // quotient is off by at most one, which the remainder tests correct.
  const int LL = L * L;
  const int rem0 = (int)((unsigned)m0 % (unsigned)LL);
  const float rl = 1.0f / (float)L, rll = 1.0f / (float)LL;
  auto quot = [](const int x, const int n, const float rn, int& rem) {
    int q = (int)((float)x * rn);
    rem = x - q * n;
    if (rem >= n) {
      ++q;
      rem -= n;
    } else if (rem < 0) {
      --q;
      rem += n;
    }
    return q;
  };
  int abase[MI];
  unsigned edge[MI];
#pragma unroll
  for (int i = 0; i < MI; ++i) {
    const int r = wm + 16 * i + fr;
    abase[i] = (r + L + 1) * RE + 8 * (CIN < KS ? (fc & 1) : fc);
    int site, col;
    quot(rem0 + r, LL, rll, site);
    const int gr = quot(site, L, rl, col);
    edge[i] = 16u | (gr == 0 ? 1u : 0u) | (gr == L - 1 ? 2u : 0u) | (col == 0 ? 4u : 0u) | (col == L - 1 ? 8u : 0u);
  }
  auto loadH = [&](const int c, u32x4 (&rh)[UH]) {
#pragma unroll
    for (int u = 0; u < UH; ++u)
      rh[u] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(xr, (int)(hoff[u] + 2 * CH * c), 0, 0));
  };
  auto storeH = [&](const int buf, const u32x4 (&rh)[UH]) {
#pragma unroll
    for (int u = 0; u < UH; ++u) {
      const int p = tid + TH * u, h = p / RP;
      if ((UH * TH <= HALO_ROWS * RP) || h < HALO_ROWS) *(u32x4*)&lds[buf * HALO + h * RE + 8 * (p % RP)] = rh[u];
    }
  };
  auto loadB = [&](const int s, u32x4 (&rb)[UB]) {
    // step s: tap s % 9, channels 32 (s / 9) .. (CIN >= 32), or taps 2 s, 2 s + 1 (CIN = 16)
    const int k0 = CIN < KS ? KS * s : (s % 9) * CIN + KS * (s / 9);
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      const int q = min(tid + TH * u, NT * 4 - 1);   // past the NT x 4 chunks: the last one again, not stored
      rb[u] = *(const u32x4*)(Wt + (int64_t)(q >> 2) * KP + k0 + 8 * (q & 3));
    }
  };
  auto storeB = [&](const int buf, const u32x4 (&rb)[UB]) {
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      const int q = tid + TH * u;
      if ((NT * 4) % TH == 0 || q < NT * 4) *(u32x4*)&Bsm[buf * BST + swz(q >> 2, q & 3)] = rb[u];
    }
  };
  f4 acc[MI][NJ];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) acc[i][j] = f4{0.0f, 0.0f, 0.0f, 0.0f};
  u32x4 rh[UH], rb0[UB], rb1[UB];
  loadH(0, rh);
  loadB(0, rb0);
  storeH(0, rh);
  storeB(0, rb0);
  loadB(1, rb1);
  if (tid < 4) *(u32x4*)&zrow[8 * tid] = (u32x4){0u, 0u, 0u, 0u};
  __syncthreads();
  // step s: chunk c = s / 9, tap t = s % 9; the weights of step s + 2 load into the set step s + 1 does not
  // need; the next chunk's halo loads at its first tap and goes to LDS after its third
  // edge bits across which tap t leaves the grid (bit 4 for the padding tap 9), and the tap's row shift
  auto off_grid = [](const int t) -> unsigned {
    return t > 8 ? 16u
                 : (t / 3 == 0 ? 1u : 0u) | (t / 3 == 2 ? 2u : 0u) | (t % 3 == 0 ? 4u : 0u) | (t % 3 == 2 ? 8u : 0u);
  };
  auto shift = [&](const int t) { return t > 8 ? 0 : ((t / 3 - 1) * L + (t % 3 - 1)) * RE; };
  auto step = [&](const int s, u32x4 (&rb_next)[UB], const u32x4 (&rb_due)[UB]) {
    const int c = CIN < KS ? 0 : s / 9, t = CIN < KS ? 2 * s : s % 9;
    if (s + 2 < NS) loadB(s + 2, rb_next);
    if (t == 0 && c + 1 < NC) loadH(c + 1, rh);
    const unsigned short* Hs = lds + (c & 1) * HALO;
    // the fragment addresses are formed anew each step: kept from the step two chunks back (same buffer, same
    // tap) they would hold 72 registers for the whole kernel
#pragma unroll
    for (int i = 0; i < MI; ++i) asm volatile("" : "+v"(abase[i]), "+v"(edge[i]));
    // this lane's tap: t, or with CIN = 16 t + 1 for lanes 32-63
    const bool second = CIN < KS && fc >= 2;
    const int sh = second ? shift(t + 1) : shift(t);
    const unsigned og = second ? off_grid(t + 1) : off_grid(t);
    const unsigned short* Bs = Bsm + (s & 1) * BST;
    bf8 a[MI], b[NJ];
#pragma unroll
    for (int i = 0; i < MI; ++i) {
      const unsigned short* pa = (edge[i] & og) ? zrow + 8 * fc : Hs + abase[i] + sh;
      a[i] = *(const bf8*)pa;
    }
#pragma unroll
    for (int j = 0; j < NJ; ++j) b[j] = *(const bf8*)&Bs[swz(16 * j + fr, fc)];
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[j], a[i], acc[i][j], 0, 0, 0);
    if (t == 2 && c + 1 < NC) storeH((c + 1) & 1, rh);
    if (s + 1 < NS) storeB((s + 1) & 1, rb_due);
    __syncthreads();
  };
#pragma unroll
  for (int s = 0; s < NS; s += 2) {
    step(s, rb0, rb1);
    if (s + 1 < NS) step(s + 1, rb1, rb0);
  }
  // epilogue: bias, activation. The weights are the MFMA's first operand, so lane l holds output channels
  // 4 (l / 16) .. +3 of site l % 16 of every 16 x 16 block: four consecutive values of one output row.
  const bool full = m0 + MT <= rows;
  if constexpr (OUT_BF) {
    // BF16 tile [MT][NT + 16] in LDS (rows padded by 32 bytes against bank conflicts of the 8-byte writes),
    // then 16-byte rows out
    constexpr int TS = NT + 16, CPR = NT / 8;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int ch = 16 * j + 4 * fc;
      const float b0 = bias[ch], b1 = bias[ch + 1], b2 = bias[ch + 2], b3 = bias[ch + 3];
#pragma unroll
      for (int i = 0; i < MI; ++i) {
        float v0 = acc[i][j][0] + b0, v1 = acc[i][j][1] + b1, v2 = acc[i][j][2] + b2, v3 = acc[i][j][3] + b3;
        if (RELU) {
          v0 = fmaxf(v0, 0.0f);
          v1 = fmaxf(v1, 0.0f);
          v2 = fmaxf(v2, 0.0f);
          v3 = fmaxf(v3, 0.0f);
        }
        // two values per v_cvt_pk_bf16_f32 (round to nearest even), each pair taken as one 32-bit word
        const unsigned p01 = __builtin_bit_cast(unsigned, __builtin_convertvector((fl2){v0, v1}, bf2));
        const unsigned p23 = __builtin_bit_cast(unsigned, __builtin_convertvector((fl2){v2, v3}, bf2));
        *(uint2*)&lds[(wm + 16 * i + fr) * TS + ch] = uint2{p01, p23};
      }
    }
    __syncthreads();
    // (kept as a loop: unrolled, its addresses raise the register pressure of the whole kernel)
    for (int q = tid; q < MT * CPR; q += TH) {
      const int row = q / CPR, c8 = q - row * CPR;
      if (full || m0 + row < rows)
        *(uint4*)((unsigned short*)Y + (m0 + row) * NT + 8 * c8) = *(const uint4*)&lds[row * TS + 8 * c8];
    }
  } else {
    // FP32: four consecutive channels are one 16-byte store. PN > 0: the channels are the head's per-site
    // projections, PN per direction (4 PN <= NT, PN a multiple of 4); they are stored direction by direction,
    // [4][rows][PN], so that a message reads the PN values of a site from one short run, and the padding
    // channels beyond 4 PN are not stored.
    static_assert(PN == 0 || (PN % 4 == 0 && 4 * PN <= NT), "projection layout");
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int ch = 16 * j + 4 * fc;
      if (PN > 0 && ch >= 4 * PN) continue;
      const float b0 = bias[ch], b1 = bias[ch + 1], b2 = bias[ch + 2], b3 = bias[ch + 3];
      constexpr int PD = PN > 0 ? PN : 1;   // projections per direction (PN = 0: the plain layout, unused)
      const int dir = ch / PD, cd = ch - dir * PD;
#pragma unroll
      for (int i = 0; i < MI; ++i) {
        const int64_t row = m0 + wm + 16 * i + fr;
        float4 v{acc[i][j][0] + b0, acc[i][j][1] + b1, acc[i][j][2] + b2, acc[i][j][3] + b3};
        if (RELU) {
          v.x = fmaxf(v.x, 0.0f);
          v.y = fmaxf(v.y, 0.0f);
          v.z = fmaxf(v.z, 0.0f);
          v.w = fmaxf(v.w, 0.0f);
        }
        float* dst = PN > 0 ? (float*)Y + (dir * rows + row) * PN + cd : (float*)Y + row * NT + ch;
        if (full || row < rows) *(float4*)dst = v;
      }
    }
  }
}

// db[c] = sum over rows of dY[row][c]; one workgroup per channel
__global__ __launch_bounds__(256) void colsum_kernel(const float* __restrict__ dY, int64_t rows, int C,
                                                     float* __restrict__ db) {
  __shared__ float red[4];
  const int c = blockIdx.x;
  float acc = 0.0f;
  for (int64_t r = threadIdx.x; r < rows; r += 256) acc += dY[r * C + c];
  acc = wsum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) db[c] = red[0] + red[1] + red[2] + red[3];
}

// Message head: one wavefront per (job, message). Leg table per message: [K, direction, a_0..a_5, b_0..b_5]
// (sites r*L + c). TRAIN: loss, d(head outputs) into `dout` [job][M][32], and d(features) into dF (atomic);
// otherwise the predicted unit message into msgs [job][M][64] (zero beyond 2^K).
template <bool TRAIN>
__global__ __launch_bounds__(64) void head_kernel(const float* __restrict__ F, const int32_t* __restrict__ legs,
                                                  int M, int L, int64_t jobs, const float* __restrict__ prm,
                                                  const float* __restrict__ targets, const uint8_t* __restrict__ use,
                                                  float inv_n, float* __restrict__ msgs, float* __restrict__ dout,
                                                  float* __restrict__ dF, float* __restrict__ loss) {
  const int64_t job = blockIdx.x / M;
  const int e = (int)(blockIdx.x - job * M), lane = threadIdx.x;
  if (job >= jobs) return;
  if (TRAIN && !use[job]) return;
  const int32_t* lg = legs + e * 14;
  const int K = lg[0], dir = lg[1];
  const float* H = prm + OFF.head + (size_t)dir * HEAD;
  const float *Wu = H, *bu = H + 2 * C3 * 2, *Wp = bu + 2, *bp = Wp + 4 * C3 * 4;
  const float* Fj = F + job * (int64_t)L * L * C3;
  // feature of input index k of leg i: [F(a_i), F(b_i)]
  auto feat = [&](int i, int k) -> float {
    const int site = (k < C3) ? lg[2 + i] : lg[2 + MAXK + i];
    return Fj[(int64_t)site * C3 + (k < C3 ? k : k - C3)];
  };
  float out[NOUT];
  for (int o = 0; o < NOUT; ++o) out[o] = 0.0f;
  // unary outputs: o = 2 i + c
  for (int i = 0; i < MAXK; ++i) {
    if (i >= K) break;
    float a0 = 0.0f, a1 = 0.0f;
    for (int k = lane; k < 2 * C3; k += 64) {
      const float f = feat(i, k);
      a0 += f * Wu[k * 2 + 0];
      a1 += f * Wu[k * 2 + 1];
    }
    out[2 * i] = wsum(a0) + bu[0];
    out[2 * i + 1] = wsum(a1) + bu[1];
  }
  // pairwise outputs: o = 2 MAXK + 4 i + q
  for (int i = 0; i < MAXK - 1; ++i) {
    if (i >= K - 1) break;
    float a[4] = {0, 0, 0, 0};
    for (int k = lane; k < 4 * C3; k += 64) {
      const float f = (k < 2 * C3) ? feat(i, k) : feat(i + 1, k - 2 * C3);
      for (int q = 0; q < 4; ++q) a[q] += f * Wp[k * 4 + q];
    }
    for (int q = 0; q < 4; ++q) out[2 * MAXK + 4 * i + q] = wsum(a[q]) + bp[q];
  }
  // scores of the lane's configuration b
  const int b = lane, nb = 1 << K;
  const bool valid = b < nb;
  float s = 0.0f;
  for (int i = 0; i < MAXK; ++i) {
    if (i >= K) break;
    const int bi = (b >> (K - 1 - i)) & 1;
    s += bi ? out[2 * i + 1] : out[2 * i];
    if (i < K - 1) {
      const int bn = (b >> (K - 2 - i)) & 1, q = 2 * bi + bn;
      const float* P = out + 2 * MAXK + 4 * i;
      s += (q == 0) ? P[0] : (q == 1) ? P[1] : (q == 2) ? P[2] : P[3];
    }
  }
  const float mx = wmax(valid ? s : -INFINITY);
  const float m = valid ? expf(s - mx) : 0.0f;
  const float nrm = sqrtf(wsum(m * m));
  const float mh = m / nrm;
  if (!TRAIN) {
    msgs[(job * M + e) * 64 + lane] = mh;
    return;
  }
  // KL(q || softmax(s)) with q = t / sum(t): the gradient in s is softmax(s) - q
  const float t = valid ? fmaxf(targets[(job * M + e) * 64 + lane], 0.0f) : 0.0f;
  const float q = t / wsum(t);
  const float zs = wsum(m);
  const float pm = m / zs;
  const float kl = wsum(q > 0.0f ? q * (logf(q) - (s - mx - logf(zs))) : 0.0f);
  if (lane == 0) loss[job * M + e] = kl * inv_n;
  const float gs = valid ? (pm - q) * inv_n : 0.0f;
  // d(outputs)
  float dO[NOUT];
  for (int o = 0; o < NOUT; ++o) dO[o] = 0.0f;
  for (int i = 0; i < MAXK; ++i) {
    if (i >= K) break;
    const int bi = (b >> (K - 1 - i)) & 1;
    dO[2 * i] = wsum(bi ? 0.0f : gs);
    dO[2 * i + 1] = wsum(bi ? gs : 0.0f);
    if (i < K - 1) {
      const int bn = (b >> (K - 2 - i)) & 1, q = 2 * bi + bn;
      for (int qq = 0; qq < 4; ++qq) dO[2 * MAXK + 4 * i + qq] = wsum(q == qq ? gs : 0.0f);
    }
  }
  if (lane < NOUT) {
    float v = 0.0f;
    for (int o = 0; o < NOUT; ++o) v = (lane == o) ? dO[o] : v;
    dout[(job * M + e) * NOUT + lane] = v;
  }
  // d(features): leg i's input vector gets Wu du_i + Wp[0:2C3] dP_i + Wp[2C3:4C3] dP_{i-1}
  float* dFj = dF + job * (int64_t)L * L * C3;
  for (int i = 0; i < MAXK; ++i) {
    if (i >= K) break;
    for (int k = lane; k < 2 * C3; k += 64) {
      float g = Wu[k * 2] * dO[2 * i] + Wu[k * 2 + 1] * dO[2 * i + 1];
      if (i < K - 1)
        for (int q = 0; q < 4; ++q) g += Wp[k * 4 + q] * dO[2 * MAXK + 4 * i + q];
      if (i > 0)
        for (int q = 0; q < 4; ++q) g += Wp[(2 * C3 + k) * 4 + q] * dO[2 * MAXK + 4 * (i - 1) + q];
      const int site = (k < C3) ? lg[2 + i] : lg[2 + MAXK + i];
      atomicAdd(&dFj[(int64_t)site * C3 + (k < C3 ? k : k - C3)], g);
    }
  }
}

// Inference head over projections. The head is linear in the features up to its scores, so for BF16
// inference the last convolution and the head's weights are composed: per direction (20 columns each),
// the features of a site projected on Wu[0:C3] (2), Wu[C3:2C3] (2), Wp[0:C3] (4), Wp[C3:2C3] (4),
// Wp[2C3:3C3] (4) and Wp[3C3:4C3] (4) -- the parts that a site contributes as a_i, b_i, a_{i+1} or
// b_{i+1} of a message. The composed layer computes those 80 projections per site directly (W3 Hc, bias
// b3 Hc), and a message's unary and pairwise outputs are sums of a few of them.
constexpr int NPROJ = 20;                  // projections per direction
constexpr int PROJ_CH = 96;                // composed layer's output channels: 4 x 20, padded to a multiple of 32

// column o of the composed head matrix Hc, entry for feature channel c (o < 4 NPROJ)
__device__ __forceinline__ float head_col(const float* prm, int o, int c) {
  const int dir = o / NPROJ, j = o - dir * NPROJ;
  const float* H = prm + OFF.head + (size_t)dir * HEAD;
  const float *Wu = H, *Wp = H + 2 * C3 * 2 + 2;
  if (j < 4) return Wu[((j >> 1) * C3 + c) * 2 + (j & 1)];
  const int q = (j - 4) & 3, part = (j - 4) >> 2;
  return Wp[(part * C3 + c) * 4 + q];
}

// Wt[o][kp] = bf16(sum_c W3[kp][c] Hc[c][o]) for o < 4 NPROJ, 0 for the padding columns; bc[o] = b3 . Hc[:, o]
__global__ void compose_head_kernel(const float* __restrict__ prm, int kpad, unsigned short* __restrict__ Wt,
                                    float* __restrict__ bc) {
  const int64_t n = (int64_t)PROJ_CH * kpad;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int o = (int)(i / kpad), kp = (int)(i - (int64_t)o * kpad);
    float v = 0.0f;
    if (o < 4 * NPROJ && kp < 9 * C2)
      for (int c = 0; c < C3; ++c) v += prm[OFF.w3 + (size_t)kp * C3 + c] * head_col(prm, o, c);
    Wt[i] = f2bf(v);
    if (kp == 0) {
      float b = 0.0f;
      if (o < 4 * NPROJ)
        for (int c = 0; c < C3; ++c) b += prm[OFF.b3 + c] * head_col(prm, o, c);
      bc[o] = b;
    }
  }
}

// one wavefront per (job, message): lanes 0 .. 2K+4(K-1)-1 form the head outputs from the projections of the
// legs' sites, every lane then scores its configuration b as head_kernel does
// Pj: projection j < NPROJ of direction dir at grid row g (= job L^2 + site) at Pj[dir dstride + g sstride + j]
__global__ __launch_bounds__(64) void head_proj_kernel(const float* __restrict__ Pj, int64_t dstride, int sstride,
                                                       const int32_t* __restrict__ legs, int M, int L, int64_t jobs,
                                                       const float* __restrict__ prm, float* __restrict__ msgs) {
  // the NPROJ projections of every leg site (a_0 .. a_{K-1}, then b_0 .. b_{K-1}), each a contiguous run of
  // five 16-byte pieces, loaded by one lane per piece into LDS: one load instruction per wave instead of
  // two to four dependent 4-byte gathers per lane
  static_assert(NPROJ == 20, "five 16-byte pieces per site");
  __shared__ float4 sp4[2 * MAXK * 5];
  const int64_t job = blockIdx.x / M;
  const int e = (int)(blockIdx.x - job * M), lane = threadIdx.x;
  if (job >= jobs) return;
  const int32_t* lg = legs + e * 14;
  const int K = lg[0], dir = lg[1];
  const float* H = prm + OFF.head + (size_t)dir * HEAD;
  const float *bu = H + 2 * C3 * 2, *bp = bu + 2 + 4 * C3 * 4;
  const float* P = Pj + dir * dstride + job * (int64_t)L * L * sstride;
  if (lane < 2 * K * 5) {
    const int m = lane / 5, part = lane - 5 * m;
    const int site = m < K ? lg[2 + m] : lg[2 + MAXK + m - K];
    sp4[lane] = *(const float4*)(P + (int64_t)site * sstride + 4 * part);
  }
  __syncthreads();
  const float* sp = (const float*)sp4;
  auto pa = [&](int i, int j) { return sp[i * NPROJ + j]; };         // leg site a_i
  auto pb = [&](int i, int j) { return sp[(K + i) * NPROJ + j]; };   // leg site b_i
  // output o = lane: unary 2 i + c, pairwise 2 MAXK + 4 i + q (as head_kernel)
  float outv = 0.0f;
  if (lane < 2 * MAXK) {
    const int i = lane >> 1, c = lane & 1;
    if (i < K) outv = pa(i, c) + pb(i, 2 + c) + bu[c];
  } else if (lane < NOUT) {
    const int i = (lane - 2 * MAXK) >> 2, q = (lane - 2 * MAXK) & 3;
    if (i < K - 1) outv = pa(i, 4 + q) + pb(i, 8 + q) + pa(i + 1, 12 + q) + pb(i + 1, 16 + q) + bp[q];
  }
  const int b = lane, nb = 1 << K;
  const bool valid = b < nb;
  float s = 0.0f;
  for (int i = 0; i < MAXK; ++i) {
    if (i >= K) break;
    const int bi = (b >> (K - 1 - i)) & 1;
    s += __shfl(outv, 2 * i + bi);
    if (i < K - 1) {
      const int bn = (b >> (K - 2 - i)) & 1;
      s += __shfl(outv, 2 * MAXK + 4 * i + 2 * bi + bn);
    }
  }
  const float mx = wmax(valid ? s : -INFINITY);
  const float m = valid ? expf(s - mx) : 0.0f;
  const float nrm = sqrtf(wsum(m * m));
  msgs[(job * M + e) * 64 + lane] = m / nrm;
}

// Head weight gradients: workgroup (direction, slice of 64 input rows of Wu (3 slices) or Wp (6 slices));
// thread = input row k; sums f_i[k] d(output) over every trained job and every message of the direction.
__global__ __launch_bounds__(64) void head_grad_kernel(const float* __restrict__ F, const int32_t* __restrict__ legs,
                                                       int M, int L, int64_t jobs, const uint8_t* __restrict__ use,
                                                       const float* __restrict__ dout, float* __restrict__ grad) {
  const int dir = blockIdx.x / 9, slice = blockIdx.x % 9, lane = threadIdx.x;
  const bool pair = slice >= 3;
  const int k = (pair ? slice - 3 : slice) * 64 + lane;
  float* G = grad + OFF.head + (size_t)dir * HEAD;
  float acc[4] = {0, 0, 0, 0};
  float bacc[4] = {0, 0, 0, 0};
  for (int64_t job = 0; job < jobs; ++job) {
    if (!use[job]) continue;
    const float* Fj = F + job * (int64_t)L * L * C3;
    for (int e = 0; e < M; ++e) {
      const int32_t* lg = legs + e * 14;
      if (lg[1] != dir) continue;
      const int K = lg[0];
      const float* dO = dout + (job * M + e) * NOUT;
      auto feat = [&](int i, int kk) -> float {
        const int site = (kk < C3) ? lg[2 + i] : lg[2 + MAXK + i];
        return Fj[(int64_t)site * C3 + (kk < C3 ? kk : kk - C3)];
      };
      if (!pair) {
        for (int i = 0; i < K; ++i) {
          const float f = feat(i, k);
          acc[0] += f * dO[2 * i];
          acc[1] += f * dO[2 * i + 1];
          bacc[0] += dO[2 * i];
          bacc[1] += dO[2 * i + 1];
        }
      } else {
        for (int i = 0; i + 1 < K; ++i) {
          const float f = (k < 2 * C3) ? feat(i, k) : feat(i + 1, k - 2 * C3);
          for (int q = 0; q < 4; ++q) {
            acc[q] += f * dO[2 * MAXK + 4 * i + q];
            bacc[q] += dO[2 * MAXK + 4 * i + q];
          }
        }
      }
    }
  }
  if (!pair) {
    G[k * 2] = acc[0];
    G[k * 2 + 1] = acc[1];
    if (slice == 0 && lane == 0) {
      G[2 * C3 * 2] = bacc[0];
      G[2 * C3 * 2 + 1] = bacc[1];
    }
  } else {
    float* Wp = G + 2 * C3 * 2 + 2;
    for (int q = 0; q < 4; ++q) Wp[k * 4 + q] = acc[q];
    if (slice == 3 && lane == 0)
      for (int q = 0; q < 4; ++q) Wp[4 * C3 * 4 + q] = bacc[q];
  }
}

__global__ void sum_kernel(const float* __restrict__ x, int64_t n, float* __restrict__ out) {
  __shared__ float red[4];
  float acc = 0.0f;
  for (int64_t i = threadIdx.x; i < n; i += 256) acc += x[i];
  acc = wsum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = red[0] + red[1] + red[2] + red[3];
}

__global__ void adam_kernel(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1,
                            float c2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi, vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// Fallback selection after a warm-started decode: syndromes with a coset whose final distance is at least
// delta1 are listed (order of the list unspecified) for a cold rerun.
// Syndromes the warm run cannot vouch for: a coset whose final distance is not below delta1, or a decided
// coset that was not among the fastest to converge (the right coset converges fastest, Sec. IV; a decided
// coset that took longer than another points to a fixed point that the predicted start led to).
__global__ void fallback_select_kernel(const double* __restrict__ delta, const int32_t* __restrict__ iters,
                                       const uint8_t* __restrict__ coset, int64_t batch, double delta1,
                                       int64_t* __restrict__ list, int64_t* __restrict__ count) {
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < batch; b += (int64_t)gridDim.x * blockDim.x) {
    bool bad = false;
    int fastest = iters[b * 4];
    for (int k = 0; k < 4; ++k) {
      bad |= !(delta[b * 4 + k] < delta1);
      fastest = min(fastest, iters[b * 4 + k]);
    }
    bad |= iters[b * 4 + coset[b]] > fastest;
    if (bad) list[atomicAdd((unsigned long long*)count, 1ull)] = b;
  }
}

// gather the listed syndromes (and their noise rates) into a compact batch
__global__ void fallback_gather_kernel(const uint8_t* __restrict__ syn, const double* __restrict__ pdev, int m,
                                       const int64_t* __restrict__ list, int64_t n, uint8_t* __restrict__ syn_out,
                                       double* __restrict__ p_out) {
  const int64_t i = blockIdx.x;
  if (i >= n) return;
  const int64_t b = list[i];
  for (int k = threadIdx.x; k < m; k += blockDim.x) syn_out[i * m + k] = syn[b * m + k];
  if (pdev && threadIdx.x == 0) p_out[i] = pdev[b];
}

// write the cold results of the listed syndromes back; their iteration counts add the warm run's
__global__ void fallback_scatter_kernel(const int64_t* __restrict__ list, int64_t n, int nq,
                                        const double* __restrict__ ll, const double* __restrict__ dl,
                                        const int32_t* __restrict__ it, const uint8_t* __restrict__ cs,
                                        const uint8_t* __restrict__ cr, double* __restrict__ ll_o,
                                        double* __restrict__ dl_o, int32_t* __restrict__ it_o, uint8_t* __restrict__ cs_o,
                                        uint8_t* __restrict__ cr_o) {
  const int64_t i = blockIdx.x;
  if (i >= n) return;
  const int64_t b = list[i];
  if (threadIdx.x < 4) {
    const int k = threadIdx.x;
    ll_o[b * 4 + k] = ll[i * 4 + k];
    dl_o[b * 4 + k] = dl[i * 4 + k];
    it_o[b * 4 + k] += it[i * 4 + k];
  }
  if (threadIdx.x == 0) cs_o[b] = cs[i];
  for (int k = threadIdx.x; k < nq; k += blockDim.x) cr_o[b * nq + k] = cr[i * nq + k];
}

// ------------------------------------------------------------------------------------------ host side
unsigned grid1(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 65536)); }

struct Legs {
  int32_t* dev = nullptr;
  int M = 0;
};
std::mutex l_mu;
std::map<std::tuple<int, int, int, int, int>, Legs> l_cache;

// leg table of every directed message of the plan (device, cached per (d, blocks, chi, device))
int legs_for(int d, const bbp_opts* o, Legs* out) {
  int dev = 0;
  W_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(l_mu);
  auto key = std::make_tuple(d, o->block_rows, o->block_cols, o->chi, dev);
  auto it = l_cache.find(key);
  if (it != l_cache.end()) {
    *out = it->second;
    return BBP_OK;
  }
  const bbp::Plan& P = bbp::cached_plan(d, o->block_rows, o->block_cols, o->chi);
  const int L = P.L;
  std::vector<int32_t> t((size_t)std::max(P.M, 1) * 14, -1);
  for (int e = 0; e < P.M; ++e) {
    const int src = P.edge_src[e], dir = P.edge_dir[e];
    const int I = src / P.nJ, J = src % P.nJ;
    const int r0 = P.row0[I], c0 = P.col0[J], kr = P.rowsz[I], kc = P.colsz[J];
    const int K = (dir <= 1) ? kr : kc;
    if (K > MAXK) return wfail(BBP_EUNSUPPORTED, "the warm start supports blocks of at most 6");
    int32_t* r = &t[(size_t)e * 14];
    r[0] = K;
    r[1] = dir;
    for (int i = 0; i < K; ++i) {
      int ar, ac, br, bc;
      switch (dir) {
        case 0: ar = r0 + i; ac = c0 + kc - 1; br = ar; bc = ac + 1; break;   // E
        case 1: ar = r0 + i; ac = c0; br = ar; bc = ac - 1; break;            // W
        case 2: ar = r0 + kr - 1; ac = c0 + i; br = ar + 1; bc = ac; break;   // S
        default: ar = r0; ac = c0 + i; br = ar - 1; bc = ac; break;           // N
      }
      r[2 + i] = ar * L + ac;
      r[2 + MAXK + i] = br * L + bc;
    }
  }
  Legs lg;
  lg.M = P.M;
  W_TRY(hipMalloc(&lg.dev, t.size() * sizeof(int32_t)));
  W_TRY(hipMemcpy(lg.dev, t.data(), t.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  l_cache[key] = lg;
  *out = lg;
  return BBP_OK;
}

// BF16 input channels per site (C0 padded to 16) and the transposed, padded BF16 weights: [C1][KP1],
// [C2][KP2], [C3][KP3]
constexpr int CS0 = 16;
#ifndef BBP_CONV_WM
#define BBP_CONV_WM 2
#endif
constexpr int CONV_WM = BBP_CONV_WM;   // waves along M in the BF16 convolutions
constexpr int KP1 = kpad(CS0), KP2 = kpad(C1), KP3 = kpad(C2);
constexpr int64_t WB1 = (int64_t)C1 * KP1, WB2 = (int64_t)C2 * KP2, WB3 = (int64_t)PROJ_CH * KP3;
constexpr int64_t WB_TOTAL = WB1 + WB2 + WB3;
static_assert(CS0 * 2 <= C0 * 4, "BF16 input channels fit the FP32 input slot of the workspace");

// syndromes per forward chunk of bbp_warm_predict (bounds its workspace)
constexpr int64_t PREDICT_CHUNK = 512;

struct WLayout {
  size_t X0, A1, A2, F, Wb, dF, dA2, dA1, dout, loss, total;
};
size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }
WLayout wlayout(int d, int64_t jobs, int M, bool train) {
  const size_t L = 2 * d - 1, rows = (size_t)jobs * L * L;
  WLayout l{};
  size_t o = 0;
  l.X0 = o; o = a256(o + rows * C0 * 4);
  l.A1 = o; o = a256(o + rows * C1 * 4);
  l.A2 = o; o = a256(o + rows * C2 * 4);
  l.F = o; o = a256(o + rows * C3 * 4);
  l.Wb = o; o = a256(o + (size_t)WB_TOTAL * 2 + PROJ_CH * 4);   // BF16 weights (transposed, padded), bias
  if (train) {
    l.dF = o; o = a256(o + rows * C3 * 4);
    l.dA2 = o; o = a256(o + rows * C2 * 4);
    l.dA1 = o; o = a256(o + rows * C1 * 4);
    l.dout = o; o = a256(o + (size_t)jobs * std::max(M, 1) * NOUT * 4);
    l.loss = o; o = a256(o + (size_t)jobs * std::max(M, 1) * 4);
  }
  l.total = o;
  return l;
}

template <int MODE, int EPI>
int conv(int L, int64_t rows, int cin, int cout, const float* X, const float* Bm, float* C, const float* aux,
         hipStream_t st) {
  const int64_t Mdim = (MODE == G_DW) ? 9 * cin : rows;
  const int Ndim = (MODE == G_DX) ? cin : cout;
  const int64_t Kdim = (MODE == G_FWD) ? 9 * cin : (MODE == G_DX) ? 9 * cout : rows;
  int64_t splits = 1;
  if (MODE == G_DW) splits = std::max<int64_t>(1, std::min<int64_t>(512, rows / 2048));
  const int64_t kchunk = ((Kdim + splits - 1) / splits + 15) / 16 * 16;
  const dim3 grid((unsigned)((Mdim + 63) / 64), (unsigned)((Ndim + 63) / 64), (unsigned)((Kdim + kchunk - 1) / kchunk));
  conv_gemm<MODE, EPI><<<grid, dim3(256), 0, st>>>(L, rows, cin, cout, kchunk, X, Bm, C, aux);
  W_TRY(hipGetLastError());
  return BBP_OK;
}

struct Args {
  int d;
  const bbp_opts* opts;
  const uint8_t* syn;
  const double* pdev;
  double p;
  int64_t batch;
  const float* prm;
  void* ws;
  size_t ws_bytes;
  hipStream_t st;
};

// forward trunk of `jobs` coset jobs starting at syndrome syn / noise rates pdev: features F [rows][C3]
// the haloed-tile kernel serves grids whose halo fits its LDS rows
bool halo_fits(int L) { return HALO_MT + 2 * L + 2 <= HALO_ROWS; }

// PN > 0 (the composed last layer): with the haloed-tile kernel the projections are stored direction-major,
// [4][rows][PN]; the gather kernel of larger grids stores them [rows][NT]
template <int CIN, int NT, int WM, int RELU, bool OUT_BF, int PN = 0>
int conv_bf16(int L, int64_t rows, const unsigned short* X, const unsigned short* Wt, const float* bias, void* Y,
              hipStream_t st) {
  // the kernel addresses the activations through one buffer descriptor with 32-bit byte offsets, the
  // out-of-grid sentinel (the buffer's size) plus a channel offset included
  if (rows * CIN > (int64_t)INT32_MAX - 512) return wfail(BBP_EINVAL, "too many sites for one BF16 convolution");
  {
    if (halo_fits(L)) {
      // the haloed-tile kernel computes only the 4 PN projection channels of the composed layer (the weight
      // rows beyond them are the padding of the gather kernel's tile)
      constexpr int NTH = PN > 0 ? 4 * PN : NT;
      conv_halo_bf16<CIN, NTH, RELU, OUT_BF, PN><<<dim3((unsigned)((rows + HALO_MT - 1) / HALO_MT)), dim3(256), 0, st>>>(
          L, rows, X, Wt, bias, Y);
      W_TRY(hipGetLastError());
      return BBP_OK;
    }
  }
  conv_fwd_bf16<CIN, NT, WM, RELU, OUT_BF><<<dim3((unsigned)((rows + 64 * WM - 1) / (64 * WM))), dim3(128 * WM), 0, st>>>(
      L, rows, X, Wt, bias, Y);
  W_TRY(hipGetLastError());
  return BBP_OK;
}

// BF16 copies of the convolution weights into the workspace, transposed to [cout][k] with k padded to a
// multiple of the stage, the last layer composed with the head (done per forward call: about 200k values)
int weights_bf16(const float* prm, const WLayout& w, char* ws, hipStream_t st) {
  unsigned short* Wb = (unsigned short*)(ws + w.Wb);
  weights_t_kernel<<<grid1(WB1), 256, 0, st>>>(prm + OFF.w1, C0, CS0, C1, KP1, Wb);
  weights_t_kernel<<<grid1(WB2), 256, 0, st>>>(prm + OFF.w2, C1, C1, C2, KP2, Wb + WB1);
  compose_head_kernel<<<grid1(WB3), 256, 0, st>>>(prm, KP3, Wb + WB1 + WB2, (float*)(Wb + WB_TOTAL));
  W_TRY(hipGetLastError());
  return BBP_OK;
}

// forward trunk in BF16 storage with FP32 accumulation: input channels, A1 and A2 in BF16; the last layer
// composed with the head gives the projections [rows][PROJ_CH] in FP32 (in the features' slot)
int trunk_bf16(int d, const uint8_t* syn, const double* pdev, double p, int64_t jobs, char* ws, const WLayout& w,
               const float* prm, hipStream_t st) {
  const int L = 2 * d - 1;
  const int64_t rows = jobs * L * L;
  unsigned short *X0 = (unsigned short*)(ws + w.X0), *A1 = (unsigned short*)(ws + w.A1),
                 *A2 = (unsigned short*)(ws + w.A2), *Wb = (unsigned short*)(ws + w.Wb);
  float* F = (float*)(ws + w.F);
  features_kernel<unsigned short, CS0><<<dim3((unsigned)(jobs / 4)), dim3(256), 0, st>>>(syn, pdev, (float)p, d, X0);
  W_TRY(hipGetLastError());
  int rc;
  if ((rc = conv_bf16<CS0, C1, CONV_WM, 1, true>(L, rows, X0, Wb, prm + OFF.b1, A1, st))) return rc;
  if ((rc = conv_bf16<C1, C2, CONV_WM, 1, true>(L, rows, A1, Wb + WB1, prm + OFF.b2, A2, st))) return rc;
  if ((rc = conv_bf16<C2, PROJ_CH, CONV_WM, 0, false, NPROJ>(L, rows, A2, Wb + WB1 + WB2,
                                                              (const float*)(Wb + WB_TOTAL), F, st)))
    return rc;
  return BBP_OK;
}

int trunk(int d, const uint8_t* syn, const double* pdev, double p, int64_t jobs, const float* prm, char* ws,
          const WLayout& w, hipStream_t st) {
  const int L = 2 * d - 1;
  const int64_t rows = jobs * L * L;
  float *X0 = (float*)(ws + w.X0), *A1 = (float*)(ws + w.A1), *A2 = (float*)(ws + w.A2), *F = (float*)(ws + w.F);
  features_kernel<float, C0><<<dim3((unsigned)(jobs / 4)), dim3(256), 0, st>>>(syn, pdev, (float)p, d, X0);
  W_TRY(hipGetLastError());
  int rc;
  if ((rc = conv<G_FWD, 1>(L, rows, C0, C1, X0, prm + OFF.w1, A1, prm + OFF.b1, st))) return rc;
  if ((rc = conv<G_FWD, 1>(L, rows, C1, C2, A1, prm + OFF.w2, A2, prm + OFF.b2, st))) return rc;
  if ((rc = conv<G_FWD, 0>(L, rows, C2, C3, A2, prm + OFF.w3, F, prm + OFF.b3, st))) return rc;
  return BBP_OK;
}

int check_common(const Args& a, Legs* lg) {
  if (!a.opts) return wfail(BBP_EINVAL, "opts is NULL");
  if (a.d < 2 || a.d > 32) return wfail(BBP_EINVAL, "d must be in [2, 32]");
  if (a.opts->block_rows < 1 || a.opts->block_cols < 1 || a.opts->block_rows > MAXK || a.opts->block_cols > MAXK)
    return wfail(BBP_EINVAL, "block sizes must be in [1, 6]");
  if (a.batch < 1) return wfail(BBP_EINVAL, "batch must be >= 1");
  if (a.batch > (int64_t)1 << 24) return wfail(BBP_EINVAL, "batch too large");
  if (!a.syn || !a.prm || !a.ws) return wfail(BBP_EINVAL, "a required pointer is NULL");
  if (!a.pdev && !(a.p > 0.0 && a.p < 1.0)) return wfail(BBP_EINVAL, "p must be in (0, 1)");
  return legs_for(a.d, a.opts, lg);
}

}  // namespace

extern "C" {

const char* bbp_warm_last_error(void) { return w_err.c_str(); }

int bbp_warm_param_count(int64_t* count) {
  if (!count) return wfail(BBP_EINVAL, "count is NULL");
  *count = (int64_t)OFF.total;
  return BBP_OK;
}

int bbp_warm_workspace_size(int32_t d, int64_t batch, const bbp_opts* opts, int32_t train, size_t* bytes) {
  if (!bytes || !opts) return wfail(BBP_EINVAL, "NULL argument");
  if (d < 2 || d > 32 || batch < 1) return wfail(BBP_EINVAL, "invalid d or batch");
  if (opts->block_rows < 1 || opts->block_cols < 1 || opts->block_rows > MAXK || opts->block_cols > MAXK)
    return wfail(BBP_EINVAL, "block sizes must be in [1, 6]");
  const bbp::Plan& P = bbp::cached_plan(d, opts->block_rows, opts->block_cols, opts->chi);
  const int64_t b = train ? batch : std::min(batch, PREDICT_CHUNK);
  *bytes = wlayout(d, 4 * b, P.M, train != 0).total;
  return BBP_OK;
}

int bbp_warm_predict(int32_t d, double p, const double* p_dev, const uint8_t* syndromes_dev, int64_t batch,
                     const bbp_opts* opts, const float* params_dev, int32_t precision, float* messages_dev,
                     void* workspace, size_t workspace_bytes, void* stream) {
  Args a{d, opts, syndromes_dev, p_dev, p, batch, params_dev, workspace, workspace_bytes, (hipStream_t)stream};
  Legs lg;
  int rc = check_common(a, &lg);
  if (rc) return rc;
  if (!messages_dev) return wfail(BBP_EINVAL, "messages_dev is NULL");
  if (precision != 0 && precision != 1) return wfail(BBP_EINVAL, "precision must be 0 (FP32) or 1 (BF16)");
  const int64_t chunk = std::min(batch, PREDICT_CHUNK);
  const WLayout w = wlayout(d, 4 * chunk, lg.M, false);
  if (workspace_bytes < w.total) return wfail(BBP_EINVAL, "workspace too small");
  const int L = 2 * d - 1, m = 2 * d * (d - 1);
  if (precision == 1 && (rc = weights_bf16(params_dev, w, (char*)workspace, a.st))) return rc;
  for (int64_t b0 = 0; b0 < batch; b0 += chunk) {
    const int64_t nb = std::min(chunk, batch - b0), jobs = 4 * nb;
    const uint8_t* sb = syndromes_dev + b0 * m;
    const double* pb = p_dev ? p_dev + b0 : nullptr;
    rc = (precision == 1) ? trunk_bf16(d, sb, pb, p, jobs, (char*)workspace, w, params_dev, a.st)
                          : trunk(d, sb, pb, p, jobs, params_dev, (char*)workspace, w, a.st);
    if (rc) return rc;
    if (lg.M > 0) {
      if (precision == 1) {
        const bool dm = halo_fits(L);   // the layout conv_bf16 stored the projections in
        const int64_t rows = jobs * (int64_t)L * L;
        head_proj_kernel<<<dim3((unsigned)(jobs * lg.M)), dim3(64), 0, a.st>>>(
            (const float*)((char*)workspace + w.F), dm ? rows * NPROJ : (int64_t)NPROJ, dm ? NPROJ : PROJ_CH, lg.dev,
            lg.M, L, jobs, params_dev, messages_dev + b0 * 4 * lg.M * 64);
      } else {
        head_kernel<false><<<dim3((unsigned)(jobs * lg.M)), dim3(64), 0, a.st>>>(
            (const float*)((char*)workspace + w.F), lg.dev, lg.M, L, jobs, params_dev, nullptr, nullptr, 0.0f,
            messages_dev + b0 * 4 * lg.M * 64, nullptr, nullptr, nullptr);
      }
      W_TRY(hipGetLastError());
    }
  }
  return BBP_OK;
}

int bbp_warm_loss_grad(int32_t d, double p, const double* p_dev, const uint8_t* syndromes_dev, int64_t batch,
                       const bbp_opts* opts, const float* params_dev, const float* targets_dev,
                       const uint8_t* use_dev, int64_t trained_messages, float* grad_dev, float* loss_dev,
                       void* workspace, size_t workspace_bytes, void* stream) {
  Args a{d, opts, syndromes_dev, p_dev, p, batch, params_dev, workspace, workspace_bytes, (hipStream_t)stream};
  Legs lg;
  int rc = check_common(a, &lg);
  if (rc) return rc;
  if (!targets_dev || !use_dev || !grad_dev || !loss_dev) return wfail(BBP_EINVAL, "a required pointer is NULL");
  if (trained_messages < 1) return wfail(BBP_EINVAL, "trained_messages must be >= 1");
  const int64_t jobs = 4 * batch;
  const int L = 2 * d - 1, M = lg.M;
  const int64_t rows = jobs * L * L;
  const WLayout w = wlayout(d, jobs, M, true);
  if (workspace_bytes < w.total) return wfail(BBP_EINVAL, "workspace too small");
  char* ws = (char*)workspace;
  float *X0 = (float*)(ws + w.X0), *A1 = (float*)(ws + w.A1), *A2 = (float*)(ws + w.A2), *F = (float*)(ws + w.F),
        *dF = (float*)(ws + w.dF), *dA2 = (float*)(ws + w.dA2), *dA1 = (float*)(ws + w.dA1),
        *dout = (float*)(ws + w.dout), *lossb = (float*)(ws + w.loss);
  hipStream_t st = a.st;
  if ((rc = trunk(d, syndromes_dev, p_dev, p, jobs, params_dev, ws, w, st))) return rc;
  W_TRY(hipMemsetAsync(grad_dev, 0, OFF.total * sizeof(float), st));
  W_TRY(hipMemsetAsync(dF, 0, (size_t)rows * C3 * sizeof(float), st));
  W_TRY(hipMemsetAsync(lossb, 0, (size_t)jobs * std::max(M, 1) * sizeof(float), st));
  W_TRY(hipMemsetAsync(dout, 0, (size_t)jobs * std::max(M, 1) * NOUT * sizeof(float), st));
  if (M > 0) {
    head_kernel<true><<<dim3((unsigned)(jobs * M)), dim3(64), 0, st>>>(
        F, lg.dev, M, L, jobs, params_dev, targets_dev, use_dev, 1.0f / (float)trained_messages, nullptr, dout, dF,
        lossb);
    head_grad_kernel<<<dim3(36), dim3(64), 0, st>>>(F, lg.dev, M, L, jobs, use_dev, dout, grad_dev);
  }
  sum_kernel<<<1, 256, 0, st>>>(lossb, jobs * std::max(M, 1), loss_dev);
  W_TRY(hipGetLastError());
  // conv3 (no activation)
  if ((rc = conv<G_DW, 0>(L, rows, C2, C3, A2, dF, grad_dev + OFF.w3, nullptr, st))) return rc;
  colsum_kernel<<<C3, 256, 0, st>>>(dF, rows, C3, grad_dev + OFF.b3);
  if ((rc = conv<G_DX, 1>(L, rows, C2, C3, dF, params_dev + OFF.w3, dA2, A2, st))) return rc;
  // conv2 (ReLU: dA2 is already the gradient of its pre-activation)
  if ((rc = conv<G_DW, 0>(L, rows, C1, C2, A1, dA2, grad_dev + OFF.w2, nullptr, st))) return rc;
  colsum_kernel<<<C2, 256, 0, st>>>(dA2, rows, C2, grad_dev + OFF.b2);
  if ((rc = conv<G_DX, 1>(L, rows, C1, C2, dA2, params_dev + OFF.w2, dA1, A1, st))) return rc;
  // conv1
  if ((rc = conv<G_DW, 0>(L, rows, C0, C1, X0, dA1, grad_dev + OFF.w1, nullptr, st))) return rc;
  colsum_kernel<<<C1, 256, 0, st>>>(dA1, rows, C1, grad_dev + OFF.b1);
  W_TRY(hipGetLastError());
  return BBP_OK;
}

int bbp_warm_adam(float* params_dev, const float* grad_dev, float* m_dev, float* v_dev, int64_t step, float lr,
                  void* stream) {
  if (!params_dev || !grad_dev || !m_dev || !v_dev) return wfail(BBP_EINVAL, "a required pointer is NULL");
  if (step < 1 || !(lr > 0.0f)) return wfail(BBP_EINVAL, "step must be >= 1 and lr > 0");
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.0f - std::pow(b1, (float)step), c2 = 1.0f - std::pow(b2, (float)step);
  adam_kernel<<<grid1((int64_t)OFF.total), 256, 0, (hipStream_t)stream>>>(params_dev, grad_dev, m_dev, v_dev,
                                                                         (int64_t)OFF.total, lr, b1, b2, 1e-8f, c1, c2);
  W_TRY(hipGetLastError());
  return BBP_OK;
}

namespace {
struct DLayout {
  size_t pred, msgs, dec, list, count, syn, pv, ll, dl, it, cs, cr, total;
};
int dlayout(int d, int64_t batch, const bbp_opts* opts, double p, DLayout* out) {
  size_t pred = 0, dec = 0;
  int rc = bbp_warm_workspace_size(d, batch, opts, 0, &pred);
  if (rc) return rc;
  bbp_group g;
  std::memset(&g, 0, sizeof(g));
  g.d = d;
  g.p = (p > 0.0 && p < 1.0) ? p : 0.1;   // the workspace size does not depend on p
  g.batch = batch;
  if ((rc = bbp_workspace_size_groups(&g, 1, opts, &dec))) return wfail(rc, bbp_last_error());
  const bbp::Plan& P = bbp::cached_plan(d, opts->block_rows, opts->block_cols, opts->chi);
  const int64_t m = 2 * d * (d - 1), nq = (int64_t)d * d + (int64_t)(d - 1) * (d - 1);
  DLayout l{};
  size_t o = 0;
  l.pred = o; o = a256(o + pred);
  l.msgs = o; o = a256(o + (size_t)batch * 4 * std::max(P.M, 1) * 64 * 4);
  l.dec = o; o = a256(o + dec);
  l.list = o; o = a256(o + (size_t)batch * 8);
  l.count = o; o = a256(o + 8);
  l.syn = o; o = a256(o + (size_t)batch * m);
  l.pv = o; o = a256(o + (size_t)batch * 8);
  l.ll = o; o = a256(o + (size_t)batch * 32);
  l.dl = o; o = a256(o + (size_t)batch * 32);
  l.it = o; o = a256(o + (size_t)batch * 16);
  l.cs = o; o = a256(o + (size_t)batch);
  l.cr = o; o = a256(o + (size_t)batch * nq);
  l.total = o;
  *out = l;
  return BBP_OK;
}
}  // namespace

int bbp_warm_decode_workspace_size(int32_t d, int64_t batch, const bbp_opts* opts, size_t* bytes) {
  if (!bytes || !opts) return wfail(BBP_EINVAL, "NULL argument");
  if (batch < 1) return wfail(BBP_EINVAL, "batch must be >= 1");
  DLayout l;
  int rc = dlayout(d, batch, opts, 0.1, &l);
  if (rc) return rc;
  *bytes = l.total;
  return BBP_OK;
}

int bbp_warm_decode(int32_t d, double p, const double* p_dev, const uint8_t* syndromes_dev, int64_t batch,
                    const bbp_opts* opts, const float* params_dev, int32_t precision, int32_t trained_d_min,
                    int32_t trained_d_max, void* workspace, size_t workspace_bytes,
                    double* loglik_dev, double* delta_dev, int32_t* iters_dev, uint8_t* coset_dev,
                    uint8_t* correction_dev, int64_t* fallback_count, void* stream) {
  if (!opts || !params_dev || !syndromes_dev || !workspace || !loglik_dev || !delta_dev || !iters_dev ||
      !coset_dev || !correction_dev)
    return wfail(BBP_EINVAL, "a required pointer is NULL");
  if (batch < 1) return wfail(BBP_EINVAL, "batch must be >= 1");
  if (trained_d_min < 0 || trained_d_max < trained_d_min || (trained_d_min == 0) != (trained_d_max == 0))
    return wfail(BBP_EINVAL, "the trained distance range must be 0 <= min <= max, both 0 for no range");
  DLayout l;
  int rc = dlayout(d, batch, opts, p, &l);
  if (rc) return rc;
  if (workspace_bytes < l.total) return wfail(BBP_EINVAL, "workspace too small");
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)workspace;
  const int m = 2 * d * (d - 1), nq = d * d + (d - 1) * (d - 1);
  if (trained_d_min > 0 && (d < trained_d_min || d > trained_d_max)) {
    // outside the distances the network was trained on its start messages can lead BP to fixed points that
    // pass every convergence test with another decision: the whole batch is decoded from the uniform start
    bbp_group g;
    std::memset(&g, 0, sizeof(g));
    g.d = d;
    g.p = p;
    g.p_dev = p_dev;
    g.syndromes_dev = syndromes_dev;
    g.batch = batch;
    g.loglik_dev = loglik_dev;
    g.delta_dev = delta_dev;
    g.iters_dev = iters_dev;
    g.coset_dev = coset_dev;
    g.correction_dev = correction_dev;
    bbp_opts co = *opts;
    co.graph = 0;
    if ((rc = bbp_decode_groups(&g, 1, &co, ws + l.dec, l.list - l.dec, stream, nullptr)))
      return wfail(rc, std::string("cold decode: ") + bbp_last_error());
    if (fallback_count) *fallback_count = batch;
    return BBP_OK;
  }
  float* msgs = (float*)(ws + l.msgs);
  if ((rc = bbp_warm_predict(d, p, p_dev, syndromes_dev, batch, opts, params_dev, precision, msgs, ws + l.pred,
                             l.msgs - l.pred, stream)))
    return rc;
  bbp_group g;
  std::memset(&g, 0, sizeof(g));
  g.d = d;
  g.p = p;
  g.p_dev = p_dev;
  g.syndromes_dev = syndromes_dev;
  g.batch = batch;
  g.loglik_dev = loglik_dev;
  g.delta_dev = delta_dev;
  g.iters_dev = iters_dev;
  g.coset_dev = coset_dev;
  g.correction_dev = correction_dev;
  g.init_messages_dev = msgs;
  const size_t dec_bytes = l.list - l.dec;
  if ((rc = bbp_decode_groups(&g, 1, opts, ws + l.dec, dec_bytes, stream, nullptr)))
    return wfail(rc, std::string("warm decode: ") + bbp_last_error());
  int64_t* list = (int64_t*)(ws + l.list);
  int64_t* cnt = (int64_t*)(ws + l.count);
  W_TRY(hipMemsetAsync(cnt, 0, 8, st));
  fallback_select_kernel<<<grid1(batch), 256, 0, st>>>(delta_dev, iters_dev, coset_dev, batch, opts->delta1, list,
                                                       cnt);
  W_TRY(hipGetLastError());
  int64_t n = 0;
  W_TRY(hipMemcpyAsync(&n, cnt, 8, hipMemcpyDeviceToHost, st));
  W_TRY(hipStreamSynchronize(st));
  if (fallback_count) *fallback_count = n;
  if (n == 0) return BBP_OK;
  uint8_t* syn = (uint8_t*)(ws + l.syn);
  double* pv = (double*)(ws + l.pv);
  fallback_gather_kernel<<<dim3((unsigned)n), dim3(256), 0, st>>>(syndromes_dev, p_dev, m, list, n, syn, pv);
  W_TRY(hipGetLastError());
  bbp_group c = g;
  c.p_dev = p_dev ? pv : nullptr;
  c.syndromes_dev = syn;
  c.batch = n;
  c.loglik_dev = (double*)(ws + l.ll);
  c.delta_dev = (double*)(ws + l.dl);
  c.iters_dev = (int32_t*)(ws + l.it);
  c.coset_dev = (uint8_t*)(ws + l.cs);
  c.correction_dev = (uint8_t*)(ws + l.cr);
  c.init_messages_dev = nullptr;
  bbp_opts co = *opts;
  co.graph = 0;   // the fallback batch changes from call to call
  if ((rc = bbp_decode_groups(&c, 1, &co, ws + l.dec, dec_bytes, stream, nullptr)))
    return wfail(rc, std::string("cold fallback: ") + bbp_last_error());
  fallback_scatter_kernel<<<dim3((unsigned)n), dim3(256), 0, st>>>(list, n, nq, c.loglik_dev, c.delta_dev,
                                                                    c.iters_dev, c.coset_dev, c.correction_dev,
                                                                    loglik_dev, delta_dev, iters_dev, coset_dev,
                                                                    correction_dev);
  W_TRY(hipGetLastError());
  return BBP_OK;
}

}  // extern "C"
