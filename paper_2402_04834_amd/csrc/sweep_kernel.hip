// sweep_kernel.hip -- block-sweep kernels for sweeps of BBP_KT steps (this file is compiled once per
// length, BBP_KT = 1..6). One wavefront runs one (job, sweep); the sweep itself is in wave_sweep.hpp.
//   mode 0: BP update of message s.msg_out (Sec. III.D): the new message is normalised (remark 3), damped
//           against the old one (remark 7) and the distance term of the convergence test stored (remark 4);
//   mode 1: closing sweep of block s.block, W_v of the Bethe estimate (Lemma 3.1).
// Grid: x = items / SWEEP_WAVES; item = one (job, sweep) of one (d, p) group of the launch.
#include <hip/hip_runtime.h>

#include "sweep_launch.hpp"
#include "wave_sweep.hpp"

#include <type_traits>
#include <utility>

#ifndef BBP_KT
#error "compile with -DBBP_KT=<sweep length 1..6>"
#endif
#ifndef BBP_WAVES_PER_EU
#define BBP_WAVES_PER_EU 4   // register budget: at least this many wavefronts per SIMD
#endif

namespace bbp {
namespace {

__device__ __forceinline__ double wave_sum_d(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// entry index of a K-leg dense message with its legs in reverse order
__device__ __forceinline__ int reverse_legs(int idx, int K) { return (int)(__brev((unsigned)idx) >> (32 - K)); }

// BF: the contractions with the side messages' middle sites take BF16 operands on the matrix cores (precision
// mode 1; FP32 everywhere else), else FP32 throughout (precision 0). BIASED: some group of the launch has
// biased Pauli noise (otherwise the depolarizing entries are compiled in and the biased selection is removed).
template <bool BF, int KT, bool TOP, bool BOT, bool SINGLE, bool Q00, bool BIASED>
__global__ __launch_bounds__(SWEEP_WAVES * 64) __attribute__((amdgpu_waves_per_eu(BBP_WAVES_PER_EU)))
void sweep_kernel(SweepArgs a) {
  const int lane = (int)__lane_id();
  const int64_t item = (int64_t)blockIdx.x * SWEEP_WAVES + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
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
      if (lane == 0) G.terms[job * G.M + s.msg_out] = 0.0;
      return;
    }
  }
  using V = float;
  const int L = 2 * G.d - 1, kp = s.kp, H = 1 << kp;
  const bool valid = lane < H;

  wave::Ctx<V> c;
  c.h = lane;
  c.kp = kp;
  c.geo = s.geo;
  if (G.pdev) {
    const float pj = (float)G.pdev[job >> 2];
    c.p00 = 1.0f - pj;
    c.pe = pj / 3.0f;
  } else {
    c.p00 = G.p00;
    c.pe = G.pe;
  }
  c.biased = BIASED ? G.biased : 0;
  for (int k = 0; k < 4; ++k) c.pib[k] = __float_as_int(G.pi[k]);
  c.exp2 = 0;
  const uint8_t* lab = G.labels + job * L * L;
  int lb = 0;
  if (lane < KT * kp) {
    const int t = lane / kp, i = lane - t * kp;
    int r, cc;
    frame_site(s.frame, s.r0, s.c0, s.kr, s.kc, t, i, r, cc);
    lb = lab[r * L + cc];
  }
  c.labv = __int_as_float(lb);
  // side messages: a sweep toward W or N walks them from their last leg, so read them leg-reversed
  const bool fwd = (s.frame == FRAME_E || s.frame == FRAME_S);
  const float* mbase = G.msgs + job * G.M * MSTRIDE;
  const int sl = fwd ? lane : reverse_legs(lane, KT);
  const bool in_msg = lane < (1 << KT);
  c.mtv = V{(TOP && in_msg) ? mbase[s.msg_top * MSTRIDE + sl] : 0.0f};
  c.mbv = V{(BOT && in_msg) ? mbase[s.msg_bot * MSTRIDE + sl] : 0.0f};

  // message index of this lane's configuration: position i is lane bit pshift(i), message bit kp-1-i
  int mi = 0;
  for (int i = 0; i < kp; ++i)
    if (lane & (1 << wave::pshift(kp, i))) mi |= 1 << (kp - 1 - i);

  float x0;
  if (s.msg_init >= 0) {
    x0 = valid ? mbase[s.msg_init * MSTRIDE + mi] : 0.0f;
  } else {
    // the sweep starts at the grid edge: checks whose in-leg leaves the grid are free variables
    const int ia = (s.geo & GEO_IN_EDGE) ? wave::check_lanes(c, Q00) : 0;
    x0 = ((lane & ~ia) == 0) ? 1.0f : 0.0f;
  }

  float fin = wave::sweep<V, KT, TOP, BOT, SINGLE, Q00, BF>(x0, c);
  fin = valid ? fin : 0.0f;

  if (a.mode == 1) {
    // closing contraction with the message from the receiver side (or the grid edge)
    double w = 0.0;
    if (s.msg_close >= 0) w = valid ? (double)mbase[s.msg_close * MSTRIDE + mi] * (double)fin : 0.0;
    else if (lane == 0) w = fin;
    w = wave_sum_d(w);
    if (lane == 0) G.lnW[job * G.nblocks + s.block] = (w > 0.0) ? c.exp2 * 0.69314718055994530942 + log(w) : NAN;
  } else {
    // normalised new message, damping against the old one (unit norm), distance term. With unit vectors
    // a, b: 2 - 2<a,b>^2 = |a - b|^2 |a + b|^2 / 2, which has no cancellation near convergence in FP32.
    float* mo = G.msgs + job * G.M * MSTRIDE + s.msg_out * MSTRIDE;
    const float old = valid ? mo[mi] : 0.0f;
    const float fn = fin * __builtin_amdgcn_rsqf(wave::wave_sum(fin * fin));
    const float dm = (1.0f - a.eta) * fn + a.eta * old;
    const float fm = dm * __builtin_amdgcn_rsqf(wave::wave_sum(dm * dm));
    const float dif = fm - old, sum = fm + old;
    const float dd = wave::wave_sum(dif * dif), ss = wave::wave_sum(sum * sum);
    if (valid) mo[mi] = fm;
    if (lane == 0) G.terms[job * G.M + s.msg_out] = 0.5 * (double)dd * (double)ss;
  }
}

}  // namespace

#define BBP_CAT2(a, b) a##b
#define BBP_CAT(a, b) BBP_CAT2(a, b)

namespace {
// variants 0..47: bit 4 BF16 middle-site contractions (precision 1), bit 5 biased noise (FP32 only)
template <int V>
void launch_variant(dim3 grid, hipStream_t st, const SweepArgs& a) {
  constexpr bool TOP = (V >> 3) & 1, BOT = (V >> 2) & 1, SINGLE = (V >> 1) & 1, Q00 = V & 1;
  constexpr bool BF = (V >> 4) & 1, BIASED = (V >> 5) & 1;
  if constexpr (BF)
    sweep_kernel<true, BBP_KT, TOP, BOT, SINGLE, Q00, false><<<grid, dim3(SWEEP_WAVES * 64), 0, st>>>(a);
  else
    sweep_kernel<false, BBP_KT, TOP, BOT, SINGLE, Q00, BIASED><<<grid, dim3(SWEEP_WAVES * 64), 0, st>>>(a);
}

template <int... I>
hipError_t dispatch(int variant, dim3 grid, hipStream_t st, const SweepArgs& a, std::integer_sequence<int, I...>) {
  bool done = false;
  ((variant == I ? (launch_variant<I>(grid, st, a), done = true) : false), ...);
  return done ? hipGetLastError() : hipErrorInvalidValue;
}
}  // namespace

// variant = (biased noise ? 32 : BF16-input products ? 16 : 0) + ((top * 2 + bottom) * 2 + single) * 2 + q00
hipError_t BBP_CAT(launch_sweeps_k, BBP_KT)(int variant, dim3 grid, hipStream_t st, const SweepArgs& a) {
  return dispatch(variant, grid, st, a, std::make_integer_sequence<int, 48>{});
}

}  // namespace bbp
