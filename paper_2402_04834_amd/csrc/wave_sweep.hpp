// wave_sweep.hpp -- one block sweep (Sec. III.D, the block update of Alg. 1) executed by a single wavefront
// with the whole boundary state in registers.
//
// Formulation. Every bond of the coset network joins a qubit and a check, and a check is a COPY tensor, so
// in a column of the sweep a check passes its crossing-bond value straight through, while a qubit maps its
// crossing-bond value h_i to h'_i with coefficient T(up, h_i, down, h'_i), up / down being the variables of
// the checks above and below it -- bits of the boundary state that the column leaves unchanged. A column
// is therefore a product of commuting 2x2 transforms, one per qubit, conditioned on neighbouring bits. At
// the two ends of the column the side messages act as caps: their sites emit the vertical bond value at
// the end site, which either equals the end check's variable or is summed against the end qubit.
//
// Mapping. Lane h of the wavefront is one crossing-bond configuration (kp <= 6 positions, 64 lanes).
// Lane bit 0 is position 0 (the top end of the column), lane bit 1 the last position, and lane bit i+1 the
// middle position i, so every qubit transform pairs lanes at a compile-time distance: 1 and 2 by DPP
// quad permutes, 4 / 8 / 16 by ds_swizzle, 32 by ds_bpermute. The cap indices of the state -- n for the
// top side message, s for the bottom one -- are register indices. The cap dimensions at each column are
// fixed by the sweep length and direction (bond j of a K-site message carries 2^min(j, K-j) values in the
// open-leg reading), so the whole sweep is instantiated per (sweep length, direction, caps present), and
// every register index is a compile-time constant. No LDS, no barriers: a workgroup holds independent
// sweeps, one per wavefront.
//
// Side-message caps: psi over the old cap index, phi over the new one and the emitted vertical bond v (see
// Cap below). Any placement of the dense core along the message gives the same exact contraction; a sweep
// that runs against the message's leg order reads the message with its legs reversed.
#pragma once
#include <utility>

#include "geom.hpp"

namespace bbp {
namespace wave {

// ---------------------------------------------------------------------------------------------- helpers
template <class F, int... I>
__device__ __forceinline__ void sfor_(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
// f(integral_constant<int, i>) for i = 0 .. N-1, each index a compile-time constant
template <int N, class F>
__device__ __forceinline__ void sfor(F&& f) {
  sfor_(f, std::make_integer_sequence<int, N>{});
}

// value of x in lane (lane ^ M)
template <int M>
__device__ __forceinline__ float xchg(float x) {
  const int xi = __float_as_int(x);
  if constexpr (M == 1) return __int_as_float(__builtin_amdgcn_mov_dpp(xi, 0xB1, 0xF, 0xF, true));   // [1,0,3,2]
  else if constexpr (M == 2) return __int_as_float(__builtin_amdgcn_mov_dpp(xi, 0x4E, 0xF, 0xF, true));  // [2,3,0,1]
  else if constexpr (M < 32) return __int_as_float(__builtin_amdgcn_ds_swizzle(xi, 0x1F | (M << 10)));
  else return __int_as_float(__builtin_amdgcn_ds_bpermute((((int)__lane_id()) ^ M) << 2, xi));
}

__device__ __forceinline__ float xchg_rt(float x, int m) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute((((int)__lane_id()) ^ m) << 2, __float_as_int(x)));
}

__device__ __forceinline__ float readlane_f(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// ------------------------------------------------------------------------------------------- cap shapes
enum : int { K_NONE = 0, K_LT, K_EQ, K_GT };

constexpr int cdim(int K, int j) { return 1 << ((j < K - j) ? j : K - j); }

// Cap at step T of a KT-step sweep. A sweep that walks a side message from its last site is run on the
// message with its legs reversed, so every cap walks its message from the first site: steps before the
// middle site D append the emitted bond as the low bit of the cap index, the middle site contracts with the
// dense message entry m[(a, v, np)], later steps strip the emitted bond from the high bit.
template <bool PRESENT, int KT, int T>
struct Cap {
  static constexpr int D = KT / 2;
  static constexpr int PO = PRESENT ? cdim(KT, T) : 1;
  static constexpr int PN = PRESENT ? cdim(KT, T + 1) : 1;
  static constexpr int R2 = 1 << (KT - D - 1);
  static constexpr int kind = !PRESENT ? K_NONE : (T < D ? K_LT : T == D ? K_EQ : K_GT);
};

// phi[NP][V] = sum_a op[a][V][NP] psi[a]; g(a) reads psi[a] (a compile-time), m(idx) reads the dense side
// message at a compile-time index.
template <class C, int NP, int V, class G, class Msg>
__device__ __forceinline__ float phi(G&& g, Msg&& m) {
  if constexpr (C::kind == K_NONE) {
    if constexpr (V == 0) return g(std::integral_constant<int, 0>{});
    else return 0.0f;
  } else if constexpr (C::kind == K_LT) {
    if constexpr (V == (NP & 1)) return g(std::integral_constant<int, (NP >> 1)>{});
    else return 0.0f;
  } else if constexpr (C::kind == K_GT) {
    return g(std::integral_constant<int, V * C::PN + NP>{});
  } else {
    float acc = 0.0f;
    sfor<C::PO>([&](auto a) { acc += m(std::integral_constant<int, (2 * a + V) * C::R2 + NP>{}) * g(a); });
    return acc;
  }
}

// ------------------------------------------------------------------------------------- sweep context
struct Ctx {
  int h;                       // lane = crossing-bond configuration (lane-bit layout above)
  int kp, kt;                  // positions across the sweep, sweep steps
  int frame, r0, c0, kr, kc, L;
  float labv;                  // lane l < kt*kp: coset label of the site at (step l / kp, position l % kp)
  float mtv, mbv;              // lane l: entry l of the top / bottom side message (0 if absent)
  float p0, p1, p2, p3;        // noise table {I, Z, X, Y} indexed x*2 + z
  double logscale;             // accumulated log of the normalisations
};

// lane bit of position i
__device__ __forceinline__ int pbit(int kp, int i) { return i == 0 ? 1 : (i == kp - 1 ? 2 : (1 << (i + 1))); }

struct SiteInfo {
  int qubit, label, swap, absent;   // absent: legs (up, in, down, out) that leave the grid, bits 0..3
};

__device__ __forceinline__ SiteInfo site_info(const Ctx& c, int t, int i) {
  int r, cc;
  frame_site(c.frame, c.r0, c.c0, c.kr, c.kc, t, i, r, cc);
  int a_up, a_in, a_dn, a_out;
  const int au = (r == 0), al = (cc == 0), ad = (r == c.L - 1), ar = (cc == c.L - 1);
  switch (c.frame) {
    case FRAME_E: a_up = au; a_in = al; a_dn = ad; a_out = ar; break;
    case FRAME_W: a_up = au; a_in = ar; a_dn = ad; a_out = al; break;
    case FRAME_S: a_up = al; a_in = au; a_dn = ar; a_out = ad; break;
    default:      a_up = al; a_in = ad; a_dn = ar; a_out = au; break;
  }
  SiteInfo s;
  s.qubit = ((r + cc) & 1) == 0;
  s.absent = a_up | (a_in << 1) | (a_dn << 2) | (a_out << 3);
  s.swap = ((r & 1) != 0) != (c.frame >= FRAME_S);
  s.label = s.qubit ? (__float_as_int(readlane_f(c.labv, t * c.kp + i)) & 3) : 0;
  return s;
}

__device__ __forceinline__ float coef(const Ctx& c, const SiteInfo& s, int vi, int hi, int vo, int ho) {
  return qubit_coef(s.label, s.swap, s.absent, c.p0, c.p1, c.p2, c.p3, vi, hi, vo, ho);
}

// lane mask of the checks of step t whose out-leg leaves the grid (their variable is summed)
__device__ __forceinline__ int out_absent_mask(const Ctx& c, int t) {
  int m = 0;
  for (int i = 0; i < c.kp; ++i) {
    const SiteInfo s = site_info(c, t, i);
    if (!s.qubit && (s.absent & 8)) m |= pbit(c.kp, i);
  }
  return m;
}

template <int N>
__device__ __forceinline__ void project_out_absent(float (&Y)[N], const Ctx& c, int oa) {
  for (int b = 1; b < 64; b <<= 1) {
    if (!(oa & b)) continue;
    const bool zero = (c.h & b) != 0;
    sfor<N>([&](auto e) {
      const float o = xchg_rt(Y[e], b);
      Y[e] = zero ? 0.0f : Y[e] + o;
    });
  }
}

// --------------------------------------------------------------------------------- column, kp >= 2
template <int KT, bool TOP, bool BOT, int T>
__device__ __forceinline__ void column_multi(const float (&X)[Cap<TOP, KT, T>::PO * Cap<BOT, KT, T>::PO],
                                             float (&Y)[Cap<TOP, KT, T>::PN * Cap<BOT, KT, T>::PN],
                                             Ctx& c) {
  using CT = Cap<TOP, KT, T>;
  using CB = Cap<BOT, KT, T>;
  constexpr int PTO = CT::PO, PTN = CT::PN, PSO = CB::PO, PSN = CB::PN;
  const int h = c.h, kp = c.kp;
  auto mt = [&](auto idx) { return readlane_f(c.mtv, idx); };
  auto mb = [&](auto idx) { return readlane_f(c.mbv, idx); };

  // top cap + site 0 (lane bit 0)
  float Z[PTN * PSO];
  const SiteInfo s0 = site_info(c, T, 0);
  if (s0.qubit) {
    const int ho = h & 1, vo = (h >> 1 + (kp > 2 ? 1 : 0)) & 1;   // position 1: lane bit 1 if kp == 2, else 2
    const float cs0 = coef(c, s0, 0, ho, vo, ho), cf0 = coef(c, s0, 0, ho ^ 1, vo, ho);
    const float cs1 = coef(c, s0, 1, ho, vo, ho), cf1 = coef(c, s0, 1, ho ^ 1, vo, ho);
    sfor<PSO>([&](auto s) {
      float Y0[PTO], Y1[PTO];
      sfor<PTO>([&](auto a) {
        const float x = X[a * PSO + s], xf = xchg<1>(x);
        Y0[a] = cs0 * x + cf0 * xf;
        Y1[a] = cs1 * x + cf1 * xf;
      });
      sfor<PTN>([&](auto n) {
        Z[n * PSO + s] = phi<CT, n, 0>([&](auto a) { return Y0[a]; }, mt) +
                         phi<CT, n, 1>([&](auto a) { return Y1[a]; }, mt);
      });
    });
  } else {
    const bool v1 = !(s0.absent & 1) && (h & 1);
    sfor<PSO>([&](auto s) {
      sfor<PTN>([&](auto n) {
        const float z0 = phi<CT, n, 0>([&](auto a) { return X[a * PSO + s]; }, mt);
        const float z1 = phi<CT, n, 1>([&](auto a) { return X[a * PSO + s]; }, mt);
        Z[n * PSO + s] = v1 ? z1 : z0;
      });
    });
  }

  // middle qubits (positions 1 .. kp-2, lane bits 2 .. kp-1)
  sfor<4>([&](auto j) {
    constexpr int i = j + 1;
    constexpr int bit = 1 << (i + 1);
    if (i <= kp - 2) {
      const SiteInfo si = site_info(c, T, i);
      if (si.qubit) {
        const int vi = (h >> (i == 1 ? 0 : i)) & 1;                    // position i-1
        const int vo = (i + 1 == kp - 1) ? ((h >> 1) & 1) : ((h >> (i + 2)) & 1);   // position i+1
        const int ho = (h >> (i + 1)) & 1;
        const float cs = coef(c, si, vi, ho, vo, ho), cf = coef(c, si, vi, ho ^ 1, vo, ho);
        sfor<PTN * PSO>([&](auto e) { Z[e] = cs * Z[e] + cf * xchg<bit>(Z[e]); });
      }
    }
  });

  // bottom cap + last site (lane bit 1)
  const SiteInfo sl = site_info(c, T, kp - 1);
  if (sl.qubit) {
    const int ho = (h >> 1) & 1, vi = (h >> (kp > 2 ? kp - 1 : 0)) & 1;   // position kp-2
    const float cs0 = coef(c, sl, vi, ho, 0, ho), cf0 = coef(c, sl, vi, ho ^ 1, 0, ho);
    const float cs1 = coef(c, sl, vi, ho, 1, ho), cf1 = coef(c, sl, vi, ho ^ 1, 1, ho);
    sfor<PTN>([&](auto n) {
      float Y0[PSO], Y1[PSO];
      sfor<PSO>([&](auto b) {
        const float z = Z[n * PSO + b], zf = xchg<2>(z);
        Y0[b] = cs0 * z + cf0 * zf;
        Y1[b] = cs1 * z + cf1 * zf;
      });
      sfor<PSN>([&](auto sp) {
        Y[n * PSN + sp] = phi<CB, sp, 0>([&](auto b) { return Y0[b]; }, mb) +
                          phi<CB, sp, 1>([&](auto b) { return Y1[b]; }, mb);
      });
    });
  } else {
    const bool v1 = !(sl.absent & 4) && (h & 2);
    sfor<PTN>([&](auto n) {
      sfor<PSN>([&](auto sp) {
        const float y0 = phi<CB, sp, 0>([&](auto b) { return Z[n * PSO + b]; }, mb);
        const float y1 = phi<CB, sp, 1>([&](auto b) { return Z[n * PSO + b]; }, mb);
        Y[n * PSN + sp] = v1 ? y1 : y0;
      });
    });
  }
  if (T == KT - 1) {
    const int oa = out_absent_mask(c, T);
    if (oa) project_out_absent(Y, c, oa);
  }
}

// --------------------------------------------------------------------------------- column, kp == 1
// The single site of the column meets both caps: a qubit sums both emitted bonds (the bottom one is kept
// as an extra index between the two cap steps), a check emits its own variable on both.
template <int KT, bool TOP, bool BOT, int T>
__device__ __forceinline__ void column_single(const float (&X)[Cap<TOP, KT, T>::PO * Cap<BOT, KT, T>::PO],
                                              float (&Y)[Cap<TOP, KT, T>::PN * Cap<BOT, KT, T>::PN], Ctx& c) {
  using CT = Cap<TOP, KT, T>;
  using CB = Cap<BOT, KT, T>;
  constexpr int PTO = CT::PO, PTN = CT::PN, PSO = CB::PO, PSN = CB::PN;
  const int h = c.h;
  auto mt = [&](auto idx) { return readlane_f(c.mtv, idx); };
  auto mb = [&](auto idx) { return readlane_f(c.mbv, idx); };
  const SiteInfo s0 = site_info(c, T, 0);
  const int ho = h & 1;
  if (s0.qubit) {
    float Z[2][PTN * PSO];   // [emitted bottom bond][np][s]
    sfor<2>([&](auto vb) {
      const float cs0 = coef(c, s0, 0, ho, vb, ho), cf0 = coef(c, s0, 0, ho ^ 1, vb, ho);
      const float cs1 = coef(c, s0, 1, ho, vb, ho), cf1 = coef(c, s0, 1, ho ^ 1, vb, ho);
      sfor<PSO>([&](auto s) {
        float Y0[PTO], Y1[PTO];
        sfor<PTO>([&](auto a) {
          const float x = X[a * PSO + s], xf = xchg<1>(x);
          Y0[a] = cs0 * x + cf0 * xf;
          Y1[a] = cs1 * x + cf1 * xf;
        });
        sfor<PTN>([&](auto n) {
          Z[vb][n * PSO + s] = phi<CT, n, 0>([&](auto a) { return Y0[a]; }, mt) +
                               phi<CT, n, 1>([&](auto a) { return Y1[a]; }, mt);
        });
      });
    });
    sfor<PTN>([&](auto n) {
      sfor<PSN>([&](auto sp) {
        Y[n * PSN + sp] = phi<CB, sp, 0>([&](auto b) { return Z[0][n * PSO + b]; }, mb) +
                          phi<CB, sp, 1>([&](auto b) { return Z[1][n * PSO + b]; }, mb);
      });
    });
  } else {
    const bool vt = !(s0.absent & 1) && ho, vb = !(s0.absent & 4) && ho;
    float Z[PTN * PSO];
    sfor<PSO>([&](auto s) {
      sfor<PTN>([&](auto n) {
        const float z0 = phi<CT, n, 0>([&](auto a) { return X[a * PSO + s]; }, mt);
        const float z1 = phi<CT, n, 1>([&](auto a) { return X[a * PSO + s]; }, mt);
        Z[n * PSO + s] = vt ? z1 : z0;
      });
    });
    sfor<PTN>([&](auto n) {
      sfor<PSN>([&](auto sp) {
        const float y0 = phi<CB, sp, 0>([&](auto b) { return Z[n * PSO + b]; }, mb);
        const float y1 = phi<CB, sp, 1>([&](auto b) { return Z[n * PSO + b]; }, mb);
        Y[n * PSN + sp] = vb ? y1 : y0;
      });
    });
  }
  if (T == KT - 1) {
    const int oa = out_absent_mask(c, T);
    if (oa) project_out_absent(Y, c, oa);
  }
}

// ------------------------------------------------------------------------------------------ the sweep
__device__ __forceinline__ float wave_sum(float v) {
  sfor<6>([&](auto k) { v += xchg<(1 << k)>(v); });
  return v;
}

template <int N>
__device__ __forceinline__ void normalise(float (&Y)[N], Ctx& c) {
  float ss = 0.0f;
  sfor<N>([&](auto e) { ss += Y[e] * Y[e]; });
  ss = wave_sum(ss);
  const float nrm = sqrtf(ss);
  const float inv = (nrm > 0.0f) ? 1.0f / nrm : 0.0f;
  c.logscale += (double)logf(nrm);
  sfor<N>([&](auto e) { Y[e] *= inv; });
}

// Absorb columns T .. KT-1 into the state X; returns the final (one-value-per-lane) state.
template <int KT, bool TOP, bool BOT, bool SINGLE, int T>
__device__ __forceinline__ float run(const float (&X)[Cap<TOP, KT, T>::PO * Cap<BOT, KT, T>::PO], Ctx& c) {
  float Y[Cap<TOP, KT, T>::PN * Cap<BOT, KT, T>::PN];
  if constexpr (SINGLE) column_single<KT, TOP, BOT, T>(X, Y, c);
  else column_multi<KT, TOP, BOT, T>(X, Y, c);
  normalise(Y, c);
  if constexpr (T + 1 < KT) return run<KT, TOP, BOT, SINGLE, T + 1>(Y, c);
  else return Y[0];
}

// The whole sweep from the entering state x0 (one value per lane); SINGLE: one position across (kp == 1).
template <int KT, bool TOP, bool BOT, bool SINGLE>
__device__ __forceinline__ float sweep(float x0, Ctx& c) {
  const float X[1] = {x0};
  return run<KT, TOP, BOT, SINGLE, 0>(X, c);
}

}  // namespace wave
}  // namespace bbp
