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
// fixed by the sweep length (bond j of a K-site message carries 2^min(j, K-j) values in the open-leg
// reading), and qubits and checks alternate along both axes, so with the sweep length, the caps present
// and the kind of the first site as template parameters every register index and every qubit/check
// decision is a compile-time constant. No LDS, no barriers: a workgroup holds independent sweeps.
//
// Side-message caps: psi over the old cap index, phi over the new one and the emitted vertical bond v (see
// Cap below). Any placement of the dense core along the message gives the same exact contraction; a sweep
// that runs against the message's leg order reads the message with its legs reversed.
//
// Noise: i.i.d. single-qubit Pauli noise; a qubit tensor entry is the probability of its label flipped by the
// adjacent bond parities. Depolarizing (p00 = 1 - p for the identity, pe = p/3 otherwise) is the default;
// a group may give four probabilities instead (biased noise), selected per qubit on the scalar unit.
//
// Middle-site caps with four new cap values (sweeps of 5 and 6 steps) contract on the matrix cores: the
// message entries are the same for every lane, so lane 4b+i supplies entry (a, v, i) and lane h = 4b+j
// its own state value; each v_mfma_f32_4x4x1f32 is one step a of the sum for all four new cap values,
// which land in the lane's four accumulator registers. FP32 products and FP32 accumulation throughout.
//
// BF16 variant (BF = true, precision mode 1): these middle-site contractions take BF16 operands on
// v_mfma_f32_4x4x4_16b_bf16 (K = 4 terms per instruction, FP32 accumulation). Where the end site is a
// qubit, its transform is folded into the message operand, A[n][(a, own / partner)] = sum_v m(a, v, n) c_v,
// with B the lane's state value and its partner's: the coefficients c_v depend only on the neighbouring
// check bit, a lane bit >= 2 when kp >= 3, so they are the same for the four lanes of an MFMA block (for
// kp < 3 the transform stays on the VALU and only the message contraction is BF16). Every other product
// -- the qubit transforms of the other columns, the routing caps -- stays FP32: on the VALU a BF16 dot
// product (v_dot2c_f32_bf16) needs its pair packed and its accumulator zeroed, three instructions where the
// FP32 transform takes two, so BF16 pays only on the matrix cores.
//
// Scaling: after every second column (odd steps, never the last) the state is rescaled by an exact power of
// two chosen from its norm (the exponent is accumulated), and the factor is folded into the first qubit
// transform of the next column, so normalisation costs one multiply-add per state entry and a wave
// reduction. Entries are non-negative, so two columns shrink a unit state by at most the product of their
// smallest coefficients and message entries, far above the FP32 range limit.
#pragma once
#include <type_traits>
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

typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf4 __attribute__((ext_vector_type(4)));
typedef float fl2 __attribute__((ext_vector_type(2)));
typedef unsigned u2 __attribute__((ext_vector_type(2)));
// (lo, hi) rounded to BF16 (round to nearest even) in one register: one v_cvt_pk_bf16_f32. Converting the
// pair as a vector is what makes the compiler emit the two-operand form (element-wise casts become two
// conversions and a v_perm), and it keeps the instruction visible to the compiler's MFMA hazard checks.
__device__ __forceinline__ unsigned cvt_pk_bf16(float lo, float hi) {
  return __builtin_bit_cast(unsigned, __builtin_convertvector((fl2){lo, hi}, bf2));
}
// (a, b, c, d) as the four BF16 values of a 4x4x4 MFMA operand, in k order
__device__ __forceinline__ bf4 pk4(float a, float b, float c, float d) {
  const u2 w = {cvt_pk_bf16(a, b), cvt_pk_bf16(c, d)};
  return __builtin_bit_cast(bf4, w);
}

template <class V>
__device__ __forceinline__ int vbits(V x) { return __builtin_bit_cast(int, x); }
template <class V>
__device__ __forceinline__ V vfrom(int i) { return __builtin_bit_cast(V, i); }
template <class V>
__device__ __forceinline__ V splat(float x) { return V{x}; }
__device__ __forceinline__ float tof(float x) { return x; }
// a * b + c, fused
__device__ __forceinline__ float fmav(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// value of x in lane (lane ^ M)
template <int M, class V>
__device__ __forceinline__ V xchg(V x) {
  const int xi = vbits(x);
  if constexpr (M == 1) return vfrom<V>(__builtin_amdgcn_mov_dpp(xi, 0xB1, 0xF, 0xF, true));   // [1,0,3,2]
  else if constexpr (M == 2) return vfrom<V>(__builtin_amdgcn_mov_dpp(xi, 0x4E, 0xF, 0xF, true));  // [2,3,0,1]
  else if constexpr (M < 32) return vfrom<V>(__builtin_amdgcn_ds_swizzle(xi, 0x1F | (M << 10)));
  else return vfrom<V>(__builtin_amdgcn_ds_bpermute((((int)__lane_id()) ^ M) << 2, xi));
}

template <class V>
__device__ __forceinline__ V xchg_rt(V x, int m) {
  return vfrom<V>(__builtin_amdgcn_ds_bpermute((((int)__lane_id()) ^ m) << 2, vbits(x)));
}

template <class V>
__device__ __forceinline__ V readlane_v(V v, int l) {
  return vfrom<V>(__builtin_amdgcn_readlane(vbits(v), l));
}
__device__ __forceinline__ float readlane_f(float v, int l) { return readlane_v(v, l); }

// value of x in lane l (ds_bpermute)
__device__ __forceinline__ float lane_get(float x, int l) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(l << 2, __float_as_int(x)));
}

typedef float f4 __attribute__((ext_vector_type(4)));

// One rank-1 step of 16 independent 4x4 products (v_mfma_f32_4x4x1f32): lanes 4b..4b+3 form block b;
// lane 4b+i supplies a (row i), lane 4b+j supplies b (column j) and holds acc[i] = D[i][j].
__device__ __forceinline__ f4 mfma4(float a, float b, f4 acc) { return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, acc, 0, 0, 0); }
// The same 16 blocks with K = 4 in BF16 (v_mfma_f32_4x4x4_16b_bf16): lane 4b+i supplies row i of A as four
// BF16 values (k = 0..3), lane 4b+j column j of B, and holds acc[i] = D[i][j] in FP32.
__device__ __forceinline__ f4 mfma4b(bf4 a, bf4 b, f4 acc) { return __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(a, b, acc, 0, 0, 0); }

__device__ __forceinline__ float wave_sum(float v) {
  sfor<6>([&](auto k) { v += xchg<(1 << k)>(v); });
  return v;
}

// ------------------------------------------------------------------------------------------- cap shapes
enum : int { K_NONE = 0, K_LT, K_EQ, K_GT };

constexpr int cdim(int K, int j) { return 1 << ((j < K - j) ? j : K - j); }

// Cap at step T of a KT-step sweep, walked from the message's first site: steps before the middle site
// D append the emitted bond as the low bit of the cap index, the middle site contracts with the dense
// message entry m[(a, v, np)], later steps strip the emitted bond from the high bit.
template <bool PRESENT, int KT, int T>
struct Cap {
  static constexpr int D = KT / 2;
  static constexpr int PO = PRESENT ? cdim(KT, T) : 1;
  static constexpr int PN = PRESENT ? cdim(KT, T + 1) : 1;
  static constexpr int R2 = 1 << (KT - D - 1);
  static constexpr int kind = !PRESENT ? K_NONE : (T < D ? K_LT : T == D ? K_EQ : K_GT);
  static constexpr int idx(int a, int v, int np) { return (2 * a + v) * R2 + np; }   // entry of m (K_EQ)
};

// phi[NP][V] = sum_a op[a][V][NP] psi[a]; g(a) reads psi[a] (a compile-time), m(idx) reads the dense side
// message at a compile-time index.
template <class C, int NP, int V, class G, class Msg>
__device__ __forceinline__ auto phi(G&& g, Msg&& m) {
  using R = decltype(g(std::integral_constant<int, 0>{}));
  if constexpr (C::kind == K_NONE) {
    if constexpr (V == 0) return g(std::integral_constant<int, 0>{});
    else return splat<R>(0.0f);
  } else if constexpr (C::kind == K_LT) {
    if constexpr (V == (NP & 1)) return g(std::integral_constant<int, (NP >> 1)>{});
    else return splat<R>(0.0f);
  } else if constexpr (C::kind == K_GT) {
    return g(std::integral_constant<int, V * C::PN + NP>{});
  } else {
    R acc = splat<R>(0.0f);
    sfor<C::PO>([&](auto a) { acc += m(std::integral_constant<int, C::idx(a, V, NP)>{}) * g(a); });
    return acc;
  }
}

// phi[NP][0] over g0 plus phi[NP][1] over g1, without adding structural zeros (routing caps).
template <class C, int NP, class G0, class G1, class Msg>
__device__ __forceinline__ auto phi2(G0&& g0, G1&& g1, Msg&& m) {
  using R = decltype(g0(std::integral_constant<int, 0>{}));
  if constexpr (C::kind == K_NONE) {
    return g0(std::integral_constant<int, 0>{});
  } else if constexpr (C::kind == K_LT) {
    if constexpr (NP & 1) return g1(std::integral_constant<int, (NP >> 1)>{});
    else return g0(std::integral_constant<int, (NP >> 1)>{});
  } else if constexpr (C::kind == K_GT) {
    return g0(std::integral_constant<int, NP>{}) + g1(std::integral_constant<int, C::PN + NP>{});
  } else {
    R acc = splat<R>(0.0f);
    sfor<C::PO>([&](auto a) {
      acc += m(std::integral_constant<int, C::idx(a, 0, NP)>{}) * g0(a);
      acc += m(std::integral_constant<int, C::idx(a, 1, NP)>{}) * g1(a);
    });
    return acc;
  }
}

// ------------------------------------------------------------------------------------- sweep context
// V = float: the value type of the state.
template <class V>
struct Ctx {
  int h;                // lane = crossing-bond configuration (lane-bit layout above)
  int kp;               // positions across the sweep
  int geo;              // GEO_* flags
  float labv;           // lane l < kt*kp: coset label of the site at (step l / kp, position l % kp)
  V mtv, mbv;           // lane l: entry l of the top / bottom side message (legs in sweep order)
  float p00, pe;        // depolarizing entries
  int biased;           // 1: entries from pib instead
  int pib[4];           // float bits of the Pauli probabilities by code x + 2z (I, X, Z, Y)
  int exp2;             // accumulated power-of-two scale (state values are true values * 2^-exp2)
};

__device__ __forceinline__ int bit(int h, int b) { return (h >> b) & 1; }
// lane-bit index of position i
__device__ __forceinline__ int pshift(int kp, int i) { return i == 0 ? 0 : (i == kp - 1 ? 1 : i + 1); }

template <class V>
struct QC {
  V cs, cf;   // coefficient of the lane's own value and of the partner lane's (crossing bit flipped)
};

// probability of Pauli code k (uniform) from the float bits of the four probabilities
__device__ __forceinline__ float pick4(const int* pib, int k) {
  const int a = (k & 1) ? pib[1] : pib[0];
  const int b = (k & 1) ? pib[3] : pib[2];
  return __int_as_float((k & 2) ? b : a);
}

// Coefficients of a qubit with coset label lb (code x + 2z) and orientation swap for a lane whose vertical
// bond parity is pv and output crossing bit ho; scaled by sc. The crossing parity (0 for the lane's own
// value, 1 for the partner's) flips x when swap and z otherwise; pv flips the other component. Depolarizing:
// the entry is p00 iff the flipped label is the identity.
__device__ __forceinline__ QC<float> qcoef(float p00, float pe, int biased, const int* pib, int lb, int swap, int pv,
                                           int ho, bool in_abs, bool out_abs, float sc) {
  QC<float> q;
  if (biased) {
    const int F = swap ? 1 : 2, G = F ^ 3;
    const float s0 = pick4(pib, lb), f0 = pick4(pib, lb ^ F), s1 = pick4(pib, lb ^ G), f1 = pick4(pib, lb ^ 3);
    q.cs = (pv ? s1 : s0) * sc;
    q.cf = (pv ? f1 : f0) * sc;
  } else {
    const int lx = lb & 1, lz = (lb >> 1) & 1;
    const int A = swap ? lx : lz, B = swap ? lz : lx;
    const bool m = (pv == B);
    const float hi = p00 * sc, lo = pe * sc;
    q.cs = (m && A == 0) ? hi : lo;
    q.cf = (m && A == 1) ? hi : lo;
  }
  if (in_abs) {   // the input crossing bit must be 0
    q.cs = ho ? 0.0f : q.cs;
    q.cf = ho ? q.cf : 0.0f;
  }
  if (out_abs) {   // the output crossing bit must be 0
    q.cs = ho ? 0.0f : q.cs;
    q.cf = ho ? 0.0f : q.cf;
  }
  return q;
}

template <class V>
__device__ __forceinline__ int label_at(const Ctx<V>& c, int t, int i) {
  return __float_as_int(readlane_f(c.labv, t * c.kp + i)) & 3;
}

// Coefficients of the qubit at (step t, position i).
template <class V>
__device__ __forceinline__ QC<V> qcoefs(const Ctx<V>& c, int t, int i, int swap, int pv, int ho, bool in_abs,
                                        bool out_abs, V sc) {
  const QC<float> q = qcoef(c.p00, c.pe, c.biased, c.pib, label_at(c, t, i), swap, pv, ho, in_abs, out_abs, tof(sc));
  return QC<V>{V{q.cs}, V{q.cf}};
}

// lane mask of the checks of a column (q0t: its site 0 is a qubit)
template <class V>
__device__ __forceinline__ int check_lanes(const Ctx<V>& c, bool q0t) {
  int m = 0;
  for (int i = 0; i < c.kp; ++i)
    if (!(q0t ^ (i & 1))) m |= 1 << pshift(c.kp, i);
  return m;
}

// Sum over the variables of the checks whose out-leg leaves the grid (lane bits oa): the result sits at
// those bits = 0.
template <class V, int N>
__device__ __forceinline__ void project_out_edge(V (&Y)[N], const Ctx<V>& c, int oa) {
  for (int b = 1; b < 64; b <<= 1) {
    if (!(oa & b)) continue;
    const bool zero = (c.h & b) != 0;
    sfor<N>([&](auto e) {
      const V o = xchg_rt(Y[e], b);
      Y[e] = zero ? splat<V>(0.0f) : Y[e] + o;
    });
  }
}

// --------------------------------------------------------------------------------- column, kp >= 2
template <class V, int KT, bool TOP, bool BOT, bool Q00, bool BF, int T>
__device__ __forceinline__ void column_multi(const V (&X)[Cap<TOP, KT, T>::PO * Cap<BOT, KT, T>::PO],
                                             V (&Y)[Cap<TOP, KT, T>::PN * Cap<BOT, KT, T>::PN], Ctx<V>& c,
                                             V sc) {
  using CT = Cap<TOP, KT, T>;
  using CB = Cap<BOT, KT, T>;
  constexpr int PTO = CT::PO, PTN = CT::PN, PSO = CB::PO, PSN = CB::PN;
  constexpr bool Q0 = Q00 ^ (T & 1);   // site 0 of this column is a qubit
  const int h = c.h, kp = c.kp;
  const int swap = ((c.geo & GEO_SWAP0) ? 1 : 0) ^ (T & 1);
  const bool in_abs = (T == 0) && (c.geo & GEO_IN_EDGE);
  const bool out_abs = (T == KT - 1) && (c.geo & GEO_OUT_EDGE);
  const bool last_q = Q0 ^ ((kp - 1) & 1);   // the last position is a qubit
  // the pending scale goes into the first qubit transform of the column
  const V one = splat<V>(1.0f);
  const V sc0 = Q0 ? sc : one;
  const V sc1 = (!Q0 && kp >= 3) ? sc : one;
  const V scl = (!Q0 && kp == 2) ? sc : one;
  auto mt = [&](auto idx) { return readlane_v(c.mtv, idx); };
  auto mb = [&](auto idx) { return readlane_v(c.mbv, idx); };

  // ---- top cap + site 0 (lane bit 0)
  V Z[PTN * PSO];
  if constexpr (Q0) {
    const int ho = bit(h, 0), vo = bit(h, pshift(kp, 1));
    const QC<V> q0 = qcoefs(c, T, 0, swap, vo, ho, in_abs, out_abs, sc0);
    QC<V> q1 = qcoefs(c, T, 0, swap, vo ^ 1, ho, in_abs, out_abs, sc0);
    if (c.geo & GEO_TOP_EDGE) q1.cs = q1.cf = splat<V>(0.0f);
    if constexpr (BF && CT::kind == K_EQ && PTN == 4) {
      // T is the middle step (never the first or last), so no edge absorption depends on the lane's own bit
      static_assert(PTO % 2 == 0, "pairs of old cap values per MFMA");
      if (kp >= 3) {
        // coefficients uniform over each block of four lanes: fold them into A, B = (x, x') per old cap value
        bf4 A[PTO / 2];
        sfor<PTO / 2>([&](auto k) {
          float ao[2], ap[2];
          sfor<2>([&](auto u) {
            const float m0 = lane_get(c.mtv, CT::idx(2 * k + u, 0, 0) + (h & 3));
            const float m1 = lane_get(c.mtv, CT::idx(2 * k + u, 1, 0) + (h & 3));
            ao[u] = m0 * q0.cs + m1 * q1.cs;
            ap[u] = m0 * q0.cf + m1 * q1.cf;
          });
          A[k] = pk4(ao[0], ap[0], ao[1], ap[1]);
        });
        sfor<PSO>([&](auto s) {
          f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
          sfor<PTO / 2>([&](auto k) {
            const float x0 = X[(2 * k) * PSO + s], x1 = X[(2 * k + 1) * PSO + s];
            acc = mfma4b(A[k], pk4(x0, xchg<1>(x0), x1, xchg<1>(x1)), acc);
          });
          sfor<4>([&](auto n) { Z[n * PSO + s] = acc[(int)n]; });
        });
      } else {
        // FP32 transform per lane, BF16 contraction with the message: K = (a, v) for two old cap values
        bf4 A[PTO / 2];
        sfor<PTO / 2>([&](auto k) {
          A[k] = pk4(lane_get(c.mtv, CT::idx(2 * k, 0, 0) + (h & 3)), lane_get(c.mtv, CT::idx(2 * k, 1, 0) + (h & 3)),
                     lane_get(c.mtv, CT::idx(2 * k + 1, 0, 0) + (h & 3)),
                     lane_get(c.mtv, CT::idx(2 * k + 1, 1, 0) + (h & 3)));
        });
        sfor<PSO>([&](auto s) {
          f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
          sfor<PTO / 2>([&](auto k) {
            const V x0 = X[(2 * k) * PSO + s], xf0 = xchg<1>(x0);
            const V x1 = X[(2 * k + 1) * PSO + s], xf1 = xchg<1>(x1);
            acc = mfma4b(A[k], pk4(q0.cs * x0 + q0.cf * xf0, q1.cs * x0 + q1.cf * xf0, q0.cs * x1 + q0.cf * xf1,
                                   q1.cs * x1 + q1.cf * xf1), acc);
          });
          sfor<4>([&](auto n) { Z[n * PSO + s] = acc[(int)n]; });
        });
      }
    } else if constexpr (CT::kind == K_EQ && PTN == 4) {
      float mA[PTO][2];
      sfor<PTO>([&](auto a) {
        mA[a][0] = lane_get(c.mtv, CT::idx(a, 0, 0) + (h & 3));
        mA[a][1] = lane_get(c.mtv, CT::idx(a, 1, 0) + (h & 3));
      });
      sfor<PSO>([&](auto s) {
        f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
        sfor<PTO>([&](auto a) {
          const V x = X[a * PSO + s], xf = xchg<1>(x);
          acc = mfma4(mA[a][0], q0.cs * x + q0.cf * xf, acc);
          acc = mfma4(mA[a][1], q1.cs * x + q1.cf * xf, acc);
        });
        sfor<4>([&](auto n) { Z[n * PSO + s] = acc[(int)n]; });
      });
    } else if constexpr (CT::kind == K_EQ) {
      // old cap index outermost: the message entries of one a are uniform (scalar) operands, and X[a][.]
      // is dead once its partner values are formed
      sfor<PTO>([&](auto a) {
        sfor<PSO>([&](auto s) {
          const V x = X[a * PSO + s], xf = xchg<1>(x);
          const V y0 = q0.cs * x + q0.cf * xf, y1 = q1.cs * x + q1.cf * xf;
          sfor<PTN>([&](auto n) {
            V& z = Z[n * PSO + s];
            const V t = mt(std::integral_constant<int, CT::idx(a, 0, n)>{}) * y0;
            z = (a == 0) ? t : z + t;
            z += mt(std::integral_constant<int, CT::idx(a, 1, n)>{}) * y1;
          });
        });
      });
    } else {
      sfor<PSO>([&](auto s) {
        V y0[PTO], y1[PTO];
        sfor<PTO>([&](auto a) {
          const V x = X[a * PSO + s], xf = xchg<1>(x);
          y0[a] = q0.cs * x + q0.cf * xf;
          y1[a] = (CT::kind != K_NONE) ? q1.cs * x + q1.cf * xf : splat<V>(0.0f);
        });
        sfor<PTN>([&](auto n) {
          Z[n * PSO + s] = phi2<CT, n>([&](auto a) { return y0[a]; }, [&](auto a) { return y1[a]; }, mt);
        });
      });
    }
  } else {
    const bool v1 = !(c.geo & GEO_TOP_EDGE) && bit(h, 0);
    if constexpr (BF && CT::kind == K_EQ && PTN == 4) {
      // K = four old cap values per MFMA, one accumulator per value of the emitted bond (the check's bit v1)
      static_assert(PTO % 4 == 0, "quads of old cap values per MFMA");
      bf4 A0[PTO / 4], A1[PTO / 4];
      sfor<PTO / 4>([&](auto k) {
        float m[2][4];
        sfor<4>([&](auto u) {
          m[0][u] = lane_get(c.mtv, CT::idx(4 * k + u, 0, 0) + (h & 3));
          m[1][u] = lane_get(c.mtv, CT::idx(4 * k + u, 1, 0) + (h & 3));
        });
        A0[k] = pk4(m[0][0], m[0][1], m[0][2], m[0][3]);
        A1[k] = pk4(m[1][0], m[1][1], m[1][2], m[1][3]);
      });
      sfor<PSO>([&](auto s) {
        f4 acc0 = {0.0f, 0.0f, 0.0f, 0.0f}, acc1 = {0.0f, 0.0f, 0.0f, 0.0f};
        sfor<PTO / 4>([&](auto k) {
          const bf4 B = pk4(X[(4 * k) * PSO + s], X[(4 * k + 1) * PSO + s], X[(4 * k + 2) * PSO + s],
                            X[(4 * k + 3) * PSO + s]);
          acc0 = mfma4b(A0[k], B, acc0);
          acc1 = mfma4b(A1[k], B, acc1);
        });
        sfor<4>([&](auto n) { Z[n * PSO + s] = v1 ? acc1[(int)n] : acc0[(int)n]; });
      });
    } else if constexpr (CT::kind == K_EQ && PTN == 4) {
      float mA[PTO][2];
      sfor<PTO>([&](auto a) {
        mA[a][0] = lane_get(c.mtv, CT::idx(a, 0, 0) + (h & 3));
        mA[a][1] = lane_get(c.mtv, CT::idx(a, 1, 0) + (h & 3));
      });
      // the emitted bond equals the check's own bit v1: one accumulator per value of v1, unmasked operands,
      // and the lane keeps the one of its own v1 (the other's products never enter)
      sfor<PSO>([&](auto s) {
        f4 acc0 = {0.0f, 0.0f, 0.0f, 0.0f}, acc1 = {0.0f, 0.0f, 0.0f, 0.0f};
        sfor<PTO>([&](auto a) {
          const float x = X[a * PSO + s];
          acc0 = mfma4(mA[a][0], x, acc0);
          acc1 = mfma4(mA[a][1], x, acc1);
        });
        sfor<4>([&](auto n) { Z[n * PSO + s] = v1 ? acc1[(int)n] : acc0[(int)n]; });
      });
    } else if constexpr (CT::kind == K_EQ) {
      sfor<PTO>([&](auto a) {
        V ms[PTN];
        sfor<PTN>([&](auto n) {
          // both entries read unconditionally: a lane read cannot sit under a lane-dependent branch
          const V m0 = mt(std::integral_constant<int, CT::idx(a, 0, n)>{});
          const V m1 = mt(std::integral_constant<int, CT::idx(a, 1, n)>{});
          ms[n] = v1 ? m1 : m0;
        });
        sfor<PSO>([&](auto s) {
          sfor<PTN>([&](auto n) {
            const V t = ms[n] * X[a * PSO + s];
            Z[n * PSO + s] = (a == 0) ? t : Z[n * PSO + s] + t;
          });
        });
      });
    } else {
      sfor<PSO>([&](auto s) {
        sfor<PTN>([&](auto n) {
          const V z0 = phi<CT, n, 0>([&](auto a) { return X[a * PSO + s]; }, mt);
          const V z1 = phi<CT, n, 1>([&](auto a) { return X[a * PSO + s]; }, mt);
          Z[n * PSO + s] = v1 ? z1 : z0;
        });
      });
    }
  }

  // ---- middle qubits (positions 1 .. kp-2, lane bits 2 .. kp-1)
  sfor<4>([&](auto j) {
    constexpr int i = j + 1;
    if constexpr (Q0 ^ (i & 1)) {
      if (i <= kp - 2) {
        const int vi = bit(h, i == 1 ? 0 : i);
        const int vo = (i + 1 == kp - 1) ? bit(h, 1) : bit(h, i + 2);
        const QC<V> q = qcoefs(c, T, i, swap, vi ^ vo, bit(h, i + 1), in_abs, out_abs, i == 1 ? sc1 : one);
        sfor<PTN * PSO>([&](auto e) {
          const V zx = xchg<(2 << i)>(Z[e]);
          Z[e] = fmav(q.cf, zx, q.cs * Z[e]);
        });
      }
    }
  });

  // ---- bottom cap + last site (lane bit 1)
  if (last_q) {
    const int ho = bit(h, 1), vi = bit(h, pshift(kp, kp - 2));
    const QC<V> q0 = qcoefs(c, T, kp - 1, swap, vi, ho, in_abs, out_abs, scl);
    QC<V> q1 = qcoefs(c, T, kp - 1, swap, vi ^ 1, ho, in_abs, out_abs, scl);
    if (c.geo & GEO_BOT_EDGE) q1.cs = q1.cf = splat<V>(0.0f);
    if constexpr (BF && CB::kind == K_EQ && PSN == 4) {
      // as for the top cap; with kp >= 3 the coefficients depend on lane bit kp-1 >= 2 only (vi)
      static_assert(PSO % 2 == 0, "pairs of old cap values per MFMA");
      if (kp >= 3) {
        bf4 A[PSO / 2];
        sfor<PSO / 2>([&](auto k) {
          float ao[2], ap[2];
          sfor<2>([&](auto u) {
            const float m0 = lane_get(c.mbv, CB::idx(2 * k + u, 0, 0) + (h & 3));
            const float m1 = lane_get(c.mbv, CB::idx(2 * k + u, 1, 0) + (h & 3));
            ao[u] = m0 * q0.cs + m1 * q1.cs;
            ap[u] = m0 * q0.cf + m1 * q1.cf;
          });
          A[k] = pk4(ao[0], ap[0], ao[1], ap[1]);
        });
        sfor<PTN>([&](auto n) {
          f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
          sfor<PSO / 2>([&](auto k) {
            const float z0 = Z[n * PSO + 2 * k], z1 = Z[n * PSO + 2 * k + 1];
            acc = mfma4b(A[k], pk4(z0, xchg<2>(z0), z1, xchg<2>(z1)), acc);
          });
          sfor<4>([&](auto sp) { Y[n * PSN + sp] = acc[(int)sp]; });
        });
      } else {
        bf4 A[PSO / 2];
        sfor<PSO / 2>([&](auto k) {
          A[k] = pk4(lane_get(c.mbv, CB::idx(2 * k, 0, 0) + (h & 3)), lane_get(c.mbv, CB::idx(2 * k, 1, 0) + (h & 3)),
                     lane_get(c.mbv, CB::idx(2 * k + 1, 0, 0) + (h & 3)),
                     lane_get(c.mbv, CB::idx(2 * k + 1, 1, 0) + (h & 3)));
        });
        sfor<PTN>([&](auto n) {
          f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
          sfor<PSO / 2>([&](auto k) {
            const V z0 = Z[n * PSO + 2 * k], zf0 = xchg<2>(z0);
            const V z1 = Z[n * PSO + 2 * k + 1], zf1 = xchg<2>(z1);
            acc = mfma4b(A[k], pk4(q0.cs * z0 + q0.cf * zf0, q1.cs * z0 + q1.cf * zf0, q0.cs * z1 + q0.cf * zf1,
                                   q1.cs * z1 + q1.cf * zf1), acc);
          });
          sfor<4>([&](auto sp) { Y[n * PSN + sp] = acc[(int)sp]; });
        });
      }
    } else if constexpr (CB::kind == K_EQ && PSN == 4) {
      float mB[PSO][2];
      sfor<PSO>([&](auto b) {
        mB[b][0] = lane_get(c.mbv, CB::idx(b, 0, 0) + (h & 3));
        mB[b][1] = lane_get(c.mbv, CB::idx(b, 1, 0) + (h & 3));
      });
      sfor<PTN>([&](auto n) {
        f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
        sfor<PSO>([&](auto b) {
          const float z = Z[n * PSO + b], zf = xchg<2>(z);
          acc = mfma4(mB[b][0], q0.cs * z + q0.cf * zf, acc);
          acc = mfma4(mB[b][1], q1.cs * z + q1.cf * zf, acc);
        });
        sfor<4>([&](auto sp) { Y[n * PSN + sp] = acc[(int)sp]; });
      });
    } else if constexpr (CB::kind == K_EQ) {
      sfor<PSO>([&](auto b) {
        sfor<PTN>([&](auto n) {
          const V z = Z[n * PSO + b], zf = xchg<2>(z);
          const V y0 = q0.cs * z + q0.cf * zf, y1 = q1.cs * z + q1.cf * zf;
          sfor<PSN>([&](auto sp) {
            V& y = Y[n * PSN + sp];
            const V t = mb(std::integral_constant<int, CB::idx(b, 0, sp)>{}) * y0;
            y = (b == 0) ? t : y + t;
            y += mb(std::integral_constant<int, CB::idx(b, 1, sp)>{}) * y1;
          });
        });
      });
    } else {
      sfor<PTN>([&](auto n) {
        V y0[PSO], y1[PSO];
        sfor<PSO>([&](auto b) {
          const V z = Z[n * PSO + b], zf = xchg<2>(z);
          y0[b] = q0.cs * z + q0.cf * zf;
          y1[b] = (CB::kind != K_NONE) ? q1.cs * z + q1.cf * zf : splat<V>(0.0f);
        });
        sfor<PSN>([&](auto sp) {
          Y[n * PSN + sp] = phi2<CB, sp>([&](auto b) { return y0[b]; }, [&](auto b) { return y1[b]; }, mb);
        });
      });
    }
  } else {
    const bool v1 = !(c.geo & GEO_BOT_EDGE) && bit(h, 1);
    if constexpr (BF && CB::kind == K_EQ && PSN == 4) {
      static_assert(PSO % 4 == 0, "quads of old cap values per MFMA");
      bf4 A0[PSO / 4], A1[PSO / 4];
      sfor<PSO / 4>([&](auto k) {
        float m[2][4];
        sfor<4>([&](auto u) {
          m[0][u] = lane_get(c.mbv, CB::idx(4 * k + u, 0, 0) + (h & 3));
          m[1][u] = lane_get(c.mbv, CB::idx(4 * k + u, 1, 0) + (h & 3));
        });
        A0[k] = pk4(m[0][0], m[0][1], m[0][2], m[0][3]);
        A1[k] = pk4(m[1][0], m[1][1], m[1][2], m[1][3]);
      });
      sfor<PTN>([&](auto n) {
        f4 acc0 = {0.0f, 0.0f, 0.0f, 0.0f}, acc1 = {0.0f, 0.0f, 0.0f, 0.0f};
        sfor<PSO / 4>([&](auto k) {
          const bf4 B = pk4(Z[n * PSO + 4 * k], Z[n * PSO + 4 * k + 1], Z[n * PSO + 4 * k + 2], Z[n * PSO + 4 * k + 3]);
          acc0 = mfma4b(A0[k], B, acc0);
          acc1 = mfma4b(A1[k], B, acc1);
        });
        sfor<4>([&](auto sp) { Y[n * PSN + sp] = v1 ? acc1[(int)sp] : acc0[(int)sp]; });
      });
    } else if constexpr (CB::kind == K_EQ && PSN == 4) {
      float mB[PSO][2];
      sfor<PSO>([&](auto b) {
        mB[b][0] = lane_get(c.mbv, CB::idx(b, 0, 0) + (h & 3));
        mB[b][1] = lane_get(c.mbv, CB::idx(b, 1, 0) + (h & 3));
      });
      sfor<PTN>([&](auto n) {
        f4 acc0 = {0.0f, 0.0f, 0.0f, 0.0f}, acc1 = {0.0f, 0.0f, 0.0f, 0.0f};
        sfor<PSO>([&](auto b) {
          const float z = Z[n * PSO + b];
          acc0 = mfma4(mB[b][0], z, acc0);
          acc1 = mfma4(mB[b][1], z, acc1);
        });
        sfor<4>([&](auto sp) { Y[n * PSN + sp] = v1 ? acc1[(int)sp] : acc0[(int)sp]; });
      });
    } else if constexpr (CB::kind == K_EQ) {
      sfor<PSO>([&](auto b) {
        V ms[PSN];
        sfor<PSN>([&](auto sp) {
          const V m0 = mb(std::integral_constant<int, CB::idx(b, 0, sp)>{});
          const V m1 = mb(std::integral_constant<int, CB::idx(b, 1, sp)>{});
          ms[sp] = v1 ? m1 : m0;
        });
        sfor<PTN>([&](auto n) {
          sfor<PSN>([&](auto sp) {
            const V t = ms[sp] * Z[n * PSO + b];
            Y[n * PSN + sp] = (b == 0) ? t : Y[n * PSN + sp] + t;
          });
        });
      });
    } else {
      sfor<PTN>([&](auto n) {
        sfor<PSN>([&](auto sp) {
          const V y0 = phi<CB, sp, 0>([&](auto b) { return Z[n * PSO + b]; }, mb);
          const V y1 = phi<CB, sp, 1>([&](auto b) { return Z[n * PSO + b]; }, mb);
          Y[n * PSN + sp] = v1 ? y1 : y0;
        });
      });
    }
  }
  if (out_abs) project_out_edge(Y, c, check_lanes(c, Q0));
}

// --------------------------------------------------------------------------------- column, kp == 1
// The single site of the column meets both caps: a qubit sums both emitted bonds (the bottom one is kept
// as an extra index between the two cap steps), a check emits its own variable on both.
template <class V, int KT, bool TOP, bool BOT, bool Q00, int T>
__device__ __forceinline__ void column_single(const V (&Xin)[Cap<TOP, KT, T>::PO * Cap<BOT, KT, T>::PO],
                                              V (&Y)[Cap<TOP, KT, T>::PN * Cap<BOT, KT, T>::PN], Ctx<V>& c,
                                              V sc) {
  using CT = Cap<TOP, KT, T>;
  using CB = Cap<BOT, KT, T>;
  constexpr int PTO = CT::PO, PTN = CT::PN, PSO = CB::PO, PSN = CB::PN;
  constexpr bool Q0 = Q00 ^ (T & 1);
  const int h = c.h, ho = h & 1;
  const int swap = ((c.geo & GEO_SWAP0) ? 1 : 0) ^ (T & 1);
  const bool in_abs = (T == 0) && (c.geo & GEO_IN_EDGE);
  const bool out_abs = (T == KT - 1) && (c.geo & GEO_OUT_EDGE);
  auto mt = [&](auto idx) { return readlane_v(c.mtv, idx); };
  auto mb = [&](auto idx) { return readlane_v(c.mbv, idx); };
  V X[PTO * PSO];
  sfor<PTO * PSO>([&](auto e) { X[e] = Xin[e] * sc; });   // no qubit transform may follow: scale here
  if constexpr (Q0) {
    const V one = splat<V>(1.0f), zero = splat<V>(0.0f);
    V Z[2][PTN * PSO];   // [emitted bottom bond][np][s]
    sfor<2>([&](auto vb) {
      QC<V> q0 = qcoefs(c, T, 0, swap, vb, ho, in_abs, out_abs, one);       // emitted top bond 0
      QC<V> q1 = qcoefs(c, T, 0, swap, vb ^ 1, ho, in_abs, out_abs, one);   // emitted top bond 1
      if (c.geo & GEO_TOP_EDGE) q1.cs = q1.cf = zero;
      if (vb == 1 && (c.geo & GEO_BOT_EDGE)) q0.cs = q0.cf = q1.cs = q1.cf = zero;
      sfor<PSO>([&](auto s) {
        V y0[PTO], y1[PTO];
        sfor<PTO>([&](auto a) {
          const V x = X[a * PSO + s], xf = xchg<1>(x);
          y0[a] = q0.cs * x + q0.cf * xf;
          y1[a] = q1.cs * x + q1.cf * xf;
        });
        sfor<PTN>([&](auto n) {
          Z[vb][n * PSO + s] = phi2<CT, n>([&](auto a) { return y0[a]; }, [&](auto a) { return y1[a]; }, mt);
        });
      });
    });
    sfor<PTN>([&](auto n) {
      sfor<PSN>([&](auto sp) {
        Y[n * PSN + sp] =
            phi2<CB, sp>([&](auto b) { return Z[0][n * PSO + b]; }, [&](auto b) { return Z[1][n * PSO + b]; }, mb);
      });
    });
  } else {
    const bool vt = !(c.geo & GEO_TOP_EDGE) && ho, vb = !(c.geo & GEO_BOT_EDGE) && ho;
    V Z[PTN * PSO];
    sfor<PSO>([&](auto s) {
      sfor<PTN>([&](auto n) {
        const V z0 = phi<CT, n, 0>([&](auto a) { return X[a * PSO + s]; }, mt);
        const V z1 = phi<CT, n, 1>([&](auto a) { return X[a * PSO + s]; }, mt);
        Z[n * PSO + s] = vt ? z1 : z0;
      });
    });
    sfor<PTN>([&](auto n) {
      sfor<PSN>([&](auto sp) {
        const V y0 = phi<CB, sp, 0>([&](auto b) { return Z[n * PSO + b]; }, mb);
        const V y1 = phi<CB, sp, 1>([&](auto b) { return Z[n * PSO + b]; }, mb);
        Y[n * PSN + sp] = vb ? y1 : y0;
      });
    });
    if (out_abs) project_out_edge(Y, c, 1);
  }
}

// ------------------------------------------------------------------------------------------ the sweep
// Power-of-two rescale of a state with squared norm ss: returns the factor to apply and accumulates its
// exponent.
template <class V>
__device__ __forceinline__ V pow2_scale(float ss, Ctx<V>& c) {
  const int e = (ss > 0.0f && ss < INFINITY) ? (__builtin_amdgcn_frexp_expf(ss) >> 1) : 0;
  c.exp2 += e;
  return V{__builtin_amdgcn_ldexpf(1.0f, -e)};
}

// Absorb columns T .. KT-1 into the state X (pending scale sc); returns the final state of this lane.
template <class V, int KT, bool TOP, bool BOT, bool SINGLE, bool Q00, bool BF, int T>
__device__ __forceinline__ V run(const V (&X)[Cap<TOP, KT, T>::PO * Cap<BOT, KT, T>::PO], Ctx<V>& c, V sc) {
  constexpr int NY = Cap<TOP, KT, T>::PN * Cap<BOT, KT, T>::PN;
  V Y[NY];
  if constexpr (SINGLE) column_single<V, KT, TOP, BOT, Q00, T>(X, Y, c, sc);
  else column_multi<V, KT, TOP, BOT, Q00, BF, T>(X, Y, c, sc);
  if constexpr (T + 1 < KT) {
    if constexpr (T & 1) {
      float ss = 0.0f;
      sfor<NY>([&](auto e) { ss += tof(Y[e]) * tof(Y[e]); });
      return run<V, KT, TOP, BOT, SINGLE, Q00, BF, T + 1>(Y, c, pow2_scale(wave_sum(ss), c));
    } else {
      return run<V, KT, TOP, BOT, SINGLE, Q00, BF, T + 1>(Y, c, splat<V>(1.0f));
    }
  } else {
    return Y[0];
  }
}

// The whole sweep from the entering state x0 (one value per lane). SINGLE: one position across
// (kp == 1); Q00: the first site of the first column is a qubit; BF: the middle-site contractions in BF16.
template <class V, int KT, bool TOP, bool BOT, bool SINGLE, bool Q00, bool BF>
__device__ __forceinline__ V sweep(V x0, Ctx<V>& c) {
  const V X[1] = {x0};
  return run<V, KT, TOP, BOT, SINGLE, Q00, BF, 0>(X, c, splat<V>(1.0f));
}

}  // namespace wave
}  // namespace bbp
