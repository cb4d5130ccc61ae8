// sweep.hpp -- one column step of an in-block sweep in the check-pass-through formulation, evaluated
// sequentially on the host (float64) by the validation hook bbp_reference_update_host. The GPU kernels
// (wave_sweep.hpp) execute the same formulation with one wavefront per sweep.
//
// Structure used. Every bond of the coset network joins a qubit and a check, and a check is a COPY tensor,
// so a bond always carries the value of the check it touches. In a column of the sweep the sites alternate
// qubit / check: a check passes its crossing-bond value straight through (its in- and out-legs and both
// vertical bonds all carry its own variable), and a qubit maps its crossing-bond value h_i to h'_i with the
// coefficient T(up, h_i, down, h'_i), where up / down are the variables of the checks above and below --
// bits of the boundary state that the column does not change. The column is therefore a product of
// commuting 2x2 transforms, one per qubit row, conditioned on neighbouring bits; no vertical bond has to be
// carried through the column. Only at the ends of the column does a vertical bond meet a side message:
// there the message's cap site emits the bond value, which either equals the end check's variable or is
// summed against the end qubit.
//
// State layout: psi[n][h][s] at ((n * H) + h) * Ps + s; h = crossing-bond values, position 0 in the most
// significant of kp bits; n / s = the top / bottom cap indices in the open-leg reading of the side messages
// (bond j of a K-site message carries its first j legs for j <= K/2 and its last K-j legs otherwise).
//
// Pass 1 (A -> B): top cap + site 0 + all middle qubits. Work item = (n', s, h with the item's group bits
//   cleared); the group bits are those of site 0 (when it is a qubit) and of the middle qubits, so every
//   pair a transform couples lies inside one item.
// Pass 2 (B -> A): bottom cap + last site, then the sum over the variable of every check whose out-leg leaves
//   the grid.
// Checks whose in-leg leaves the grid (first column at the lattice edge) read the state with their bit
// cleared: their variable is free.
#pragma once
#include "geom.hpp"

namespace bbp {

enum : int { CAP_NONE = 0, CAP_F_LT, CAP_F_EQ, CAP_F_GT, CAP_B_GT, CAP_B_EQ, CAP_B_LT };

struct CapInfo {
  int kind;     // CAP_*
  int Pold;     // cap dimension before the site
  int Pnew;     // after
  int R2;       // 2^(K - K/2 - 1): stride of the legs after the middle site in the dense message
};

BBP_HD CapInfo cap_info(bool present, bool fwd, int K, int t) {
  CapInfo c;
  if (!present) { c.kind = CAP_NONE; c.Pold = 1; c.Pnew = 1; c.R2 = 1; return c; }
  const int D = K / 2;
  const int js = fwd ? t : K - 1 - t;
  c.R2 = 1 << (K - D - 1);
  if (fwd) {
    c.Pold = cap_dim(K, t);
    c.Pnew = cap_dim(K, t + 1);
    c.kind = (js < D) ? CAP_F_LT : (js == D) ? CAP_F_EQ : CAP_F_GT;
  } else {
    c.Pold = cap_dim(K, K - t);
    c.Pnew = cap_dim(K, K - t - 1);
    c.kind = (js > D) ? CAP_B_GT : (js == D) ? CAP_B_EQ : CAP_B_LT;
  }
  return c;
}

// Value of phi[np][v] = sum_n op[n][v][np] * psi[n] for one cap site, reading psi[n] through get(n).
// m: the dense side message (entry (v_0..v_{K-1}), first leg most significant).
template <class V, class Get>
BBP_HD V cap_phi(const CapInfo& c, const float* m, int np, int v, Get get) {
  switch (c.kind) {
    case CAP_NONE: return v == 0 ? get(0) : V(0);
    case CAP_F_LT: return v == (np & 1) ? get(np >> 1) : V(0);
    case CAP_F_EQ: {
      V acc = V(0);
      for (int a = 0; a < c.Pold; ++a) acc += V(m[(a * 2 + v) * c.R2 + np]) * get(a);
      return acc;
    }
    case CAP_F_GT: return get(v * c.Pnew + np);
    case CAP_B_GT: return (v == np / c.Pold) ? get(np % c.Pold) : V(0);
    case CAP_B_EQ: {
      V acc = V(0);
      for (int b = 0; b < c.Pold; ++b) acc += V(m[(np * 2 + v) * c.R2 + b]) * get(b);
      return acc;
    }
    default: return get(2 * np + v);   // CAP_B_LT
  }
}

// Per-column constants of a sweep.
struct Column {
  int kp, H;
  CapInfo top, bot;
  int q0;            // site 0 is a qubit
  int up_absent0;    // site 0's up leg leaves the grid
  int qlast;         // last site is a qubit
  int dn_absent_last;
  int single;        // kp == 1
  int gmask;         // group bits of pass 1
  int ng;            // number of group bits
  int g0, g1, g2;    // group bit masks, low to high (0 when unused)
  int m0, m1, m2;    // positions of the middle qubits (inside the group)
  int nmid;
  int in_absent;     // mask of check bits whose in-leg leaves the grid (free variables)
  int out_absent;    // mask of check bits whose out-leg leaves the grid (summed variables)
};

BBP_HD int pos_bit(int kp, int i) { return 1 << (kp - 1 - i); }

BBP_HD void site_flags(int frame, int L, int r, int c, int& a_up, int& a_in, int& a_dn, int& a_out) {
  const int au = (r == 0), al = (c == 0), ad = (r == L - 1), ar = (c == L - 1);
  switch (frame) {
    case FRAME_E: a_up = au; a_in = al; a_dn = ad; a_out = ar; break;
    case FRAME_W: a_up = au; a_in = ar; a_dn = ad; a_out = al; break;
    case FRAME_S: a_up = al; a_in = au; a_dn = ar; a_out = ad; break;
    default:      a_up = al; a_in = ad; a_dn = ar; a_out = au; break;
  }
}

BBP_HD void make_column(Column& col, int frame, int r0, int c0, int kr, int kc, int kt, int kp, int L, int t,
                        bool has_top, bool has_bot) {
  const bool fwd = (frame == FRAME_E || frame == FRAME_S);
  col.kp = kp;
  col.H = 1 << kp;
  col.top = cap_info(has_top, fwd, kt, t);
  col.bot = cap_info(has_bot, fwd, kt, t);
  col.single = (kp == 1);
  col.gmask = 0;
  col.ng = 0;
  col.nmid = 0;
  col.g0 = col.g1 = col.g2 = 0;
  col.m0 = col.m1 = col.m2 = 0;
  col.in_absent = 0;
  col.out_absent = 0;
  for (int i = 0; i < kp; ++i) {
    int r, c;
    frame_site(frame, r0, c0, kr, kc, t, i, r, c);
    int a_up, a_in, a_dn, a_out;
    site_flags(frame, L, r, c, a_up, a_in, a_dn, a_out);
    const int q = ((r + c) & 1) == 0;
    if (i == 0) { col.q0 = q; col.up_absent0 = a_up; }
    if (i == kp - 1) { col.qlast = q; col.dn_absent_last = a_dn; }
    if (!q) {
      if (a_in) col.in_absent |= pos_bit(kp, i);
      if (a_out) col.out_absent |= pos_bit(kp, i);
    }
    if (kp > 1 && q && i < kp - 1) {
      if (i > 0) {
        if (col.nmid == 0) col.m0 = i;
        else if (col.nmid == 1) col.m1 = i;
        else col.m2 = i;
        ++col.nmid;
      }
      col.gmask |= pos_bit(kp, i);
    }
  }
  // group bits in increasing bit order (scalars only: no dynamically indexed arrays on the device)
  for (int b = 0; b < kp; ++b)
    if (col.gmask & (1 << b)) {
      if (col.ng == 0) col.g0 = 1 << b;
      else if (col.ng == 1) col.g1 = 1 << b;
      else col.g2 = 1 << b;
      ++col.ng;
    }
}

// Pass 1 for one work item. T: frame tables of this column's sites (16 floats each, position-major).
// getA(n, h, s) returns the (scaled) input state; put(np, h, s, value) stores an output.
// For kp == 1 pass 1 stores phi[np][vt][h][s] instead (put(np * 2 + vt, h, s, value)).
template <class V, class GetA, class Put>
BBP_HD void pass1_item(const Column& col, const float* T, const float* mtop, int np, int hb, int s, GetA getA,
                       Put put) {
  const int kp = col.kp;
  auto src = [&](int n, int h) -> V { return getA(n, h & ~col.in_absent, s); };
  if (col.single) {
    for (int vt = 0; vt < 2; ++vt)
      for (int h = 0; h < 2; ++h)
        put(np * 2 + vt, h, s, cap_phi<V>(col.top, mtop, np, vt, [&](int n) { return src(n, h); }));
    return;
  }
  // register arrays below are indexed only with compile-time indices (fully unrolled, runtime guards)
  V val[8];
  const int ne = 1 << col.ng;
  const int b0 = pos_bit(kp, 0);
  const int g0 = col.g0, g1 = col.g1, g2 = col.g2;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    val[e] = V(0);
    if (e < ne) {
      const int h = hb | ((e & 1) ? g0 : 0) | ((e & 2) ? g1 : 0) | ((e & 4) ? g2 : 0);
      V out;
      if (col.q0) {
        // site 0 qubit: sum over the emitted top leg v and its own input bit
        const int vo = (h & pos_bit(kp, 1)) ? 1 : 0;
        const int ho = (h & b0) ? 1 : 0;
        out = V(0);
        for (int v = 0; v < 2; ++v)
          for (int hi = 0; hi < 2; ++hi) {
            const float coef = T[v * 8 + hi * 4 + vo * 2 + ho];
            if (coef == 0.0f) continue;
            const int hs = hi ? (h | b0) : (h & ~b0);
            out += V(coef) * cap_phi<V>(col.top, mtop, np, v, [&](int n) { return src(n, hs); });
          }
      } else {
        // site 0 check: the emitted top leg equals the check's variable (its own bit), unless the leg is absent
        const int v = col.up_absent0 ? 0 : ((h & b0) ? 1 : 0);
        out = cap_phi<V>(col.top, mtop, np, v, [&](int n) { return src(n, h); });
      }
      val[e] = out;
    }
  }
  // middle qubits: 2x2 transforms conditioned on the check bits above and below
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    if (j < col.nmid) {
      const int i = (j == 0) ? col.m0 : (j == 1) ? col.m1 : col.m2;
      const int bi = pos_bit(kp, i);
      const int vi = (hb & pos_bit(kp, i - 1)) ? 1 : 0;
      const int vo = (hb & pos_bit(kp, i + 1)) ? 1 : 0;
      const float* Ti = T + i * 16;
      const V c00 = V(Ti[vi * 8 + 0 * 4 + vo * 2 + 0]), c10 = V(Ti[vi * 8 + 1 * 4 + vo * 2 + 0]);
      const V c01 = V(Ti[vi * 8 + 0 * 4 + vo * 2 + 1]), c11 = V(Ti[vi * 8 + 1 * 4 + vo * 2 + 1]);
#pragma unroll
      for (int g = 0; g < 3; ++g) {
        const int gb = (g == 0) ? g0 : (g == 1) ? g1 : g2;
        if (g < col.ng && gb == bi) {
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            if (!(e & (1 << g)) && e < ne) {
              const V a = val[e], b = val[e | (1 << g)];
              val[e] = c00 * a + c10 * b;
              val[e | (1 << g)] = c01 * a + c11 * b;
            }
          }
        }
      }
    }
  }
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    if (e < ne) {
      const int h = hb | ((e & 1) ? g0 : 0) | ((e & 2) ? g1 : 0) | ((e & 4) ? g2 : 0);
      put(np, h, s, val[e]);
    }
  }
}

// Pass 2 for one output element (n, h, sp): bottom cap + last site, then the out-leg projections.
// getB(n, h, s) reads pass 1's output (for kp == 1: getB(np * 2 + vt, h, s)).
template <class V, class GetB>
BBP_HD V pass2_output(const Column& col, const float* T, const float* mbot, int n, int h, int sp, GetB getB) {
  const int kp = col.kp;
  if (h & col.out_absent) return V(0);
  const int bl = pos_bit(kp, kp - 1);
  const float* Tl = T + (kp - 1) * 16;
  const int noa = __builtin_popcount(col.out_absent);
  V total = V(0);
  for (int comb = 0; comb < (1 << noa); ++comb) {
    // deposit the bits of comb into the positions of the summed check variables
    int hh = h, k = 0;
    for (int b = 0; b < 6; ++b)
      if (col.out_absent & (1 << b)) { if (comb & (1 << k)) hh |= 1 << b; ++k; }
    V out = V(0);
    if (col.single) {
      const int ho = hh & 1;
      if (col.qlast) {
        for (int vt = 0; vt < 2; ++vt)
          for (int vb = 0; vb < 2; ++vb)
            for (int hi = 0; hi < 2; ++hi) {
              const float coef = Tl[vt * 8 + hi * 4 + vb * 2 + ho];
              if (coef == 0.0f) continue;
              out += V(coef) * cap_phi<V>(col.bot, mbot, sp, vb, [&](int s) { return getB(n * 2 + vt, hi, s); });
            }
      } else {
        const int vt = col.up_absent0 ? 0 : ho;
        const int vb = col.dn_absent_last ? 0 : ho;
        out = cap_phi<V>(col.bot, mbot, sp, vb, [&](int s) { return getB(n * 2 + vt, hh, s); });
      }
    } else if (col.qlast) {
      const int vi = (hh & pos_bit(kp, kp - 2)) ? 1 : 0;
      const int ho = (hh & bl) ? 1 : 0;
      for (int v = 0; v < 2; ++v)
        for (int hi = 0; hi < 2; ++hi) {
          const float coef = Tl[vi * 8 + hi * 4 + v * 2 + ho];
          if (coef == 0.0f) continue;
          const int hs = hi ? (hh | bl) : (hh & ~bl);
          out += V(coef) * cap_phi<V>(col.bot, mbot, sp, v, [&](int s) { return getB(n, hs, s); });
        }
    } else {
      const int v = col.dn_absent_last ? 0 : ((hh & bl) ? 1 : 0);
      out = cap_phi<V>(col.bot, mbot, sp, v, [&](int s) { return getB(n, hh, s); });
    }
    total += out;
  }
  return total;
}

}  // namespace bbp
