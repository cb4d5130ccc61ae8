// plan.cpp -- block plan and plan-time rank analysis of the blockBP decoder (host, C++17).
//
// Partition (Alg. 1, remark 1): block rows/columns of size k, the last one holding the remainder.
// Directed messages: for every block and every existing neighbour in the order E, W, S, N.
// Schedule (remark 8): blocks with (I+J) even update first, then the others.
//
// Rank analysis. The boundary state of an in-block sweep is compressed to bond chi after every column
// (Sec. III.A, III.D). The compression changes the state only where its Schmidt rank across a cut exceeds
// chi. Every entry of the (untruncated) boundary state is a polynomial with integer coefficients in the
// noise-table entries of the qubits and in the entries of the incoming messages, so its rank across a cut
// is at most the rank at a random point of the parameter space, with equality for all points off a
// proper algebraic subset. The plan evaluates every distinct sweep (same shape, position parity,
// neighbour pattern and frame) at random parameters modulo the prime 2^31-1 -- exact arithmetic, no
// tolerance -- with an independent random 2x2 noise table per qubit, and computes the rank of every cut
// whose dimensions both exceed chi by Gaussian elimination. If no cut can exceed chi, truncation is the
// identity for every syndrome, noise model and message, and the GPU contracts blocks exactly.
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>

#include "geom.hpp"
#include "sweep.hpp"
#include "trunc_shape.hpp"

namespace bbp {

namespace {

std::vector<std::pair<int, int>> splits(int L, int k) {
  std::vector<std::pair<int, int>> out;
  for (int s = 0; s < L; s += k) out.push_back({s, (s + k <= L) ? k : L - s});
  return out;
}

const int DI[4] = {0, 0, 1, -1};   // E, W, S, N
const int DJ[4] = {1, -1, 0, 0};

// ---------------------------------------------------------------------------------------------------
// Arithmetic for the generic sweep: exact modular ints and float64.
struct ModP {
  using V = uint64_t;
  static constexpr uint64_t P = 2147483647ull;
  static V zero() { return 0; }
  static V one() { return 1; }
  static V add(V a, V b) { V s = a + b; return s >= P ? s - P : s; }
  static V mul(V a, V b) { return (a * b) % P; }
};
struct F64 {
  using V = double;
  static V zero() { return 0.0; }
  static V one() { return 1.0; }
  static V add(V a, V b) { return a + b; }
  static V mul(V a, V b) { return a * b; }
};

// One block sweep with the device's index arithmetic. tables[(t*kp+i)*16 + e]; init/top/bot are dense
// messages (nullptr when absent). After every column `col(t, A, Pt, H, Ps)` is called.
template <class Fld, class Col>
void generic_sweep(const SweepDesc& s, const typename Fld::V* tables, const typename Fld::V* init,
                   const typename Fld::V* top, const typename Fld::V* bot,
                   std::vector<typename Fld::V>& A, Col&& col) {
  using V = typename Fld::V;
  const int kt = s.kt, kp = s.kp, H = 1 << kp, K = kt, D = K / 2;
  const bool fwd = (s.frame == FRAME_E || s.frame == FRAME_S);
  std::vector<V> B;
  A.assign(H, Fld::zero());
  if (init) for (int h = 0; h < H; ++h) A[h] = init[h];
  else A[0] = Fld::one();
  int Pt = 1, Ps = 1;
  for (int t = 0; t < kt; ++t) {
    const int js = fwd ? t : kt - 1 - t;
    const int bnew = fwd ? t + 1 : kt - 1 - t;
    const int Ptn = top ? cap_dim(K, bnew) : 1;
    const int Psn = bot ? cap_dim(K, bnew) : 1;
    const int HS = H * Ps;
    const int R2 = 1 << (K - D - 1);
    // top cap: B[(n'*2+v)*HS + hs]
    B.assign((size_t)Ptn * 2 * HS, Fld::zero());
    for (int np = 0; np < Ptn; ++np)
      for (int v = 0; v < 2; ++v)
        for (int hs = 0; hs < HS; ++hs) {
          V val = Fld::zero();
          if (!top) {
            if (v == 0) val = A[hs];
          } else if (fwd) {
            if (js < D) { if (v == (np & 1)) val = A[(size_t)(np >> 1) * HS + hs]; }
            else if (js == D) {
              for (int a = 0; a < (1 << D); ++a)
                val = Fld::add(val, Fld::mul(top[(a * 2 + v) * R2 + np], A[(size_t)a * HS + hs]));
            } else { const int R = 1 << (K - js - 1); val = A[(size_t)(v * R + np) * HS + hs]; }
          } else {
            if (js > D) { const int R = 1 << (K - js - 1); if (v == np / R) val = A[(size_t)(np % R) * HS + hs]; }
            else if (js == D) {
              for (int b = 0; b < R2; ++b)
                val = Fld::add(val, Fld::mul(top[(np * 2 + v) * R2 + b], A[(size_t)b * HS + hs]));
            } else { val = A[(size_t)(2 * np + v) * HS + hs]; }
          }
          B[((size_t)np * 2 + v) * HS + hs] = val;
        }
    // sites, top to bottom: in-place 4x4 transforms on (v, h_i)
    for (int i = 0; i < kp; ++i) {
      const V* T = tables + (size_t)(t * kp + i) * 16;
      const int hbit = 1 << (kp - 1 - i);
      for (int np = 0; np < Ptn; ++np)
        for (int h = 0; h < H; ++h) {
          if (h & hbit) continue;
          for (int sb = 0; sb < Ps; ++sb) {
            size_t idx[4];
            V in[4];
            for (int q = 0; q < 4; ++q) {
              const int v = q >> 1, hb = q & 1;
              idx[q] = (((size_t)np * 2 + v) * H + (h | (hb ? hbit : 0))) * Ps + sb;
              in[q] = B[idx[q]];
            }
            for (int o = 0; o < 4; ++o) {       // o = vo*2 + ho
              V acc = Fld::zero();
              for (int q = 0; q < 4; ++q) acc = Fld::add(acc, Fld::mul(T[q * 4 + o], in[q]));
              B[idx[o]] = acc;
            }
          }
        }
    }
    // bottom cap: A[(n'*H + h)*Psn + s']
    A.assign((size_t)Ptn * H * Psn, Fld::zero());
    auto Bat = [&](int np, int v, int h, int sb) -> V { return B[(((size_t)np * 2 + v) * H + h) * Ps + sb]; };
    for (int np = 0; np < Ptn; ++np)
      for (int h = 0; h < H; ++h)
        for (int sp = 0; sp < Psn; ++sp) {
          V val = Fld::zero();
          if (!bot) {
            val = Bat(np, 0, h, 0);
          } else if (fwd) {
            if (js < D) val = Bat(np, sp & 1, h, sp >> 1);
            else if (js == D) {
              for (int a = 0; a < (1 << D); ++a)
                for (int v = 0; v < 2; ++v)
                  val = Fld::add(val, Fld::mul(bot[(a * 2 + v) * R2 + sp], Bat(np, v, h, a)));
            } else { const int R = 1 << (K - js - 1); for (int v = 0; v < 2; ++v) val = Fld::add(val, Bat(np, v, h, v * R + sp)); }
          } else {
            if (js > D) { const int R = 1 << (K - js - 1); val = Bat(np, sp / R, h, sp % R); }
            else if (js == D) {
              for (int b = 0; b < R2; ++b)
                for (int v = 0; v < 2; ++v)
                  val = Fld::add(val, Fld::mul(bot[(sp * 2 + v) * R2 + b], Bat(np, v, h, b)));
            } else { for (int v = 0; v < 2; ++v) val = Fld::add(val, Bat(np, v, h, 2 * sp + v)); }
          }
          A[((size_t)np * H + h) * Psn + sp] = val;
        }
    Pt = Ptn;
    Ps = Psn;
    col(t, A, Pt, H, Ps);
  }
}

int rank_modp(std::vector<uint64_t> M, int rows, int cols) {
  const uint64_t P = ModP::P;
  auto inv = [&](uint64_t a) {
    uint64_t r = 1, e = P - 2;
    while (e) { if (e & 1) r = r * a % P; a = a * a % P; e >>= 1; }
    return r;
  };
  int rank = 0;
  for (int c = 0; c < cols && rank < rows; ++c) {
    int piv = -1;
    for (int r = rank; r < rows; ++r) if (M[(size_t)r * cols + c]) { piv = r; break; }
    if (piv < 0) continue;
    if (piv != rank) for (int k = 0; k < cols; ++k) std::swap(M[(size_t)piv * cols + k], M[(size_t)rank * cols + k]);
    const uint64_t iv = inv(M[(size_t)rank * cols + c]);
    for (int k = c; k < cols; ++k) M[(size_t)rank * cols + k] = M[(size_t)rank * cols + k] * iv % P;
    for (int r = 0; r < rows; ++r) {
      if (r == rank) continue;
      const uint64_t f = M[(size_t)r * cols + c];
      if (!f) continue;
      for (int k = c; k < cols; ++k)
        M[(size_t)r * cols + k] = (M[(size_t)r * cols + k] + (P - f) * M[(size_t)rank * cols + k]) % P;
    }
    ++rank;
  }
  return rank;
}

struct Rng {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  uint64_t modp() { return 1 + next() % (ModP::P - 1); }
};

// Largest generic rank over the cuts of sweep s that could exceed chi (0 if none can).
int analyse_sweep(const Plan& p, const SweepDesc& s, Rng& rng) {
  const int kt = s.kt, kp = s.kp;
  std::vector<uint64_t> tables((size_t)kt * kp * 16);
  for (int t = 0; t < kt; ++t)
    for (int i = 0; i < kp; ++i) {
      int r, c;
      frame_site(s.frame, s.r0, s.c0, s.kr, s.kc, t, i, r, c);
      // a generic noise table per qubit: mark the four entries, then substitute random residues
      float marks[4] = {1.0f, 2.0f, 3.0f, 4.0f};
      float T[16];
      site_table(s.frame, p.L, r, c, 0, marks, T);
      uint64_t vals[4] = {rng.modp(), rng.modp(), rng.modp(), rng.modp()};
      for (int e = 0; e < 16; ++e) {
        const bool qubit = ((r + c) & 1) == 0;
        uint64_t v = 0;
        if (T[e] != 0.0f) v = qubit ? vals[(int)T[e] - 1] : 1;
        tables[(size_t)(t * kp + i) * 16 + e] = v;
      }
    }
  auto rand_msg = [&](int K) {
    std::vector<uint64_t> m((size_t)1 << K);
    for (auto& x : m) x = rng.modp();
    return m;
  };
  std::vector<uint64_t> mi, mt, mb;
  if (s.msg_init >= 0) mi = rand_msg(kp);
  if (s.msg_top >= 0) mt = rand_msg(kt);
  if (s.msg_bot >= 0) mb = rand_msg(kt);
  int worst = 0;
  std::vector<uint64_t> A;
  generic_sweep<ModP>(s, tables.data(), mi.empty() ? nullptr : mi.data(), mt.empty() ? nullptr : mt.data(),
                      mb.empty() ? nullptr : mb.data(), A,
                      [&](int, const std::vector<uint64_t>& St, int Pt, int H, int Ps) {
                        const int total = Pt * H * Ps;
                        for (int cut = 1; cut <= kp + 1; ++cut) {
                          const int left = Pt << (cut - 1);
                          const int right = total / left;
                          if (left <= p.chi || right <= p.chi) continue;
                          std::vector<uint64_t> M(St.begin(), St.begin() + total);
                          int rk;
                          if (left <= right) rk = rank_modp(M, left, right);
                          else {
                            std::vector<uint64_t> Mt((size_t)total);
                            for (int a = 0; a < left; ++a)
                              for (int b = 0; b < right; ++b) Mt[(size_t)b * left + a] = M[(size_t)a * right + b];
                            rk = rank_modp(Mt, right, left);
                          }
                          if (rk > worst) worst = rk;
                        }
                      });
  return worst;
}

// Algorithmic flops of one block sweep in the check-pass-through formulation (a multiply-add counts 2):
// per column, with PT / PS the top / bottom cap dimensions before (o) and after (n) the column and H the
// crossing-bond configurations,
//   end qubit (site 0 against the top cap, last site against the bottom cap): each emitted-bond value v
//     the cap uses needs y_v = T(own) x + T(partner) x' (2 multiply-adds) per input entry -- both v for a
//     cap that appends the bond or contracts the dense core, one for a cap that strips it (plus one add
//     per output), only v = 0 without a cap;
//   dense-core contraction (middle site of a side message): sum over (old cap index, v) per output entry,
//     with both v for a qubit, the check's own v for a check;
//   middle qubit: 2 multiply-adds per state entry; checks and the routing caps move data only.
// The closing work (normalisation, damping and distance term, or the closing overlap) is 10 flops per
// configuration. Normalisation inside the sweep (a range device) is not counted.
double sweep_flops(const Plan& p, const SweepDesc& s) {
  (void)p;
  const int kt = s.kt, kp = s.kp, D = kt / 2;
  const double H = (double)(1 << kp);
  auto cdim = [](int K, int j) { return (double)(1 << std::min(j, K - j)); };
  const bool top = s.msg_top >= 0, bot = s.msg_bot >= 0, q00 = (s.geo & GEO_Q00) != 0;
  double f = 0.0;
  for (int t = 0; t < kt; ++t) {
    const bool q0 = q00 ^ (t & 1), ql = q0 ^ (((kp - 1) & 1) != 0);
    const int kind = t < D ? 1 : (t == D ? 2 : 3);   // 1 append, 2 dense core, 3 strip
    const double PTo = top ? cdim(kt, t) : 1, PTn = top ? cdim(kt, t + 1) : 1;
    const double PSo = bot ? cdim(kt, t) : 1, PSn = bot ? cdim(kt, t + 1) : 1;
    const double in = PTo * PSo * H, z = PTn * PSo * H, out = PTn * PSn * H;
    // top cap + site 0
    if (q0) {
      if (!top) f += 4.0 * in;
      else if (kind == 1) f += 8.0 * in;
      else if (kind == 3) f += 4.0 * in + z;
      else f += 8.0 * in + 4.0 * PTo * z;
    } else if (top && kind == 2) {
      f += 2.0 * PTo * z;
    }
    // middle qubits: positions 1 .. kp-2 of the qubit parity
    int nmid = 0;
    for (int i = 1; i <= kp - 2; ++i) nmid += (q0 ^ ((i & 1) != 0)) ? 1 : 0;
    f += 4.0 * nmid * z;
    // bottom cap + last site (for one position across, the single site counts once, at the top)
    if (kp > 1 && ql) {
      if (!bot) f += 4.0 * z;
      else if (kind == 1) f += 8.0 * z;
      else if (kind == 3) f += 4.0 * z + out;
      else f += 8.0 * z + 4.0 * PSo * out;
    } else if (bot && kind == 2) {
      f += 2.0 * PSo * out;
    }
  }
  f += 10.0 * H;
  return f;
}

// Algorithmic flops of one sweep in the truncating kernel (bonds padded to 2 chi_max = 32 before the
// compression, as the kernel executes them): per column, every crossing site and the top cap is factored by
// Householder QR of a 64 x 32 matrix (2 m n^2 - 2 n^3 / 3), the reflections are applied to the 32 x 16 carry
// (4 (64 - j) 16 per reflection j), and every site below the top cap takes one-sided Jacobi SVD of a 32 x 32
// matrix, counted at six sweeps of 496 rotations (a 2 x 32 product and a 4 x 32 rotation each); the absorption
// products (R times the column tensor) add 2 x 32 x 32 x 64 per site. Narrow sweeps (trunc_shape.hpp) execute
// the nonzero blocks only: QR of 32 x 16, reflections on the carry's 32 x 8 block, 120 rotations of 16-entry
// rows per Jacobi sweep, absorption into 32 x 16 from 16 terms.
double trunc_sweep_flops(const SweepDesc& s, int chi) {
  double qr, apply = 0.0, svd, absorb;
  if (trunc_narrow(chi, s.kt, s.kp)) {
    // the 32 x 16 site matrix with 16 reflections, the reflections on the carry's 32 x 8 block, 16 Jacobi rows
    // of 2 x 8 nonzero entries, absorption into the 32 x 16 matrix from 16 terms
    qr = 0.0;
    for (int j = 0; j < 16; ++j) qr += 4.0 * (32 - j) * (16 - j);
    for (int j = 0; j < 16; ++j) apply += 4.0 * (32 - j) * 8;
    svd = 6.0 * 120 * (2.0 * 16 + 6.0 * 16);
    absorb = 2.0 * 16 * 32 * 16;
  } else {
    qr = 2.0 * 64 * 32 * 32 - 2.0 * 32 * 32 * 32 / 3.0;
    for (int j = 0; j < 32; ++j) apply += 4.0 * (64 - j) * 16;
    svd = 6.0 * 496 * (2.0 * 32 + 6.0 * 32);
    absorb = 2.0 * 32 * 32 * 64;
  }
  return (double)s.kt * (s.kp + 1) * (qr + apply + svd + absorb);
}

}  // namespace

Plan make_plan(int d, int kr, int kc, int chi) {
  Plan p;
  p.d = d;
  p.L = 2 * d - 1;
  p.kr = kr;
  p.kc = kc;
  p.chi = chi;
  auto rs = splits(p.L, kr), cs = splits(p.L, kc);
  p.nI = (int)rs.size();
  p.nJ = (int)cs.size();
  for (auto& x : rs) { p.row0.push_back(x.first); p.rowsz.push_back(x.second); }
  for (auto& x : cs) { p.col0.push_back(x.first); p.colsz.push_back(x.second); }
  p.nblocks = p.nI * p.nJ;
  std::map<std::pair<int, int>, int> id;
  for (int I = 0; I < p.nI; ++I)
    for (int J = 0; J < p.nJ; ++J)
      for (int dir = 0; dir < 4; ++dir) {
        const int I2 = I + DI[dir], J2 = J + DJ[dir];
        if (I2 < 0 || I2 >= p.nI || J2 < 0 || J2 >= p.nJ) continue;
        const int src = I * p.nJ + J, dst = I2 * p.nJ + J2;
        id[{src, dst}] = (int)p.edge_src.size();
        p.edge_src.push_back(src);
        p.edge_dst.push_back(dst);
        p.edge_dir.push_back(dir);
        const int K = (dir <= 1) ? p.rowsz[I] : p.colsz[J];
        p.edge_len.push_back(K);
        if (K > p.max_msg_len) p.max_msg_len = K;
      }
  p.M = (int)p.edge_src.size();
  auto msg = [&](int I, int J, int I2, int J2) -> int {
    if (I2 < 0 || I2 >= p.nI || J2 < 0 || J2 >= p.nJ) return -1;
    return id[{I2 * p.nJ + J2, I * p.nJ + J}];
  };
  auto make = [&](int I, int J, int frame, int out) {
    SweepDesc s;
    std::memset(&s, 0, sizeof(s));
    s.r0 = p.row0[I];
    s.c0 = p.col0[J];
    s.kr = p.rowsz[I];
    s.kc = p.colsz[J];
    s.frame = frame;
    const bool ew = frame <= 1;
    s.kt = ew ? s.kc : s.kr;
    s.kp = ew ? s.kr : s.kc;
    s.msg_out = out;
    const int opp[4] = {1, 0, 3, 2};
    const int o = opp[frame];
    s.msg_init = msg(I, J, I + DI[o], J + DJ[o]);
    if (ew) {
      s.msg_top = msg(I, J, I - 1, J);
      s.msg_bot = msg(I, J, I + 1, J);
    } else {
      s.msg_top = msg(I, J, I, J - 1);
      s.msg_bot = msg(I, J, I, J + 1);
    }
    s.msg_close = (out < 0) ? msg(I, J, I + DI[frame], J + DJ[frame]) : -1;
    s.block = I * p.nJ + J;
    // geometry flags, uniform over the sweep's steps
    int r, c, a_up, a_in, a_dn, a_out;
    frame_site(frame, s.r0, s.c0, s.kr, s.kc, 0, 0, r, c);
    site_flags(frame, p.L, r, c, a_up, a_in, a_dn, a_out);
    s.geo = ((((r + c) & 1) == 0) ? GEO_Q00 : 0) | ((ew ? (c & 1) : !(r & 1)) ? GEO_SWAP0 : 0) |
            (a_up ? GEO_TOP_EDGE : 0) | (a_in ? GEO_IN_EDGE : 0);
    frame_site(frame, s.r0, s.c0, s.kr, s.kc, 0, s.kp - 1, r, c);
    site_flags(frame, p.L, r, c, a_up, a_in, a_dn, a_out);
    if (a_dn) s.geo |= GEO_BOT_EDGE;
    frame_site(frame, s.r0, s.c0, s.kr, s.kc, s.kt - 1, 0, r, c);
    site_flags(frame, p.L, r, c, a_up, a_in, a_dn, a_out);
    if (a_out) s.geo |= GEO_OUT_EDGE;
    return s;
  };
  for (int e = 0; e < p.M; ++e) {
    const int I = p.edge_src[e] / p.nJ, J = p.edge_src[e] % p.nJ;
    SweepDesc s = make(I, J, p.edge_dir[e], e);
    s.flops = (float)sweep_flops(p, s);
    p.round[(I + J) & 1].push_back(s);
    p.flops_iter += s.flops;
  }
  for (int I = 0; I < p.nI; ++I)
    for (int J = 0; J < p.nJ; ++J) {
      SweepDesc s = make(I, J, FRAME_E, -1);
      s.flops = (float)sweep_flops(p, s);
      p.bethe.push_back(s);
      p.flops_bethe += s.flops;
    }
  for (int e = 0; e < p.M; ++e)
    if (p.edge_src[e] < p.edge_dst[e]) {
      p.pair_ids.push_back(e);
      p.pair_ids.push_back(id[{p.edge_dst[e], p.edge_src[e]}]);
    }

  // rank analysis, once per distinct sweep class; a sweep whose boundary state can exceed chi is marked for
  // the truncating kernel, and so is every sweep of a plan with blocks wider than 6 (the dense kernels hold
  // at most 64 crossing configurations)
  const int kmax = std::max(*std::max_element(p.rowsz.begin(), p.rowsz.end()),
                            *std::max_element(p.colsz.begin(), p.colsz.end()));
  p.mstride = 1 << std::max(6, kmax);
  std::map<std::tuple<int, int, int, int, int, int, int, int>, int> seen;
  Rng rng{0x5eed0fb10cb9ull};
  int worst = 0;
  auto visit = [&](SweepDesc& s) {
    auto key = std::make_tuple(s.kr, s.kc, s.r0 & 1, s.c0 & 1, s.frame, s.msg_init >= 0, s.msg_top >= 0,
                               (s.msg_bot >= 0) * 2 + (s.r0 + s.kr == p.L) * 4 + (s.c0 + s.kc == p.L) * 8 +
                                   (s.r0 == 0) * 16 + (s.c0 == 0) * 32);
    auto it = seen.find(key);
    int r;
    if (it != seen.end()) {
      r = it->second;
    } else {
      r = analyse_sweep(p, s, rng);
      r = std::max(r, analyse_sweep(p, s, rng));   // two independent random points
      seen[key] = r;
    }
    worst = std::max(worst, r);
    s.trunc = (r > chi || kmax > 6) ? (trunc_narrow(chi, s.kt, s.kp) ? 2 : 1) : 0;
    if (s.trunc) {
      s.flops = (float)trunc_sweep_flops(s, chi);
      p.trunc_sweeps += 1;
    }
    p.max_kp = std::max(p.max_kp, s.kp);
  };
  for (int c = 0; c < 2; ++c) for (auto& s : p.round[c]) visit(s);
  for (auto& s : p.bethe) visit(s);
  p.flops_iter = 0.0;
  p.flops_bethe = 0.0;
  for (int c = 0; c < 2; ++c) for (auto& s : p.round[c]) p.flops_iter += s.flops;
  for (auto& s : p.bethe) p.flops_bethe += s.flops;
  p.max_rank = worst;
  p.exact = (worst <= chi);
  // dense messages are exact when no message MPS can exceed chi
  const bool msg_exact = (1 << (p.max_msg_len / 2)) <= chi;
  // largest dense boundary state of any sweep (the device keeps it in 4096-entry LDS buffers)
  size_t max_state = 0, max_mid = 0;
  auto state_size = [&](const SweepDesc& s) {
    int Ps = 1;
    for (int t = 0; t < s.kt; ++t) {
      Column col;
      make_column(col, s.frame, s.r0, s.c0, s.kr, s.kc, s.kt, s.kp, p.L, t, s.msg_top >= 0, s.msg_bot >= 0);
      const size_t H = 64;   // the device stores rows of 64 lanes
      max_mid = std::max(max_mid, (size_t)col.top.Pnew * H * Ps * (col.single ? 2 : 1));
      max_state = std::max(max_state, (size_t)col.top.Pnew * H * col.bot.Pnew);
      Ps = col.bot.Pnew;
    }
  };
  for (int c = 0; c < 2; ++c) for (auto& s : p.round[c]) if (!s.trunc) state_size(s);
  for (auto& s : p.bethe) if (!s.trunc) state_size(s);
  if (kmax > TRUNC_KMAX) {
    p.gpu_ok = false;
    p.why = "blocks larger than 8 tensors per side are not implemented on the GPU";
  } else if (max_state > 4096 || max_mid > 2048) {
    p.gpu_ok = false;
    p.why = "a dense block sweep exceeds the device's state buffers";
  } else if (!msg_exact) {
    p.gpu_ok = false;
    p.why = "chi below 2^(k/2): message MPSs would be truncated, not implemented on the GPU";
  } else if (p.trunc_sweeps > 0 && chi > TRUNC_CHI_MAX) {
    p.gpu_ok = false;
    p.why = "the truncating block sweeps (blocks wider than 6, or chi below a block's boundary rank) hold chi "
            "up to 16";
  } else {
    p.gpu_ok = true;
  }
  return p;
}

int host_sweep(const Plan& p, const SweepDesc& s, const uint8_t* labels, const float* pi, const double* msgs,
               double* out, double* logscale) {
  // the kernel's algorithm (sweep.hpp), evaluated sequentially in float64 with float32 inputs
  const int kt = s.kt, kp = s.kp, H = 1 << kp, L = p.L;
  std::vector<float> tables((size_t)kt * kp * 16);
  for (int t = 0; t < kt; ++t)
    for (int i = 0; i < kp; ++i) {
      int r, c;
      frame_site(s.frame, s.r0, s.c0, s.kr, s.kc, t, i, r, c);
      site_table(s.frame, L, r, c, labels[r * L + c], pi, &tables[(size_t)(t * kp + i) * 16]);
    }
  std::vector<float> mt(64, 0.0f), mb(64, 0.0f);
  if (s.msg_top >= 0) for (int h = 0; h < 64; ++h) mt[h] = (float)msgs[(size_t)s.msg_top * 64 + h];
  if (s.msg_bot >= 0) for (int h = 0; h < 64; ++h) mb[h] = (float)msgs[(size_t)s.msg_bot * 64 + h];
  std::vector<double> A(H, 0.0), B;
  if (s.msg_init >= 0) for (int h = 0; h < H; ++h) A[h] = (float)msgs[(size_t)s.msg_init * 64 + h];
  else A[0] = 1.0;
  int Ps = 1;
  double scale = 1.0, ls = 0.0;
  for (int t = 0; t < kt; ++t) {
    Column col;
    make_column(col, s.frame, s.r0, s.c0, s.kr, s.kc, kt, kp, L, t, s.msg_top >= 0, s.msg_bot >= 0);
    const float* T = &tables[(size_t)t * kp * 16];
    const int Ptn = col.top.Pnew, Psn = col.bot.Pnew;
    const int HB = col.single ? 2 * H : H;
    B.assign((size_t)Ptn * HB * Ps, 0.0);
    auto getA = [&](int n, int h, int sb) { return scale * A[((size_t)n * H + h) * Ps + sb]; };
    auto put = [&](int np, int h, int sb, double v) { B[((size_t)np * H + h) * Ps + sb] = v; };
    if (col.single) {
      for (int np = 0; np < Ptn; ++np)
        for (int sb = 0; sb < Ps; ++sb) pass1_item<double>(col, T, mt.data(), np, 0, sb, getA, put);
    } else {
      for (int np = 0; np < Ptn; ++np)
        for (int h = 0; h < H; ++h) {
          if (h & col.gmask) continue;
          for (int sb = 0; sb < Ps; ++sb) pass1_item<double>(col, T, mt.data(), np, h, sb, getA, put);
        }
    }
    auto getB = [&](int n, int h, int sb) { return B[((size_t)n * H + h) * Ps + sb]; };
    A.assign((size_t)Ptn * H * Psn, 0.0);
    double ss = 0.0;
    for (int n = 0; n < Ptn; ++n)
      for (int h = 0; h < H; ++h)
        for (int sp = 0; sp < Psn; ++sp) {
          const double v = pass2_output<double>(col, T, mb.data(), n, h, sp, getB);
          A[((size_t)n * H + h) * Psn + sp] = v;
          ss += v * v;
        }
    const double nrm = std::sqrt(ss);
    scale = 1.0 / nrm;
    ls += std::log(nrm);
    Ps = Psn;
  }
  for (int h = 0; h < H; ++h) out[h] = A[h] * scale;
  *logscale = ls;
  return 0;
}

const Plan& cached_plan(int d, int kr, int kc, int chi) {
  static std::map<std::tuple<int, int, int, int>, Plan> cache;
  static std::mutex mu;
  std::lock_guard<std::mutex> lk(mu);
  auto key = std::make_tuple(d, kr, kc, chi);
  auto it = cache.find(key);
  if (it == cache.end()) it = cache.emplace(key, make_plan(d, kr, kc, chi)).first;
  return it->second;
}

}  // namespace bbp
