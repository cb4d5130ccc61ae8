// trunc_shape.hpp -- the shape decision shared by the truncating-sweep kernel (trunc_sweep.hip) and the
// planner's flop model (plan.cpp).
#pragma once

namespace bbp {

// A truncating sweep is narrow when every bond of its state stays within 8: chi <= 8, and the chains of the
// entering message over its kp sites and of the side messages over its kt steps have bonds
// min(2^j, 2^(K - j)) <= 8 (kp, kt <= 7). A site that has absorbed its column then spans at most 16 x 2 x 16
// values: its factorisation is 32 x 16 inside the padded 64 x 32 (16 reflections), and the matrices of its
// SVDs have at most 16 nonzero rows and 8 nonzero entries per half-row.
constexpr bool trunc_narrow(int chi, int kt, int kp) { return chi <= 8 && kt <= 7 && kp <= 7; }

}  // namespace bbp
