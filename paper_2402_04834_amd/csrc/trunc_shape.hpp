// trunc_shape.hpp -- the shape decision shared by the truncating-sweep kernel (trunc_sweep.hip) and the
// planner's flop model (plan.cpp).
#pragma once

namespace bbp {

// A truncating sweep is narrow when every bond of its state stays within 8: chi <= 8, and the chain of the
// entering message over its kp sites has bonds min(2^j, 2^(kp - j)) <= 8 (kp <= 7). A site that has absorbed
// its column then spans at most 16 x 2 x 16 values: its factorisation is 32 x 16 inside the padded 64 x 32
// (16 reflections) and its SVD has at most 16 nonzero rows.
constexpr bool trunc_narrow(int chi, int kp) { return chi <= 8 && kp <= 7; }

}  // namespace bbp
