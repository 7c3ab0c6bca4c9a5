// log1p_poly.hpp -- written by gen_log1p.py; do not edit.
// log(m) = f - s (f - z P(z)), s = f/(2+f), z = s^2, m = 1 + f in
// [sqrt(1/2), sqrt(2)); P of degree 6.  Max relative error of a plain
// double evaluation on t in (-1, 1e12]: 1.98e-16.
#pragma once

namespace sabr {

constexpr double kLn2Hi = 0.6931471803691238;
constexpr double kLn2Lo = 1.9082149292705877e-10;
constexpr int kLog1pDeg = 6;
constexpr double kLog1pPoly[kLog1pDeg + 1] = {
    0.666666666666667,
    0.39999999999899505,
    0.28571428625975487,
    0.2222221113479508,
    0.18182889125261723,
    0.15331721600556042,
    0.14616449685043406,
};

}  // namespace sabr
