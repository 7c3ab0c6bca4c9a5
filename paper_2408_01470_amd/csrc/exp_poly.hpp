// exp_poly.hpp -- written by gen_exp.py; do not edit.
// exp(x) = 2^k p(r), k = rint(x/ln2), r = x - k ln2_hi - k ln2_lo,
// p of degree 11.  Max relative error of a plain double evaluation on
// the normal range: 1.77e-16.
#pragma once

namespace sabr {

constexpr double kExpLn2Hi = 0.6931471803691238;
constexpr double kExpLn2Lo = 1.9082149292705877e-10;
constexpr double kExpInvLn2 = 1.4426950408889634;
constexpr int kExpDeg = 11;
constexpr double kExpPoly[kExpDeg + 1] = {
    1.0,
    1.0,
    0.5000000000000019,
    0.1666666666666668,
    0.0416666666664881,
    0.008333333333319601,
    0.0013888888952314775,
    0.00019841269890047113,
    2.4801485482328494e-05,
    2.755724091857897e-06,
    2.763263963904103e-07,
    2.5110037605963777e-08,
};

}  // namespace sabr
