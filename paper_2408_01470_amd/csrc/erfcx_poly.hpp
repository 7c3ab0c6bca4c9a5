// erfcx_poly.hpp -- written by gen_erfcx.py; do not edit.
// h(t) = erfcx(x) (x + K), t = (x - K)/(x + K), as a polynomial in t
// of degree 24 (Chebyshev interpolant, monomial basis, Horner).
// Max relative error of the double evaluation on [0, 1e21]: 4.12e-16.
#pragma once

namespace sabr {

constexpr double kErfcxK = 4.0;
constexpr int kErfcxDeg = 24;
constexpr double kErfcxPoly[kErfcxDeg + 1] = {
    1.095995661000491,
    -0.976548729080882,
    0.7732087022652369,
    -0.5408538313132345,
    0.33085158787802266,
    -0.17401093723993213,
    0.0763815149091835,
    -0.02637005334070314,
    0.00611205565561393,
    -0.0002809588591250074,
    -0.0004550526714402559,
    0.00017681276781310884,
    -3.6352864144616853e-06,
    -1.8860655174390427e-05,
    4.6949536005148395e-06,
    1.4235437808888834e-06,
    -8.477202827598295e-07,
    -7.440134079315679e-08,
    1.2678363974294932e-07,
    -2.762829273945234e-10,
    -1.8096905734635933e-08,
    7.054882560385151e-10,
    2.282283310732059e-09,
    -7.652918351368929e-11,
    -1.791502752209178e-10,
};

}  // namespace sabr
