#!/usr/bin/env python
"""Writes exp_poly.hpp: the constants of the device exp.

Method (Cody & Waite, Software Manual for the Elementary Functions, 1980):
k = rint(x / ln2), r = x - k ln2 evaluated as two fma steps with
ln2 = ln2_hi + ln2_lo (ln2_hi of 32 significant bits, so k ln2_hi is exact
for |k| < 2^21), |r| <= ln2/2, exp(x) = 2^k p(r) with p the degree-11
polynomial interpolating exp at the Chebyshev nodes of [-ln2/2, ln2/2]
(80 digits, rounded to double; relative error 4e-18 before rounding).
The script reports the maximum relative error of a double evaluation
(Python floats, no fma) against mpmath on [-745, 709].
"""
import math
import os

import mpmath as mp

DEG = 11
HERE = os.path.dirname(os.path.abspath(__file__))


def fit():
    h = mp.log(2) / 2
    n = DEG + 1
    nodes = [h * mp.cos(mp.pi * (j + mp.mpf(1) / 2) / n) for j in range(n)]
    A = mp.matrix([[x ** i for i in range(n)] for x in nodes])
    b = mp.matrix([mp.exp(x) for x in nodes])
    a = mp.lu_solve(A, b)
    return [a[i] for i in range(n)]


def split_ln2():
    ln2 = mp.log(2)
    hi = mp.floor(ln2 * 2 ** 32) / 2 ** 32
    return float(hi), float(ln2 - hi), float(1 / ln2)


def exp_double(x, a, hi, lo, il2):
    k = round(x * il2)
    r = (x - k * hi) - k * lo
    p = a[-1]
    for c in reversed(a[:-1]):
        p = p * r + c
    return math.ldexp(p, int(k))


def main():
    mp.mp.dps = 80
    a = [float(v) for v in fit()]
    hi, lo, il2 = split_ln2()
    worst = 0.0
    for i in range(20001):
        x = -745.0 + (709.0 + 745.0) * i / 20000
        ref = mp.exp(mp.mpf(x))
        if ref < mp.mpf(2) ** -1022:
            continue            # subnormal results: absolute, not relative, accuracy
        got = exp_double(x, a, hi, lo, il2)
        worst = max(worst, float(abs((got - ref) / ref)))
    lines = [
        "// exp_poly.hpp -- written by gen_exp.py; do not edit.",
        "// exp(x) = 2^k p(r), k = rint(x/ln2), r = x - k ln2_hi - k ln2_lo,",
        f"// p of degree {DEG}.  Max relative error of a plain double evaluation on",
        f"// the normal range: {worst:.2e}.",
        "#pragma once",
        "",
        "namespace sabr {",
        "",
        f"constexpr double kExpLn2Hi = {hi!r};",
        f"constexpr double kExpLn2Lo = {lo!r};",
        f"constexpr double kExpInvLn2 = {il2!r};",
        f"constexpr int kExpDeg = {DEG};",
        "constexpr double kExpPoly[kExpDeg + 1] = {",
    ]
    lines += [f"    {v!r}," for v in a]
    lines += ["};", "", "}  // namespace sabr", ""]
    with open(os.path.join(HERE, "exp_poly.hpp"), "w") as fh:
        fh.write("\n".join(lines))
    print(f"degree {DEG}, max rel err {worst:.2e}")


if __name__ == "__main__":
    main()
