#!/usr/bin/env python
"""Writes log1p_poly.hpp: the constants of the device log1p.

Method (argument reduction by the binary exponent, then the atanh series; the
scheme of Tang, ACM TOMS 16 (1990), without the table): v = 1 + t = 2^k m
with m in [sqrt(1/2), sqrt(2)), f = m - 1 (exact), s = f/(2 + f),
log(m) = 2 atanh(s) = f - s (f - R(s^2)) with
R(z) = sum_{j>=1} 2 z^j/(2j + 1) = z P(z), |s| <= (sqrt2 - 1)/(sqrt2 + 1).

P is the degree-6 polynomial interpolating P(z) = (log((1+s)/(1-s))/s - 2)/z
at the Chebyshev nodes of [0, z_max] (80 digits, rounded to double); its
error on R is below 1e-17 absolute, i.e. under 0.05 ulp of the result.
ln 2 is split as ln2_hi (32 significant bits, so k ln2_hi is exact) plus
ln2_lo.  The script reports the maximum relative error of a double
evaluation (Python floats, no fma) against mpmath.
"""
import os

import mpmath as mp

DEG = 6
HERE = os.path.dirname(os.path.abspath(__file__))


def p_exact(z):
    if z == 0:
        return mp.mpf(2) / 3
    s = mp.sqrt(z)
    return (mp.log((1 + s) / (1 - s)) / s - 2) / z


def fit():
    smax = (mp.sqrt(2) - 1) / (mp.sqrt(2) + 1)
    zmax = smax * smax
    n = DEG + 1
    nodes = [zmax / 2 * (1 + mp.cos(mp.pi * (j + mp.mpf(1) / 2) / n)) for j in range(n)]
    A = mp.matrix([[x ** i for i in range(n)] for x in nodes])
    b = mp.matrix([p_exact(x) for x in nodes])
    a = mp.lu_solve(A, b)
    return [a[i] for i in range(n)]


def split_ln2():
    ln2 = mp.log(2)
    hi = mp.floor(ln2 * 2 ** 32) / 2 ** 32
    return float(hi), float(ln2 - hi)


def log1p_double(t, a, hi, lo):
    import math
    v = 1.0 + t
    vv = v - 1.0
    e = (1.0 - (v - vv)) + (t - vv)
    m, k = math.frexp(v)
    if m < math.sqrt(0.5):
        m, k = 2 * m, k - 1
    f = m - 1.0
    s = f / (2.0 + f)
    z = s * s
    p = a[-1]
    for c in reversed(a[:-1]):
        p = p * z + c
    lf = f - s * (f - z * p)
    return k * hi + (lf + (k * lo + e / v))


def main():
    mp.mp.dps = 80
    a_mp = fit()
    a = [float(v) for v in a_mp]
    hi, lo = split_ln2()
    worst = 0.0
    for i in range(1, 6001):
        if i <= 2000:
            t = -1 + 10 ** (-16 + 16 * i / 2000)        # (-1, 0)
        elif i <= 4000:
            t = 10 ** (-12 + 12 * (i - 2000) / 2000)    # (0, 1]
        else:
            t = 10 ** (12 * (i - 4000) / 2000)          # [1, 1e12]
        for tt in (t, -t if t < 1 else t):
            if tt == 0.0:
                continue
            got = log1p_double(tt, a, hi, lo)
            ref = mp.log1p(mp.mpf(tt))
            worst = max(worst, float(abs((got - ref) / ref)))
    lines = [
        "// log1p_poly.hpp -- written by gen_log1p.py; do not edit.",
        "// log(m) = f - s (f - z P(z)), s = f/(2+f), z = s^2, m = 1 + f in",
        f"// [sqrt(1/2), sqrt(2)); P of degree {DEG}.  Max relative error of a plain",
        f"// double evaluation on t in (-1, 1e12]: {worst:.2e}.",
        "#pragma once",
        "",
        "namespace sabr {",
        "",
        f"constexpr double kLn2Hi = {hi!r};",
        f"constexpr double kLn2Lo = {lo!r};",
        f"constexpr int kLog1pDeg = {DEG};",
        "constexpr double kLog1pPoly[kLog1pDeg + 1] = {",
    ]
    lines += [f"    {v!r}," for v in a]
    lines += ["};", "", "}  // namespace sabr", ""]
    with open(os.path.join(HERE, "log1p_poly.hpp"), "w") as fh:
        fh.write("\n".join(lines))
    print(f"degree {DEG}, ln2 = {hi!r} + {lo!r}, max rel err {worst:.2e}")


if __name__ == "__main__":
    main()
