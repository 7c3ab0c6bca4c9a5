"""Algorithmic FP64 work of the calibrator, for the roofline.

Counts follow the formulas as the kernels state them, each operation counted
once where the definition needs it: add, sub and mul count 1, fma counts 2,
a hardware reciprocal or reciprocal square root seed counts 1, comparisons,
selects, negations, exponent manipulation and integer work (the Philox
generator) count 0; of two forms selected between, the common one counts
(the |z| <= 1 quotient of z/x(z)).  Elementary functions count the FP64
operations of their implementation (``ELEMENTARY``): the kernels' own
branch-free exp, log1p, sqrt, reciprocal and erfcx (counted from their
definitions, and confirmed by the hardware counters
SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_F64 of a kernel calling only one of them,
as ADD + MUL + TRANS + 2 FMA per call), and the device library's division,
measured the same way.  Units: FLOP per quote evaluation, per underlying,
per chain step (parameter map, proposal, Metropolis) and per launch of the
per-level annealing kernel.
"""
from __future__ import annotations

import numpy as np

# FP64 FLOP per call (confirmed by the counters of the pricing program).
#   exp   : x/ln2, two-step Cody-Waite reduction, degree-11 Horner      1+4+22
#   log1p : two-sum (6), m + m (1), f with the two-sum's error (2),
#           s = f/(2 + f) (9), s^2 (1), degree-6 Horner (12), the two fma
#           (4), k ln2 (4)                                                  39
#   sqrt  : rsq seed, one Goldschmidt pass, final correction          1+2+10
#   rcp   : rcp seed, r0 + r0 (e + e^2)                                  1+6
#   erfcx : x +- K, reciprocal, degree-24 Horner, scale              2+7+48+2
#   erfcx2: a pair sharing one reciprocal of the product (the two
#           arguments' x +- K 4, product 1, reciprocal 7, the two
#           reciprocals 2, t 2, Horner 96, scales 2)                      114
#   div   : device library division                                        14
ELEMENTARY = {"exp": 27.0, "log1p": 39.0, "sqrt": 13.0, "rcp": 7.0, "erfcx": 59.0,
              "erfcx2": 114.0, "div": 14.0}


def _e(name, n=1):
    return n * ELEMENTARY[name]


def sabr_const(model: int, formula: int = 0) -> float:
    """Constants of one (alpha, beta, rho, nu): rho^2 and 2 - 3 rho^2 (3),
    nu/alpha (a reciprocal and a product), the three corr coefficients
    alpha^2 (1-b)^2/24, rho b nu alpha/4, (2 - 3 rho^2) nu^2/24 (3 + 4 + 3);
    (1-b) and (1-b)^2 add 2 when beta is a parameter (GLOBAL4).  Eq.
    (sigmaHagan) with beta fixed instead takes the three coefficients of its
    quadratic in k: nu/alpha (reciprocal and product), w = fp/alpha (1),
    alpha/fp (reciprocal and product), d = 1-b - rho nu w (3), nu w (1), the
    linear coefficient (2) and the quadratic one (13)."""
    if model == 0:
        return 16.0 + _e("rcp")
    if formula == 1:
        return 22.0 + _e("rcp", 2)
    return 15.0 + _e("rcp")


def hagan_quote(fixed_beta: bool) -> float:
    """Hagan 2002 vol fraction for one quote: z = (nu/alpha) q L (2),
    s = sqrt(1 - 2 rho z + z^2) (4), the log1p argument 2z/(s + 1 - z)
    (3 and a division), P = q^2 + T (ca + cb q + cc q^2) (7), the numerator
    alpha P z (2) and the denominator (q^3 D1) x (1: q^3 D1 is the quote's
    constant when beta is fixed); with beta a parameter also q^3 D1 (3),
    q = exp((1-b)/2 ln(fK)) (2) and D1 = 1 + u/24 + u^2/1920,
    u = (1-b)^2 L^2 (6).  The quotient is a reciprocal and a product."""
    f = 19 + _e("sqrt") + _e("log1p") + _e("rcp")
    if not fixed_beta:
        f += 3 + 2 + _e("exp") + 6
    return f


def eq3_quote(fixed_beta: bool) -> float:
    """Paper eq. (sigmaHagan) for one quote.  beta a parameter: nu =
    (nu/alpha) alpha (1), w = f^(1-b)/alpha (a library division), rho nu w
    (2), the two bracket coefficients (2 and 12), the quadratic in k (4),
    the numerator scale (1) and fp = exp((1-b) ln f) (1).  beta fixed: the
    quadratic in k with the underlying's coefficients (two fma, 4)."""
    if fixed_beta:
        return 4.0
    return 23 + _e("div") + _e("exp")


def black_quote(direct: bool = False) -> float:
    """sigma and 1/sigma from the vol fraction (5 and one reciprocal; one
    reciprocal when the formula gives sigma itself), then the Black-76
    out-of-the-money price: sd, d1, d2 (6), the two erfcx arguments
    x = |d|/sqrt(2) (2), E = exp(-x1^2) (1), f E/2 (2), the combination (3)
    and the discount (1); the two erfcx share one reciprocal (erfcx2)."""
    return (1 if direct else 5) + _e("rcp") + 15 + _e("exp") + _e("erfcx2")


RESIDUAL = 4.0   # r = m - target, acc += (w r) r


def quote_flops(model: int, formula: int, residual: int) -> float:
    fixed = model != 0          # LMM12 and PERFWD fix beta
    direct = fixed and formula == 1   # the formula gives sigma itself
    f = hagan_quote(fixed) if formula == 0 else eq3_quote(fixed)
    if residual == 1:
        f += black_quote(direct)
    elif not direct:
        f += 1 + _e("rcp")
    return f + RESIDUAL


def map_flops_inst(market: dict, inst: int) -> float:
    """Parameter map per chain step.  GLOBAL4: the SABR constants once.
    LMM12: per forward the two abcd forms (10 and 2 exp), per gap between
    consecutive forwards the two correlation factors (3 and 2 exp); per
    underlying its SABR constants; for a swap over n forwards the O(n)
    frozen-weight recursion (4 per forward forward, 14 per forward
    backward) and its closing Nb, alpha_S, nu_S, rho_S (12, 2 sqrt,
    3 reciprocals).  PERFWD: per underlying the SABR constants of its
    forward's triple (fixed beta)."""
    if int(market["model"]) == 0:
        return sabr_const(0) + 2
    f0, f1 = market["fwd_off"][inst], market["fwd_off"][inst + 1]
    u0, u1 = market["und_off"][inst], market["und_off"][inst + 1]
    formula = int(market["formula"])
    if int(market["model"]) == 2:
        return (u1 - u0) * sabr_const(2, formula)
    if int(market["model"]) == 3:
        # per forward: phi alpha w (2), the running sum (1), sigma D (1),
        # exp, the product (1); per underlying its SABR constants
        nf = f1 - f0
        return nf * (5 + _e("exp")) + (u1 - u0) * sabr_const(3, formula)
    if int(market["model"]) == 4:
        # per underlying: G and Qh(T) (two square integrals), 32 quadrature
        # nodes (g: exp + 4; Qh(tau): square integral; term: 5), the sum and
        # alpha, nu (2 sqrt, 2 reciprocals, 5)
        sq = SQ_INT
        return (u1 - u0) * (2 * sq + 32 * (_e("exp") + 4 + sq + 5) + 31 + _e("sqrt", 2) +
                            _e("rcp", 2) + 5 + sabr_const(4, formula))
    nf = f1 - f0
    lens = np.asarray(market["und_len"][u0:u1])
    fwd = nf * (10 + _e("exp", 2)) + max(nf - 1, 0) * (3 + _e("exp", 2))
    und = len(lens) * sabr_const(1, formula)
    swp = lens[lens > 1]
    und += float(np.sum(18 * swp)) + len(swp) * (12 + _e("sqrt", 2) + _e("rcp", 3))
    return fwd + und


# Square integral of an abcd function (abcd_sq_int): two psi triples (the
# 17-term series by Horner's rule, 16 fma = 32, the closed form 10 with a
# reciprocal, the downward recurrence 4) at 2cx and cx sharing one
# exponential (given), and the combination (14).
SQ_INT = 2 * (32 + 10 + _e("rcp") + 4) + 14


def num_params(market: dict) -> int:
    model = int(market["model"])
    nf = int(market["fwd_off"][1] - market["fwd_off"][0])
    if model == 2:
        return 3 * nf
    if model == 3:
        return 2 * nf + 1
    if model == 4:
        return 2 * nf + 8
    return 4 if model == 0 else 12


def step_overhead(P: int) -> float:
    """Proposal (6 per coordinate), uniform conversion (1 per uniform, P+1),
    Metropolis (dE, a library division and exponential)."""
    return 6 * P + (P + 1) + 1 + _e("div") + _e("exp")


def level_launch_flops(market: dict, chains, n_steps: int) -> float:
    """FLOP of one launch of the per-level annealing kernel: every chain of
    every instance takes n_steps steps."""
    model, formula, residual = (int(market["model"]), int(market["formula"]),
                                int(market["residual"]))
    nq = np.diff(np.asarray(market["q_off"]))
    n = len(nq)
    ch = np.broadcast_to(np.asarray(chains), (n,))
    qf = quote_flops(model, formula, residual)
    tot = 0.0
    for i in range(n):
        per_step = nq[i] * qf + map_flops_inst(market, i) + step_overhead(num_params(market))
        tot += float(ch[i]) * n_steps * per_step
    return tot


def cost_launch_flops(market: dict, pt_inst) -> float:
    """FLOP of one sabr_cost_batch launch over the given points."""
    model, formula, residual = (int(market["model"]), int(market["formula"]),
                                int(market["residual"]))
    nq = np.diff(np.asarray(market["q_off"]))
    qf = quote_flops(model, formula, residual)
    pt_inst = np.asarray(pt_inst)
    return float(sum(nq[i] * qf + map_flops_inst(market, i) for i in pt_inst))


# ---------------------------------------------------------------------------
# Monte Carlo pricer (the Hagan SABR/LIBOR dynamics of Sec. 2.1)
# ---------------------------------------------------------------------------
# The path step's own functions, counted from their definitions:
#   log        : m + m, m - 1, 2 + f, rcp, s, s^2, degree-6 Horner, two fma,
#                k ln2 in two fma                               1+1+1+7+1+1+12+4+4 = 32
#   sincos 2pi u: 4u, q/4, u - q/4, 2 pi r, x^2, x z, two degree-8 Horner
#                chains and their closing fma                     5+1+16+2+16+2 = 42
MC_LOG = 32.0
MC_SINCOS = 42.0
MC_BOX_MULLER = MC_LOG + _e("sqrt") + MC_SINCOS + 5          # per normal pair: 92
MC_PER_FORWARD_REST = (1 + 4 + _e("rcp")          # s = V F^beta, d = tau s / (1 + tau F)
                       + 6                         # the three drift recursions
                       + 10                        # the F update
                       + 10 + _e("exp"))           # the V update: 65


def mc_power_flops(beta: float) -> float:
    """max(F, 0)^beta: sqrt at beta = 1/2, F itself at 1, else exp(beta log F)."""
    if beta == 0.5:
        return _e("sqrt")
    if beta == 1.0:
        return 0.0
    return 1 + MC_LOG + _e("exp")


def mc_step_flops(M: int, betas_alive) -> float:
    """One path step with the n forwards of betas_alive alive (of M): n
    normal pairs, pair m adding its two factor columns into the alive rows
    2m..2n-1 (lower triangular: two fma per row, 4 n (n + 1) FLOP in all),
    and each alive forward's power, drift and updates."""
    n = len(betas_alive)
    return (n * MC_BOX_MULLER + 4 * n * (n + 1)
            + sum(mc_power_flops(b) + MC_PER_FORWARD_REST for b in betas_alive))


def mc_steps(T, dt, amax):
    """Steps of each fixing interval 0..amax (the pricer's grid)."""
    out = []
    for j in range(amax + 1):
        length = T[j] - (T[j - 1] if j > 0 else 0.0)
        out.append(max(1, int(np.ceil(length / dt))))
    return out


def mc_launch_flops(prob: dict, n_paths: int, dt: float) -> float:
    """Algorithmic FLOP of one pricing call (path steps only; the payoffs,
    once per option and path, are left out)."""
    M = len(prob["T"])
    amax = int(np.max(prob["opt_a"]))
    n = mc_steps(prob["T"], dt, amax)
    beta = [float(b) for b in prob["beta"]]
    return float(n_paths) * sum(n[j] * mc_step_flops(M, beta[j:]) for j in range(amax + 1))


def mc_path_steps(prob: dict, n_paths: int, dt: float) -> float:
    amax = int(np.max(prob["opt_a"]))
    return float(n_paths) * sum(mc_steps(prob["T"], dt, amax))
