"""Algorithmic FP64 work of the calibrator, for the roofline.

Counts follow the formulas as the kernels evaluate them: add, sub and mul
count 1, fma counts 2, comparisons and selects count 0.  An elementary
function counts the FP64 operations of one call of the device math library
(``ELEMENTARY``), measured once on MI355X with the hardware counters
(SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_F64 of a kernel that only calls the
function; see the profiles directory).  Units: FLOP per quote evaluation, per
chain step (parameter maps, proposal, Metropolis) and per launch of the
per-level annealing kernel.
"""
from __future__ import annotations

import numpy as np

# FP64 FLOP per call (ADD + MUL + TRANS + 2 FMA), measured: see module docstring.
ELEMENTARY = {"exp": 27.0, "log1p": 45.0, "sqrt": 9.0, "div": 13.0, "erfc": 60.0}


def _e(name, n=1):
    return n * ELEMENTARY[name]


# SABR constants of one (alpha, beta, rho, nu): (1-b), (1-b)^2, the three
# corr coefficients and the five z/x(z) series coefficients.
SABR_CONST = 34.0


def hagan_quote(fixed_beta: bool) -> float:
    """Hagan 2002 vol for one quote: z, s = sqrt(1 - 2 rho z + z^2), the
    log1p argument (one division), the series, corr q^2 and the final
    division; plus q = exp(...) and D1 when beta is a parameter."""
    arith = 2 + 4 + 3 + 10 + 7 + 2 + 4
    f = arith + _e("sqrt") + _e("log1p") + _e("div", 2)
    if not fixed_beta:
        f += 2 + _e("exp") + 6
    return f


def eq3_quote(fixed_beta: bool) -> float:
    """Paper eq. (sigmaHagan) for one quote: w = f^(1-b)/alpha, two bracket
    coefficients, the quadratic in k and the scale."""
    f = 1 + 2 + 2 + 9 + 4 + 1 + _e("div", 2)
    if not fixed_beta:
        f += 1 + _e("exp")
    return f


def black_quote() -> float:
    """Black-76 out-of-the-money price: sd, d1 (one division), d2, two erfc
    and the combination."""
    return 14 + _e("div") + _e("erfc", 2)


RESIDUAL = 4.0   # r = m - mkt, acc += w r r


def quote_flops(model: int, formula: int, residual: int) -> float:
    fixed = model == 1
    f = hagan_quote(fixed) if formula == 0 else eq3_quote(fixed)
    if model == 1:
        f += SABR_CONST          # per underlying constants, evaluated per quote
    if residual == 1:
        f += black_quote()
    return f + RESIDUAL


def map_flops_inst(market: dict, inst: int) -> float:
    """LMM12 map per chain step: abcd forms and correlation gap factors per
    forward; per underlying nu/alpha, and for a swap over n forwards the O(n)
    frozen-weight recursion (21 n) plus its closing square roots and
    divisions."""
    if int(market["model"]) == 0:
        return SABR_CONST + _e("div")
    f0, f1 = market["fwd_off"][inst], market["fwd_off"][inst + 1]
    u0, u1 = market["und_off"][inst], market["und_off"][inst + 1]
    nf = f1 - f0
    lens = np.asarray(market["und_len"][u0:u1])
    fwd = nf * (10 + _e("exp", 2)) + max(nf - 1, 0) * (3 + _e("exp", 2))
    und = len(lens) * _e("div")
    swp = lens[lens > 1]
    und += float(np.sum(21 * swp)) + len(swp) * (8 + _e("sqrt", 2) + _e("div", 3))
    return fwd + und


def step_overhead(model: int) -> float:
    """Proposal (7 per coordinate), uniform conversion, Metropolis."""
    P = 4 if model == 0 else 12
    return 7 * P + (P + 1) + 2 + _e("div") + _e("exp")


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
        per_step = nq[i] * qf + map_flops_inst(market, i) + step_overhead(model)
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
