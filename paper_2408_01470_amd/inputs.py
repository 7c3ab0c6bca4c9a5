"""Seeded synthetic market generators (shared by the GPU path and its checks).

This module only lays out market *structure* and draws random numbers: forward
curves, fixing grids, strikes, quote kinds, true parameters, noise draws and
random search-box points.  It holds none of the calibration method's
arithmetic (no implied-vol formula, no Black price, no parameter map, no
cost): market quotes are completed by the caller from model vols at the true
parameters (``complete_market``), computed by whichever implementation the
caller is exercising.

Workload shapes follow the paper's caplet/swaption calibration (Sec. 4:
semiannual EURIBOR forwards, smiles over a moneyness grid ln(K/F) of
-80%..80%, Table "Smiles of forward rates") at the sizes of the benchmark
configurations:

* ``caplet_market``      -- 10 semiannual forwards, 3% + N(0, 0.002),
  11 strikes F +- 200 bp (ATM included), GLOBAL4 (alpha, beta, rho, nu).
* ``lmm_market``         -- M semiannual forwards on an upward 2%..4% curve,
  caplet smiles on forwards 1..M-1 plus an expiry x tenor swaption grid,
  LMM12 parameters, price residuals (optionally both option sides).
* ``batch_markets``      -- many caplet markets of uneven size
  (10..40 forwards x 5..15 strikes).
* ``perfwd_markets``     -- equal-size caplet markets with per-forward
  (alpha, rho, nu) truths, for the PERFWD model.
* ``mm_markets``         -- equal-size caplet markets with Mercurio-Morini
  truths (alpha_i, phi_i per forward, one sigma).
* ``paper_caplet_market`` -- not synthetic: the paper's own 6M EURIBOR
  caplet data of 21/11/2011 (13 forwards x 9 moneyness values, Sec. 4,
  Tables "Discount factor curve" and "Smiles of forward rates"), for the
  per-forward (PERFWD) Hagan model calibrated in Sec. 4.1.1.

All randomness comes from ``numpy.random.Generator(Philox(key))``.
"""
from __future__ import annotations

import datetime
import os

import numpy as np

MODEL_GLOBAL4 = 0
MODEL_LMM12 = 1
MODEL_PERFWD = 2
MODEL_MM = 3
MODEL_REB = 4
FORMULA_HAGAN2002 = 0
FORMULA_PAPER_EQ3 = 1
RESID_VOL = 0
RESID_PRICE = 1
KIND_CALL = 0
KIND_PUT = 1

SEED_BASE = 2408014700

GLOBAL4_NAMES = ("alpha", "beta", "rho", "nu")
LMM12_NAMES = ("a", "b", "c", "d", "a_nu", "b_nu", "c_nu", "d_nu", "rho", "lambda1", "eta2",
               "lambda2")


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=int(seed)))


def num_params(model: int, n_fwd: int | None = None) -> int:
    if model == MODEL_PERFWD:
        return 3 * int(n_fwd)
    if model == MODEL_MM:
        return 2 * int(n_fwd) + 1
    if model == MODEL_REB:
        return 2 * int(n_fwd) + 8
    return 4 if model == MODEL_GLOBAL4 else 12


def box(model: int, n_fwd: int | None = None):
    """Search box (lb, ub).  The paper prints no box; values sitting on round
    bounds in its calibrated tables (sigma_1 = 1, phi = -1, kappa = 0.001)
    suggest plain interval bounds, chosen here wide enough to hold the
    synthetic true parameters.  PERFWD (n_fwd triples (alpha, rho, nu)):
    alpha in [0.001, 0.2] as for GLOBAL4, rho in [-0.99, 0.99], nu in
    [0.001, 1] (the printed sigma_1 = 1.0000 of Sec. 4.1.1 sits on that
    bound).  MM (n_fwd pairs (alpha, phi), then sigma): alpha and phi as for
    PERFWD, sigma in [0.001, 1].  REB (n_fwd pairs (kappa, phi), then g's
    (a, b, c, d) and h's (a_h, b_h, c_h, d_h)): kappa in [0.001, 0.2] (the
    printed kappa_i = 0.0010 sit on that bound), phi as above, a, b in
    [0, 50], c in [0.01, 10], d in [0.001, 50] (the printed g has b = 44.8,
    d = 25.3), a_h in [0.001, 5], b_h in [0, 50], c_h in [0.01, 10], d_h in
    [0.001, 5]."""
    if model == MODEL_PERFWD:
        lb = np.tile([0.001, -0.99, 0.001], int(n_fwd))
        ub = np.tile([0.2, 0.99, 1.0], int(n_fwd))
        return lb, ub
    if model == MODEL_MM:
        lb = np.concatenate([np.tile([0.001, -0.99], int(n_fwd)), [0.001]])
        ub = np.concatenate([np.tile([0.2, 0.99], int(n_fwd)), [1.0]])
        return lb, ub
    if model == MODEL_REB:
        lb = np.concatenate([np.tile([0.001, -0.99], int(n_fwd)),
                             [0.0, 0.0, 0.01, 0.001, 0.001, 0.0, 0.01, 0.001]])
        ub = np.concatenate([np.tile([0.2, 0.99], int(n_fwd)),
                             [50.0, 50.0, 10.0, 50.0, 5.0, 50.0, 10.0, 5.0]])
        return lb, ub
    if model == MODEL_GLOBAL4:
        lb = np.array([0.001, 0.0, -0.99, 0.001])
        ub = np.array([0.2, 1.0, 0.99, 1.5])
    else:
        lb = np.array([0.0, -0.05, 0.01, 0.001, 0.0, -0.5, 0.01, 0.001, -0.99, 0.001, 0.0, 0.001])
        ub = np.array([0.1, 0.1, 3.0, 0.1, 1.0, 1.0, 3.0, 1.0, 0.99, 5.0, 0.999, 5.0])
    return lb, ub


def _curve_discounts(T, tau, F):
    """Payment discount factors P(0, T_i + tau_i) of a curve whose forwards
    are F (simple compounding), starting from P(0, T_0) given by the caller's
    first entry of ``T`` at 3%: a curve consistent with its own forwards."""
    P = np.empty_like(F)
    d = 1.0 / (1.0 + T[0] * 0.03) if T[0] > 0 else 1.0
    for i in range(len(F)):
        d = d / (1.0 + tau[i] * F[i])
        P[i] = d
    return P


def _empty():
    return dict(fwd_T=[], fwd_tau=[], fwd_F=[], fwd_P=[], und_first=[], und_len=[], q_und=[],
                q_kind=[], q_K=[], q_w=[], fwd_off=[0], und_off=[0], q_off=[0])


def _finish(parts, model, formula, residual, beta):
    m = {}
    for k in ("fwd_T", "fwd_tau", "fwd_F", "fwd_P", "q_K", "q_w"):
        m[k] = np.ascontiguousarray(np.concatenate(parts[k]) if parts[k] else np.zeros(0),
                                    dtype=np.float64)
    for k in ("und_first", "und_len", "q_und", "q_kind"):
        m[k] = np.ascontiguousarray(np.concatenate(parts[k]) if parts[k] else np.zeros(0),
                                    dtype=np.int32)
    for k in ("fwd_off", "und_off", "q_off"):
        m[k] = np.asarray(parts[k], dtype=np.int32)
    m["q_vol"] = np.ones_like(m["q_K"])  # placeholder until complete_market
    m["model"] = int(model)
    m["formula"] = int(formula)
    m["residual"] = int(residual)
    m["beta"] = float(beta)
    return m


def _append(parts, T, tau, F, P, und_first, und_len, q_und, q_kind, q_K):
    parts["fwd_T"].append(np.asarray(T, float))
    parts["fwd_tau"].append(np.asarray(tau, float))
    parts["fwd_F"].append(np.asarray(F, float))
    parts["fwd_P"].append(np.asarray(P, float))
    parts["und_first"].append(np.asarray(und_first, np.int32))
    parts["und_len"].append(np.asarray(und_len, np.int32))
    parts["q_und"].append(np.asarray(q_und, np.int32))
    parts["q_kind"].append(np.asarray(q_kind, np.int32))
    parts["q_K"].append(np.asarray(q_K, float))
    parts["q_w"].append(np.ones(len(q_K)))
    parts["fwd_off"].append(parts["fwd_off"][-1] + len(T))
    parts["und_off"].append(parts["und_off"][-1] + len(und_first))
    parts["q_off"].append(parts["q_off"][-1] + len(q_K))


def _caplet_instance(g, M, nK, spread=0.02):
    T = 0.5 * np.arange(1, M + 1)
    tau = np.full(M, 0.5)
    F = 0.03 + g.normal(0.0, 0.002, M)
    P = _curve_discounts(T, tau, F)
    und_first = np.arange(M)
    und_len = np.ones(M, np.int32)
    offs = np.linspace(-spread, spread, nK)
    q_und = np.repeat(np.arange(M), nK)
    q_K = (F[:, None] + offs[None, :]).reshape(-1)
    # the ATM strike (offset exactly 0 when nK is odd) is F itself
    if nK % 2 == 1:
        q_K.reshape(M, nK)[:, nK // 2] = F
    q_kind = np.zeros(M * nK, np.int32)
    return T, tau, F, P, und_first, und_len, q_und, q_kind, q_K


def _global4_truth(g):
    return np.array([g.uniform(0.02, 0.05), 0.5, g.uniform(-0.5, 0.0), g.uniform(0.2, 0.6)])


def caplet_market(seed=SEED_BASE + 1000, M=10, nK=11, formula=FORMULA_HAGAN2002,
                  residual=RESID_VOL):
    """One caplet market: M semiannual forwards (fixings 0.5..0.5M years),
    F_i = 3% + N(0, 0.002), nK strikes evenly spread over F +- 200 bp."""
    g = rng(seed)
    parts = _empty()
    _append(parts, *_caplet_instance(g, M, nK))
    m = _finish(parts, MODEL_GLOBAL4, formula, residual, 0.5)
    truth = _global4_truth(g)[None, :]
    noise = g.normal(0.0, 0.002, m["q_K"].shape[0])
    return m, truth, noise


def batch_markets(n_markets=256, seed=SEED_BASE + 3000, M_range=(10, 40), nK_range=(5, 15)):
    """Independent caplet markets of uneven size (per-market seeds): M ~ U{10..40},
    nK ~ U{5..15}, so each holds 50..600 quotes."""
    parts = _empty()
    truths, noises = [], []
    for j in range(n_markets):
        g = rng(seed + j)
        M = int(g.integers(M_range[0], M_range[1] + 1))
        nK = int(g.integers(nK_range[0], nK_range[1] + 1))
        _append(parts, *_caplet_instance(g, M, nK))
        truths.append(_global4_truth(g))
        noises.append(g.normal(0.0, 0.002, M * nK))
    m = _finish(parts, MODEL_GLOBAL4, FORMULA_HAGAN2002, RESID_VOL, 0.5)
    return m, np.array(truths), np.concatenate(noises)


def _lmm12_truth(g):
    return np.array([
        g.uniform(0.01, 0.03), g.uniform(0.0, 0.02), g.uniform(0.5, 1.5), g.uniform(0.02, 0.04),
        g.uniform(0.1, 0.3), g.uniform(0.0, 0.2), g.uniform(0.5, 1.5), g.uniform(0.2, 0.4),
        g.uniform(-0.4, 0.0), g.uniform(0.05, 0.3), g.uniform(0.5, 0.9), g.uniform(0.1, 1.0),
    ])


def _moneyness_grid(n, lo=-0.8, hi=0.8):
    g = np.linspace(lo, hi, n)
    if n % 2 == 1:
        g[n // 2] = 0.0          # exact ATM strike
    return g


def _lmm_instance(M, n_cap_K, n_exp, n_ten, n_swp_K, both_sides):
    T = 0.5 * np.arange(M)
    tau = np.full(M, 0.5)
    F = 0.02 + 0.02 * np.arange(M) / (M - 1)
    P = _curve_discounts(T, tau, F)
    und_first, und_len, is_swp = [], [], []
    for i in range(1, M):                    # caplets on forwards 1..M-1
        und_first.append(i)
        und_len.append(1)
        is_swp.append(False)
    for e in range(1, n_exp + 1):            # swaptions: expiry T_e, n periods
        for n in range(1, n_ten + 1):
            if e + n - 1 <= M - 1:
                und_first.append(e)
                und_len.append(n)
                is_swp.append(True)
    und_first = np.array(und_first, np.int32)
    und_len = np.array(und_len, np.int32)
    cap_m = _moneyness_grid(n_cap_K)
    swp_m = _moneyness_grid(n_swp_K)
    sides = (KIND_CALL, KIND_PUT) if both_sides else (KIND_CALL,)
    q_und, q_kind, q_K = [], [], []
    for u in range(len(und_first)):
        f0, n = und_first[u], und_len[u]
        # strike centre: the forward itself for a caplet, the plain mean of
        # the swap's forwards for a swaption (close to, not equal to, S0)
        centre = F[f0] if n == 1 else float(np.mean(F[f0:f0 + n]))
        for mny in (swp_m if is_swp[u] else cap_m):
            for kind in sides:
                q_und.append(u)
                q_kind.append(kind)
                q_K.append(centre if mny == 0.0 else centre * np.exp(mny))
    return T, tau, F, P, und_first, und_len, np.array(q_und, np.int32), \
        np.array(q_kind, np.int32), np.array(q_K)


def lmm_market(seed=SEED_BASE + 2000, n_markets=1, M=20, n_cap_K=15, n_exp=10, n_ten=10,
               n_swp_K=7, both_sides=False, residual=RESID_PRICE, beta=0.5):
    """LMM12 markets: caplet smiles (n_cap_K strikes) on forwards 1..M-1 and an
    n_exp x n_ten swaption grid (n_swp_K strikes), strikes K = centre exp(m),
    m evenly spread over [-0.8, 0.8] (the paper's moneyness range)."""
    parts = _empty()
    truths, noises = [], []
    for j in range(n_markets):
        g = rng(seed + j)
        inst = _lmm_instance(M, n_cap_K, n_exp, n_ten, n_swp_K, both_sides)
        _append(parts, *inst)
        truths.append(_lmm12_truth(g))
        noises.append(g.normal(0.0, 0.002, len(inst[-1])))
    m = _finish(parts, MODEL_LMM12, FORMULA_HAGAN2002, residual, beta)
    return m, np.array(truths), np.concatenate(noises)


def perfwd_markets(seed=SEED_BASE + 6000, n_markets=3, M=13, nK=9, formula=FORMULA_HAGAN2002,
                   residual=RESID_VOL):
    """PERFWD caplet markets (equal size: M forwards x nK strikes each, the
    shape of the paper's 13 x 9 data), per-forward true triples
    alpha ~ U[0.02, 0.05], rho ~ U[-0.5, 0], nu ~ U[0.2, 0.6]."""
    parts = _empty()
    truths, noises = [], []
    for j in range(n_markets):
        g = rng(seed + j)
        _append(parts, *_caplet_instance(g, M, nK))
        truths.append(np.column_stack([g.uniform(0.02, 0.05, M), g.uniform(-0.5, 0.0, M),
                                       g.uniform(0.2, 0.6, M)]).ravel())
        noises.append(g.normal(0.0, 0.002, M * nK))
    m = _finish(parts, MODEL_PERFWD, formula, residual, 0.5)
    return m, np.array(truths), np.concatenate(noises)


def mm_markets(seed=SEED_BASE + 7000, n_markets=3, M=13, nK=9, formula=FORMULA_HAGAN2002,
               residual=RESID_VOL):
    """Mercurio-Morini caplet markets (equal size: M forwards x nK strikes
    each), true alpha_i ~ U[0.02, 0.05], phi_i ~ U[-0.5, 0], sigma ~
    U[0.2, 0.6]; point layout (alpha_1, phi_1, ..., alpha_M, phi_M, sigma)."""
    parts = _empty()
    truths, noises = [], []
    for j in range(n_markets):
        g = rng(seed + j)
        _append(parts, *_caplet_instance(g, M, nK))
        pairs = np.column_stack([g.uniform(0.02, 0.05, M), g.uniform(-0.5, 0.0, M)]).ravel()
        truths.append(np.concatenate([pairs, [g.uniform(0.2, 0.6)]]))
        noises.append(g.normal(0.0, 0.002, M * nK))
    m = _finish(parts, MODEL_MM, formula, residual, 0.5)
    return m, np.array(truths), np.concatenate(noises)


def reb_markets(seed=SEED_BASE + 8000, n_markets=3, M=13, nK=9, formula=FORMULA_HAGAN2002,
                residual=RESID_VOL):
    """Rebonato caplet markets (equal size), true kappa_i ~ U[0.001, 0.003],
    phi_i ~ U[-0.5, 0], g = (a, b, c, d) ~ (U[2, 6], U[20, 60], U[0.2, 0.5],
    U[15, 35]), h = (a_h, b_h, c_h, d_h) ~ (U[0.001, 0.1], U[10, 30],
    U[3, 8], U[0.3, 0.8]) (around the paper's calibrated values); point
    layout (kappa_1, phi_1, ..., kappa_M, phi_M, a, b, c, d, a_h, b_h, c_h,
    d_h)."""
    parts = _empty()
    truths, noises = [], []
    for j in range(n_markets):
        g = rng(seed + j)
        _append(parts, *_caplet_instance(g, M, nK))
        pairs = np.column_stack([g.uniform(0.001, 0.003, M), g.uniform(-0.5, 0.0, M)]).ravel()
        gh = [g.uniform(2, 6), g.uniform(20, 60), g.uniform(0.2, 0.5), g.uniform(15, 35),
              g.uniform(0.001, 0.1), g.uniform(10, 30), g.uniform(3, 8), g.uniform(0.3, 0.8)]
        truths.append(np.concatenate([pairs, gh]))
        noises.append(g.normal(0.0, 0.002, M * nK))
    m = _finish(parts, MODEL_REB, formula, residual, 0.5)
    return m, np.array(truths), np.concatenate(noises)


def complete_market(market, model_vols, noise):
    """Market vols = model vols at the true parameters + noise."""
    m = dict(market)
    m["q_vol"] = np.ascontiguousarray(np.asarray(model_vols, float) + np.asarray(noise, float))
    return m


def as_vol_market(market):
    """Same market, vol residuals (used to read model vols)."""
    m = dict(market)
    m["residual"] = RESID_VOL
    return m


def random_box_points(model, n, seed, lb=None, ub=None):
    lb0, ub0 = box(model)
    lb = lb0 if lb is None else np.asarray(lb, float)
    ub = ub0 if ub is None else np.asarray(ub, float)
    g = rng(seed)
    u = g.random((n, len(lb)))
    return lb + (ub - lb) * u


def select_instances(market, idx):
    """The sub-batch of instances idx (in that order) of a CSR market."""
    idx = [int(i) for i in np.atleast_1d(idx)]
    out = {k: v for k, v in market.items() if not isinstance(v, np.ndarray)}
    spans = {"fwd": ("fwd_off", ("fwd_T", "fwd_tau", "fwd_F", "fwd_P")),
             "und": ("und_off", ("und_first", "und_len")),
             "q": ("q_off", ("q_und", "q_kind", "q_K", "q_w", "q_vol"))}
    for off_key, keys in spans.values():
        off = np.asarray(market[off_key])
        out[off_key] = np.concatenate([[0], np.cumsum([off[i + 1] - off[i] for i in idx])]
                                      ).astype(np.int32)
        for k in keys:
            if k in market:
                a = np.asarray(market[k])
                out[k] = np.ascontiguousarray(np.concatenate(
                    [a[off[i]:off[i + 1]] for i in idx]) if idx else a[:0])
    return out


def n_quotes(market):
    return np.diff(np.asarray(market["q_off"]))


def n_inst(market):
    return len(market["q_off"]) - 1


# ---------------------------------------------------------------------------
# The paper's market data (Sec. 4): 6M EURIBOR, valuation date 21/11/2011.
# ---------------------------------------------------------------------------
GOLDEN_DIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "tests",
                          "golden")
PAPER_MONEYNESS = (-0.8, -0.6, -0.4, -0.2, 0.0, 0.2, 0.4, 0.6, 0.8)
_VALUATION = datetime.date(2011, 11, 21)


def _rows(name, golden_dir=None):
    rows = []
    with open(os.path.join(golden_dir or GOLDEN_DIR, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def _date(text):
    d, m, y = (int(v) for v in text.replace("-", "/").split("/"))
    return datetime.date(y + 2000 if y < 100 else y, m, d)


def paper_discount(dates, golden_dir=None):
    """P(0, t) on the paper's discount factor curve at the given dates:
    log-linear interpolation in calendar days between pillars (the paper
    names no interpolation; this one reproduces the forward F_1 = 1.196%
    implied by its calibrated Hagan parameters)."""
    pts = [(_date(r[0]), float(r[1])) for r in _rows("paper_discount_curve.txt", golden_dir)]
    days = np.array([(d - _VALUATION).days for d, _ in pts], float)
    logp = np.log([p for _, p in pts])
    x = np.array([(d - _VALUATION).days for d in dates], float)
    return np.exp(np.interp(x, days, logp))


def paper_caplet_market(golden_dir=None, model=MODEL_PERFWD, formula=FORMULA_PAPER_EQ3,
                        residual=RESID_VOL, beta=0.5, fwd_F=None):
    """The caplet market of the paper's Sec. 4.1.1 calibration, one instance.

    Forward i (i = 1..13) fixes on the i-th date of the smiles table and pays
    six months later on the next one (the 13th: 21/11/2018).  T_i = ACT/365
    years from 21/11/2011; tau_i = ACT/360 accrual; F_i = (P(0, T_i) /
    P(0, T_i + tau_i) - 1) / tau_i from the discount curve; P = P(0, pay).
    Quotes: K = F_i exp(m), m = -80%..80% (the table's moneyness ln(K/F)),
    market vols in % / 100, weight 1 (the paper's f_c: plain sum of squared
    vol differences), out-of-the-money side (put below F, call above).
    Quote order: forward-major, moneyness ascending.  ``fwd_F`` replaces
    the curve's forwards (strikes follow them)."""
    smiles = _rows("paper_forward_smiles.txt", golden_dir)
    fix = [_date(r[0]) for r in smiles]
    pay = fix[1:] + [datetime.date(fix[-1].year, fix[-1].month + 6, fix[-1].day)
                     if fix[-1].month <= 6 else
                     datetime.date(fix[-1].year + 1, fix[-1].month - 6, fix[-1].day)]
    P0 = paper_discount(fix, golden_dir)
    P1 = paper_discount(pay, golden_dir)
    T = np.array([(d - _VALUATION).days / 365.0 for d in fix])
    tau = np.array([(b - a).days / 360.0 for a, b in zip(fix, pay)])
    F = (P0 / P1 - 1.0) / tau if fwd_F is None else np.asarray(fwd_F, float)
    n = len(fix)
    mny = np.array(PAPER_MONEYNESS)
    q_und = np.repeat(np.arange(n), len(mny)).astype(np.int32)
    q_K = (F[:, None] * np.exp(mny)[None, :]).ravel()
    q_kind = np.where(np.tile(mny, n) < 0.0, KIND_PUT, KIND_CALL).astype(np.int32)
    parts = _empty()
    _append(parts, T, tau, F, P1, np.arange(n), np.ones(n, np.int32), q_und, q_kind, q_K)
    m = _finish(parts, model, formula, residual, beta)
    m["q_vol"] = np.array([[float(v) / 100.0 for v in r[1:]] for r in smiles]).ravel()
    return m


def perfwd_as_global4(market):
    """A PERFWD market re-laid as a GLOBAL4 market with one instance per
    forward (that forward and its caplets): the PERFWD cost is the sum of
    these instances' costs at (alpha_i, beta, rho_i, nu_i).  Single-instance
    PERFWD markets only."""
    assert len(market["fwd_off"]) == 2, "one PERFWD instance"
    nf = int(market["fwd_off"][1])
    q_und = np.asarray(market["q_und"])
    first = np.asarray(market["und_first"])
    parts = _empty()
    q_idx = []
    for i in range(nf):
        us = np.nonzero(first == i)[0]
        qs = np.nonzero(np.isin(q_und, us))[0]
        q_idx.append(qs)
        local_u = np.searchsorted(us, q_und[qs])
        _append(parts, [market["fwd_T"][i]], [market["fwd_tau"][i]], [market["fwd_F"][i]],
                [market["fwd_P"][i]], np.zeros(len(us), np.int32), np.ones(len(us), np.int32),
                local_u, np.asarray(market["q_kind"])[qs], np.asarray(market["q_K"])[qs])
    m = _finish(parts, MODEL_GLOBAL4, market["formula"], market["residual"], market["beta"])
    qi = np.concatenate(q_idx)
    m["q_vol"] = np.asarray(market["q_vol"], float)[qi].copy()
    m["q_w"] = np.asarray(market["q_w"], float)[qi].copy()
    return m


def perfwd_points_as_global4(x, beta):
    """(n_fwd * 3,) PERFWD point -> (n_fwd, 4) GLOBAL4 points (alpha, beta,
    rho, nu), one per forward instance of ``perfwd_as_global4``."""
    t = np.asarray(x, float).reshape(-1, 3)
    return np.column_stack([t[:, 0], np.full(len(t), beta), t[:, 1], t[:, 2]])


def global4_points_as_perfwd(y):
    """Inverse of ``perfwd_points_as_global4`` (drops beta)."""
    y = np.asarray(y, float)
    return y[:, [0, 2, 3]].ravel()


# ---------------------------------------------------------------------------
# Monte Carlo pricing problems (the Hagan SABR/LIBOR dynamics of Sec. 2.1)
# ---------------------------------------------------------------------------
# Correlation parameters y = (eta1, lambda1, eta2, lambda2, lambda3) of the
# paper's Hagan swaption calibration (Sec. 4.1.2).
PAPER_HAGAN_CORR = (0.814904, 3.378797, 0.975928, 3.777324, 0.013940)


def mc_problem_arrays(T, tau, F0, alpha, beta, phi, sigma, y, P0, opt_a, opt_b, opt_K):
    """A Monte Carlo pricing problem as a dict of arrays (forward arrays [M],
    y [5], options (a, b, K): payer swaption expiring at T_a on forwards
    a..b-1, b = a + 1 the caplet on F_a)."""
    M = len(T)

    def f(v):
        v = np.asarray(v, float)
        if v.ndim == 0:
            return np.full(M, float(v))
        assert v.shape == (M,), "forward arrays need one entry per forward"
        return v.copy()
    return dict(T=f(T), tau=f(tau), F0=f(F0), alpha=f(alpha), beta=f(beta), phi=f(phi),
                sigma=f(sigma), y=np.asarray(y, float).copy(), P0=float(P0),
                opt_a=np.asarray(opt_a, np.int32).copy(), opt_b=np.asarray(opt_b, np.int32).copy(),
                opt_K=np.asarray(opt_K, float).copy())


def paper_mc_problem(golden_dir=None, moneyness=PAPER_MONEYNESS, y=PAPER_HAGAN_CORR):
    """The paper's caplet market (Sec. 4.1.1: 13 EURIBOR forwards, fixing
    dates, accruals and forwards from the printed curve) under the Hagan
    model with its printed caplet calibration (phi_ii, sigma_i, alpha_i;
    beta = 0.5) and swaption correlations y; options: the 13 x 9 caplets
    K = F_i exp(m) of the smiles table.  P0 = P(0, T_1) from the curve."""
    m = paper_caplet_market(golden_dir)
    prm = np.array([[float(v) for v in r[1:]] for r in _rows("paper_hagan_caplet_params.txt",
                                                             golden_dir)])
    T, tau, F = m["fwd_T"], m["fwd_tau"], m["fwd_F"]
    P0 = float(m["fwd_P"][0] * (1.0 + tau[0] * F[0]))
    M = len(T)
    mny = np.asarray(moneyness, float)
    a = np.repeat(np.arange(M), len(mny))
    return mc_problem_arrays(T, tau, F, prm[:, 2], 0.5, prm[:, 0], prm[:, 1], y, P0, a, a + 1,
                             F[a] * np.exp(np.tile(mny, M)))


def mc_problem(seed=SEED_BASE + 9000, M=10, n_cap_K=3, n_swaptions=6, beta=None):
    """Synthetic pricing problem: semi-annual fixings from 0.5y with jitter,
    forwards 1-4%, lognormal-equivalent vols 15-40%, phi_ii in (-0.7, 0.3),
    sigma_i in (0.1, 0.8), beta 0.5 (or uniform in [0.2, 1] when beta is
    'random'); caplets on every forward at n_cap_K strikes around the
    forward and n_swaptions random payer swaptions (a < b <= M) at strikes
    around the mean of their forwards."""
    g = rng(seed)
    T = 0.5 * np.arange(1, M + 1) + g.uniform(-0.02, 0.02, M)
    tau = 0.5 + g.uniform(0.0, 0.02, M)
    F = g.uniform(0.01, 0.04, M)
    if beta == "random":
        bet = g.uniform(0.2, 1.0, M)
    else:
        bet = np.full(M, 0.5 if beta is None else float(beta))
    alpha = g.uniform(0.15, 0.40, M) * F ** (1.0 - bet)
    phi = g.uniform(-0.7, 0.3, M)
    sigma = g.uniform(0.1, 0.8, M)
    y = (g.uniform(0.5, 0.9), g.uniform(0.5, 4.0), g.uniform(0.5, 0.95), g.uniform(0.5, 4.0),
         g.uniform(0.0, 0.5))
    P0 = float(np.exp(-0.02 * T[0]))
    mny = np.linspace(-0.3, 0.3, n_cap_K) if n_cap_K > 1 else np.zeros(1)
    ca = np.repeat(np.arange(M), len(mny))
    K = list(F[ca] * np.exp(np.tile(mny, M)))
    a = list(ca)
    b = list(ca + 1)
    for _ in range(n_swaptions):
        sa = int(g.integers(0, M - 1)) if M > 1 else 0
        sb = int(g.integers(sa + 1, M + 1))
        a.append(sa)
        b.append(sb)
        K.append(float(F[sa:sb].mean() * np.exp(g.uniform(-0.3, 0.3))))
    return mc_problem_arrays(T, tau, F, alpha, bet, phi, sigma, y, P0, a, b, K)


def paper_mc_swaption_problem(golden_dir=None, y=PAPER_HAGAN_CORR):
    """The fourteen swaptions of the paper's Hagan swaption table (Sec. 4.1.2:
    expiries 0.5-2 years, tenors 1-4 years, moneyness -40%..40%) on its
    EURIBOR market under the printed caplet calibration and correlations.
    Swaption x by L expires at the fixing x years out (fixing index 2x - 1)
    and covers the 2L semi-annual forwards from there; K = S0 exp(m), S0 the
    forward swap rate of those forwards with their own accruals as the fixed
    leg's (the paper does not state the fixed leg's conventions).  Also
    returns the printed market and Monte Carlo prices (% of notional)."""
    base = paper_mc_problem(golden_dir, y=y)
    rows = [[float(v) for v in r] for r in _rows("paper_hagan_swaption_prices.txt", golden_dir)]
    tau, F = base["tau"], base["F0"]
    P = [base["P0"]]
    for k in range(len(F)):
        P.append(P[-1] / (1.0 + tau[k] * F[k]))
    a, b, K = [], [], []
    for e, t, m, _, _ in rows:
        sa = int(round(2 * e)) - 1
        sb = sa + int(round(2 * t))
        A = sum(tau[i] * P[i + 1] for i in range(sa, sb))
        S0 = (P[sa] - P[sb]) / A
        a.append(sa)
        b.append(sb)
        K.append(S0 * np.exp(m / 100.0))
    prob = mc_problem_arrays(base["T"], tau, F, base["alpha"], base["beta"], base["phi"],
                             base["sigma"], y, base["P0"], a, b, K)
    printed = np.array([[r[3], r[4]] for r in rows])
    return prob, printed
