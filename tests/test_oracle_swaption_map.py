"""Pins of the oracle's frozen-weight swaption map against the dynamics it
freezes (Sec. 2.1: eqs. (dinamicasHagan1), (dinamicasHagan2) with the
correlations of eqs. (rhoij), (thetaij), (phiij)).

The map gives the swap rate S = sum_k w_k F_k (weights frozen at t = 0) the
SABR parameters of its instantaneous dynamics at t = 0.  Two routes that share
nothing with the map's closed form check it:

* Ito's lemma evaluated numerically.  With g_k = w_k F_k^beta, the normal vol
  of S is a(V) = sqrt(sum_kl g_k V_k g_l V_l C^WW_kl) as a function of the
  forwards' vols V (C the block correlation matrix of (W, Z), built by the
  oracle's Monte Carlo from the three equations and pinned there against the
  paper's printed swaption prices).  Then alpha_S S0^beta = a(alpha); the
  log-vol of S moves by sum_k d_k dV_k / V_k with d_k = d ln a / d ln V_k,
  taken here by central differences; nu_S^2 = sum_kl d_k nu_k d_l nu_l C^ZZ_kl
  and rho_S = sum_kl g_k alpha_k d_l nu_l C^WZ_kl / (a nu_S).
* The oracle's Monte Carlo of the full dynamics (its forwards simulated
  jointly under the spot measure) prices short-dated swaptions; Black's
  formula at the Hagan vol of the mapped parameters must match them.

A dropped correlation kernel exp(-lambda1 |dT|), a theta on index gaps
instead of time gaps, or a wrong rho_S fails the first pin; the first of
those also fails the second.
"""
import math

import numpy as np
import pytest

from paper_2408_01470_amd import inputs as I

BETA = 0.5


def _market(M=6, seed=3):
    """Forwards fixing at 0.25 + 0.5 k with slightly uneven accruals, caplets
    on every forward (they expose alpha_k and nu_k), swaps from the first
    fixing over 2..M forwards and two swaps starting later."""
    g = np.random.default_rng(seed)
    T = 0.25 + 0.5 * np.arange(M)
    tau = 0.5 + g.uniform(-0.01, 0.02, M)
    F = 0.02 + 0.02 * np.arange(M) / (M - 1) + g.uniform(-0.002, 0.002, M)
    P0 = math.exp(-0.02 * T[0])
    P = P0 / np.cumprod(1.0 + tau * F)
    first = list(range(M)) + [0] * (M - 1) + [1, 2]
    length = [1] * M + list(range(2, M + 1)) + [3, 4]
    n_u = len(first)
    mk = dict(fwd_T=T, fwd_tau=tau, fwd_F=F, fwd_P=P,
              und_first=np.array(first, np.int32), und_len=np.array(length, np.int32),
              q_und=np.arange(n_u, dtype=np.int32), q_kind=np.zeros(n_u, np.int32),
              q_K=np.array([F[f:f + n].mean() for f, n in zip(first, length)]),
              q_w=np.ones(n_u), q_vol=np.full(n_u, 0.3),
              fwd_off=np.array([0, M], np.int32), und_off=np.array([0, n_u], np.int32),
              q_off=np.array([0, n_u], np.int32), model=I.MODEL_LMM12,
              formula=I.FORMULA_HAGAN2002, residual=I.RESID_VOL, beta=BETA)
    return mk, P0


# (a, b, c, d, a_nu, b_nu, c_nu, d_nu, rho, lambda1, eta2, lambda2): humped
# alpha and nu term structures, strong decorrelation, eta2 < 1
POINTS = [
    np.array([0.02, 0.05, 1.0, 0.03, 0.3, 0.2, 1.0, 0.3, -0.4, 2.0, 0.4, 1.5]),
    np.array([0.01, 0.08, 1.8, 0.025, 0.5, -0.3, 0.6, 0.25, 0.3, 0.7, 0.2, 3.0]),
    np.array([0.03, 0.0, 0.5, 0.02, 0.1, 0.4, 2.0, 0.2, -0.5, 1.2, 0.7, 0.5]),
]


def _swap(mk, first, n):
    """Annuity, frozen weights and swap rate (Sec. 2: the market's own
    definitions)."""
    sl = slice(first, first + n)
    tP = mk["fwd_tau"][sl] * mk["fwd_P"][sl]
    A = float(tP.sum())
    w = tP / A
    return A, w, float(w @ mk["fwd_F"][sl])


def _ito(oracle, mk, th, p, first, n):
    """(alpha_S, rho_S, nu_S) of the swap on forwards [first, first + n) by
    Ito's lemma with numerical derivatives."""
    M = len(mk["fwd_T"])
    al, nv = th[:M, 0], th[:M, 3]       # the caplets' (forwards') alpha_k, nu_k
    rho, lam1, eta2, lam2 = p[8], p[9], p[10], p[11]
    sl = slice(first, first + n)
    _, w, S0 = _swap(mk, first, n)
    C = oracle.mc_corr_matrix(mk["fwd_T"][sl], np.full(n, rho), (0.0, lam1, eta2, lam2, 0.0))
    CW, CWZ, CZ = C[:n, :n], C[:n, n:], C[n:, n:]
    g = w * mk["fwd_F"][sl] ** BETA

    def log_a(V):
        return 0.5 * math.log((g * V) @ CW @ (g * V))

    V0 = al[sl]
    h = 1e-5
    d = np.array([(log_a(V0 * np.exp(h * e)) - log_a(V0 * np.exp(-h * e))) / (2.0 * h)
                  for e in np.eye(n)])
    a = math.exp(log_a(V0))
    dn = d * nv[sl]
    nuS = math.sqrt(dn @ CZ @ dn)
    rhoS = (g * V0) @ CWZ @ dn / (a * nuS)
    return a / S0 ** BETA, rhoS, nuS


@pytest.mark.parametrize("k", range(len(POINTS)))
def test_swaption_map_is_the_instantaneous_dynamics(oracle, k):
    mk, _ = _market()
    p = POINTS[k]
    th, ok = oracle.map_params(mk, 0, p)
    assert ok
    M = len(mk["fwd_T"])
    for u in range(M, len(mk["und_first"])):
        first, n = int(mk["und_first"][u]), int(mk["und_len"][u])
        aS, rS, nS = _ito(oracle, mk, th, p, first, n)
        assert th[u, 0] == pytest.approx(aS, rel=1e-12), (u, "alpha_S")
        assert th[u, 1] == BETA
        assert th[u, 2] == pytest.approx(rS, abs=1e-8), (u, "rho_S")
        assert th[u, 3] == pytest.approx(nS, rel=1e-8), (u, "nu_S")


def test_swaption_map_nontrivial_case(oracle):
    """The pinned case is far from the degenerate ones: rho_S differs from rho
    and nu_S from the weighted mean of the nu_k, by more than the pins'
    tolerances many times over."""
    mk, _ = _market()
    p = POINTS[0]
    th, _ = oracle.map_params(mk, 0, p)
    M = len(mk["fwd_T"])
    for u in range(M, len(mk["und_first"])):
        first, n = int(mk["und_first"][u]), int(mk["und_len"][u])
        _, w, _ = _swap(mk, first, n)
        assert abs(th[u, 2] - p[8]) > 0.05
        assert abs(th[u, 3] / float(w @ th[first:first + n, 3]) - 1.0) > 0.02


def test_swaption_map_prices_short_swaptions_like_the_full_dynamics(oracle):
    """Swaptions expiring at the first fixing (T = 0.25) on 2..6 forwards,
    priced by the oracle's Monte Carlo of the joint spot-measure dynamics
    (eta1 = 0, phi_ii = rho, lambda3 = 0, beta = 1/2: the LMM12 model) and by
    Black-76 at the Hagan 2002 vol of the mapped parameters, at the money and
    0.15 in log-moneyness in the money.  Agreement within 1.2% plus three
    standard errors (the frozen-weight and Hagan expansions are first order
    in T; the observed gaps are 0.1-0.9%)."""
    mk, P0 = _market()
    p = POINTS[0]
    th, ok = oracle.map_params(mk, 0, p)
    assert ok
    M = len(mk["fwd_T"])
    rho, lam1, eta2, lam2 = p[8], p[9], p[10], p[11]
    opt_a, opt_b, opt_K, ref = [], [], [], []
    for u in range(M, 2 * M - 1):
        first, n = int(mk["und_first"][u]), int(mk["und_len"][u])
        A, _, S0 = _swap(mk, first, n)
        Te = float(mk["fwd_T"][first])
        for m in (-0.15, 0.0):
            K = S0 * math.exp(m)
            sig = oracle.hagan2002_vol(S0, K, Te, th[u, 0], BETA, th[u, 2], th[u, 3])
            opt_a.append(first)
            opt_b.append(first + n)
            opt_K.append(K)
            ref.append(oracle.black(0, S0, K, Te, sig, A))
    prob = I.mc_problem_arrays(mk["fwd_T"], mk["fwd_tau"], mk["fwd_F"], th[:M, 0], BETA,
                               np.full(M, rho), th[:M, 3], (0.0, lam1, eta2, lam2, 0.0), P0,
                               opt_a, opt_b, opt_K)
    price, se = oracle.mc_price(prob, 400_000, 0.0125, 7)
    ref = np.array(ref)
    gap = np.abs(price / ref - 1.0)
    assert np.all(gap <= 0.012 + 3.0 * se / ref), np.column_stack([opt_b, opt_K, gap, se / ref])
