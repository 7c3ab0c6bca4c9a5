"""Pins of the oracle's Monte Carlo pricer under the Hagan SABR/LIBOR dynamics
(Sec. 2.1; the swaption pricer S_MC of Sec. 3 and the caplet pricer of Table
haganMCpricer).  Against what the mathematics fixes, not against itself:
Philox4x32-10 known-answer vectors (Random123), the law of the normals, the
correlation factor against the block matrix of eqs. (rhoij), (thetaij),
(phiij), the spot-measure identities (a zero-strike swaption is worth
P(0, T_a) - P(0, T_b) whatever the model parameters), the Black-76 caplet at
beta = 1 and sigma = 0, the Bachelier caplet at beta = 0 and sigma = 0, the
covariance of the forwards after one step, the skew of the SABR smile
against Hagan's expansion, and path-slice invariance of the counter-based
streams."""
import math

import numpy as np
import pytest
from scipy import optimize, stats

from paper_2408_01470_amd import inputs as I

RANDOM123_KAT = [  # philox4x32-10 known-answer vectors of the Random123 distribution
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


@pytest.mark.parametrize("ctr,key,out", RANDOM123_KAT)
def test_philox4x32_known_answers(oracle, ctr, key, out):
    assert tuple(int(v) for v in oracle.philox4x32(ctr, key)) == out


def test_normals_layout(oracle):
    """Pairs 2b and 2b + 1 of step s on path p: Box-Muller of block (b, s,
    p_lo, p_hi) under key (seed_lo, seed_hi), words (w0, w1) and (w2, w3),
    32-bit uniforms u1 = (w + 1) 2^-32, u2 = w' 2^-32."""
    seed, path, step, M = (7 << 32) + 3, (1 << 32) + 5, 11, 5
    xi = oracle.mc_normals(seed, path, step, M)
    for m in range(M):
        w = [int(v) for v in oracle.philox4x32((m // 2, step, path & 0xFFFFFFFF, path >> 32),
                                               (seed & 0xFFFFFFFF, seed >> 32))]
        u1 = (w[2 * (m % 2)] + 1) / 2.0 ** 32
        u2 = w[2 * (m % 2) + 1] / 2.0 ** 32
        r = math.sqrt(-2.0 * math.log(u1))
        assert xi[2 * m] == pytest.approx(r * math.cos(2 * math.pi * u2), rel=1e-15, abs=1e-15)
        assert xi[2 * m + 1] == pytest.approx(r * math.sin(2 * math.pi * u2), rel=1e-15,
                                              abs=1e-15)


def test_normals_are_standard_normal(oracle):
    z = np.array([oracle.mc_normals(123, p, s, 4) for p in range(2500) for s in range(4)])
    n = z.size
    flat = z.ravel()
    assert abs(flat.mean()) < 5 / math.sqrt(n)
    assert abs(flat.var() - 1.0) < 5 * math.sqrt(2.0 / n)
    assert stats.kstest(flat, "norm").pvalue > 1e-3
    c = np.corrcoef(z.T)
    assert np.max(np.abs(c - np.eye(8))) < 5 / math.sqrt(z.shape[0])


def test_step_counts(oracle):
    for length, dt in ((0.5, 0.1), (0.49863014, 0.1), (1.0, 1e-3), (0.3, 1.0), (2.0, 0.7),
                       (1e-9, 0.01)):
        n = oracle.mc_steps(length, dt)
        assert n >= 1 and n * dt >= length * (1 - 1e-15) and (n - 1) * dt < length


def test_factor_reproduces_a_valid_correlation(oracle):
    """Positive-definite block matrix: B B^T is the matrix."""
    T = 0.5 * np.arange(1, 9)
    phi = np.full(8, -0.4)
    y = (0.7, 1.0, 0.8, 1.5, 0.2)
    C = oracle.mc_corr_matrix(T, phi, y)
    assert np.linalg.eigvalsh(C).min() > 0
    B = oracle.mc_factor(T, phi, y)
    np.testing.assert_allclose(B @ B.T, C, atol=1e-13)
    # the blocks by their equations
    assert C[2, 5] == pytest.approx(0.7 + 0.3 * math.exp(-1.0 * 1.5))
    assert C[8 + 2, 8 + 5] == pytest.approx(0.8 + 0.2 * math.exp(-1.5 * 1.5))
    assert C[2, 8 + 5] == pytest.approx(-0.4 * math.exp(-0.2 * 1.5))


def test_factor_alive_rows_are_leading(oracle):
    """The forwards alive during [T_{j-1}, T_j) (k >= j) draw on the first
    2(M - j) normals only: their rows of the factor vanish beyond."""
    for p in (I.paper_mc_problem(), I.mc_problem()):
        M = len(p["T"])
        B = oracle.mc_factor(p["T"], p["phi"], p["y"])
        for j in range(M):
            for k in range(j, M):
                assert not np.any(B[k, 2 * (M - j):]) and not np.any(B[M + k, 2 * (M - j):])


def test_factor_repairs_the_paper_correlation(oracle):
    """The paper's calibrated phi_ii (mixed signs) and y give an indefinite
    matrix; the repaired B B^T is a correlation matrix (unit diagonal,
    positive semi-definite) that keeps the positive spectrum's part."""
    pm = I.paper_mc_problem()
    C = oracle.mc_corr_matrix(pm["T"], pm["phi"], pm["y"])
    lam, Q = np.linalg.eigh(C)
    assert lam.min() < -1.0
    B = oracle.mc_factor(pm["T"], pm["phi"], pm["y"])
    R = B @ B.T
    np.testing.assert_allclose(np.diag(R), 1.0, atol=1e-14)
    assert np.linalg.eigvalsh(R).min() > -1e-12
    Cp = (Q * np.maximum(lam, 0)) @ Q.T
    d = np.sqrt(np.diag(Cp))
    np.testing.assert_allclose(R, Cp / d[:, None] / d[None, :], atol=1e-12)


def _discounts(p):
    """P(0, T_k) for k = 0..M from P(0, T_0) and the initial forwards."""
    out = [p["P0"]]
    for k in range(len(p["T"])):
        out.append(out[-1] / (1.0 + p["tau"][k] * p["F0"][k]))
    return np.array(out)


def _within(mc, se, exact, bias=0.0, k=4.5):
    assert np.all(np.abs(mc - exact) <= k * se + bias), np.c_[mc, exact, se]


def test_zero_strike_swaptions_are_bond_spreads(oracle):
    """K = 0: the payoff is the floating leg 1 - P(T_a, T_b), worth
    P(0, T_a) - P(0, T_b) under the spot measure for any volatility model;
    the drift and the numeraire must match for this to hold."""
    p = I.mc_problem(seed=I.SEED_BASE + 9100, M=8, n_cap_K=1, n_swaptions=0, beta="random")
    p["sigma"] *= 1.5
    ab = [(0, 1), (0, 8), (2, 3), (2, 8), (4, 6), (7, 8), (1, 5)]
    p["opt_a"] = np.array([a for a, _ in ab], np.int32)
    p["opt_b"] = np.array([b for _, b in ab], np.int32)
    p["opt_K"] = np.zeros(len(ab))
    m, se = oracle.mc_price(p, 40000, 0.02, 11)
    P = _discounts(p)
    exact = np.array([P[a] - P[b] for a, b in ab])
    _within(m, se, exact, bias=2e-5 * exact)
    assert np.all(se < 1e-2 * exact)


def _black(F, K, T, vol):
    sd = vol * math.sqrt(T)
    d1 = (math.log(F / K) + 0.5 * sd * sd) / sd
    return F * stats.norm.cdf(d1) - K * stats.norm.cdf(d1 - sd)


def _bachelier(F, K, T, vol):
    sd = vol * math.sqrt(T)
    d = (F - K) / sd
    return (F - K) * stats.norm.cdf(d) + sd * stats.norm.pdf(d)


@pytest.mark.parametrize("beta", [1.0, 0.0], ids=["black", "bachelier"])
def test_caplets_match_closed_forms(oracle, beta):
    """sigma = 0 freezes V at alpha: beta = 1 is the lognormal LIBOR model
    (Black-76 caplets), beta = 0 the normal one (Bachelier caplets), both
    under the forward measure of the payment date."""
    M = 4
    p = I.mc_problem(seed=I.SEED_BASE + 9200, M=M, n_cap_K=3, n_swaptions=0, beta=beta)
    p["sigma"][:] = 0.0
    if beta == 0.0:
        p["alpha"] = 0.0035 + 0.0005 * np.arange(M)      # 35-50 bp normal vols
        p["F0"] = 0.03 + 0.002 * np.arange(M)
        p["opt_K"] = p["F0"][p["opt_a"]] + np.tile([-0.004, 0.0, 0.004], M)
    m, se = oracle.mc_price(p, 40000, 0.01, 5)
    P = _discounts(p)
    f = _black if beta == 1.0 else _bachelier
    exact = np.array([P[a + 1] * p["tau"][a] * f(p["F0"][a], K, p["T"][a], p["alpha"][a])
                      for a, K in zip(p["opt_a"], p["opt_K"])])
    _within(m, se, exact, bias=3e-3 * exact)
    assert np.all(se < 0.05 * exact)


def test_one_step_forward_covariance(oracle):
    """beta = 0, sigma = 0 and one step to T_0: F(T_0) = F(0) + drift h +
    alpha sqrt(T_0) (B xi)_W with a drift that is the same on every path, so
    Cov(F_k, F_l) = alpha_k alpha_l T_0 rho_{k,l} (eq. rhoij).  The forwards
    are read back from zero-strike swaptions (0, b), b = 1..M."""
    M = 5
    p = I.mc_problem(seed=I.SEED_BASE + 9300, M=M, n_cap_K=1, n_swaptions=0, beta=0.0)
    p["sigma"][:] = 0.0
    p["alpha"] = np.full(M, 0.002)
    p["F0"] = np.full(M, 0.04)
    p["phi"] = np.full(M, -0.3)                 # one sign: a positive-definite block matrix
    assert np.linalg.eigvalsh(oracle.mc_corr_matrix(p["T"], p["phi"], p["y"])).min() > 0
    p["opt_a"] = np.zeros(M, np.int32)
    p["opt_b"] = np.arange(1, M + 1, dtype=np.int32)
    p["opt_K"] = np.zeros(M)
    n = 40000
    X = oracle.mc_paths(p, n, 10.0, 3)
    Q = 1.0 - X / p["P0"]                       # P(T_0, T_b) per path
    Qp = np.column_stack([np.ones(n), Q])
    F = (Qp[:, :-1] / Qp[:, 1:] - 1.0) / p["tau"][None, :]
    C = np.cov(F.T) / (np.outer(p["alpha"], p["alpha"]) * p["T"][0])
    rho = oracle.mc_corr_matrix(p["T"], p["phi"], p["y"])[:M, :M]
    np.testing.assert_allclose(C, rho, atol=6 / math.sqrt(n))


def _implied(price, F, K, T, disc):
    return optimize.brentq(lambda v: disc * _black(F, K, T, v) - price, 1e-4, 3.0)


@pytest.mark.parametrize("phi", [-0.5, 0.5])
def test_sabr_smile_skew(oracle, phi):
    """One forward: (F, V) under its payment measure is the SABR model with
    correlation phi_ii, so the Monte Carlo smile follows Hagan's expansion
    (to its O(T) accuracy, here 0.5 vol points) and its skew has the sign
    of phi."""
    p = I.mc_problem_arrays(T=[1.0], tau=[0.5], F0=[0.03], alpha=[0.3 * math.sqrt(0.03)],
                            beta=0.5, phi=[phi], sigma=[0.5], y=(0.8, 1.0, 0.9, 1.0, 0.1),
                            P0=0.98, opt_a=[0, 0, 0], opt_b=[1, 1, 1],
                            opt_K=0.03 * np.exp([-0.2, 0.0, 0.2]))
    m, se = oracle.mc_price(p, 100000, 0.005, 21)
    disc = p["P0"] / (1 + 0.5 * 0.03) * 0.5
    mc_vol = np.array([_implied(v, 0.03, K, 1.0, disc) for v, K in zip(m, p["opt_K"])])
    hagan = np.array([oracle.hagan2002_vol(0.03, K, 1.0, p["alpha"][0], 0.5, phi, 0.5)
                      for K in p["opt_K"]])
    assert np.max(np.abs(mc_vol - hagan)) < 0.005
    assert np.sign(mc_vol[2] - mc_vol[0]) == np.sign(phi)
    assert abs((mc_vol[2] - mc_vol[0]) - (hagan[2] - hagan[0])) < 0.004


def test_path_slices_are_the_same_paths(oracle):
    p = I.mc_problem(seed=I.SEED_BASE + 9400, M=6, n_cap_K=2, n_swaptions=3)
    X = oracle.mc_paths(p, 40, 0.1, 9)
    Y = oracle.mc_paths(p, 15, 0.1, 9, path0=25)
    assert np.array_equal(X[25:], Y)
    Z = oracle.mc_paths(p, 40, 0.1, 10)
    assert not np.array_equal(X, Z)


def test_mc_rejects_bad_options(oracle):
    p = I.mc_problem(seed=I.SEED_BASE + 9500, M=4, n_cap_K=1, n_swaptions=0)
    p["opt_b"][0] = 5
    with pytest.raises(ValueError):
        oracle.mc_paths(p, 2, 0.1, 1)


@pytest.mark.parametrize("phi", [[0.4, 0.4, 0.4, 0.4, -0.4], [-0.5] * 5],
                         ids=["mixed-signs", "one-sign"])
def test_caplet_does_not_depend_on_the_other_forwards(oracle, phi):
    """Under its payment measure (F_k, V_k) is the SABR model with phi_kk
    whatever the other forwards do, so a caplet priced in the joint spot-
    measure simulation equals the same caplet priced with its forward alone.
    This fixes the drift of V_k: the coefficient of d_i is the covariance of
    Z_k with W_i, phi_{i,k} of eq. (phiij) (signs mixed here, so phi_{k,i}
    would differ; with one sign, dropping that drift shows)."""
    M = 5
    phi = np.array(phi)
    F, alpha = 0.10, 0.6 * math.sqrt(0.10)
    p = I.mc_problem_arrays(T=np.arange(1.0, M + 1), tau=1.0, F0=F, alpha=alpha,
                            beta=0.5, phi=phi, sigma=0.8, y=(0.0, 1.0, 0.0, 1.0, 0.3), P0=0.97,
                            opt_a=[M - 1, M - 1], opt_b=[M, M], opt_K=[F, 1.5 * F])
    assert np.linalg.eigvalsh(oracle.mc_corr_matrix(p["T"], p["phi"], p["y"])).min() > 0
    m, se = oracle.mc_price(p, 60000, 0.02, 31)
    P = _discounts(p)
    q = I.mc_problem_arrays(T=[float(M)], tau=1.0, F0=F, alpha=alpha, beta=0.5,
                            phi=[phi[-1]], sigma=0.8, y=p["y"], P0=P[M - 1], opt_a=[0, 0],
                            opt_b=[1, 1], opt_K=[F, 1.5 * F])
    m1, se1 = oracle.mc_price(q, 60000, 0.02, 32)
    assert np.all(np.abs(m - m1) <= 4.5 * np.hypot(se, se1)), np.c_[m, m1, se, se1]


def test_paper_swaption_prices(oracle):
    """Sec. 4.1.2: at the printed caplet calibration and swaption
    correlations, the Monte Carlo prices of the paper's fourteen swaptions x
    five strikes (70 cells, % of notional) reproduce the printed S_MC within
    5% each and 3% on average (the fixed leg's conventions are not printed:
    the remainder is a common +2.4%), while the printed market prices S_Black
    lie up to 20% away: the pin follows the model, not the market."""
    p, printed = I.paper_mc_swaption_problem()
    m, se = oracle.mc_price(p, 100000, 0.01, 5)
    mc = 100.0 * m
    rel = mc / printed[:, 1] - 1.0
    assert np.max(np.abs(rel)) < 0.05 and np.mean(np.abs(rel)) < 0.03, rel
    assert np.max(np.abs(mc / printed[:, 0] - 1.0)) > 0.10


def _sabr_forward_measure(F0, alpha, beta, phi, sigma, T, K, n, dt, seed):
    """Plain numpy Monte Carlo of one forward's SABR pair under its payment
    measure (no drifts: dF = V F^beta dW, dV = sigma V dZ, corr phi), the
    textbook form a caplet sees; E[(F_T - K)^+] per strike with its error."""
    g = np.random.default_rng(seed)
    steps = int(np.ceil(T / dt))
    h = T / steps
    F = np.full(n, F0)
    V = np.full(n, alpha)
    for _ in range(steps):
        z1 = g.standard_normal(n)
        z2 = phi * z1 + math.sqrt(1.0 - phi * phi) * g.standard_normal(n)
        s = V * np.maximum(F, 0.0) ** beta
        F = np.maximum(F + s * math.sqrt(h) * z1, 0.0)
        V = V * np.exp(-0.5 * sigma * sigma * h + sigma * math.sqrt(h) * z2)
    pay = np.maximum(F[:, None] - np.asarray(K)[None, :], 0.0)
    return pay.mean(axis=0), pay.std(axis=0, ddof=1) / math.sqrt(n)


def test_caplet_matches_its_forward_measure_sabr(oracle):
    """The joint spot-measure simulation of five forwards prices the last
    forward's caplets as the SABR model under that caplet's payment measure
    does (an independent drift-free simulation): the spot-measure drifts of
    F and of V (mu^F, mu^V of Sec. 2.1) are exactly the change of measure."""
    M = 5
    phi = np.array([-0.5] * M)
    F, alpha = 0.10, 0.6 * math.sqrt(0.10)
    K = [F, 1.5 * F]
    p = I.mc_problem_arrays(T=np.arange(1.0, M + 1), tau=1.0, F0=F, alpha=alpha, beta=0.5,
                            phi=phi, sigma=0.8, y=(0.0, 1.0, 0.0, 1.0, 0.3), P0=0.97,
                            opt_a=[M - 1, M - 1], opt_b=[M, M], opt_K=K)
    assert np.linalg.eigvalsh(oracle.mc_corr_matrix(p["T"], p["phi"], p["y"])).min() > 0
    m, se = oracle.mc_price(p, 100000, 0.02, 41)
    P = _discounts(p)
    ref, rse = _sabr_forward_measure(F, alpha, 0.5, -0.5, 0.8, float(M), K, 100000, 0.02, 42)
    ref, rse = P[M] * ref, P[M] * rse            # tau = 1: the caplet is P(0, pay) E[(F - K)^+]
    assert np.all(np.abs(m - ref) <= 4.5 * np.hypot(se, rse)), np.c_[m, ref, se, rse]


def test_paths_do_not_depend_on_threads(oracle):
    """Each path's numbers come from its own counters: one host thread and
    all of them give the same paths bit for bit."""
    p = I.mc_problem(seed=I.SEED_BASE + 9450, M=7, n_cap_K=2, n_swaptions=4)
    n = oracle.max_threads()
    try:
        oracle.set_threads(1)
        X1 = oracle.mc_paths(p, 300, 0.05, 13)
    finally:
        oracle.set_threads(n)
    Xn = oracle.mc_paths(p, 300, 0.05, 13)
    assert np.array_equal(X1, Xn)
