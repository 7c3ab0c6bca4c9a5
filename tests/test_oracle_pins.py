"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: the paper's
worked example (its printed calibrated parameters and model vols), closed
forms, special cases that reduce to a library routine, high-precision
arithmetic, or brute force.
"""
import math

import numpy as np
import pytest
from scipy import special, stats

from conftest import load_golden
from paper_2408_01470_amd import inputs as I


# --------------------------------------------------------------------------
# Paper eq. (sigmaHagan), Sec. 2.1, against the worked example of Sec. 4.1.1
# --------------------------------------------------------------------------
def _hagan_table():
    params = {int(r[0]): tuple(map(float, r[1:])) for r in load_golden(
        "paper_hagan_caplet_params.txt")}
    vols = [(int(r[0]), int(r[1]), float(r[2]), float(r[3])) for r in load_golden(
        "paper_hagan_caplet_vols.txt")]
    return params, vols


def _eq3_table_errors(oracle, params, vols, beta):
    """Eq. (sigmaHagan) with the printed (phi_ii, sigma_i), the printed ATM model
    vol A_i = alpha_i / F_i^(1-beta) (so omega_i = 1/A_i), k = printed moneyness."""
    atm = {i: smod / 100.0 for i, mny, _, smod in vols if mny == 0}
    errs = []
    for i, mny, _, smod in vols:
        if mny == 0:
            continue
        phi, sig, _ = params[i]
        k = mny / 100.0
        # f = 1 makes alpha / f^(1-beta) = alpha = A_i for every beta
        model = oracle.paper_eq3_vol(1.0, math.exp(k), atm[i], beta, phi, sig) * 100.0
        errs.append(abs(model - smod))
    return np.array(errs)


def test_paper_eq3_reproduces_hagan_caplet_table(oracle):
    params, vols = _hagan_table()
    errs = _eq3_table_errors(oracle, params, vols, beta=0.5)
    assert len(errs) == 52                   # 13 forwards x 4 off-ATM strikes
    assert errs.max() <= 0.011               # printed to 2 decimals


@pytest.mark.parametrize("beta", [0.0, 0.3, 0.7, 1.0])
def test_paper_eq3_table_rejects_other_betas(oracle, beta):
    # the pin discriminates: the printed table is not reproduced for beta != 0.5
    params, vols = _hagan_table()
    assert _eq3_table_errors(oracle, params, vols, beta=beta).max() > 1.0


def test_paper_mre_of_hagan_fit(oracle):
    """MRE of Sec. 4.1.1 (printed 1.80e-2): mean |sigma_mkt - sigma_model| /
    sigma_mkt over all 13 x 9 cells of the forward smiles table, with the model
    of the worked example."""
    params, vols = _hagan_table()
    atm = {i: smod / 100.0 for i, mny, _, smod in vols if mny == 0}
    smiles = load_golden("paper_forward_smiles.txt")
    mny = [-80, -60, -40, -20, 0, 20, 40, 60, 80]
    rel = []
    for i, row in enumerate(smiles, start=1):
        phi, sig, _ = params[i]
        for k, s in zip(mny, row[1:]):
            mkt = float(s) / 100.0
            model = oracle.paper_eq3_vol(1.0, math.exp(k / 100.0), atm[i], 0.5, phi, sig)
            rel.append(abs(mkt - model) / mkt)
    assert len(rel) == 117
    assert abs(np.mean(rel) - 1.80e-2) <= 0.5e-4


def test_paper_eq3_reproduces_mercurio_morini_table(oracle):
    """Sec. 4.2.1: with the Mercurio-Morini map (phi^SABR = phi_i, sigma^SABR =
    sigma, beta = 0.5) eq. (sigmaHagan) reproduces the printed off-ATM vols."""
    rows = load_golden("paper_mm_caplet_params.txt")
    params = {int(r[0]): float(r[1]) for r in rows}
    sigma = 0.5986
    vols = [(int(r[0]), int(r[1]), float(r[2]), float(r[3])) for r in load_golden(
        "paper_mm_caplet_vols.txt")]
    atm = {i: smod / 100.0 for i, mny, _, smod in vols if mny == 0}
    errs = [abs(oracle.paper_eq3_vol(1.0, math.exp(mny / 100.0), atm[i], 0.5, params[i], sigma)
                * 100.0 - smod) for i, mny, _, smod in vols if mny != 0]
    assert len(errs) == 48
    assert max(errs) <= 0.011


# --------------------------------------------------------------------------
# Hagan 2002 lognormal formula (cited, Sec. 2.1): closed forms
# --------------------------------------------------------------------------
CASES = [(0.03, 0.025, 1.5, 0.04, 0.5, -0.3, 0.5), (0.02, 0.035, 4.0, 0.02, 0.3, 0.4, 0.9),
         (0.05, 0.05, 0.5, 0.2, 0.8, -0.8, 0.2), (0.03, 0.012, 9.5, 0.01, 0.0, 0.6, 1.4)]


@pytest.mark.parametrize("f,K,T,alpha,_b,rho,_n", CASES)
def test_hagan2002_lognormal_limit(oracle, f, K, T, alpha, _b, rho, _n):
    # nu = 0 and beta = 1: the model is Black with constant vol alpha
    assert oracle.hagan2002_vol(f, K, T, alpha, 1.0, rho, 0.0) == pytest.approx(alpha, rel=1e-15)


@pytest.mark.parametrize("f,K,T,alpha,_b,_r,nu", CASES)
def test_hagan2002_beta1_rho0(oracle, f, K, T, alpha, _b, _r, nu):
    # beta = 1, rho = 0: x(z) = asinh(z), sigma = alpha z/asinh(z) (1 + nu^2 T/12)
    z = nu / alpha * math.log(f / K)
    chi = 1.0 if z == 0 else z / np.arcsinh(z)
    expect = alpha * chi * (1.0 + nu * nu * T / 12.0)
    assert oracle.hagan2002_vol(f, K, T, alpha, 1.0, 0.0, nu) == pytest.approx(expect, rel=2e-15)


@pytest.mark.parametrize("f,_K,T,alpha,beta,rho,nu", CASES)
def test_hagan2002_atm_limit_and_continuity(oracle, f, _K, T, alpha, beta, rho, nu):
    # ATM value: alpha/f^(1-beta) [1 + ((1-beta)^2 alpha^2/(24 f^(2-2beta))
    #            + rho beta nu alpha/(4 f^(1-beta)) + (2 - 3 rho^2) nu^2/24) T]
    fb = f ** (1 - beta)
    atm = alpha / fb * (1 + ((1 - beta) ** 2 * alpha ** 2 / (24 * fb * fb)
                             + rho * beta * nu * alpha / (4 * fb) + (2 - 3 * rho ** 2) * nu ** 2
                             / 24) * T)
    assert oracle.hagan2002_vol(f, f, T, alpha, beta, rho, nu) == pytest.approx(atm, rel=1e-14)
    for eps in (1e-12, 1e-9, 1e-6):   # the removable singularity is continuous
        for s in (-1, 1):
            v = oracle.hagan2002_vol(f, f * (1 + s * eps), T, alpha, beta, rho, nu)
            assert v == pytest.approx(atm, rel=5 * eps + 1e-14)


@pytest.mark.parametrize("f,_K,_T,alpha,beta,rho,nu", CASES)
def test_hagan2002_small_moneyness_expansion(oracle, f, _K, _T, alpha, beta, rho, nu):
    """At T = 0 the k = ln(K/f) Taylor coefficients are Hagan et al.'s
    sigma0 {1 - (1/2)(1 - beta - rho lam) k + (1/12)[(1-beta)^2 + (2-3rho^2) lam^2] k^2},
    sigma0 = alpha/f^(1-beta), lam = nu f^(1-beta)/alpha."""
    s0 = alpha / f ** (1 - beta)
    lam = nu / alpha * f ** (1 - beta)
    h = 1e-3
    sig = lambda k: oracle.hagan2002_vol(f, f * math.exp(k), 0.0, alpha, beta, rho, nu)
    d1 = (sig(h) - sig(-h)) / (2 * h)
    d2 = (sig(h) - 2 * sig(0) + sig(-h)) / h ** 2
    assert d1 / s0 == pytest.approx(-0.5 * (1 - beta - rho * lam), abs=1e-5)
    assert d2 / s0 == pytest.approx(((1 - beta) ** 2 + (2 - 3 * rho ** 2) * lam ** 2) / 6,
                                    rel=1e-4, abs=1e-5)


def test_chi_against_high_precision(oracle):
    """z / x(z) against 50-digit arithmetic over z in [-50, 50], rho in [-0.99, 0.99]."""
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 50

    def ref(z, rho):
        if z == 0:
            return 1.0
        z, rho = mp.mpf(z), mp.mpf(rho)
        return float(z / mp.log((mp.sqrt(1 - 2 * rho * z + z * z) + z - rho) / (1 - rho)))

    worst = 0.0
    for rho in np.linspace(-0.99, 0.99, 12):
        for z in np.concatenate([-np.logspace(-12, 1.7, 40), [0.0], np.logspace(-12, 1.7, 40)]):
            r = ref(float(z), float(rho))
            worst = max(worst, abs(oracle.chi(float(z), float(rho)) - r) / r)
    assert worst <= 1e-15


# --------------------------------------------------------------------------
# Black-76
# --------------------------------------------------------------------------
BL = [(0.03, 0.02, 1.0, 0.3, 0.95), (0.03, 0.045, 5.0, 0.2, 0.8), (0.02, 0.02, 0.5, 0.6, 0.99),
      (0.04, 0.01, 10.0, 0.15, 0.6), (0.03, 0.09, 0.25, 0.25, 0.97)]


@pytest.mark.parametrize("f,K,T,s,D", BL)
def test_black_put_call_parity(oracle, f, K, T, s, D):
    c, p = oracle.black(0, f, K, T, s, D), oracle.black(1, f, K, T, s, D)
    assert c - p == pytest.approx(D * (f - K), abs=1e-15 * D * f)


@pytest.mark.parametrize("f,K,T,s,D", BL)
def test_black_against_scipy_normal(oracle, f, K, T, s, D):
    sd = s * math.sqrt(T)
    d1 = (math.log(f / K) + 0.5 * s * s * T) / sd
    d2 = d1 - sd
    call = D * (f * special.ndtr(d1) - K * special.ndtr(d2))
    put = D * (K * special.ndtr(-d2) - f * special.ndtr(-d1))
    assert oracle.black(0, f, K, T, s, D) == pytest.approx(call, rel=1e-12, abs=1e-18)
    assert oracle.black(1, f, K, T, s, D) == pytest.approx(put, rel=1e-12, abs=1e-18)
    vega = D * f * stats.norm.pdf(d1) * math.sqrt(T)
    assert oracle.black_vega(f, K, T, s, D) == pytest.approx(vega, rel=1e-13)


def test_black_atm_closed_form_and_limits(oracle):
    f, T, s, D = 0.03, 2.0, 0.4, 0.9
    # K = f: C = D f erf(sigma sqrt(T) / (2 sqrt 2))
    assert oracle.black(0, f, f, T, s, D) == pytest.approx(
        D * f * math.erf(s * math.sqrt(T) / (2 * math.sqrt(2))), rel=1e-14)
    # sigma -> 0: intrinsic value
    assert oracle.black(0, f, 0.02, T, 1e-9, D) == pytest.approx(D * 0.01, rel=1e-12)
    assert oracle.black(1, f, 0.02, T, 1e-9, D) == pytest.approx(0.0, abs=1e-20)
    # bounds and monotonicity in sigma and K
    prev = 0.0
    for sig in np.linspace(0.05, 2.0, 20):
        c = oracle.black(0, f, 0.035, T, sig, D)
        assert prev < c <= D * f
        prev = c
    prices = [oracle.black(0, f, K, T, s, D) for K in np.linspace(0.01, 0.08, 15)]
    assert np.all(np.diff(prices) < 0)


# --------------------------------------------------------------------------
# Philox4x64-10 against numpy's library implementation
# --------------------------------------------------------------------------
def test_philox_matches_numpy(oracle):
    g = np.random.default_rng(5)
    for _ in range(20):
        ctr = g.integers(0, 2 ** 63, 4, dtype=np.uint64)
        ctr[0] = ctr[0] % (2 ** 62)
        key = g.integers(0, 2 ** 63, 2, dtype=np.uint64)
        bg = np.random.Philox(counter=ctr, key=key)
        raw = np.array([bg.random_raw() for _ in range(4)], dtype=np.uint64)
        nxt = ctr.copy()
        nxt[0] += np.uint64(1)        # numpy increments the counter before use
        assert np.array_equal(oracle.philox(nxt, key), raw)


# --------------------------------------------------------------------------
# LMM12 parameter map: abcd forms and the frozen-weight swaption map
# --------------------------------------------------------------------------
def _lmm_small(n_fwd=6, F=None, seed=1):
    m, truth, noise = I.lmm_market(M=n_fwd, n_cap_K=3, n_exp=2, n_ten=3, n_swp_K=3)
    if F is not None:
        m = dict(m)
        m["fwd_F"] = np.asarray(F, float)
    return m, truth[0]


def test_lmm_caplet_map_is_abcd(oracle):
    m, p = _lmm_small()
    th, ok = oracle.map_params(m, 0, p)
    assert ok
    T = m["fwd_T"]
    for u, (first, ln) in enumerate(zip(m["und_first"], m["und_len"])):
        if ln != 1:
            continue
        t = T[first]
        a, b, c, d, an, bn, cn, dn, rho = p[:9]
        assert th[u, 0] == pytest.approx((a + b * t) * math.exp(-c * t) + d, rel=1e-15)
        assert th[u, 1] == 0.5
        assert th[u, 2] == rho
        assert th[u, 3] == pytest.approx((an + bn * t) * math.exp(-cn * t) + dn, rel=1e-15)


def test_swaption_map_identity_for_identical_forwards(oracle):
    # identical forwards and SABR parameters, perfect correlation (lambda1 =
    # lambda2 = 0): the swap rate equals every forward, so its SABR parameters
    # are the forwards' own
    m, p = _lmm_small(F=np.full(6, 0.03))
    p = p.copy()
    p[1] = 0.0
    p[2] = 1.0
    p[5] = 0.0           # b = b_nu = 0 and c_nu irrelevant
    p[0] = 0.0
    p[4] = 0.0           # a = a_nu = 0 -> alpha_i = d, nu_i = d_nu for every i
    p[9] = 0.0
    p[11] = 0.0          # lambda1 = lambda2 = 0
    th, ok = oracle.map_params(m, 0, p)
    assert ok
    np.testing.assert_allclose(th[:, 0], p[3], rtol=1e-14)
    np.testing.assert_allclose(th[:, 2], p[8], rtol=1e-14)
    np.testing.assert_allclose(th[:, 3], p[7], rtol=1e-14)


def test_swaption_map_vol_of_vol_is_weighted_average(oracle):
    # identical forwards and alphas, lambda1 = 0, theta = 1 (eta2 = 1): the
    # vol-of-vol of the swap rate is sum_k w_k nu_k, with the annuity weights
    m, p = _lmm_small(F=np.full(6, 0.03))
    p = p.copy()
    p[0] = p[1] = 0.0
    p[9] = 0.0
    p[10] = 1.0
    th, ok = oracle.map_params(m, 0, p)
    assert ok
    T = m["fwd_T"]
    nu = (p[4] + p[5] * T) * np.exp(-p[6] * T) + p[7]
    tauP = m["fwd_tau"] * m["fwd_P"]
    for u, (first, ln) in enumerate(zip(m["und_first"], m["und_len"])):
        sl = slice(first, first + ln)
        w = tauP[sl] / tauP[sl].sum()
        assert th[u, 3] == pytest.approx(float(np.dot(w, nu[sl])), rel=1e-13)
        assert th[u, 2] == pytest.approx(p[8], rel=1e-13)
        assert th[u, 0] == pytest.approx(p[3], rel=1e-13)


def test_swaption_map_correlation_bounded(oracle):
    m, _ = _lmm_small()
    lb, ub = I.box(I.MODEL_LMM12)
    pts = I.random_box_points(I.MODEL_LMM12, 300, 11)
    n_ok = 0
    for p in pts:
        th, ok = oracle.map_params(m, 0, p)
        if ok:
            n_ok += 1
            assert np.all(np.abs(th[:, 2]) < 1.0)
            assert np.all(th[:, 0] > 0) and np.all(th[:, 3] >= 0)
    assert n_ok > 20


# --------------------------------------------------------------------------
# Cost
# --------------------------------------------------------------------------
def test_cost_zero_on_noise_free_market(oracle):
    m, truth, noise = I.caplet_market()
    mv, _, _, ok = oracle.model_values(m, 0, truth[0])
    exact = I.complete_market(m, mv, np.zeros_like(noise))
    assert oracle.cost_batch(exact, truth)[0] == 0.0
    for resid_mode in (I.RESID_PRICE,):
        pm = dict(exact)
        pm["residual"] = resid_mode
        assert oracle.cost_batch(pm, truth)[0] <= 1e-28


def test_cost_is_weighted_sum_of_squares(oracle, c1_market):
    mk, truth = c1_market
    pts = I.random_box_points(I.MODEL_GLOBAL4, 50, 3)
    c, r = oracle.cost_batch(mk, pts, resid=True)
    fin = np.isfinite(c)
    assert fin.sum() > 10
    np.testing.assert_allclose(c[fin], np.sum(r[fin] ** 2, axis=1), rtol=1e-13)
    # residual = Hagan vol - market vol, quote by quote
    S0, A, T = oracle.underlyings(mk, 0)
    p = pts[np.argmax(fin)]
    for q in (0, 5, 57, 109):
        u = mk["q_und"][q]
        v = oracle.hagan2002_vol(S0[u], mk["q_K"][q], T[u], *p)
        assert r[np.argmax(fin), q] == pytest.approx(v - mk["q_vol"][q], rel=1e-15, abs=1e-18)


def test_out_of_domain_gives_infinite_cost(oracle, c1_market):
    mk, truth = c1_market
    bad = np.array([[-0.01, 0.5, 0.0, 0.3], [0.03, 0.5, 1.0, 0.3], [0.03, 1.2, 0.0, 0.3],
                    [0.03, 0.5, 0.0, -0.1]])
    assert np.all(np.isinf(oracle.cost_batch(mk, bad)))


@pytest.mark.parametrize("which", ["c1", "c2"])
def test_dual_gradient_matches_central_differences(oracle, c1_market, c2_market, which):
    mk, truth = c1_market if which == "c1" else c2_market
    model = mk["model"]
    lb, ub = I.box(model)
    pts = np.vstack([truth, I.random_box_points(model, 40, 17)])
    c, g = oracle.cost_grad(mk, pts)
    fin = np.isfinite(c)
    checked = 0
    for i in np.nonzero(fin)[0][:12]:
        for k in range(len(lb)):
            h = 1e-6 * max(1.0, abs(pts[i, k]))
            e = np.zeros(len(lb))
            e[k] = h
            cp, cm = oracle.cost_batch(mk, np.vstack([pts[i] + e, pts[i] - e]))
            if not (np.isfinite(cp) and np.isfinite(cm)):
                continue
            fd = (cp - cm) / (2 * h)
            scale = max(abs(fd), 1e-6 * np.max(np.abs(g[i])), 1e-12 * c[i])
            assert abs(g[i, k] - fd) <= 2e-5 * scale + 1e-10 * c[i] / h * 1e-6
            checked += 1
    assert checked > 20


def test_gradient_equals_twice_jtwr(oracle, c2_market):
    mk, truth = c2_market
    c, g, A, b = oracle.cost_grad(mk, truth, normal=True)
    np.testing.assert_allclose(g[0], 2 * b[0], rtol=1e-11, atol=1e-14 * np.abs(g).max())
    assert np.allclose(A[0], A[0].T)
    assert np.all(np.linalg.eigvalsh(A[0]) > -1e-12 * np.abs(A[0]).max())
