"""The per-forward Hagan model (PERFWD) of Sec. 3, calibrated to caplets in
Sec. 4.1.1, in the CPU oracle: pinned against the paper's worked example
(printed calibrated parameters, model vol table and MRE), against the
separation of its cost into one GLOBAL4 problem per forward, and against its
domain; plus the host-side validation of PERFWD plans and the E2 replay's
schedule arithmetic."""
import ctypes
import os

import numpy as np
import pytest

from conftest import ROOT, load_golden
from paper_2408_01470_amd import inputs as I
from paper_2408_01470_amd import workloads as W


def _printed():
    """Printed (phi_ii, sigma_i, alpha_i) per forward as a PERFWD point
    (alpha, rho, nu) and the printed model ATM vols A_i."""
    prm = np.array([[float(v) for v in r[1:]] for r in load_golden(
        "paper_hagan_caplet_params.txt")])
    x = np.column_stack([prm[:, 2], prm[:, 0], prm[:, 1]]).ravel()
    vols = [(int(r[0]), int(r[1]), float(r[2]), float(r[3])) for r in load_golden(
        "paper_hagan_caplet_vols.txt")]
    atm = np.array([sm for i, mny, _, sm in sorted(v for v in vols if v[1] == 0)]) / 100.0
    return x, atm, vols


def _implied_market():
    """The paper market with F_i = (alpha_i / A_i)^2: the forwards its
    printed alpha_i and ATM model vols imply at beta = 0.5."""
    x, atm, _ = _printed()
    return I.paper_caplet_market(fwd_F=(x[0::3] / atm) ** 2)


def test_perfwd_reproduces_paper_fit_table(oracle):
    """At the printed parameters the PERFWD cost path gives the printed model
    vols (Sec. 4.1.1 table, 13 forwards x 5 strikes, 2 decimals in %)."""
    x, _, vols = _printed()
    mk = _implied_market()
    mv, tgt, w, ok = oracle.model_values(oracle.Market(mk), 0, x)
    assert ok
    mv = mv.reshape(13, 9) * 100.0
    col = {m: j for j, m in enumerate((-80, -60, -40, -20, 0, 20, 40, 60, 80))}
    errs = [abs(mv[i - 1, col[mny]] - smod) for i, mny, _, smod in vols]
    assert len(errs) == 65
    assert max(errs) <= 0.011


def test_perfwd_paper_mre(oracle):
    """MRE of the printed fit over all 117 quotes: 1.80e-2 (Sec. 4.1.1)."""
    x, _, _ = _printed()
    mk = _implied_market()
    mv, tgt, _, ok = oracle.model_values(oracle.Market(mk), 0, x)
    assert ok and len(mv) == 117
    assert abs(np.mean(np.abs(mv - tgt) / tgt) - 1.80e-2) <= 0.5e-4


def test_perfwd_triple_order_matters(oracle):
    """Swapping rho and nu in every triple, or shifting triples by one forward,
    moves the fit far from the printed table: the pin above discriminates."""
    x, _, _ = _printed()
    mk = _implied_market()
    M = oracle.Market(mk)
    base = np.mean(np.abs(np.subtract(*oracle.model_values(M, 0, x)[:2])))
    t = x.reshape(13, 3)
    for y in (t[:, [0, 2, 1]].ravel(), np.roll(t, 1, axis=0).ravel()):
        y = np.clip(y, *I.box(I.MODEL_PERFWD, 13))
        mv, tgt, _, ok = oracle.model_values(M, 0, y)
        assert not ok or np.mean(np.abs(mv - tgt)) > 3 * base


@pytest.mark.parametrize("formula,residual", [(1, 0), (0, 0), (0, 1)],
                         ids=["eq3-vol", "hagan-vol", "hagan-price"])
def test_perfwd_cost_separates_per_forward(oracle, formula, residual):
    """f(x) = sum_i f_i(alpha_i, beta, rho_i, nu_i): the PERFWD cost is the sum
    of the GLOBAL4 costs of each forward's caplets (Sec. 3: f_c sums over
    forwards, each forward's smile depends on its own triple only)."""
    mk = I.paper_caplet_market(formula=formula, residual=residual)
    g4 = I.perfwd_as_global4(mk)
    lb, ub = I.box(I.MODEL_PERFWD, 13)
    pts = I.rng(I.SEED_BASE + 9100).uniform(lb, ub, (16, 39))
    c = oracle.cost_batch(mk, pts)
    n_fin = 0
    for k in range(len(pts)):
        y = I.perfwd_points_as_global4(pts[k], 0.5)
        c4 = oracle.cost_batch(g4, y, np.arange(13, dtype=np.int32))
        if np.isfinite(c[k]):
            n_fin += 1
            np.testing.assert_allclose(c[k], c4.sum(), rtol=1e-13)
        else:                       # a forward's model vol left the domain
            assert c[k] == np.inf and not np.all(np.isfinite(c4))
    assert n_fin >= 4
    np.testing.assert_array_equal(I.global4_points_as_perfwd(
        I.perfwd_points_as_global4(pts[0], 0.5)), pts[0])


def test_perfwd_domain_covers_unquoted_forwards(oracle):
    """A triple outside the domain gives +inf, also on a forward with no
    quotes (its parameters do not enter any model value)."""
    mk = I.paper_caplet_market()
    keep = mk["q_und"] != 4                     # forward 5 unquoted
    m2 = dict(mk)
    for k in ("q_und", "q_kind", "q_K", "q_vol", "q_w"):
        m2[k] = np.asarray(mk[k])[keep]
    m2["q_off"] = np.array([0, int(keep.sum())], np.int32)
    x, _, _ = _printed()
    assert np.isfinite(oracle.cost_batch(m2, x[None, :])[0])
    for k, v in ((12, 0.0), (13, 1.0), (14, -1e-3), (0, -0.01), (37, -1.0)):
        y = x.copy()
        y[k] = v
        assert oracle.cost_batch(m2, y[None, :])[0] == np.inf, (k, v)


def test_perfwd_has_no_gradient_entry(oracle):
    mk = I.paper_caplet_market()
    x, _, _ = _printed()
    with pytest.raises(ValueError):
        oracle.cost_grad(mk, x[None, :])


def test_curve_forwards_near_implied_forwards():
    """The discount-curve forwards (log-linear interpolation, ACT/360 accrual)
    agree with those the printed parameters imply: F_1 = 1.196% to 0.1%,
    every forward to 2.5% (eq. (sigmaHagan) depends on alpha and F only
    through alpha / F^(1-beta), so this only rescales the fitted alpha_i)."""
    x, atm, _ = _printed()
    Fi = (x[0::3] / atm) ** 2
    F = I.paper_caplet_market()["fwd_F"]
    assert abs(F[0] / Fi[0] - 1.0) < 1e-3
    assert np.max(np.abs(F / Fi - 1.0)) < 0.025


def test_paper_e2_schedule_count():
    """T0 = 10, Tmin = 0.01, rho = 0.99, N = 10, 16384 chains: 112,738,304
    cost evaluations (Sec. 4.1.1)."""
    w = W.paper_e2()
    assert w.n_levels == 688
    assert w.chains * (1 + w.n_steps * w.n_levels) == w.extra["paper_evals"] == 112738304
    assert I.n_quotes(w.market).tolist() == [117]


# --------------------------------------------------------------------------
# Host-side validation of PERFWD plans (no GPU work: plan creation only)
# --------------------------------------------------------------------------
LIB = os.path.join(ROOT, "paper_2408_01470_amd", "libsabr_hip.so")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(LIB):
        pytest.skip("HIP library not built")
    from paper_2408_01470_amd import _lib
    return _lib.lib()


def _create(L, m):
    from test_abi import _problem
    prob, keep = _problem(m)
    h = ctypes.c_void_p()
    rc = L.sabr_plan_create(ctypes.byref(prob), ctypes.byref(h))
    if rc == 0:
        n = L.sabr_plan_num_params(h)
        L.sabr_plan_destroy(h)
        return rc, n
    return rc, None


def _perfwd_batch(Ms, nK=5):
    g = I.rng(I.SEED_BASE + 9200)
    parts = I._empty()
    for M in Ms:
        T = 0.5 * np.arange(1, M + 1)
        F = 0.03 + 0.001 * np.arange(M)
        P = np.exp(-0.03 * (T + 0.5))
        K = (F[:, None] * np.exp(np.linspace(-0.5, 0.5, nK))[None, :]).ravel()
        I._append(parts, T, np.full(M, 0.5), F, P, np.arange(M), np.ones(M, np.int32),
                  np.repeat(np.arange(M), nK), np.zeros(M * nK, np.int32), K)
    m = I._finish(parts, I.MODEL_PERFWD, I.FORMULA_HAGAN2002, I.RESID_VOL, 0.5)
    m["q_vol"] = g.uniform(0.2, 0.4, len(m["q_K"]))
    return m


def test_plan_create_perfwd(L):
    assert _create(L, I.paper_caplet_market()) == (0, 39)
    assert _create(L, _perfwd_batch([21, 21])) == (0, 63)
    assert L.sabr_num_params(2) == -1


@pytest.mark.parametrize("Ms", [[10, 11], [22]], ids=["unequal", "too-many-forwards"])
def test_plan_create_perfwd_rejects(L, Ms):
    rc, _ = _create(L, _perfwd_batch(Ms))
    assert rc == -1
    assert b"PERFWD" in L.sabr_last_error()


def test_plan_create_perfwd_rejects_swaps(L):
    m = _perfwd_batch([6])
    m["und_len"] = m["und_len"].copy()
    m["und_len"][0] = 2
    rc, _ = _create(L, m)
    assert rc == -1 and b"only LMM12 markets hold swaptions" in L.sabr_last_error()
