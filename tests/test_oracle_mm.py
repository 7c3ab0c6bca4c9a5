"""The Mercurio-Morini model (MM) of Sec. 2.2 with the SABR parameters of eq.
(haganForMercurio), in the CPU oracle: pinned against the paper's caplet
calibration of Sec. 4.2.1 (printed parameters, model vol table and MRE), the
special cases that reduce it to the per-forward and common-parameter Hagan
models, and its domain; plus host-side validation of MM plans."""
import ctypes
import os

import numpy as np
import pytest

from conftest import ROOT, load_golden
from paper_2408_01470_amd import inputs as I
from paper_2408_01470_amd import workloads as W

MNY = (-80, -60, -40, -20, 0, 20, 40, 60, 80)


def _printed_mm():
    """Printed (phi_i, alpha_i) and sigma as an MM point (alpha_1, phi_1, ...,
    sigma), and the printed model vol table."""
    rows = load_golden("paper_mm_caplet_params.txt")
    prm = np.array([[float(v) for v in r[1:]] for r in rows])
    x = np.concatenate([np.column_stack([prm[:, 1], prm[:, 0]]).ravel(), [0.5986]])
    vols = [(int(r[0]), int(r[1]), float(r[2]), float(r[3])) for r in load_golden(
        "paper_mm_caplet_vols.txt")]
    return x, vols


def _implied_forwards():
    """F_i = (alpha_i / A_i)^2 from the printed Hagan-model calibration of the
    same data (Sec. 4.1.1): the forwards the paper's tables imply."""
    prm = np.array([[float(v) for v in r[1:]] for r in load_golden(
        "paper_hagan_caplet_params.txt")])
    vols = [(int(r[0]), int(r[1]), float(r[3])) for r in load_golden(
        "paper_hagan_caplet_vols.txt")]
    atm = np.array([v[2] for v in sorted(t for t in vols if t[1] == 0)]) / 100.0
    return (prm[:, 2] / atm) ** 2


def _model_table(oracle, mk, x):
    mv, tgt, _, ok = oracle.model_values(oracle.Market(mk), 0, x)
    assert ok
    return mv, tgt


def test_mm_reproduces_paper_fit_table(oracle):
    """The 60 printed MM model vols (12 forwards x 5 strikes) at the printed
    parameters, to 0.25% relative (alpha_i printed to 3 digits; the forwards
    implied from the Hagan tables carry their own rounding)."""
    x, vols = _printed_mm()
    mk = I.paper_caplet_market(model=I.MODEL_MM, fwd_F=_implied_forwards())
    mv, _ = _model_table(oracle, mk, x)
    mv = mv.reshape(13, 9) * 100.0
    col = {m: j for j, m in enumerate(MNY)}
    rel = [abs(mv[i - 1, col[m]] / sm - 1.0) for i, m, _, sm in vols]
    assert len(rel) == 60
    assert max(rel) <= 2.5e-3


def test_mm_paper_mre(oracle):
    """MRE over the 117 quotes: printed 3.11e-2 (Sec. 4.2.1)."""
    x, _ = _printed_mm()
    mk = I.paper_caplet_market(model=I.MODEL_MM, fwd_F=_implied_forwards())
    mv, tgt = _model_table(oracle, mk, x)
    assert abs(np.mean(np.abs(mv - tgt) / tgt) - 3.11e-2) <= 1.0e-4


def test_mm_drift_reading_discriminates(oracle):
    """The printed ATM levels separate the drift conventions: with the drift
    sum starting at the first unfixed forward itself (forward j entering
    until its own fixing T_j) the ATM levels of F_11, F_12 miss by > 0.5%,
    while the reading used (from the forward after it) stays within 0.25%.
    The literal variant is evaluated through the PERFWD oracle with its
    alpha^SABR computed here."""
    x, vols = _printed_mm()
    F = _implied_forwards()
    mk = I.paper_caplet_market(model=I.MODEL_PERFWD, fwd_F=F)
    al, ph, sig = x[0:26:2], x[1:26:2], x[26]
    c = mk["fwd_tau"] * ph * al * F ** 0.5 / (1.0 + mk["fwd_tau"] * F)
    a_lit = al * np.exp(-sig * np.cumsum(c * mk["fwd_T"]))
    y = np.column_stack([a_lit, ph, np.full(13, sig)]).ravel()
    mv, _ = _model_table(oracle, mk, y)
    atm = {i: sm for i, m, _, sm in vols if m == 0}
    dev = [abs(mv.reshape(13, 9)[i - 1, 4] * 100.0 / atm[i] - 1.0) for i in (11, 12)]
    assert min(dev) > 5e-3


@pytest.mark.parametrize("formula,residual", [(1, 0), (0, 0), (0, 1)],
                         ids=["eq3-vol", "hagan-vol", "hagan-price"])
def test_mm_special_cases(oracle, formula, residual):
    """sigma = 0 or all phi = 0 remove the drift: MM equals PERFWD at
    (alpha_i, phi_i, sigma); one forward: MM equals GLOBAL4 at
    (alpha, beta, phi, sigma) (its drift weight T_0 is 0)."""
    mk_mm = I.paper_caplet_market(model=I.MODEL_MM, formula=formula, residual=residual)
    mk_pf = I.paper_caplet_market(model=I.MODEL_PERFWD, formula=formula, residual=residual)
    g = I.rng(I.SEED_BASE + 9600)
    lb, ub = I.box(I.MODEL_MM, 13)
    for _ in range(6):
        x = g.uniform(lb, ub)
        x[-1] = 0.0 if _ % 2 == 0 else x[-1]
        if _ % 2 == 1:
            x[1:26:2] = 0.0
        y = np.column_stack([x[0:26:2], x[1:26:2], np.full(13, x[26])]).ravel()
        c_mm = oracle.cost_batch(mk_mm, x[None, :])[0]
        c_pf = oracle.cost_batch(mk_pf, y[None, :])[0]
        assert c_mm == c_pf or abs(c_mm - c_pf) <= 1e-13 * abs(c_pf)
    g4 = I.perfwd_as_global4(mk_pf)
    for k in (0, 5, 12):   # forward k alone, as a one-forward MM market
        sel = slice(int(g4["q_off"][k]), int(g4["q_off"][k + 1]))
        m1 = dict(g4, fwd_off=np.array([0, 1], np.int32), und_off=np.array([0, 1], np.int32),
                  q_off=np.array([0, 9], np.int32))
        for key in ("fwd_T", "fwd_tau", "fwd_F", "fwd_P", "und_first", "und_len"):
            m1[key] = np.asarray(g4[key])[k:k + 1]
        for key in ("q_und", "q_kind", "q_K", "q_vol", "q_w"):
            m1[key] = np.asarray(g4[key])[sel]
        c_mm = oracle.cost_batch(dict(m1, model=I.MODEL_MM), np.array([[0.05, -0.3, 0.4]]))[0]
        c_g4 = oracle.cost_batch(m1, np.array([[0.05, 0.5, -0.3, 0.4]]))[0]
        assert c_mm == c_g4 or abs(c_mm - c_g4) <= 1e-13 * abs(c_g4)


def test_mm_drift_grows_with_negative_phi(oracle):
    """All phi_j < 0 make every drift term positive: alpha_i^SABR / alpha_i =
    exp(-sigma D_i) > 1 and increasing in i (model ATM vol above the
    drift-free one by a growing factor)."""
    mk_mm = I.paper_caplet_market(model=I.MODEL_MM)
    mk_pf = I.paper_caplet_market(model=I.MODEL_PERFWD)
    x = np.concatenate([np.tile([0.07, -0.6], 13), [0.6]])
    y = np.column_stack([np.full(13, 0.07), np.full(13, -0.6), np.full(13, 0.6)]).ravel()
    a, _ = _model_table(oracle, mk_mm, x)
    b, _ = _model_table(oracle, mk_pf, y)
    ratio = a.reshape(13, 9)[:, 4] / b.reshape(13, 9)[:, 4]
    assert ratio[0] == pytest.approx(1.0, abs=1e-15)
    assert np.all(np.diff(ratio) > 0.0) and ratio[-1] > 1.02


def test_mm_domain(oracle):
    mk = I.paper_caplet_market(model=I.MODEL_MM)
    x, _ = _printed_mm()
    assert np.isfinite(oracle.cost_batch(mk, x[None, :])[0])
    for k, v in ((26, -1e-3), (0, 0.0), (1, 1.0), (25, -1.0), (24, -0.01)):
        y = x.copy()
        y[k] = v
        assert oracle.cost_batch(mk, y[None, :])[0] == np.inf, (k, v)
    with pytest.raises(ValueError):
        oracle.cost_grad(mk, x[None, :])


def test_paper_mm_schedule():
    w = W.paper_mm()
    assert w.n_levels == 688 and w.chains * (1 + w.n_steps * w.n_levels) == 112738304
    assert I.num_params(I.MODEL_MM, 13) == 27


LIB = os.path.join(ROOT, "paper_2408_01470_amd", "libsabr_hip.so")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(LIB):
        pytest.skip("HIP library not built")
    from paper_2408_01470_amd import _lib
    return _lib.lib()


def test_plan_create_mm(L):
    from test_oracle_perfwd import _create, _perfwd_batch
    assert _create(L, I.paper_caplet_market(model=I.MODEL_MM)) == (0, 27)
    m = dict(_perfwd_batch([31, 31]), model=I.MODEL_MM)
    assert _create(L, m) == (0, 63)
    rc, _ = _create(L, dict(_perfwd_batch([32]), model=I.MODEL_MM))
    assert rc == -1 and b"MM needs 1..31" in L.sabr_last_error()
    rc, _ = _create(L, dict(_perfwd_batch([8, 9]), model=I.MODEL_MM))
    assert rc == -1 and b"MM instances" in L.sabr_last_error()
