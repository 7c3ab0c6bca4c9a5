"""The Rebonato model (REB) of Sec. 2.2 with the SABR parameters of eq.
(haganForRebonato), in the CPU oracle: its two integrals against mpmath
quadrature of their definitions, the closed forms of constant g and h, the
paper's calibrated Rebonato table (Sec. 4.3.1: with the printed ATM levels,
phi_ii and the printed g and h, the map's nu reproduces the printed off-ATM
model vols; kappa_i, printed to one or two digits, does not enter), its
domain, and host-side validation of REB plans."""
import math
import os

import mpmath as mp
import numpy as np
import pytest

from conftest import ROOT, load_golden
from paper_2408_01470_amd import inputs as I
from paper_2408_01470_amd import workloads as W

GH = [3.7789, 44.7668, 0.3076, 25.3412, 0.0010, 19.5812, 6.2339, 0.5533]


def _market():
    return I.paper_caplet_market(model=I.MODEL_REB)


def _point(kap, phi, gh):
    return np.concatenate([np.column_stack([kap, phi]).ravel(), gh])


def _mp_alpha_nu(T, kap, gh):
    """eq. (haganForRebonato) by mpmath quadrature of its definitions."""
    mp.mp.dps = 30
    a, b, c, d, ah, bh, ch, dh = [mp.mpf(v) for v in gh]
    g = lambda t: (a + b * (T - t)) * mp.e ** (-c * (T - t)) + d
    h = lambda s: (ah + bh * (T - s)) * mp.e ** (-ch * (T - s)) + dh
    G = mp.quad(lambda t: g(t) ** 2, [0, T])
    H = lambda t: mp.quad(lambda s: h(s) ** 2, [0, t])
    J = mp.quad(lambda t: g(t) ** 2 * H(t), [0, T])
    alpha = kap * mp.sqrt(G / T)
    nu = mp.sqrt(2 * J) / (alpha * T) * kap   # kappa / (alpha T) sqrt(2 J)
    return float(alpha), float(nu)


@pytest.mark.parametrize("gh", [GH, [0.1, 0.5, 3.0, 0.1, 0.5, 2.0, 10.0, 0.2],
                                [0.05, 0.1, 0.01, 0.05, 0.3, 0.5, 0.01, 0.1],
                                [1.0, 10.0, 1.0, 5.0, 0.2, 5.0, 2.0, 0.5]],
                         ids=["printed", "steep-h", "flat", "mid"])
def test_reb_map_against_quadrature(oracle, gh):
    mk = _market()
    kap = np.full(13, 0.002)
    phi = np.linspace(-0.5, 0.3, 13)
    th, ok = oracle.map_params(mk, 0, _point(kap, phi, gh))
    assert ok
    T = mk["fwd_T"]
    for i in (0, 4, 12):
        alpha, nu = _mp_alpha_nu(T[i], kap[i], gh)
        assert th[i, 0] == pytest.approx(alpha, rel=1e-13)
        assert th[i, 3] == pytest.approx(nu, rel=1e-12)
        assert th[i, 2] == phi[i] and th[i, 1] == 0.5


def test_reb_constant_g_and_h(oracle):
    """b = c = 0 and b_h = c_h = 0: g = a + d, h = a_h + d_h, so alpha =
    kappa (a + d) and nu = a_h + d_h at every expiry."""
    mk = _market()
    kap = np.linspace(0.001, 0.004, 13)
    gh = [0.3, 0.0, 0.0, 0.2, 0.25, 0.0, 0.0, 0.15]
    th, ok = oracle.map_params(mk, 0, _point(kap, np.zeros(13), gh))
    assert ok
    np.testing.assert_allclose(th[:, 0], kap * 0.5, rtol=1e-14)
    np.testing.assert_allclose(th[:, 3], np.full(13, 0.4), rtol=1e-13)


def test_reb_reproduces_paper_smile_shapes(oracle):
    """Sec. 4.3.1: eq. (sigmaHagan) with the printed ATM model vols, the
    printed phi_ii and nu from the map at the printed g and h gives the
    printed off-ATM model vols (48 cells) to 0.05 vol points on average and
    0.35 at most (the worst: the shortest expiries, whose nu is largest);
    dropping the factor 2 under the square root of nu breaks it."""
    prm = np.array([[float(v) for v in r[1:]] for r in load_golden(
        "paper_rebonato_caplet_params.txt")])
    vols = [(int(r[0]), int(r[1]), float(r[2]), float(r[3])) for r in load_golden(
        "paper_rebonato_caplet_vols.txt")]
    phi = np.clip(prm[:, 0], -0.9999, 0.9999)     # phi_13 = -1 printed, on the bound
    th, ok = oracle.map_params(_market(), 0, _point(prm[:, 1], phi, GH))
    assert ok
    atm = {i: sm / 100.0 for i, m, _, sm in vols if m == 0}

    def errs(nu):
        return np.array([oracle.paper_eq3_vol(1.0, math.exp(m / 100.0), atm[i], 0.5, phi[i - 1],
                                              nu[i - 1]) * 100.0 - sm
                         for i, m, _, sm in vols if m != 0])
    e = errs(th[:, 3])
    assert len(e) == 48
    assert np.mean(np.abs(e)) <= 0.05 and np.max(np.abs(e)) <= 0.35
    assert np.max(np.abs(errs(th[:, 3] / math.sqrt(2.0)))) > 2.0


def test_reb_domain(oracle):
    mk = _market()
    x = _point(np.full(13, 0.002), np.full(13, -0.3), GH)
    assert np.isfinite(oracle.cost_batch(mk, x[None, :])[0])
    for k, v in ((0, 0.0), (1, 1.0), (25, -1.0), (28, -0.1), (32, -0.1)):
        y = x.copy()
        y[k] = v
        assert oracle.cost_batch(mk, y[None, :])[0] == np.inf, (k, v)
    y = x.copy()
    y[26:30] = 0.0        # g = 0: G = 0
    assert oracle.cost_batch(mk, y[None, :])[0] == np.inf
    with pytest.raises(ValueError):
        oracle.cost_grad(mk, x[None, :])


def test_paper_reb_schedule():
    w = W.paper_reb()
    assert w.chains * (1 + w.n_steps * w.n_levels) == w.extra["paper_evals"] == 2254471168
    assert I.num_params(I.MODEL_REB, 13) == 34


LIB = os.path.join(ROOT, "paper_2408_01470_amd", "libsabr_hip.so")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(LIB):
        pytest.skip("HIP library not built")
    from paper_2408_01470_amd import _lib
    return _lib.lib()


def test_plan_create_reb(L):
    from test_oracle_perfwd import _create, _perfwd_batch
    assert _create(L, _market()) == (0, 34)
    assert _create(L, dict(_perfwd_batch([27, 27]), model=I.MODEL_REB)) == (0, 62)
    rc, _ = _create(L, dict(_perfwd_batch([28]), model=I.MODEL_REB))
    assert rc == -1 and b"REB needs 1..27" in L.sabr_last_error()
