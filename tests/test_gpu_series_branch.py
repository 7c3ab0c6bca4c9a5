"""Parity in the removable singularity of Hagan's formula (Sec. 2.1, eq.
(sigmaHagan) cites Hagan 2002): chi = z/x(z) at z = (nu/alpha) q ln(f/K)
-> 0.  The cost kernels keep the log1p quotient down to |z| = 2^-60 (only
the exact at-the-money z = 0 goes below it, where |z| is floored and chi
rounds to its limit 1); the adjoint takes the series of chi below
|z| = 2^-18 and of its derivatives below 2^-10.  These tests place quotes
so that |z| spans both sides of each switch (both signs of z), down to the
smallest nonzero |z| a strike can give and z = 0, and compare with the
oracle: model values and costs to 1e-12 relative, gradients, J^T W J and
J^T W r to 1e-10."""
import numpy as np
import pytest

from paper_2408_01470_amd import inputs as I

torch = pytest.importorskip("torch")

F0, T_EXP = 0.031, 2.5
POINT = np.array([0.035, 0.5, -0.35, 0.45])        # GLOBAL4 (alpha, beta, rho, nu)


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_01470_amd import api as A
    return A


def _log_moneyness(z, p, f=F0):
    """ln(f/K) whose z = (nu/alpha) (f K)^((1-b)/2) ln(f/K) equals the target."""
    a, b, _, n = p
    L = z * a / (n * f ** (1.0 - b))
    for _ in range(50):   # q depends on K = f e^-L weakly
        q = (f * f * np.exp(-L)) ** (0.5 * (1.0 - b))
        L = z * a / (n * q)
    return L


def _near_atm_market(zs, residual, p=POINT):
    L = np.array([_log_moneyness(z, p) for z in zs])
    K = F0 * np.exp(-L)
    T, tau = np.array([T_EXP]), np.array([0.5])
    P = np.array([0.92])
    parts = I._empty()
    I._append(parts, T, tau, np.array([F0]), P, [0], [1], np.zeros(len(K), np.int32),
              np.zeros(len(K), np.int32), K)
    m = I._finish(parts, I.MODEL_GLOBAL4, I.FORMULA_HAGAN2002, residual, 0.5)
    return m, L


def _targets(switch):
    mags = switch * np.array([2.0 ** -2, 2.0 ** -1, 1 - 1e-3, 1 - 1e-9, 1.0, 1 + 1e-9, 1 + 1e-3,
                              2.0, 4.0])
    return np.concatenate([mags, -mags])


def _completed(oracle, zs, residual):
    m, L = _near_atm_market(zs, residual)
    vm = I.as_vol_market(m)
    mv, _, _, ok = oracle.model_values(vm, 0, POINT)
    assert ok
    g = np.random.default_rng(7)
    return I.complete_market(m, mv, g.normal(0.0, 0.002, len(mv))), L


def _points(n, seed):
    g = np.random.default_rng(seed)
    lb, ub = I.box(0)
    pts = np.clip(POINT[None, :] * g.uniform(0.999, 1.001, (n, 4)), lb, ub)
    return np.vstack([POINT[None, :], pts])


@pytest.mark.gpu
@pytest.mark.parametrize("residual", [I.RESID_VOL, I.RESID_PRICE])
def test_cost_series_switch_parity(api, oracle, residual):
    zs = np.concatenate([_targets(2.0 ** -18), [1e-15, -1e-15, 0.0]])
    mk, L = _completed(oracle, zs, residual)
    plan = api.Plan(mk)
    # at the point itself every |z| is on target; the nearby points move z
    # by up to 0.2%, so the quotes next to the switch fall on either side
    pts = _points(16, 3)
    c, mvals = plan.cost(torch.tensor(pts, device="cuda"), model=True)
    c = c.cpu().numpy()
    mvals = mvals.cpu().numpy()
    c_o = oracle.cost_batch(mk, pts)
    assert np.all(np.isfinite(c_o)) and np.all(np.isfinite(c))
    np.testing.assert_allclose(c, c_o, rtol=1e-12)
    for i, p in enumerate(pts):
        mo, _, _, ok = oracle.model_values(mk, 0, p)
        assert ok
        err = np.abs(mvals[i, :len(mo)] - mo) / np.abs(mo)
        j = int(np.argmax(err))
        assert err[j] <= 1e-12, (f"point {i}, quote {j} (target z {zs[j]:.6g}, ln(f/K) "
                                 f"{L[j]:.6g}): gpu {mvals[i, j]!r} oracle {mo[j]!r}")


@pytest.mark.gpu
@pytest.mark.parametrize("residual", [I.RESID_VOL, I.RESID_PRICE])
def test_adjoint_series_switch_parity(api, oracle, residual):
    zs = np.concatenate([_targets(2.0 ** -10), _targets(2.0 ** -18)])
    mk, L = _completed(oracle, zs, residual)
    plan = api.Plan(mk)
    pts = _points(16, 4)
    c_o, g_o, A_o, b_o = oracle.cost_grad(mk, pts, normal=True)
    out = plan.vjp(torch.tensor(pts, device="cuda"), normal=True)
    np.testing.assert_allclose(out["cost"].cpu().numpy(), c_o, rtol=1e-12)
    g_g = out["grad"].cpu().numpy()
    scale = np.maximum(np.abs(g_o), 1e-6 * np.abs(g_o).max(axis=1, keepdims=True))
    err = np.abs(g_g - g_o) / scale
    i, k = np.unravel_index(np.argmax(err), err.shape)
    assert err.max() <= 1e-10, f"gradient: point {i} param {k}: {g_g[i, k]!r} vs {g_o[i, k]!r}"
    A_g = out["jtwj"].cpu().numpy()
    sA = np.abs(A_o).max(axis=(1, 2), keepdims=True)
    assert np.max(np.abs(A_g - A_o) / sA) <= 1e-10
    b_g = out["jtwr"].cpu().numpy()
    sb = np.maximum(np.abs(b_o), 1e-6 * np.abs(b_o).max(axis=1, keepdims=True))
    assert np.max(np.abs(b_g - b_o) / sb) <= 1e-10


def test_targets_straddle_the_switches():
    """The fixture's strikes put |z| on both sides of each switch (host)."""
    for switch in (2.0 ** -18, 2.0 ** -10):
        zs = _targets(switch)
        m, L = _near_atm_market(zs, I.RESID_VOL)
        a, b, _, n = POINT
        q = (F0 * m["q_K"]) ** (0.5 * (1.0 - b))
        z = n / a * q * L
        np.testing.assert_allclose(z, zs, rtol=1e-12)
        assert np.any(np.abs(z) < switch) and np.any(np.abs(z) > switch)
        assert np.any(z > 0) and np.any(z < 0)
