"""Pins of the oracle's Nelder-Mead polish (the paper's local minimizer after
the annealing, Sec. 3): it reaches the minimum that scipy's Nelder-Mead and
the oracle's Levenberg-Marquardt reach, the grid minimum of a two-parameter
problem, keeps frozen coordinates and the start at zero iterations, and never
ends above its start."""
import numpy as np
import pytest
from scipy.optimize import minimize

from paper_2408_01470_amd import inputs as I


@pytest.fixture(scope="module")
def caplets(oracle):
    m, truth, noise = I.caplet_market()
    mv, _, _, ok = oracle.model_values(I.as_vol_market(m), 0, truth[0])
    assert ok
    return I.complete_market(m, mv, noise), truth[0]


def test_nm_reaches_scipy_and_lm_minimum(oracle, caplets):
    mk, truth = caplets
    lb, ub = I.box(0)
    x0 = np.clip(truth * np.array([1.2, 0.9, 0.8, 1.3]), lb, ub)
    x, f, it = oracle.nm_polish(mk, x0[None, :], None, lb, ub, max_iter=2000, step=0.05,
                                tol=1e-14)
    ref = minimize(lambda z: oracle.cost_batch(mk, np.clip(z, lb, ub)[None, :])[0], x0,
                   method="Nelder-Mead", bounds=list(zip(lb, ub)),
                   options=dict(xatol=1e-12, fatol=1e-16, maxiter=20000, maxfev=40000))
    xl, fl, _ = oracle.lm_polish(mk, x0[None, :], None, lb, ub, max_iter=200)
    assert 0 < it[0] < 2000
    assert f[0] == pytest.approx(ref.fun, rel=1e-8)
    assert f[0] == pytest.approx(fl[0], rel=1e-8)
    np.testing.assert_allclose(x[0], ref.x, rtol=1e-5)
    np.testing.assert_allclose(x[0], xl[0], rtol=1e-5)


def test_nm_two_parameter_grid_minimum(oracle, caplets):
    """beta and nu frozen (lb = ub): NM over (alpha, rho) against a 201 x 201
    brute-force grid of the same cost."""
    mk, truth = caplets
    lb = np.array([0.01, truth[1], -0.9, truth[3]])
    ub = np.array([0.06, truth[1], 0.5, truth[3]])
    a = np.linspace(lb[0], ub[0], 201)
    r = np.linspace(lb[2], ub[2], 201)
    A, R = np.meshgrid(a, r, indexing="ij")
    pts = np.column_stack([A.ravel(), np.full(A.size, truth[1]), R.ravel(),
                           np.full(A.size, truth[3])])
    c = oracle.cost_batch(mk, pts)
    k = int(np.argmin(c))
    x0 = np.array([0.05, truth[1], 0.3, truth[3]])
    x, f, _ = oracle.nm_polish(mk, x0[None, :], None, lb, ub, max_iter=2000, tol=1e-15)
    assert f[0] <= c[k]
    assert abs(x[0, 0] - pts[k, 0]) <= a[1] - a[0]
    assert abs(x[0, 2] - pts[k, 2]) <= r[1] - r[0]
    assert x[0, 1] == truth[1] and x[0, 3] == truth[3]


def test_nm_zero_iterations_and_monotone(oracle, caplets):
    mk, truth = caplets
    lb, ub = I.box(0)
    x0 = np.clip(truth * np.array([1.3, 1.1, 0.7, 0.8]), lb, ub)
    f0 = oracle.cost_batch(mk, x0[None, :])[0]
    x, f, it = oracle.nm_polish(mk, x0[None, :], None, lb, ub, max_iter=0)
    assert it[0] == 0            # the best vertex of the initial simplex
    assert f[0] <= f0 and f[0] == oracle.cost_batch(mk, x)[0]
    assert np.count_nonzero(x[0] != x0) <= 1
    prev = f[0]
    for k in (5, 20, 80, 320):
        _, fk, itk = oracle.nm_polish(mk, x0[None, :], None, lb, ub, max_iter=k)
        assert fk[0] <= prev and itk[0] <= k
        prev = fk[0]


@pytest.mark.parametrize("model", [I.MODEL_PERFWD, I.MODEL_MM], ids=["perfwd", "mm"])
def test_nm_improves_paper_models(oracle, model):
    mk = I.paper_caplet_market(model=model)
    lb, ub = I.box(model, 13)
    x0 = (lb + ub) / 2
    f0 = oracle.cost_batch(mk, x0[None, :])[0]
    x, f, it = oracle.nm_polish(mk, x0[None, :], None, lb, ub, max_iter=300)
    assert f[0] < f0 and np.all(x[0] >= lb) and np.all(x[0] <= ub)
    assert f[0] == pytest.approx(oracle.cost_batch(mk, x)[0], rel=0, abs=0)
