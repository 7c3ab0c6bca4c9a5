"""GPU parity of the Nelder-Mead polish (sabr_nm_polish) against the oracle's
Nelder-Mead, for every model: the same iteration count, best vertex and cost
(the simplex arithmetic is evaluated in the same IEEE order on both sides, so
the runs agree while no cost comparison falls within rounding of a tie), the
initial simplex's best vertex at zero iterations, frozen coordinates, and
invalid instances."""
import numpy as np
import pytest

from paper_2408_01470_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_01470_amd import api as A
    return A


def _complete(oracle, m, truth, noise):
    M = oracle.Market(I.as_vol_market(m))
    mv = np.concatenate([oracle.model_values(M, i, truth[i])[0] for i in range(M.n_inst)])
    return I.complete_market(m, mv, noise)


def _compare(api, oracle, mk, x0, pt_inst, lb, ub, max_iter, step=0.05):
    plan = api.Plan(mk)
    x, f, it = plan.nm(torch.tensor(x0, device="cuda"), lb, ub,
                       pt_inst=torch.tensor(pt_inst, device="cuda"), max_iter=max_iter,
                       step=step, tol=1e-13)
    xo, fo, ito = oracle.nm_polish(mk, x0, pt_inst, lb, ub, max_iter=max_iter, step=step,
                                   tol=1e-13)
    x, f, it = x.cpu().numpy(), f.cpu().numpy(), it.cpu().numpy()
    assert np.array_equal(it, ito)
    np.testing.assert_allclose(f, fo, rtol=1e-11)
    np.testing.assert_allclose(x, xo, rtol=1e-11, atol=1e-15)
    return f, it


@pytest.mark.parametrize("formula,residual", [(0, 0), (0, 1), (1, 0)],
                         ids=["hagan-vol", "hagan-price", "eq3-vol"])
def test_nm_parity_global4(api, oracle, formula, residual):
    m, truth, noise = I.batch_markets(n_markets=3, M_range=(6, 12), nK_range=(5, 9))
    m = dict(m, formula=formula, residual=residual)
    mk = _complete(oracle, m, truth, noise)
    lb, ub = I.box(0)
    g = I.rng(I.SEED_BASE + 9910)
    pt = np.repeat(np.arange(3, dtype=np.int32), 2)
    x0 = np.clip(truth[pt] * g.uniform(0.8, 1.2, (6, 4)), lb, ub)
    f, it = _compare(api, oracle, mk, x0, pt, lb, ub, 150)
    assert np.all(it > 10)


def test_nm_parity_lmm12(api, oracle):
    m, truth, noise = I.lmm_market(seed=I.SEED_BASE + 2100, M=8, n_cap_K=5, n_exp=3, n_ten=3,
                                   n_swp_K=3)
    mk = _complete(oracle, m, truth, noise)
    lb, ub = I.box(1)
    g = I.rng(I.SEED_BASE + 9920)
    x0 = np.clip(truth[[0, 0, 0]] * g.uniform(0.9, 1.1, (3, 12)), lb, ub)
    _compare(api, oracle, mk, x0, np.zeros(3, np.int32), lb, ub, 80)


@pytest.mark.parametrize("model", [I.MODEL_PERFWD, I.MODEL_MM], ids=["perfwd", "mm"])
def test_nm_parity_paper_models(api, oracle, model):
    mk = I.paper_caplet_market(model=model)
    lb, ub = I.box(model, 13)
    g = I.rng(I.SEED_BASE + 9930 + model)
    x0 = lb + (ub - lb) * g.uniform(0.3, 0.7, (2, len(lb)))
    f, it = _compare(api, oracle, mk, x0, np.zeros(2, np.int32), lb, ub, 60)
    assert np.all(it == 60)


def test_nm_edges(api, oracle):
    m, truth, noise = I.caplet_market()
    mk = _complete(oracle, m, truth, noise)
    plan = api.Plan(mk)
    lb, ub = I.box(0)
    lb = lb.copy()
    ub = ub.copy()
    lb[1] = ub[1] = 0.5                      # beta frozen
    x0 = np.clip(truth * np.array([[1.1, 1.0, 0.9, 1.2]]), lb, ub)
    x, f, it = plan.nm(torch.tensor(x0, device="cuda"), lb, ub, max_iter=0)
    xo, fo, _ = oracle.nm_polish(mk, x0, None, lb, ub, max_iter=0)
    assert int(it.cpu()[0]) == 0                # the best vertex of the initial simplex
    assert np.array_equal(x.cpu().numpy(), xo)
    assert float(f.cpu()[0]) <= oracle.cost_batch(mk, x0)[0]
    x, f, it = plan.nm(torch.tensor(x0, device="cuda"), lb, ub, max_iter=200)
    assert np.all(x.cpu().numpy()[:, 1] == 0.5)
    assert float(f.cpu()[0]) < oracle.cost_batch(mk, x0)[0]
    bad = torch.tensor([0, 3], dtype=torch.int32, device="cuda")
    x, f, it = plan.nm(torch.tensor(np.vstack([x0, x0]), device="cuda"), lb, ub, pt_inst=bad,
                       max_iter=10)
    f = f.cpu().numpy()
    assert np.isfinite(f[0]) and np.isnan(f[1])
