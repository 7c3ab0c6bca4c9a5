"""GPU parity of the per-forward Hagan model (PERFWD, P = 3 per forward) against
the oracle: costs on the paper's EURIBOR caplet data and on synthetic
multi-market batches (up to P = 63, the largest a wave holds), annealing
accept decisions bit for bit (P + 1 uniforms from (P + 4) / 4 Philox blocks,
step counts that leave a ragged last Philox pass), sampled chains of level 0
at the paper's full E2 size (16384 chains), and the LM polish of each forward
as a GLOBAL4 instance."""
import numpy as np
import pytest

from paper_2408_01470_amd import inputs as I
from paper_2408_01470_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RTOL = 1e-12


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_01470_amd import api as A
    return A


def _printed_point():
    from conftest import load_golden
    prm = np.array([[float(v) for v in r[1:]] for r in load_golden(
        "paper_hagan_caplet_params.txt")])
    return np.column_stack([prm[:, 2], prm[:, 0], prm[:, 1]]).ravel()


def _oracle_vols(oracle, vm, truth):
    M = oracle.Market(vm)
    out = []
    for i in range(M.n_inst):
        mv, _, _, ok = oracle.model_values(M, i, truth[i])
        assert ok
        out.append(mv)
    return np.concatenate(out)


def _synthetic(oracle, n_markets, M, nK, formula=0, residual=0):
    m, truth, noise = I.perfwd_markets(n_markets=n_markets, M=M, nK=nK, formula=formula,
                                       residual=residual)
    return I.complete_market(m, _oracle_vols(oracle, I.as_vol_market(m), truth), noise), truth


def _cost_compare(api, oracle, mk, pts, pt_inst=None):
    plan = api.Plan(mk)
    c_g = plan.cost(torch.tensor(pts, device="cuda"),
                    None if pt_inst is None else torch.tensor(pt_inst, device="cuda"))
    c_g = c_g.cpu().numpy()
    c_o = oracle.cost_batch(mk, pts, pt_inst)
    fin = np.isfinite(c_o)
    assert np.array_equal(fin, np.isfinite(c_g))
    np.testing.assert_allclose(c_g[fin], c_o[fin], rtol=RTOL)
    return fin


@pytest.mark.parametrize("formula,residual", [(1, 0), (0, 0), (0, 1), (1, 1)],
                         ids=["eq3-vol", "hagan-vol", "hagan-price", "eq3-price"])
def test_paper_market_cost_parity(api, oracle, formula, residual):
    mk = I.paper_caplet_market(formula=formula, residual=residual)
    lb, ub = I.box(I.MODEL_PERFWD, 13)
    x = _printed_point()
    g = I.rng(I.SEED_BASE + 9300)
    pts = np.vstack([x, np.clip(x * g.uniform(0.8, 1.2, (40, 39)), lb, ub),
                     g.uniform(lb, ub, (24, 39))])
    fin = _cost_compare(api, oracle, mk, pts)
    assert fin[:41].all()


@pytest.mark.parametrize("M,nK", [(13, 9), (21, 7), (1, 5)], ids=["P39", "P63", "P3"])
def test_multi_market_cost_parity(api, oracle, M, nK):
    mk, truth = _synthetic(oracle, 3, M, nK)
    g = I.rng(I.SEED_BASE + 9400 + M)
    pt_inst = g.integers(0, 3, 96).astype(np.int32)
    pts = truth[pt_inst] * g.uniform(0.9, 1.1, (96, 3 * M))
    pts = np.clip(pts, *I.box(I.MODEL_PERFWD, M))
    _cost_compare(api, oracle, mk, pts, pt_inst)


def test_domain_failures_match(api, oracle):
    mk = I.paper_caplet_market()
    x = _printed_point()
    pts = np.tile(x, (6, 1))
    pts[1, 0] = 0.0        # alpha_1 = 0
    pts[2, 1] = 1.0        # rho_1 = 1
    pts[3, 38] = -1e-3     # nu_13 < 0
    pts[4, 37] = -1.0      # rho_13 = -1
    c = api.Plan(mk).cost(torch.tensor(pts, device="cuda")).cpu().numpy()
    assert np.isfinite(c[0]) and np.isfinite(c[5])
    assert np.all(c[1:5] == np.inf)
    np.testing.assert_allclose(c[0], oracle.cost_batch(mk, x[None, :])[0], rtol=RTOL)


def _sa_compare(g, o):
    assert np.array_equal(g["accept"].cpu().numpy(), o["accept"])
    assert np.array_equal(g["level_best"].cpu().numpy(), o["level_best"])
    np.testing.assert_allclose(g["best_f"].cpu().numpy(), o["best_f"], rtol=RTOL)
    assert np.array_equal(g["best_x"].cpu().numpy(), o["best_x"])
    np.testing.assert_allclose(g["chain_best_f"].cpu().numpy(), o["chain_best_f"], rtol=RTOL)


@pytest.mark.parametrize("T0", [10.0, 1e-3], ids=["paper-T0", "cold"])
def test_paper_market_accept_parity(api, oracle, T0):
    """P = 39: 10 Philox blocks a step, 6 steps a pass, N = 10 (ragged)."""
    mk = I.paper_caplet_market()
    lb, ub = I.box(I.MODEL_PERFWD, 13)
    kw = dict(T0=T0, cool=0.99, n_levels=5, n_steps=10, seed=6)
    g = api.Plan(mk).sa(40, lb, ub, record=True, chain_best=True, **kw)
    o = oracle.sa_calibrate(mk, 40, lb, ub, record=True, **kw)
    _sa_compare(g, o)
    acc = g["accept"].cpu().numpy()
    assert 0.0 < acc.mean() < 1.0


def test_max_params_accept_parity(api, oracle):
    """P = 63: 16 Philox blocks a step, 4 steps a pass, N = 7 (ragged), two
    markets, given starts and per-market temperatures."""
    mk, truth = _synthetic(oracle, 2, 21, 5)
    lb, ub = I.box(I.MODEL_PERFWD, 21)
    lb2, ub2 = np.tile(lb, (2, 1)), np.tile(ub, (2, 1))
    x0 = np.clip(truth * 1.05, lb2, ub2)
    kw = dict(T0=1.0, cool=0.7, n_levels=3, n_steps=7, seed=61, x0=x0, step_frac=0.01,
              T0_per_inst=np.array([0.01, 0.1]))
    chains = np.array([24, 9], np.int32)
    g = api.Plan(mk).sa(chains, lb2, ub2, record=True, chain_best=True, **kw)
    o = oracle.sa_calibrate(mk, chains, lb2, ub2, record=True, **kw)
    _sa_compare(g, o)
    assert 0.0 < g["accept"].cpu().numpy().mean() < 1.0


@pytest.mark.parametrize("waves,occ", [(4, 4), (1, 1)])
def test_e2_full_size_sampled_chains(api, oracle, waves, occ):
    """The paper's E2 launch: 16384 chains of the P = 39 market at T0 = 10;
    sampled chains of level 0 against the oracle's replay of those chains."""
    w = W.paper_e2()
    mk = w.market
    lb, ub = I.box(I.MODEL_PERFWD, 13)
    g = I.rng(I.SEED_BASE + 9500)
    sc = np.concatenate([g.choice(w.chains, 10, replace=False), [0, w.chains - 1]])
    sc = sc.astype(np.int32)
    si = np.zeros(len(sc), np.int32)
    r = api.Plan(mk).sa(w.chains, lb, ub, T0=w.extra["T0"], cool=1.0, n_levels=1,
                        n_steps=w.n_steps, seed=w.seed, record=True, chain_best=True,
                        waves=waves, occupancy=occ)
    o = oracle.sa_level0_sample(mk, w.chains, lb, ub, T0=w.extra["T0"], n_steps=w.n_steps,
                                seed=w.seed, sample_inst=si, sample_chain=sc)
    acc = r["accept"].cpu().numpy().reshape(w.n_steps, w.chains)
    cbf = r["chain_best_f"].cpu().numpy()
    cbx = r["chain_best_x"].cpu().numpy().reshape(w.chains, -1)
    for j, c in enumerate(sc):
        assert np.array_equal(acc[:, c], o["accept"][j]), f"chain {c}"
        assert abs(cbf[c] - o["BF"][j]) <= RTOL * abs(o["BF"][j]), f"chain {c}"
        assert np.array_equal(cbx[c], o["BX"][j]), f"chain {c}"
    assert 0.0 < acc.mean() < 1.0


def test_adjoint_and_lm_refuse_perfwd(api):
    mk = I.paper_caplet_market()
    plan = api.Plan(mk)
    x = torch.tensor(_printed_point()[None, :], device="cuda")
    lb, ub = I.box(I.MODEL_PERFWD, 13)
    with pytest.raises(api._lib.SabrError, match="GLOBAL4 and LMM12"):
        plan.vjp(x)
    with pytest.raises(api._lib.SabrError, match="GLOBAL4 and LMM12"):
        plan.lm(x, lb, ub)


def test_polish_per_forward_as_global4(api, oracle):
    """The E2 polish: each forward's triple refined by LM as a GLOBAL4
    instance with beta frozen at 0.5; the PERFWD cost of the polished point
    (GPU) equals the sum of the polished GLOBAL4 costs, does not exceed the
    start's, and the GLOBAL4 costs agree with the oracle's at the GPU's
    polished points."""
    mk = I.paper_caplet_market()
    plan = api.Plan(mk)
    lb, ub = I.box(I.MODEL_PERFWD, 13)
    r = plan.sa(64, lb, ub, T0=10.0, cool=0.9, n_levels=20, n_steps=10, seed=7)
    x = r["best_x"].cpu().numpy()[0]
    f0 = float(r["best_f"].cpu().numpy()[0])
    g4 = I.perfwd_as_global4(mk)
    plan4 = api.Plan(g4)
    lb4 = np.tile([0.001, 0.5, -0.99, 0.001], (13, 1))
    ub4 = np.tile([0.2, 0.5, 0.99, 1.0], (13, 1))
    starts = torch.tensor(I.perfwd_points_as_global4(x, 0.5), device="cuda")
    y, f4, it = plan4.lm(starts, lb4, ub4, pt_inst=torch.arange(13, dtype=torch.int32,
                                                                  device="cuda"),
                         max_iter=100)
    y = y.cpu().numpy()
    f4 = f4.cpu().numpy()
    assert np.all(y[:, 1] == 0.5)
    xp = I.global4_points_as_perfwd(y)
    fp = float(plan.cost(torch.tensor(xp[None, :], device="cuda")).cpu().numpy()[0])
    np.testing.assert_allclose(fp, f4.sum(), rtol=1e-12)
    assert fp <= f0
    np.testing.assert_allclose(f4, oracle.cost_batch(g4, y, np.arange(13, dtype=np.int32)),
                               rtol=RTOL)
