"""Chains split over several waves (sa_config.waves_per_chain > 1): each
chain is a workgroup whose waves take every k-th block of 64 quotes and
combine their partial costs in LDS before the Metropolis test of Sec. 3's
SA box.  The accept/reject sequences must still match the oracle's, over
the whole c1 schedule, on the c2 market, with waves that hold no quote at
all, on a ragged batch under hipGraph replay and through the entry point
that allocates nothing."""
import numpy as np
import pytest

from paper_2408_01470_amd import inputs as I
from paper_2408_01470_amd import workloads as W
from sa_divergence import check_restarts, first_mismatch
from test_gpu_schedules import _full_schedule

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RTOL = 1e-12


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_01470_amd import api as A
    return A


def test_c1_full_schedule_two_waves_per_chain(api, oracle):
    """c1's 110 quotes: wave 0 takes 64, wave 1 the other 46."""
    w = W.config1()
    _full_schedule(api, oracle, w, w.chains, 0, waves_per_chain=2)


def test_c2_market_four_waves_per_chain(api, oracle):
    """LMM12 with the chunked map: every wave maps the point, the quotes of
    each chunk go round the four waves."""
    w = W.config2()
    _full_schedule(api, oracle, w, 64, 0, waves_per_chain=4, n_levels=60)


def _ragged(oracle):
    from conftest import complete_with_oracle
    m, truth, noise = I.batch_markets(n_markets=5, M_range=(3, 20), nK_range=(3, 11),
                                      seed=I.SEED_BASE + 90)
    return complete_with_oracle(oracle, m, truth, noise)


@pytest.mark.parametrize("wpc", [3, 8])
def test_ragged_batch_with_idle_waves(api, oracle, wpc):
    """Markets of 30..160 quotes: with 3 or 8 waves per chain some waves hold
    no quote (their partial is 0); uneven chain counts per instance."""
    mk = _ragged(oracle)
    nq = I.n_quotes(mk)
    assert nq.min() < 64 and nq.max() > 128, nq
    lb, ub = I.box(0)
    chains = np.array([5, 1, 12, 3, 7], np.int32)
    T0s = np.array([0.05, 0.02, 0.08, 0.01, 0.03])
    kw = dict(T0=0.05, T0_per_inst=T0s, cool=0.8, n_levels=6, n_steps=15, seed=17, record=True)
    plan = api.Plan(mk)
    g = plan.sa(chains, lb, ub, chain_best=True, waves_per_chain=wpc, **kw)
    torch.cuda.synchronize()
    o = oracle.sa_calibrate(mk, chains, lb, ub, **kw)
    where = first_mismatch(g["accept"].cpu().numpy(), o["accept"], 6, 15, chains)
    assert where is None, f"first mismatch at {where}"
    msg = check_restarts(g["level_best"].cpu().numpy(), o["level_best"])
    assert msg is None, msg
    assert np.array_equal(g["best_x"].cpu().numpy(), o["best_x"])
    np.testing.assert_allclose(g["best_f"].cpu().numpy(), o["best_f"], rtol=RTOL)
    np.testing.assert_allclose(g["chain_best_f"].cpu().numpy(), o["chain_best_f"], rtol=RTOL)


def test_split_graph_replay_and_noalloc_match_eager(api, oracle):
    """The same split launches replayed from a hipGraph (other eager work in
    between) and run through sa_calibrate_noalloc give the eager results
    bit for bit."""
    mk = _ragged(oracle)
    lb, ub = I.box(0)
    chains = np.array([5, 1, 12, 3, 7], np.int32)
    kw = dict(T0=0.05, cool=0.8, n_levels=5, n_steps=11, seed=23, record=True, chain_best=True,
              waves_per_chain=2)
    plan = api.Plan(mk)
    eager = plan.sa(chains, lb, ub, **kw)
    torch.cuda.synchronize()
    keys = ("accept", "level_best", "best_x", "best_f", "chain_best_x", "chain_best_f")
    na = plan.sa(chains, lb, ub, noalloc=True, **kw)
    torch.cuda.synchronize()
    for k in keys:
        assert torch.equal(na[k], eager[k]), f"noalloc: {k}"
    side = torch.cuda.Stream()
    ws, outs = eager["workspace"], None
    pts = torch.tensor(I.random_box_points(0, 64, 3), device="cuda")
    for rep in range(3):
        with torch.cuda.stream(side):
            g = plan.sa(chains, lb, ub, use_graph=True, stream=side, workspace=ws, out=outs, **kw)
        outs = g
        side.synchronize()
        plan.cost(pts)
        torch.cuda.synchronize()
        for k in keys:
            assert torch.equal(g[k], eager[k]), f"replay {rep}: {k}"


@pytest.mark.parametrize("n_ten", [22, 30])
def test_long_swaps_split_over_waves(api, oracle, n_ten):
    """Swaps of 22 forwards (the 24-register swap column) and of 30 (the LDS
    column, one per wave) with their quotes split over three waves."""
    m, truth, noise = I.lmm_market(M=n_ten + 4, n_cap_K=3, n_exp=3, n_ten=n_ten, n_swp_K=3,
                                   residual=I.RESID_PRICE)
    vm = I.as_vol_market(m)
    mv, _, _, ok = oracle.model_values(vm, 0, truth[0])
    assert ok
    mk = I.complete_market(m, mv, noise[:len(mv)])
    assert max(mk["und_len"]) == n_ten
    lb, ub = I.box(1)
    x0 = np.clip(truth[0], lb, ub)
    kw = dict(T0=0.02, cool=0.8, n_levels=3, n_steps=8, seed=29, x0=x0, record=True)
    plan = api.Plan(mk)
    g = plan.sa(6, lb, ub, chain_best=True, waves_per_chain=3, **kw)
    torch.cuda.synchronize()
    o = oracle.sa_calibrate(mk, 6, lb, ub, **kw)
    where = first_mismatch(g["accept"].cpu().numpy(), o["accept"], 3, 8, [6])
    assert where is None, f"first mismatch at {where}"
    assert np.array_equal(g["level_best"].cpu().numpy(), o["level_best"])
    np.testing.assert_allclose(g["best_f"].cpu().numpy(), o["best_f"], rtol=RTOL)
