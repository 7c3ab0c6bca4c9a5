"""Two chains per wave (sa_config.chains_per_wave = 2, GLOBAL4): lanes 0-31
carry one chain and lanes 32-63 the next, each half drawing its own Philox
uniforms, pricing the quotes 32 at a time and taking its own Metropolis
decision of Sec. 3's SA box.  The accept/reject sequences must match the
oracle's over the whole c1 schedule, on sampled instances of c3 at full
size, on a ragged batch whose odd chain counts leave the upper half of an
instance's last wave without a chain, in both residual modes and with
eq. (3), on markets smaller than one 32-lane pass, under hipGraph replay and
through the entry point that allocates nothing; and the results must equal
those of one chain per wave bit for bit."""
import numpy as np
import pytest

from paper_2408_01470_amd import inputs as I
from paper_2408_01470_amd import workloads as W
from sa_divergence import check_restarts, first_mismatch
from test_gpu_schedules import _full_schedule, _sampled_instances

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RTOL = 1e-12


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_01470_amd import api as A
    return A


def test_c1_full_schedule_paired(api, oracle):
    """c1's 64 chains, 200 levels x 100 steps, 32 waves of two chains."""
    w = W.config1()
    _full_schedule(api, oracle, w, w.chains, 4, chains_per_wave=2)


def test_c3_full_size_two_levels_paired(api, oracle):
    """c3 at full size (256 markets, 1024 chains each) with paired chains:
    the smallest, the largest and two more instances against the oracle."""
    w = W.config3()
    nq = I.n_quotes(w.market)
    sample = sorted({0, int(np.argmax(nq)), int(np.argmin(nq)), w.n_inst - 1})
    _sampled_instances(api, oracle, w, sample, 4, 1, chains_per_wave=2)


def _ragged(oracle, residual=I.RESID_VOL, formula=0):
    from conftest import complete_with_oracle
    m, truth, noise = I.batch_markets(n_markets=5, M_range=(3, 20), nK_range=(3, 11),
                                      seed=I.SEED_BASE + 92)
    m = dict(m, residual=residual, formula=formula)
    return complete_with_oracle(oracle, m, truth, noise)


@pytest.mark.parametrize("residual,formula,waves", [(I.RESID_VOL, 0, 4), (I.RESID_PRICE, 0, 2),
                                                    (I.RESID_VOL, 1, 8)])
def test_ragged_batch_odd_chains(api, oracle, residual, formula, waves):
    """Markets of 36..160 quotes (a partial 32-lane pass in most), odd chain
    counts (a half-wave with no chain at each instance's end), per-instance
    temperatures."""
    mk = _ragged(oracle, residual, formula)
    lb, ub = I.box(0)
    chains = np.array([5, 1, 12, 3, 7], np.int32)
    T0s = np.array([0.05, 0.02, 0.08, 0.01, 0.03])
    kw = dict(T0=0.05, T0_per_inst=T0s, cool=0.8, n_levels=6, n_steps=15, seed=19, record=True)
    plan = api.Plan(mk)
    g = plan.sa(chains, lb, ub, chain_best=True, waves=waves, chains_per_wave=2, **kw)
    torch.cuda.synchronize()
    o = oracle.sa_calibrate(mk, chains, lb, ub, **kw)
    where = first_mismatch(g["accept"].cpu().numpy(), o["accept"], 6, 15, chains)
    assert where is None, f"first mismatch at {where}"
    msg = check_restarts(g["level_best"].cpu().numpy(), o["level_best"])
    assert msg is None, msg
    assert np.array_equal(g["best_x"].cpu().numpy(), o["best_x"])
    np.testing.assert_allclose(g["best_f"].cpu().numpy(), o["best_f"], rtol=RTOL)
    np.testing.assert_allclose(g["chain_best_f"].cpu().numpy(), o["chain_best_f"], rtol=RTOL)
    np.testing.assert_array_equal(g["trace"].cpu().numpy()[:, :, 1], o["trace"][:, :, 1])


def test_paired_graph_replay_and_noalloc_match_eager(api, oracle):
    """The paired launches replayed from a hipGraph (other eager work in
    between) and run through sa_calibrate_noalloc give the eager results bit
    for bit."""
    mk = _ragged(oracle)
    lb, ub = I.box(0)
    chains = np.array([5, 1, 12, 3, 7], np.int32)
    kw = dict(T0=0.05, cool=0.8, n_levels=5, n_steps=11, seed=23, record=True, chain_best=True,
              waves=4, chains_per_wave=2)
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


def test_paired_and_single_chains_agree(api, oracle):
    """The same calibration with one chain per wave and with two gives the
    same results bit for bit: each half keeps the partial sums of the 64
    lanes it stands for and adds them in the one-wave order."""
    mk = _ragged(oracle, I.RESID_PRICE)
    lb, ub = I.box(0)
    chains = np.array([9, 4, 16, 2, 11], np.int32)
    kw = dict(T0=0.05, cool=0.8, n_levels=4, n_steps=10, seed=41, record=True, chain_best=True,
              waves=4)
    plan = api.Plan(mk)
    a = plan.sa(chains, lb, ub, **kw)
    b = plan.sa(chains, lb, ub, chains_per_wave=2, **kw)
    torch.cuda.synchronize()
    for k in ("accept", "level_best", "best_x", "best_f", "chain_best_x", "chain_best_f"):
        assert torch.equal(a[k], b[k]), k
    assert torch.equal(a["trace"][:, :, :2], b["trace"][:, :, :2])   # not the device times


def test_paired_full_size_c3_equals_one_chain_per_wave(api, oracle):
    """c3 at full size (256 markets of 65-585 quotes, 1024 chains each), two
    levels at the benchmark's temperatures: paired and one-wave launches
    agree bit for bit."""
    from test_gpu_schedules import _workload
    w = W.config3()
    mk, T0s, cool = _workload(oracle, w)
    lb, ub = I.box(0)
    kw = dict(T0=T0s[0], T0_per_inst=T0s, cool=cool, n_levels=2, n_steps=w.n_steps, seed=w.seed,
              step_frac=w.step_frac, record=True, chain_best=True)
    plan = api.Plan(mk)
    a = plan.sa(w.chains, lb, ub, waves=4, occupancy=1, **kw)
    b = plan.sa(w.chains, lb, ub, waves=4, occupancy=4, chains_per_wave=2, **kw)
    torch.cuda.synchronize()
    for k in ("accept", "level_best", "best_x", "best_f", "chain_best_f"):
        assert torch.equal(a[k], b[k]), k


def test_paired_tiny_markets_and_lone_chains(api, oracle):
    """Markets of 6..9 quotes (one 32-lane pass, most lanes idle) and
    instances of one and three chains (the upper half of their last wave
    holds no chain): the oracle's accept flags, and one chain per wave bit
    for bit."""
    from conftest import complete_with_oracle
    m, truth, noise = I.batch_markets(n_markets=4, M_range=(2, 3), nK_range=(2, 4),
                                      seed=I.SEED_BASE + 93)
    mk = complete_with_oracle(oracle, m, truth, noise)
    assert I.n_quotes(mk).max() < 32
    lb, ub = I.box(0)
    chains = np.array([1, 3, 2, 1], np.int32)
    kw = dict(T0=0.02, cool=0.7, n_levels=5, n_steps=12, seed=43, record=True)
    plan = api.Plan(mk)
    g = plan.sa(chains, lb, ub, chain_best=True, waves=2, chains_per_wave=2, **kw)
    one = plan.sa(chains, lb, ub, chain_best=True, waves=2, **kw)
    torch.cuda.synchronize()
    o = oracle.sa_calibrate(mk, chains, lb, ub, **kw)
    where = first_mismatch(g["accept"].cpu().numpy(), o["accept"], 5, 12, chains)
    assert where is None, f"first mismatch at {where}"
    np.testing.assert_allclose(g["best_f"].cpu().numpy(), o["best_f"], rtol=RTOL)
    for k in ("accept", "level_best", "best_x", "best_f", "chain_best_x", "chain_best_f"):
        assert torch.equal(g[k], one[k]), k
