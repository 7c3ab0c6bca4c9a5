"""GPU parity at the benchmark workloads' full sizes, in the launch shapes the
benchmark's tuner chooses from.

c2 (LMM12, 985 quotes, 4096 chains): every accept decision of the first
three levels against the oracle's annealing, bit for bit, plus the level-end
restart indices and per-chain best-ever costs.  c3 (256 caplet markets) and
c5 (64 LMM12 markets x 8838 quotes, swaps of up to 20 forwards, the map's
LDS column): sampled chains of level 0 against the oracle's replay of those
chains alone.  Markets are completed with oracle model vols."""
import numpy as np
import pytest

from paper_2408_01470_amd import inputs as I
from paper_2408_01470_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RTOL = 1e-12
SHAPES = [(4, 4), (4, 1), (1, 3)]


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_01470_amd import api as A
    return A


def _oracle_vols(oracle, vm, truth):
    out = []
    M = oracle.Market(vm)
    for i in range(M.n_inst):
        mv, _, _, ok = oracle.model_values(M, i, truth[i])
        assert ok
        out.append(mv)
    return np.concatenate(out)


def _schedule_T0(oracle, w, mk):
    """T0 per instance by the benchmark's rule, with oracle costs."""
    pts = W.schedule_points(w.model, w.seed)
    nq = I.n_quotes(mk)
    T0s = []
    for i in range(w.n_inst):
        c = oracle.cost_batch(mk, pts, np.full(len(pts), i, np.int32))
        T0s.append(W.schedule(c, nq[i], w.n_levels)[0])
    return np.array(T0s), W.schedule(c, nq[-1], w.n_levels)[1]


@pytest.fixture(scope="module")
def c2_full(oracle):
    w = W.config2()
    mk = W.synthesize(w, lambda vm, t: _oracle_vols(oracle, vm, t))
    T0s, cool = _schedule_T0(oracle, w, mk)
    lb, ub = I.box(w.model)
    kw = dict(T0=T0s[0], cool=cool, n_levels=3, n_steps=w.n_steps, seed=w.seed,
              step_frac=w.step_frac, T0_per_inst=T0s)
    o = oracle.sa_calibrate(mk, w.chains, lb, ub, record=True, **kw)
    return w, mk, lb, ub, kw, o


@pytest.mark.parametrize("waves,occ", SHAPES)
def test_c2_full_size_accept_parity(api, c2_full, waves, occ):
    w, mk, lb, ub, kw, o = c2_full
    plan = api.Plan(mk)
    g = plan.sa(w.chains, lb, ub, record=True, chain_best=True, waves=waves, occupancy=occ, **kw)
    acc = g["accept"].cpu().numpy().reshape(3, w.n_steps, w.chains)
    ref = o["accept"].reshape(3, w.n_steps, w.chains)
    bad = np.argwhere(acc != ref)
    assert len(bad) == 0, f"first divergence (level, step, chain) = {tuple(bad[0])}"
    assert 0.0 < acc.mean() < 1.0
    assert np.array_equal(g["level_best"].cpu().numpy(), o["level_best"])
    np.testing.assert_allclose(g["chain_best_f"].cpu().numpy(), o["chain_best_f"], rtol=RTOL)
    assert np.array_equal(g["best_x"].cpu().numpy(), o["best_x"])


def _sampled_level0(api, oracle, w, waves, occ, n_inst_sample, n_chain_sample, seed):
    mk = W.synthesize(w, lambda vm, t: _oracle_vols(oracle, vm, t))
    lb, ub = I.box(w.model)
    T0s = np.full(w.n_inst, 1e-3)
    g = np.random.default_rng(seed)
    insts = np.sort(g.choice(w.n_inst, n_inst_sample, replace=False))
    si = np.repeat(insts, n_chain_sample).astype(np.int32)
    sc = np.concatenate([g.choice(w.chains, n_chain_sample, replace=False)
                         for _ in insts]).astype(np.int32)
    si = np.concatenate([si, [w.n_inst - 1]]).astype(np.int32)   # last chain of the last market
    sc = np.concatenate([sc, [w.chains - 1]]).astype(np.int32)
    plan = api.Plan(mk)
    r = plan.sa(w.chains, lb, ub, T0=1.0, cool=1.0, n_levels=1, n_steps=w.n_steps, seed=w.seed,
                step_frac=w.step_frac, T0_per_inst=T0s, record=True, chain_best=True,
                waves=waves, occupancy=occ)
    o = oracle.sa_level0_sample(mk, w.chains, lb, ub, T0=1.0, n_steps=w.n_steps, seed=w.seed,
                                sample_inst=si, sample_chain=sc, step_frac=w.step_frac,
                                T0_per_inst=T0s)
    acc = r["accept"].cpu().numpy().reshape(w.n_inst, w.n_steps, w.chains)
    cbf = r["chain_best_f"].cpu().numpy().reshape(w.n_inst, w.chains)
    cbx = r["chain_best_x"].cpu().numpy().reshape(w.n_inst, w.chains, -1)
    for j, (i, c) in enumerate(zip(si, sc)):
        assert np.array_equal(acc[i, :, c], o["accept"][j]), f"instance {i} chain {c}"
        assert abs(cbf[i, c] - o["BF"][j]) <= RTOL * abs(o["BF"][j]), f"instance {i} chain {c}"
        assert np.array_equal(cbx[i, c], o["BX"][j]), f"instance {i} chain {c}"
    return acc


@pytest.mark.parametrize("waves,occ", [(4, 4), (1, 1)])
def test_c3_full_size_sampled_chains(api, oracle, waves, occ):
    acc = _sampled_level0(api, oracle, W.config3(), waves, occ, 6, 4, 3)
    assert 0.0 < acc.mean() < 1.0


@pytest.mark.parametrize("waves,occ", [(4, 4), (1, 1)])
def test_c5_full_size_sampled_chains(api, oracle, waves, occ):
    w = W.config5()
    assert max(w.market["und_len"]) > 16      # long swaps: the map's LDS column
    acc = _sampled_level0(api, oracle, w, waves, occ, 3, 4, 5)
    assert 0.0 < acc.mean() < 1.0


def test_long_swaps_accept_parity(api, oracle):
    """Swaps of 20 forwards (the map's LDS column) over several levels."""
    m, truth, noise = I.lmm_market(seed=I.SEED_BASE + 77, M=24, n_cap_K=3, n_exp=3, n_ten=20,
                                   n_swp_K=3)
    assert max(m["und_len"]) == 20
    vm = I.as_vol_market(m)
    mk = I.complete_market(m, _oracle_vols(oracle, vm, truth), noise)
    lb, ub = I.box(1)
    kw = dict(T0=1e-3, cool=0.7, n_levels=4, n_steps=6, seed=19)
    plan = api.Plan(mk)
    g = plan.sa(16, lb, ub, record=True, **kw)
    o = oracle.sa_calibrate(mk, 16, lb, ub, record=True, **kw)
    assert np.array_equal(g["accept"].cpu().numpy(), o["accept"])
    assert np.array_equal(g["level_best"].cpu().numpy(), o["level_best"])
    np.testing.assert_allclose(g["best_f"].cpu().numpy(), o["best_f"], rtol=RTOL)
    pts = np.clip(truth[0][None, :] * np.random.default_rng(2).uniform(0.9, 1.1, (8, 12)), lb, ub)
    c_g = plan.cost(torch.tensor(pts, device="cuda")).cpu().numpy()
    np.testing.assert_allclose(c_g, oracle.cost_batch(mk, pts), rtol=RTOL)
