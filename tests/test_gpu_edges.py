"""GPU edge cases against the oracle: zero steps, zero levels, one chain,
given starting points with per-instance temperatures, frozen coordinates,
empty inputs, LM with no iterations, and costs at every corner of the
search box (the degenerate parameter values: beta = 0 and 1, |rho| = 0.99,
the smallest nu and alpha)."""
import itertools

import numpy as np
import pytest

from conftest import complete_with_oracle
from paper_2408_01470_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RTOL = 1e-12


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_01470_amd import api as A
    return A


def _compare(g, o, C_total):
    assert np.array_equal(g["level_best"].cpu().numpy(), o["level_best"])
    np.testing.assert_allclose(g["best_f"].cpu().numpy(), o["best_f"], rtol=RTOL)
    assert np.array_equal(g["best_x"].cpu().numpy(), o["best_x"])
    if g.get("accept") is not None and o["accept"] is not None:
        assert np.array_equal(g["accept"].cpu().numpy(), o["accept"])


@pytest.mark.parametrize("L,N,C", [(3, 0, 8), (0, 5, 8), (4, 6, 1)],
                         ids=["no-steps", "no-levels", "one-chain"])
def test_sa_degenerate_schedules(api, oracle, c1_market, L, N, C):
    mk, _ = c1_market
    lb, ub = I.box(0)
    plan = api.Plan(mk)
    kw = dict(T0=0.05, cool=0.8, n_levels=L, n_steps=N, seed=23)
    g = plan.sa(C, lb, ub, record=True, chain_best=True, **kw)
    o = oracle.sa_calibrate(mk, C, lb, ub, record=True, **kw)
    _compare(g, o, C)
    np.testing.assert_allclose(g["chain_best_f"].cpu().numpy(), o["chain_best_f"], rtol=RTOL)
    if L > 0:
        tr = g["trace"].cpu().numpy()
        np.testing.assert_allclose(tr[0, :, 0], o["trace"][0, :, 0], rtol=RTOL)
        np.testing.assert_array_equal(tr[0, :, 1], o["trace"][0, :, 1])


def test_sa_given_start_per_instance_T0_and_frozen_coordinate(api, oracle):
    m, truth, noise = I.batch_markets(n_markets=3, M_range=(4, 12), nK_range=(3, 9))
    mk = complete_with_oracle(oracle, m, truth, noise)
    lb, ub = I.box(0)
    lb3 = np.tile(lb, (3, 1))
    ub3 = np.tile(ub, (3, 1))
    lb3[1, 1] = ub3[1, 1] = 0.5          # beta fixed on instance 1
    x0 = np.clip(truth * 1.05, lb3, ub3)
    T0s = np.array([0.02, 0.05, 0.1])
    chains = np.array([5, 12, 3], np.int32)
    kw = dict(T0=1.0, cool=0.7, n_levels=5, n_steps=8, seed=29, x0=x0, T0_per_inst=T0s)
    plan = api.Plan(mk)
    g = plan.sa(chains, lb3, ub3, record=True, chain_best=True, **kw)
    o = oracle.sa_calibrate(mk, chains, lb3, ub3, record=True, **kw)
    _compare(g, o, int(chains.sum()))
    cbx = g["chain_best_x"].cpu().numpy()
    assert np.all(cbx[5:17, 1] == 0.5)
    assert 0.0 < g["accept"].cpu().numpy().mean() < 1.0


def test_empty_inputs(api, c1_market):
    mk, _ = c1_market
    plan = api.Plan(mk)
    e = torch.zeros((0, 4), dtype=torch.float64, device="cuda")
    assert plan.cost(e).numel() == 0
    out = plan.vjp(e, normal=True)
    assert out["cost"].numel() == 0 and out["grad"].numel() == 0
    x, f, it = plan.lm(e, *I.box(0), max_iter=5)
    assert x.numel() == 0 and f.numel() == 0


def test_lm_zero_iterations_returns_start(api, oracle, c1_market):
    mk, truth = c1_market
    plan = api.Plan(mk)
    lb, ub = I.box(0)
    starts = np.clip(truth[0][None, :] * np.array([[1.1, 0.9, 1.0, 1.2]]), lb, ub)
    x, f, it = plan.lm(torch.tensor(starts, device="cuda"), lb, ub, max_iter=0)
    assert np.array_equal(x.cpu().numpy(), starts)
    assert int(it.cpu().numpy()[0]) == 0
    np.testing.assert_allclose(f.cpu().numpy(), oracle.cost_batch(mk, starts), rtol=RTOL)


@pytest.mark.parametrize("residual", [0, 1], ids=["vol", "price"])
def test_cost_at_box_corners(api, oracle, residual):
    m, truth, noise = I.caplet_market(residual=residual)
    mk = complete_with_oracle(oracle, m, truth, noise)
    lb, ub = I.box(0)
    corners = np.array([[ub[k] if b else lb[k] for k, b in enumerate(bits)]
                        for bits in itertools.product([0, 1], repeat=4)])
    plan = api.Plan(mk)
    c_g = plan.cost(torch.tensor(corners, device="cuda")).cpu().numpy()
    c_o = oracle.cost_batch(mk, corners)
    fin = np.isfinite(c_o)
    assert np.array_equal(fin, np.isfinite(c_g))
    np.testing.assert_allclose(c_g[fin], c_o[fin], rtol=RTOL)


def test_lmm_cost_at_box_corners_sampled(api, oracle, c2_market):
    mk, _ = c2_market
    lb, ub = I.box(1)
    g = np.random.default_rng(41)
    bits = g.integers(0, 2, (64, 12))
    corners = np.where(bits == 1, ub[None, :], lb[None, :])
    plan = api.Plan(mk)
    c_g = plan.cost(torch.tensor(corners, device="cuda")).cpu().numpy()
    c_o = oracle.cost_batch(mk, corners)
    fin = np.isfinite(c_o)
    assert np.array_equal(fin, np.isfinite(c_g))
    scale = np.maximum(np.abs(c_o[fin]), 1e-300)
    assert np.max(np.abs(c_g[fin] - c_o[fin]) / scale) <= RTOL


def test_calls_on_a_stream_other_than_the_current_one(api, oracle, c1_market, c2_market):
    """Every entry point given a side stream while torch's current stream is
    another: the launch waits for the current stream's allocations and
    fills, its tensors are recorded on the side stream, and the results
    equal those of the same calls on the current stream."""
    mk, truth = c1_market
    plan = api.Plan(mk)
    side = torch.cuda.Stream()
    cur = torch.cuda.current_stream()
    pts = torch.tensor(I.random_box_points(0, 300, 9), device="cuda")
    lb, ub = I.box(0)
    ref_c, ref_r = plan.cost(pts, resid=True)
    ref_v = plan.vjp(pts)
    kw = dict(T0=0.05, cool=0.8, n_levels=3, n_steps=10, seed=5, record=True)
    ref_s = plan.sa(32, lb, ub, **kw)
    ref_l = plan.lm(pts[:8], lb, ub, max_iter=5)
    got_c, got_r = plan.cost(pts, resid=True, stream=side)
    got_v = plan.vjp(pts, stream=side)
    got_s = plan.sa(32, lb, ub, stream=side, **kw)
    got_l = plan.lm(pts[:8], lb, ub, max_iter=5, stream=side)
    cur.wait_stream(side)
    assert torch.equal(ref_c, got_c) and torch.equal(ref_r.nan_to_num(), got_r.nan_to_num())
    assert torch.equal(ref_v["grad"], got_v["grad"])
    assert torch.equal(ref_s["accept"], got_s["accept"]) and torch.equal(ref_s["best_x"],
                                                                          got_s["best_x"])
    assert torch.equal(ref_l[0], got_l[0])
    mk2, _ = c2_market
    plan2 = api.Plan(mk2, stream=side)        # upload on the side stream
    p2 = torch.tensor(np.clip(I.random_box_points(1, 64, 4), *I.box(1)), device="cuda")
    g2 = plan2.vjp(p2, stream=side)
    cur.wait_stream(side)
    np.testing.assert_array_equal(g2["grad"].cpu().numpy(), plan2.vjp(p2)["grad"].cpu().numpy())
    mc = api.McPlan(I.mc_problem(M=6, n_cap_K=2, n_swaptions=3), stream=side)
    pr, _ = mc.price(1000, 0.05, 3, stream=side)
    cur.wait_stream(side)
    pr0, _ = mc.price(1000, 0.05, 3)
    assert torch.equal(pr, pr0)
