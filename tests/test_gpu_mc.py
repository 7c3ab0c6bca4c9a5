"""GPU parity of the Monte Carlo pricer (sabr_mc_price) against the oracle's
Monte Carlo under the Hagan SABR/LIBOR dynamics (Sec. 2.1): the same paths
(the counter-based normals of both sides, the same scheme), so every price
and standard error agrees to rounding (the elementary functions and the
order of the sums differ: relative 1e-9 is allowed); across path counts
that leave ragged waves and select 4, 2 or 1 lanes per path (up to 16384,
131072 and beyond; 8 lanes on the 13- and 16-forward cases), one forward and the most forwards, expiries at the
first and last fixing, and the paper's market.  At the replay's full size
(1e6 paths, dt = 1e-3) the prices are checked by properties that hold at any
size: a zero-strike swaption is worth P(0, T_a) - P(0, T_b), and the
paper's caplets agree with the oracle's estimate on the first paths within
their standard errors; runs are bitwise repeatable."""
import math

import numpy as np
import pytest

from paper_2408_01470_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RTOL = 1e-9


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_01470_amd import api as A
    return A


def _compare(api, oracle, p, n_paths, dt, seed):
    plan = api.McPlan(p)
    m, se = plan.price(n_paths, dt, seed)
    m, se = m.cpu().numpy(), se.cpu().numpy()
    mo, seo = oracle.mc_price(p, n_paths, dt, seed)
    scale = max(float(np.max(np.abs(mo))), 1e-300)
    np.testing.assert_allclose(m, mo, rtol=RTOL, atol=1e-12 * scale)
    np.testing.assert_allclose(se, seo, rtol=1e-7, atol=1e-12 * scale)
    return m, se


@pytest.mark.parametrize("n_paths", [1, 63, 64, 65, 1000, 4099, 16385, 131073])
def test_mc_parity_path_counts(api, oracle, n_paths):
    p = I.mc_problem(seed=I.SEED_BASE + 9800, M=8, n_cap_K=3, n_swaptions=6)
    m, se = _compare(api, oracle, p, n_paths, 0.05, 17)
    if n_paths == 1:
        assert np.all(se == 0.0)


@pytest.mark.parametrize("M,beta", [(1, None), (5, "random"), (16, None), (24, None)],
                         ids=["one-forward", "random-beta", "sixteen-forwards", "most-forwards"])
def test_mc_parity_shapes(api, oracle, M, beta):
    p = I.mc_problem(seed=I.SEED_BASE + 9810 + M, M=M, n_cap_K=2, n_swaptions=0 if M == 1 else 5,
                     beta=beta)
    if M > 1:   # expiries at the first and the last fixing, the longest swap
        p["opt_a"] = np.concatenate([p["opt_a"], [0, M - 1, 0]]).astype(np.int32)
        p["opt_b"] = np.concatenate([p["opt_b"], [M, M, 1]]).astype(np.int32)
        p["opt_K"] = np.concatenate([p["opt_K"], [p["F0"].mean(), p["F0"][-1], 0.0]])
    _compare(api, oracle, p, 700, 0.1, 23)


@pytest.mark.parametrize("M", [13, 16, 24])
@pytest.mark.parametrize("n_paths", [4096, 4097, 16385, 131073])
def test_mc_parity_lanes_per_path_by_register_budget(api, oracle, M, n_paths):
    """Every lanes-per-path variant (8, 4, 2 and 1 lanes at these path counts)
    of the kernels of each register budget (up to 13 forwards, 14 to 16,
    beyond 16) against the oracle on the same paths, at a coarse step."""
    p = I.mc_problem(seed=I.SEED_BASE + 9830 + M, M=M, n_cap_K=2, n_swaptions=4)
    p["opt_a"] = np.concatenate([p["opt_a"], [0, M - 1]]).astype(np.int32)
    p["opt_b"] = np.concatenate([p["opt_b"], [M, M]]).astype(np.int32)
    p["opt_K"] = np.concatenate([p["opt_K"], [p["F0"].mean(), p["F0"][-1]]])
    _compare(api, oracle, p, n_paths, 0.25, 29)


def test_mc_parity_paper_market(api, oracle):
    p = I.paper_mc_problem()
    _compare(api, oracle, p, 512, 0.02, 2408)
    q, _ = I.paper_mc_swaption_problem()       # the paper's fourteen swaptions
    _compare(api, oracle, q, 300, 0.01, 2408)


def test_mc_parity_coarse_and_fine_steps(api, oracle):
    p = I.mc_problem(seed=I.SEED_BASE + 9820, M=4, n_cap_K=3, n_swaptions=3)
    _compare(api, oracle, p, 300, 10.0, 5)       # one step per fixing interval
    _compare(api, oracle, p, 100, 0.003, 5)


def test_mc_full_size_properties(api, oracle):
    """The replay's full size: 1e6 paths, dt = 1e-3, the paper's market."""
    p = I.paper_mc_problem()
    M = len(p["T"])
    n, dt, seed = 1_000_000, 1e-3, 2408
    plan = api.McPlan(p)
    m, se = [t.cpu().numpy() for t in plan.price(n, dt, seed)]
    m2, se2 = [t.cpu().numpy() for t in plan.price(n, dt, seed)]
    assert np.array_equal(m, m2) and np.array_equal(se, se2)
    mo, seo = oracle.mc_price(p, 1000, dt, seed)
    assert np.all(np.abs(m - mo) <= 4.5 * seo + 1e-12)
    assert np.all(se <= 2.0 * seo * math.sqrt(1000 / n) + 1e-12)   # se ~ 1/sqrt(n)
    # zero-strike swaptions: the floating leg, P(0, T_a) - P(0, T_b)
    q = dict(p)
    ab = [(0, 1), (0, M), (5, 9), (M - 1, M)]
    q["opt_a"] = np.array([a for a, _ in ab], np.int32)
    q["opt_b"] = np.array([b for _, b in ab], np.int32)
    q["opt_K"] = np.zeros(len(ab))
    mz, sz = [t.cpu().numpy() for t in api.McPlan(q).price(n, dt, seed)]
    P = [q["P0"]]
    for k in range(M):
        P.append(P[-1] / (1.0 + q["tau"][k] * q["F0"][k]))
    exact = np.array([P[a] - P[b] for a, b in ab])
    assert np.all(np.abs(mz - exact) <= 4.5 * sz + 1e-5 * exact), np.c_[mz, exact, sz]


def test_mc_errors(api):
    p = I.mc_problem(seed=I.SEED_BASE + 9830, M=3, n_swaptions=1)
    plan = api.McPlan(p)
    with pytest.raises(Exception) as e:
        plan.price(0, 0.1, 1)
    assert "n_paths" in str(e.value)
    with pytest.raises(Exception) as e:
        plan.price(10, 0.0, 1)
    assert "dt" in str(e.value)
    with pytest.raises(Exception) as e:       # rejected before any allocation or launch
        plan.price((1 << 38) + 1, 0.1, 1)
    assert "n_paths" in str(e.value)
    from paper_2408_01470_amd import _lib
    L = _lib.lib()
    out = torch.empty(plan.n_opt, dtype=torch.float64, device="cuda")
    ws = torch.empty(8, dtype=torch.uint8, device="cuda")
    import ctypes
    rc = L.sabr_mc_price(plan._h, 1000, 0.1, 1, ctypes.c_void_p(out.data_ptr()), None,
                         ctypes.c_void_p(ws.data_ptr()), 8, None)
    assert rc == -5 and b"workspace" in L.sabr_last_error()


def test_mc_cost(api, oracle):
    """sabr_mc_cost: the swaption cost of Sec. 3 over the same paths, against
    the oracle's prices; with and without weights, with the prices kept in
    the workspace."""
    p, printed = I.paper_mc_swaption_problem()
    tgt = printed[:, 0] / 100.0                  # the printed market prices
    w = np.linspace(0.5, 2.0, len(tgt))
    plan = api.McPlan(p)
    mo, _ = oracle.mc_price(p, 400, 0.02, 9)
    for weight in (None, w):
        c, pr = plan.cost(400, 0.02, 9, tgt, weight)
        ww = np.ones(len(tgt)) if weight is None else w
        np.testing.assert_allclose(pr.cpu().numpy(), mo, rtol=RTOL, atol=1e-15)
        assert float(c.cpu()[0]) == pytest.approx(float(np.sum(ww * (mo - tgt) ** 2)), rel=1e-8)
    from paper_2408_01470_amd import _lib
    import ctypes
    L = _lib.lib()
    ws, n = plan.workspace(400)
    t = torch.tensor(tgt, device="cuda")
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    assert L.sabr_mc_cost(plan._h, 400, 0.02, 9, ctypes.c_void_p(t.data_ptr()), None, None,
                          ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.data_ptr()), n,
                          None) == 0
    torch.cuda.synchronize()
    c, _ = plan.cost(400, 0.02, 9, tgt)
    assert float(out.cpu()[0]) == float(c.cpu()[0])


def test_mc_full_size_paper_swaptions(api):
    """The paper's fourteen swaptions x five strikes at its printed
    parameters, at the replay's full size (1e6 paths, dt = 1e-3): every cell
    within 5% of the printed Monte Carlo prices (the fixed leg's conventions
    are not printed; the oracle's pin has the same bound)."""
    p, printed = I.paper_mc_swaption_problem()
    m, se = [t.cpu().numpy() for t in api.McPlan(p).price(1_000_000, 1e-3, 2408)]
    rel = 100.0 * m / printed[:, 1] - 1.0
    assert np.max(np.abs(rel)) < 0.05 and np.mean(np.abs(rel)) < 0.03, rel
    assert np.all(100.0 * se < 0.01 * printed[:, 1])
