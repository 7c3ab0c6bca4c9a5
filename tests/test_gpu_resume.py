"""Checkpoint and resume of the annealing (sa_config.level0, state_in and
state_out): the Philox counters are functions of (instance, level, step,
chain, block) and a level boundary leaves every chain of an instance at its
restart point, so L levels in one run equal l levels, the state saved, and
L - l more from it, bit for bit; the saved state matches the CPU oracle's
(its points bit for bit, its costs to the parity tolerance), and a state the
oracle saved resumes on the GPU into the oracle's own run (Sec. 3's SA box,
levels after level l)."""
import numpy as np
import pytest

from paper_2408_01470_amd import inputs as I
from sa_divergence import check_restarts, first_mismatch

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RTOL = 1e-12


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_01470_amd import api as A
    return A


def _ragged(oracle):
    from conftest import complete_with_oracle
    m, truth, noise = I.batch_markets(n_markets=5, M_range=(3, 20), nK_range=(3, 11),
                                      seed=I.SEED_BASE + 94)
    return complete_with_oracle(oracle, m, truth, noise)


def _blocks(acc, chains, L, N):
    """Accept flags per instance as [L][N][C] arrays."""
    out, off = [], 0
    for C in chains:
        out.append(acc[off:off + L * N * C].reshape(L, N, C))
        off += L * N * C
    return out


def _state_parts(st, chains, P):
    """A state array split per instance into X, F, BX, BF, T."""
    out, off = [], 0
    for C in chains:
        s = st[off:off + 2 * C * (P + 1) + 1]
        out.append((s[:C * P], s[C * P:C * (P + 1)], s[C * (P + 1):C * (2 * P + 1)],
                    s[C * (2 * P + 1):C * (2 * P + 2)], s[-1]))
        off += 2 * C * (P + 1) + 1
    return out


@pytest.mark.parametrize("cpw", [1, 2])
def test_resume_equals_one_run(api, oracle, cpw):
    """7 levels in one run against 3 levels, their state, then 4 more from
    level 3, with one chain per wave and with two (the resumed init kernel's
    paired variant)."""
    mk = _ragged(oracle)
    lb, ub = I.box(0)
    chains = np.array([5, 1, 12, 3, 7], np.int32)
    L, l, N = 7, 3, 11
    kw = dict(T0=0.05, cool=0.8, n_steps=N, seed=29, record=True, chain_best=True, waves=4,
              chains_per_wave=cpw)
    plan = api.Plan(mk)
    full = plan.sa(chains, lb, ub, n_levels=L, state_out=True, **kw)
    first = plan.sa(chains, lb, ub, n_levels=l, state_out=True, **kw)
    rest = plan.sa(chains, lb, ub, n_levels=L - l, level0=l, state_in=first["state"],
                   state_out=True, **kw)
    torch.cuda.synchronize()
    af = _blocks(full["accept"].cpu().numpy(), chains, L, N)
    a1 = _blocks(first["accept"].cpu().numpy(), chains, l, N)
    a2 = _blocks(rest["accept"].cpu().numpy(), chains, L - l, N)
    for i in range(len(chains)):
        assert np.array_equal(af[i], np.concatenate([a1[i], a2[i]])), f"instance {i}"
    lbf = full["level_best"].cpu().numpy()
    assert np.array_equal(lbf[:, :l], first["level_best"].cpu().numpy())
    assert np.array_equal(lbf[:, l:], rest["level_best"].cpu().numpy())
    for k in ("best_x", "best_f", "chain_best_x", "chain_best_f", "state"):
        assert torch.equal(full[k], rest[k]), k
    assert torch.equal(full["trace"][:, l:, :2], rest["trace"][:, :, :2])
    assert list(rest["n_evals"]) == list(chains.astype(np.int64) * N * (L - l))


def test_state_matches_oracle_and_oracle_state_resumes(api, oracle):
    """The GPU's state after 2 levels against the oracle's; then the GPU
    resumes from the oracle's state for 3 more levels and follows the
    oracle's 5-level run."""
    mk = _ragged(oracle)
    lb, ub = I.box(0)
    chains = np.array([4, 9, 2, 6, 3], np.int32)
    L, l, N = 5, 2, 10
    kw = dict(T0=0.04, cool=0.75, n_steps=N, seed=31, record=True)
    plan = api.Plan(mk)
    P = plan.P
    g = plan.sa(chains, lb, ub, n_levels=l, state_out=True, **kw)
    torch.cuda.synchronize()
    o1 = oracle.sa_calibrate(mk, chains, lb, ub, n_levels=l, keep_state=True, **kw)
    where = first_mismatch(g["accept"].cpu().numpy(), o1["accept"], l, N, chains)
    assert where is None, f"first mismatch at {where}"
    for i, (gs, os_) in enumerate(zip(_state_parts(g["state"].cpu().numpy(), chains, P),
                                      _state_parts(o1["state"], chains, P))):
        assert np.array_equal(gs[0], os_[0]) and np.array_equal(gs[2], os_[2]), f"points, {i}"
        np.testing.assert_allclose(gs[1], os_[1], rtol=RTOL)
        np.testing.assert_allclose(gs[3], os_[3], rtol=RTOL)
        assert gs[4] == os_[4], f"temperature, instance {i}"
    o = oracle.sa_calibrate(mk, chains, lb, ub, n_levels=L, **kw)
    r = plan.sa(chains, lb, ub, n_levels=L - l, level0=l,
                state_in=torch.tensor(o1["state"], device="cuda"), **kw)
    torch.cuda.synchronize()
    ob = _blocks(o["accept"], chains, L, N)
    o_rest = np.concatenate([b[l:].ravel() for b in ob])
    where = first_mismatch(r["accept"].cpu().numpy(), o_rest, L - l, N, chains)
    assert where is None, f"first mismatch at {where}"
    np.testing.assert_allclose(r["best_f"].cpu().numpy(), o["best_f"], rtol=RTOL)
    msg = check_restarts(r["level_best"].cpu().numpy(), o["level_best"][:, l:])
    assert msg is None, msg


def test_state_in_size_is_checked(api, oracle):
    plan = api.Plan(_ragged(oracle))
    lb, ub = I.box(0)
    with pytest.raises(ValueError):
        plan.sa(3, lb, ub, T0=0.05, cool=0.8, n_levels=1, n_steps=2, seed=1, level0=1,
                state_in=torch.zeros(5, dtype=torch.float64, device="cuda"))


@pytest.mark.parametrize("L,N", [(0, 5), (3, 0), (2, 6)])
def test_level0_without_state_and_degenerate_schedules(api, oracle, L, N):
    """A run that starts at level 4 without a state (temperature T0 cool^4,
    the Philox counters of levels 4, 5, ...), also with no level at all (the
    state is the evaluated start) and with levels of no step (restarts and
    cooling only): the oracle's flags and state."""
    mk = _ragged(oracle)
    lb, ub = I.box(0)
    chains = np.array([3, 2, 5, 1, 4], np.int32)
    kw = dict(T0=0.05, cool=0.8, n_levels=L, n_steps=N, seed=37, record=True, level0=4)
    plan = api.Plan(mk)
    g = plan.sa(chains, lb, ub, state_out=True, **kw)
    torch.cuda.synchronize()
    o = oracle.sa_calibrate(mk, chains, lb, ub, keep_state=True, **kw)
    if L * N:
        where = first_mismatch(g["accept"].cpu().numpy(), o["accept"], L, N, chains)
        assert where is None, f"first mismatch at {where}"
    for i, (gs, os_) in enumerate(zip(_state_parts(g["state"].cpu().numpy(), chains, plan.P),
                                      _state_parts(o["state"], chains, plan.P))):
        assert np.array_equal(gs[0], os_[0]) and np.array_equal(gs[2], os_[2]), f"points, {i}"
        np.testing.assert_allclose(gs[1], os_[1], rtol=RTOL)
        np.testing.assert_allclose(gs[3], os_[3], rtol=RTOL)
        assert gs[4] == os_[4], f"temperature, instance {i}"
    np.testing.assert_allclose(g["best_f"].cpu().numpy(), o["best_f"], rtol=RTOL)


def test_resume_under_graph_replay_and_noalloc(api, oracle):
    """The resumed run (state in, state out) replayed from a hipGraph, with
    other eager work between replays, and through sa_calibrate_noalloc gives
    the eager results bit for bit."""
    mk = _ragged(oracle)
    lb, ub = I.box(0)
    chains = np.array([5, 1, 12, 3, 7], np.int32)
    kw = dict(T0=0.05, cool=0.8, n_steps=9, seed=47, record=True, chain_best=True, waves=4)
    plan = api.Plan(mk)
    first = plan.sa(chains, lb, ub, n_levels=2, state_out=True, **kw)
    st = first["state"].clone()
    rkw = dict(kw, n_levels=3, level0=2, state_in=st, state_out=True)
    eager = plan.sa(chains, lb, ub, **rkw)
    torch.cuda.synchronize()
    keys = ("accept", "level_best", "best_x", "best_f", "chain_best_x", "chain_best_f", "state")
    na = plan.sa(chains, lb, ub, noalloc=True, **rkw)
    torch.cuda.synchronize()
    for k in keys:
        assert torch.equal(na[k], eager[k]), f"noalloc: {k}"
    side = torch.cuda.Stream()
    ws, outs = eager["workspace"], None
    pts = torch.tensor(I.random_box_points(0, 64, 5), device="cuda")
    for rep in range(3):
        with torch.cuda.stream(side):
            g = plan.sa(chains, lb, ub, use_graph=True, stream=side, workspace=ws, out=outs,
                        **rkw)
        outs = g
        side.synchronize()
        plan.cost(pts)
        torch.cuda.synchronize()
        for k in keys:
            assert torch.equal(g[k], eager[k]), f"replay {rep}: {k}"
