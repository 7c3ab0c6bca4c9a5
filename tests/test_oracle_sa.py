"""Pins of the oracle's simulated annealing and Levenberg-Marquardt polish."""
import math

import numpy as np
import pytest
from scipy import optimize

from paper_2408_01470_amd import inputs as I


def test_paper_eval_count_matches_loop_structure(oracle, c1_market):
    """Sec. 4.1.1: T0 = 10, Tmin = 0.01, rho = 0.99, N = 10, w = 256 x 64 chains
    evaluated the cost 112738304 times.  The do-while loop of the SA box runs
    until T <= Tmin; every chain evaluates x0 once and each step once, and the
    level-end restart copies the best point without re-evaluating it."""
    T, levels = 10.0, 0
    while True:
        levels += 1
        T = 0.99 * T
        if not T > 0.01:
            break
    assert levels == 688
    # the oracle's count for a small run has the same structure C (1 + N L)
    mk, _ = c1_market
    lb, ub = I.box(0)
    r = oracle.sa_calibrate(mk, 7, lb, ub, T0=1.0, cool=0.9, n_levels=3, n_steps=4, seed=2)
    assert r["n_evals"][0] == 7 * (1 + 4 * 3)
    assert 256 * 64 * (1 + 10 * levels) == 112738304


def _minus_one(ctr):
    """numpy's Philox adds one to its 256-bit counter before each block."""
    v = sum(int(w) << (64 * i) for i, w in enumerate(ctr)) - 1
    v %= 1 << 256
    return np.array([(v >> (64 * i)) & ((1 << 64) - 1) for i in range(4)], np.uint64)


def _python_sa_replay(oracle, mk, C, L, N, T0, cool, seed, step_frac, lb, ub):
    """The SA loop written out in Python with numpy's Philox (counter
    pre-incremented by numpy, hence ctr - 1) and the oracle's cost."""
    P = len(lb)
    x0 = 0.5 * (lb + ub)
    X = np.tile(x0, (C, 1))
    F = np.full(C, oracle.cost_batch(mk, x0)[0])
    acc_all = []
    best = []
    T = T0
    for l in range(L):
        for s in range(N):
            flags = []
            for c in range(C):
                u = []
                for b in range((P + 1 + 3) // 4):
                    bg = np.random.Philox(counter=_minus_one([l * N + s, c, b, 0]),
                                          key=np.array([seed, 0], np.uint64))
                    u += [(int(bg.random_raw()) >> 11) * 2.0 ** -53 for _ in range(4)]
                xp = X[c] + step_frac * (ub - lb) * (2 * np.array(u[:P]) - 1)
                xp = np.where(xp > ub, 2 * ub - xp, xp)
                xp = np.where(xp < lb, 2 * lb - xp, xp)
                xp = np.clip(xp, lb, ub)
                fp = oracle.cost_batch(mk, xp)[0]
                dE = fp - F[c]
                a = dE <= 0 or u[P] < math.exp(-dE / T)
                if a:
                    X[c], F[c] = xp, fp
                flags.append(a)
            acc_all.append(flags)
        b = int(np.argmin(F))
        best.append(b)
        X[:] = X[b]
        F[:] = F[b]
        T = cool * T
    return np.array(acc_all, np.uint8).reshape(-1), np.array(best)


def test_sa_loop_replay_with_library_philox(oracle, c1_market):
    mk, _ = c1_market
    lb, ub = I.box(0)
    C, L, N = 3, 3, 4
    acc, best = _python_sa_replay(oracle, mk, C, L, N, 0.05, 0.5, 99, 0.05, lb, ub)
    r = oracle.sa_calibrate(mk, C, lb, ub, T0=0.05, cool=0.5, n_levels=L, n_steps=N, seed=99,
                            record=True)
    assert np.array_equal(r["accept"], acc)
    assert np.array_equal(r["level_best"][0], best)
    assert 0 < acc.sum() < acc.size


def test_sa_deterministic_and_restart_semantics(oracle, c1_market):
    mk, _ = c1_market
    lb, ub = I.box(0)
    kw = dict(T0=0.05, cool=0.8, n_levels=6, n_steps=20, seed=5, record=True)
    a = oracle.sa_calibrate(mk, 16, lb, ub, **kw)
    b = oracle.sa_calibrate(mk, 16, lb, ub, **kw)
    for k in ("best_x", "best_f", "accept", "trace", "chain_best_f"):
        assert np.array_equal(a[k], b[k])
    # best ever is the minimum of the per-chain bests, and the trace is monotone
    assert a["best_f"][0] == a["chain_best_f"].min()
    assert np.all(np.diff(a["trace"][0, :, 0]) <= 0)
    acc = a["accept"].reshape(6, 20, 16)
    np.testing.assert_allclose(acc.mean(axis=(1, 2)), a["trace"][0, :, 1])
    # different seed, different path
    c = oracle.sa_calibrate(mk, 16, lb, ub, **dict(kw, seed=6))
    assert not np.array_equal(a["accept"], c["accept"])


def test_sa_and_lm_beat_brute_force_grid_on_two_parameter_toy(oracle, c1_market):
    """beta and rho fixed at their true values (lb = ub); a 401 x 401 grid over
    (alpha, nu) bounds the global minimum; SA must reach the grid minimum and
    LM from the grid argmin converges to the continuous minimum below it."""
    mk, truth = c1_market
    lb, ub = I.box(0)
    lb, ub = lb.copy(), ub.copy()
    lb[1] = ub[1] = truth[0, 1]
    lb[2] = ub[2] = truth[0, 2]
    al = np.linspace(lb[0], ub[0], 401)
    nu = np.linspace(lb[3], ub[3], 401)
    A, Nn = np.meshgrid(al, nu, indexing="ij")
    pts = np.stack([A.ravel(), np.full(A.size, lb[1]), np.full(A.size, lb[2]), Nn.ravel()], 1)
    cost = oracle.cost_batch(mk, pts)
    gmin = np.nanmin(cost)
    r = oracle.sa_calibrate(mk, 32, lb, ub, T0=0.05, cool=0.9, n_levels=60, n_steps=25, seed=3)
    assert r["best_f"][0] <= gmin * (1 + 1e-6)
    x, f, it = oracle.lm_polish(mk, pts[np.nanargmin(cost)], None, lb, ub)
    assert f[0] <= gmin
    x2, f2, _ = oracle.lm_polish(mk, r["best_x"], None, lb, ub)
    assert f2[0] == pytest.approx(f[0], rel=1e-8)
    np.testing.assert_allclose(x2[0], x[0], rtol=1e-5)


def test_lm_matches_scipy_on_unconstrained_toy(oracle, c1_market):
    """With an inactive box, projected LM is plain LM: it reaches the local
    minimum scipy's MINPACK LM reaches from the same start."""
    mk, truth = c1_market
    lb = np.array([1e-4, 0.0, -0.999, 1e-4])
    ub = np.array([1.0, 1.0, 0.999, 5.0])
    lb[1] = ub[1] = 0.5                      # fix beta, free alpha, rho, nu
    start = truth[0] * np.array([1.3, 1.0, 0.7, 0.8])
    x, f, it = oracle.lm_polish(mk, start, None, lb, ub, max_iter=200, tol=1e-15)

    def resid(q):
        p = np.array([q[0], 0.5, q[1], q[2]])
        _, r = oracle.cost_batch(mk, p, resid=True)
        return r[0]

    sol = optimize.least_squares(resid, start[[0, 2, 3]], method="lm", xtol=1e-15, ftol=1e-15,
                                 gtol=1e-15)
    assert f[0] == pytest.approx(2 * sol.cost, rel=1e-9)
    np.testing.assert_allclose(x[0, [0, 2, 3]], sol.x, rtol=1e-5)


def test_lm_decreases_cost(oracle, c2_market):
    mk, truth = c2_market
    lb, ub = I.box(1)
    start = np.clip(truth[0] * 1.1, lb, ub)
    f0 = oracle.cost_batch(mk, start)[0]
    x, f, it = oracle.lm_polish(mk, start, None, lb, ub, max_iter=15)
    assert f[0] < f0
    assert np.all(x >= lb) and np.all(x <= ub)


def test_level0_sample_matches_full_annealing(oracle, c1_market):
    """The sampled-chain replay of level 0 reproduces sa_calibrate's level 0
    (accept flags, per-chain best-ever cost and point) chain by chain."""
    mk, _ = c1_market
    lb, ub = I.box(0)
    C, N = 40, 12
    full = oracle.sa_calibrate(mk, C, lb, ub, T0=0.05, cool=0.8, n_levels=1, n_steps=N,
                               seed=31, record=True)
    chains = np.array([0, 7, 39, 12], np.int32)
    smp = oracle.sa_level0_sample(mk, C, lb, ub, T0=0.05, n_steps=N, seed=31,
                                  sample_inst=np.zeros(len(chains), np.int32),
                                  sample_chain=chains)
    acc = full["accept"].reshape(N, C)
    for j, c in enumerate(chains):
        assert np.array_equal(smp["accept"][j], acc[:, c])
        assert smp["BF"][j] == full["chain_best_f"][c]
        assert np.array_equal(smp["BX"][j], full["chain_best_x"][c])


def _small_batch(oracle):
    from conftest import complete_with_oracle
    m, truth, noise = I.batch_markets(n_markets=3, M_range=(3, 8), nK_range=(3, 7))
    return complete_with_oracle(oracle, m, truth, noise)


@pytest.mark.parametrize("split", [1, 4, 9])
def test_checkpoint_resume_equals_one_run(oracle, split):
    """L levels in one call equal `split` levels, then the saved state resumed
    for L - split more (the Philox counters and temperatures continue): the
    same accept flags, restart chains, best points and final state, bit for
    bit, on a ragged batch."""
    mk = _small_batch(oracle)
    lb, ub = I.box(0)
    chains = np.array([5, 12, 3], np.int32)
    L, N = 10, 7
    kw = dict(T0=0.05, cool=0.8, n_steps=N, seed=17, record=True)
    full = oracle.sa_calibrate(mk, chains, lb, ub, n_levels=L, keep_state=True, **kw)
    a = oracle.sa_calibrate(mk, chains, lb, ub, n_levels=split, keep_state=True, **kw)
    b = oracle.sa_calibrate(mk, chains, lb, ub, n_levels=L - split, level0=split,
                            state_in=a["state"], keep_state=True, **kw)
    # accept flags: per instance [L][N][C] blocks
    off_f = off_a = off_b = 0
    for C in chains:
        C = int(C)
        fa = full["accept"][off_f:off_f + L * N * C]
        aa = a["accept"][off_a:off_a + split * N * C]
        bb = b["accept"][off_b:off_b + (L - split) * N * C]
        assert np.array_equal(fa, np.concatenate([aa, bb]))
        off_f += L * N * C
        off_a += split * N * C
        off_b += (L - split) * N * C
    assert np.array_equal(full["level_best"], np.hstack([a["level_best"], b["level_best"]]))
    assert np.array_equal(full["best_x"], b["best_x"])
    assert np.array_equal(full["best_f"], b["best_f"])
    assert np.array_equal(full["chain_best_f"], b["chain_best_f"])
    assert np.array_equal(full["state"], b["state"])
    assert np.array_equal(full["n_evals"], a["n_evals"] + b["n_evals"])
    # the state's temperature is the schedule's, by repeated multiplication
    T = 0.05
    for _ in range(L):
        T = 0.8 * T
    for (_, F, _, BF, Ts) in oracle.sa_state_split(full["state"], chains, 4):
        assert Ts == T
        assert np.all(F == F[0])            # every chain restarted at one point
        assert BF.min() <= F[0]          # the restart point was evaluated by some chain


def test_instance_key_runs_one_instance_alone(oracle):
    """An instance of a batch, run alone with its Philox key word and
    temperature, repeats its part of the batch run exactly; with the default
    key (index 0) it draws other numbers."""
    mk = _small_batch(oracle)
    lb, ub = I.box(0)
    chains = np.array([5, 12, 3], np.int32)
    T0s = np.array([0.05, 0.02, 0.08])
    L, N = 4, 9
    kw = dict(T0=1.0, cool=0.8, n_levels=L, n_steps=N, seed=5, record=True)
    full = oracle.sa_calibrate(mk, chains, lb, ub, T0_per_inst=T0s, **kw)
    one = oracle.sa_calibrate(I.select_instances(mk, [1]), [12], lb, ub, T0_per_inst=T0s[1:2],
                              inst_key=[1], **kw)
    o = L * N * 5
    assert np.array_equal(full["accept"][o:o + L * N * 12], one["accept"])
    assert np.array_equal(full["level_best"][1], one["level_best"][0])
    assert np.array_equal(full["best_x"][1], one["best_x"][0])
    other = oracle.sa_calibrate(I.select_instances(mk, [1]), [12], lb, ub,
                                T0_per_inst=T0s[1:2], **kw)
    assert not np.array_equal(other["accept"], one["accept"])


def test_chain_steps_replay_a_level(oracle, c1_market):
    """The step-by-step replay of one chain's level reproduces the accept
    flags of the full annealing, and each flag is the Metropolis rule applied
    to the reported costs and uniform (accept iff dE <= 0 or u < exp(-dE/T))."""
    mk, _ = c1_market
    lb, ub = I.box(0)
    C, N, T0, cool = 6, 15, 0.05, 0.8
    kw = dict(T0=T0, cool=cool, n_steps=N, seed=29, record=True)
    full = oracle.sa_calibrate(mk, C, lb, ub, n_levels=3, **kw)
    st = oracle.sa_calibrate(mk, C, lb, ub, n_levels=2, keep_state=True, **kw)["state"]
    X, F, _, _, T = oracle.sa_state_split(st, [C], 4)[0]
    acc = full["accept"].reshape(3, N, C)
    for c in range(C):
        r = oracle.sa_chain_steps(mk, 0, c, 2, T, lb, ub, X[c], F[c], N, 29)
        assert np.array_equal(r["accept"], acc[2, :, c])
        f = F[c]
        for s in range(N):
            dE = r["fp"][s] - f
            assert bool(r["accept"][s]) == bool(dE <= 0 or r["u"][s] < math.exp(-dE / T))
            if r["accept"][s]:
                f = r["fp"][s]


def test_divergence_report_names_the_planted_step(oracle):
    """The divergence report finds a flag planted into one run's record and
    replays that chain to it: dE, T and -T ln u come from the replay, and with
    identical costs on both sides a flipped flag is a real divergence."""
    from sa_divergence import describe, first_mismatch
    mk = _small_batch(oracle)
    lb, ub = I.box(0)
    chains = np.array([5, 12, 3], np.int32)
    T0s = np.array([0.05, 0.02, 0.08])
    L, N, cool, seed = 4, 9, 0.8, 5
    r = oracle.sa_calibrate(mk, chains, lb, ub, T0=1.0, cool=cool, n_levels=L, n_steps=N,
                            seed=seed, T0_per_inst=T0s, record=True)
    acc = r["accept"].copy()
    where = (1, 2, 4, 7)
    acc[L * N * 5 + (2 * N + 4) * 12 + 7] ^= 1
    assert first_mismatch(acc, r["accept"], L, N, chains) == where

    def ora_cost(pts, inst):
        return oracle.cost_batch(mk, pts, np.full(len(pts), inst, np.int32))
    msg = describe(ora_cost, 4, 3, oracle, mk, chains, lb, ub, T0s, cool, N, seed, 0.05, where)
    assert "instance 1, level 2, step 4, chain 7" in msg
    assert msg.endswith("real divergence")
    T = 0.02 * cool * cool
    assert f"T {T:.17g}" in msg
