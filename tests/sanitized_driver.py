"""Driver run under AddressSanitizer and UndefinedBehaviorSanitizer by
test_sanitizers.py (a child process with the sanitizer runtime preloaded).

    python sanitized_driver.py oracle <liboracle.so>
    python sanitized_driver.py host <libsabr_hip.so>

`oracle`: every entry point of the CPU oracle on small problems (the cost of
each model and formula, dual-number gradients, annealing with a resumed
state and a step-by-step chain replay, LM, Nelder-Mead, the Monte Carlo
paths and prices).  `host`: the HIP library's host-side code without a GPU
(plan validation and packing, its queries, the refusals of bad markets and
annealing configurations, the Monte Carlo plan and its host factor).
"""
import ctypes
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

from paper_2408_01470_amd import inputs as I  # noqa: E402


def run_oracle(path):
    from oracle import oracle as O
    O.LIB_PATH = path
    O.lib()
    m, truth, noise = I.caplet_market(M=4, nK=5)
    mv, _, _, ok = O.model_values(m, 0, truth[0])
    assert ok
    mk = I.complete_market(m, mv, noise[:len(mv)])
    pts = I.random_box_points(0, 8, 3)
    O.cost_batch(mk, pts, resid=True)
    O.cost_grad(mk, pts, normal=True)
    lb, ub = I.box(0)
    kw = dict(T0=0.05, cool=0.8, n_steps=5, seed=3)
    r1 = O.sa_calibrate(mk, 6, lb, ub, n_levels=2, record=True, keep_state=True, **kw)
    O.sa_calibrate(mk, 6, lb, ub, n_levels=2, level0=2, state_in=r1["state"], record=True, **kw)
    x = 0.5 * (lb + ub)
    f = float(O.cost_batch(mk, x[None, :])[0])
    O.sa_chain_steps(mk, 0, 1, 0, 0.05, lb[None, :], ub[None, :], x, f, 5, 3)
    O.lm_polish(mk, pts[:2], None, lb, ub, max_iter=3)
    O.nm_polish(mk, pts[:2], np.zeros(2, np.int32), lb, ub, max_iter=20)
    # LMM12 with swaptions, both residual modes
    for resid in (I.RESID_VOL, I.RESID_PRICE):
        m2, t2, n2 = I.lmm_market(M=8, n_cap_K=3, n_exp=3, n_ten=4, n_swp_K=3, residual=resid)
        vm = I.as_vol_market(m2)
        v2, _, _, ok = O.model_values(vm, 0, t2[0])
        assert ok
        mk2 = I.complete_market(m2, v2, n2)
        p2 = np.clip(t2[0][None, :] * np.linspace(0.9, 1.1, 3)[:, None], *I.box(1))
        O.cost_batch(mk2, p2)
        O.cost_grad(mk2, p2, normal=True)
        O.map_params(mk2, 0, p2[0])
    # the per-forward, Mercurio-Morini and Rebonato models
    for gen in (I.perfwd_markets, I.mm_markets, I.reb_markets):
        m3, t3, n3 = gen(n_markets=1, M=4, nK=3)
        v3, _, _, ok = O.model_values(m3, 0, t3[0])
        assert ok
        mk3 = I.complete_market(m3, v3, n3)
        O.cost_batch(mk3, t3[:1])
    # Monte Carlo
    prob = I.mc_problem(M=4, n_cap_K=2, n_swaptions=2)
    O.mc_price(prob, 64, 0.1, 5)
    print("oracle ok", flush=True)


def run_host(path):
    from paper_2408_01470_amd import _lib
    _lib.LIB_PATH = path
    L = _lib.lib()
    from test_abi import _create
    for m in (I.caplet_market()[0], I.lmm_market()[0], I.batch_markets(n_markets=4)[0],
              I.perfwd_markets(n_markets=2)[0], I.mm_markets(n_markets=2)[0],
              I.reb_markets(n_markets=2)[0]):
        rc, h = _create(L, m)
        assert rc == 0, L.sabr_last_error()
        L.sabr_plan_device_bytes(h)
        n = int(m["und_off"][-1])
        S0, A, T = np.zeros(n), np.zeros(n), np.zeros(n)
        f64 = ctypes.POINTER(ctypes.c_double)
        assert L.sabr_plan_underlyings(h, S0.ctypes.data_as(f64), A.ctypes.data_as(f64),
                                       T.ctypes.data_as(f64)) == 0
        L.sabr_plan_destroy(h)
    bad = dict(I.caplet_market()[0])
    bad["q_K"] = bad["q_K"].copy()
    bad["q_K"][3] = -1.0
    rc, _ = _create(L, bad)
    assert rc == -1
    from paper_2408_01470_amd._lib import SAConfig
    m = I.caplet_market()[0]
    rc, h = _create(L, m)
    i32 = ctypes.POINTER(ctypes.c_int32)
    ch = np.array([16], np.int32)
    cfg = SAConfig(1.0, 0.9, 0.05, 10, 10, 1, None, 0, 0, None, 0)
    assert L.sa_workspace_size(h, ctypes.byref(cfg), ch.ctypes.data_as(i32)) > 0
    L.sabr_plan_destroy(h)
    # the Monte Carlo plan and its host-side correlation factor
    from paper_2408_01470_amd import api
    B = api.McProblem(I.mc_problem(M=6, n_cap_K=2, n_swaptions=3)).factor()
    assert np.all(np.isfinite(B))
    print("host ok", flush=True)


if __name__ == "__main__":
    {"oracle": run_oracle, "host": run_host}[sys.argv[1]](sys.argv[2])
