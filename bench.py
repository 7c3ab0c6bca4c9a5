#!/usr/bin/env python
"""Benchmark of the MI355X SA calibrator (one JSON line on stdout).

A step is one full calibration of the workload: simulated annealing over all
levels (proposal, parameter map, swaption map, Hagan vol, Black price,
weighted residual reduction, Metropolis, level-end restart).  The default
workload is the joint caplet + swaption LMM12 calibration (985 quotes, 4096
chains, 688 levels x 10 steps).  Throughput is quote-evaluations per second
with the market already resident in HBM.

Also reported: the dominant kernel (the per-level annealing kernel) against
the FP64 vector roofline, timed with HIP events recorded on its own stream,
and the CPU oracle's throughput on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "quote-evals/s + time-to-RMSE (SA vs SA+adjoint polish), 1 MI355X"
FP64_VECTOR_PEAK_TFLOPS = 78.6
EVENT_STRIDE = 8


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c5", choices=["c1", "c2", "c3", "c5"],
                    help="the headline workload (default: the largest, c5)")
    ap.add_argument("--graph", action="store_true",
                    help="time the headline as hipGraph replays")
    ap.add_argument("--no-extra-configs", action="store_true",
                    help="skip c1, c2 and c3 beside the headline")
    ap.add_argument("--levels", type=int, default=None, help="override the level count")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-time-to-rmse", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the cost / adjoint / LM measurement")
    ap.add_argument("--adjoint-config", default="c5", choices=["c2", "c5"])
    ap.add_argument("--no-paper-e2", action="store_true",
                    help="skip the replay of the paper's timed caplet calibration")
    ap.add_argument("--paper-e2-only", action="store_true")
    ap.add_argument("--no-paper-mc", action="store_true",
                    help="skip the replay of the paper's Monte Carlo pricing table")
    ap.add_argument("--paper-mc-only", action="store_true")
    ap.add_argument("--paper-reb-only", action="store_true",
                    help="replay the paper's Rebonato caplet calibration (2.25e9 evaluations)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only the cost / adjoint / LM measurement (one JSON line)")
    ap.add_argument("--waves", type=int, default=None,
                    help="fixed waves per workgroup of the level kernel (skips the autotuner)")
    ap.add_argument("--occupancy", type=int, default=None,
                    help="fixed register budget in waves per SIMD (with --waves)")
    ap.add_argument("--waves-per-chain", type=int, default=1,
                    help="fixed waves per chain (with --waves; > 1 splits each chain's quotes)")
    ap.add_argument("--chains-per-wave", type=int, default=1,
                    help="fixed chains per wave (with --waves; 2 pairs chains in half-waves, "
                         "GLOBAL4 workloads)")
    return ap.parse_args()


def gpu_vols(api, vol_market, truth):
    import torch
    plan = api.Plan(vol_market)
    n = plan.n_inst
    _, mv = plan.cost(torch.tensor(truth, device="cuda"),
                      pt_inst=torch.arange(n, dtype=torch.int32, device="cuda"), model=True)
    mv = mv.cpu().numpy()
    return np.concatenate([mv[i, :plan.nq[i]] for i in range(n)])


def oracle_vols(O, vol_market, truth):
    M = O.Market(vol_market)
    out = []
    for i in range(M.n_inst):
        mv, _, _, ok = O.model_values(M, i, truth[i])
        assert ok
        out.append(mv)
    return np.concatenate(out)


# The oracle's bounded sample per headline workload: (instances from the
# first, levels, chains per instance or None for all) -- about 1e9 quote
# evaluations, 10-20 s on 16 host threads.
CPU_SAMPLE = {"c1": (1, None, None), "c2": (1, 6, None), "c3": (8, 1, None), "c5": (1, 1, None)}


def cpu_baseline(config, levels=None):
    """The oracle, as it stands, on a bounded sample of the same calibration
    (its own copy of the market and schedule): the first levels of the first
    instances, every chain, OpenMP over chains; and on one host thread the
    first level of 64 chains of the first instance."""
    from oracle import oracle as O
    from paper_2408_01470_amd import inputs as I
    from paper_2408_01470_amd import workloads as W

    w = W.CONFIGS[config]()
    if levels is not None:
        w.n_levels = levels
    mk = W.synthesize(w, lambda vm, t: oracle_vols(O, vm, t))
    lb, ub = I.box(w.model)
    pts = W.schedule_points(w.model, w.seed)
    nq = I.n_quotes(mk)
    T0s, cool = [], None
    for i in range(w.n_inst):
        c = O.cost_batch(mk, pts, np.full(len(pts), i, np.int32))
        T0, cool = W.schedule(c, nq[i], w.n_levels)
        T0s.append(T0)
    n_i, n_lv, n_ch = CPU_SAMPLE[config]
    n_lv = w.n_levels if n_lv is None else min(n_lv, w.n_levels)
    C = w.chains if n_ch is None else n_ch
    idx = list(range(n_i))
    sub = I.select_instances(mk, idx)
    threads = int(O.max_threads())
    kw = dict(cool=cool, n_steps=w.n_steps, seed=w.seed, step_frac=w.step_frac, inst_key=idx)
    t = time.perf_counter()
    O.sa_calibrate(sub, C, lb, ub, T0=T0s[0], T0_per_inst=np.array(T0s[:n_i]),
                   n_levels=n_lv, **kw)
    dt = time.perf_counter() - t
    qe = int(np.sum(np.int64(C) * (1 + np.int64(w.n_steps) * n_lv) * nq[:n_i]))
    # one core: the first level of 64 chains of the first instance
    one = I.select_instances(mk, [0])
    c1 = min(64, w.chains)
    O.set_threads(1)
    t = time.perf_counter()
    O.sa_calibrate(one, c1, lb, ub, T0=T0s[0], n_levels=1, cool=cool, n_steps=w.n_steps,
                   seed=w.seed, step_frac=w.step_frac, inst_key=[0])
    dt1 = time.perf_counter() - t
    O.set_threads(threads)
    qe1 = c1 * (1 + w.n_steps) * int(nq[0])
    return dict(value=qe / dt, unit="quote-evals/s", cores=threads, kind="oracle",
                sample=f"{w.name.split(':')[0]}: the first {n_lv} of {w.n_levels} levels of the "
                       f"first {n_i} of {w.n_inst} instances, {C} chains each, the headline's "
                       f"market and schedule ({qe:.3e} quote-evals, {dt:.1f} s, OpenMP over "
                       "chains)",
                single_core={"value": qe1 / dt1, "sample": f"first level, {c1} chains of the "
                                                          f"first instance ({qe1:.3e} "
                                                          f"quote-evals, {dt1:.1f} s)"},
                host_cpu=host_cpu())


def host_cpu():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cost_and_adjoint(api, W, I, config="c5"):
    """sabr_cost_batch, sabr_cost_vjp and sabr_lm_polish on an LMM12 workload
    (default c5, 64 markets x 8838 quotes): cost and gradient of `chains`
    points per market near its true parameters, then LM on 128 such points
    per market.  Rates are n_pts x Q per second (device time, HIP events)."""
    import torch
    w = W.CONFIGS[config]()
    mk = W.synthesize(w, lambda vm, t: gpu_vols(api, vm, t))
    plan = api.Plan(mk)
    lb, ub = I.box(w.model)
    Q = int(I.n_quotes(mk)[0])
    per = w.chains
    g = np.random.default_rng(I.SEED_BASE + 5001)
    pts = np.clip(np.repeat(w.truth, per, axis=0) * g.uniform(0.95, 1.05, (w.n_inst * per, 12)),
                  lb, ub)
    inst = np.repeat(np.arange(w.n_inst, dtype=np.int32), per)
    P = torch.tensor(pts, device="cuda")
    pi = torch.tensor(inst, device="cuda")
    s = torch.cuda.current_stream()

    def timed(fn):
        fn()                                  # warm-up (first-call costs)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        r = fn()
        e1.record(s)
        torch.cuda.synchronize()
        return r, e0.elapsed_time(e1) / 1e3

    n = len(pts)
    c, t_cost = timed(lambda: plan.cost(P, pt_inst=pi))
    o, t_vjp = timed(lambda: plan.vjp(P, pt_inst=pi))
    k = 128
    sel = np.concatenate([np.arange(i * per, i * per + k) for i in range(w.n_inst)])
    X0 = P[torch.tensor(sel, device="cuda")].contiguous()
    I0 = pi[torch.tensor(sel, device="cuda")].contiguous()
    (x, f, it), t_lm = timed(lambda: plan.lm(X0, lb, ub, pt_inst=I0, max_iter=50))
    f0 = c[torch.tensor(sel, device="cuda")].cpu().numpy()
    f = f.cpu().numpy()
    it = it.cpu().numpy()
    return {
        "workload": w.name.split(",")[0],
        "cost_batch": {"points": n, "s": t_cost, "quote_evals_per_s": n * Q / t_cost},
        "cost_vjp": {"points": n, "s": t_vjp, "quote_evals_per_s": n * Q / t_vjp,
                     "finite_gradients": int(np.isfinite(o["grad"].cpu().numpy()).all(axis=1).sum())},
        "lm_polish": {"points": len(sel), "max_iter": 50, "s": t_lm,
                      "iterations_mean": float(it.mean()), "iterations_max": int(it.max()),
                      "median_cost_ratio": float(np.median(f / f0))},
    }


def measured_traffic(config, shape):
    """HBM bytes per launch of the level kernel from the committed counter
    records (FETCH_SIZE and WRITE_SIZE passes scaled by a copy kernel's
    readings; one record per launch shape), or None when there is no record
    for this workload and launch shape or the kernel sources changed since
    the counters were taken."""
    from paper_2408_01470_amd import build
    path = os.path.join(ROOT, "profiles", f"sa_level_kernel_{config}_counters.md")
    try:
        text = open(path).read()
        recs = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, IndexError, ValueError):
        return None
    digest = build.source_digest()
    for rec in (recs if isinstance(recs, list) else [recs]):
        if (rec.get("source_sha256") == digest
                and rec.get("waves_per_group") == shape.get("waves_per_group")
                and rec.get("occupancy") == shape.get("occupancy")
                and rec.get("waves_per_chain", 1) == shape.get("waves_per_chain", 1)
                and rec.get("chains_per_wave", 1) == shape.get("chains_per_wave", 1)):
            return float(rec["traffic_bytes_per_launch"])
    return None


def time_to_rmse(api, W, I, autotune):
    """Config c4: SA (512 chains, 50 levels x 100 steps) then LM polish of the
    64 best chain points (the hybrid), against plain SA (same chains) run for
    up to 4 x 200 levels.  Times are device times (HIP events; plain SA's
    from its level trace: the first level whose best-ever RMSE reaches the
    target).

    * the ratio at the plain run's own final RMSE R_plain: t_plain = when the
      plain run first reaches R_plain, t_hybrid = when the hybrid does (the
      first level of its SA part, else the end of its polish);
    * the ratios at (1 + 1e-2) R* and (1 + 1e-3) R*, R* the RMSE of the
      polished optimum: t_hybrid = the end of the polish; where the plain run
      never gets there the ratio is a lower bound (its full time);
    * plain SA's best-ever RMSE against time (every 20th level)."""
    import torch
    w = W.config4()
    mk = W.synthesize(w, lambda vm, t: gpu_vols(api, vm, t))
    plan = api.Plan(mk)
    lb, ub = I.box(w.model)
    Q = int(I.n_quotes(mk)[0])
    c = plan.cost(torch.tensor(W.schedule_points(w.model, w.seed), device="cuda")).cpu().numpy()
    T0, cool_h = W.schedule(c, Q, w.n_levels)
    L_plain = 4 * 200
    _, cool_p = W.schedule(c, Q, L_plain)
    shape = {}
    if autotune:
        from paper_2408_01470_amd import autotune as AT
        t = AT.tune(plan, w.chains, lb, ub, w.n_steps,
                    candidates=AT.CANDIDATES + AT.split_candidates(plan, w.chains) +
                    AT.pair_candidates(plan, w.chains))
        shape = dict(waves=t["waves"], occupancy=t["occupancy"],
                     waves_per_chain=t["waves_per_chain"], chains_per_wave=t["chains_per_wave"])
    kw = dict(T0=T0, n_steps=w.n_steps, seed=w.seed, step_frac=w.step_frac, **shape)
    k = w.extra["polish"]

    def hybrid():
        r = plan.sa(w.chains, lb, ub, cool=cool_h, n_levels=w.n_levels, chain_best=True, **kw)
        idx = torch.topk(-r["chain_best_f"], k).indices
        return r, plan.lm(r["chain_best_x"][idx], lb, ub, max_iter=50)

    hybrid()                    # warm-up: first-call costs stay out of the timing
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    e0.record(s)
    r = plan.sa(w.chains, lb, ub, cool=cool_h, n_levels=w.n_levels, chain_best=True, **kw)
    e1.record(s)
    idx = torch.topk(-r["chain_best_f"], k).indices
    x, f, it = plan.lm(r["chain_best_x"][idx], lb, ub, max_iter=50)
    e2.record(s)
    torch.cuda.synchronize()
    t_sa = e0.elapsed_time(e1) / 1e3
    t_hyb = e0.elapsed_time(e2) / 1e3
    tr_h = r["trace"].cpu().numpy()[0]
    rmse_h = np.sqrt(tr_h[:, 0] / Q)
    # the hybrid's level-trace clock starts at its own initial evaluation
    f_opt = float(f.min())
    rmse_opt = np.sqrt(f_opt / Q)
    rp = plan.sa(w.chains, lb, ub, cool=cool_p, n_levels=L_plain, **kw)
    torch.cuda.synchronize()
    tr = rp["trace"].cpu().numpy()[0]
    rmse_p = np.sqrt(tr[:, 0] / Q)
    t_lv = tr[:, 2] / 1e9

    def plain_time(target):
        hit = np.nonzero(rmse_p <= target)[0]
        return (float(t_lv[hit[0]]), True) if len(hit) else (float(t_lv[-1]), False)

    ratios = {}
    for tag, target in (("1e-2", (1 + 1e-2) * rmse_opt), ("1e-3", (1 + 1e-3) * rmse_opt)):
        tp, reached = plain_time(target)
        ratios[tag] = {"rmse_target": target, "t_plain_s": tp, "plain_reached": reached,
                       "t_hybrid_s": t_hyb, "speedup": tp / t_hyb,
                       "speedup_is_lower_bound": not reached}
    R_plain = float(rmse_p[-1])
    tp, _ = plain_time(R_plain)
    hit_h = np.nonzero(rmse_h <= R_plain)[0]
    th = float(tr_h[hit_h[0], 2] / 1e9) if len(hit_h) else t_hyb
    assert rmse_opt <= R_plain or len(hit_h), "the hybrid never reaches plain SA's RMSE"
    curve = [[round(float(t_lv[l]), 6), float(rmse_p[l])] for l in range(0, L_plain, 20)]
    return {
        "workload": w.name,
        "rmse_sa_plus_lm": rmse_opt,
        "rmse_sa_before_polish": float(np.sqrt(r["best_f"].item() / Q)),
        "rmse_plain_sa_final": R_plain,
        "t_sa_plus_lm_s": t_hyb,
        "t_sa_part_s": t_sa,
        "lm_iterations_max": int(it.max()),
        "at_plain_final_rmse": {"rmse": R_plain, "t_plain_s": tp, "t_hybrid_s": th,
                                "speedup": tp / th},
        "at_polished_rmse": ratios,
        "plain_rmse_vs_time": curve,
        "speedup": tp / th,
        "launch_shape": shape,
    }


NM_ITERS = 20000


def paper_e2(api, W, I, flops, autotune, shape=None, which="e2"):
    """The paper's own timed caplet calibrations on its printed EURIBOR data
    (Sec. 4.1.1 and 4.2.1), eq. (sigmaHagan), SA with T0 = 10, Tmin = 0.01,
    rho = 0.99 (688 levels), N = 10, 16384 chains (112,738,304 cost
    evaluations).  which = "e2": the per-forward Hagan model (PERFWD, P = 39),
    then LM on each forward as a GLOBAL4 instance with beta frozen at 0.5.
    which = "mm": the Mercurio-Morini model (P = 27).  Both are also polished
    the paper's way, by Nelder-Mead on the whole point (sabr_nm_polish, at
    most NM_ITERS iterations).  Device time of the annealing (HIP events) and
    wall time of each polish including its host-side re-layout; MRE = mean
    |sigma_model - sigma_market| / sigma_market over the 117 quotes."""
    import torch
    w = {"e2": W.paper_e2, "mm": W.paper_mm, "reb": W.paper_reb}[which]()
    mk = w.market
    plan = api.Plan(mk)
    tuning = None
    n_fwd = int(mk["fwd_off"][1])
    lb, ub = I.box(int(mk["model"]), n_fwd)
    kw = dict(T0=w.extra["T0"], cool=w.extra["cool"], n_levels=w.n_levels, n_steps=w.n_steps,
              seed=w.seed, step_frac=w.step_frac)
    if shape is None:
        shape = {}
        if autotune:
            from paper_2408_01470_amd import autotune as AT
            t = AT.tune(plan, w.chains, lb, ub, w.n_steps)
            shape = dict(waves=t["waves"], occupancy=t["occupancy"])
            tuning = [[d["waves"], d["occupancy"], round(d["level_ms"], 4)] for d in t["all"]]
    g4 = I.perfwd_as_global4(mk) if which == "e2" else None
    plan4 = api.Plan(g4) if which == "e2" else None
    beta = float(mk["beta"])
    lb4 = np.tile([lb[0], beta, lb[1], lb[2]], (n_fwd, 1))
    ub4 = np.tile([ub[0], beta, ub[1], ub[2]], (n_fwd, 1))
    inst4 = torch.arange(n_fwd, dtype=torch.int32, device="cuda")
    vol = np.asarray(mk["q_vol"])

    def nm(x):
        y, f, it = plan.nm(torch.tensor(x[None, :], device="cuda"), lb, ub, max_iter=NM_ITERS,
                           tol=1e-12)
        return y.cpu().numpy()[0], it.cpu().numpy()

    def polish(x):
        if which != "e2":
            return x, np.zeros(1, np.int32)
        starts = torch.tensor(I.perfwd_points_as_global4(x, beta), device="cuda")
        y, f4, it = plan4.lm(starts, lb4, ub4, pt_inst=inst4, max_iter=100)
        return I.global4_points_as_perfwd(y.cpu().numpy()), it.cpu().numpy()

    def mre(x):
        _, mv = plan.cost(torch.tensor(x[None, :], device="cuda"), model=True)
        mv = mv.cpu().numpy()[0, :len(vol)]
        return float(np.mean(np.abs(mv - vol) / vol))

    warm = dict(kw, n_levels=2) if which == "reb" else kw   # the long replay warms on 2 levels
    r = plan.sa(w.chains, lb, ub, trace=False, **shape, **warm)        # warm-up
    polish(r["best_x"].cpu().numpy()[0])
    nm(r["best_x"].cpu().numpy()[0])
    ws = r["workspace"]
    L = w.n_levels
    sampled = list(range(0, L, EVENT_STRIDE))
    s = torch.cuda.current_stream()
    evs = [None] * (2 * L)
    for l in sampled:
        evs[2 * l] = torch.cuda.Event(enable_timing=True)
        evs[2 * l + 1] = torch.cuda.Event(enable_timing=True)
        evs[2 * l].record(s)
        evs[2 * l + 1].record(s)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    r = plan.sa(w.chains, lb, ub, trace=False, workspace=ws, level_events=evs, **shape, **kw)
    e1.record(s)
    torch.cuda.synchronize()
    t_sa = e0.elapsed_time(e1) / 1e3
    x_sa = r["best_x"].cpu().numpy()[0]
    t0 = time.perf_counter()
    x_pol, it = polish(x_sa)
    t_pol = time.perf_counter() - t0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x_nm, it_nm = nm(x_sa)
    t_nm = time.perf_counter() - t0
    lvl_ms = np.array([evs[2 * l].elapsed_time(evs[2 * l + 1]) for l in sampled])
    flop_launch = flops.level_launch_flops(mk, w.chains, w.n_steps)
    achieved = flop_launch / (float(lvl_ms.mean()) / 1e3) / 1e12
    evals = w.chains * (1 + w.n_steps * L)
    if which == "e2":
        t = x_pol.reshape(-1, 3)
        params = {"alpha": t[:, 0].round(5).tolist(), "phi": t[:, 1].round(4).tolist(),
                  "sigma": t[:, 2].round(4).tolist()}
    else:
        params = None
    out = {
        "workload": w.name,
        "cost_evaluations": evals,
        "quote_evals": w.quote_evals(),
        "t_sa_s": t_sa,
        "cost_evals_per_s": evals / t_sa,
        "quote_evals_per_s": w.quote_evals() / t_sa,
        "level_kernel_avg_ms": float(lvl_ms.mean()),
        "level_kernel_fp64_frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
        "mre_sa": mre(x_sa),
        "cost_sa": float(r["best_f"].item()),
        "launch_shape": shape,
        "tuning_level_ms": tuning,
        "paper": {"t_sa_s": w.extra["paper_sa_s"],
                  "t_nelder_mead_s": w.extra.get("paper_nm_s"),
                  "t_total_s": w.extra.get("paper_total_s"),
                  "cost_evaluations": w.extra["paper_evals"], "mre": w.extra["paper_mre"],
                  "hardware": ("two GTX 470" if which == "reb" else "one GTX 470")
                  + " (context, not a target)"},
    }
    out.update({"t_nelder_mead_s": t_nm, "nelder_mead_iterations": int(it_nm[0]),
                "mre_nelder_mead": mre(x_nm)})
    if which == "e2":
        out.update({"t_polish_s": t_pol, "polish_lm_iterations_max": int(it.max()),
                    "mre_polished": mre(x_pol), "params_polished": params})
    elif which == "mm":
        t = x_nm[:-1].reshape(-1, 2)
        out["params_nelder_mead"] = {"alpha": t[:, 0].round(5).tolist(),
                                     "phi": t[:, 1].round(4).tolist(),
                                     "sigma": round(float(x_nm[-1]), 4)}
    else:
        t = x_nm[:-8].reshape(-1, 2)
        out["params_nelder_mead"] = {"kappa": t[:, 0].round(5).tolist(),
                                     "phi": t[:, 1].round(4).tolist(),
                                     "g_abcd": x_nm[-8:-4].round(4).tolist(),
                                     "h_abcd": x_nm[-4:].round(4).tolist()}
    return out


# Table (haganMCpricer): caplet pricing by Monte Carlo in the Hagan model,
# (paths, dt, CPU s, GPU s) on an Intel E5620 and one GTX 470 (single
# precision; context, not a target).
PAPER_MC_TABLE = [
    (10**3, 1e-1, 0.558, 0.094), (10**3, 1e-2, 5.580, 0.222), (10**3, 1e-3, 55.956, 1.406),
    (10**4, 1e-1, 5.572, 0.119), (10**4, 1e-2, 55.740, 0.390), (10**4, 1e-3, 557.698, 3.081),
    (10**5, 1e-1, 55.692, 0.323), (10**5, 1e-2, 558.331, 2.886), (10**5, 1e-3, 5601.292, 28.550),
    (10**6, 1e-1, 557.696, 2.375), (10**6, 1e-2, 5588.070, 27.950),
    (10**6, 1e-3, 55904.184, 283.970),
]


def paper_mc(api, I, flops, cpu=True):
    """Replay of the paper's Monte Carlo pricing table: the 117 caplets of its
    EURIBOR market (13 forwards, fixings to 6.5 years) under the Hagan model
    at its printed calibration (phi_ii, sigma_i, alpha_i, beta = 0.5) and
    swaption correlations, every (paths, dt) cell of the table, FP64.  Device
    time of sabr_mc_price (HIP events on the launch stream; the plan is
    resident); path-steps/s; the level of the largest cell against the 78.6
    TFLOP/s FP64 peak (algorithmic FLOP of flops.mc_launch_flops); the mean
    absolute error of the 1e6-path prices against the market's Black prices
    (caplet price = P(0, pay) tau Black(F, K, T, vol), in % of notional as the
    paper prints it); the paper's fourteen swaptions x five strikes at the same
    parameters against its printed market and Monte Carlo prices; and, with
    cpu, the oracle on a bounded sample."""
    import torch
    from scipy.stats import norm
    prob = I.paper_mc_problem()
    plan = api.McPlan(prob)
    stream = torch.cuda.current_stream()
    seed = 2408
    plan.price(1000, 0.1, seed)
    torch.cuda.synchronize()
    cells = []
    big = None
    for n, dt, cpu_s, gpu_s in PAPER_MC_TABLE:
        reps = 3 if n * (0.1 / dt) <= 10**6 else 1
        ms = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            price, se = plan.price(n, dt, seed)
            e1.record(stream)
            e1.synchronize()
            ms.append(e0.elapsed_time(e1))
        t = min(ms) / 1e3
        steps = flops.mc_path_steps(prob, n, dt)
        cells.append({"paths": n, "dt": dt, "s": t, "path_steps_per_s": steps / t,
                      "paper_gpu_s": gpu_s, "paper_cpu_s": cpu_s,
                      "speedup_vs_paper_gpu": gpu_s / t})
        if n == 10**6 and dt == 1e-3:
            big = (t, price.cpu().numpy(), se.cpu().numpy())
    t, price, se = big
    fl = flops.mc_launch_flops(prob, 10**6, 1e-3)
    # market prices from the smiles table's vols
    mk = I.paper_caplet_market()
    a = prob["opt_a"]
    F, T, tau, K = prob["F0"][a], prob["T"][a], prob["tau"][a], prob["opt_K"]
    pay = mk["fwd_P"][a]
    vol = mk["q_vol"]
    sd = vol * np.sqrt(T)
    d1 = (np.log(F / K) + 0.5 * sd * sd) / sd
    mkt = pay * tau * (F * norm.cdf(d1) - K * norm.cdf(d1 - sd))
    out = {
        "workload": "the paper's Monte Carlo caplet pricing: 117 caplets, 13 EURIBOR forwards, "
                    "Hagan model at the printed calibration, spot measure, FP64",
        "cells": cells,
        "largest_cell": {"paths": 10**6, "dt": 1e-3, "s": t,
                         "tflops": fl / t / 1e12, "fp64_frac": fl / t / 78.6e12,
                         "flop": fl},
        "mae_vs_market_pct": float(np.mean(np.abs(price - mkt)) * 100.0),
        "max_stderr_pct": float(se.max() * 100.0),
        "paper": {"mae_mc_pct": 4.08e-2, "mae_formula_pct": 4.14e-2,
                  "hardware": "one GTX 470, single precision (context, not a target)"},
    }
    # the paper's fourteen swaptions x five strikes at the same parameters
    sprob, printed = I.paper_mc_swaption_problem()
    splan = api.McPlan(sprob)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    sp, sse = splan.price(10**6, 1e-3, seed)
    e1.record(stream)
    e1.synchronize()
    sp = 100.0 * sp.cpu().numpy()
    out["swaptions"] = {
        "cells": int(len(sp)), "paths": 10**6, "dt": 1e-3, "s": e0.elapsed_time(e1) / 1e3,
        "mean_rel_dev_vs_paper_mc": float(np.mean(sp / printed[:, 1] - 1.0)),
        "max_abs_rel_dev_vs_paper_mc": float(np.max(np.abs(sp / printed[:, 1] - 1.0))),
        "mae_vs_market_pct": float(np.mean(np.abs(sp - printed[:, 0]))),
        "paper_mae_vs_market_pct_these_cells": float(np.mean(np.abs(printed[:, 1] - printed[:, 0]))),
        "paper_mae_all_swaptions_pct": 6.19e-2,
    }
    if cpu:
        from oracle import oracle as O
        n_cpu, dt_cpu = 2000, 1e-2
        t0 = time.perf_counter()
        O.mc_paths(prob, n_cpu, dt_cpu, seed)
        tc = time.perf_counter() - t0
        out["cpu_oracle"] = {"paths": n_cpu, "dt": dt_cpu, "s": tc,
                             "path_steps_per_s": flops.mc_path_steps(prob, n_cpu, dt_cpu) / tc,
                             "threads": int(O.max_threads()), "kind": "oracle"}
    return out


# launch shapes the tuner tries per workload (waves per workgroup, waves per
# SIMD); the large LMM12 batch keeps to the shapes its LDS and registers allow
TUNE_CANDIDATES = {"c5": ((8, 3), (8, 4), (4, 3), (4, 4))}


def measure_sa(api, W, I, flops, config, steps, warmup, autotune=True, fixed_shape=None,
               levels=None, use_graph=False):
    """One workload's calibration, timed: `steps` whole calibrations after
    `warmup` untimed ones, with the market resident in HBM.  Eager launches
    carry HIP events around every EVENT_STRIDE-th level kernel (the roofline
    of the dominant kernel); with use_graph the timed calibrations are
    hipGraph replays on a side stream, and one eager calibration after them
    supplies the per-launch kernel time."""
    import torch
    w = W.CONFIGS[config]()
    if levels is not None:
        w.n_levels = levels
    mk = W.synthesize(w, lambda vm, t: gpu_vols(api, vm, t))
    plan = api.Plan(mk)
    lb, ub = I.box(w.model)
    nq = I.n_quotes(mk)
    pts = torch.tensor(W.schedule_points(w.model, w.seed), device="cuda")
    T0s, cool = [], None
    for i in range(w.n_inst):
        c = plan.cost(pts, pt_inst=torch.full((len(pts),), i, dtype=torch.int32,
                                              device="cuda")).cpu().numpy()
        T0, cool = W.schedule(c, nq[i], w.n_levels)
        T0s.append(T0)
    T0s = np.array(T0s)
    kw = dict(T0=T0s[0], cool=cool, n_levels=w.n_levels, n_steps=w.n_steps, seed=w.seed,
              step_frac=w.step_frac, T0_per_inst=T0s, trace=True)
    tuned = None
    if fixed_shape is not None:
        kw.update(waves=fixed_shape["waves"], occupancy=fixed_shape["occupancy"],
                  waves_per_chain=fixed_shape.get("waves_per_chain", 1),
                  chains_per_wave=fixed_shape.get("chains_per_wave", 1))
    elif autotune:
        from paper_2408_01470_amd import autotune as AT
        cand = TUNE_CANDIDATES.get(config, AT.CANDIDATES + AT.split_candidates(plan, w.chains) +
                                   AT.pair_candidates(plan, w.chains))
        tuned = AT.tune(plan, w.chains, lb, ub, w.n_steps, levels=3 if config == "c5" else 4,
                        candidates=cand)
        kw.update(waves=tuned["waves"], occupancy=tuned["occupancy"],
                  waves_per_chain=tuned["waves_per_chain"],
                  chains_per_wave=tuned["chains_per_wave"])
    L = w.n_levels
    sampled = list(range(0, L, EVENT_STRIDE))

    def level_events(stream):
        evs = [None] * (2 * L)
        for l in sampled:
            evs[2 * l] = torch.cuda.Event(enable_timing=True)
            evs[2 * l + 1] = torch.cuda.Event(enable_timing=True)
            evs[2 * l].record(stream)       # create the HIP events on this stream
            evs[2 * l + 1].record(stream)
        return evs

    stream = torch.cuda.Stream() if use_graph else torch.cuda.current_stream()
    ws, outs = None, None
    with torch.cuda.stream(stream):
        for _ in range(warmup):
            r = plan.sa(w.chains, lb, ub, workspace=ws, out=outs, use_graph=use_graph,
                        stream=stream, **kw)
            ws = r["workspace"]
            outs = r if use_graph else None
        events = [None if use_graph else level_events(stream) for _ in range(steps)]
        torch.cuda.synchronize()
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        start.record(stream)
        results = []
        for k in range(steps):
            r = plan.sa(w.chains, lb, ub, workspace=ws, out=outs, level_events=events[k],
                        use_graph=use_graph, stream=stream, **kw)
            ws = r["workspace"]
            outs = r if use_graph else None
            results.append(r)
        end.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        if use_graph:     # one eager calibration for the per-launch kernel time
            events = [level_events(stream)]
            plan.sa(w.chains, lb, ub, workspace=ws, level_events=events[0], stream=stream, **kw)
            torch.cuda.synchronize()
    ms_per_step = start.elapsed_time(end) / steps
    qe = w.quote_evals()
    lvl_ms = np.array([[evs[2 * l].elapsed_time(evs[2 * l + 1]) for l in sampled]
                       for evs in events])
    avg_launch_s = float(lvl_ms.mean()) / 1e3
    flop_launch = flops.level_launch_flops(mk, w.chains, w.n_steps)
    achieved = flop_launch / avg_launch_s / 1e12
    best_f = results[-1]["best_f"].cpu().numpy()
    shape = {"waves_per_group": kw.get("waves", 0), "occupancy": kw.get("occupancy", 0),
             "waves_per_chain": max(1, kw.get("waves_per_chain", 1)),
             "chains_per_wave": max(1, kw.get("chains_per_wave", 1))}
    return {
        "workload": w.name,
        "value": qe / (ms_per_step / 1e3),
        "unit": "quote-evals/s",
        "ms_per_step": ms_per_step,
        "steps": steps,
        "launch": "hipGraph replay" if use_graph else "eager",
        "config": {
            "workload": w.name,
            "instances": int(w.n_inst),
            "quotes_per_instance": int(nq.max()),
            "quotes_total": int(nq.sum()),
            "chains_per_instance": int(w.chains),
            "levels": int(w.n_levels),
            "steps_per_level": int(w.n_steps),
            "quote_evals_per_step": qe,
        },
        "roofline": {
            "bound": "alu",
            "kernel": "sa_level_kernel",
            "achieved": achieved,
            "peak": FP64_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
            "traffic": measured_traffic(config, shape),
            "flop_per_launch": flop_launch,
            "avg_launch_ms": avg_launch_s * 1e3,
            "launches_timed": int(lvl_ms.size),
        },
        "calibration": {"rmse_best": float(np.sqrt(best_f / nq).max()),
                        "wall_s_per_step": wall / steps},
        "launch_shape": dict(shape, autotuned=tuned is not None),
        "_market": mk,
    }


# the other workloads reported beside the headline: (config, timed steps,
# level count override, graph replay)
EXTRA_SA = (("c1", 3, None, False), ("c2", 3, None, False), ("c3", 2, 20, True))


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the "
              "sharding of chains, markets and paths across GPUs is designed, not built",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2408_01470_amd import api, flops
    from paper_2408_01470_amd import inputs as I
    from paper_2408_01470_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.adjoint_only:
        print(json.dumps(cost_and_adjoint(api, W, I, args.adjoint_config)))
        return
    fixed_shape = (dict(waves=args.waves, occupancy=args.occupancy or 1,
                        waves_per_chain=args.waves_per_chain,
                        chains_per_wave=args.chains_per_wave)
                   if args.waves is not None else None)
    if args.paper_e2_only:
        print(json.dumps(paper_e2(api, W, I, flops, not args.no_autotune, fixed_shape)))
        print(json.dumps(paper_e2(api, W, I, flops, not args.no_autotune, fixed_shape, "mm")))
        return
    if args.paper_mc_only:
        print(json.dumps(paper_mc(api, I, flops, not args.no_cpu_baseline)))
        return
    if args.paper_reb_only:
        print(json.dumps(paper_e2(api, W, I, flops, not args.no_autotune, fixed_shape, "reb")))
        return
    head = measure_sa(api, W, I, flops, args.config, args.steps, args.warmup,
                      not args.no_autotune, fixed_shape, args.levels, args.graph)
    mk = head.pop("_market")
    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "quote-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": head["config"],
        "roofline": head["roofline"],
        "calibration": head["calibration"],
        "launch_shape": head["launch_shape"],
        "launch": head["launch"],
    }
    if not args.no_extra_configs:
        out["other_workloads"] = {}
        for cfg, steps, levels, graph in EXTRA_SA:
            if cfg == args.config:
                continue
            r = measure_sa(api, W, I, flops, cfg, steps, 1, not args.no_autotune, None, levels,
                           graph)
            r.pop("_market")
            out["other_workloads"][cfg] = r
    if not args.no_time_to_rmse:
        out["time_to_rmse"] = time_to_rmse(api, W, I, not args.no_autotune)
    if not args.no_adjoint:
        out["cost_and_adjoint"] = cost_and_adjoint(api, W, I, args.adjoint_config)
    if not args.no_paper_e2:
        out["paper_e2"] = paper_e2(api, W, I, flops, not args.no_autotune, fixed_shape)
        out["paper_mm"] = paper_e2(api, W, I, flops, not args.no_autotune, fixed_shape, "mm")
    if not args.no_paper_mc:
        out["paper_mc"] = paper_mc(api, I, flops, not args.no_cpu_baseline)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.config, args.levels)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
