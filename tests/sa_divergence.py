"""Where two runs of the same annealing part (the GPU's and the oracle's), and
why.

Sec. 3's SA box accepts a proposal iff dE <= 0 or u < exp(-dE / T).  Both
sides draw the same Philox uniforms, so their accept flags agree unless the
two cost evaluations straddle the threshold -T ln u.  At the first differing
flag this module reports the instance, level, step and chain, both dE values,
T and -T ln u, and classifies the mismatch:

* "ulp tie": |dE_gpu - dE_oracle| >= |dE_oracle + T ln u| -- the costs'
  rounding difference alone can move dE across the threshold (or the level-end
  argmin picked chains whose final costs differ by at most 4 ulp);
* "real divergence": otherwise.

Everything here is test infrastructure: the oracle replays the chain from the
start of the level (its own run to that level), and the GPU's dE comes from
the library's cost entry point at the same two points.
"""
import math

import numpy as np

from paper_2408_01470_amd import inputs as I


def first_mismatch(acc_gpu, acc_ora, L, N, chains):
    """(instance, level, step, chain) of the first differing flag, or None.
    Flags are laid out per instance as [L][N][chains[i]] blocks."""
    off = 0
    for i, C in enumerate(np.atleast_1d(chains)):
        C = int(C)
        a = np.asarray(acc_gpu[off:off + L * N * C]).reshape(L, N, C)
        b = np.asarray(acc_ora[off:off + L * N * C]).reshape(L, N, C)
        d = np.argwhere(a != b)
        if len(d):
            lv, s, c = (int(v) for v in d[0])
            return i, lv, s, c
        off += L * N * C
    return None


def gpu_cost_fn(plan):
    """Costs of points of one instance by the library (numpy in, numpy out)."""
    import torch

    def f(pts, inst):
        t = torch.tensor(np.asarray(pts), device="cuda")
        return plan.cost(t, pt_inst=torch.full((len(pts),), inst, dtype=torch.int32,
                                                device="cuda")).cpu().numpy()
    return f


def describe(cost_fn, P, n_inst, oracle, mk, chains, lb, ub, T0s, cool, N, seed, step_frac,
             where):
    """The report of the mismatch at `where` = (instance, level, step, chain);
    cost_fn(points, instance) gives the other side's costs."""
    i, lv, s, c = where
    C = int(np.atleast_1d(chains)[i] if np.ndim(chains) else chains)
    one = I.select_instances(mk, [i])
    lbi = np.broadcast_to(lb, (n_inst, P))[i:i + 1]
    ubi = np.broadcast_to(ub, (n_inst, P))[i:i + 1]
    kw = dict(T0=float(T0s[i]), cool=cool, n_steps=N, seed=seed, step_frac=step_frac,
              inst_key=[i])
    if lv > 0:
        st = oracle.sa_calibrate(one, [C], lbi, ubi, n_levels=lv, keep_state=True, **kw)["state"]
        X, F, _, _, T = oracle.sa_state_split(st, [C], P)[0]
        x, f = X[c], float(F[c])
    else:
        x = 0.5 * (lbi[0] + ubi[0])
        f = float(oracle.cost_batch(one, x[None, :])[0])
        T = float(T0s[i])
    r = oracle.sa_chain_steps(one, 0, c, lv, T, lbi, ubi, x, f, N, seed, step_frac=step_frac,
                              inst_key=[i])
    for k in range(s):
        if r["accept"][k]:
            x, f = r["xp"][k], float(r["fp"][k])
    xp, fp_o, u = r["xp"][s], float(r["fp"][s]), float(r["u"][s])
    f_g, fp_g = (float(v) for v in cost_fn(np.vstack([x, xp]), i))
    dE_o, dE_g = fp_o - f, fp_g - f_g
    thr = -T * math.log(u) if u > 0 else math.inf
    tie = abs(dE_g - dE_o) >= abs(dE_o - thr)
    return (f"first divergence at instance {i}, level {lv}, step {s}, chain {c}: "
            f"dE oracle {dE_o:.17g}, dE gpu {dE_g:.17g}, T {T:.17g}, -T ln u {thr:.17g}, "
            f"oracle accepts {bool(r['accept'][s])}: "
            + ("ulp tie" if tie else "real divergence"))


def check_restarts(lbest_gpu, lbest_ora, final_costs=None):
    """Level-end argmin chains per (instance, level); a differing pair is a
    tie when the two chains' final costs lie within 4 ulp."""
    a = np.asarray(lbest_gpu)
    b = np.asarray(lbest_ora)
    d = np.argwhere(a != b)
    if not len(d):
        return None
    i, lv = (int(v) for v in d[0])
    msg = f"restart chain differs at instance {i}, level {lv}: gpu {a[i, lv]}, oracle {b[i, lv]}"
    if final_costs is not None:
        fa, fb = final_costs
        ulps = abs(fa - fb) / math.ulp(max(abs(fa), abs(fb)))
        msg += f" ({'tie' if ulps <= 4 else 'real divergence'}: {ulps:.1f} ulp apart)"
    return msg
