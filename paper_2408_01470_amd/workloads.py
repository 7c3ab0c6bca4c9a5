"""Benchmark workloads: synthetic markets shaped like the paper's caplet and
swaption calibrations (Sec. 4: semiannual forwards, 9-point moneyness smiles
over -80%..80%, swap smiles by expiry and tenor), at the sizes of the five
benchmark configurations, plus the annealing settings of each.

Market quotes are model vols at the true parameters plus N(0, 0.002) noise;
the model vols come from whichever implementation the caller passes
(``vols_fn``), so the GPU path and the CPU oracle each synthesise their own
copy of the same market.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import inputs as I

SIGMA_NOISE = 0.002


@dataclass
class Workload:
    name: str
    market: dict                 # structure (q_vol placeholder until synthesised)
    truth: np.ndarray            # [n_inst, P] (None for the paper's market data)
    noise: np.ndarray            # [total quotes] (None for the paper's market data)
    chains: int
    n_levels: int
    n_steps: int
    seed: int
    step_frac: float = 0.05
    extra: dict = field(default_factory=dict)

    @property
    def model(self):
        return int(self.market["model"])

    @property
    def n_inst(self):
        return I.n_inst(self.market)

    def quote_evals(self, n_levels=None, chains=None):
        """Quote evaluations of one calibration: sum_i C (1 + N L) Q_i."""
        L = self.n_levels if n_levels is None else n_levels
        C = self.chains if chains is None else chains
        q = I.n_quotes(self.market).astype(np.int64)
        return int(np.sum(np.int64(C) * (1 + np.int64(self.n_steps) * L) * q))


def config1():
    """Plain caplet calibration: 10 forwards x 11 strikes, GLOBAL4, 64 chains,
    200 levels x 100 steps."""
    m, truth, noise = I.caplet_market(seed=I.SEED_BASE + 1000)
    return Workload("c1: caplets 10x11, GLOBAL4, 64 chains, L=200, N=100", m, truth, noise,
                    chains=64, n_levels=200, n_steps=100, seed=1)


def config2():
    """Joint caplet + swaption calibration: 20 forwards, 19 x 15 caplets and a
    10 x 10 swaption grid x 7 strikes (985 quotes), LMM12, Black-price residuals
    with vega weights, 4096 chains, the paper's 688 levels (T0 = 10, Tmin =
    0.01, rho = 0.99) of N = 10 steps."""
    m, truth, noise = I.lmm_market(seed=I.SEED_BASE + 2000, M=20, n_cap_K=15, n_exp=10,
                                   n_ten=10, n_swp_K=7, residual=I.RESID_PRICE)
    return Workload("c2: LMM12 caplets 19x15 + swaptions 10x10x7 (985 quotes), 4096 chains, "
                    "L=688, N=10, price residuals", m, truth, noise,
                    chains=4096, n_levels=688, n_steps=10, seed=2)


def config3(n_markets=256):
    """256 caplet markets of uneven size (10..40 forwards x 5..15 strikes),
    1024 chains each."""
    m, truth, noise = I.batch_markets(n_markets=n_markets, seed=I.SEED_BASE + 3000)
    return Workload(f"c3: {n_markets} caplet markets, 50-600 quotes, 1024 chains each, "
                    "L=200, N=100", m, truth, noise, chains=1024, n_levels=200, n_steps=100,
                    seed=3)


def config4():
    """Config-1 market; 512 chains, 50 levels x 100 steps, then LM on the best 64."""
    m, truth, noise = I.caplet_market(seed=I.SEED_BASE + 1000)
    return Workload("c4: caplets 10x11, SA 512 chains L=50 N=100 + LM polish of the best 64",
                    m, truth, noise, chains=512, n_levels=50, n_steps=100, seed=4,
                    extra=dict(polish=64, fd_points=1000))


def config5(n_markets=64):
    """64 LMM12 markets x 40 forwards: 39 x 21 caplets + 20 x 20 swaptions x 9
    strikes, both option sides (8838 quotes each), 8192 chains each."""
    m, truth, noise = I.lmm_market(seed=I.SEED_BASE + 5000, n_markets=n_markets, M=40,
                                   n_cap_K=21, n_exp=20, n_ten=20, n_swp_K=9, both_sides=True,
                                   residual=I.RESID_PRICE)
    return Workload(f"c5: {n_markets} LMM12 markets x 8838 quotes, 8192 chains each, "
                    "L=20, N=10 slice", m, truth, noise, chains=8192, n_levels=20, n_steps=10,
                    seed=5, extra=dict(polish=128))


def paper_levels(T0, T_min, cool):
    """Temperature levels of the paper's schedule T_l = T0 cool^l while
    T_l >= T_min (Sec. 3)."""
    L = 0
    T = T0
    while T >= T_min:
        L += 1
        T *= cool
    return L


def paper_e2(chains=16384):
    """The paper's own timed caplet calibration (Sec. 4.1.1) replayed on its
    printed data: the per-forward Hagan model (PERFWD, 13 forwards, P = 39,
    beta = 0.5) on the 13 x 9 EURIBOR caplet smiles with eq. (sigmaHagan),
    SA with T0 = 10, Tmin = 0.01, rho = 0.99 (688 levels), N = 10 and
    256 x 64 = 16384 chains: 16384 (1 + 10 x 688) = 112,738,304 cost
    evaluations, as printed.  The paper then polishes with Nelder-Mead; here
    LM polishes each forward as a GLOBAL4 instance with beta frozen.
    Printed for comparison: SA 8.565 s and Nelder-Mead 0.174 s on one
    GTX 470, MRE 1.80e-2."""
    m = I.paper_caplet_market()
    T0, T_min, cool = 10.0, 0.01, 0.99
    return Workload("e2: the paper's EURIBOR caplets 13x9, PERFWD P=39, eq. (sigmaHagan), "
                    f"{chains} chains, T0=10, Tmin=0.01, rho=0.99, N=10", m, None, None,
                    chains=chains, n_levels=paper_levels(T0, T_min, cool), n_steps=10, seed=6,
                    extra=dict(T0=T0, T_min=T_min, cool=cool, paper_sa_s=8.565,
                               paper_nm_s=0.174, paper_evals=112738304, paper_mre=1.80e-2))


def paper_mm(chains=16384):
    """The paper's Mercurio-Morini caplet calibration (Sec. 4.2.1) replayed on
    its printed data: MM (13 forwards, P = 27, beta = 0.5), eq.
    (sigmaHagan), the same annealing settings as E2 (T0 = 10, Tmin = 0.01,
    rho = 0.99, 688 levels, N = 10, 16384 chains: 112,738,304 cost
    evaluations).  Printed for comparison: SA 9.124 s and Nelder-Mead
    0.041 s on one GTX 470, MRE 3.11e-2."""
    m = I.paper_caplet_market(model=I.MODEL_MM)
    T0, T_min, cool = 10.0, 0.01, 0.99
    return Workload("mm: the paper's EURIBOR caplets 13x9, Mercurio-Morini P=27, eq. "
                    f"(sigmaHagan), {chains} chains, T0=10, Tmin=0.01, rho=0.99, N=10", m, None,
                    None, chains=chains, n_levels=paper_levels(T0, T_min, cool), n_steps=10,
                    seed=7, extra=dict(T0=T0, T_min=T_min, cool=cool, paper_sa_s=9.124,
                                       paper_nm_s=0.041, paper_evals=112738304,
                                       paper_mre=3.11e-2))


def paper_reb(chains=32768, n_steps=100):
    """The paper's Rebonato caplet calibration (Sec. 4.3.1) replayed on its
    printed data: REB (13 forwards, P = 34, beta = 0.5), eq. (sigmaHagan),
    T0 = 10, Tmin = 0.01, rho = 0.99 (688 levels), N = 100, and the chains of
    its two GPUs (2 x 256 x 64 = 32768) on one: 32768 (1 + 100 x 688) =
    2,254,471,168 cost evaluations ("roughly two billion").  Printed for
    comparison: SA 119.913 s on two GTX 470, MRE 2.93e-2."""
    m = I.paper_caplet_market(model=I.MODEL_REB)
    T0, T_min, cool = 10.0, 0.01, 0.99
    return Workload(f"reb: the paper's EURIBOR caplets 13x9, Rebonato P=34, eq. (sigmaHagan), "
                    f"{chains} chains, T0=10, Tmin=0.01, rho=0.99, N={n_steps}", m, None, None,
                    chains=chains, n_levels=paper_levels(T0, T_min, cool), n_steps=n_steps,
                    seed=8, extra=dict(T0=T0, T_min=T_min, cool=cool, paper_sa_s=119.913,
                                       paper_total_s=146.729, paper_evals=2254471168,
                                       paper_mre=2.93e-2))


CONFIGS = {"c1": config1, "c2": config2, "c3": config3, "c4": config4, "c5": config5}


def synthesize(w: Workload, vols_fn):
    """Complete the market: q_vol = vols_fn(vol-mode market, truth) + noise.
    ``vols_fn`` returns the concatenated model vols of every instance."""
    vols = vols_fn(I.as_vol_market(w.market), w.truth)
    return I.complete_market(w.market, vols, w.noise)


def schedule(costs_at_random_points, n_quotes, n_levels):
    """Temperature schedule (the paper's T0 = 10 suits its own cost units;
    these markets use decimal vols or vega-scaled prices): T0 = 0.1 x the
    median cost over random box points, T_end = 0.01 Q sigma_noise^2, and
    cool = (T_end / T0)^(1/(L-1)) so the last level runs at T_end."""
    c = np.asarray(costs_at_random_points, float)
    c = c[np.isfinite(c)]
    T0 = 0.1 * float(np.median(c))
    T_end = 0.01 * float(n_quotes) * SIGMA_NOISE ** 2
    cool = (T_end / T0) ** (1.0 / max(n_levels - 1, 1)) if T_end < T0 else 1.0
    return T0, cool


def schedule_points(model, seed):
    return I.random_box_points(model, 1024, seed)
