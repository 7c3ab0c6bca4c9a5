"""Host side of the Monte Carlo pricer's C ABI (no GPU): the plan's
correlation factor against the oracle's (the same spectral repair, computed
by the library's own Jacobi eigen-solver), and validation of the problem."""
import os

import numpy as np
import pytest

from conftest import ROOT
from paper_2408_01470_amd import inputs as I

LIB = os.path.join(ROOT, "paper_2408_01470_amd", "libsabr_hip.so")


@pytest.fixture(scope="module")
def api():
    if not os.path.exists(LIB):
        pytest.skip("HIP library not built")
    from paper_2408_01470_amd import api as A
    return A


@pytest.mark.parametrize("which", ["paper", "synthetic", "max", "one", "seven-clipped"])
def test_factor_matches_oracle(api, oracle, which):
    """The plan's factor (its own Jacobi eigen-solver, repair and semi-definite
    Cholesky) against the oracle's (numpy's eigh); with seven clipped
    eigenvalues the zero pivots are rounding noise and the rest agrees to
    1e-10."""
    p = {"paper": lambda: I.paper_mc_problem(),
         "synthetic": lambda: I.mc_problem(),
         "max": lambda: I.mc_problem(seed=I.SEED_BASE + 9600, M=16, n_swaptions=4),
         "one": lambda: I.mc_problem(seed=I.SEED_BASE + 9601, M=1, n_swaptions=0),
         "seven-clipped": lambda: I.mc_problem(seed=I.SEED_BASE + 9826, M=16, n_cap_K=2,
                                               n_swaptions=5)}[which]()
    B = api.McProblem(p).factor()
    Bo = oracle.mc_factor(p["T"], p["phi"], p["y"])
    np.testing.assert_allclose(B, Bo, rtol=0, atol=1e-10 if which == "seven-clipped" else 1e-12)
    np.testing.assert_allclose((B * B).sum(axis=1), 1.0, atol=1e-11)


@pytest.mark.parametrize("mutate,msg", [
    (lambda p: p["T"].__setitem__(3, p["T"][2]), "increasing"),
    (lambda p: p["T"].__setitem__(0, 0.0), "increasing"),
    (lambda p: p["F0"].__setitem__(1, -0.01), "positive"),
    (lambda p: p["alpha"].__setitem__(1, 0.0), "positive"),
    (lambda p: p["beta"].__setitem__(2, 1.5), "beta"),
    (lambda p: p["phi"].__setitem__(2, -1.2), "phi"),
    (lambda p: p["sigma"].__setitem__(2, -0.1), "sigma"),
    (lambda p: p["y"].__setitem__(0, 1.2), "eta1"),
    (lambda p: p["y"].__setitem__(4, -1.0), "lambda"),
    (lambda p: p["opt_b"].__setitem__(0, 7), "a < b"),
    (lambda p: p["opt_b"].__setitem__(0, p["opt_a"][0]), "a < b"),
    (lambda p: p["opt_K"].__setitem__(0, np.nan), "strike"),
], ids=["T-equal", "T0-zero", "F0", "alpha", "beta", "phi", "sigma", "eta", "lambda", "b>M",
        "b=a", "K-nan"])
def test_plan_rejects_bad_problem(api, mutate, msg):
    p = I.mc_problem(seed=I.SEED_BASE + 9700, M=6, n_swaptions=2)
    mutate(p)
    with pytest.raises(Exception) as e:
        api.McProblem(p)
    assert msg in str(e.value)


def test_plan_limits(api):
    with pytest.raises(Exception) as e:
        api.McProblem(I.mc_problem(seed=I.SEED_BASE + 9701, M=25, n_swaptions=0))
    assert "n_fwd must be 1..24" in str(e.value)
    p = I.mc_problem(seed=I.SEED_BASE + 9702, M=3, n_swaptions=0)
    for k in ("opt_a", "opt_b", "opt_K"):
        p[k] = p[k][:0]
    with pytest.raises(Exception) as e:
        api.McProblem(p)
    assert "at least one option" in str(e.value)
