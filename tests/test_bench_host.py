"""Host side of bench.py's report (no GPU): the one-GPU guard, the traffic
records of the level kernel's counter profile, and the accounting behind
roofline.achieved -- the algorithmic FLOP of flops.py against the FP64
operations the hardware counters executed, as committed under profiles/
(executed may exceed algorithmic by at most 1.5x, and the algorithmic count
may not exceed what ran), and the launch shapes the autotuner proposes."""
import os
import re
import subprocess
import sys

import pytest

from conftest import ROOT
from paper_2408_01470_amd import flops, inputs as I, workloads as W


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2 and "one GPU only" in r.stderr and r.stdout == ""


@pytest.fixture(scope="module")
def bench():
    sys.path.insert(0, ROOT)
    import bench as B
    return B


def _records(config):
    import json
    text = open(os.path.join(ROOT, "profiles", f"sa_level_kernel_{config}_counters.md")).read()
    return json.loads(text.split("```json", 1)[1].split("```", 1)[0])


@pytest.mark.parametrize("config,lo,hi", [("c2", 1e6, 1e7), ("c5", 1e7, 1e11)])
def test_traffic_records(bench, monkeypatch, config, lo, hi):
    """Each committed record gives the HBM bytes of its launch shape while the
    sources hash to its digest, and nothing otherwise."""
    from paper_2408_01470_amd import build
    recs = _records(config)
    assert recs
    for rec in recs:
        monkeypatch.setattr(build, "source_digest", lambda d=rec["source_sha256"]: d)
        shape = {"waves_per_group": rec["waves_per_group"], "occupancy": rec["occupancy"]}
        v = bench.measured_traffic(config, shape)
        assert v is not None and lo < v < hi, (config, shape, v)
        assert v == pytest.approx(1024 * (rec["fetch_kib_per_dispatch"] * rec["fetch_scale"] +
                                          rec["write_kib_per_dispatch"] * rec["write_scale"]),
                                  rel=1e-5)
        assert bench.measured_traffic(config, {"waves_per_group": 3, "occupancy": 2}) is None
        monkeypatch.setattr(build, "source_digest", lambda: "0" * 64)
        assert bench.measured_traffic(config, shape) is None
    assert bench.measured_traffic("c9", {"waves_per_group": 4, "occupancy": 4}) is None


def _executed(name, unit):
    text = open(os.path.join(ROOT, "profiles", name)).read()
    m = re.search(r"executed FP64 FLOP[^=]*= 64 \(ADD \+ MUL \+ TRANS \+ 2 FMA\) = ([0-9.]+) " + unit,
                  text)
    assert m, name
    return float(m.group(1))


def test_level_kernel_flop_accounting():
    w = W.config2()
    alg = flops.level_launch_flops(w.market, [w.chains], w.n_steps)
    ex = _executed("sa_level_kernel_c2_counters.md", "G") * 1e9
    assert 1.0 <= ex / alg <= 1.5, (ex, alg)


def test_monte_carlo_flop_accounting():
    alg = flops.mc_launch_flops(I.paper_mc_problem(), 10**6, 1e-3)
    ex = _executed("mc_kernel_paper_table.md", "T") * 1e12
    assert 0.98 <= ex / alg <= 1.5, (ex, alg)


class _PlanShape:
    """The attributes of api.Plan the tuner's candidate lists read."""

    def __init__(self, n_inst, max_q, model):
        self.n_inst, self.max_q, self.model = n_inst, max_q, model


def test_autotune_split_and_pair_candidates():
    """Split shapes (several waves per chain) only when the chains leave most
    of the 1024 SIMDs idle and a chain has two or more blocks of 64 quotes;
    paired shapes (two chains per wave) only for GLOBAL4 plans whose chains
    fill the chip four times over."""
    from paper_2408_01470_amd import autotune as AT
    c1 = _PlanShape(1, 110, 0)
    assert AT.split_candidates(c1, 64) == ((2, 1, 2), (2, 3, 2))
    assert AT.pair_candidates(c1, 64) == ()
    assert AT.split_candidates(_PlanShape(1, 60, 0), 64) == ()          # one block of quotes
    assert AT.split_candidates(_PlanShape(1, 985, 1), 4096) == ()        # the chip is full
    wide = AT.split_candidates(_PlanShape(1, 8838, 1), 64)
    assert {k for k, _, _ in wide} == {2, 4, 8} and all(w == k for w, _, k in wide)
    c3 = _PlanShape(256, 585, 0)
    pairs = AT.pair_candidates(c3, 1024)
    assert pairs and all(len(p) == 4 and p[2] == 1 and p[3] == 2 for p in pairs)
    assert AT.pair_candidates(_PlanShape(64, 8838, 1), 8192) == ()       # LMM12: no pairing
    assert AT.pair_candidates(_PlanShape(1, 110, 0), 512) == ()          # too few chains
    assert AT.split_candidates(c3, 1024) == ()
