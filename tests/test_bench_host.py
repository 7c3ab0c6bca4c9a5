"""Host side of bench.py's report (no GPU): the one-GPU guard, the traffic
records of the level kernel's counter profile, and the accounting behind
roofline.achieved -- the algorithmic FLOP of flops.py against the FP64
operations the hardware counters executed, as committed under profiles/
(executed may exceed algorithmic by at most 1.5x, and the algorithmic count
may not exceed what ran)."""
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


def test_traffic_records(bench, monkeypatch):
    shapes = [(4, 4), (8, 4), (6, 4), (4, 3), (8, 3)]
    vals = [bench.measured_traffic("c2", {"waves_per_group": w, "occupancy": o})
            for w, o in shapes]
    assert all(v is not None and 1e6 < v < 1e7 for v in vals), vals
    assert bench.measured_traffic("c2", {"waves_per_group": 2, "occupancy": 4}) is None
    assert bench.measured_traffic("c9", {"waves_per_group": 4, "occupancy": 4}) is None
    from paper_2408_01470_amd import build
    monkeypatch.setattr(build, "source_digest", lambda: "0" * 64)
    assert bench.measured_traffic("c2", {"waves_per_group": 4, "occupancy": 4}) is None


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
