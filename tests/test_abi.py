"""C-ABI checks that need no GPU: the built library loads, exports every
function include/sabr.h declares, and host-side validation rejects bad input
before anything would be enqueued."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from conftest import ROOT
from paper_2408_01470_amd import inputs as I

HEADER = os.path.join(ROOT, "include", "sabr.h")
LIB = os.path.join(ROOT, "paper_2408_01470_amd", "libsabr_hip.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", text)
    keywords = {"if", "sizeof", "return", "defined"}
    return sorted(set(n for n in names if n not in keywords and (n.startswith("sabr_") or
                                                                  n.startswith("sa_"))))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(LIB):
        pytest.skip("HIP library not built")
    from paper_2408_01470_amd import _lib
    return _lib.lib()


def test_library_exports_every_declared_function(L):
    names = declared_functions()
    assert len(names) >= 12
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if line.strip())
    missing = [n for n in names if n not in exported]
    assert not missing, f"declared but not exported: {missing}"
    for n in names:
        getattr(L, n)


def _problem(m):
    from paper_2408_01470_amd._lib import SabrProblem
    keep = {}
    for k in ("fwd_off", "und_off", "q_off", "und_first", "und_len", "q_und", "q_kind"):
        keep[k] = np.ascontiguousarray(m[k], dtype=np.int32)
    for k in ("fwd_T", "fwd_tau", "fwd_F", "fwd_P", "q_K", "q_vol", "q_w"):
        keep[k] = np.ascontiguousarray(m[k], dtype=np.float64)
    i32 = ctypes.POINTER(ctypes.c_int32)
    f64 = ctypes.POINTER(ctypes.c_double)
    p = lambda k, t: keep[k].ctypes.data_as(t)
    prob = SabrProblem(len(keep["q_off"]) - 1, p("fwd_off", i32), p("fwd_T", f64),
                       p("fwd_tau", f64), p("fwd_F", f64), p("fwd_P", f64), p("und_off", i32),
                       p("und_first", i32), p("und_len", i32), p("q_off", i32), p("q_und", i32),
                       p("q_kind", i32), p("q_K", f64), p("q_vol", f64), p("q_w", f64),
                       int(m["model"]), int(m["formula"]), int(m["residual"]), float(m["beta"]))
    return prob, keep


def _create(L, m):
    prob, keep = _problem(m)
    h = ctypes.c_void_p()
    rc = L.sabr_plan_create(ctypes.byref(prob), ctypes.byref(h))
    return rc, h


def test_plan_create_and_queries(L):
    m, truth, noise = I.lmm_market()
    rc, h = _create(L, m)
    assert rc == 0
    assert L.sabr_plan_num_params(h) == 12
    assert L.sabr_plan_num_inst(h) == 1
    assert L.sabr_plan_max_quotes(h) == 985
    assert L.sabr_plan_device_bytes(h) > 985 * 8 * 10
    n = int(m["und_off"][-1])
    S0, A, T = np.zeros(n), np.zeros(n), np.zeros(n)
    f64 = ctypes.POINTER(ctypes.c_double)
    assert L.sabr_plan_underlyings(h, S0.ctypes.data_as(f64), A.ctypes.data_as(f64),
                                   T.ctypes.data_as(f64)) == 0
    # caplets: the swap rate of a one-period swap is the forward itself
    cap = m["und_len"] == 1
    np.testing.assert_array_equal(S0[cap], m["fwd_F"][m["und_first"][cap]])
    L.sabr_plan_destroy(h)
    assert L.sabr_num_params(0) == 4 and L.sabr_num_params(1) == 12 and L.sabr_num_params(7) == -1


@pytest.mark.parametrize("mutate,msg", [
    (lambda m: m["q_K"].__setitem__(3, -1.0), "strike"),
    (lambda m: m["q_vol"].__setitem__(0, np.nan), "vol"),
    (lambda m: m["fwd_F"].__setitem__(2, 0.0), "forward"),
    (lambda m: m["q_und"].__setitem__(0, 5), "sorted"),
    (lambda m: m["q_und"].__setitem__(109, 10), "underlying out of range"),
    (lambda m: m["und_first"].__setitem__(9, 10), "forward range"),
    (lambda m: m["q_kind"].__setitem__(4, 2), "kind"),
    (lambda m: m["q_w"].__setitem__(4, -1.0), "weight"),
    (lambda m: m.__setitem__("model", 5), "model"),
    (lambda m: m.__setitem__("beta", 1.5), "beta"),
])
def test_plan_rejects_bad_market(L, mutate, msg):
    m, _, _ = I.caplet_market()
    m = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in m.items()}
    mutate(m)
    rc, h = _create(L, m)
    assert rc == -1, msg
    assert L.sabr_last_error().decode()


def test_plan_rejects_non_monotone_offsets(L):
    m, _, _ = I.batch_markets(n_markets=2)
    m = dict(m)
    m["q_off"] = np.array([0, m["q_off"][2], m["q_off"][1]], np.int32)
    rc, _ = _create(L, m)
    assert rc == -1
    assert "monotone" in L.sabr_last_error().decode()


def test_global4_rejects_swaptions(L):
    m, _, _ = I.lmm_market(M=6, n_cap_K=3, n_exp=2, n_ten=2, n_swp_K=3)
    m = dict(m, model=0)
    rc, _ = _create(L, m)
    assert rc == -1
    assert "only LMM12 markets hold swaptions" in L.sabr_last_error().decode()


def test_sa_rejects_bad_config_without_gpu(L):
    from paper_2408_01470_amd._lib import SAConfig
    m, _, _ = I.caplet_market()
    rc, h = _create(L, m)
    assert rc == 0
    ch = np.array([0], np.int32)
    i32 = ctypes.POINTER(ctypes.c_int32)
    cfg = SAConfig(1.0, 0.9, 0.05, 10, 10, 1, None, 0, 0, None, 0)
    assert L.sa_workspace_size(h, ctypes.byref(cfg), ch.ctypes.data_as(i32)) == 0  # 0 chains
    ch[0] = 16
    assert L.sa_workspace_size(h, ctypes.byref(cfg), ch.ctypes.data_as(i32)) > 16 * 8
    bad = SAConfig(1.0, 1.5, 0.05, 10, 10, 1, None, 0, 0, None, 0)   # cool > 1
    assert L.sa_workspace_size(h, ctypes.byref(bad), ch.ctypes.data_as(i32)) == 0
    # waves per chain: 0..8, and a one-chain workgroup per chain (more tiles)
    split = SAConfig(1.0, 0.9, 0.05, 10, 10, 1, None, 4, 0, None, 0, 2)
    many = np.array([4096], np.int32)
    assert (L.sa_workspace_size(h, ctypes.byref(split), many.ctypes.data_as(i32)) >
            L.sa_workspace_size(h, ctypes.byref(cfg), many.ctypes.data_as(i32)))
    for wpc in (-1, 9):
        bad = SAConfig(1.0, 0.9, 0.05, 10, 10, 1, None, 0, 0, None, 0, wpc)
        assert L.sa_workspace_size(h, ctypes.byref(bad), ch.ctypes.data_as(i32)) == 0
        assert "waves_per_chain" in L.sabr_last_error().decode()
    # not uploaded: sa_calibrate refuses before touching the GPU
    f64 = ctypes.POINTER(ctypes.c_double)
    lb, ub = (np.ascontiguousarray(b) for b in I.box(0))
    rc = L.sa_calibrate(h, ctypes.byref(cfg), ch.ctypes.data_as(i32), lb.ctypes.data_as(f64),
                        ub.ctypes.data_as(f64), None, None, None, None, None, None, None, None,
                        None, 0, None)
    assert rc == -1
    L.sabr_plan_destroy(h)


def test_sa_split_chain_lds_refusal_without_gpu(L):
    """A chain split over more waves than one workgroup's LDS holds is
    refused by name (the per-wave tables of a large LMM12 market)."""
    from paper_2408_01470_amd._lib import SAConfig
    m, _, _ = I.lmm_market(M=60, n_cap_K=3, n_exp=12, n_ten=12, n_swp_K=3)
    rc, h = _create(L, m)
    assert rc == 0
    ch = np.array([4], np.int32)
    i32 = ctypes.POINTER(ctypes.c_int32)
    ok = SAConfig(1.0, 0.9, 0.05, 10, 10, 1, None, 0, 0, None, 0, 1)
    assert L.sa_workspace_size(h, ctypes.byref(ok), ch.ctypes.data_as(i32)) > 0
    big = SAConfig(1.0, 0.9, 0.05, 10, 10, 1, None, 0, 0, None, 0, 8)
    assert L.sa_workspace_size(h, ctypes.byref(big), ch.ctypes.data_as(i32)) == 0
    assert "LDS" in L.sabr_last_error().decode()
    L.sabr_plan_destroy(h)


def test_shutdown_forgets_process_state_without_gpu(L):
    """sabr_shutdown clears the calling thread's last error and the library
    keeps working after it (its caches are looked up again)."""
    m, _, _ = I.caplet_market()
    bad = dict(m)
    bad["q_K"] = bad["q_K"].copy()
    bad["q_K"][0] = -1.0
    rc, _ = _create(L, bad)
    assert rc == -1 and L.sabr_last_error().decode()
    assert L.sabr_shutdown() == 0
    assert L.sabr_last_error().decode() == ""
    rc, h = _create(L, m)
    assert rc == 0
    L.sabr_plan_destroy(h)


def test_sa_paired_chain_refusals_without_gpu(L):
    """chains_per_wave: 2 pairs two GLOBAL4 chains in one wave and halves the
    workgroups (tiles) of the workspace; other values, other models and the
    combination with split chains are refused by name."""
    from paper_2408_01470_amd._lib import SAConfig
    i32 = ctypes.POINTER(ctypes.c_int32)
    m = I.caplet_market()[0]
    rc, h = _create(L, m)
    assert rc == 0
    ch = np.array([4096], np.int32)
    one = SAConfig(1.0, 0.9, 0.05, 10, 10, 1, None, 4, 0, None, 0, 1, 1)
    two = SAConfig(1.0, 0.9, 0.05, 10, 10, 1, None, 4, 0, None, 0, 1, 2)
    s1 = L.sa_workspace_size(h, ctypes.byref(one), ch.ctypes.data_as(i32))
    s2 = L.sa_workspace_size(h, ctypes.byref(two), ch.ctypes.data_as(i32))
    # 4096 chains: 1024 tiles of 4 waves, or 512 of 4 paired waves; each
    # tile holds 2 doubles and 3 ints of level-end partials
    assert s1 > 0 and s2 > 0
    assert s1 - s2 >= 512 * (2 * 8 + 3 * 4) - 5 * 256
    for cpw in (-1, 3):
        bad = SAConfig(1.0, 0.9, 0.05, 10, 10, 1, None, 4, 0, None, 0, 1, cpw)
        assert L.sa_workspace_size(h, ctypes.byref(bad), ch.ctypes.data_as(i32)) == 0
        assert "chains_per_wave" in L.sabr_last_error().decode()
    neg = SAConfig(1.0, 0.9, 0.05, 10, 10, 1, None, 4, 0, None, 0, 1, 1, -1)
    assert L.sa_workspace_size(h, ctypes.byref(neg), ch.ctypes.data_as(i32)) == 0
    assert "level0" in L.sabr_last_error().decode()
    both = SAConfig(1.0, 0.9, 0.05, 10, 10, 1, None, 4, 0, None, 0, 2, 2)
    assert L.sa_workspace_size(h, ctypes.byref(both), ch.ctypes.data_as(i32)) == 0
    assert "waves_per_chain" in L.sabr_last_error().decode()
    L.sabr_plan_destroy(h)
    rc, h = _create(L, I.lmm_market()[0])
    assert rc == 0
    assert L.sa_workspace_size(h, ctypes.byref(two), ch.ctypes.data_as(i32)) == 0
    assert "GLOBAL4" in L.sabr_last_error().decode()
    L.sabr_plan_destroy(h)
