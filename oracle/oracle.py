"""ctypes binding of the CPU oracle (``liboracle_sabr.so``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg.  The product path never loads it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle_sabr.so")
SRC = os.path.join(HERE, "sabr_oracle.cpp")

_i32p = ctypes.POINTER(ctypes.c_int32)
_f64p = ctypes.POINTER(ctypes.c_double)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_i64p = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (FP64, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(LIB_PATH):
        cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-o", LIB_PATH + ".tmp", SRC]
        subprocess.run(cmd, check=True)
        os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class OracleMarket(ctypes.Structure):
    _fields_ = [
        ("n_inst", ctypes.c_int32),
        ("fwd_off", _i32p), ("fwd_T", _f64p), ("fwd_tau", _f64p), ("fwd_F", _f64p),
        ("fwd_P", _f64p),
        ("und_off", _i32p), ("und_first", _i32p), ("und_len", _i32p),
        ("q_off", _i32p), ("q_und", _i32p), ("q_kind", _i32p),
        ("q_K", _f64p), ("q_vol", _f64p), ("q_w", _f64p),
        ("model", ctypes.c_int32), ("formula", ctypes.c_int32), ("residual", ctypes.c_int32),
        ("beta", ctypes.c_double),
    ]


class OracleSAConfig(ctypes.Structure):
    _fields_ = [
        ("T0", ctypes.c_double), ("cool", ctypes.c_double), ("step_frac", ctypes.c_double),
        ("n_levels", ctypes.c_int32), ("n_steps", ctypes.c_int32), ("seed", ctypes.c_uint64),
        ("T0_per_inst", _f64p), ("level0", ctypes.c_int32), ("inst_key", _i32p),
        ("state_in", _f64p), ("state_out", _f64p),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=True)
        L = ctypes.CDLL(LIB_PATH)
        L.oracle_last_error.restype = ctypes.c_char_p
        L.oracle_hagan2002_vol.restype = ctypes.c_double
        L.oracle_hagan2002_vol.argtypes = [ctypes.c_double] * 7
        L.oracle_paper_eq3_vol.restype = ctypes.c_double
        L.oracle_paper_eq3_vol.argtypes = [ctypes.c_double] * 6
        L.oracle_chi.restype = ctypes.c_double
        L.oracle_chi.argtypes = [ctypes.c_double] * 2
        L.oracle_black.restype = ctypes.c_double
        L.oracle_black.argtypes = [ctypes.c_int32] + [ctypes.c_double] * 5
        L.oracle_black_vega.restype = ctypes.c_double
        L.oracle_black_vega.argtypes = [ctypes.c_double] * 5
        L.oracle_philox4x64_10.argtypes = [_u64p, _u64p, _u64p]
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t) if a is not None else None


class Market:
    """Keeps the numpy arrays alive while the C struct points into them."""

    def __init__(self, m: dict):
        self.arrays = {}
        for k in ("fwd_off", "und_off", "q_off", "und_first", "und_len", "q_und", "q_kind"):
            self.arrays[k] = np.ascontiguousarray(m[k], dtype=np.int32)
        for k in ("fwd_T", "fwd_tau", "fwd_F", "fwd_P", "q_K", "q_vol", "q_w"):
            self.arrays[k] = np.ascontiguousarray(m[k], dtype=np.float64)
        a = self.arrays
        self.n_inst = len(a["q_off"]) - 1
        self.model = int(m["model"])
        fo = a["fwd_off"]
        nf = int(fo[1] - fo[0]) if len(fo) > 1 else -1
        self.P = {0: 4, 1: 12, 2: 3 * nf, 3: 2 * nf + 1, 4: 2 * nf + 8}.get(self.model, -1)
        self.nq = np.diff(a["q_off"])
        self.nu = np.diff(a["und_off"])
        self.s = OracleMarket(
            self.n_inst,
            _p(a["fwd_off"], _i32p), _p(a["fwd_T"], _f64p), _p(a["fwd_tau"], _f64p),
            _p(a["fwd_F"], _f64p), _p(a["fwd_P"], _f64p),
            _p(a["und_off"], _i32p), _p(a["und_first"], _i32p), _p(a["und_len"], _i32p),
            _p(a["q_off"], _i32p), _p(a["q_und"], _i32p), _p(a["q_kind"], _i32p),
            _p(a["q_K"], _f64p), _p(a["q_vol"], _f64p), _p(a["q_w"], _f64p),
            self.model, int(m["formula"]), int(m["residual"]), float(m["beta"]))


def _check(rc):
    if rc < 0:
        raise ValueError("oracle: " + lib().oracle_last_error().decode())
    return rc


def _mk(m):
    return m if isinstance(m, Market) else Market(m)


def max_threads():
    return lib().oracle_max_threads()


def set_threads(n):
    lib().oracle_set_threads(int(n))


def hagan2002_vol(f, K, T, alpha, beta, rho, nu):
    return lib().oracle_hagan2002_vol(f, K, T, alpha, beta, rho, nu)


def paper_eq3_vol(f, K, alpha, beta, rho, nu):
    return lib().oracle_paper_eq3_vol(f, K, alpha, beta, rho, nu)


def chi(z, rho):
    return lib().oracle_chi(z, rho)


def black(kind, f, K, T, sigma, D):
    return lib().oracle_black(kind, f, K, T, sigma, D)


def black_vega(f, K, T, sigma, D):
    return lib().oracle_black_vega(f, K, T, sigma, D)


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().oracle_philox4x64_10(_p(c, _u64p), _p(k, _u64p), _p(out, _u64p))
    return out


def underlyings(m, inst=0):
    M = _mk(m)
    n = int(M.nu[inst])
    S0, A, T = np.zeros(n), np.zeros(n), np.zeros(n)
    _check(lib().oracle_underlyings(ctypes.byref(M.s), inst, _p(S0, _f64p), _p(A, _f64p),
                                    _p(T, _f64p)))
    return S0, A, T


def map_params(m, inst, p):
    M = _mk(m)
    out = np.zeros(int(M.nu[inst]) * 4)
    p = np.ascontiguousarray(p, dtype=np.float64)
    rc = _check(lib().oracle_map_params(ctypes.byref(M.s), inst, _p(p, _f64p), _p(out, _f64p)))
    return out.reshape(-1, 4), rc == 0


def model_values(m, inst, p):
    """(model, target, weight) per quote of instance `inst`."""
    M = _mk(m)
    n = int(M.nq[inst])
    mv, tg, w = np.zeros(n), np.zeros(n), np.zeros(n)
    p = np.ascontiguousarray(p, dtype=np.float64)
    rc = _check(lib().oracle_model_values(ctypes.byref(M.s), inst, _p(p, _f64p), _p(mv, _f64p),
                                          _p(tg, _f64p), _p(w, _f64p)))
    return mv, tg, w, rc == 0


def cost_batch(m, params, pt_inst=None, resid=False):
    M = _mk(m)
    params = np.ascontiguousarray(np.atleast_2d(params), dtype=np.float64)
    n = params.shape[0]
    pt = np.zeros(n, np.int32) if pt_inst is None else np.ascontiguousarray(pt_inst, np.int32)
    cost = np.zeros(n)
    stride = int(M.nq.max()) if len(M.nq) else 0
    r = np.full((n, stride), np.nan) if resid else None
    _check(lib().oracle_cost_batch(ctypes.byref(M.s), n, _p(pt, _i32p), _p(params, _f64p),
                                   _p(cost, _f64p), _p(r, _f64p), stride))
    return (cost, r) if resid else cost


def cost_grad(m, params, pt_inst=None, normal=False):
    M = _mk(m)
    params = np.ascontiguousarray(np.atleast_2d(params), dtype=np.float64)
    n, P = params.shape
    pt = np.zeros(n, np.int32) if pt_inst is None else np.ascontiguousarray(pt_inst, np.int32)
    cost, grad = np.zeros(n), np.zeros((n, P))
    A = np.zeros((n, P, P)) if normal else None
    g = np.zeros((n, P)) if normal else None
    _check(lib().oracle_cost_grad(ctypes.byref(M.s), n, _p(pt, _i32p), _p(params, _f64p),
                                  _p(cost, _f64p), _p(grad, _f64p), _p(A, _f64p), _p(g, _f64p)))
    return (cost, grad, A, g) if normal else (cost, grad)


def sabr_cost_batch(m, params, pt_inst=None, resid=False, model=False):
    """The mirror of the library's sabr_cost_batch: cost, and the residuals
    and model values ([n, stride], the caller's quote order) when asked."""
    M = _mk(m)
    params = np.ascontiguousarray(np.atleast_2d(params), dtype=np.float64)
    n = params.shape[0]
    pt = np.zeros(n, np.int32) if pt_inst is None else np.ascontiguousarray(pt_inst, np.int32)
    cost = np.zeros(n)
    stride = int(M.nq.max()) if len(M.nq) else 0
    r = np.full((n, stride), np.nan) if resid else None
    mv = np.full((n, stride), np.nan) if model else None
    _check(lib().oracle_sabr_cost_batch(ctypes.byref(M.s), n, _p(pt, _i32p), _p(params, _f64p),
                                        _p(cost, _f64p), _p(r, _f64p), _p(mv, _f64p), stride))
    return cost, r, mv


def sabr_cost_vjp(m, params, pt_inst=None, g_cost=None, normal=False):
    """The mirror of the library's sabr_cost_vjp: cost, g_cost-weighted
    gradient and (normal) J^T W J, J^T W r."""
    M = _mk(m)
    params = np.ascontiguousarray(np.atleast_2d(params), dtype=np.float64)
    n, P = params.shape
    pt = np.zeros(n, np.int32) if pt_inst is None else np.ascontiguousarray(pt_inst, np.int32)
    gc = None if g_cost is None else np.ascontiguousarray(g_cost, dtype=np.float64)
    cost, gp = np.zeros(n), np.zeros((n, P))
    A = np.zeros((n, P, P)) if normal else None
    g = np.zeros((n, P)) if normal else None
    _check(lib().oracle_sabr_cost_vjp(ctypes.byref(M.s), n, _p(pt, _i32p), _p(params, _f64p),
                                      _p(gc, _f64p), _p(cost, _f64p), _p(gp, _f64p),
                                      _p(A, _f64p), _p(g, _f64p)))
    return cost, gp, A, g


def sa_state_doubles(chains, P):
    """Doubles of the annealing state of instances with these chain counts:
    per instance X [C][P], F [C], BX [C][P], BF [C], T."""
    return int(sum(2 * int(c) * (P + 1) + 1 for c in np.atleast_1d(chains)))


def sa_calibrate(m, chains, lb, ub, T0, cool, n_levels, n_steps, seed, step_frac=0.05,
                 x0=None, T0_per_inst=None, record=False, level0=0, inst_key=None,
                 state_in=None, keep_state=False):
    """Synchronous parallel SA (Sec. 3).  level0 > 0 starts at that level of
    the schedule (Philox counters and temperature); state_in resumes from the
    state a previous call returned with keep_state (then no initial
    evaluation); inst_key overrides the Philox key word 1 of each instance."""
    M = _mk(m)
    P = M.P
    ch = np.ascontiguousarray(np.broadcast_to(np.asarray(chains, np.int32), (M.n_inst,)),
                              dtype=np.int32)
    lb = np.ascontiguousarray(np.broadcast_to(lb, (M.n_inst, P)), dtype=np.float64)
    ub = np.ascontiguousarray(np.broadcast_to(ub, (M.n_inst, P)), dtype=np.float64)
    x0a = None if x0 is None else np.ascontiguousarray(np.broadcast_to(x0, (M.n_inst, P)),
                                                       dtype=np.float64)
    t0i = None if T0_per_inst is None else np.ascontiguousarray(T0_per_inst, dtype=np.float64)
    key = None if inst_key is None else np.ascontiguousarray(inst_key, dtype=np.int32)
    nst = sa_state_doubles(ch, P)
    sin = None if state_in is None else np.ascontiguousarray(state_in, dtype=np.float64)
    if sin is not None and sin.size != nst:
        raise ValueError(f"state_in holds {sin.size} doubles, need {nst}")
    sout = np.zeros(nst) if keep_state else None
    cfg = OracleSAConfig(T0, cool, step_frac, n_levels, n_steps, seed, _p(t0i, _f64p),
                         level0, _p(key, _i32p), _p(sin, _f64p), _p(sout, _f64p))
    best_x = np.zeros((M.n_inst, P))
    best_f = np.zeros(M.n_inst)
    tot = int(ch.sum())
    cbx = np.zeros((tot, P))
    cbf = np.zeros(tot)
    acc = np.zeros(int(n_levels) * int(n_steps) * tot, np.uint8) if record else None
    trace = np.zeros((M.n_inst, n_levels, 3))
    lbest = np.zeros((M.n_inst, n_levels), np.int32)
    nev = np.zeros(M.n_inst, np.int64)
    _check(lib().oracle_sa_calibrate(
        ctypes.byref(M.s), ctypes.byref(cfg), _p(ch, _i32p), _p(lb, _f64p), _p(ub, _f64p),
        _p(x0a, _f64p), _p(best_x, _f64p), _p(best_f, _f64p), _p(cbx, _f64p), _p(cbf, _f64p),
        _p(acc, _u8p), _p(trace, _f64p), _p(lbest, _i32p), _p(nev, _i64p)))
    out = dict(best_x=best_x, best_f=best_f, chain_best_x=cbx, chain_best_f=cbf, accept=acc,
               trace=trace, level_best=lbest, n_evals=nev)
    if keep_state:
        out["state"] = sout
    return out


def sa_state_split(state, chains, P):
    """Per instance (X [C][P], F [C], BX [C][P], BF [C], T) of a state vector."""
    out, o = [], 0
    for C in np.atleast_1d(chains):
        C = int(C)
        X = state[o:o + C * P].reshape(C, P)
        o += C * P
        F = state[o:o + C]
        o += C
        BX = state[o:o + C * P].reshape(C, P)
        o += C * P
        BF = state[o:o + C]
        o += C
        out.append((X, F, BX, BF, float(state[o])))
        o += 1
    return out


def sa_chain_steps(m, inst, chain, level, T, lb, ub, x, f, n_steps, seed, step_frac=0.05,
                   inst_key=None):
    """One chain's steps of one level, step by step, from point x (cost f):
    proposals, their costs, the acceptance uniforms and the accept flags."""
    M = _mk(m)
    P = M.P
    lb = np.ascontiguousarray(np.broadcast_to(lb, (M.n_inst, P)), dtype=np.float64)
    ub = np.ascontiguousarray(np.broadcast_to(ub, (M.n_inst, P)), dtype=np.float64)
    key = None if inst_key is None else np.ascontiguousarray(inst_key, dtype=np.int32)
    cfg = OracleSAConfig(1.0, 1.0, step_frac, 1, n_steps, seed, None, 0, _p(key, _i32p),
                         None, None)
    xa = np.ascontiguousarray(x, dtype=np.float64)
    xp = np.zeros((n_steps, P))
    fp = np.zeros(n_steps)
    u = np.zeros(n_steps)
    acc = np.zeros(n_steps, np.uint8)
    _check(lib().oracle_sa_chain_steps(
        ctypes.byref(M.s), ctypes.byref(cfg), int(inst), int(chain), int(level),
        ctypes.c_double(T), _p(lb, _f64p), _p(ub, _f64p), _p(xa, _f64p), ctypes.c_double(f),
        _p(xp, _f64p), _p(fp, _f64p), _p(u, _f64p), _p(acc, _u8p)))
    return dict(xp=xp, fp=fp, u=u, accept=acc)


def sa_level0_sample(m, chains, lb, ub, T0, n_steps, seed, sample_inst, sample_chain,
                     step_frac=0.05, x0=None, T0_per_inst=None):
    """Level 0 of sa_calibrate for sampled (instance, chain) pairs."""
    M = _mk(m)
    P = M.P
    ch = np.ascontiguousarray(np.broadcast_to(np.asarray(chains, np.int32), (M.n_inst,)),
                              dtype=np.int32)
    lb = np.ascontiguousarray(np.broadcast_to(lb, (M.n_inst, P)), dtype=np.float64)
    ub = np.ascontiguousarray(np.broadcast_to(ub, (M.n_inst, P)), dtype=np.float64)
    x0a = None if x0 is None else np.ascontiguousarray(np.broadcast_to(x0, (M.n_inst, P)),
                                                       dtype=np.float64)
    t0i = None if T0_per_inst is None else np.ascontiguousarray(T0_per_inst, dtype=np.float64)
    cfg = OracleSAConfig(T0, 1.0, step_frac, 1, n_steps, seed, _p(t0i, _f64p))
    si = np.ascontiguousarray(sample_inst, np.int32)
    sc = np.ascontiguousarray(sample_chain, np.int32)
    n = len(si)
    acc = np.zeros((n, int(n_steps)), np.uint8)
    F = np.zeros(n)
    BF = np.zeros(n)
    BX = np.zeros((n, P))
    _check(lib().oracle_sa_level0_sample(
        ctypes.byref(M.s), ctypes.byref(cfg), _p(ch, _i32p), _p(lb, _f64p), _p(ub, _f64p),
        _p(x0a, _f64p), n, _p(si, _i32p), _p(sc, _i32p), _p(acc, _u8p), _p(F, _f64p),
        _p(BF, _f64p), _p(BX, _f64p)))
    return dict(accept=acc, F=F, BF=BF, BX=BX)


def nm_polish(m, params, pt_inst, lb, ub, max_iter=1000, step=0.05, tol=1e-12):
    M = _mk(m)
    P = M.P
    x = np.ascontiguousarray(np.atleast_2d(params), dtype=np.float64).copy()
    n = x.shape[0]
    pt = np.zeros(n, np.int32) if pt_inst is None else np.ascontiguousarray(pt_inst, np.int32)
    lb = np.ascontiguousarray(np.broadcast_to(lb, (M.n_inst, P)), dtype=np.float64)
    ub = np.ascontiguousarray(np.broadcast_to(ub, (M.n_inst, P)), dtype=np.float64)
    f = np.zeros(n)
    it = np.zeros(n, np.int32)
    _check(lib().oracle_nm_polish(ctypes.byref(M.s), n, _p(pt, _i32p), _p(x, _f64p),
                                  _p(lb, _f64p), _p(ub, _f64p), int(max_iter),
                                  ctypes.c_double(step), ctypes.c_double(tol), _p(f, _f64p),
                                  _p(it, _i32p)))
    return x, f, it


def lm_polish(m, params, pt_inst, lb, ub, max_iter=50, mu0=1e-3, tol=1e-12):
    M = _mk(m)
    P = M.P
    x = np.ascontiguousarray(np.atleast_2d(params), dtype=np.float64).copy()
    n = x.shape[0]
    pt = np.zeros(n, np.int32) if pt_inst is None else np.ascontiguousarray(pt_inst, np.int32)
    lb = np.ascontiguousarray(np.broadcast_to(lb, (M.n_inst, P)), dtype=np.float64)
    ub = np.ascontiguousarray(np.broadcast_to(ub, (M.n_inst, P)), dtype=np.float64)
    f = np.zeros(n)
    it = np.zeros(n, np.int32)
    _check(lib().oracle_lm_polish(ctypes.byref(M.s), n, _p(pt, _i32p), _p(x, _f64p),
                                  _p(lb, _f64p), _p(ub, _f64p), int(max_iter), ctypes.c_double(mu0),
                                  ctypes.c_double(tol), _p(f, _f64p), _p(it, _i32p)))
    return x, f, it


# ---------------------------------------------------------------------------
# Monte Carlo under the Hagan SABR/LIBOR dynamics (Sec. 2.1)
# ---------------------------------------------------------------------------
_u32p = ctypes.POINTER(ctypes.c_uint32)


def _mc_lib():
    L = lib()
    if not getattr(L, "_mc_ready", False):
        L.oracle_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
        L.oracle_mc_normals.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64,
                                        ctypes.c_int32, _f64p]
        L.oracle_mc_steps.argtypes = [ctypes.c_double, ctypes.c_double]
        L.oracle_mc_steps.restype = ctypes.c_int32
        L.oracle_mc_paths.argtypes = ([ctypes.c_int32] + [_f64p] * 8 + [ctypes.c_double, _f64p,
                                      ctypes.c_int32, _i32p, _i32p, _f64p, ctypes.c_int64,
                                      ctypes.c_int64, ctypes.c_double, ctypes.c_uint64, _f64p])
        L.oracle_mc_paths.restype = ctypes.c_int32
        L._mc_ready = True
    return L


def philox4x32(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _mc_lib().oracle_philox4x32_10(_p(c, _u32p), _p(k, _u32p), _p(out, _u32p))
    return out


def mc_normals(seed, path, step, M):
    xi = np.zeros(2 * M)
    _mc_lib().oracle_mc_normals(int(seed), int(path), int(step), int(M), _p(xi, _f64p))
    return xi


def mc_steps(length, dt):
    return _mc_lib().oracle_mc_steps(float(length), float(dt))


def mc_corr_matrix(T, phi, y):
    """The 2M x 2M correlation of (W_1..W_M, Z_1..Z_M) of Sec. 2.1: blocks rho
    (eq. rhoij), phi with phi_{i,j} = E[dW_i dZ_j] (eq. phiij) and theta
    (eq. thetaij)."""
    T = np.asarray(T, float)
    phi = np.asarray(phi, float)
    eta1, lam1, eta2, lam2, lam3 = [float(v) for v in y]
    dT = np.abs(T[:, None] - T[None, :])
    rho = eta1 + (1.0 - eta1) * np.exp(-lam1 * dT)
    theta = eta2 + (1.0 - eta2) * np.exp(-lam2 * dT)
    ph = (np.sign(phi)[:, None] * np.sqrt(np.abs(phi[:, None] * phi[None, :]))
          * np.exp(-lam3 * dT))
    return np.block([[rho, ph], [ph.T, theta]])


def mc_repaired_corr(T, phi, y):
    """The spectral repair of Rebonato and Jaeckel (1999) of the matrix above:
    eigenvalues clipped at zero, then rescaled to unit diagonal (the matrix
    itself when it is positive semi-definite)."""
    C = mc_corr_matrix(T, phi, y)
    lam, Q = np.linalg.eigh(C)
    R = (Q * np.maximum(lam, 0.0)[None, :]) @ Q.T
    d = np.sqrt(np.diag(R))
    d = np.where(d > 0.0, d, 1.0)
    return R / d[:, None] / d[None, :]


def mc_factor(T, phi, y):
    """Correlation factor B with x = B xi (xi iid standard normal), rows W_0..
    W_{M-1}, Z_0..Z_{M-1}: the Cholesky factor of the repaired matrix with its
    components ordered W_{M-1}, Z_{M-1}, W_{M-2}, ..., W_0, Z_0 (a pivot at or
    below 1e-9 leaves its column zero: the semi-definite case, whose zero
    pivots come out as rounding noise of order 1e-12), rows put back
    in the natural order.  In that ordering the forwards alive during
    [T_{j-1}, T_j) (k >= j) are the leading 2(M - j) components, so they use
    the first 2(M - j) normals only."""
    R = mc_repaired_corr(T, phi, y)
    M = len(T)
    rows = [t * M + k for k in range(M - 1, -1, -1) for t in (0, 1)]
    A = R[np.ix_(rows, rows)]
    n = 2 * M
    L = np.zeros((n, n))
    for c in range(n):
        dd = A[c, c] - float(np.dot(L[c, :c], L[c, :c]))
        if dd <= 1e-9:
            continue
        L[c, c] = np.sqrt(dd)
        for r in range(c + 1, n):
            L[r, c] = (A[r, c] - float(np.dot(L[r, :c], L[c, :c]))) / L[c, c]
    B = np.zeros((n, n))
    B[rows, :] = L
    return B


def mc_paths(prob, n_paths, dt, seed, path0=0, B=None):
    """Discounted payoff [n_paths][n_opt] of every option on paths path0 ..
    path0 + n_paths - 1 (see oracle_mc_paths)."""
    f = {k: np.ascontiguousarray(prob[k], dtype=np.float64)
         for k in ("T", "tau", "F0", "alpha", "beta", "phi", "sigma", "y", "opt_K")}
    a = np.ascontiguousarray(prob["opt_a"], dtype=np.int32)
    b = np.ascontiguousarray(prob["opt_b"], dtype=np.int32)
    M = len(f["T"])
    if B is None:
        B = mc_factor(f["T"], f["phi"], f["y"])
    B = np.ascontiguousarray(B, dtype=np.float64)
    X = np.zeros((int(n_paths), len(a)))
    _check(_mc_lib().oracle_mc_paths(
        M, _p(f["T"], _f64p), _p(f["tau"], _f64p), _p(f["F0"], _f64p), _p(f["alpha"], _f64p),
        _p(f["beta"], _f64p), _p(f["phi"], _f64p), _p(f["sigma"], _f64p), _p(f["y"], _f64p),
        float(prob["P0"]), _p(B, _f64p), len(a), _p(a, _i32p), _p(b, _i32p), _p(f["opt_K"], _f64p),
        int(path0), int(n_paths), float(dt), int(seed), _p(X, _f64p)))
    return X


def mc_price(prob, n_paths, dt, seed, B=None):
    """Monte Carlo price and standard error of every option."""
    X = mc_paths(prob, n_paths, dt, seed, B=B)
    n = X.shape[0]
    mean = X.mean(axis=0)
    se = X.std(axis=0, ddof=1) / np.sqrt(n) if n > 1 else np.zeros(X.shape[1])
    return mean, se
