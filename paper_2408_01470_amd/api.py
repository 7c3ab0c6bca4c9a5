"""Python front end of the HIP calibrator: torch tensors in, torch tensors out.

Argument marshalling only -- every step of the calibration runs in the HIP
kernels behind the C ABI (include/sabr.h).  PyTorch supplies device memory and
streams.  There is no CPU fallback: without the built library or a GPU these
calls raise.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import SAConfig, SabrMcProblem, SabrProblem, check, lib

_i32p = ctypes.POINTER(ctypes.c_int32)
_f64p = ctypes.POINTER(ctypes.c_double)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream=None, *tensors):
    """The stream a launch runs on: the caller's, or torch's current one.  On
    a stream other than the current one the launch first waits for the
    current stream (where torch allocated and filled the tensors), and every
    tensor it touches is recorded on that stream, so torch's caching
    allocator does not hand the memory out while the launch may still use
    it."""
    cur = torch.cuda.current_stream()
    if stream is None or stream == cur:
        return ctypes.c_void_p(cur.cuda_stream)
    stream.wait_stream(cur)
    for t in tensors:
        if t is not None:
            t.record_stream(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _require_gpu():
    if not torch.cuda.is_available():
        raise RuntimeError("the HIP calibrator needs a GPU (no CPU fallback)")


class Plan:
    """A validated market batch uploaded to device memory."""

    def __init__(self, market: dict, device: str = "cuda", stream=None):
        _require_gpu()
        L = lib()
        self.device = torch.device(device)
        self._keep = {}
        for k in ("fwd_off", "und_off", "q_off", "und_first", "und_len", "q_und", "q_kind"):
            self._keep[k] = np.ascontiguousarray(market[k], dtype=np.int32)
        for k in ("fwd_T", "fwd_tau", "fwd_F", "fwd_P", "q_K", "q_vol", "q_w"):
            self._keep[k] = np.ascontiguousarray(market[k], dtype=np.float64)
        a = self._keep
        p = lambda k, t: a[k].ctypes.data_as(t)
        self._prob = SabrProblem(
            len(a["q_off"]) - 1,
            p("fwd_off", _i32p), p("fwd_T", _f64p), p("fwd_tau", _f64p), p("fwd_F", _f64p),
            p("fwd_P", _f64p), p("und_off", _i32p), p("und_first", _i32p), p("und_len", _i32p),
            p("q_off", _i32p), p("q_und", _i32p), p("q_kind", _i32p), p("q_K", _f64p),
            p("q_vol", _f64p), p("q_w", _f64p), int(market["model"]), int(market["formula"]),
            int(market["residual"]), float(market["beta"]))
        h = ctypes.c_void_p()
        check(L.sabr_plan_create(ctypes.byref(self._prob), ctypes.byref(h)))
        self._h = h
        self.model = int(market["model"])
        self.formula = int(market["formula"])
        self.residual = int(market["residual"])
        self.P = int(L.sabr_plan_num_params(h))
        self.n_inst = int(L.sabr_plan_num_inst(h))
        self.max_q = int(L.sabr_plan_max_quotes(h))
        self.nq = np.diff(a["q_off"])
        nbytes = int(L.sabr_plan_device_bytes(h))
        self._dev = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        check(L.sabr_plan_upload(h, _ptr(self._dev), nbytes, _stream(stream, self._dev)))

    def __del__(self):
        h = getattr(self, "_h", None)
        try:
            if h is not None and _lib is not None and _lib._lib is not None:
                _lib._lib.sabr_plan_destroy(h)
        except Exception:  # interpreter shutdown: modules may be gone
            pass
        self._h = None

    # ------------------------------------------------------------------
    def underlyings(self):
        n = int(self._keep["und_off"][-1])
        S0, A, T = np.zeros(n), np.zeros(n), np.zeros(n)
        check(lib().sabr_plan_underlyings(self._h, S0.ctypes.data_as(_f64p),
                                          A.ctypes.data_as(_f64p), T.ctypes.data_as(_f64p)))
        return S0, A, T

    def _pts(self, params, pt_inst):
        params = torch.as_tensor(params, dtype=torch.float64, device=self.device)
        params = params.reshape(-1, self.P).contiguous()
        n = params.shape[0]
        if pt_inst is None:
            pt_inst = torch.zeros(n, dtype=torch.int32, device=self.device)
        else:
            pt_inst = torch.as_tensor(pt_inst, dtype=torch.int32, device=self.device).contiguous()
        return params, pt_inst, n

    def cost(self, params, pt_inst=None, resid=False, model=False, stream=None):
        """cost[n] (and optionally resid[n, max_q], model[n, max_q])."""
        params, pt_inst, n = self._pts(params, pt_inst)
        cost = torch.empty(n, dtype=torch.float64, device=self.device)
        r = torch.full((n, self.max_q), float("nan"), dtype=torch.float64,
                       device=self.device) if resid else None
        m = torch.full((n, self.max_q), float("nan"), dtype=torch.float64,
                       device=self.device) if model else None
        check(lib().sabr_cost_batch(self._h, n, _ptr(pt_inst), _ptr(params), _ptr(cost), _ptr(r),
                                    _ptr(m), self.max_q,
                                    _stream(stream, self._dev, params, pt_inst, cost, r, m)))
        out = [cost]
        if resid:
            out.append(r)
        if model:
            out.append(m)
        return out[0] if len(out) == 1 else tuple(out)

    # ------------------------------------------------------------------
    def sa_config(self, T0, cool, n_levels, n_steps, seed, step_frac=0.05, T0_per_inst=None,
                  waves=0, use_graph=False, level_events=None, occupancy=0, waves_per_chain=0,
                  chains_per_wave=0, level0=0, state_in=None, state_out=None):
        t0i = None
        if T0_per_inst is not None:
            t0i = np.ascontiguousarray(T0_per_inst, dtype=np.float64)
            self._keep["_t0i"] = t0i
        ev = None
        if level_events is not None:
            # torch.cuda.Event objects, created (recorded once) on the caller's stream
            # None entries (in pairs) skip a level
            ev = (ctypes.c_void_p * len(level_events))(
                *[e.cuda_event if e is not None else None for e in level_events])
            self._keep["_ev"] = ev
        return SAConfig(float(T0), float(cool), float(step_frac), int(n_levels), int(n_steps),
                        int(seed), t0i.ctypes.data_as(_f64p) if t0i is not None else None,
                        int(waves), 1 if use_graph else 0,
                        ctypes.cast(ev, ctypes.POINTER(ctypes.c_void_p)) if ev is not None
                        else None, int(occupancy), int(waves_per_chain), int(chains_per_wave),
                        int(level0), _ptr(state_in), _ptr(state_out))

    def sa_workspace_bytes(self, cfg, chains):
        ch = np.ascontiguousarray(np.broadcast_to(chains, (self.n_inst,)), dtype=np.int32)
        return int(lib().sa_workspace_size(self._h, ctypes.byref(cfg), ch.ctypes.data_as(_i32p)))

    def _sa_outputs(self, tot, n_levels, n_steps, record, trace, chain_best):
        n, P, dev = self.n_inst, self.P, self.device
        f64 = dict(dtype=torch.float64, device=dev)
        return dict(
            best_x=torch.empty((n, P), **f64),
            best_f=torch.empty(n, **f64),
            chain_best_x=torch.empty((tot, P), **f64) if chain_best else None,
            chain_best_f=torch.empty(tot, **f64) if chain_best else None,
            accept=torch.empty(int(n_levels) * int(n_steps) * tot, dtype=torch.uint8,
                               device=dev) if record else None,
            trace=torch.zeros((n, int(n_levels), 3), **f64) if trace else None,
            level_best=torch.empty((n, int(n_levels)), dtype=torch.int32, device=dev)
            if record else None,
        )

    def sa(self, chains, lb, ub, T0, cool, n_levels, n_steps, seed, step_frac=0.05, x0=None,
           T0_per_inst=None, record=False, trace=True, chain_best=False, waves=0,
           use_graph=False, stream=None, workspace=None, out=None, level_events=None,
           occupancy=0, noalloc=False, waves_per_chain=0, chains_per_wave=0, level0=0,
           state_in=None, state_out=False):
        """Synchronous parallel simulated annealing on every instance.  ``out``
        (a dict returned by an earlier call with the same shapes) reuses its
        output tensors, so a captured graph can be replayed.  noalloc: run
        through sa_calibrate_noalloc (the library's fixed device scratch, no
        workspace; the returned "workspace" is None).  waves_per_chain > 1:
        each chain's quotes split over that many waves of one workgroup;
        chains_per_wave = 2 (GLOBAL4): two chains per wave, one per half.
        Resume: level0 is the first level's index; state_in (a float64 device
        tensor of state_doubles(chains) values, as a run with state_out=True
        returned in "state") replaces the evaluation of x0."""
        L = lib()
        n, P = self.n_inst, self.P
        cfg = self.sa_config(T0, cool, n_levels, n_steps, seed, step_frac, T0_per_inst, waves,
                             use_graph, level_events, occupancy, waves_per_chain,
                             chains_per_wave)
        ch = np.ascontiguousarray(np.broadcast_to(chains, (n,)), dtype=np.int32)
        lb = np.ascontiguousarray(np.broadcast_to(lb, (n, P)), dtype=np.float64)
        ub = np.ascontiguousarray(np.broadcast_to(ub, (n, P)), dtype=np.float64)
        x0a = None if x0 is None else np.ascontiguousarray(np.broadcast_to(x0, (n, P)),
                                                           dtype=np.float64)
        tot = int(ch.sum())
        out = dict(out) if out is not None else self._sa_outputs(tot, n_levels, n_steps,
                                                                  record, trace, chain_best)
        nst = self.state_doubles(ch)
        if state_in is not None and (state_in.dtype != torch.float64 or state_in.numel() != nst
                                     or not state_in.is_contiguous()):
            raise ValueError(f"state_in: a contiguous float64 tensor of {nst} values")
        if state_out and out.get("state") is None:
            out["state"] = torch.empty(nst, dtype=torch.float64, device=self.device)
        elif not state_out:
            out["state"] = None
        cfg.level0, cfg.state_in, cfg.state_out = int(level0), _ptr(state_in), _ptr(out["state"])
        o = out
        args = (lb.ctypes.data_as(_f64p), ub.ctypes.data_as(_f64p),
                x0a.ctypes.data_as(_f64p) if x0a is not None else None,
                _ptr(o["best_x"]), _ptr(o["best_f"]), _ptr(o["chain_best_x"]),
                _ptr(o["chain_best_f"]), _ptr(o["accept"]), _ptr(o["trace"]),
                _ptr(o["level_best"]))
        if noalloc:
            check(L.sa_calibrate_noalloc(
                self._h, ctypes.byref(cfg), ch.ctypes.data_as(_i32p), *args,
                _stream(stream, self._dev, state_in,
                        *[v for v in o.values() if isinstance(v, torch.Tensor)])))
            out["workspace"] = None
            out["n_evals"] = ch.astype(np.int64) * (int(state_in is None) +
                                                    int(n_steps) * int(n_levels))
            return out
        ws = int(L.sa_workspace_size(self._h, ctypes.byref(cfg), ch.ctypes.data_as(_i32p)))
        if ws == 0:
            check(-1 if L.sabr_last_error() else 0)
            raise _lib.SabrError("sa_workspace_size: " + L.sabr_last_error().decode())
        if workspace is None or workspace.numel() < ws:
            workspace = torch.empty(ws, dtype=torch.uint8, device=self.device)
        check(L.sa_calibrate(self._h, ctypes.byref(cfg), ch.ctypes.data_as(_i32p),
                             lb.ctypes.data_as(_f64p), ub.ctypes.data_as(_f64p),
                             x0a.ctypes.data_as(_f64p) if x0a is not None else None,
                             _ptr(o["best_x"]), _ptr(o["best_f"]), _ptr(o["chain_best_x"]),
                             _ptr(o["chain_best_f"]), _ptr(o["accept"]), _ptr(o["trace"]),
                             _ptr(o["level_best"]), _ptr(workspace), workspace.numel(),
                             _stream(stream, self._dev, workspace, state_in,
                                     *[v for v in o.values() if isinstance(v, torch.Tensor)])))
        out["workspace"] = workspace
        out["n_evals"] = ch.astype(np.int64) * (int(state_in is None) +
                                                int(n_steps) * int(n_levels))
        return out

    def state_doubles(self, chains):
        """Doubles of an annealing state (sa_config.state_in/state_out) for
        these chain counts: 2 C (P + 1) + 1 per instance."""
        ch = np.broadcast_to(np.asarray(chains, dtype=np.int64), (self.n_inst,))
        return int(np.sum(2 * ch * (self.P + 1) + 1))

    # ------------------------------------------------------------------
    def _adj_workspace(self, n, workspace=None):
        ws = int(lib().sabr_adjoint_workspace_size(self._h, n))
        if workspace is None or workspace.numel() < ws:
            workspace = torch.empty(max(ws, 256), dtype=torch.uint8, device=self.device)
        return workspace

    def vjp(self, params, pt_inst=None, g_cost=None, normal=False, stream=None, workspace=None,
            want_jtwr=False):
        """Hand-written adjoint: dict(cost, grad = g_cost * d cost/d p, and with
        normal=True jtwj [n,P,P], jtwr [n,P]; want_jtwr: jtwr alone)."""
        params, pt_inst, n = self._pts(params, pt_inst)
        f64 = dict(dtype=torch.float64, device=self.device)
        cost = torch.empty(n, **f64)
        grad = torch.empty((n, self.P), **f64)
        jtwj = torch.empty((n, self.P, self.P), **f64) if normal else None
        jtwr = torch.empty((n, self.P), **f64) if (normal or want_jtwr) else None
        if g_cost is not None:
            g_cost = torch.as_tensor(g_cost, **f64).reshape(n).contiguous()
        check(lib().sabr_cost_vjp(self._h, n, _ptr(pt_inst), _ptr(params), _ptr(g_cost),
                                  _ptr(cost), _ptr(grad), _ptr(jtwj), _ptr(jtwr), None, 0,
                                  _stream(stream, self._dev, params, pt_inst, g_cost, cost, grad,
                                          jtwj, jtwr)))
        return dict(cost=cost, grad=grad, jtwj=jtwj, jtwr=jtwr)

    def lm(self, params, lb, ub, pt_inst=None, max_iter=50, mu0=1e-3, tol=1e-12, stream=None,
           workspace=None):
        """Projected Levenberg-Marquardt polish; returns (params, cost, iterations)."""
        params, pt_inst, n = self._pts(params, pt_inst)
        x = params.clone()
        lb = np.ascontiguousarray(np.broadcast_to(lb, (self.n_inst, self.P)), dtype=np.float64)
        ub = np.ascontiguousarray(np.broadcast_to(ub, (self.n_inst, self.P)), dtype=np.float64)
        cost = torch.empty(n, dtype=torch.float64, device=self.device)
        iters = torch.empty(n, dtype=torch.int32, device=self.device)
        ws = self._adj_workspace(n, workspace)
        check(lib().sabr_lm_polish(self._h, n, _ptr(pt_inst), _ptr(x), lb.ctypes.data_as(_f64p),
                                   ub.ctypes.data_as(_f64p), int(max_iter), float(mu0),
                                   float(tol), _ptr(cost), _ptr(iters), _ptr(ws), ws.numel(),
                                   _stream(stream, self._dev, pt_inst, x, cost, iters, ws)))
        return x, cost, iters

    def nm(self, params, lb, ub, pt_inst=None, max_iter=1000, step=0.05, tol=1e-12, stream=None,
           workspace=None):
        """Nelder-Mead polish (the paper's local minimizer, every model);
        returns (params, cost, iterations)."""
        params, pt_inst, n = self._pts(params, pt_inst)
        x = params.clone()
        lb = np.ascontiguousarray(np.broadcast_to(lb, (self.n_inst, self.P)), dtype=np.float64)
        ub = np.ascontiguousarray(np.broadcast_to(ub, (self.n_inst, self.P)), dtype=np.float64)
        cost = torch.empty(n, dtype=torch.float64, device=self.device)
        iters = torch.empty(n, dtype=torch.int32, device=self.device)
        need = int(lib().sabr_nm_workspace_size(self._h))
        if workspace is None or workspace.numel() < need:
            workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=self.device)
        check(lib().sabr_nm_polish(self._h, n, _ptr(pt_inst), _ptr(x), lb.ctypes.data_as(_f64p),
                                   ub.ctypes.data_as(_f64p), int(max_iter), float(step),
                                   float(tol), _ptr(cost), _ptr(iters), _ptr(workspace),
                                   workspace.numel(),
                                   _stream(stream, self._dev, pt_inst, x, cost, iters, workspace)))
        return x, cost, iters


class SabrCost(torch.autograd.Function):
    """cost = f(params) through sabr_cost_batch; backward through the
    hand-written adjoint sabr_cost_vjp."""

    @staticmethod
    def forward(ctx, params, plan, pt_inst):
        params = params.contiguous()
        cost = plan.cost(params, pt_inst)
        ctx.plan = plan
        ctx.save_for_backward(params, pt_inst)
        return cost

    @staticmethod
    def backward(ctx, g):
        params, pt_inst = ctx.saved_tensors
        out = ctx.plan.vjp(params, pt_inst, g_cost=g.contiguous())
        return out["grad"], None, None


def sabr_cost(plan: Plan, params, pt_inst=None):
    """Differentiable cost of points (torch.float64 [n, P] on the GPU)."""
    n = params.reshape(-1, plan.P).shape[0]
    if pt_inst is None:
        pt_inst = torch.zeros(n, dtype=torch.int32, device=plan.device)
    return SabrCost.apply(params.reshape(-1, plan.P), plan, pt_inst)


class McProblem:
    """A validated Monte Carlo pricing problem (host only: the plan and its
    correlation factor; see sabr_mc_plan_create)."""

    def __init__(self, prob: dict):
        L = lib()
        self._keep = {k: np.ascontiguousarray(prob[k], dtype=np.float64)
                      for k in ("T", "tau", "F0", "alpha", "beta", "phi", "sigma", "opt_K")}
        for k in ("opt_a", "opt_b"):
            self._keep[k] = np.ascontiguousarray(prob[k], dtype=np.int32)
        a = self._keep
        f = lambda k: a[k].ctypes.data_as(_lib._f64p)
        y = [float(v) for v in prob["y"]]
        self.M = len(a["T"])
        self.n_opt = len(a["opt_a"])
        self._prob = SabrMcProblem(self.M, f("T"), f("tau"), f("F0"), f("alpha"), f("beta"),
                                   f("phi"), f("sigma"), *y, float(prob["P0"]), self.n_opt,
                                   a["opt_a"].ctypes.data_as(_lib._i32p),
                                   a["opt_b"].ctypes.data_as(_lib._i32p), f("opt_K"))
        h = ctypes.c_void_p()
        check(L.sabr_mc_plan_create(ctypes.byref(self._prob), ctypes.byref(h)))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        try:
            if h is not None and _lib is not None and _lib._lib is not None:
                _lib._lib.sabr_mc_plan_destroy(h)
        except Exception:  # interpreter shutdown
            pass
        self._h = None

    def factor(self):
        B = np.zeros((2 * self.M, 2 * self.M))
        check(lib().sabr_mc_factor(self._h, B.ctypes.data_as(_lib._f64p)))
        return B


class McPlan(McProblem):
    """A Monte Carlo pricing problem uploaded to device memory.  Its calls
    share one workspace: issue them on one stream (or synchronise between
    streams), as concurrent calls would overwrite each other's sums."""

    def __init__(self, prob: dict, device: str = "cuda", stream=None):
        _require_gpu()
        super().__init__(prob)
        self.device = torch.device(device)
        nbytes = int(lib().sabr_mc_plan_device_bytes(self._h))
        self._dev = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        check(lib().sabr_mc_plan_upload(self._h, _ptr(self._dev), nbytes,
                                        _stream(stream, self._dev)))
        self._ws = None

    def workspace(self, n_paths):
        n = int(lib().sabr_mc_workspace_size(self._h, int(n_paths)))
        if self._ws is None or self._ws.numel() < n:
            self._ws = torch.empty(max(n, 256), dtype=torch.uint8, device=self.device)
        return self._ws, n

    def price(self, n_paths, dt, seed, stream=None):
        """(price, standard error) of every option, float64 device tensors."""
        price = torch.empty(self.n_opt, dtype=torch.float64, device=self.device)
        se = torch.empty(self.n_opt, dtype=torch.float64, device=self.device)
        ws, n = self.workspace(n_paths)
        check(lib().sabr_mc_price(self._h, int(n_paths), float(dt), int(seed), _ptr(price),
                                  _ptr(se), _ptr(ws), ws.numel(),
                                  _stream(stream, self._dev, price, se, ws)))
        return price, se

    def cost(self, n_paths, dt, seed, target, weight=None, stream=None):
        """The swaption cost sum_o w_o (price_o - target_o)^2 over the same
        paths as price(); returns (cost, price) as float64 device tensors."""
        target = torch.as_tensor(target, dtype=torch.float64, device=self.device).contiguous()
        w = None if weight is None else torch.as_tensor(weight, dtype=torch.float64,
                                                        device=self.device).contiguous()
        price = torch.empty(self.n_opt, dtype=torch.float64, device=self.device)
        cost = torch.empty(1, dtype=torch.float64, device=self.device)
        ws, n = self.workspace(n_paths)
        check(lib().sabr_mc_cost(self._h, int(n_paths), float(dt), int(seed), _ptr(target),
                                 _ptr(w), _ptr(price), _ptr(cost), _ptr(ws), ws.numel(),
                                 _stream(stream, self._dev, target, w, price, cost, ws)))
        return cost, price
