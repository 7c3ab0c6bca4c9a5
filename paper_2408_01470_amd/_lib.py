"""ctypes declarations of the C ABI in include/sabr.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsabr_hip.so")

_i32p = ctypes.POINTER(ctypes.c_int32)
_f64p = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_vp = ctypes.c_void_p


class SabrProblem(ctypes.Structure):
    _fields_ = [
        ("n_inst", ctypes.c_int32),
        ("fwd_off", _i32p), ("fwd_T", _f64p), ("fwd_tau", _f64p), ("fwd_F", _f64p),
        ("fwd_P", _f64p),
        ("und_off", _i32p), ("und_first", _i32p), ("und_len", _i32p),
        ("q_off", _i32p), ("q_und", _i32p), ("q_kind", _i32p),
        ("q_K", _f64p), ("q_vol", _f64p), ("q_w", _f64p),
        ("model", ctypes.c_int32), ("vol_formula", ctypes.c_int32), ("residual", ctypes.c_int32),
        ("beta", ctypes.c_double),
    ]


class SabrMcProblem(ctypes.Structure):
    _fields_ = [
        ("n_fwd", ctypes.c_int32),
        ("T", _f64p), ("tau", _f64p), ("F0", _f64p), ("alpha", _f64p), ("beta", _f64p),
        ("phi", _f64p), ("sigma", _f64p),
        ("eta1", ctypes.c_double), ("lambda1", ctypes.c_double), ("eta2", ctypes.c_double),
        ("lambda2", ctypes.c_double), ("lambda3", ctypes.c_double), ("P0", ctypes.c_double),
        ("n_opt", ctypes.c_int32), ("opt_a", _i32p), ("opt_b", _i32p), ("opt_K", _f64p),
    ]


class SAConfig(ctypes.Structure):
    _fields_ = [
        ("T0", ctypes.c_double), ("cool", ctypes.c_double), ("step_frac", ctypes.c_double),
        ("n_levels", ctypes.c_int32), ("n_steps", ctypes.c_int32), ("seed", ctypes.c_uint64),
        ("T0_per_inst", _f64p), ("waves_per_group", ctypes.c_int32),
        ("use_graph", ctypes.c_int32), ("level_events", ctypes.POINTER(ctypes.c_void_p)),
        ("occupancy", ctypes.c_int32), ("waves_per_chain", ctypes.c_int32),
        ("chains_per_wave", ctypes.c_int32), ("level0", ctypes.c_int32),
        ("state_in", ctypes.c_void_p), ("state_out", ctypes.c_void_p),   # device pointers
    ]


SA_NOALLOC_MAX_BYTES = 64 << 20   # include/sabr.h

_lib = None


class LibraryMissing(RuntimeError):
    pass


def lib():
    """Load the in-tree HIP library; fail loudly if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LibraryMissing(
            f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; "
            "g.build()'` (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    L.sabr_last_error.restype = ctypes.c_char_p
    L.sabr_shutdown.restype = ctypes.c_int32
    L.sabr_shutdown.argtypes = []
    L.sabr_plan_create.argtypes = [ctypes.POINTER(SabrProblem), ctypes.POINTER(_vp)]
    L.sabr_plan_destroy.argtypes = [_vp]
    L.sabr_plan_destroy.restype = None
    L.sabr_plan_device_bytes.argtypes = [_vp]
    L.sabr_plan_device_bytes.restype = ctypes.c_size_t
    L.sabr_plan_upload.argtypes = [_vp, _vp, ctypes.c_size_t, _vp]
    L.sabr_num_params.argtypes = [ctypes.c_int32]
    for f in ("sabr_plan_num_params", "sabr_plan_num_inst", "sabr_plan_max_quotes"):
        getattr(L, f).argtypes = [_vp]
    L.sabr_plan_underlyings.argtypes = [_vp, _f64p, _f64p, _f64p]
    L.sabr_cost_batch.argtypes = [_vp, ctypes.c_int32, _vp, _vp, _vp, _vp, _vp, ctypes.c_int32,
                                  _vp]
    L.sa_workspace_size.argtypes = [_vp, ctypes.POINTER(SAConfig), _i32p]
    L.sa_workspace_size.restype = ctypes.c_size_t
    L.sa_calibrate.argtypes = [_vp, ctypes.POINTER(SAConfig), _i32p, _f64p, _f64p, _f64p,
                               _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
    L.sa_calibrate_noalloc.argtypes = [_vp, ctypes.POINTER(SAConfig), _i32p, _f64p, _f64p,
                                       _f64p, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
    L.sabr_adjoint_workspace_size.argtypes = [_vp, ctypes.c_int32]
    L.sabr_adjoint_workspace_size.restype = ctypes.c_size_t
    L.sabr_cost_vjp.argtypes = [_vp, ctypes.c_int32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                ctypes.c_size_t, _vp]
    L.sabr_lm_polish.argtypes = [_vp, ctypes.c_int32, _vp, _vp, _f64p, _f64p, ctypes.c_int32,
                                 ctypes.c_double, ctypes.c_double, _vp, _vp, _vp,
                                 ctypes.c_size_t, _vp]
    L.sabr_nm_workspace_size.argtypes = [_vp]
    L.sabr_nm_workspace_size.restype = ctypes.c_size_t
    L.sabr_nm_polish.argtypes = [_vp, ctypes.c_int32, _vp, _vp, _f64p, _f64p, ctypes.c_int32,
                                 ctypes.c_double, ctypes.c_double, _vp, _vp, _vp,
                                 ctypes.c_size_t, _vp]
    L.sabr_mc_plan_create.argtypes = [ctypes.POINTER(SabrMcProblem), ctypes.POINTER(_vp)]
    L.sabr_mc_plan_destroy.argtypes = [_vp]
    L.sabr_mc_plan_destroy.restype = None
    L.sabr_mc_plan_device_bytes.argtypes = [_vp]
    L.sabr_mc_plan_device_bytes.restype = ctypes.c_size_t
    L.sabr_mc_plan_upload.argtypes = [_vp, _vp, ctypes.c_size_t, _vp]
    L.sabr_mc_factor.argtypes = [_vp, _f64p]
    L.sabr_mc_workspace_size.argtypes = [_vp, ctypes.c_int64]
    L.sabr_mc_workspace_size.restype = ctypes.c_size_t
    L.sabr_mc_price.argtypes = [_vp, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64, _vp, _vp,
                                _vp, ctypes.c_size_t, _vp]
    L.sabr_mc_cost.argtypes = [_vp, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64, _vp, _vp,
                               _vp, _vp, _vp, ctypes.c_size_t, _vp]
    _lib = L
    return _lib


class SabrError(RuntimeError):
    pass


def check(rc: int) -> None:
    if rc != 0:
        raise SabrError(f"sabr status {rc}: {lib().sabr_last_error().decode()}")
