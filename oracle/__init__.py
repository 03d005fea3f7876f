"""CPU oracle of the Dual-Mode Single Gaussian Model update (TEST INFRASTRUCTURE).

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline leg
may import this package.  The GPU library never calls it and shares no code
with it.

Two implementations, both written from the paper (Henderson & Vertescher,
arXiv:1702.05156, Sec. 2.2-2.3 and the appendix's inner-update listing):

* ``liboracle.so`` (``dsgm_oracle.c``): plain scalar FP64 C, forward, forced
  decisions, decision margins, reverse-mode and forward-mode derivatives.
* ``oracle.exact``: the same steps in exact rational arithmetic (fractions),
  for tiny inputs.

Parameter readings (see ``dsgm_oracle.c`` for the list): the weight rule,
the mask reference, the age cap as min(a+1, age_max), no fused multiply-add.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

WEIGHT_EQ, WEIGHT_APPENDIX = 0, 1
MASK_VARIANCE, MASK_PRINTED = 0, 1
HIT_A, HIT_C, RESET, SWAP, FG = 1, 2, 4, 8, 16


@dataclass
class Params:
    theta_s: float = 2.0
    theta_d: float = 4.0
    var_init: float = 255.0
    var_floor: float = 0.1
    mask_floor: float = 0.25
    age_max: int = 30
    weight_rule: int = WEIGHT_EQ
    mask_rule: int = MASK_VARIANCE


def default_params(intensity_range: float = 255.0, mask_rule: int = MASK_VARIANCE) -> Params:
    """The paper's constants on an intensity scale of width ``intensity_range``.

    The paper works on 8-bit intensities: initial variance 255 (Sec. 2.3), age
    cap 30 (Sec. 2.2), variance floor 0.1 and background floor 0.25 (appendix).
    Variances scale with the square of the intensity scale s = range/255; the
    printed background rule floors an intensity, which scales with s.  The paper
    prints no values for theta_s and theta_d; 2 and 4 are assumed.
    """
    s = intensity_range / 255.0
    return Params(theta_s=2.0, theta_d=4.0, var_init=255.0 * s * s, var_floor=0.1 * s * s,
                  mask_floor=(0.25 * s * s if mask_rule == MASK_VARIANCE else 0.25 * s),
                  age_max=30, weight_rule=WEIGHT_EQ, mask_rule=mask_rule)


class _CParams(ctypes.Structure):
    _fields_ = [("theta_s", ctypes.c_double), ("theta_d", ctypes.c_double),
                ("var_init", ctypes.c_double), ("var_floor", ctypes.c_double),
                ("mask_floor", ctypes.c_double), ("age_max", ctypes.c_int32),
                ("weight_rule", ctypes.c_int32), ("mask_rule", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        _lib = ctypes.CDLL(LIB_PATH)
        dp = ctypes.c_void_p
        _lib.orc_forward.argtypes = [ctypes.c_int64, ctypes.c_int64] + [dp] * 13 + [ctypes.c_int]
        _lib.orc_backward.argtypes = [ctypes.c_int64, ctypes.c_int64] + [dp] * 14 + [ctypes.c_int]
        _lib.orc_jvp.argtypes = ([ctypes.c_int64, ctypes.c_int64] + [dp] * 11 +
                                 [ctypes.c_double, dp, dp, ctypes.c_int])
        _lib.orc_max_threads.restype = ctypes.c_int
        _lib.orc_warp_state.argtypes = [ctypes.c_int64, ctypes.c_int64] + [dp] * 9 + \
            [dp] * 6 + [ctypes.c_int]
        _lib.orc_warp_state.restype = ctypes.c_int
        _lib.orc_forward_grid.argtypes = ([ctypes.c_int64] * 3 + [ctypes.c_int32] + [dp] * 10 +
                                          [ctypes.c_int])
        _lib.orc_forward_grid.restype = ctypes.c_int
        _lib.orc_forward_u8.argtypes = [ctypes.c_int64, ctypes.c_int64] + [dp] * 10 + [ctypes.c_int]
        _lib.orc_forward_u8.restype = ctypes.c_int
        _lib.orc_gauss_weights.argtypes = [ctypes.c_int32, ctypes.c_double, dp]
        _lib.orc_gauss_weights.restype = ctypes.c_int
        _lib.orc_preprocess.argtypes = ([ctypes.c_int64] * 3 + [dp, dp, ctypes.c_int32, dp,
                                        ctypes.c_int32, ctypes.c_int])
        _lib.orc_preprocess.restype = ctypes.c_int
        _lib.orc_preprocess_u8.argtypes = ([ctypes.c_int64] * 3 + [dp, dp, ctypes.c_int32, dp,
                                           ctypes.c_int32, ctypes.c_int])
        _lib.orc_preprocess_u8.restype = ctypes.c_int
        for f in (_lib.orc_forward, _lib.orc_backward, _lib.orc_jvp):
            f.restype = ctypes.c_int
    return _lib


def max_threads() -> int:
    return int(lib().orc_max_threads())


def _cp(p: Params) -> _CParams:
    return _CParams(p.theta_s, p.theta_d, p.var_init, p.var_floor, p.mask_floor,
                    p.age_max, p.weight_rule, p.mask_rule)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _state_arrays(state: dict, N: int):
    return (_f64(state["mean_a"], (N,)).copy(), _f64(state["var_a"], (N,)).copy(),
            np.ascontiguousarray(state["age_a"], dtype=np.int32).reshape(N).copy(),
            _f64(state["mean_c"], (N,)).copy(), _f64(state["var_c"], (N,)).copy(),
            np.ascontiguousarray(state["age_c"], dtype=np.int32).reshape(N).copy())


def forward(frames, state: dict, params: Params, *, bg=True, codes=True, forced=None,
            margins=False, nthreads: int = 0) -> dict:
    """Run T frames over N pixels.  ``frames`` has shape (T, N) (or (T, H, W)).

    Returns a dict with the final state (same keys as ``state``), ``masks``
    (uint8 0/255), and optionally ``bg`` (apparent mean after each frame),
    ``codes`` (decision bits) and ``margins`` (T, N, 3).
    """
    x = np.asarray(frames)
    T = x.shape[0]
    N = int(np.prod(x.shape[1:])) if x.ndim > 1 else 0
    x = _f64(x, (T, N))
    mA, vA, aA, mC, vC, aC = _state_arrays(state, N)
    out_masks = np.empty((T, N), np.uint8)
    out_bg = np.empty((T, N), np.float64) if bg else None
    out_codes = np.empty((T, N), np.uint8) if codes else None
    out_marg = np.empty((T, N, 3), np.float64) if margins else None
    f = None if forced is None else np.ascontiguousarray(forced, dtype=np.uint8).reshape(T, N)
    cp = _cp(params)
    rc = lib().orc_forward(T, N, _ptr(x), _ptr(mA), _ptr(vA), _ptr(aA), _ptr(mC), _ptr(vC),
                           _ptr(aC), ctypes.byref(cp), _ptr(out_masks), _ptr(out_bg),
                           _ptr(out_codes), _ptr(f), _ptr(out_marg), int(nthreads))
    if rc != 0:
        raise ValueError(f"orc_forward failed ({rc})")
    res = {"mean_a": mA, "var_a": vA, "age_a": aA, "mean_c": mC, "var_c": vC, "age_c": aC,
           "masks": out_masks}
    if bg:
        res["bg"] = out_bg
    if codes:
        res["codes"] = out_codes
    if margins:
        res["margins"] = out_marg
    return res


def backward(frames, state0: dict, params: Params, grad_bg=None, grad_state_T=None, *,
             forced=None, nthreads: int = 0) -> dict:
    """Reverse-mode derivative with the decisions held fixed.

    Returns ``grad_frames`` (T, N), ``grad_state0`` (4, N) for (mean_a, var_a,
    mean_c, var_c), ``grad_var_init`` (float, compensated sum over pixels) and
    ``grad_var_init_px`` (N,).
    """
    x = np.asarray(frames)
    T = x.shape[0]
    N = int(np.prod(x.shape[1:])) if x.ndim > 1 else 0
    x = _f64(x, (T, N))
    mA, vA, aA, mC, vC, aC = _state_arrays(state0, N)
    gbg = None if grad_bg is None else _f64(grad_bg, (T, N))
    gsT = None if grad_state_T is None else _f64(grad_state_T, (4, N))
    f = None if forced is None else np.ascontiguousarray(forced, dtype=np.uint8).reshape(T, N)
    gx = np.empty((T, N), np.float64)
    gs0 = np.empty((4, N), np.float64)
    gvi = np.empty((N,), np.float64)
    cp = _cp(params)
    rc = lib().orc_backward(T, N, _ptr(x), _ptr(mA), _ptr(vA), _ptr(aA), _ptr(mC), _ptr(vC),
                            _ptr(aC), ctypes.byref(cp), _ptr(f), _ptr(gbg), _ptr(gsT), _ptr(gx),
                            _ptr(gs0), _ptr(gvi), int(nthreads))
    if rc != 0:
        raise ValueError(f"orc_backward failed ({rc})")
    return {"grad_frames": gx, "grad_state0": gs0, "grad_var_init": math.fsum(gvi.tolist()),
            "grad_var_init_px": gvi}


def jvp(frames, state0: dict, params: Params, dframes, dstate0, dvar_init: float = 0.0, *,
        forced=None, nthreads: int = 0) -> dict:
    """Forward-mode derivative with the decisions held fixed."""
    x = np.asarray(frames)
    T = x.shape[0]
    N = int(np.prod(x.shape[1:])) if x.ndim > 1 else 0
    x = _f64(x, (T, N))
    mA, vA, aA, mC, vC, aC = _state_arrays(state0, N)
    dx = _f64(dframes, (T, N))
    ds0 = _f64(dstate0, (4, N))
    f = None if forced is None else np.ascontiguousarray(forced, dtype=np.uint8).reshape(T, N)
    dbg = np.empty((T, N), np.float64)
    dsT = np.empty((4, N), np.float64)
    cp = _cp(params)
    rc = lib().orc_jvp(T, N, _ptr(x), _ptr(mA), _ptr(vA), _ptr(aA), _ptr(mC), _ptr(vC), _ptr(aC),
                       ctypes.byref(cp), _ptr(f), _ptr(dx), _ptr(ds0), float(dvar_init),
                       _ptr(dbg), _ptr(dsT), int(nthreads))
    if rc != 0:
        raise ValueError(f"orc_jvp failed ({rc})")
    return {"dbg": dbg, "dstate_T": dsT}


# ------------------------------------------------------------- preprocessing
def gauss_weights(n: int, sigma: float) -> np.ndarray:
    """Normalised Gaussian weights of length n (odd), Sec. 2.1 density sampled
    at integer offsets from the centre (preprocess_oracle.c)."""
    w = np.empty(n, np.float64)
    if lib().orc_gauss_weights(int(n), float(sigma), _ptr(w)) != 0:
        raise ValueError("orc_gauss_weights: bad arguments")
    return w


def preprocess(frames, weights=None, median: bool = True, nthreads: int = 0) -> np.ndarray:
    """Separable blur with `weights` (rows, then columns; None = no blur), then
    the 3 x 3 median (if `median`), borders clamped; frames (T, H, W) -> same."""
    x = np.ascontiguousarray(frames, dtype=np.float64)
    if x.ndim == 2:
        x = x[None]
    T, H, W = x.shape
    out = np.empty_like(x)
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
    n = 0 if w is None else int(w.size)
    rc = lib().orc_preprocess(T, H, W, _ptr(x), _ptr(out), n, _ptr(w), int(bool(median)),
                              int(nthreads))
    if rc != 0:
        raise ValueError(f"orc_preprocess failed ({rc})")
    return out


def preprocess_u8(frames, weights=None, median: bool = True, nthreads: int = 0) -> np.ndarray:
    """The appendix's 8-bit preprocessing (preprocess_oracle.c,
    orc_preprocess_u8): a two-dimensional single-precision blur with the
    window weights float(w_i * w_j), written back to 8 bits by dropping the
    fraction, then the 3 x 3 median of the 8-bit image (None = no blur);
    uint8 frames (T, H, W) -> same."""
    x = np.ascontiguousarray(frames, dtype=np.uint8)
    if x.ndim == 2:
        x = x[None]
    T, H, W = x.shape
    out = np.empty_like(x)
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
    n = 0 if w is None else int(w.size)
    rc = lib().orc_preprocess_u8(T, H, W, _ptr(x), _ptr(out), n, _ptr(w), int(bool(median)),
                                 int(nthreads))
    if rc != 0:
        raise ValueError(f"orc_preprocess_u8 failed ({rc})")
    return out


# ------------------------------------------------------------ motion compensation
def warp_state(state: dict, frame, inv_map, params: Params, H: int, W: int,
               nthreads: int = 0) -> dict:
    """The model after motion compensation (dsgm_oracle.c, orc_warp_state):
    `inv_map` (3 x 3) takes a current pixel (column, row, 1) to its position in
    the previous frame; bilinear means and variances, nearest ages, uncovered
    pixels restarted from `frame` (H*W values)."""
    N = H * W
    mA, vA, aA, mC, vC, aC = _state_arrays(state, N)
    m = np.ascontiguousarray(inv_map, dtype=np.float64).reshape(9)
    x = _f64(frame, (N,))
    out = {k: np.empty(N, np.float64) for k in ("mean_a", "var_a", "mean_c", "var_c")}
    out["age_a"] = np.empty(N, np.int32)
    out["age_c"] = np.empty(N, np.int32)
    cp = _cp(params)
    rc = lib().orc_warp_state(H, W, _ptr(m), _ptr(x), _ptr(mA), _ptr(vA), _ptr(aA), _ptr(mC),
                              _ptr(vC), _ptr(aC), ctypes.byref(cp), _ptr(out["mean_a"]),
                              _ptr(out["var_a"]), _ptr(out["age_a"]), _ptr(out["mean_c"]),
                              _ptr(out["var_c"]), _ptr(out["age_c"]), int(nthreads))
    if rc != 0:
        raise ValueError(f"orc_warp_state failed ({rc})")
    return out


# --------------------------------------------------------------- grid model
def forward_grid(frames, state: dict, params: Params, block: int, *, codes=True,
                 nthreads: int = 0) -> dict:
    """Yi et al.'s grid model (blocks of block x block pixels; dsgm_oracle.c,
    orc_forward_grid).  frames (T, H, W); state arrays hold Hb x Wb blocks.
    Returns the final state, masks (T, H, W) and codes (T, Hb*Wb)."""
    x = np.ascontiguousarray(frames, dtype=np.float64)
    T, H, W = x.shape
    Hb, Wb = -(-H // block), -(-W // block)
    mA, vA, aA, mC, vC, aC = _state_arrays(state, Hb * Wb)
    masks = np.empty((T, H, W), np.uint8)
    cd = np.empty((T, Hb * Wb), np.uint8) if codes else None
    cp = _cp(params)
    rc = lib().orc_forward_grid(T, H, W, int(block), _ptr(x), _ptr(mA), _ptr(vA), _ptr(aA),
                                _ptr(mC), _ptr(vC), _ptr(aC), ctypes.byref(cp), _ptr(masks),
                                _ptr(cd), int(nthreads))
    if rc != 0:
        raise ValueError(f"orc_forward_grid failed ({rc})")
    res = {"mean_a": mA, "var_a": vA, "age_a": aA, "mean_c": mC, "var_c": vC, "age_c": aC,
           "masks": masks}
    if codes:
        res["codes"] = cd
    return res


# ------------------------------------------------------- 8-bit as-run model
def forward_u8(frames, state: dict, params: Params, *, codes=True, nthreads: int = 0) -> dict:
    """The appendix's 8-bit as-run model (dsgm_oracle.c, orc_forward_u8):
    uint8 frames (T, N); state means/variances uint8, ages int."""
    x = np.ascontiguousarray(frames, dtype=np.uint8)
    T = x.shape[0]
    N = int(np.prod(x.shape[1:])) if x.ndim > 1 else 0
    x = x.reshape(T, N)
    u8 = lambda k: np.ascontiguousarray(state[k], dtype=np.uint8).reshape(N).copy()
    i32 = lambda k: np.ascontiguousarray(state[k], dtype=np.int32).reshape(N).copy()
    mA, vA, mC, vC, aA, aC = u8("mean_a"), u8("var_a"), u8("mean_c"), u8("var_c"), i32("age_a"), i32("age_c")
    masks = np.empty((T, N), np.uint8)
    cd = np.empty((T, N), np.uint8) if codes else None
    cp = _cp(params)
    rc = lib().orc_forward_u8(T, N, _ptr(x), _ptr(mA), _ptr(vA), _ptr(aA), _ptr(mC), _ptr(vC),
                              _ptr(aC), ctypes.byref(cp), _ptr(masks), _ptr(cd), int(nthreads))
    if rc != 0:
        raise ValueError(f"orc_forward_u8 failed ({rc})")
    res = {"mean_a": mA, "var_a": vA, "age_a": aA, "mean_c": mC, "var_c": vC, "age_c": aC,
           "masks": masks}
    if codes:
        res["codes"] = cd
    return res
