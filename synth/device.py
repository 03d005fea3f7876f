"""Device twin of the seeded generator: ctypes binding of libsynth.so.

Fills torch CUDA tensors with exactly the values that ``synth`` (numpy) returns
for the same logical indices.  Test and benchmark infrastructure.
"""
from __future__ import annotations

import ctypes
import os

import torch

from . import STREAM_AGE_A, STREAM_AGE_C, STREAM_FRAMES, STREAM_MEAN_A, STREAM_MEAN_C, \
    STREAM_VAR_A, STREAM_VAR_C, STREAM_GRAD_BG, STREAM_GRAD_STATE

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsynth.so")
_DT = {torch.float64: 0, torch.float32: 1, torch.bfloat16: 2}
UNIFORM, ABS_UNIFORM, NORMAL = 0, 1, 2

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run the build first")
        _lib = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
        _lib.synth_fill.argtypes = [vp, i32, i32, i64, i64, i64, i64, i64, u64, u64, vp]
        _lib.synth_ages.argtypes = [vp, i64, i32, u64, u64, vp]
        _lib.synth_video.argtypes = [vp, i32, i64, i64, i64, i64, i64, u64, vp]
        _lib.synth_probe_forward.argtypes = [vp, i32, i32, vp, vp, i64, i64, vp]
        _lib.synth_probe_backward.argtypes = [vp, vp, vp, i32, i64, i64, vp]
    return _lib


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def fill(t: torch.Tensor, seed: int, stream_id: int, kind: int = UNIFORM) -> torch.Tensor:
    """Fill a (T, H, W) or (H, W) tensor (last dim contiguous) in place."""
    v = t if t.dim() == 3 else t.unsqueeze(0)
    T, H, W = v.shape
    fs, rs, cs = v.stride()
    assert cs == 1 or W <= 1
    rc = lib().synth_fill(ctypes.c_void_p(v.data_ptr()), _DT[v.dtype], kind, T, H, W,
                          rs if H > 1 else W, fs if T > 1 else H * max(rs, W), seed, stream_id,
                          _stream())
    if rc != 0:
        raise RuntimeError(f"synth_fill failed ({rc})")
    return t


def ages(t: torch.Tensor, seed: int, stream_id: int, age_max: int) -> torch.Tensor:
    assert t.dtype == torch.uint8 and t.is_contiguous()
    rc = lib().synth_ages(ctypes.c_void_p(t.data_ptr()), t.numel(), age_max, seed, stream_id,
                          _stream())
    if rc != 0:
        raise RuntimeError(f"synth_ages failed ({rc})")
    return t


def frames(seed: int, T: int, H: int, W: int, dtype=torch.float64, device="cuda") -> torch.Tensor:
    return fill(torch.empty((T, H, W), dtype=dtype, device=device), seed, STREAM_FRAMES)


def video(seed: int, T: int, H: int, W: int, dtype=torch.float64, device="cuda") -> torch.Tensor:
    """The structured video of ``synth.video`` (values q/128, exact in every dtype)."""
    v = torch.empty((T, H, W), dtype=dtype, device=device)
    fs, rs, _ = v.stride()
    rc = lib().synth_video(ctypes.c_void_p(v.data_ptr()), _DT[dtype], T, H, W, rs if H > 1 else W,
                           fs if T > 1 else H * max(rs, W), seed, _stream())
    if rc != 0:
        raise RuntimeError(f"synth_video failed ({rc})")
    return v


def state(seed: int, H: int, W: int, dtype=torch.float64, age_max: int = 30, device="cuda"):
    """The random mid-run state of ``synth.state`` as a tuple of six device tensors
    (mean_a, var_a, mean_c, var_c, age_a, age_c)."""
    f = lambda s, k: fill(torch.empty((H, W), dtype=dtype, device=device), seed, s, k)
    a = lambda s: ages(torch.empty((H, W), dtype=torch.uint8, device=device), seed, s, age_max)
    return (f(STREAM_MEAN_A, UNIFORM), f(STREAM_VAR_A, ABS_UNIFORM), f(STREAM_MEAN_C, UNIFORM),
            f(STREAM_VAR_C, ABS_UNIFORM), a(STREAM_AGE_A), a(STREAM_AGE_C))


def grad_bg(seed: int, T: int, H: int, W: int, dtype=torch.float64, device="cuda") -> torch.Tensor:
    return fill(torch.empty((T, H, W), dtype=dtype, device=device), seed, STREAM_GRAD_BG, NORMAL)


def grad_state(seed: int, H: int, W: int, dtype=torch.float64, device="cuda") -> torch.Tensor:
    """(4, H, W): upstream gradient of the final (mean_a, var_a, mean_c, var_c)."""
    return fill(torch.empty((4, H, W), dtype=dtype, device=device), seed, STREAM_GRAD_STATE, NORMAL)


def probe_forward(frames: torch.Tensor, pixels_per_lane: int, masks: torch.Tensor,
                  sink: torch.Tensor) -> None:
    """The forward kernel's memory traffic with no model arithmetic (dense T x H x W)."""
    T = frames.shape[0]
    npx = frames[0].numel()
    assert frames.is_contiguous() and masks.is_contiguous() and masks.numel() == T * npx
    assert masks.dtype == torch.uint8 and sink.numel() >= 1
    rc = lib().synth_probe_forward(ctypes.c_void_p(frames.data_ptr()), frames.element_size(),
                                   pixels_per_lane, ctypes.c_void_p(masks.data_ptr()),
                                   ctypes.c_void_p(sink.data_ptr()), T, npx, _stream())
    if rc != 0:
        raise RuntimeError(f"synth_probe_forward failed ({rc})")


def probe_backward(x: torch.Tensor, g: torch.Tensor, gx: torch.Tensor) -> None:
    """The backward kernel's frame-sized traffic (x, g in; gx out) with no arithmetic."""
    T = x.shape[0]
    npx = x[0].numel()
    for t in (g, gx):
        assert t.is_contiguous() and t.shape == x.shape and t.dtype == x.dtype
    assert x.is_contiguous()
    rc = lib().synth_probe_backward(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(g.data_ptr()),
                                    ctypes.c_void_p(gx.data_ptr()), x.element_size(), T, npx,
                                    _stream())
    if rc != 0:
        raise RuntimeError(f"synth_probe_backward failed ({rc})")
