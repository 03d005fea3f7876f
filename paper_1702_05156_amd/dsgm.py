"""ctypes binding of libdsgm.so (argument marshalling only).

Every function named ``dsgm_*`` here is the C entry point of the same name in
``include/dsgm.h``: it takes torch tensors, checks that they are CUDA (HIP)
tensors of the right dtype and layout, and passes their device pointers, the
sizes and strides, and the current HIP stream.  All computation happens in the
library's kernels; if the library is missing, importing this module fails.

PyTorch is used for device memory and streams only.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdsgm.so")

DSGM_OK = 0
STATUS = {0: "DSGM_OK", -1: "DSGM_E_ARG", -2: "DSGM_E_SHAPE", -3: "DSGM_E_DTYPE",
          -4: "DSGM_E_ALIGN", -5: "DSGM_E_WORKSPACE", -6: "DSGM_E_HIP", -7: "DSGM_E_UNSUPPORTED"}
IN_F64, IN_F32, IN_BF16, IN_U8 = 0, 1, 2, 3
ACC_F64, ACC_F32, ACC_F64_IO32, ACC_U8, ACC_F32X2 = 0, 1, 2, 3, 4
WEIGHT_EQ, WEIGHT_APPENDIX = 0, 1
MASK_VARIANCE, MASK_PRINTED = 0, 1
CODE_HIT_A, CODE_HIT_C, CODE_RESET, CODE_SWAP, CODE_FG = 1, 2, 4, 8, 16

_IN_DTYPES = {torch.float64: IN_F64, torch.float32: IN_F32, torch.bfloat16: IN_BF16,
              torch.uint8: IN_U8}
# F32X2 state planes are complex64 tensors: the (hi, lo) float pairs of the
# library's layout, hi in the real part and lo in the imaginary part
_ACC_DTYPES = {torch.float64: ACC_F64, torch.float32: ACC_F32, torch.uint8: ACC_U8,
               torch.complex64: ACC_F32X2}
# dtype of bg and of the gradient arrays, and of the model state, per dsgm_acc
ACC_TORCH = {ACC_F64: torch.float64, ACC_F32: torch.float32, ACC_F64_IO32: torch.float32,
             ACC_U8: torch.uint8, ACC_F32X2: torch.float32}
STATE_TORCH = {ACC_F64: torch.float64, ACC_F32: torch.float32, ACC_F64_IO32: torch.float64,
               ACC_U8: torch.uint8, ACC_F32X2: torch.complex64}


def x2_from_f64(t: torch.Tensor) -> torch.Tensor:
    """The nearest (hi, lo) float pairs of a float64 tensor, as complex64:
    hi = fl32(t), lo = fl32(t - hi); hi + lo is exact in float64."""
    hi = t.to(torch.float32)
    lo = (t - hi.double()).to(torch.float32)
    return torch.complex(hi, lo)


def x2_to_f64(t: torch.Tensor) -> torch.Tensor:
    """hi + lo of complex64 pairs, in float64 (exact)."""
    return t.real.double() + t.imag.double()


class DSGMError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__(f"{fn}: {STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    """dsgm_params (host struct)."""
    _fields_ = [("theta_s", ctypes.c_double), ("theta_d", ctypes.c_double),
                ("var_init", ctypes.c_double), ("var_floor", ctypes.c_double),
                ("mask_floor", ctypes.c_double), ("age_max", ctypes.c_int32),
                ("weight_rule", ctypes.c_int32), ("mask_rule", ctypes.c_int32)]

    def __repr__(self):
        return "Params(" + ", ".join(f"{n}={getattr(self, n)!r}" for n, _ in self._fields_) + ")"


class Shape(ctypes.Structure):
    _fields_ = [("T", ctypes.c_int64), ("H", ctypes.c_int64), ("W", ctypes.c_int64),
                ("row_stride", ctypes.c_int64), ("frame_stride", ctypes.c_int64)]


class Filter(ctypes.Structure):
    """dsgm_filter (host struct): n-tap separable blur, then an optional 3 x 3 median."""
    _fields_ = [("n", ctypes.c_int32), ("median", ctypes.c_int32),
                ("weights", ctypes.c_double * 7)]


class _State(ctypes.Structure):
    _fields_ = [("mean_a", ctypes.c_void_p), ("var_a", ctypes.c_void_p),
                ("mean_c", ctypes.c_void_p), ("var_c", ctypes.c_void_p),
                ("age_a", ctypes.c_void_p), ("age_c", ctypes.c_void_p)]


class _GradState(ctypes.Structure):
    _fields_ = [("mean_a", ctypes.c_void_p), ("var_a", ctypes.c_void_p),
                ("mean_c", ctypes.c_void_p), ("var_c", ctypes.c_void_p)]


class Instance(ctypes.Structure):
    """dsgm_instance"""
    _fields_ = [("shape", Shape), ("frames", ctypes.c_void_p), ("state", _State),
                ("masks", ctypes.c_void_p), ("bg", ctypes.c_void_p),
                ("fg_counts", ctypes.c_void_p)]


class BatchPlan(ctypes.Structure):
    """dsgm_batch_plan (host handle)"""
    _fields_ = [("device_plan", ctypes.c_void_p), ("n_items", ctypes.c_int64),
                ("total_elements", ctypes.c_int64), ("n_instances", ctypes.c_int32),
                ("in_dtype", ctypes.c_int32), ("acc", ctypes.c_int32), ("vector", ctypes.c_int32),
                ("grid", ctypes.c_int32), ("has_bg", ctypes.c_int32),
                ("has_counts", ctypes.c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.dsgm_params_default.argtypes = [ctypes.POINTER(Params), ctypes.c_double, i32]
    lib.dsgm_state_init_from_frame.argtypes = [vp, i32, Shape, i32, ctypes.POINTER(Params),
                                               ctypes.POINTER(_State), vp]
    sz = ctypes.c_size_t
    lib.dsgm_forward.argtypes = [vp, i32, Shape, i32, ctypes.POINTER(Params),
                                 ctypes.POINTER(_State), vp, vp, vp, sz, i32, vp, vp]
    lib.dsgm_gauss_weights.argtypes = [i32, ctypes.c_double, ctypes.POINTER(ctypes.c_double)]
    lib.dsgm_forward_filtered.argtypes = [vp, i32, Shape, i32, ctypes.POINTER(Params),
                                          ctypes.POINTER(Filter), ctypes.POINTER(_State), vp, vp,
                                          vp, vp, vp]
    lib.dsgm_forward_warped.argtypes = [vp, i32, Shape, i32, ctypes.POINTER(Params),
                                        ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_State),
                                        ctypes.POINTER(_State), vp, vp, vp, vp]
    lib.dsgm_forward_grid.argtypes = [vp, i32, Shape, i32, ctypes.POINTER(Params), i32,
                                      ctypes.POINTER(_State), vp, vp, vp, vp]
    lib.dsgm_ckpt_bytes.argtypes = [Shape, i32, i32]
    lib.dsgm_ckpt_bytes.restype = ctypes.c_size_t
    lib.dsgm_workspace_bytes.argtypes = [Shape, i32]
    lib.dsgm_workspace_bytes.restype = ctypes.c_size_t
    lib.dsgm_backward.argtypes = [vp, i32, Shape, i32, ctypes.POINTER(Params), vp, sz, i32, vp,
                                  ctypes.POINTER(_GradState), vp, ctypes.POINTER(_GradState), vp,
                                  vp, sz, vp]
    lib.dsgm_backward_noalloc.argtypes = [vp, i32, Shape, i32, ctypes.POINTER(Params), vp, sz,
                                          i32, vp, ctypes.POINTER(_GradState), vp,
                                          ctypes.POINTER(_GradState), vp, vp]
    lib.dsgm_batch_plan_bytes.argtypes = [ctypes.POINTER(Instance), i32, i32, i32]
    lib.dsgm_batch_plan_bytes.restype = ctypes.c_size_t
    lib.dsgm_plan_batched.argtypes = [ctypes.POINTER(Instance), i32, i32, i32, vp, ctypes.c_size_t,
                                      ctypes.POINTER(BatchPlan), vp]
    lib.dsgm_forward_batched.argtypes = [ctypes.POINTER(BatchPlan), ctypes.POINTER(Params), vp]
    lib.dsgm_status_string.argtypes = [ctypes.c_int]
    lib.dsgm_status_string.restype = ctypes.c_char_p
    lib.dsgm_last_error.restype = ctypes.c_char_p
    lib.dsgm_set_launch.argtypes = [i32, i32]
    lib.dsgm_count_nonfinite.argtypes = [vp, i32, Shape, vp, vp]
    lib.dsgm_autotune_bytes.argtypes = [i32, i32, Shape, i32]
    lib.dsgm_autotune_bytes.restype = ctypes.c_size_t
    lib.dsgm_autotune.argtypes = [i32, i32, Shape, i32, vp, ctypes.c_size_t,
                                  ctypes.POINTER(ctypes.c_int32), vp]
    lib.dsgm_autotune_lookup.argtypes = [i32, i32, Shape, i32, ctypes.POINTER(ctypes.c_int32)]
    lib.dsgm_autotune_clear.argtypes = []
    for f in ("dsgm_params_default", "dsgm_state_init_from_frame", "dsgm_forward",
              "dsgm_backward", "dsgm_backward_noalloc", "dsgm_plan_batched", "dsgm_forward_batched", "dsgm_version",
              "dsgm_set_launch", "dsgm_gauss_weights", "dsgm_forward_filtered",
              "dsgm_forward_warped", "dsgm_forward_grid", "dsgm_autotune",
              "dsgm_autotune_lookup", "dsgm_autotune_clear", "dsgm_count_nonfinite"):
        getattr(lib, f).restype = ctypes.c_int
    del i64
    return lib


lib = _load()

# names of every C entry point declared in include/dsgm.h
EXPORTS = ["dsgm_params_default", "dsgm_state_init_from_frame", "dsgm_forward",
           "dsgm_ckpt_bytes", "dsgm_workspace_bytes", "dsgm_backward", "dsgm_batch_plan_bytes",
           "dsgm_plan_batched", "dsgm_forward_batched", "dsgm_status_string", "dsgm_last_error",
           "dsgm_version", "dsgm_set_launch", "dsgm_gauss_weights", "dsgm_forward_filtered",
           "dsgm_forward_warped", "dsgm_forward_grid", "dsgm_autotune_bytes", "dsgm_autotune",
           "dsgm_autotune_lookup", "dsgm_autotune_clear", "dsgm_count_nonfinite",
           "dsgm_backward_noalloc"]

# largest H*W dsgm_backward_noalloc accepts (the library's own buffer)
NOALLOC_MAX_PIXELS = 1 << 23


def _check(fn: str, rc: int):
    if rc != DSGM_OK:
        raise DSGMError(fn, rc, lib.dsgm_last_error().decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


# ------------------------------------------------------------------ params
def dsgm_params_default(intensity_range: float = 2.0, mask_rule: int = MASK_VARIANCE) -> Params:
    p = Params()
    _check("dsgm_params_default", lib.dsgm_params_default(ctypes.byref(p), intensity_range, mask_rule))
    return p


def dsgm_version() -> int:
    return lib.dsgm_version()


def dsgm_set_launch(block: int = 0, vector: int = 0) -> None:
    _check("dsgm_set_launch", lib.dsgm_set_launch(block, vector))


TUNE_BG, TUNE_CKPT, TUNE_PRINTED = 1, 2, 4


def _tune_shape(T: int, H: int, W: int) -> Shape:
    return Shape(int(T), int(H), int(W), int(W), int(H) * int(W))


def dsgm_autotune_bytes(in_dtype: int, acc: int, T: int, H: int, W: int, flags: int = 0) -> int:
    return int(lib.dsgm_autotune_bytes(in_dtype, acc, _tune_shape(T, H, W), flags))


def dsgm_autotune(in_dtype: int, acc: int, T: int, H: int, W: int, flags: int = 0) -> tuple:
    """Time dsgm_forward's launch shapes on a synthetic T x H x W problem and keep
    the fastest for later calls with these types, sizes and outputs; returns
    (block, pixels per lane).  Allocates its workspace with torch."""
    n = dsgm_autotune_bytes(in_dtype, acc, T, H, W, flags)
    ws = torch.empty(max(n, 1), dtype=torch.uint8, device="cuda")
    chosen = (ctypes.c_int32 * 2)()
    _check("dsgm_autotune", lib.dsgm_autotune(in_dtype, acc, _tune_shape(T, H, W), flags,
                                              _ptr(ws), n, chosen, _stream()))
    return int(chosen[0]), int(chosen[1])


def dsgm_autotune_lookup(in_dtype: int, acc: int, T: int, H: int, W: int, flags: int = 0) -> tuple:
    chosen = (ctypes.c_int32 * 2)()
    _check("dsgm_autotune_lookup",
           lib.dsgm_autotune_lookup(in_dtype, acc, _tune_shape(T, H, W), flags, chosen))
    return int(chosen[0]), int(chosen[1])


def dsgm_autotune_clear() -> None:
    _check("dsgm_autotune_clear", lib.dsgm_autotune_clear())


# ------------------------------------------------------------------ state
@dataclass
class State:
    """The six state planes (H x W each) as device tensors."""
    mean_a: torch.Tensor
    var_a: torch.Tensor
    mean_c: torch.Tensor
    var_c: torch.Tensor
    age_a: torch.Tensor
    age_c: torch.Tensor

    @property
    def acc(self) -> int:
        return _ACC_DTYPES[self.mean_a.dtype]

    def clone(self) -> "State":
        return State(*(t.clone() for t in self.planes()))

    def planes(self):
        return (self.mean_a, self.var_a, self.mean_c, self.var_c, self.age_a, self.age_c)

    @staticmethod
    def empty(H: int, W: int, dtype=torch.float64, device="cuda") -> "State":
        f = lambda: torch.empty((H, W), dtype=dtype, device=device)
        u = lambda: torch.empty((H, W), dtype=torch.uint8, device=device)
        return State(f(), f(), f(), f(), u(), u())


def _resolve_acc(state: State, acc) -> int:
    if acc is None:
        return state.acc
    if STATE_TORCH[acc] != state.mean_a.dtype:
        raise ValueError(f"acc={acc} needs a {STATE_TORCH[acc]} state, got {state.mean_a.dtype}")
    return acc


def _cstate(st: State, H: int, W: int) -> _State:
    acc_dt = st.mean_a.dtype
    if acc_dt not in _ACC_DTYPES:
        raise TypeError(f"state dtype {acc_dt} not supported")
    for name, t in zip(("mean_a", "var_a", "mean_c", "var_c", "age_a", "age_c"), st.planes()):
        want = torch.uint8 if name.startswith("age") else acc_dt
        if t.dtype != want or not t.is_cuda or not t.is_contiguous() or t.numel() != H * W:
            raise ValueError(f"state.{name}: need a contiguous {want} CUDA tensor of {H}x{W}")
    return _State(*(t.data_ptr() for t in st.planes()))


def _frames_shape(frames: torch.Tensor) -> Shape:
    if frames.dim() != 3:
        raise ValueError("frames must be T x H x W")
    T, H, W = frames.shape
    fs, rs, cs = frames.stride()
    if cs != 1 and W > 1:
        raise ValueError("frames: the last dimension must be contiguous")
    return Shape(T, H, W, rs if H > 1 else W, fs if T > 1 else max(H * rs, 1))


def _same_layout(name: str, t: torch.Tensor, frames: torch.Tensor, dtype):
    if t is None:
        return
    if t.dtype != dtype or not t.is_cuda or tuple(t.shape) != tuple(frames.shape):
        raise ValueError(f"{name}: need a CUDA {dtype} tensor of shape {tuple(frames.shape)}")
    T, H, W = frames.shape
    for d, n in ((0, T), (1, H), (2, W)):
        if n > 1 and t.stride(d) != frames.stride(d):
            raise ValueError(f"{name}: strides {t.stride()} differ from the frames' {frames.stride()}")


def dsgm_state_init_from_frame(frame0: torch.Tensor, state: State, params: Params) -> None:
    if frame0.dim() != 2:
        raise ValueError("frame0 must be H x W")
    H, W = frame0.shape
    sh = Shape(1, H, W, frame0.stride(0) if H > 1 else W, H * W)
    _check("dsgm_state_init_from_frame",
           lib.dsgm_state_init_from_frame(_ptr(frame0), _IN_DTYPES[frame0.dtype], sh, state.acc,
                                          ctypes.byref(params), ctypes.byref(_cstate(state, H, W)),
                                          _stream()))


def dsgm_ckpt_bytes(T: int, H: int, W: int, acc: int, ckpt_every: int) -> int:
    return int(lib.dsgm_ckpt_bytes(Shape(T, H, W, W, H * W), acc, ckpt_every))


def dsgm_forward(frames: torch.Tensor, state: State, params: Params, masks: torch.Tensor,
                 bg: torch.Tensor | None = None, ckpt: torch.Tensor | None = None,
                 ckpt_every: int = 0, codes: torch.Tensor | None = None, acc=None) -> None:
    """Run the T frames of ``frames`` (T x H x W) through the model in ``state``
    (updated in place); writes ``masks`` and the optional outputs.  ``acc``
    defaults to the state's type (ACC_F64_IO32 must be asked for)."""
    if frames.dtype not in _IN_DTYPES:
        raise TypeError(f"frames dtype {frames.dtype} not supported")
    sh = _frames_shape(frames)
    acc = _resolve_acc(state, acc)
    _same_layout("masks", masks, frames, torch.uint8)
    _same_layout("bg", bg, frames, ACC_TORCH[acc])
    _same_layout("codes", codes, frames, torch.uint8)
    if ckpt is not None and (ckpt.dtype != torch.uint8 or not ckpt.is_cuda):
        raise ValueError("ckpt: need a CUDA uint8 tensor")
    cs = _cstate(state, sh.H, sh.W)
    _check("dsgm_forward",
           lib.dsgm_forward(_ptr(frames), _IN_DTYPES[frames.dtype], sh, acc, ctypes.byref(params),
                            ctypes.byref(cs), _ptr(masks), _ptr(bg), _ptr(ckpt),
                            0 if ckpt is None else ckpt.numel(), int(ckpt_every), _ptr(codes),
                            _stream()))


def dsgm_count_nonfinite(frames: torch.Tensor, count: torch.Tensor | None = None) -> torch.Tensor:
    """Count the NaN and infinite elements of ``frames`` (T x H x W) into a
    device int64 scalar (``count``, or a new one), asynchronously."""
    if frames.dtype not in _IN_DTYPES:
        raise TypeError(f"frames dtype {frames.dtype} not supported")
    sh = _frames_shape(frames)
    if count is None:
        count = torch.empty((), dtype=torch.int64, device=frames.device)
    elif count.dtype != torch.int64 or count.numel() != 1 or not count.is_cuda:
        raise ValueError("count: need a CUDA int64 scalar")
    _check("dsgm_count_nonfinite",
           lib.dsgm_count_nonfinite(_ptr(frames), _IN_DTYPES[frames.dtype], sh, _ptr(count),
                                    _stream()))
    return count


def dsgm_gauss_weights(n: int = 5, sigma: float = 1.0) -> list:
    """The n normalised Gaussian taps (Sec. 2.1 density at integer offsets)."""
    w = (ctypes.c_double * 7)()
    _check("dsgm_gauss_weights", lib.dsgm_gauss_weights(int(n), float(sigma), w))
    return [w[i] for i in range(n)]


def gauss_filter(n: int = 5, sigma: float = 1.0, median: bool = True) -> Filter:
    """The paper's preprocessing: an n-tap Gaussian blur, then a 3 x 3 median."""
    f = Filter()
    f.n = int(n)
    f.median = int(bool(median))
    for i, v in enumerate(dsgm_gauss_weights(n, sigma) if n else []):
        f.weights[i] = v
    return f


def dsgm_forward_filtered(frames: torch.Tensor, state: State, params: Params, filt: Filter,
                          masks: torch.Tensor, bg: torch.Tensor | None = None,
                          filtered: torch.Tensor | None = None, codes: torch.Tensor | None = None,
                          acc=None) -> None:
    """dsgm_forward on the preprocessed frames (blur, then median), fused in one pass;
    ``filtered`` (optional) receives the preprocessed frames."""
    if frames.dtype not in _IN_DTYPES:
        raise TypeError(f"frames dtype {frames.dtype} not supported")
    sh = _frames_shape(frames)
    acc = _resolve_acc(state, acc)
    _same_layout("masks", masks, frames, torch.uint8)
    _same_layout("bg", bg, frames, ACC_TORCH[acc])
    _same_layout("filtered", filtered, frames, ACC_TORCH[acc])
    _same_layout("codes", codes, frames, torch.uint8)
    cs = _cstate(state, sh.H, sh.W)
    _check("dsgm_forward_filtered",
           lib.dsgm_forward_filtered(_ptr(frames), _IN_DTYPES[frames.dtype], sh, acc,
                                     ctypes.byref(params), ctypes.byref(filt), ctypes.byref(cs),
                                     _ptr(masks), _ptr(bg), _ptr(filtered), _ptr(codes),
                                     _stream()))


def dsgm_forward_warped(frame: torch.Tensor, src: State, dst: State, params: Params, inv_map,
                        masks: torch.Tensor, bg: torch.Tensor | None = None,
                        codes: torch.Tensor | None = None, acc=None) -> None:
    """One frame (H x W) of the update on the model in ``src`` mapped through the
    3 x 3 ``inv_map`` (current pixel -> previous frame); the new model goes to
    ``dst`` (distinct planes), masks/bg/codes are H x W like the frame."""
    if frame.dtype not in _IN_DTYPES:
        raise TypeError(f"frame dtype {frame.dtype} not supported")
    if frame.dim() != 2:
        raise ValueError("frame must be H x W")
    H, W = frame.shape
    f3 = frame.unsqueeze(0)
    sh = _frames_shape(f3)
    acc = _resolve_acc(src, acc)
    if _resolve_acc(dst, acc) != acc:
        raise ValueError("src and dst must have the same state type")
    _same_layout("masks", masks.unsqueeze(0), f3, torch.uint8)
    _same_layout("bg", None if bg is None else bg.unsqueeze(0), f3, ACC_TORCH[acc])
    _same_layout("codes", None if codes is None else codes.unsqueeze(0), f3, torch.uint8)
    m = (ctypes.c_double * 9)(*[float(v) for v in torch.as_tensor(inv_map, dtype=torch.float64).reshape(9).tolist()])
    cs, cd = _cstate(src, H, W), _cstate(dst, H, W)
    _check("dsgm_forward_warped",
           lib.dsgm_forward_warped(_ptr(frame), _IN_DTYPES[frame.dtype], sh, acc,
                                   ctypes.byref(params), m, ctypes.byref(cs), ctypes.byref(cd),
                                   _ptr(masks), _ptr(bg), _ptr(codes), _stream()))


def dsgm_forward_grid(frames: torch.Tensor, state: State, params: Params, block: int,
                      masks: torch.Tensor, bg: torch.Tensor | None = None,
                      codes: torch.Tensor | None = None, acc=None) -> None:
    """Yi et al.'s grid model: one dual model per block x block pixels; ``state``
    holds ceil(H/b) x ceil(W/b) planes; masks like the frames; bg and codes
    (optional) dense T x Hb x Wb."""
    if frames.dtype not in _IN_DTYPES:
        raise TypeError(f"frames dtype {frames.dtype} not supported")
    sh = _frames_shape(frames)
    T, H, W = frames.shape
    Hb, Wb = -(-H // block), -(-W // block)
    acc = _resolve_acc(state, acc)
    _same_layout("masks", masks, frames, torch.uint8)
    for name, t, dt in (("bg", bg, ACC_TORCH[acc]), ("codes", codes, torch.uint8)):
        if t is not None and (t.dtype != dt or not t.is_cuda or not t.is_contiguous()
                              or tuple(t.shape) != (T, Hb, Wb)):
            raise ValueError(f"{name}: need a contiguous CUDA {dt} tensor of shape {(T, Hb, Wb)}")
    cs = _cstate(state, Hb, Wb)
    _check("dsgm_forward_grid",
           lib.dsgm_forward_grid(_ptr(frames), _IN_DTYPES[frames.dtype], sh, acc,
                                 ctypes.byref(params), int(block), ctypes.byref(cs), _ptr(masks),
                                 _ptr(bg), _ptr(codes), _stream()))


def dsgm_workspace_bytes(T: int, H: int, W: int, acc: int) -> int:
    return int(lib.dsgm_workspace_bytes(Shape(T, H, W, W, H * W), acc))


def _planes4(name, planes, H, W, dtype):
    if planes is None:
        return None
    planes = tuple(planes)
    if len(planes) != 4:
        raise ValueError(f"{name}: need 4 planes (mean_a, var_a, mean_c, var_c)")
    for t in planes:
        if t.dtype != dtype or not t.is_cuda or not t.is_contiguous() or t.numel() != H * W:
            raise ValueError(f"{name}: need contiguous {dtype} CUDA planes of {H}x{W}")
    return _GradState(*(t.data_ptr() for t in planes))


def dsgm_backward(frames: torch.Tensor, params: Params, ckpt: torch.Tensor, ckpt_every: int,
                  acc: int, grad_bg, grad_state_T, grad_frames: torch.Tensor, grad_state0,
                  grad_var_init: torch.Tensor, workspace: torch.Tensor) -> None:
    """Adjoint of dsgm_forward with the decisions held fixed.  ``grad_state_T``
    and ``grad_state0`` are 4-tuples of (mean_a, var_a, mean_c, var_c) planes;
    ``grad_var_init`` is a one-element float64 CUDA tensor."""
    if frames.dtype not in _IN_DTYPES:
        raise TypeError(f"frames dtype {frames.dtype} not supported")
    sh = _frames_shape(frames)
    adt = ACC_TORCH[acc]
    _same_layout("grad_bg", grad_bg, frames, adt)
    _same_layout("grad_frames", grad_frames, frames, adt)
    gsT = _planes4("grad_state_T", grad_state_T, sh.H, sh.W, adt)
    gs0 = _planes4("grad_state0", grad_state0, sh.H, sh.W, adt)
    if grad_var_init.dtype != torch.float64 or not grad_var_init.is_cuda or grad_var_init.numel() != 1:
        raise ValueError("grad_var_init: need a one-element float64 CUDA tensor")
    need = dsgm_workspace_bytes(sh.T, sh.H, sh.W, acc)
    if workspace.dtype != torch.uint8 or not workspace.is_cuda or workspace.numel() < need:
        raise ValueError(f"workspace: need a CUDA uint8 tensor of at least {need} bytes")
    if ckpt is not None and (ckpt.dtype != torch.uint8 or not ckpt.is_cuda):
        raise ValueError("ckpt: need a CUDA uint8 tensor")
    _check("dsgm_backward",
           lib.dsgm_backward(_ptr(frames), _IN_DTYPES[frames.dtype], sh, acc, ctypes.byref(params),
                             _ptr(ckpt), 0 if ckpt is None else ckpt.numel(), int(ckpt_every),
                             _ptr(grad_bg),
                             ctypes.byref(gsT) if gsT is not None else None, _ptr(grad_frames),
                             ctypes.byref(gs0) if gs0 is not None else None, _ptr(grad_var_init),
                             _ptr(workspace), workspace.numel(), _stream()))


def dsgm_backward_noalloc(frames: torch.Tensor, params: Params, ckpt: torch.Tensor,
                          ckpt_every: int, acc: int, grad_bg, grad_state_T,
                          grad_frames: torch.Tensor, grad_state0,
                          grad_var_init: torch.Tensor) -> None:
    """dsgm_backward without a workspace: the library uses a buffer of its own
    on the current device (H*W <= NOALLOC_MAX_PIXELS).  Calls that overlap on
    one device race on that buffer."""
    if frames.dtype not in _IN_DTYPES:
        raise TypeError(f"frames dtype {frames.dtype} not supported")
    sh = _frames_shape(frames)
    adt = ACC_TORCH[acc]
    _same_layout("grad_bg", grad_bg, frames, adt)
    _same_layout("grad_frames", grad_frames, frames, adt)
    gsT = _planes4("grad_state_T", grad_state_T, sh.H, sh.W, adt)
    gs0 = _planes4("grad_state0", grad_state0, sh.H, sh.W, adt)
    if grad_var_init.dtype != torch.float64 or not grad_var_init.is_cuda or grad_var_init.numel() != 1:
        raise ValueError("grad_var_init: need a one-element float64 CUDA tensor")
    if ckpt is not None and (ckpt.dtype != torch.uint8 or not ckpt.is_cuda):
        raise ValueError("ckpt: need a CUDA uint8 tensor")
    _check("dsgm_backward_noalloc",
           lib.dsgm_backward_noalloc(_ptr(frames), _IN_DTYPES[frames.dtype], sh, acc,
                                     ctypes.byref(params), _ptr(ckpt),
                                     0 if ckpt is None else ckpt.numel(), int(ckpt_every),
                                     _ptr(grad_bg),
                                     ctypes.byref(gsT) if gsT is not None else None,
                                     _ptr(grad_frames),
                                     ctypes.byref(gs0) if gs0 is not None else None,
                                     _ptr(grad_var_init), _stream()))


# ------------------------------------------------------------------ convenience
def forward(frames: torch.Tensor, state: State, params: Params, *, bg: bool = False,
            codes: bool = False, ckpt_every: int = 0, acc=None) -> dict:
    """Allocate the outputs (same layout as ``frames``) and call dsgm_forward."""
    T, H, W = frames.shape
    acc = _resolve_acc(state, acc)
    like = lambda dt: torch.empty_strided(frames.shape, frames.stride(), dtype=dt, device=frames.device)
    out = {"masks": like(torch.uint8)}
    if bg:
        out["bg"] = like(ACC_TORCH[acc])
    if codes:
        out["codes"] = like(torch.uint8)
    if ckpt_every:
        out["ckpt"] = torch.empty(max(dsgm_ckpt_bytes(T, H, W, acc, ckpt_every), 1),
                                  dtype=torch.uint8, device=frames.device)
    dsgm_forward(frames, state, params, out["masks"], out.get("bg"), out.get("ckpt"), ckpt_every,
                 out.get("codes"), acc=acc)
    return out


def forward_filtered(frames: torch.Tensor, state: State, params: Params, filt: Filter, *,
                     bg: bool = False, filtered: bool = False, codes: bool = False,
                     acc=None) -> dict:
    """Allocate the outputs and call dsgm_forward_filtered."""
    acc = _resolve_acc(state, acc)
    like = lambda dt: torch.empty_strided(frames.shape, frames.stride(), dtype=dt, device=frames.device)
    out = {"masks": like(torch.uint8)}
    if bg:
        out["bg"] = like(ACC_TORCH[acc])
    if filtered:
        out["filtered"] = like(ACC_TORCH[acc])
    if codes:
        out["codes"] = like(torch.uint8)
    dsgm_forward_filtered(frames, state, params, filt, out["masks"], out.get("bg"),
                          out.get("filtered"), out.get("codes"), acc=acc)
    return out


def backward(frames: torch.Tensor, params: Params, ckpt: torch.Tensor, ckpt_every: int, acc: int,
             grad_bg=None, grad_state_T=None) -> dict:
    """Allocate the gradients and call dsgm_backward."""
    T, H, W = frames.shape
    adt = ACC_TORCH[acc]
    gx = torch.empty_strided(frames.shape, frames.stride(), dtype=adt, device=frames.device)
    gs0 = tuple(torch.empty((H, W), dtype=adt, device=frames.device) for _ in range(4))
    gvi = torch.empty((1,), dtype=torch.float64, device=frames.device)
    ws = torch.empty(max(dsgm_workspace_bytes(T, H, W, acc), 1), dtype=torch.uint8,
                     device=frames.device)
    dsgm_backward(frames, params, ckpt, ckpt_every, acc, grad_bg, grad_state_T, gx, gs0, gvi, ws)
    return {"grad_frames": gx, "grad_state0": gs0, "grad_var_init": gvi, "workspace": ws}


def _like_frames(t, frames, dtype):
    """t (or zeros) in the frames' layout and the given dtype."""
    out = torch.empty_strided(frames.shape, frames.stride(), dtype=dtype, device=frames.device)
    if t is None:
        return None
    out.copy_(t)
    return out


class DSGMFunction(torch.autograd.Function):
    """Differentiable DSGM forward (Sec. 2.2-2.3 of arXiv:1702.05156).

    apply(frames, mean_a, var_a, mean_c, var_c, age_a, age_c, var_init, params, ckpt_every, acc)
    returns (masks, bg, mean_a_T, var_a_T, mean_c_T, var_c_T, age_a_T, age_c_T).
    The input state is not modified.  masks and ages are not differentiable;
    the gradient flows to frames, the four float planes and var_init (a 0-d or
    one-element tensor), with the decisions held at the forward pass's values.
    theta_s, theta_d and the floors get no gradient (it is zero almost
    everywhere).
    """

    @staticmethod
    def forward(ctx, frames, mean_a, var_a, mean_c, var_c, age_a, age_c, var_init, params,
                ckpt_every=32, acc=None):
        p = Params(*(getattr(params, n) for n, _ in Params._fields_))
        p.var_init = float(var_init.detach().reshape(()).item()) if torch.is_tensor(var_init) \
            else float(var_init)
        st = State(mean_a.detach().clone(), var_a.detach().clone(), mean_c.detach().clone(),
                   var_c.detach().clone(), age_a.detach().clone(), age_c.detach().clone())
        acc = _resolve_acc(st, acc)
        if acc == ACC_F32X2:
            raise NotImplementedError("DSGMFunction: F32X2 state has no autograd form; call "
                                      "forward() and backward() directly")
        out = forward(frames.detach(), st, p, bg=True, ckpt_every=ckpt_every, acc=acc)
        ctx.save_for_backward(frames, out["ckpt"])
        ctx.params, ctx.K, ctx.acc = p, ckpt_every, acc
        ctx.var_init_like = var_init if torch.is_tensor(var_init) else None
        ctx.mark_non_differentiable(out["masks"], st.age_a, st.age_c)
        return (out["masks"], out["bg"], st.mean_a, st.var_a, st.mean_c, st.var_c, st.age_a,
                st.age_c)

    @staticmethod
    def backward(ctx, g_masks, g_bg, g_mA, g_vA, g_mC, g_vC, g_aA, g_aC):
        frames, ckpt = ctx.saved_tensors
        adt = ACC_TORCH[ctx.acc]
        gbg = _like_frames(g_bg, frames, adt)
        gsT = None
        if any(g is not None for g in (g_mA, g_vA, g_mC, g_vC)):
            ref = frames.new_zeros((frames.shape[1], frames.shape[2]), dtype=adt)
            gsT = tuple((g if g is not None else ref).to(adt).contiguous()
                        for g in (g_mA, g_vA, g_mC, g_vC))
        r = backward(frames, ctx.params, ckpt, ctx.K, ctx.acc, gbg, gsT)
        gx = r["grad_frames"].to(frames.dtype)
        gvi = None
        if ctx.var_init_like is not None:
            gvi = r["grad_var_init"].to(ctx.var_init_like.dtype).reshape(ctx.var_init_like.shape)
        gs = r["grad_state0"]
        gs = tuple(g.to(STATE_TORCH[ctx.acc]) for g in gs)
        return (gx, gs[0], gs[1], gs[2], gs[3], None, None, gvi, None, None, None)


# ------------------------------------------------------------------ batched
def _instance(frames: torch.Tensor, state: State, masks: torch.Tensor, bg=None, counts=None,
              acc=None) -> Instance:
    sh = _frames_shape(frames)
    acc = _resolve_acc(state, acc)
    _same_layout("masks", masks, frames, torch.uint8)
    _same_layout("bg", bg, frames, ACC_TORCH[acc])
    if counts is not None and (counts.dtype != torch.int32 or not counts.is_cuda or
                               not counts.is_contiguous() or counts.numel() != sh.T):
        raise ValueError(f"counts: need a contiguous int32 CUDA tensor of {sh.T} entries")
    return Instance(sh, frames.data_ptr(), _cstate(state, sh.H, sh.W), masks.data_ptr(),
                    None if bg is None else bg.data_ptr(),
                    None if counts is None else counts.data_ptr())


class Batch:
    """Many independent instances planned for one persistent launch.

    ``items`` is a list of (frames, state, masks, bg-or-None[, counts-or-None]);
    counts is an int32 tensor of T entries that each run fills with the
    foreground pixels of every frame.  Every tensor is kept alive by this
    object.  ``run(params)`` calls dsgm_forward_batched on the
    current stream (capturable into a CUDA/HIP graph).
    """

    def __init__(self, items, in_dtype=None, acc=None, vector: int = 0, grid: int = 0):
        """``vector`` (pixels per lane, 1/2/4; 0 = the library's default) is the
        tile width of the plan and ``grid`` (0 = the planner's device-filling
        count) the number of persistent workgroups; ``tune.tune_batched`` picks
        both by measurement."""
        self.items = list(items)
        if not self.items:
            raise ValueError("empty batch")
        fr0, st0 = self.items[0][0], self.items[0][1]
        self.in_dtype = _IN_DTYPES[fr0.dtype] if in_dtype is None else in_dtype
        self.acc = st0.acc if acc is None else acc
        for fr, st, *_ in self.items:
            if _IN_DTYPES[fr.dtype] != self.in_dtype or st.mean_a.dtype != STATE_TORCH[self.acc]:
                raise ValueError("all instances of a batch share the frame and state dtypes")
        arr = (Instance * len(self.items))(*(_instance(*it, acc=self.acc) for it in self.items))
        self._arr = arr
        if vector:
            dsgm_set_launch(0, vector)  # the width the plan's size and items are made for
        try:
            nbytes = int(lib.dsgm_batch_plan_bytes(arr, len(self.items), self.in_dtype, self.acc))
            if nbytes == 0:
                raise DSGMError("dsgm_batch_plan_bytes", -1, lib.dsgm_last_error().decode())
            self.plan_buffer = torch.empty(nbytes, dtype=torch.uint8, device=fr0.device)
            self.plan = BatchPlan()
            _check("dsgm_plan_batched",
                   lib.dsgm_plan_batched(arr, len(self.items), self.in_dtype, self.acc,
                                         _ptr(self.plan_buffer), nbytes, ctypes.byref(self.plan),
                                         _stream()))
        finally:
            if vector:
                dsgm_set_launch(0, 0)
        if grid:
            if grid < 1:
                raise ValueError(f"grid = {grid}: at least one workgroup")
            self.plan.grid = int(grid)

    def run(self, params: Params) -> None:
        _check("dsgm_forward_batched",
               lib.dsgm_forward_batched(ctypes.byref(self.plan), ctypes.byref(params), _stream()))
