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
IN_F64, IN_F32, IN_BF16 = 0, 1, 2
ACC_F64, ACC_F32 = 0, 1
WEIGHT_EQ, WEIGHT_APPENDIX = 0, 1
MASK_VARIANCE, MASK_PRINTED = 0, 1
CODE_HIT_A, CODE_HIT_C, CODE_RESET, CODE_SWAP, CODE_FG = 1, 2, 4, 8, 16

_IN_DTYPES = {torch.float64: IN_F64, torch.float32: IN_F32, torch.bfloat16: IN_BF16}
_ACC_DTYPES = {torch.float64: ACC_F64, torch.float32: ACC_F32}
ACC_TORCH = {ACC_F64: torch.float64, ACC_F32: torch.float32}


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


class _State(ctypes.Structure):
    _fields_ = [("mean_a", ctypes.c_void_p), ("var_a", ctypes.c_void_p),
                ("mean_c", ctypes.c_void_p), ("var_c", ctypes.c_void_p),
                ("age_a", ctypes.c_void_p), ("age_c", ctypes.c_void_p)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.dsgm_params_default.argtypes = [ctypes.POINTER(Params), ctypes.c_double, i32]
    lib.dsgm_state_init_from_frame.argtypes = [vp, i32, Shape, i32, ctypes.POINTER(Params),
                                               ctypes.POINTER(_State), vp]
    lib.dsgm_forward.argtypes = [vp, i32, Shape, i32, ctypes.POINTER(Params),
                                 ctypes.POINTER(_State), vp, vp, vp, i32, vp, vp]
    lib.dsgm_ckpt_bytes.argtypes = [Shape, i32, i32]
    lib.dsgm_ckpt_bytes.restype = ctypes.c_size_t
    lib.dsgm_status_string.argtypes = [ctypes.c_int]
    lib.dsgm_status_string.restype = ctypes.c_char_p
    lib.dsgm_last_error.restype = ctypes.c_char_p
    lib.dsgm_set_launch.argtypes = [i32, i32]
    for f in ("dsgm_params_default", "dsgm_state_init_from_frame", "dsgm_forward",
              "dsgm_version", "dsgm_set_launch"):
        getattr(lib, f).restype = ctypes.c_int
    del i64
    return lib


lib = _load()

# names of every C entry point declared in include/dsgm.h
EXPORTS = ["dsgm_params_default", "dsgm_state_init_from_frame", "dsgm_forward",
           "dsgm_ckpt_bytes", "dsgm_status_string", "dsgm_last_error", "dsgm_version",
           "dsgm_set_launch"]


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
                 ckpt_every: int = 0, codes: torch.Tensor | None = None) -> None:
    """Run the T frames of ``frames`` (T x H x W) through the model in ``state``
    (updated in place); writes ``masks`` and the optional outputs."""
    if frames.dtype not in _IN_DTYPES:
        raise TypeError(f"frames dtype {frames.dtype} not supported")
    sh = _frames_shape(frames)
    acc = state.acc
    _same_layout("masks", masks, frames, torch.uint8)
    _same_layout("bg", bg, frames, ACC_TORCH[acc])
    _same_layout("codes", codes, frames, torch.uint8)
    if ckpt is not None:
        need = dsgm_ckpt_bytes(sh.T, sh.H, sh.W, acc, ckpt_every)
        if ckpt.dtype != torch.uint8 or not ckpt.is_cuda or ckpt.numel() < need:
            raise ValueError(f"ckpt: need a CUDA uint8 tensor of at least {need} bytes")
    cs = _cstate(state, sh.H, sh.W)
    _check("dsgm_forward",
           lib.dsgm_forward(_ptr(frames), _IN_DTYPES[frames.dtype], sh, acc, ctypes.byref(params),
                            ctypes.byref(cs), _ptr(masks), _ptr(bg), _ptr(ckpt), int(ckpt_every),
                            _ptr(codes), _stream()))


# ------------------------------------------------------------------ convenience
def forward(frames: torch.Tensor, state: State, params: Params, *, bg: bool = False,
            codes: bool = False, ckpt_every: int = 0) -> dict:
    """Allocate the outputs (same layout as ``frames``) and call dsgm_forward."""
    T, H, W = frames.shape
    like = lambda dt: torch.empty_strided(frames.shape, frames.stride(), dtype=dt, device=frames.device)
    out = {"masks": like(torch.uint8)}
    if bg:
        out["bg"] = like(ACC_TORCH[state.acc])
    if codes:
        out["codes"] = like(torch.uint8)
    if ckpt_every:
        out["ckpt"] = torch.empty(max(dsgm_ckpt_bytes(T, H, W, state.acc, ckpt_every), 1),
                                  dtype=torch.uint8, device=frames.device)
    dsgm_forward(frames, state, params, out["masks"], out.get("bg"), out.get("ckpt"), ckpt_every,
                 out.get("codes"))
    return out
