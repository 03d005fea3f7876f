"""The C ABI on the CPU: the library loads, exports every declared symbol, and
rejects bad arguments with the documented status before any HIP call."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

from paper_1702_05156_amd import dsgm
lib = dsgm.lib


def _declared():
    text = open(os.path.join(ROOT, "include", "dsgm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dsgm_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = _declared()
    assert "dsgm_forward" in names and "dsgm_params_default" in names
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(dsgm.EXPORTS) == names


def test_version_and_status_strings():
    assert dsgm.dsgm_version() >= 100
    assert lib.dsgm_status_string(0) == b"DSGM_OK"
    assert lib.dsgm_status_string(-4) == b"DSGM_E_ALIGN"
    assert lib.dsgm_status_string(123) == b"DSGM_UNKNOWN"


def test_params_default_values():
    p = dsgm.dsgm_params_default(255.0)
    assert (p.theta_s, p.theta_d, p.var_init, p.var_floor, p.mask_floor, p.age_max) == \
        (2.0, 4.0, 255.0, 0.1, 0.25, 30)
    p = dsgm.dsgm_params_default(2.0)
    s = 2.0 / 255.0
    assert p.var_init == 255.0 * s * s and p.var_floor == 0.1 * s * s and p.mask_floor == 0.25 * s * s
    p = dsgm.dsgm_params_default(2.0, dsgm.MASK_PRINTED)
    assert p.mask_floor == 0.25 * s and p.mask_rule == dsgm.MASK_PRINTED
    # agrees with the oracle's own derivation of the same constants
    import oracle
    o = oracle.default_params(2.0)
    q = dsgm.dsgm_params_default(2.0)
    assert (o.var_init, o.var_floor, o.mask_floor) == (q.var_init, q.var_floor, q.mask_floor)


def test_params_default_rejects():
    p = dsgm.Params()
    assert lib.dsgm_params_default(None, 2.0, 0) == -1
    assert lib.dsgm_params_default(ctypes.byref(p), 0.0, 0) == -1
    assert lib.dsgm_params_default(ctypes.byref(p), 2.0, 7) == -1
    assert b"mask_rule" in lib.dsgm_last_error()


FAKE = 1 << 20  # never dereferenced: every call below fails validation first


def _state(ptr=FAKE):
    return dsgm._State(ptr, ptr, ptr, ptr, ptr, ptr)


def _fwd(frames=FAKE, in_dtype=0, shape=(4, 8, 8, 8, 64), acc=0, params=None, state="ok",
         masks=FAKE, bg=None, ckpt=None, K=0, codes=None, ckpt_bytes=1 << 30):
    p = params if params is not None else dsgm.dsgm_params_default(2.0)
    st = _state() if state == "ok" else state
    return lib.dsgm_forward(frames, in_dtype, dsgm.Shape(*shape), acc,
                            ctypes.byref(p) if p is not False else None,
                            ctypes.byref(st) if st is not None else None, masks, bg, ckpt,
                            ckpt_bytes, K, codes, None)


def test_forward_validation():
    assert _fwd(in_dtype=5) == -3
    assert _fwd(acc=3) == -3
    assert _fwd(in_dtype=0, acc=1) == -3                  # f64 frames, f32 state
    assert _fwd(params=False) == -1
    assert _fwd(state=None) == -1
    assert _fwd(shape=(-1, 8, 8, 8, 64)) == -2
    assert _fwd(shape=(4, 8, 8, 7, 64)) == -2             # row_stride < W
    assert _fwd(shape=(4, 8, 8, 8, 63)) == -2             # frame_stride < extent
    assert _fwd(shape=(4, 1 << 16, 1 << 15, 1 << 15, 1 << 31)) == -2  # frame > 2^31 bytes
    assert _fwd(frames=None) == -1
    assert _fwd(masks=None) == -1
    assert _fwd(state=_state(0)) == -1
    assert _fwd(frames=FAKE + 4) == -4                   # f64 frames not 8-aligned
    assert _fwd(bg=FAKE + 2) == -4
    assert _fwd(ckpt=FAKE, K=0) == -1
    assert _fwd(ckpt=FAKE, K=2, ckpt_bytes=100) == -5     # checkpoint buffer too small
    for bad in (dict(age_max=0), dict(age_max=256), dict(weight_rule=2), dict(mask_rule=-1),
                dict(theta_s=-1.0), dict(var_init=float("nan")), dict(var_floor=float("inf"))):
        p = dsgm.dsgm_params_default(2.0)
        for k, v in bad.items():
            setattr(p, k, v)
        assert _fwd(params=p) == -1, bad
    assert b"age_max" in lib.dsgm_last_error() or lib.dsgm_last_error()


def test_empty_problems_need_no_gpu():
    # nothing to do: returns OK without touching the device
    assert _fwd(shape=(0, 8, 8, 8, 64)) == 0
    assert _fwd(shape=(4, 0, 8, 8, 64)) == 0
    assert _fwd(shape=(4, 8, 0, 0, 0), frames=None, masks=None) == 0
    assert lib.dsgm_last_error() == b""


def test_ckpt_bytes():
    sh = dsgm.Shape(100, 3, 5, 5, 15)
    # ceil(100/32) = 4 checkpoints of 4 f64 planes + 2 age planes, each padded to 256 B
    assert lib.dsgm_ckpt_bytes(sh, 0, 32) == 4 * (4 * 256 + 2 * 256)
    assert lib.dsgm_ckpt_bytes(sh, 0, 0) == 0
    sh = dsgm.Shape(64, 100, 100, 100, 10000)
    assert lib.dsgm_ckpt_bytes(sh, 1, 8) == 8 * (4 * 40192 + 2 * 10240)


def test_set_launch_validation():
    assert lib.dsgm_set_launch(100, 0) == -1
    assert lib.dsgm_set_launch(64, 3) == -1
    assert lib.dsgm_set_launch(0, 0) == 0


def _bwd(frames=FAKE, shape=(4, 8, 8, 8, 64), ckpt=FAKE, K=2, gfr=FAKE, gs0="ok", gvi=FAKE,
         ws=FAKE, ws_bytes=1 << 20, acc=0, in_dtype=0, ckpt_bytes=1 << 30):
    p = dsgm.dsgm_params_default(2.0)
    g = dsgm._GradState(FAKE, FAKE, FAKE, FAKE) if gs0 == "ok" else gs0
    return lib.dsgm_backward(frames, in_dtype, dsgm.Shape(*shape), acc, ctypes.byref(p), ckpt,
                             ckpt_bytes, K, None, None, gfr, ctypes.byref(g) if g is not None else None, gvi,
                             ws, ws_bytes, None)


def test_backward_validation():
    assert _bwd(ws_bytes=16) == -5                       # DSGM_E_WORKSPACE
    assert _bwd(ckpt_bytes=1000) == -5                   # checkpoint buffer too small
    assert _bwd(ws=None) == -1
    assert _bwd(gvi=None) == -1
    assert _bwd(ckpt=None) == -1
    assert _bwd(K=0) == -1
    assert _bwd(gfr=None) == -1
    assert _bwd(gs0=None) == -1
    assert _bwd(gs0=dsgm._GradState(FAKE, None, FAKE, FAKE)) == -1
    assert _bwd(frames=FAKE + 3) == -4
    assert _bwd(in_dtype=0, acc=1) == -3
    sh = dsgm.Shape(4, 8, 8, 8, 64)
    assert lib.dsgm_workspace_bytes(sh, 0) == 512 + 4096
    assert lib.dsgm_workspace_bytes(sh, 9) == 0


def _bwd_na(frames=FAKE, shape=(4, 8, 8, 8, 64), ckpt=FAKE, K=2, gfr=FAKE, gs0="ok", gvi=FAKE,
            acc=0, in_dtype=0, ckpt_bytes=1 << 40):
    p = dsgm.dsgm_params_default(2.0)
    g = dsgm._GradState(FAKE, FAKE, FAKE, FAKE) if gs0 == "ok" else gs0
    return lib.dsgm_backward_noalloc(frames, in_dtype, dsgm.Shape(*shape), acc, ctypes.byref(p),
                                     ckpt, ckpt_bytes, K, None, None, gfr,
                                     ctypes.byref(g) if g is not None else None, gvi, None)


def test_backward_noalloc_validation():
    """The entry point without a workspace rejects what dsgm_backward rejects,
    and frames larger than its own buffer, before any HIP call."""
    assert _bwd_na(gvi=None) == -1
    assert _bwd_na(ckpt=None) == -1
    assert _bwd_na(K=0) == -1
    assert _bwd_na(gfr=None) == -1
    assert _bwd_na(gs0=None) == -1
    assert _bwd_na(ckpt_bytes=1000) == -5
    assert _bwd_na(frames=FAKE + 3) == -4
    assert _bwd_na(in_dtype=0, acc=1) == -3
    big = dsgm.NOALLOC_MAX_PIXELS
    # one pixel over the limit: 2^23 + 1 = 3 * 2796203 (frames of one row)
    assert _bwd_na(shape=(1, 1, big + 1, big + 1, big + 1)) == -5
    assert b"at most" in lib.dsgm_last_error()
    assert _bwd_na(shape=(1, 3, 2796203, 2796203, 3 * 2796203)) == -5


def test_f32x2_validation():
    """The compensated pair state: F32 or BF16 frames, 8-byte values (the
    checkpoint size of FP64 state), dsgm_forward/dsgm_backward only."""
    assert _fwd(in_dtype=1, acc=4, shape=(0, 8, 8, 8, 64)) == 0
    assert _fwd(in_dtype=0, acc=4) == -3                 # FP64 frames
    assert _fwd(in_dtype=3, acc=4) == -3                 # 8-bit frames
    assert _fwd(in_dtype=1, acc=4, bg=FAKE + 2) == -4    # FP32 bg alignment
    assert _bwd(in_dtype=0, acc=4) == -3
    assert _bwd(in_dtype=1, acc=4, ws_bytes=16) == -5
    sh = dsgm.Shape(100, 3, 5, 5, 15)
    assert lib.dsgm_ckpt_bytes(sh, 4, 32) == lib.dsgm_ckpt_bytes(sh, 0, 32)
    assert lib.dsgm_workspace_bytes(sh, 4) == lib.dsgm_workspace_bytes(sh, 0)
    one = (dsgm.Instance * 1)(_inst())
    assert lib.dsgm_batch_plan_bytes(one, 1, 1, 4) == 0
    assert b"F32X2" in lib.dsgm_last_error()
    p = dsgm.dsgm_params_default(2.0)
    st = _state()
    f = dsgm.gauss_filter(5, 1.0, True)
    rc = lib.dsgm_forward_filtered(FAKE, 1, dsgm.Shape(2, 8, 8, 8, 64), 4, ctypes.byref(p),
                                   ctypes.byref(f), ctypes.byref(st), FAKE, None, None, None, None)
    assert rc == -3
    rc = lib.dsgm_forward_grid(FAKE, 1, dsgm.Shape(2, 8, 8, 8, 64), 4, ctypes.byref(p), 4,
                               ctypes.byref(st), FAKE, None, None, None)
    assert rc == -3


def _inst(T=4, H=8, W=8, ptr=FAKE, bg=None):
    return dsgm.Instance(dsgm.Shape(T, H, W, W, H * W), ptr, _state(ptr), ptr, bg)


def test_batched_validation():
    one = (dsgm.Instance * 2)(_inst(), _inst(T=3, H=4, W=12))
    n = lib.dsgm_batch_plan_bytes(one, 2, 1, 1)
    # header + 2 descriptors of 136 B (padded) + items: 8*8/4 = 16 groups -> 1 item;
    # 4*12/4 -> 1 item
    assert n == 256 + 512 + 256
    # foreground counters add 256 stripes of T counters per instance (padded)
    cnt = (dsgm.Instance * 2)(_inst(), _inst(T=3, H=4, W=12))
    cnt[1].fg_counts = FAKE
    assert lib.dsgm_batch_plan_bytes(cnt, 2, 1, 1) == n + 3 * 256 * 4
    cnt[1].fg_counts = FAKE + 2
    assert lib.dsgm_batch_plan_bytes(cnt, 2, 1, 1) == 0   # misaligned counters
    assert lib.dsgm_batch_plan_bytes(None, 2, 1, 1) == 0
    bad = (dsgm.Instance * 1)(_inst(ptr=FAKE + 2))
    assert lib.dsgm_batch_plan_bytes(bad, 1, 1, 1) == 0   # misaligned f32 frames
    neg = (dsgm.Instance * 1)(_inst(T=-1))
    assert lib.dsgm_batch_plan_bytes(neg, 1, 1, 1) == 0
    plan = dsgm.BatchPlan()
    assert lib.dsgm_plan_batched(one, 2, 1, 1, None, 1 << 20, ctypes.byref(plan), None) == -1
    assert lib.dsgm_plan_batched(one, 2, 1, 1, FAKE, 16, ctypes.byref(plan), None) == -5
    assert lib.dsgm_plan_batched(one, 2, 1, 1, FAKE + 8, 1 << 20, ctypes.byref(plan), None) == -4
    p = dsgm.dsgm_params_default(2.0)
    assert lib.dsgm_forward_batched(None, ctypes.byref(p), None) == -1
    assert lib.dsgm_forward_batched(ctypes.byref(plan), ctypes.byref(p), None) == -1  # not planned
    plan.device_plan = FAKE
    plan.vector = 3
    assert lib.dsgm_forward_batched(ctypes.byref(plan), ctypes.byref(p), None) == -1
    plan.vector, plan.n_items, plan.grid = 4, 0, 0
    assert lib.dsgm_forward_batched(ctypes.byref(plan), ctypes.byref(p), None) == -1  # no workgroups
    plan.grid = 1
    assert lib.dsgm_forward_batched(ctypes.byref(plan), ctypes.byref(p), None) == 0  # nothing to do


E_ARG, E_UNSUPPORTED = -1, -7


def test_gauss_weights_match_the_oracle():
    """The library's Gaussian taps (host code) equal the oracle's bit for bit
    (both evaluate the Sec. 2.1 density in the same stated order)."""
    import oracle
    for n, sigma in [(1, 1.0), (3, 0.7), (5, 1.0), (7, 1.5)]:
        got = np.array(dsgm.dsgm_gauss_weights(n, sigma))
        assert np.array_equal(got, oracle.gauss_weights(n, sigma)), (n, sigma)


def test_filtered_forward_validation():
    """Argument checks of dsgm_forward_filtered run before any HIP call."""
    p = dsgm.dsgm_params_default(2.0)
    sh = dsgm.Shape(4, 8, 8, 8, 64)
    st = dsgm._State(16, 16, 16, 16, 16, 16)
    for n, med, want in [(4, 1, E_ARG), (9, 1, E_UNSUPPORTED), (5, 2, E_ARG),
                         (-1, 0, E_ARG)]:
        f = dsgm.Filter()
        f.n, f.median = n, med
        for i in range(7):
            f.weights[i] = 0.2
        rc = dsgm.lib.dsgm_forward_filtered(16, 0, sh, 0, ctypes.byref(p), ctypes.byref(f),
                                            ctypes.byref(st), 16, None, None, None, None)
        assert rc == want, (n, med, rc)
    f = dsgm.gauss_filter(5, 1.0)
    rc = dsgm.lib.dsgm_forward_filtered(16, 0, sh, 0, ctypes.byref(p), None, ctypes.byref(st),
                                        16, None, None, None, None)
    assert rc == E_ARG
    f.n, f.weights[0] = 1, 0.5
    rc = dsgm.lib.dsgm_forward_filtered(16, 0, sh, 0, ctypes.byref(p), ctypes.byref(f),
                                        ctypes.byref(st), 16, None, None, None, None)
    assert rc == E_UNSUPPORTED
    for n, s in [(4, 1.0), (9, 1.0), (5, 0.0)]:
        with pytest.raises(dsgm.DSGMError):
            dsgm.dsgm_gauss_weights(n, s)


def test_warped_forward_validation():
    """dsgm_forward_warped rejects T != 1, overlapping src/dst planes and a
    non-finite map before any HIP call."""
    p = dsgm.dsgm_params_default(2.0)
    m = (ctypes.c_double * 9)(1, 0, 0, 0, 1, 0, 0, 0, 1)
    base = 1 << 20
    src = dsgm._State(base, base + 4096, base + 8192, base + 12288, base + 16384, base + 16640)
    dst = dsgm._State(base + 32768, base + 36864, base + 40960, base + 45056, base + 49152,
                      base + 49408)
    sh = dsgm.Shape(1, 8, 8, 8, 64)
    rc = dsgm.lib.dsgm_forward_warped(base, 0, dsgm.Shape(2, 8, 8, 8, 64), 0, ctypes.byref(p), m,
                                      ctypes.byref(src), ctypes.byref(dst), base, None, None, None)
    assert rc == -2
    rc = dsgm.lib.dsgm_forward_warped(base, 0, sh, 0, ctypes.byref(p), m, ctypes.byref(src),
                                      ctypes.byref(src), base, None, None, None)
    assert rc == E_ARG
    bad = (ctypes.c_double * 9)(1, 0, float("nan"), 0, 1, 0, 0, 0, 1)
    rc = dsgm.lib.dsgm_forward_warped(base, 0, sh, 0, ctypes.byref(p), bad, ctypes.byref(src),
                                      ctypes.byref(dst), base, None, None, None)
    assert rc == E_ARG
    rc = dsgm.lib.dsgm_forward_warped(base, 0, sh, 0, ctypes.byref(p), None, ctypes.byref(src),
                                      ctypes.byref(dst), base, None, None, None)
    assert rc == E_ARG


def test_grid_forward_validation():
    p = dsgm.dsgm_params_default(2.0)
    st = dsgm._State(1 << 20, 1 << 21, 1 << 22, 1 << 23, 1 << 24, 1 << 25)
    for b, want in [(3, -7), (8, -7), (0, -7)]:
        rc = dsgm.lib.dsgm_forward_grid(1 << 20, 0, dsgm.Shape(2, 8, 8, 8, 64), 0,
                                        ctypes.byref(p), b, ctypes.byref(st), 1 << 20, None, None,
                                        None)
        assert rc == want, (b, rc)


def test_empty_problems_of_the_extensions_need_no_gpu():
    """T = 0, H = 0 or W = 0: every extension entry point returns OK at once."""
    p = dsgm.dsgm_params_default(2.0)
    st = dsgm._State(1 << 20, 1 << 21, 1 << 22, 1 << 23, 1 << 24, 1 << 25)
    f = dsgm.gauss_filter(5, 1.0, True)
    for sh in ((0, 8, 8, 8, 64), (4, 0, 8, 8, 64), (4, 8, 0, 0, 0)):
        rc = lib.dsgm_forward_filtered(None, 0, dsgm.Shape(*sh), 0, ctypes.byref(p),
                                       ctypes.byref(f), ctypes.byref(st), None, None, None, None,
                                       None)
        assert rc == 0, sh
        rc = lib.dsgm_forward_grid(None, 0, dsgm.Shape(*sh), 0, ctypes.byref(p), 4,
                                   ctypes.byref(st), None, None, None, None)
        assert rc == 0, sh
    m = (ctypes.c_double * 9)(1, 0, 0, 0, 1, 0, 0, 0, 1)
    st2 = dsgm._State(1 << 26, 1 << 27, 1 << 28, 1 << 29, 1 << 30, 1 << 31)
    rc = lib.dsgm_forward_warped(None, 0, dsgm.Shape(1, 0, 8, 8, 0), 0, ctypes.byref(p), m,
                                 ctypes.byref(st), ctypes.byref(st2), None, None, None, None)
    assert rc == 0
    p8 = dsgm.dsgm_params_default(255.0, 1)
    rc = lib.dsgm_forward(None, 3, dsgm.Shape(0, 8, 8, 8, 64), 3, ctypes.byref(p8),
                          ctypes.byref(st), None, None, None, 0, 0, None, None)
    assert rc == 0
    # the 8-bit model goes with 8-bit frames only, and has no bg or checkpoints
    rc = lib.dsgm_forward(1 << 20, 1, dsgm.Shape(2, 8, 8, 8, 64), 3, ctypes.byref(p8),
                          ctypes.byref(st), 1 << 20, None, None, 0, 0, None, None)
    assert rc == -3
    rc = lib.dsgm_forward(1 << 20, 3, dsgm.Shape(2, 8, 8, 8, 64), 3, ctypes.byref(p8),
                          ctypes.byref(st), 1 << 20, 1 << 21, None, 0, 0, None, None)
    assert rc == -7
    rc = lib.dsgm_backward(1 << 20, 3, dsgm.Shape(2, 8, 8, 8, 64), 3, ctypes.byref(p8), None, 0,
                           1, None, None, 1 << 20, None, None, None, 0, None)
    assert rc == -3
    # the 8-bit preprocessing pipeline: U8 frames with U8 state only, no bg
    f = dsgm.gauss_filter(5, 1.0, True)
    rc = lib.dsgm_forward_filtered(1 << 20, 3, dsgm.Shape(2, 8, 8, 8, 64), 1, ctypes.byref(p8),
                                   ctypes.byref(f), ctypes.byref(st), 1 << 20, None, None, None,
                                   None)
    assert rc == -3
    rc = lib.dsgm_forward_filtered(1 << 20, 1, dsgm.Shape(2, 8, 8, 8, 64), 3, ctypes.byref(p8),
                                   ctypes.byref(f), ctypes.byref(st), 1 << 20, None, None, None,
                                   None)
    assert rc == -3
    rc = lib.dsgm_forward_filtered(1 << 20, 3, dsgm.Shape(2, 8, 8, 8, 64), 3, ctypes.byref(p8),
                                   ctypes.byref(f), ctypes.byref(st), 1 << 20, 1 << 21, None, None,
                                   None)
    assert rc == -7
    rc = lib.dsgm_forward_filtered(None, 3, dsgm.Shape(0, 8, 8, 8, 64), 3, ctypes.byref(p8),
                                   ctypes.byref(f), ctypes.byref(st), None, None, None, None, None)
    assert rc == 0


def test_autotune_arguments_rejected_before_any_hip_call():
    S = dsgm._tune_shape
    i32x2 = ctypes.c_int32 * 2
    chosen = i32x2(7, 7)
    # sizes of the tuner's workspace: dense min(T, 64) frames + outputs + state
    n = dsgm.dsgm_autotune_bytes(dsgm.IN_F64, dsgm.ACC_F64, 500, 48, 64)
    assert n >= 64 * 48 * 64 * (8 + 1) + 48 * 64 * (4 * 8 + 2)
    assert dsgm.dsgm_autotune_bytes(dsgm.IN_F64, dsgm.ACC_F64, 500, 48, 64, dsgm.TUNE_BG) > n
    assert dsgm.dsgm_autotune_bytes(dsgm.IN_F64, dsgm.ACC_F64, 0, 48, 64) == 0
    assert dsgm.dsgm_autotune_bytes(dsgm.IN_F64, dsgm.ACC_F32, 5, 48, 64) == 0  # bad pair
    # empty problem: nothing to tune, chosen = {0, 0}
    assert lib.dsgm_autotune(dsgm.IN_F32, dsgm.ACC_F32, S(0, 8, 8), 0, None, 0, chosen, None) == 0
    assert list(chosen) == [0, 0]
    bad = [
        ((dsgm.IN_F64, dsgm.ACC_F32, S(4, 8, 8), 0, None, 0), -3),
        ((9, dsgm.ACC_F32, S(4, 8, 8), 0, None, 0), -3),
        ((dsgm.IN_F32, dsgm.ACC_F32, S(4, 8, 8), 8, None, 0), -1),
        ((dsgm.IN_U8, dsgm.ACC_U8, S(4, 8, 8), dsgm.TUNE_CKPT, None, 0), -7),
        ((dsgm.IN_F32, dsgm.ACC_F32, S(-1, 8, 8), 0, None, 0), -2),
        ((dsgm.IN_F32, dsgm.ACC_F32, S(4, 8, 8), 0, None, 0), -1),      # no workspace
        ((dsgm.IN_F32, dsgm.ACC_F32, S(4, 8, 8), 0, ctypes.c_void_p(256), 16),
         -5),
        ((dsgm.IN_F32, dsgm.ACC_F32, S(4, 8, 8), 0, ctypes.c_void_p(260), 1 << 20),
         -4),
    ]
    for args, want in bad:
        assert lib.dsgm_autotune(*args, chosen, None) == want, (args, lib.dsgm_last_error())
    # the table: empty until a tuning run fills it; lookups need no GPU
    assert dsgm.dsgm_autotune_clear() is None
    assert dsgm.dsgm_autotune_lookup(dsgm.IN_F64, dsgm.ACC_F64, 500, 1920, 2560) == (0, 0)
    assert lib.dsgm_autotune_lookup(dsgm.IN_F64, dsgm.ACC_F64, S(5, 8, 8), 0, None) == -1
    with pytest.raises(dsgm.DSGMError):
        dsgm.dsgm_autotune_lookup(dsgm.IN_F64, dsgm.ACC_F64, 5, 8, 8, 16)


def test_host_tables_are_thread_safe():
    """The process-wide launch override and the tuner's table are shared by all
    threads: concurrent setters, lookups and clears from many threads (ctypes
    drops the GIL around each call) leave them consistent."""
    import threading
    S = dsgm._tune_shape
    errors = []

    def worker(k):
        try:
            chosen = (ctypes.c_int32 * 2)()
            for i in range(2000):
                assert lib.dsgm_set_launch(64 * (1 + (i + k) % 4), (1, 2, 4)[(i * k) % 3]) == 0
                assert lib.dsgm_autotune_lookup(dsgm.IN_F32, dsgm.ACC_F32, S(4, 8, 8 + k), 0,
                                                chosen) == 0
                assert list(chosen) == [0, 0]
                if i % 97 == 0:
                    assert lib.dsgm_autotune_clear() == 0
        except AssertionError as e:  # pragma: no cover - reported below
            errors.append((k, e))

    threads = [threading.Thread(target=worker, args=(k,)) for k in range(8)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors
    assert lib.dsgm_set_launch(0, 0) == 0


def test_count_nonfinite_rejects_before_any_hip_call():
    S = lambda T, H, W: dsgm.Shape(T, H, W, W, H * W)
    fake = ctypes.c_void_p(256)
    assert lib.dsgm_count_nonfinite(fake, 9, S(2, 3, 4), fake, None) == -3          # dtype
    assert lib.dsgm_count_nonfinite(fake, 0, S(-1, 3, 4), fake, None) == -2         # shape
    assert lib.dsgm_count_nonfinite(fake, 0, dsgm.Shape(2, 3, 4, 3, 12), fake, None) == -2
    assert lib.dsgm_count_nonfinite(fake, 0, S(2, 3, 4), None, None) == -1          # no count
    assert lib.dsgm_count_nonfinite(fake, 0, S(2, 3, 4), ctypes.c_void_p(260), None) == -4
    assert lib.dsgm_count_nonfinite(None, 0, S(2, 3, 4), fake, None) == -1          # no frames
    assert lib.dsgm_count_nonfinite(ctypes.c_void_p(258), 1, S(2, 3, 4), fake, None) == -4
    assert b"frames" in lib.dsgm_last_error()
