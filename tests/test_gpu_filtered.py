"""GPU parity of the forward with fused preprocessing (dsgm_forward_filtered):
the separable blur and the 3 x 3 median (Sec. 2.1, 3.3.1) feeding the update,
against the preprocessing oracle followed by the update oracle.  FP64 is
bit-exact (same sums in the same order, exact median selection); FP32 state
is held to the certified tolerance."""
import numpy as np
import pytest
import torch

import oracle
import synth
from synth import device as sdev
from tests import gpu_util as G

pytestmark = pytest.mark.gpu

from paper_1702_05156_amd import dsgm



def _case(seed, T, H, W, n, median, in_dtype=torch.float64, sigma=1.0, frames=None, params=None):
    p = params or dsgm.dsgm_params_default(2.0)
    filt = dsgm.gauss_filter(n, sigma, median) if n else dsgm.gauss_filter(0, 1.0, median)
    fr, st = G.device_case(seed, T, H, W, in_dtype, torch.float64)
    if frames is not None:
        fr = frames(fr)
    out = dsgm.forward_filtered(fr, st, p, filt, bg=True, filtered=True, codes=True)
    torch.cuda.synchronize()
    x, st0 = G.host_case(seed, T, H, W, in_dtype, torch.float64)
    w = oracle.gauss_weights(n, sigma) if n else None
    xf = oracle.preprocess(x.reshape(T, H, W), w, median=bool(median)).reshape(T, H * W)
    return p, out, st, xf, st0


@pytest.mark.parametrize("n,median", [(5, 1), (3, 1), (7, 1), (5, 0), (0, 1), (0, 0), (1, 1)])
def test_filtered_frames_and_update_f64_bit_exact(n, median):
    T, H, W = 23, 37, 150   # several tiles, ragged in both directions
    p, out, st, xf, st0 = _case(41, T, H, W, n, median)
    G.assert_bit_exact("filtered", G.flat(out["filtered"]), xf)
    ref = oracle.forward(xf, st0, G.oracle_params(p))
    G.assert_bit_exact("codes", G.flat(out["codes"]), ref["codes"])
    G.assert_bit_exact("masks", G.flat(out["masks"]), ref["masks"])
    G.assert_bit_exact("bg", G.flat(out["bg"]), ref["bg"])
    hs = G.state_to_host(st)
    for k in ("mean_a", "var_a", "mean_c", "var_c", "age_a", "age_c"):
        G.assert_bit_exact(k, hs[k], ref[k])


@pytest.mark.parametrize("wr,mr", [(1, 0), (0, 1), (1, 1)])
def test_filtered_other_rules_f64_bit_exact(wr, mr):
    """The appendix's weights (1/a) and its printed mask rule on the fused path
    (the mask rule selects a compiled variant of the kernel)."""
    p = dsgm.dsgm_params_default(2.0, mr)
    p.weight_rule = wr
    T, H, W = 15, 37, 150
    p, out, st, xf, st0 = _case(42, T, H, W, 5, 1, params=p)
    G.assert_bit_exact("filtered", G.flat(out["filtered"]), xf)
    ref = oracle.forward(xf, st0, G.oracle_params(p))
    G.assert_bit_exact("codes", G.flat(out["codes"]), ref["codes"])
    G.assert_bit_exact("masks", G.flat(out["masks"]), ref["masks"])
    hs = G.state_to_host(st)
    for k in ("mean_a", "var_a", "mean_c", "var_c", "age_a", "age_c"):
        G.assert_bit_exact(k, hs[k], ref[k])


@pytest.mark.parametrize("T,H,W", [(3, 1, 1), (4, 1, 70), (4, 70, 1), (5, 16, 64), (2, 17, 65),
                                   (1, 2, 3)])
def test_filtered_edge_shapes(T, H, W):
    p, out, st, xf, st0 = _case(42, T, H, W, 5, 1)
    G.assert_bit_exact("filtered", G.flat(out["filtered"]), xf)
    ref = oracle.forward(xf, st0, G.oracle_params(p))
    G.assert_bit_exact("masks", G.flat(out["masks"]), ref["masks"])
    hs = G.state_to_host(st)
    for k in ("mean_a", "var_a", "age_a", "age_c"):
        G.assert_bit_exact(k, hs[k], ref[k])


def test_filtered_strided_frames():
    """Frames that are a view with row and frame padding (scalar stores)."""
    T, H, W = 9, 20, 70

    def pad(fr):
        big = torch.zeros((T, H + 3, W + 5), dtype=fr.dtype, device=fr.device)
        big[:, :H, :W] = fr
        return big[:, :H, :W]
    p, out, st, xf, st0 = _case(43, T, H, W, 5, 1, frames=pad)
    G.assert_bit_exact("filtered", G.flat(out["filtered"]), xf)
    ref = oracle.forward(xf, st0, G.oracle_params(p))
    G.assert_bit_exact("masks", G.flat(out["masks"]), ref["masks"])


def test_filtered_video_f64_bit_exact():
    """The structured video from a state initialised on the first filtered frame."""
    T, H, W = 120, 48, 96
    p = dsgm.dsgm_params_default(2.0)
    filt = dsgm.gauss_filter(5, 1.0, True)
    fr = sdev.video(44, T, H, W, torch.float64)
    x = synth.video(44, T, H, W)
    xf = oracle.preprocess(x.reshape(T, H, W), oracle.gauss_weights(5, 1.0)).reshape(T, H * W)
    st = dsgm.State.empty(H, W)
    ff0 = torch.as_tensor(xf[0].reshape(H, W), device="cuda")
    dsgm.dsgm_state_init_from_frame(ff0, st, p)
    out = dsgm.forward_filtered(fr, st, p, filt, filtered=True, codes=True)
    torch.cuda.synchronize()
    G.assert_bit_exact("filtered", G.flat(out["filtered"]), xf)
    n = H * W
    st0 = {"mean_a": xf[0].copy(), "mean_c": xf[0].copy(), "var_a": np.full(n, p.var_init),
           "var_c": np.full(n, p.var_init), "age_a": np.ones(n, np.int32),
           "age_c": np.ones(n, np.int32)}
    ref = oracle.forward(xf, st0, G.oracle_params(p))
    G.assert_bit_exact("codes", G.flat(out["codes"]), ref["codes"])


@pytest.mark.parametrize("in_dtype", [torch.bfloat16, torch.float32])
def test_filtered_fp32_within_tolerance(in_dtype):
    """FP32 state and arithmetic (the blur with fused multiply-adds): the
    filtered frames agree with the FP64 oracle to 1e-6; decisions that differ
    are certified near ties of the oracle run on the oracle's filtered frames."""
    from tests.test_gpu_forward import _certify_fp32
    T, H, W, seed = 60, 64, 128, 45
    p = dsgm.dsgm_params_default(2.0)
    filt = dsgm.gauss_filter(5, 1.0, True)
    fr, st = G.device_case(seed, T, H, W, in_dtype, torch.float32)
    out = dsgm.forward_filtered(fr, st, p, filt, bg=True, filtered=True, codes=True)
    torch.cuda.synchronize()
    x, st0 = G.host_case(seed, T, H, W, in_dtype, torch.float32)
    xf = oracle.preprocess(x.reshape(T, H, W), oracle.gauss_weights(5, 1.0)).reshape(T, H * W)
    assert np.max(np.abs(G.flat(out["filtered"]) - xf)) <= 1e-6
    ref = oracle.forward(xf, st0, G.oracle_params(p), margins=True)
    div = _certify_fp32(G.flat(out["codes"]), ref, tol_margin=1e-5)
    assert div.mean() <= 1e-3, div.mean()


@pytest.mark.slow
def test_full_size_filtered_f64_sampled_bit_exact():
    """1920x2560x500, FP64, 5-tap Gaussian (sigma 1) and 3x3 median fused, masks
    only -- the launch the benchmark times.  A filtered pixel depends on the raw
    frame within 3 rows and columns, so the oracle filters a 7x7 crop around each
    sampled pixel (cut at the frame edges, where both clamp alike) and runs the
    update on the crop's centre."""
    T, H, W, seed = 500, 1920, 2560, 1
    p = dsgm.dsgm_params_default(2.0)
    filt = dsgm.gauss_filter(5, 1.0, True)
    fr, st = G.device_case(seed, T, H, W)
    masks = torch.empty((T, H, W), dtype=torch.uint8, device="cuda")
    dsgm.dsgm_forward_filtered(fr, st, p, filt, masks)
    torch.cuda.synchronize()
    rng = np.random.default_rng(11)
    pix = np.unique(np.concatenate([rng.choice(H * W, 256, replace=False),
                                    [0, 1, W - 1, W, H * W - W, H * W - 1, 2 * W + 2]]))
    w = oracle.gauss_weights(5, 1.0)
    xf = np.empty((T, pix.size))
    for k, q in enumerate(pix):
        y, x = divmod(int(q), W)
        ys = np.arange(max(0, y - 3), min(H, y + 4))
        xs = np.arange(max(0, x - 3), min(W, x + 4))
        crop_pix = (ys[:, None] * W + xs[None, :]).ravel()
        raw = synth.frames(seed, T, H, W, "f64", pix=crop_pix).reshape(T, ys.size, xs.size)
        xf[:, k] = oracle.preprocess(raw, w)[:, y - ys[0], x - xs[0]]
    _, st0 = G.host_case(seed, 1, H, W, pix=pix)
    ref = oracle.forward(xf, st0, G.oracle_params(p), bg=False, codes=False)
    pix_t = torch.as_tensor(pix, device="cuda")
    G.assert_bit_exact("masks", masks.view(T, H * W)[:, pix_t].cpu().numpy(), ref["masks"])
    hs = G.state_to_host(st)
    for k in ("mean_a", "var_a", "mean_c", "var_c", "age_a", "age_c"):
        G.assert_bit_exact(k, hs[k][pix], ref[k])
    del fr, masks


# ---------------------------------------- the appendix's 8-bit pipeline, end to end
def _u8_case(seed, T, H, W):
    x = (synth.video_levels(seed, T, H, W) + 128).astype(np.uint8).reshape(T, H, W)
    rng = np.random.default_rng(seed)
    st = {k: rng.integers(0, 256, H * W).astype(np.uint8) for k in ("mean_a", "var_a", "mean_c", "var_c")}
    st["age_a"] = rng.integers(1, 31, H * W).astype(np.uint8)
    st["age_c"] = rng.integers(1, 31, H * W).astype(np.uint8)
    return x, st


def _u8_state(st, H, W):
    t = lambda k: torch.as_tensor(st[k].reshape(H, W), device="cuda").contiguous()
    return dsgm.State(t("mean_a"), t("var_a"), t("mean_c"), t("var_c"), t("age_a"), t("age_c"))


def _u8_check(out, dst, x, st, p, n, median, sigma=1.0):
    T = x.shape[0]
    w = oracle.gauss_weights(n, sigma) if n > 1 else None
    xf = oracle.preprocess_u8(x, w, median=bool(median))
    G.assert_bit_exact("filtered", G.flat(out["filtered"]).astype(np.int64),
                       xf.reshape(T, -1).astype(np.int64))
    ref = oracle.forward_u8(xf.reshape(T, -1), st, G.oracle_params(p))
    G.assert_bit_exact("codes", G.flat(out["codes"]).astype(np.int64), ref["codes"].astype(np.int64))
    G.assert_bit_exact("masks", G.flat(out["masks"]).astype(np.int64), ref["masks"].astype(np.int64))
    for k in ("mean_a", "var_a", "mean_c", "var_c", "age_a", "age_c"):
        got = getattr(dst, k).cpu().numpy().ravel()
        G.assert_bit_exact(k, got.astype(np.int64), ref[k].astype(np.int64))


@pytest.mark.parametrize("n,median", [(5, 1), (3, 1), (7, 1), (5, 0), (0, 1), (0, 0), (1, 1)])
def test_u8_filtered_pipeline_bit_exact(n, median):
    """U8 frames and state: the appendix's two-dimensional single-precision
    blur written back to 8 bits, the 3 x 3 median of the 8-bit image and the
    8-bit as-run update, all integer outputs identical to the oracle's."""
    T, H, W = 23, 37, 150   # several tiles, ragged in both directions
    x, st = _u8_case(51, T, H, W)
    p = dsgm.dsgm_params_default(255.0)
    filt = dsgm.gauss_filter(n, 1.0, median) if n else dsgm.gauss_filter(0, 1.0, median)
    dst = _u8_state(st, H, W)
    out = dsgm.forward_filtered(torch.as_tensor(x, device="cuda"), dst, p, filt, filtered=True,
                                codes=True)
    torch.cuda.synchronize()
    _u8_check(out, dst, x, st, p, n, median)


@pytest.mark.parametrize("wr,mr", [(1, 1), (1, 0), (0, 1)])
def test_u8_filtered_other_rules_and_sigma(wr, mr):
    p = dsgm.dsgm_params_default(255.0, mr)
    p.weight_rule = wr
    T, H, W = 19, 21, 70
    x, st = _u8_case(52 + wr + 2 * mr, T, H, W)
    filt = dsgm.gauss_filter(5, 1.7, True)
    dst = _u8_state(st, H, W)
    out = dsgm.forward_filtered(torch.as_tensor(x, device="cuda"), dst, p, filt, filtered=True,
                                codes=True)
    torch.cuda.synchronize()
    _u8_check(out, dst, x, st, p, 5, 1, sigma=1.7)


@pytest.mark.parametrize("T,H,W", [(3, 1, 1), (4, 1, 70), (4, 70, 1), (5, 16, 64), (2, 17, 65),
                                   (1, 2, 3)])
def test_u8_filtered_edge_shapes(T, H, W):
    x, st = _u8_case(53, T, H, W)
    p = dsgm.dsgm_params_default(255.0)
    filt = dsgm.gauss_filter(5, 1.0, True)
    dst = _u8_state(st, H, W)
    out = dsgm.forward_filtered(torch.as_tensor(x, device="cuda"), dst, p, filt, filtered=True,
                                codes=True)
    torch.cuda.synchronize()
    _u8_check(out, dst, x, st, p, 5, 1)


def test_u8_filtered_strided_frames_and_rejections():
    """A padded view of the frames (scalar stores), and the argument checks of
    the 8-bit pairing."""
    T, H, W = 9, 20, 70
    x, st = _u8_case(54, T, H, W)
    big = torch.zeros((T, H + 3, W + 5), dtype=torch.uint8, device="cuda")
    big[:, :H, :W] = torch.as_tensor(x, device="cuda")
    fr = big[:, :H, :W]
    p = dsgm.dsgm_params_default(255.0)
    filt = dsgm.gauss_filter(3, 0.8, True)
    dst = _u8_state(st, H, W)
    out = dsgm.forward_filtered(fr, dst, p, filt, filtered=True, codes=True)
    torch.cuda.synchronize()
    _u8_check(out, dst, x, st, p, 3, 1, sigma=0.8)
    with pytest.raises(dsgm.DSGMError) as e:      # no bg in the 8-bit model
        dsgm.forward_filtered(fr, _u8_state(st, H, W), p, filt, bg=True)
    assert e.value.status == -7
    f32 = dsgm.State(*[torch.zeros((H, W), dtype=torch.float32, device="cuda") for _ in range(4)],
                     *[torch.ones((H, W), dtype=torch.uint8, device="cuda") for _ in range(2)])
    with pytest.raises(dsgm.DSGMError) as e:      # U8 frames need U8 state
        dsgm.forward_filtered(fr, f32, p, filt, acc=dsgm.ACC_F32)
    assert e.value.status == -3


@pytest.mark.slow
def test_full_size_u8_filtered_sampled_bit_exact():
    """1920x2560x60 U8 frames of the structured video, 5-tap Gaussian and 3x3
    median as the appendix runs them on 8-bit images, fused with the 8-bit
    update.  A filtered pixel depends on the raw frame within 3 rows and
    columns, so the oracle filters a 7x7 crop around each sampled pixel (cut at
    the frame edges, where both clamp alike) and runs the update on its centre."""
    T, H, W, seed = 60, 1920, 2560, 5
    p = dsgm.dsgm_params_default(255.0)
    filt = dsgm.gauss_filter(5, 1.0, True)
    fr = (sdev.video(seed, T, H, W, torch.float32) * 128 + 128).to(torch.uint8)
    rng = np.random.default_rng(12)
    st = {k: rng.integers(0, 256, H * W).astype(np.uint8) for k in ("mean_a", "var_a", "mean_c", "var_c")}
    st["age_a"] = rng.integers(1, 31, H * W).astype(np.uint8)
    st["age_c"] = rng.integers(1, 31, H * W).astype(np.uint8)
    dst = _u8_state(st, H, W)
    masks = torch.empty((T, H, W), dtype=torch.uint8, device="cuda")
    dsgm.dsgm_forward_filtered(fr, dst, p, filt, masks)
    torch.cuda.synchronize()
    pix = np.unique(np.concatenate([rng.choice(H * W, 256, replace=False),
                                    [0, 1, W - 1, W, H * W - W, H * W - 1, 2 * W + 2]]))
    w = oracle.gauss_weights(5, 1.0)
    xf = np.empty((T, pix.size), np.uint8)
    for k, q in enumerate(pix):
        y, x = divmod(int(q), W)
        ys = np.arange(max(0, y - 3), min(H, y + 4))
        xs = np.arange(max(0, x - 3), min(W, x + 4))
        crop_pix = (ys[:, None] * W + xs[None, :]).ravel()
        raw = (synth.video_levels(seed, T, H, W, pix=crop_pix) + 128).astype(np.uint8)
        xf[:, k] = oracle.preprocess_u8(raw.reshape(T, ys.size, xs.size), w)[:, y - ys[0], x - xs[0]]
    st0 = {k: v[pix] for k, v in st.items()}
    ref = oracle.forward_u8(xf, st0, G.oracle_params(p), codes=False)
    pix_t = torch.as_tensor(pix, device="cuda")
    G.assert_bit_exact("masks", masks.view(T, H * W)[:, pix_t].cpu().numpy().astype(np.int64),
                       ref["masks"].astype(np.int64))
    for k in ("mean_a", "var_a", "mean_c", "var_c", "age_a", "age_c"):
        got = getattr(dst, k).cpu().numpy().ravel()[pix]
        G.assert_bit_exact(k, got.astype(np.int64), ref[k].astype(np.int64))
    del fr, masks
