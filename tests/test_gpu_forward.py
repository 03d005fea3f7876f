"""GPU forward parity: the HIP path against the FP64 oracle, through the C ABI.

FP64 accumulation is bit-exact by construction (every operation rounded on
its own in the same order as the oracle), so masks, decision codes, bg and the
final state must be identical.  FP32/BF16 frames with FP64 accumulation are
fed to the oracle as the same (exactly upcast) values and must be identical
too.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from synth import device as sdev
from tests import gpu_util as G

pytestmark = pytest.mark.gpu

from paper_1702_05156_amd import dsgm


def _run_and_compare(seed, T, H, W, in_dtype=torch.float64, params=None, frames=None):
    p = params or dsgm.dsgm_params_default(2.0)
    fr, st = G.device_case(seed, T, H, W, in_dtype, torch.float64, p.age_max)
    if frames is not None:
        fr = frames(fr)
    x, st0 = G.host_case(seed, T, H, W, in_dtype, torch.float64, p.age_max)
    out = dsgm.forward(fr, st, p, bg=True, codes=True)
    torch.cuda.synchronize()
    ref = oracle.forward(x, st0, G.oracle_params(p))
    G.assert_bit_exact("codes", G.flat(out["codes"]), ref["codes"])
    G.assert_bit_exact("masks", G.flat(out["masks"]), ref["masks"])
    G.assert_bit_exact("bg", G.flat(out["bg"]), ref["bg"])
    hs = G.state_to_host(st)
    for k in ("mean_a", "var_a", "mean_c", "var_c", "age_a", "age_c"):
        G.assert_bit_exact(k, hs[k], ref[k])
    return out, ref


def test_generator_twin_bit_identical():
    T, H, W = 3, 17, 29
    for dt in (torch.float64, torch.float32, torch.bfloat16):
        d = sdev.frames(5, T, H, W, dt)
        h = synth.frames(5, T, H, W, G.GRID[dt])
        G.assert_bit_exact(f"frames {dt}", G.flat(d), h)
    st = sdev.state(6, H, W, torch.float64)
    hs = synth.state(6, H, W, "f64", 30)
    for t, k in zip(st, ("mean_a", "var_a", "mean_c", "var_c", "age_a", "age_c")):
        G.assert_bit_exact(k, t.double().cpu().numpy().ravel() if k[0] != "a" else
                           t.cpu().numpy().ravel().astype(np.int32), hs[k])
    g = sdev.grad_bg(7, T, H, W, torch.float32)
    G.assert_bit_exact("grad_bg", G.flat(g), synth.grad_bg(7, T, H, W))
    gs = sdev.grad_state(7, H, W, torch.float64)
    G.assert_bit_exact("grad_state", gs.cpu().numpy().reshape(4, -1), synth.grad_state(7, H, W))


def test_smallest_paper_size_f64_bit_exact():
    """320x240 frames, 500 of them (the paper's test sequence size), seed 0."""
    out, ref = _run_and_compare(0, 500, 240, 320)
    c = ref["codes"]
    for bit in (oracle.HIT_A, oracle.HIT_C, oracle.RESET, oracle.SWAP, oracle.FG):
        assert np.any(c & bit)


@pytest.mark.parametrize("T,H,W", [(37, 7, 13), (9, 5, 6), (5, 3, 4), (1, 1, 1), (2, 1, 3),
                                   (13, 64, 257), (6, 2, 4096)])
def test_ragged_shapes_bit_exact(T, H, W):
    _run_and_compare(11, T, H, W)


@pytest.mark.parametrize("in_dtype", [torch.float32, torch.bfloat16])
def test_low_precision_frames_f64_state_bit_exact(in_dtype):
    _run_and_compare(12, 41, 19, 24, in_dtype)


@pytest.mark.parametrize("rule,mrule", [(0, 1), (1, 0), (1, 1)])
def test_other_rules_bit_exact(rule, mrule):
    p = dsgm.dsgm_params_default(2.0, mrule)
    p.weight_rule = rule
    _run_and_compare(13, 60, 16, 40, params=p)


def test_age_cap_and_thresholds_bit_exact():
    p = dsgm.dsgm_params_default(2.0)
    p.age_max = 3
    p.theta_s = 5.0
    p.theta_d = 0.5
    _run_and_compare(14, 50, 8, 64, params=p)
    p = dsgm.dsgm_params_default(2.0)
    p.theta_s = 0.0
    _run_and_compare(15, 20, 4, 16, params=p)


def test_strided_frames_bit_exact():
    """Frames that are a view into a larger buffer (row and frame padding)."""
    T, H, W = 23, 9, 20

    def view(fr):
        big = torch.zeros((T, H + 3, W + 12), dtype=fr.dtype, device=fr.device)
        big[:, :H, :W] = fr
        return big[:, :H, :W]

    _run_and_compare(16, T, H, W, frames=view)


def test_empty_inputs():
    p = dsgm.dsgm_params_default(2.0)
    for T, H, W in ((0, 4, 4), (3, 0, 4), (3, 4, 0)):
        fr, st = G.device_case(1, max(T, 1), max(H, 1), max(W, 1))
        fr = torch.zeros((T, H, W), dtype=torch.float64, device="cuda")
        st = dsgm.State.empty(H, W)
        dsgm.dsgm_forward(fr, st, p, torch.empty((T, H, W), dtype=torch.uint8, device="cuda"))
    torch.cuda.synchronize()


def test_launch_shapes_do_not_change_results():
    T, H, W = 64, 24, 256
    p = dsgm.dsgm_params_default(2.0)
    results = []
    try:
        for block, vec in ((0, 0), (64, 1), (128, 2), (256, 4), (192, 1)):
            dsgm.dsgm_set_launch(block, vec)
            fr, st = G.device_case(17, T, H, W)
            out = dsgm.forward(fr, st, p, bg=True, ckpt_every=7)
            results.append((out, st))
    finally:
        dsgm.dsgm_set_launch(0, 0)
    torch.cuda.synchronize()
    o0, s0 = results[0]
    for o, s in results[1:]:
        for k in ("masks", "bg"):
            assert torch.equal(o[k], o0[k]), k
        assert torch.equal(G.ckpt_payload(o["ckpt"], T, H, W, 7, 8),
                           G.ckpt_payload(o0["ckpt"], T, H, W, 7, 8))
        for a, b in zip(s.planes(), s0.planes()):
            assert torch.equal(a, b)
    # the debug codes variant (one pixel per lane) gives the same results
    fr, st = G.device_case(17, T, H, W)
    oc = dsgm.forward(fr, st, p, bg=True, codes=True)
    assert torch.equal(oc["masks"], o0["masks"]) and torch.equal(oc["bg"], o0["bg"])
    assert torch.equal((oc["codes"] & 16) != 0, o0["masks"] == 255)


def test_streaming_equals_fused():
    T, H, W = 30, 12, 40
    p = dsgm.dsgm_params_default(2.0)
    fr, st = G.device_case(18, T, H, W)
    st2 = st.clone()
    fused = dsgm.forward(fr, st, p, bg=True, codes=True)
    for t in range(T):
        one = dsgm.forward(fr[t:t + 1], st2, p, bg=True, codes=True)
        for k in ("masks", "bg", "codes"):
            assert torch.equal(one[k][0], fused[k][t]), (t, k)
    for a, b in zip(st.planes(), st2.planes()):
        assert torch.equal(a, b)


@pytest.mark.parametrize("in_dtype,acc_dtype,acc", [
    (torch.float64, torch.float64, dsgm.ACC_F64), (torch.bfloat16, torch.float32, dsgm.ACC_F32),
    (torch.float32, torch.float64, dsgm.ACC_F64_IO32)])
@pytest.mark.parametrize("W", [40, 37])
@pytest.mark.parametrize("bg,printed", [(False, False), (True, False), (False, True), (True, True)])
def test_one_frame_calls_equal_the_fused_call(in_dtype, acc_dtype, acc, W, bg, printed):
    """One-frame calls without checkpoints or codes run their own kernel
    variant: frame by frame it gives the masks, bg and state of one call over
    all frames, for every output and mask-rule variant, at the widest pixels
    per lane the type allows (W = 40) and at one (W = 37)."""
    T, H = 12, 9
    p = dsgm.dsgm_params_default(2.0, dsgm.MASK_PRINTED if printed else dsgm.MASK_VARIANCE)
    fr, st = G.device_case(21, T, H, W, in_dtype, acc_dtype)
    st2 = st.clone()
    fused = dsgm.forward(fr, st, p, bg=bg, acc=acc)
    for t in range(T):
        one = dsgm.forward(fr[t:t + 1], st2, p, bg=bg, acc=acc)
        assert torch.equal(one["masks"][0], fused["masks"][t]), t
        if bg:
            assert torch.equal(one["bg"][0], fused["bg"][t]), t
    for a, b in zip(st.planes(), st2.planes()):
        assert torch.equal(a, b)


def test_checkpoints_hold_the_oracle_state():
    T, H, W, K = 45, 6, 32, 8
    p = dsgm.dsgm_params_default(2.0)
    fr, st = G.device_case(19, T, H, W)
    x, st0 = G.host_case(19, T, H, W)
    out = dsgm.forward(fr, st, p, ckpt_every=K)
    torch.cuda.synchronize()
    ck = out["ckpt"].cpu().numpy()
    px = H * W
    fpl = (px * 8 + 255) // 256 * 256
    apl = (px + 255) // 256 * 256
    slot = 4 * fpl + 2 * apl
    cur = st0
    for j in range((T + K - 1) // K):
        base = j * slot
        planes = [ck[base + i * fpl: base + i * fpl + px * 8].view(np.float64) for i in range(4)]
        ages = [ck[base + 4 * fpl + i * apl: base + 4 * fpl + i * apl + px].astype(np.int32)
                for i in range(2)]
        for name, got in zip(("mean_a", "var_a", "mean_c", "var_c"), planes):
            G.assert_bit_exact(f"ckpt{j}.{name}", got, cur[name])
        G.assert_bit_exact(f"ckpt{j}.age_a", ages[0], cur["age_a"])
        G.assert_bit_exact(f"ckpt{j}.age_c", ages[1], cur["age_c"])
        r = oracle.forward(x[j * K:(j + 1) * K], cur, G.oracle_params(p), bg=False, codes=False)
        cur = {k: r[k] for k in st0}


def test_state_init_from_frame():
    H, W = 7, 9
    p = dsgm.dsgm_params_default(2.0)
    fr = sdev.frames(20, 1, H, W)[0]
    st = dsgm.State.empty(H, W)
    dsgm.dsgm_state_init_from_frame(fr, st, p)
    torch.cuda.synchronize()
    assert torch.equal(st.mean_a, fr) and torch.equal(st.mean_c, fr)
    assert torch.all(st.var_a == p.var_init) and torch.all(st.var_c == p.var_init)
    assert torch.all(st.age_a == 1) and torch.all(st.age_c == 1)


@pytest.mark.slow
def test_full_size_f64_sampled_bit_exact():
    """1920x2560 pixels x 500 frames, FP64, seed 1, masks only -- the launch
    configuration the benchmark times.  Pixels are independent, so checking a
    random sample of pixels against the oracle over all 500 frames is an exact
    check for those pixels."""
    T, H, W = 500, 1920, 2560
    p = dsgm.dsgm_params_default(2.0)
    fr, st = G.device_case(1, T, H, W)
    masks = torch.empty((T, H, W), dtype=torch.uint8, device="cuda")
    dsgm.dsgm_forward(fr, st, p, masks)
    torch.cuda.synchronize()
    rng = np.random.default_rng(1)
    pix = np.unique(np.concatenate([rng.choice(H * W, 4096, replace=False),
                                    [0, W - 1, H * W - W, H * W - 1]]))
    x, st0 = G.host_case(1, T, H, W, pix=pix)
    ref = oracle.forward(x, st0, G.oracle_params(p), bg=False, codes=False)
    pix_t = torch.as_tensor(pix, device="cuda")
    got_masks = masks.view(T, H * W)[:, pix_t].cpu().numpy()
    G.assert_bit_exact("masks", got_masks, ref["masks"])
    hs = G.state_to_host(st)
    for k in ("mean_a", "var_a", "mean_c", "var_c", "age_a", "age_c"):
        G.assert_bit_exact(k, hs[k][pix], ref[k])
    # a property that holds at any size: masks are 0/255 everywhere
    assert int(((masks != 0) & (masks != 255)).sum()) == 0
    del fr, masks


def test_streaming_full_size_f64_bit_exact():
    """One dsgm_forward call per frame, as the streaming benchmark makes them:
    1920 x 2560 FP64 frames of the structured video (seed 1), three calls
    from a random mid-run state; every pixel's masks and final state equal
    the oracle's."""
    T, H, W, seed = 3, 1920, 2560, 1
    p = dsgm.dsgm_params_default(2.0)
    fr = sdev.video(seed, T, H, W, torch.float64)
    st = dsgm.State(*sdev.state(seed, H, W, torch.float64))
    masks = torch.empty((T, H, W), dtype=torch.uint8, device="cuda")
    for t in range(T):
        dsgm.dsgm_forward(fr[t:t + 1], st, p, masks[t:t + 1])
    torch.cuda.synchronize()
    x = synth.video(seed, T, H, W).reshape(T, -1)
    st0 = synth.state(seed, H, W, "f64", p.age_max)
    ref = oracle.forward(x, st0, G.oracle_params(p), bg=False, codes=False)
    G.assert_bit_exact("masks", masks.cpu().numpy().reshape(T, -1), ref["masks"])
    hs = G.state_to_host(st)
    for k in ("mean_a", "var_a", "mean_c", "var_c", "age_a", "age_c"):
        G.assert_bit_exact(k, hs[k], ref[k])


def _certify_fp32(codes_gpu, ref, tol_margin=1e-5):
    """Decision certification for a reduced-precision run.  For every pixel
    whose decision codes differ from the FP64 oracle's, the first differing
    frame must differ in a decision whose FP64 margin is within tol_margin of
    its threshold (the A test, the C test, or the background test); a swap or
    reset can only differ after a differing match decision.  Returns the
    boolean mask of diverged pixels (structural decisions differ)."""
    c_gpu = codes_gpu.astype(np.int32)
    c_ref = ref["codes"].astype(np.int32)
    m = ref["margins"]
    T, N = c_ref.shape
    struct = (c_gpu & 0x0F) != (c_ref & 0x0F)
    diverged = struct.any(axis=0)
    first = np.where(diverged, struct.argmax(axis=0), T)
    for j in np.nonzero(diverged)[0]:
        t = first[j]
        a_differs = (c_gpu[t, j] & 1) != (c_ref[t, j] & 1)
        mg = abs(m[t, j, 0]) if a_differs else abs(m[t, j, 1])
        assert mg <= tol_margin, (j, t, c_gpu[t, j], c_ref[t, j], m[t, j])
    # foreground flips before the pixel diverges must be background-test near ties
    fgdiff = ((c_gpu & 16) != (c_ref & 16)) & (np.arange(T)[:, None] < first[None, :])
    for t, j in zip(*np.nonzero(fgdiff)):
        assert abs(m[t, j, 2]) <= tol_margin, (t, j, m[t, j])
    return diverged


@pytest.mark.parametrize("in_dtype", [torch.float32, torch.bfloat16])
def test_fp32_state_certified_against_oracle(in_dtype):
    """FP32 state and arithmetic on the paper-size sequence (320x240x500): the
    oracle runs in FP64 on the same values (frames on the storage grid, state
    on the FP32 grid).  Every pixel whose decisions differ is certified as a
    near tie; at most 1e-3 of the pixels may diverge; the others must agree
    to |dm| <= 1e-5 and |dv| <= 1e-5 * max(v, var_init) over all frames."""
    T, H, W, seed = 500, 240, 320, 31
    p = dsgm.dsgm_params_default(2.0)
    fr, st = G.device_case(seed, T, H, W, in_dtype, torch.float32)
    x, s0 = G.host_case(seed, T, H, W, in_dtype, torch.float32)
    out = dsgm.forward(fr, st, p, bg=True, codes=True)
    torch.cuda.synchronize()
    ref = oracle.forward(x, s0, G.oracle_params(p), margins=True)
    div = _certify_fp32(G.flat(out["codes"]), ref)
    assert div.mean() <= 1e-3, div.mean()
    ok = ~div
    bg = G.flat(out["bg"])
    assert np.max(np.abs(bg[:, ok] - ref["bg"][:, ok])) <= 1e-5
    hs = G.state_to_host(st)
    for k in ("mean_a", "mean_c"):
        assert np.max(np.abs(hs[k][ok] - ref[k][ok])) <= 1e-5, k
    for k in ("var_a", "var_c"):
        assert np.max(np.abs(hs[k][ok] - ref[k][ok]) / np.maximum(ref[k][ok], p.var_init)) <= 1e-5, k
    for k in ("age_a", "age_c"):
        G.assert_bit_exact(k, hs[k][ok], ref[k][ok])


@pytest.mark.parametrize("in_dtype", [torch.float32, torch.bfloat16])
def test_io32_forward_is_fp64_rounded_once(in_dtype):
    """FP64 state and arithmetic with an FP32 bg array: codes, masks and state
    bit-identical to the FP64 oracle, bg equal to the oracle's bg rounded to
    FP32 (round to nearest even)."""
    T, H, W, seed = 300, 48, 160, 32
    p = dsgm.dsgm_params_default(2.0)
    fr, st = G.device_case(seed, T, H, W, in_dtype, torch.float64)
    x, s0 = G.host_case(seed, T, H, W, in_dtype, torch.float64)
    out = dsgm.forward(fr, st, p, bg=True, codes=True, acc=dsgm.ACC_F64_IO32)
    assert out["bg"].dtype == torch.float32
    torch.cuda.synchronize()
    ref = oracle.forward(x, s0, G.oracle_params(p))
    G.assert_bit_exact("codes", G.flat(out["codes"]), ref["codes"])
    G.assert_bit_exact("masks", G.flat(out["masks"]), ref["masks"])
    G.assert_bit_exact("bg", out["bg"].cpu().numpy().reshape(T, -1),
                       ref["bg"].astype(np.float32))
    hs = G.state_to_host(st)
    for k in ("mean_a", "var_a", "mean_c", "var_c", "age_a", "age_c"):
        G.assert_bit_exact(k, hs[k], ref[k])


def _sample_pixels(seed, H, W, n):
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([rng.choice(H * W, n, replace=False),
                                     [0, W - 1, H * W - W, H * W - 1]]))


@pytest.mark.slow
def test_full_size_bf16_fp32_masks_only_certified():
    """1920x2560 pixels x 500 frames, BF16 frames, FP32 state, masks only, seed
    1: the launch the benchmark's mixed leg times (four pixels per lane, no
    decision codes).  Sampled pixels are certified against the FP64 oracle
    from the masks alone: identical masks until the oracle's first near tie
    (FP64 margin <= 1e-5), the final state within 1e-5 on pixels with none.
    Over all pixels at most 1e-3 may show any mask difference from the FP64
    path (the oracle's arithmetic bit for bit, tested at this size), and the
    same pass with decision codes gives the same bits."""
    T, H, W, seed = 500, 1920, 2560, 1
    p = dsgm.dsgm_params_default(2.0)
    fr = sdev.frames(seed, T, H, W, torch.bfloat16)
    st = dsgm.State(*sdev.state(seed, H, W, torch.float32))
    st_cd = st.clone()
    st64 = dsgm.State(*(t.double() if t.is_floating_point() else t.clone() for t in st.planes()))
    masks = torch.empty((T, H, W), dtype=torch.uint8, device="cuda")
    dsgm.dsgm_forward(fr, st, p, masks)
    pix = _sample_pixels(1, H, W, 2048)
    x, st0 = G.host_case(seed, T, H, W, torch.bfloat16, torch.float32, pix=pix)
    ref = oracle.forward(x, st0, G.oracle_params(p), margins=True)
    pt = torch.as_tensor(pix, device="cuda")
    clear, differs = G.certify_masks(masks.view(T, -1)[:, pt].cpu().numpy(), ref)
    hs = G.state_to_host(st)
    hs = {k: v[pix] for k, v in hs.items()}
    G.assert_state_close(hs, ref, clear, p.var_init)
    assert clear.mean() > 0.9 and not differs[clear].any()
    # every pixel: mask differences against the FP64 path
    m64 = torch.empty_like(masks)
    dsgm.dsgm_forward(fr, st64, p, m64)
    frac = float((masks != m64).any(dim=0).float().mean().item())
    assert frac <= 1e-3, frac
    del st64, m64
    # the one-pixel-per-lane variant with decision codes: the same bits
    m_cd, codes = torch.empty_like(masks), torch.empty_like(masks)
    dsgm.dsgm_forward(fr, st_cd, p, m_cd, codes=codes)
    torch.cuda.synchronize()
    assert torch.equal(m_cd, masks)
    for a, b in zip(st_cd.planes(), st.planes()):
        assert torch.equal(a, b)
    del fr, masks, m_cd, codes
