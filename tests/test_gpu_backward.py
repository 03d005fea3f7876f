"""GPU adjoint parity: dsgm_backward against the oracle's reverse mode, central
differences of the GPU forward, and torch.autograd.

With FP64 accumulation the adjoint is bit-identical to the oracle's (same chain
rule, same operation order); with FP32 it is compared with the oracle run
under the GPU's own decisions (forced codes), relative L2 error <= 1e-5.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from synth import device as sdev
from tests import gpu_util as G

pytestmark = pytest.mark.gpu

from paper_1702_05156_amd import dsgm


def _grads(seed, T, H, W, dt):
    gbg = sdev.grad_bg(seed, T, H, W, dt)
    gst = sdev.grad_state(seed, H, W, dt)
    return gbg, tuple(gst[i].contiguous() for i in range(4))


def _gpu_fwd_bwd(seed, T, H, W, K, in_dtype, acc_dtype, params=None, use_gbg=True, use_gst=True):
    p = params or dsgm.dsgm_params_default(2.0)
    fr, st = G.device_case(seed, T, H, W, in_dtype, acc_dtype, p.age_max)
    out = dsgm.forward(fr, st, p, bg=True, codes=True, ckpt_every=K)
    gbg, gst = _grads(seed + 100, T, H, W, acc_dtype)
    acc = dsgm.ACC_F64 if acc_dtype == torch.float64 else dsgm.ACC_F32
    r = dsgm.backward(fr, p, out["ckpt"], K, acc, gbg if use_gbg else None, gst if use_gst else None)
    torch.cuda.synchronize()
    return p, out, r, (gbg if use_gbg else None), (gst if use_gst else None)


def _oracle_bwd(seed, T, H, W, in_dtype, acc_dtype, p, codes, gbg, gst):
    x, st0 = G.host_case(seed, T, H, W, in_dtype, acc_dtype, p.age_max)
    gb = None if gbg is None else G.flat(gbg)
    gs = None if gst is None else np.stack([g.double().cpu().numpy().ravel() for g in gst])
    return oracle.backward(x, st0, G.oracle_params(p), gb, gs, forced=G.flat(codes).astype(np.uint8))


@pytest.mark.parametrize("K", [1, 7, 16, 17, 40, 100])
def test_f64_adjoint_bit_exact(K):
    T, H, W, seed = 100, 12, 40, 21
    p, out, r, gbg, gst = _gpu_fwd_bwd(seed, T, H, W, K, torch.float64, torch.float64)
    ref = _oracle_bwd(seed, T, H, W, torch.float64, torch.float64, p, out["codes"], gbg, gst)
    G.assert_bit_exact("grad_frames", G.flat(r["grad_frames"]), ref["grad_frames"])
    for i, name in enumerate(("mean_a", "var_a", "mean_c", "var_c")):
        G.assert_bit_exact(f"grad_{name}0", r["grad_state0"][i].cpu().numpy().ravel(),
                           ref["grad_state0"][i])
    px = r["workspace"][: H * W * 8].view(torch.float64).cpu().numpy()
    G.assert_bit_exact("grad_var_init per pixel", px, ref["grad_var_init_px"])
    gvi = float(r["grad_var_init"].item())
    assert gvi == pytest.approx(ref["grad_var_init"], rel=1e-15, abs=1e-300)


@pytest.mark.parametrize("in_dtype", [torch.float64, torch.float32])
def test_f64_adjoint_appendix_weights_bit_exact(in_dtype):
    """The adjoint under the appendix's weights (w = 1/a), FP64 arithmetic,
    against the oracle's reverse mode under the same decisions."""
    T, H, W, K, seed = 60, 10, 24, 16, 28
    p = dsgm.dsgm_params_default(2.0, dsgm.MASK_PRINTED)
    p.weight_rule = dsgm.WEIGHT_APPENDIX
    p_, out, r, gbg, gst = _gpu_fwd_bwd(seed, T, H, W, K, in_dtype, torch.float64, params=p)
    ref = _oracle_bwd(seed, T, H, W, in_dtype, torch.float64, p, out["codes"], gbg, gst)
    G.assert_bit_exact("grad_frames", G.flat(r["grad_frames"]), ref["grad_frames"])
    for i, name in enumerate(("mean_a", "var_a", "mean_c", "var_c")):
        G.assert_bit_exact(f"grad_{name}0", r["grad_state0"][i].cpu().numpy().ravel(),
                           ref["grad_state0"][i])
    px = r["workspace"][: H * W * 8].view(torch.float64).cpu().numpy()
    G.assert_bit_exact("grad_var_init per pixel", px, ref["grad_var_init_px"])


@pytest.mark.parametrize("in_dtype", [torch.float32, torch.bfloat16])
def test_adjoint_does_not_depend_on_checkpoint_interval(in_dtype):
    """FP32 state: the replay recomputes the forward's values exactly, so every
    checkpoint interval gives the same bits.  The intervals cover chunks of
    every kind the 32-frame tape has: full, shorter than the half loaded before
    the sweep (1, 5, 10), longer than it (20, 25, 31), and segments longer than
    the tape, whose later chunks replay a prefix (33, 45, 70)."""
    T, H, W, seed = 70, 8, 64, 22
    res = [_gpu_fwd_bwd(seed, T, H, W, K, in_dtype, torch.float32)[2]
           for K in (1, 5, 20, 31, 32, 33, 45, 70)]
    for r in res[1:]:
        assert torch.equal(r["grad_frames"], res[0]["grad_frames"])
        for a, b in zip(r["grad_state0"], res[0]["grad_state0"]):
            assert torch.equal(a, b)
        assert torch.equal(r["grad_var_init"], res[0]["grad_var_init"])


@pytest.mark.parametrize("opt", [dict(use_gbg=False), dict(use_gst=False)])
def test_f64_adjoint_optional_upstreams(opt):
    T, H, W, seed = 30, 4, 16, 23
    p, out, r, gbg, gst = _gpu_fwd_bwd(seed, T, H, W, 16, torch.float64, torch.float64, **opt)
    ref = _oracle_bwd(seed, T, H, W, torch.float64, torch.float64, p, out["codes"], gbg, gst)
    G.assert_bit_exact("grad_frames", G.flat(r["grad_frames"]), ref["grad_frames"])


def _rel_l2(a, b):
    a, b = np.asarray(a, np.float64).ravel(), np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("in_dtype", [torch.float32, torch.bfloat16])
def test_f32_adjoint_vs_oracle_same_decisions(in_dtype):
    T, H, W, seed = 200, 16, 64, 24
    p, out, r, gbg, gst = _gpu_fwd_bwd(seed, T, H, W, 32, in_dtype, torch.float32)
    ref = _oracle_bwd(seed, T, H, W, in_dtype, torch.float32, p, out["codes"], gbg, gst)
    e = _rel_l2(G.flat(r["grad_frames"]), ref["grad_frames"])
    assert e <= 1e-5, e
    gs = np.stack([g.double().cpu().numpy().ravel() for g in r["grad_state0"]])
    assert _rel_l2(gs, ref["grad_state0"]) <= 1e-5
    assert float(r["grad_var_init"].item()) == pytest.approx(ref["grad_var_init"], rel=1e-5)


def test_f64_adjoint_matches_central_difference_of_gpu_forward():
    """d/dh of <gbg, bg(x + h u)> + <gst, state_T(x + h u)> at h = 0 by central
    differences of the GPU forward (h = 1e-6), against <u, grad> from the GPU
    adjoint.  The map is quadratic between decision changes, so the difference
    quotient is exact up to rounding; pixels whose decisions change under the
    perturbation are left out of the direction."""
    T, H, W, seed, h = 60, 8, 32, 25, 1e-6
    p = dsgm.dsgm_params_default(2.0)
    fr, st = G.device_case(seed, T, H, W)
    gbg, gst = _grads(seed + 100, T, H, W, torch.float64)
    dirx = sdev.fill(torch.empty_like(fr), seed, synth.STREAM_DIRECTION)
    keep = torch.ones((H, W), dtype=torch.float64, device="cuda")

    def objective(frames, want_codes=False):
        s = st.clone()
        o = dsgm.forward(frames, s, p, bg=True, codes=True)
        val = (gbg * o["bg"]).sum(dtype=torch.float64)
        for gi, pl in zip(gst, (s.mean_a, s.var_a, s.mean_c, s.var_c)):
            val = val + (gi * pl).sum(dtype=torch.float64)
        return float(val.item()), o["codes"]

    base, codes0 = objective(fr)
    for _ in range(3):
        u = dirx * keep
        fp, cp = objective(fr + h * u)
        fm, cm = objective(fr - h * u)
        changed = ((cp != codes0) | (cm != codes0)).any(dim=0)
        if not bool(changed.any()):
            break
        keep = keep * (~changed).double()
    assert not bool(changed.any())
    fd = (fp - fm) / (2 * h)
    s = st.clone()
    o = dsgm.forward(fr, s, p, bg=True, ckpt_every=16)
    r = dsgm.backward(fr, p, o["ckpt"], 16, dsgm.ACC_F64, gbg, gst)
    an = float((u * r["grad_frames"]).sum(dtype=torch.float64).item())
    assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (fd, an)
    assert float(keep.mean()) > 0.9


def test_autograd_function_matches_direct_calls():
    T, H, W, seed = 40, 6, 24, 26
    p = dsgm.dsgm_params_default(2.0)
    fr, st = G.device_case(seed, T, H, W)
    fr = fr.clone().requires_grad_(True)
    mA, vA, mC, vC = (t.clone().requires_grad_(True) for t in (st.mean_a, st.var_a, st.mean_c, st.var_c))
    vi = torch.tensor(p.var_init, dtype=torch.float64, device="cuda", requires_grad=True)
    gbg, gst = _grads(seed + 100, T, H, W, torch.float64)
    masks, bg, mAT, vAT, mCT, vCT, aAT, aCT = dsgm.DSGMFunction.apply(
        fr, mA, vA, mC, vC, st.age_a, st.age_c, vi, p, 16)
    loss = (bg * gbg).sum() + sum((g * t).sum() for g, t in zip(gst, (mAT, vAT, mCT, vCT)))
    loss.backward()
    # the same through the C ABI directly
    s = st.clone()
    o = dsgm.forward(fr.detach(), s, p, bg=True, ckpt_every=16)
    r = dsgm.backward(fr.detach(), p, o["ckpt"], 16, dsgm.ACC_F64, gbg, gst)
    assert torch.equal(masks, o["masks"]) and torch.equal(bg.detach(), o["bg"])
    assert torch.equal(fr.grad, r["grad_frames"])
    for leaf, g in zip((mA, vA, mC, vC), r["grad_state0"]):
        assert torch.equal(leaf.grad, g)
    assert float(vi.grad) == float(r["grad_var_init"].item())
    # the inputs were not modified
    assert torch.equal(mA.detach(), st.mean_a)


def test_torch_gradcheck_tiny():
    """torch.autograd.gradcheck on a tiny FP64 instance whose decision margins
    are all far from zero (so +-eps never flips a decision)."""
    T, H, W = 8, 2, 4
    for seed in range(200, 260):
        x, st0 = G.host_case(seed, T, H, W)
        ref = oracle.forward(x, st0, oracle.default_params(2.0), margins=True)
        if np.min(np.abs(ref["margins"])) > 1e-4:
            break
    else:
        pytest.skip("no seed with large margins")
    p = dsgm.dsgm_params_default(2.0)
    fr, st = G.device_case(seed, T, H, W)
    vi = torch.tensor(p.var_init, dtype=torch.float64, device="cuda")

    def f(frames, mA, vA, mC, vC, v):
        out = dsgm.DSGMFunction.apply(frames, mA, vA, mC, vC, st.age_a, st.age_c, v, p, 4)
        return out[1], out[2], out[3], out[4], out[5]

    inputs = tuple(t.clone().requires_grad_(True) for t in (fr, st.mean_a, st.var_a, st.mean_c, st.var_c, vi))
    assert torch.autograd.gradcheck(f, inputs, eps=1e-6, atol=1e-7, rtol=1e-6)


def test_backward_validation_errors():
    T, H, W = 4, 2, 8
    p = dsgm.dsgm_params_default(2.0)
    fr, st = G.device_case(1, T, H, W)
    o = dsgm.forward(fr, st, p, ckpt_every=2)
    gx = torch.empty_like(fr)
    gs0 = tuple(torch.empty((H, W), dtype=torch.float64, device="cuda") for _ in range(4))
    gvi = torch.empty(1, dtype=torch.float64, device="cuda")
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError):
        dsgm.dsgm_backward(fr, p, o["ckpt"], 2, dsgm.ACC_F64, None, None, gx, gs0, gvi, small)
    cs = dsgm._GradState(*(t.data_ptr() for t in gs0))
    nck = o["ckpt"].numel()
    rc = dsgm.lib.dsgm_backward(fr.data_ptr(), 0, dsgm._frames_shape(fr), 0, p, o["ckpt"].data_ptr(), nck,
                                2, None, None, gx.data_ptr(), cs, gvi.data_ptr(), small.data_ptr(), 16, None)
    assert rc == -5  # DSGM_E_WORKSPACE
    rc = dsgm.lib.dsgm_backward(fr.data_ptr(), 0, dsgm._frames_shape(fr), 0, p, None, 0, 2,
                                None, None, gx.data_ptr(), cs, gvi.data_ptr(), small.data_ptr(), 1 << 20, None)
    assert rc == -1  # no checkpoints
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    rc = dsgm.lib.dsgm_backward(fr.data_ptr(), 0, dsgm._frames_shape(fr), 0, p, o["ckpt"].data_ptr(), nck,
                                1, None, None, gx.data_ptr(), cs, gvi.data_ptr(), ws.data_ptr(), 1 << 20, None)
    assert rc == -5  # K = 1 needs more checkpoints than a K = 2 forward wrote


@pytest.mark.slow
def test_full_size_f32_forward_and_adjoint_sampled():
    """1920x2560 pixels x 500 frames, FP32 frames and state, bg on, K = 32,
    upstream gradients N(0,1) (seed 2): the forward the benchmark's adjoint
    leg times (two pixels per lane, bg and checkpoints, no decision codes)
    and dsgm_backward on that forward's own checkpoints.  Sampled pixels are
    certified against the FP64 oracle from the masks alone (identical masks
    until the oracle's first near tie, FP64 margin <= 1e-5); on the pixels
    with no near tie -- where the run provably took the oracle's decisions --
    bg, every checkpoint and the final state agree within 1e-5 and the
    gradients to relative L2 1e-5 of the oracle's reverse mode.  The same
    forward with decision codes gives the same bits."""
    T, H, W, K, seed = 500, 1920, 2560, 32, 2
    p = dsgm.dsgm_params_default(2.0)
    fr, st = G.device_case(seed, T, H, W, torch.float32, torch.float32)
    st_cd = st.clone()
    masks = torch.empty((T, H, W), dtype=torch.uint8, device="cuda")
    bg = torch.empty((T, H, W), dtype=torch.float32, device="cuda")
    ck = torch.empty(dsgm.dsgm_ckpt_bytes(T, H, W, dsgm.ACC_F32, K), dtype=torch.uint8, device="cuda")
    dsgm.dsgm_forward(fr, st, p, masks, bg, ck, K)
    gbg, gst = _grads(seed + 100, T, H, W, torch.float32)
    r = dsgm.backward(fr, p, ck, K, dsgm.ACC_F32, gbg, gst)
    torch.cuda.synchronize()
    rng = np.random.default_rng(2)
    pix = np.unique(np.concatenate([rng.choice(H * W, 2048, replace=False), [0, H * W - 1]]))
    pt = torch.as_tensor(pix, device="cuda")
    x, st0 = G.host_case(seed, T, H, W, torch.float32, torch.float32, pix=pix)
    op = G.oracle_params(p)
    # the oracle chunk by chunk, keeping the state at every checkpoint
    cur, parts, ckref = st0, [], []
    for j in range(0, T, K):
        ckref.append(cur)
        rj = oracle.forward(x[j:j + K], cur, op, margins=True)
        parts.append(rj)
        cur = {k: rj[k] for k in st0}
    ref = {k: np.concatenate([q[k] for q in parts]) for k in ("masks", "bg", "codes", "margins")}
    ref.update(cur)
    clear, differs = G.certify_masks(masks.view(T, -1)[:, pt].cpu().numpy(), ref)
    assert clear.mean() > 0.9 and not differs[clear].any()
    bgs = bg.view(T, -1)[:, pt].double().cpu().numpy()
    assert np.max(np.abs(bgs[:, clear] - ref["bg"][:, clear])) <= 1e-5
    hs = {k: v[pix] for k, v in G.state_to_host(st).items()}
    G.assert_state_close(hs, ref, clear, p.var_init)
    # checkpoints: slot j holds the state before frame j*K
    cb = ck.cpu().numpy()
    px = H * W
    fpl, apl = (px * 4 + 255) // 256 * 256, (px + 255) // 256 * 256
    slot = 4 * fpl + 2 * apl
    for j, want in enumerate(ckref):
        b0 = j * slot
        got = {name: cb[b0 + i * fpl: b0 + i * fpl + px * 4].view(np.float32)[pix].astype(np.float64)
               for i, name in enumerate(("mean_a", "var_a", "mean_c", "var_c"))}
        for i, name in enumerate(("age_a", "age_c")):
            got[name] = cb[b0 + 4 * fpl + i * apl: b0 + 4 * fpl + i * apl + px][pix].astype(np.int32)
        G.assert_state_close(got, want, clear, p.var_init)
    # the adjoint under the oracle's decisions, which the clear pixels took
    gb = gbg.view(T, -1)[:, pt].double().cpu().numpy()
    gs = np.stack([g.view(-1)[pt].double().cpu().numpy() for g in gst])
    rb = oracle.backward(x, st0, op, gb, gs, forced=ref["codes"])
    gx = r["grad_frames"].view(T, -1)[:, pt].double().cpu().numpy()
    assert _rel_l2(gx[:, clear], rb["grad_frames"][:, clear]) <= 1e-5
    g0 = np.stack([g.view(-1)[pt].double().cpu().numpy() for g in r["grad_state0"]])
    assert _rel_l2(g0[:, clear], rb["grad_state0"][:, clear]) <= 1e-5
    gpx = r["workspace"][: H * W * 8].view(torch.float64)[pt].cpu().numpy()
    assert _rel_l2(gpx[clear], rb["grad_var_init_px"][clear]) <= 1e-5
    # the one-pixel-per-lane variant with decision codes: the same bits
    m2, bg2, codes = torch.empty_like(masks), torch.empty_like(bg), torch.empty_like(masks)
    ck2 = torch.empty_like(ck)
    dsgm.dsgm_forward(fr, st_cd, p, m2, bg2, ck2, K, codes)
    torch.cuda.synchronize()
    assert torch.equal(m2, masks) and torch.equal(bg2, bg)
    assert torch.equal(G.ckpt_payload(ck2, T, H, W, K, 4), G.ckpt_payload(ck, T, H, W, K, 4))
    for a_, b_ in zip(st_cd.planes(), st.planes()):
        assert torch.equal(a_, b_)
    del fr, st, st_cd, masks, bg, ck, m2, bg2, ck2, codes, gbg, gst, r


def test_io32_adjoint_is_fp64_rounded_once():
    """FP64 adjoint arithmetic with FP32 gradient arrays: every gradient equals
    the FP64 oracle's (under the same decisions, fed the same FP32 upstream
    values) rounded once to FP32."""
    T, H, W, K, seed = 120, 16, 40, 32, 27
    p = dsgm.dsgm_params_default(2.0)
    fr, st = G.device_case(seed, T, H, W, torch.float32, torch.float64)
    out = dsgm.forward(fr, st, p, bg=True, codes=True, ckpt_every=K, acc=dsgm.ACC_F64_IO32)
    gbg, gst = _grads(seed + 100, T, H, W, torch.float32)
    r = dsgm.backward(fr, p, out["ckpt"], K, dsgm.ACC_F64_IO32, gbg, gst)
    torch.cuda.synchronize()
    ref = _oracle_bwd(seed, T, H, W, torch.float32, torch.float64, p, out["codes"], gbg, gst)
    G.assert_bit_exact("grad_frames", r["grad_frames"].cpu().numpy().reshape(T, -1),
                       ref["grad_frames"].astype(np.float32))
    for i in range(4):
        G.assert_bit_exact(f"grad_state0[{i}]", r["grad_state0"][i].cpu().numpy().ravel(),
                           ref["grad_state0"][i].astype(np.float32))
    px = r["workspace"][: H * W * 8].view(torch.float64).cpu().numpy()
    G.assert_bit_exact("grad_var_init per pixel", px, ref["grad_var_init_px"])


@pytest.mark.slow
def test_full_size_io32_forward_and_adjoint_sampled():
    """The largest single instance: 2160 x 3840 pixels x 1344 frames (11.1 G
    elements), FP32 frames, FP64 state and arithmetic, FP32 bg and gradient
    arrays, checkpoints every 32 frames, upstream gradients N(0,1), seed 4 --
    about 200 GB resident.  Sampled pixels: masks and final state bit-identical
    to the FP64 oracle, bg and gradients equal to its values rounded to FP32."""
    T, H, W, K, seed = 1344, 2160, 3840, 32, 4
    acc = dsgm.ACC_F64_IO32
    p = dsgm.dsgm_params_default(2.0)
    fr, st = G.device_case(seed, T, H, W, torch.float32, torch.float64)
    st0 = st.clone()
    masks = torch.empty((T, H, W), dtype=torch.uint8, device="cuda")
    bg = torch.empty((T, H, W), dtype=torch.float32, device="cuda")
    ck = torch.empty(dsgm.dsgm_ckpt_bytes(T, H, W, acc, K), dtype=torch.uint8, device="cuda")
    dsgm.dsgm_forward(fr, st, p, masks, bg, ck, K, acc=acc)
    gbg, gst = _grads(seed + 100, T, H, W, torch.float32)
    r = dsgm.backward(fr, p, ck, K, acc, gbg, gst)
    torch.cuda.synchronize()
    rng = np.random.default_rng(4)
    pix = np.sort(rng.choice(H * W, 256, replace=False))
    pt = torch.as_tensor(pix, device="cuda")
    x, s0 = G.host_case(seed, T, H, W, torch.float32, torch.float64, pix=pix)
    op = G.oracle_params(p)
    ref = oracle.forward(x, s0, op)
    G.assert_bit_exact("masks", masks.view(T, -1)[:, pt].cpu().numpy(), ref["masks"])
    G.assert_bit_exact("bg", bg.view(T, -1)[:, pt].cpu().numpy(), ref["bg"].astype(np.float32))
    hs = G.state_to_host(st)
    for k in ("mean_a", "var_a", "mean_c", "var_c", "age_a", "age_c"):
        G.assert_bit_exact(k, hs[k][pix], ref[k])
    gb = gbg.view(T, -1)[:, pt].double().cpu().numpy()
    gs = np.stack([g.view(-1)[pt].double().cpu().numpy() for g in gst])
    rb = oracle.backward(x, s0, op, gb, gs, forced=ref["codes"])
    G.assert_bit_exact("grad_frames", r["grad_frames"].view(T, -1)[:, pt].cpu().numpy(),
                       rb["grad_frames"].astype(np.float32))
    for i in range(4):
        G.assert_bit_exact(f"grad_state0[{i}]", r["grad_state0"][i].view(-1)[pt].cpu().numpy(),
                           rb["grad_state0"][i].astype(np.float32))
    del fr, st, st0, masks, bg, ck, gbg, gst, r


@pytest.mark.parametrize("in_dtype,acc_dtype", [(torch.float64, torch.float64),
                                                (torch.bfloat16, torch.float32)])
def test_run_to_run_determinism(in_dtype, acc_dtype):
    """Two runs of the forward and the adjoint on the same inputs give the same
    bits, the two-pass reduction of d/d var_init included (no atomics anywhere
    in a floating-point result)."""
    T, H, W, K, seed = 90, 33, 200, 16, 29
    runs = [_gpu_fwd_bwd(seed, T, H, W, K, in_dtype, acc_dtype) for _ in range(2)]
    (_, o1, r1, _, _), (_, o2, r2, _, _) = runs
    for k in ("masks", "bg", "codes"):
        assert torch.equal(o1[k], o2[k]), k
    eb = 8 if acc_dtype == torch.float64 else 4
    assert torch.equal(G.ckpt_payload(o1["ckpt"], T, H, W, K, eb),
                       G.ckpt_payload(o2["ckpt"], T, H, W, K, eb))
    assert torch.equal(r1["grad_frames"], r2["grad_frames"])
    for a, b in zip(r1["grad_state0"], r2["grad_state0"]):
        assert torch.equal(a, b)
    assert r1["grad_var_init"].cpu().numpy().tobytes() == r2["grad_var_init"].cpu().numpy().tobytes()


def test_pixel_permutation_equivariance():
    """Pixels are independent: mirroring the frames and the state left-right
    mirrors every per-pixel output and gradient, and leaves d/d var_init equal
    up to the summation order of its reduction."""
    T, H, W, K, seed = 50, 20, 72, 16, 30
    p = dsgm.dsgm_params_default(2.0)
    fr, st = G.device_case(seed, T, H, W)
    gbg, gst = _grads(seed + 100, T, H, W, torch.float64)
    flip = lambda t: t.flip(-1).contiguous()
    st_f = dsgm.State(*(flip(t) for t in st.planes()))
    out = dsgm.forward(fr, st, p, bg=True, codes=True, ckpt_every=K)
    out_f = dsgm.forward(flip(fr), st_f, p, bg=True, codes=True, ckpt_every=K)
    r = dsgm.backward(fr, p, out["ckpt"], K, dsgm.ACC_F64, gbg, gst)
    r_f = dsgm.backward(flip(fr), p, out_f["ckpt"], K, dsgm.ACC_F64, flip(gbg),
                        tuple(flip(g) for g in gst))
    torch.cuda.synchronize()
    for k in ("masks", "bg", "codes"):
        assert torch.equal(flip(out[k]), out_f[k]), k
    for a, b in zip(st.planes(), st_f.planes()):
        assert torch.equal(flip(a), b)
    assert torch.equal(flip(r["grad_frames"]), r_f["grad_frames"])
    for a, b in zip(r["grad_state0"], r_f["grad_state0"]):
        assert torch.equal(flip(a), b)
    assert float(r["grad_var_init"].item()) == pytest.approx(float(r_f["grad_var_init"].item()),
                                                            rel=1e-13)
