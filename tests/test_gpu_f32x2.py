"""GPU parity of the compensated single-precision state (DSGM_ACC_F32X2): state
values are (hi, lo) float pairs and every operation is built from error-free
FP32 transformations.  The oracle runs in FP64 on the same inputs (frames on
their storage grid, the initial state as the exact values hi + lo of the
pairs the GPU starts from).  Tolerance contract of the compensated mode:
decisions identical to the oracle's except at certified near ties (FP64
margin <= 1e-12 at the first differing decision), final means and variances
within 1e-12 of the oracle's, bg and gradient arrays (FP32) within half an
FP32 ulp of the oracle's FP64 values (one rounding, up to 1e-12 of slack)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from synth import device as sdev
from tests import gpu_util as G
from tests.test_gpu_forward import _certify_fp32

pytestmark = pytest.mark.gpu

from paper_1702_05156_amd import dsgm

X2 = dsgm.ACC_F32X2
TOL = 1e-12


def _pairs_host(v):
    """The exact value hi + lo of the pair the GPU makes from a float64 value."""
    hi = v.astype(np.float32)
    lo = (v - hi.astype(np.float64)).astype(np.float32)
    return hi.astype(np.float64) + lo.astype(np.float64)


def _case(seed, T, H, W, in_dtype, age_max=30, pix=None):
    fr = sdev.frames(seed, T, H, W, in_dtype)
    mA, vA, mC, vC, aA, aC = sdev.state(seed, H, W, torch.float64, age_max)
    st = dsgm.State(dsgm.x2_from_f64(mA), dsgm.x2_from_f64(vA), dsgm.x2_from_f64(mC),
                    dsgm.x2_from_f64(vC), aA, aC)
    x = synth.frames(seed, T, H, W, G.GRID[in_dtype], pix=pix)
    s0 = synth.state(seed, H, W, "f64", age_max, pix=pix)
    for k in ("mean_a", "var_a", "mean_c", "var_c"):
        s0[k] = _pairs_host(s0[k])
    return fr, st, x, s0


def _host_state(st):
    return {"mean_a": dsgm.x2_to_f64(st.mean_a).cpu().numpy().ravel(),
            "var_a": dsgm.x2_to_f64(st.var_a).cpu().numpy().ravel(),
            "mean_c": dsgm.x2_to_f64(st.mean_c).cpu().numpy().ravel(),
            "var_c": dsgm.x2_to_f64(st.var_c).cpu().numpy().ravel(),
            "age_a": st.age_a.cpu().numpy().ravel().astype(np.int32),
            "age_c": st.age_c.cpu().numpy().ravel().astype(np.int32)}


def _assert_rounded_once(name, got32, ref64, tol=TOL):
    """FP32 values within half an ulp (plus tol) of the FP64 reference: the
    reference rounded once, up to the pair arithmetic's own error."""
    got = np.asarray(got32, dtype=np.float64)
    ref = np.asarray(ref64, dtype=np.float64)
    half_ulp = 0.5 * np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
    err = np.abs(got - ref) - half_ulp
    worst = float(np.max(err, initial=-1.0))
    assert worst <= tol, (name, worst)


def _assert_state(hs, ref, sel, tol=TOL):
    for k in ("mean_a", "var_a", "mean_c", "var_c"):
        d = np.max(np.abs(hs[k][sel] - ref[k][sel]), initial=0.0)
        assert d <= tol, (k, d)
    for k in ("age_a", "age_c"):
        G.assert_bit_exact(k, hs[k][sel], ref[k][sel])


@pytest.mark.parametrize("in_dtype", [torch.float32, torch.bfloat16])
@pytest.mark.parametrize("T,H,W", [(200, 37, 61), (160, 48, 160)])
def test_f32x2_forward_against_oracle(in_dtype, T, H, W):
    """Codes, masks, state and bg against the FP64 oracle; the masks-only
    launch (two pixels per lane where the width allows) gives the codes
    variant's bits."""
    seed = 51
    p = dsgm.dsgm_params_default(2.0)
    fr, st, x, s0 = _case(seed, T, H, W, in_dtype)
    st_m = st.clone()
    out = dsgm.forward(fr, st, p, bg=True, codes=True)
    masks = torch.empty_like(out["masks"])
    dsgm.dsgm_forward(fr, st_m, p, masks)
    torch.cuda.synchronize()
    assert out["bg"].dtype == torch.float32
    ref = oracle.forward(x, s0, G.oracle_params(p), margins=True)
    div = _certify_fp32(G.flat(out["codes"]), ref, tol_margin=TOL)
    assert torch.equal(masks, out["masks"])
    for a, b in zip(st_m.planes(), st.planes()):
        assert torch.equal(a, b)
    ok = ~div
    G.assert_bit_exact("masks", G.flat(out["masks"])[:, ok], ref["masks"][:, ok])
    _assert_state(_host_state(st), ref, ok)
    _assert_rounded_once("bg", G.flat(out["bg"])[:, ok], ref["bg"][:, ok])
    # on these inputs no decision comes within 1e-12 of a tie
    assert div.sum() == 0


@pytest.mark.parametrize("wr,mr", [(1, 0), (0, 1), (1, 1)])
def test_f32x2_other_rules(wr, mr):
    T, H, W, seed = 120, 24, 64, 52
    p = dsgm.dsgm_params_default(2.0, mr)
    p.weight_rule = wr
    fr, st, x, s0 = _case(seed, T, H, W, torch.float32)
    out = dsgm.forward(fr, st, p, bg=True, codes=True)
    torch.cuda.synchronize()
    ref = oracle.forward(x, s0, G.oracle_params(p), margins=True)
    div = _certify_fp32(G.flat(out["codes"]), ref, tol_margin=TOL)
    ok = ~div
    _assert_state(_host_state(st), ref, ok)
    _assert_rounded_once("bg", G.flat(out["bg"])[:, ok], ref["bg"][:, ok])


def test_f32x2_paper_size_and_streaming():
    """320 x 240 x 500 (the paper's sequence size) from a random mid-run state:
    certified against the oracle; one-frame calls give the fused call's bits."""
    T, H, W, seed = 500, 240, 320, 53
    p = dsgm.dsgm_params_default(2.0)
    fr, st, x, s0 = _case(seed, T, H, W, torch.float32)
    st_s = st.clone()
    out = dsgm.forward(fr, st, p, codes=True)
    ms = torch.empty_like(out["masks"])
    for t in range(T):
        dsgm.dsgm_forward(fr[t:t + 1], st_s, p, ms[t:t + 1])
    torch.cuda.synchronize()
    assert torch.equal(ms, out["masks"])
    for a, b in zip(st_s.planes(), st.planes()):
        assert torch.equal(a, b)
    ref = oracle.forward(x, s0, G.oracle_params(p), margins=True)
    div = _certify_fp32(G.flat(out["codes"]), ref, tol_margin=TOL)
    assert div.mean() <= 1e-4
    _assert_state(_host_state(st), ref, ~div)


@pytest.mark.parametrize("K", [7, 32])
@pytest.mark.parametrize("in_dtype", [torch.float32, torch.bfloat16])
def test_f32x2_adjoint_against_oracle(K, in_dtype):
    """The adjoint with the forward's decisions: frame and initial-state
    gradients within half an FP32 ulp of the oracle's FP64 reverse mode,
    d/d var_init (FP64, compensated sum) to 1e-10 relative."""
    T, H, W, seed = 100, 12, 40, 54
    p = dsgm.dsgm_params_default(2.0)
    fr, st, x, s0 = _case(seed, T, H, W, in_dtype)
    out = dsgm.forward(fr, st, p, bg=True, codes=True, ckpt_every=K)
    gbg = sdev.grad_bg(seed + 100, T, H, W, torch.float32)
    gst = tuple(g.contiguous() for g in sdev.grad_state(seed + 100, H, W, torch.float32))
    r = dsgm.backward(fr, p, out["ckpt"], K, X2, gbg, gst)
    torch.cuda.synchronize()
    gs = np.stack([g.double().cpu().numpy().ravel() for g in gst])
    rb = oracle.backward(x, s0, G.oracle_params(p), G.flat(gbg), gs,
                         forced=G.flat(out["codes"]).astype(np.uint8))
    # relative to the gradients' scale: the pair arithmetic's error grows with
    # the magnitude the reverse sweep accumulates
    _assert_rounded_once("grad_frames", G.flat(r["grad_frames"]), rb["grad_frames"], tol=1e-11)
    for i in range(4):
        _assert_rounded_once(f"grad_state0[{i}]", r["grad_state0"][i].cpu().numpy().ravel(),
                             rb["grad_state0"][i], tol=1e-11)
    assert float(r["grad_var_init"].item()) == pytest.approx(rb["grad_var_init"], rel=1e-10)
    # the decisions the adjoint replays are the oracle's (no near tie here)
    ref = oracle.forward(x, s0, G.oracle_params(p))
    G.assert_bit_exact("codes", G.flat(out["codes"]), ref["codes"])


def test_f32x2_state_init_and_rejections():
    T, H, W = 3, 9, 30
    p = dsgm.dsgm_params_default(2.0)
    fr = sdev.frames(55, T, H, W, torch.float32)
    st = dsgm.State.empty(H, W, torch.complex64)
    dsgm.dsgm_state_init_from_frame(fr[0], st, p)
    torch.cuda.synchronize()
    x0 = fr[0].double().cpu().numpy().ravel()
    hs = _host_state(st)
    G.assert_bit_exact("mean_a", hs["mean_a"], x0)
    G.assert_bit_exact("mean_c", hs["mean_c"], x0)
    G.assert_bit_exact("var_a", hs["var_a"], np.full(H * W, _pairs_host(np.array([p.var_init]))[0]))
    assert int(st.age_a.max()) == 1 and int(st.age_c.min()) == 1
    # FP64 frames do not go with the pair state; the extensions do not take it
    with pytest.raises(dsgm.DSGMError, match="DTYPE"):
        dsgm.dsgm_forward(fr.double(), st, p, torch.empty((T, H, W), dtype=torch.uint8,
                                                          device="cuda"))
    with pytest.raises(dsgm.DSGMError, match="DTYPE"):
        dsgm.forward_filtered(fr, st, p, dsgm.gauss_filter(5, 1.0, True))


@pytest.mark.slow
def test_full_size_f32x2_forward_and_adjoint_sampled():
    """1920 x 2560 pixels x 500 frames, FP32 frames, bg and checkpoints every 32
    frames, then the adjoint on those checkpoints (the launches the benchmark
    times for the compensated mode).  256 sampled pixels against the oracle:
    masks identical, state within 1e-12, bg and gradients rounded once."""
    T, H, W, K, seed = 500, 1920, 2560, 32, 56
    p = dsgm.dsgm_params_default(2.0)
    rng = np.random.default_rng(56)
    pix = np.unique(np.concatenate([rng.choice(H * W, 256, replace=False),
                                    [0, W - 1, H * W - W, H * W - 1]]))
    fr, st, x, s0 = _case(seed, T, H, W, torch.float32, pix=pix)
    masks = torch.empty((T, H, W), dtype=torch.uint8, device="cuda")
    bg = torch.empty((T, H, W), dtype=torch.float32, device="cuda")
    ck = torch.empty(dsgm.dsgm_ckpt_bytes(T, H, W, X2, K), dtype=torch.uint8, device="cuda")
    dsgm.dsgm_forward(fr, st, p, masks, bg, ck, K)
    gbg = sdev.grad_bg(seed + 100, T, H, W, torch.float32)
    gst = tuple(g.contiguous() for g in sdev.grad_state(seed + 100, H, W, torch.float32))
    r = dsgm.backward(fr, p, ck, K, X2, gbg, gst)
    torch.cuda.synchronize()
    pt = torch.as_tensor(pix, device="cuda")
    op = G.oracle_params(p)
    ref = oracle.forward(x, s0, op, margins=True)
    clear, differs = G.certify_masks(masks.view(T, -1)[:, pt].cpu().numpy(), ref, tol=TOL)
    assert clear.all() and not differs.any()
    hs = {k: v[pix] for k, v in _host_state(st).items()}
    _assert_state(hs, ref, np.ones(pix.size, bool))
    _assert_rounded_once("bg", bg.view(T, -1)[:, pt].cpu().numpy(), ref["bg"])
    gb = gbg.view(T, -1)[:, pt].double().cpu().numpy()
    gs = np.stack([g.view(-1)[pt].double().cpu().numpy() for g in gst])
    rb = oracle.backward(x, s0, op, gb, gs, forced=ref["codes"])
    _assert_rounded_once("grad_frames", r["grad_frames"].view(T, -1)[:, pt].cpu().numpy(),
                         rb["grad_frames"], tol=1e-11)
    for i in range(4):
        _assert_rounded_once(f"grad_state0[{i}]", r["grad_state0"][i].view(-1)[pt].cpu().numpy(),
                             rb["grad_state0"][i], tol=1e-11)
    del fr, st, masks, bg, ck, gbg, gst, r


def test_f32x2_adjoint_matches_central_difference_of_the_pair_forward():
    """The compensated adjoint against central differences of the compensated
    forward, independently of the oracle: d/dh <gst, state_T(s0 + h u)> for a
    direction u over the four initial float planes, h = 1e-6, against
    <u, grad_state0>.  With the decisions fixed the final state is quadratic
    in the initial one, so the quotient is exact up to rounding (the pairs
    carry about 48 bits); pixels whose decisions change under the
    perturbation are left out of the direction."""
    T, H, W, seed, h = 60, 8, 32, 57, 1e-6
    p = dsgm.dsgm_params_default(2.0)
    fr, st, _, _ = _case(seed, T, H, W, torch.float32)
    gst = tuple(g.contiguous() for g in sdev.grad_state(seed + 100, H, W, torch.float32))
    s0 = [dsgm.x2_to_f64(t) for t in st.planes()[:4]]
    dirs = [sdev.fill(torch.empty((H, W), dtype=torch.float64, device="cuda"), seed + i,
                      synth.STREAM_DIRECTION) for i in range(4)]
    keep = torch.ones((H, W), dtype=torch.float64, device="cuda")

    def objective(step):
        planes = [dsgm.x2_from_f64(s0[i] + step * dirs[i] * keep) for i in range(4)]
        s = dsgm.State(*planes, st.age_a.clone(), st.age_c.clone())
        o = dsgm.forward(fr, s, p, codes=True)
        val = sum((g.double() * dsgm.x2_to_f64(pl)).sum(dtype=torch.float64)
                  for g, pl in zip(gst, (s.mean_a, s.var_a, s.mean_c, s.var_c)))
        return float(val.item()), o["codes"]

    _, codes0 = objective(0.0)
    for _ in range(3):
        fp, cp = objective(h)
        fm, cm = objective(-h)
        changed = ((cp != codes0) | (cm != codes0)).any(dim=0)
        if not bool(changed.any()):
            break
        keep = keep * (~changed).double()
    assert not bool(changed.any())
    fd = (fp - fm) / (2 * h)
    s = st.clone()
    o = dsgm.forward(fr, s, p, ckpt_every=16)
    r = dsgm.backward(fr, p, o["ckpt"], 16, X2, None, gst)
    an = sum(float((dirs[i] * keep * r["grad_state0"][i].double()).sum(dtype=torch.float64).item())
             for i in range(4))
    assert abs(fd - an) <= 1e-5 * max(1.0, abs(an)), (fd, an)
    assert float(keep.mean()) > 0.9
