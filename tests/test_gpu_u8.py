"""GPU parity of the appendix's 8-bit as-run model (DSGM_IN_U8 frames with
DSGM_ACC_U8 state through dsgm_forward) against the 8-bit oracle: integer
work, so masks, codes and the stored state must be identical."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests import gpu_util as G

pytestmark = pytest.mark.gpu

from paper_1702_05156_amd import dsgm


def _case(seed, T, H, W):
    x = (synth.video_levels(seed, T, H, W) + 128).astype(np.uint8).reshape(T, H, W)
    rng = np.random.default_rng(seed)
    st = {k: rng.integers(0, 256, H * W).astype(np.uint8) for k in ("mean_a", "var_a", "mean_c", "var_c")}
    st["age_a"] = rng.integers(1, 31, H * W).astype(np.uint8)
    st["age_c"] = rng.integers(1, 31, H * W).astype(np.uint8)
    return x, st


def _dev_state(st, H, W):
    t = lambda k: torch.as_tensor(st[k].reshape(H, W), device="cuda").contiguous()
    return dsgm.State(t("mean_a"), t("var_a"), t("mean_c"), t("var_c"), t("age_a"), t("age_c"))


def _params(weight_rule, mask_rule):
    p = dsgm.dsgm_params_default(255.0, mask_rule)
    p.weight_rule = weight_rule
    return p


@pytest.mark.parametrize("wr,mr", [(1, 1), (0, 0), (1, 0), (0, 1)])
@pytest.mark.parametrize("T,H,W", [(120, 48, 64), (37, 11, 30)])
def test_u8_forward_bit_exact(wr, mr, T, H, W):
    x, st = _case(71 + wr + 2 * mr, T, H, W)
    p = _params(wr, mr)
    fr = torch.as_tensor(x, device="cuda")
    dst = _dev_state(st, H, W)
    out = dsgm.forward(fr, dst, p, codes=True)
    torch.cuda.synchronize()
    ref = oracle.forward_u8(x.reshape(T, -1), st, G.oracle_params(p))
    G.assert_bit_exact("codes", G.flat(out["codes"]).astype(np.uint8), ref["codes"])
    G.assert_bit_exact("masks", G.flat(out["masks"]).astype(np.uint8), ref["masks"])
    for k in ("mean_a", "var_a", "mean_c", "var_c", "age_a", "age_c"):
        got = getattr(dst, k).cpu().numpy().ravel()
        G.assert_bit_exact(k, got.astype(np.int64), ref[k].astype(np.int64))


def test_u8_streaming_equals_fused_and_no_codes_path():
    T, H, W = 40, 16, 128
    x, st = _case(75, T, H, W)
    p = _params(1, 1)
    fr = torch.as_tensor(x, device="cuda")
    a = _dev_state(st, H, W)
    b = _dev_state(st, H, W)
    m_fused = torch.empty((T, H, W), dtype=torch.uint8, device="cuda")
    dsgm.dsgm_forward(fr, a, p, m_fused)
    m_stream = torch.empty_like(m_fused)
    for t in range(T):
        dsgm.dsgm_forward(fr[t:t + 1], b, p, m_stream[t:t + 1])
    torch.cuda.synchronize()
    assert torch.equal(m_fused, m_stream)
    for u, v in zip(a.planes(), b.planes()):
        assert torch.equal(u, v)


@pytest.mark.parametrize("wr,mr", [(1, 1), (0, 0)])
@pytest.mark.parametrize("H,W", [(16, 128), (9, 30), (5, 37), (1, 1)])
def test_u8_one_frame_steps_against_the_oracle(wr, mr, H, W):
    """One call per frame (the persistent one-frame kernel; widths of 4, 2 and
    1 pixel per lane) with codes: every frame's masks and codes and the final
    stored state equal the 8-bit oracle's."""
    T = 12
    x, st = _case(76, T, H, W)
    p = _params(wr, mr)
    fr = torch.as_tensor(x, device="cuda")
    s = _dev_state(st, H, W)
    m = torch.empty((T, H, W), dtype=torch.uint8, device="cuda")
    c = torch.empty_like(m)
    for t in range(T):
        dsgm.dsgm_forward(fr[t:t + 1], s, p, m[t:t + 1], codes=c[t:t + 1])
    torch.cuda.synchronize()
    ref = oracle.forward_u8(x.reshape(T, -1), st, G.oracle_params(p))
    G.assert_bit_exact("masks", m.cpu().numpy().reshape(T, -1), ref["masks"])
    G.assert_bit_exact("codes", c.cpu().numpy().reshape(T, -1), ref["codes"])
    for k, plane in zip(("mean_a", "var_a", "mean_c", "var_c", "age_a", "age_c"), s.planes()):
        G.assert_bit_exact(k, plane.cpu().numpy().ravel().astype(ref[k].dtype), ref[k])


def test_u8_one_frame_steps_full_size_against_the_oracle():
    """The one-frame kernel as the streaming benchmark runs it (1920 x 2560
    frames, no codes, the appendix's rules), where every lane of the
    persistent grid takes several pixel groups in turn: three calls, and the
    masks of each and the stored state after them equal the 8-bit oracle's."""
    T, H, W = 3, 1920, 2560
    x, st = _case(77, T, H, W)
    p = _params(1, 1)
    fr = torch.as_tensor(x, device="cuda")
    s = _dev_state(st, H, W)
    m = torch.empty((T, H, W), dtype=torch.uint8, device="cuda")
    for t in range(T):
        dsgm.dsgm_forward(fr[t:t + 1], s, p, m[t:t + 1])
    torch.cuda.synchronize()
    ref = oracle.forward_u8(x.reshape(T, -1), st, G.oracle_params(p), codes=False)
    G.assert_bit_exact("masks", m.cpu().numpy().reshape(T, -1), ref["masks"])
    for k, plane in zip(("mean_a", "var_a", "mean_c", "var_c", "age_a", "age_c"), s.planes()):
        G.assert_bit_exact(k, plane.cpu().numpy().ravel().astype(ref[k].dtype), ref[k])


def test_u8_init_from_frame_and_rejections():
    H, W = 5, 9
    p = _params(1, 1)
    p.var_init = 300.5
    f0 = torch.as_tensor((np.arange(H * W) % 256).astype(np.uint8).reshape(H, W), device="cuda")
    st = dsgm.State.empty(H, W, torch.uint8)
    dsgm.dsgm_state_init_from_frame(f0, st, p)
    torch.cuda.synchronize()
    assert torch.equal(st.mean_a, f0) and torch.all(st.var_c == 255)
    assert torch.all(st.age_a == 1)
    fr = f0.unsqueeze(0).repeat(3, 1, 1).contiguous()
    with pytest.raises(dsgm.DSGMError):
        dsgm.dsgm_forward(fr, st, p, torch.empty_like(fr), bg=torch.empty_like(fr))
