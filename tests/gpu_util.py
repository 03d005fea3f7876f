"""Helpers shared by the GPU parity tests (not collected by pytest)."""
from __future__ import annotations

import numpy as np
import torch

import oracle
import synth
from synth import device as sdev

GRID = {torch.float64: "f64", torch.float32: "f32", torch.bfloat16: "bf16"}
ACC_NAME = {torch.float64: "f64", torch.float32: "f32"}


def oracle_params(p) -> "oracle.Params":
    return oracle.Params(theta_s=p.theta_s, theta_d=p.theta_d, var_init=p.var_init,
                         var_floor=p.var_floor, mask_floor=p.mask_floor, age_max=p.age_max,
                         weight_rule=p.weight_rule, mask_rule=p.mask_rule)


def device_case(seed, T, H, W, in_dtype=torch.float64, acc_dtype=torch.float64, age_max=30):
    """Frames and a random mid-run state on the device (from the device generator)."""
    from paper_1702_05156_amd.dsgm import State
    fr = sdev.frames(seed, T, H, W, in_dtype)
    st = State(*sdev.state(seed, H, W, acc_dtype, age_max))
    return fr, st


def host_case(seed, T, H, W, in_dtype=torch.float64, acc_dtype=torch.float64, age_max=30,
              pix=None, t=None):
    """The same inputs from the host generator, as float64 numpy arrays
    (frames: (len(t), len(pix))), for the oracle."""
    x = synth.frames(seed, T, H, W, GRID[in_dtype], t=t, pix=pix)
    st = synth.state(seed, H, W, ACC_NAME[acc_dtype], age_max, pix=pix)
    return x, st


def state_to_host(st) -> dict:
    return {"mean_a": st.mean_a.double().cpu().numpy().ravel(),
            "var_a": st.var_a.double().cpu().numpy().ravel(),
            "mean_c": st.mean_c.double().cpu().numpy().ravel(),
            "var_c": st.var_c.double().cpu().numpy().ravel(),
            "age_a": st.age_a.cpu().numpy().ravel().astype(np.int32),
            "age_c": st.age_c.cpu().numpy().ravel().astype(np.int32)}


def flat(t: torch.Tensor) -> np.ndarray:
    """(T, H, W) device tensor -> (T, H*W) numpy (float64 for floats)."""
    a = t.detach()
    if a.is_floating_point():
        a = a.double()
    a = a.cpu().numpy()
    return a.reshape(a.shape[0], -1)


def assert_bit_exact(name, got, want):
    got = np.asarray(got)
    want = np.asarray(want)
    assert got.shape == want.shape, (name, got.shape, want.shape)
    bad = got != want
    if np.any(bad):
        idx = np.argwhere(bad)[:5]
        raise AssertionError(f"{name}: {int(bad.sum())} of {bad.size} differ; first at "
                             f"{idx.tolist()}: got {got[bad][:5]} want {want[bad][:5]}")


def ckpt_payload(ck: torch.Tensor, T, H, W, K, elt_bytes) -> torch.Tensor:
    """The defined bytes of a checkpoint buffer: per slot (the state before
    frames 0, K, 2K, ...) four float planes of elt_bytes * H*W bytes and two
    age planes of H*W bytes, each plane starting on a 256-byte boundary.  The
    padding between planes is never written, so whole buffers are not
    comparable."""
    px = H * W
    fpl = (px * elt_bytes + 255) // 256 * 256
    apl = (px + 255) // 256 * 256
    slot = 4 * fpl + 2 * apl
    parts = []
    for j in range((T + K - 1) // K):
        b = j * slot
        parts += [ck[b + i * fpl: b + i * fpl + px * elt_bytes] for i in range(4)]
        parts += [ck[b + 4 * fpl + i * apl: b + 4 * fpl + i * apl + px] for i in range(2)]
    return torch.cat(parts)


def first_near_tie(ref, tol=1e-5) -> np.ndarray:
    """Per pixel, the first frame at which the oracle takes a decision whose
    FP64 margin (squared distance minus threshold) is within `tol` of zero:
    the A test on every frame, the C test on frames where A did not match,
    the background test on every frame.  T where there is none."""
    m, c = ref["margins"], ref["codes"]
    T = c.shape[0]
    a_missed = (c & oracle.HIT_A) == 0
    near = ((np.abs(m[..., 0]) <= tol) | (a_missed & (np.abs(m[..., 1]) <= tol)) |
            (np.abs(m[..., 2]) <= tol))
    return np.where(near.any(axis=0), near.argmax(axis=0), T)


def certify_masks(masks_gpu, ref, tol=1e-5):
    """Certification of a reduced-precision run from its masks alone (no
    decision codes, so the launch under test is the one without them).  The
    FP32 state error is far below `tol`, so the run must take the oracle's
    decisions until the oracle's first near tie of a pixel: masks identical
    before that frame, and identical throughout on pixels with no near tie.
    Returns (clear, mask_differs): pixels with no near tie, and pixels
    whose masks differ somewhere."""
    masks_gpu = np.asarray(masks_gpu)
    T = masks_gpu.shape[0]
    first = first_near_tie(ref, tol)
    diff = masks_gpu != ref["masks"]
    early = diff & (np.arange(T)[:, None] < first[None, :])
    if early.any():
        t, j = np.argwhere(early)[0]
        raise AssertionError(f"mask differs at frame {t}, sample pixel {j}, before its first "
                             f"near tie (frame {first[j]}): margins {ref['margins'][t, j]}")
    return first == T, diff.any(axis=0)


def assert_state_close(hs, ref, sel, var_init, tol=1e-5):
    """Final model state of the reduced-precision run on the pixels `sel`:
    means within tol, variances within tol * max(v, var_init), ages equal."""
    for k in ("mean_a", "mean_c"):
        assert np.max(np.abs(hs[k][sel] - ref[k][sel]), initial=0.0) <= tol, k
    for k in ("var_a", "var_c"):
        d = np.abs(hs[k][sel] - ref[k][sel]) / np.maximum(ref[k][sel], var_init)
        assert np.max(d, initial=0.0) <= tol, k
    for k in ("age_a", "age_c"):
        assert_bit_exact(k, hs[k][sel], ref[k][sel])
