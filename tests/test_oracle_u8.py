"""Pins of the 8-bit as-run oracle (the appendix keeps means and variances in
8-bit images, so every write drops the fraction): frame by frame it is the
real-valued oracle's step from the same integer state followed by that
storage rule; its masks equal the real-valued step's wherever the stored
apparent model did not need rounding."""
import numpy as np
import pytest

import oracle
import synth


def _u8(v):
    return np.clip(np.trunc(v), 0, 255)


def _setup(seed, T, N):
    x = (synth.video_levels(seed, T, 1, N) + 128).astype(np.uint8)   # 0..255 levels
    rng = np.random.default_rng(seed)
    st = {"mean_a": rng.integers(0, 256, N), "var_a": rng.integers(0, 256, N),
          "mean_c": rng.integers(0, 256, N), "var_c": rng.integers(0, 256, N),
          "age_a": rng.integers(1, 31, N), "age_c": rng.integers(1, 31, N)}
    return x, st


@pytest.mark.parametrize("rule,mrule,var_init", [(1, 1, None), (0, 0, None), (1, 0, None),
                                                  (1, 1, 100.5), (0, 1, 101.9)])
def test_each_frame_is_the_real_step_then_the_storage_rule(rule, mrule, var_init):
    """Per-frame calls (state stored between frames) equal one call over all
    frames; a fractional var_init exercises the storage of reset and swapped
    candidates within a call."""
    T, N = 60, 500
    x, st = _setup(1, T, N)
    p = oracle.default_params(255.0, mask_rule=mrule)
    p.weight_rule = rule
    if var_init is not None:
        p.var_init = var_init
    full = oracle.forward_u8(x, st, p)
    cur = {k: np.asarray(v) for k, v in st.items()}
    for t in range(T):
        real = oracle.forward(x[t:t + 1].astype(np.float64), {k: v.astype(np.float64) if "age" not in k else v
                                                               for k, v in cur.items()}, p)
        step = oracle.forward_u8(x[t:t + 1], cur, p)
        assert np.array_equal(step["codes"][0] & 15, real["codes"][0] & 15)
        for k in ("mean_a", "var_a", "mean_c", "var_c"):
            assert np.array_equal(step[k], _u8(real[k]).astype(np.uint8)), (t, k)
        for k in ("age_a", "age_c"):
            assert np.array_equal(step[k], real[k]), (t, k)
        # where the stored apparent model is the real one, the masks agree
        same = real["mean_a"] == step["mean_a"]
        if mrule == 0:
            same &= real["var_a"] == step["var_a"]
        assert np.array_equal(step["masks"][0][same], real["masks"][0][same])
        assert np.array_equal(step["masks"][0], full["masks"][t])
        cur = {k: step[k] for k in ("mean_a", "var_a", "mean_c", "var_c", "age_a", "age_c")}
    for k in cur:
        assert np.array_equal(cur[k], full[k]), k


def test_storage_rule_saturates_and_truncates():
    """A variance blend above 255 is stored as 255; fractions are dropped."""
    p = oracle.default_params(255.0, mask_rule=1)
    p.weight_rule = 1
    st = {"mean_a": [100], "var_a": [250], "mean_c": [0], "var_c": [0], "age_a": [2],
          "age_c": [1]}
    # |x - 100|^2 = 400 < 2*250: A matches with alpha = 1/2
    out = oracle.forward_u8(np.array([[120]], np.uint8), st, p)
    assert out["codes"][0, 0] & 1
    assert out["mean_a"][0] == 110                       # (100 + 120) / 2
    assert out["var_a"][0] == 175                        # (250 + 100) / 2
    out = oracle.forward_u8(np.array([[115]], np.uint8), st, p)
    assert out["codes"][0, 0] & 1
    assert out["mean_a"][0] == 107                       # 107.5 truncated
    assert out["var_a"][0] == 153                        # 125 + 56.25 / 2 = 153.125
    # a reset candidate takes var_init, stored through the same rule
    p.var_init = 300.7
    out = oracle.forward_u8(np.array([[10]], np.uint8), dict(st, var_a=[0], mean_c=[200]), p)
    assert out["codes"][0, 0] & 4 and out["var_c"][0] == 255 and out["mean_c"][0] == 10
    p.var_init = 17.9
    out = oracle.forward_u8(np.array([[10]], np.uint8), dict(st, var_a=[0], mean_c=[200]), p)
    assert out["var_c"][0] == 17


def test_swapped_in_candidate_is_stored_before_it_is_used():
    """Frame 0 swaps (C older than A) and resets C to (x, var_init); frame 1 fails
    A and matches C, whose stored variance is trunc(var_init): 101.9 -> 101.
    One call over both frames equals two one-frame calls (state stored between
    them), and the hand result: mean (100 + 111) / 2 = 105.5 -> 105, variance
    101 / 2 + (105.5 - 111)^2 / 2 = 65.625 -> 65."""
    p = oracle.default_params(255.0, mask_rule=1)
    p.weight_rule = 0
    p.var_init = 101.9
    st = {"mean_a": [10], "var_a": [1], "mean_c": [100], "var_c": [1], "age_a": [1],
          "age_c": [5]}
    x = np.array([[100], [111]], np.uint8)
    both = oracle.forward_u8(x, st, p)
    one = oracle.forward_u8(x[:1], st, p)
    assert one["codes"][0, 0] & 8 and one["var_c"][0] == 101
    two = oracle.forward_u8(x[1:], {k: one[k] for k in st}, p)
    assert two["codes"][0, 0] & 2
    assert two["mean_c"][0] == 105 and two["var_c"][0] == 65
    for k in st:
        assert np.array_equal(both[k], two[k]), k
