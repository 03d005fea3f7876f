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


@pytest.mark.parametrize("rule,mrule", [(1, 1), (0, 0), (1, 0)])
def test_each_frame_is_the_real_step_then_the_storage_rule(rule, mrule):
    T, N = 60, 500
    x, st = _setup(1, T, N)
    p = oracle.default_params(255.0, mask_rule=mrule)
    p.weight_rule = rule
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
