"""Pins of the grid-model oracle (Yi et al.'s block model of Sec. 2.2): with
blocks of one pixel it is the per-pixel oracle exactly; on frames that are
constant over each block it is the per-pixel oracle on the block-sampled
frames; the block's mean and V do not depend on the order of its pixels when
sums are exact; partial edge blocks average the pixels they have."""
import numpy as np
import pytest

import oracle
import synth

P = oracle.default_params(2.0)


def _state(seed, n):
    return {k: np.asarray(v) for k, v in synth.state(seed, 1, n, "f64", 30).items()}


def test_block_of_one_is_the_pixel_model():
    T, H, W = 40, 6, 7
    x = synth.frames(1, T, H, W, "f64").reshape(T, H, W)
    st = _state(1, H * W)
    g = oracle.forward_grid(x, st, P, 1)
    r = oracle.forward(x.reshape(T, H * W), st, P)
    assert np.array_equal(g["masks"].reshape(T, -1), r["masks"])
    assert np.array_equal(g["codes"], r["codes"] & 15)
    for k in ("mean_a", "var_a", "mean_c", "var_c", "age_a", "age_c"):
        assert np.array_equal(g[k], r[k]), k


@pytest.mark.parametrize("b,H,W", [(2, 6, 8), (4, 8, 12), (4, 9, 10), (2, 5, 7)])
def test_block_constant_frames_reduce_to_the_pixel_model(b, H, W):
    """Frames constant on every block (8-bit levels, so block sums are exact):
    the block model is the pixel model run on one pixel per block, and every
    pixel of a block gets that pixel's mask."""
    T = 50
    Hb, Wb = -(-H // b), -(-W // b)
    lv = synth.video_levels(2, T, Hb, Wb) / 128.0           # (T, Hb*Wb)
    blocks = lv.reshape(T, Hb, Wb)
    x = np.repeat(np.repeat(blocks, b, axis=1), b, axis=2)[:, :H, :W]
    st = _state(2, Hb * Wb)
    g = oracle.forward_grid(x, st, P, b)
    r = oracle.forward(lv, st, P)
    for k in ("mean_a", "var_a", "mean_c", "var_c", "age_a", "age_c"):
        assert np.array_equal(g[k], r[k]), k
    assert np.array_equal(g["codes"], r["codes"] & 15)
    want = np.repeat(np.repeat(r["masks"].reshape(T, Hb, Wb), b, axis=1), b, axis=2)[:, :H, :W]
    assert np.array_equal(g["masks"], want)


def test_pixel_order_inside_a_block_does_not_matter_with_exact_sums():
    T, H, W, b = 30, 8, 8, 4
    x = synth.video_levels(3, T, H, W).reshape(T, H, W) / 128.0
    st = _state(3, 4)
    g = oracle.forward_grid(x, st, P, b)
    # mirror every 4x4 block left-right and top-bottom: same block sums and maxima
    xm = x.reshape(T, 2, 4, 2, 4)[:, :, ::-1, :, ::-1].reshape(T, H, W)
    gm = oracle.forward_grid(xm, st, P, b)
    for k in ("mean_a", "var_a", "mean_c", "var_c", "age_a", "age_c"):
        assert np.array_equal(g[k], gm[k]), k
    assert np.array_equal(g["codes"], gm["codes"])


def test_block_variance_term_dominates_the_mean_distance():
    """V = max_j (m' - I_j)^2 >= (m' - M)^2: a block with spread reaches a
    larger variance than the same block collapsed to its mean."""
    T, b = 1, 2
    x = np.array([[[0.0, 0.5], [0.25, 0.25]]])
    st = {"mean_a": np.array([0.2]), "var_a": np.array([1.0]), "mean_c": np.array([0.0]),
          "var_c": np.array([1.0]), "age_a": np.array([5]), "age_c": np.array([1])}
    g = oracle.forward_grid(x, st, P, b)
    flat = oracle.forward(np.full((1, 1), 0.25), st, P)
    assert g["codes"][0, 0] & 1 and flat["codes"][0, 0] & 1
    assert g["mean_a"][0] == flat["mean_a"][0]
    assert g["var_a"][0] > flat["var_a"][0]
    w = 1 / 6
    mean = (1 - w) * 0.2 + w * 0.25
    want = (1 - w) * 1.0 + w * max((mean - v) ** 2 for v in (0.0, 0.5, 0.25, 0.25))
    assert g["var_a"][0] == pytest.approx(want, rel=1e-15)


def test_masks_are_per_pixel_against_the_block_model():
    """A block of equal pixels with one outlier: the block model matches and
    stays near the common value, so only the outlier is foreground."""
    T, H, W, b = 1, 4, 4, 4
    x = np.full((T, H, W), 0.25)
    x[0, 2, 1] = 0.9
    st = {"mean_a": np.array([0.25]), "var_a": np.array([0.01]), "mean_c": np.array([-1.0]),
          "var_c": np.array([0.01]), "age_a": np.array([30]), "age_c": np.array([1])}
    g = oracle.forward_grid(x, st, P, b)
    assert g["codes"][0, 0] & 1                  # the block matched A
    fg = g["masks"][0] != 0
    assert fg[2, 1] and fg.sum() == 1
