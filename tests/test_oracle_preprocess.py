"""Pins of the preprocessing oracle (Gaussian blur, then 3 x 3 median; Sec.
2.1 and the CUDA preprocessing of Sec. 3.3.1) against what the mathematics
fixes: closed forms of the weights, the exact impulse response of a separable
filter, the 2-D definition of the blur, an independent library implementation
(scipy.ndimage), and the median by brute force."""
import numpy as np
import pytest

import oracle

from scipy import ndimage as scipy_ndimage


@pytest.mark.parametrize("n,sigma", [(3, 0.8), (5, 1.0), (7, 1.5), (9, 2.0)])
def test_weights_closed_forms(n, sigma):
    w = oracle.gauss_weights(n, sigma)
    r = (n - 1) // 2
    assert np.array_equal(w, w[::-1])                       # symmetric, exactly
    assert abs(w.sum() - 1.0) <= 4 * n * np.finfo(float).eps
    # ratio of neighbouring samples of the density: exp(-(2d+1) / (2 sigma^2))
    for d in range(r):
        want = np.exp(-(2 * d + 1) / (2 * sigma * sigma))
        assert w[r + d + 1] / w[r + d] == pytest.approx(want, rel=1e-14)
    assert np.argmax(w) == r


def test_weights_reject_bad_arguments():
    for n, s in [(4, 1.0), (0, 1.0), (5, 0.0), (5, -1.0), (33, 1.0)]:
        with pytest.raises(ValueError):
            oracle.gauss_weights(n, s)


def test_impulse_response_is_the_outer_product():
    n, sigma = 5, 1.0
    w = oracle.gauss_weights(n, sigma)
    H, W, y0, x0 = 11, 13, 5, 6
    img = np.zeros((1, H, W))
    img[0, y0, x0] = 1.0
    out = oracle.preprocess(img, w, median=False)[0]
    want = np.zeros((H, W))
    for a in range(-2, 3):
        for b in range(-2, 3):
            want[y0 + a, x0 + b] = w[2 + a] * w[2 + b]
    assert np.array_equal(out, want)


@pytest.mark.parametrize("n,sigma", [(5, 1.0), (7, 1.3)])
def test_blur_matches_2d_definition_and_scipy(n, sigma):
    rng = np.random.default_rng(3)
    x = rng.uniform(-1, 1, size=(3, 17, 23))
    w = oracle.gauss_weights(n, sigma)
    got = oracle.preprocess(x, w, median=False)
    r = (n - 1) // 2
    k2 = np.outer(w, w)
    for t in range(x.shape[0]):
        p = np.pad(x[t], r, mode="edge")      # clamp-to-edge borders
        ref = np.zeros_like(x[t])
        for i in range(n):
            for j in range(n):
                ref += k2[i, j] * p[i:i + x.shape[1], j:j + x.shape[2]]
        assert np.max(np.abs(got[t] - ref)) <= 1e-15
        sc = scipy_ndimage.correlate1d(x[t], w, axis=1, mode="nearest")
        sc = scipy_ndimage.correlate1d(sc, w, axis=0, mode="nearest")
        assert np.max(np.abs(got[t] - sc)) <= 1e-15


def test_median_brute_force():
    rng = np.random.default_rng(4)
    x = rng.integers(-5, 6, size=(2, 9, 12)).astype(np.float64) / 8   # many ties
    got = oracle.preprocess(x, None, median=True)
    for t in range(2):
        p = np.pad(x[t], 1, mode="edge")
        win = np.stack([p[dy:dy + 9, dx:dx + 12] for dy in range(3) for dx in range(3)])
        assert np.array_equal(got[t], np.median(win, axis=0))


def test_blur_then_median_order():
    rng = np.random.default_rng(5)
    x = rng.uniform(-1, 1, size=(2, 10, 14))
    w = oracle.gauss_weights(5, 1.0)
    both = oracle.preprocess(x, w, median=True)
    blurred = oracle.preprocess(x, w, median=False)
    assert np.array_equal(both, oracle.preprocess(blurred, None, median=True))
    assert not np.array_equal(both, oracle.preprocess(oracle.preprocess(x, None, median=True), w,
                                                      median=False))


def test_constant_and_identity():
    c = np.full((2, 6, 7), 0.375)
    w = oracle.gauss_weights(7, 1.2)
    out = oracle.preprocess(c, w, median=True)
    assert np.max(np.abs(out - 0.375)) <= 16 * np.finfo(float).eps
    rng = np.random.default_rng(6)
    x = rng.uniform(-1, 1, size=(3, 5, 8))
    assert np.array_equal(oracle.preprocess(x, None, median=False), x)


def test_single_pixel_and_thin_frames():
    w = oracle.gauss_weights(5, 1.0)
    x = np.array([[[0.25]], [[-0.5]]])
    out = oracle.preprocess(x, w, median=True)
    assert np.allclose(out, x, rtol=0, atol=1e-15)
    rng = np.random.default_rng(7)
    row = rng.uniform(-1, 1, size=(1, 1, 9))
    out = oracle.preprocess(row, w, median=False)
    # one row: the column pass sees the same row five times
    ref = scipy_ndimage.correlate1d(row[0], w, axis=1, mode="nearest")
    assert np.max(np.abs(out[0] - ref)) <= 1e-15


# ------------------------------------------------ the appendix's 8-bit pipeline
def _exact_blur_u8(x, w):
    """The 2-D blur of one uint8 frame in exact rational arithmetic with the
    single-precision window weights float(w_i * w_j) (exact binary fractions),
    borders clamped to the last row and column: the real value the
    single-precision sum approximates."""
    from fractions import Fraction
    n = w.size
    r = (n - 1) // 2
    H, W = x.shape
    w2 = [[Fraction(float(np.float32(w[i] * w[j]))) for j in range(n)] for i in range(n)]
    out = np.empty((H, W), dtype=object)
    for y in range(H):
        for c in range(W):
            acc = Fraction(0)
            for i in range(n):
                for j in range(n):
                    yy = min(max(y + i - r, 0), H - 1)
                    xx = min(max(c + j - r, 0), W - 1)
                    acc += int(x[yy, xx]) * w2[i][j]
            out[y, c] = acc
    return out


@pytest.mark.parametrize("n,sigma,seed", [(3, 0.8, 1), (5, 1.0, 2), (7, 1.5, 3)])
def test_u8_blur_is_the_truncated_exact_sum(n, sigma, seed):
    """Each 8-bit blurred value is the integer part of the exact 2-D weighted
    sum, except where that sum lies within the single-precision rounding of
    25-49 terms of an integer (there it may be one less or one more)."""
    w = oracle.gauss_weights(n, sigma)
    rng = np.random.default_rng(seed)
    x = rng.integers(0, 256, size=(1, 9, 11), dtype=np.uint8)
    got = oracle.preprocess_u8(x, w, median=False)[0].astype(int)
    ex = _exact_blur_u8(x[0], w)
    near = 0
    for y in range(x.shape[1]):
        for c in range(x.shape[2]):
            e = ex[y, c]
            fl = e.numerator // e.denominator
            if abs(float(e - round(e))) < 1e-3:   # float rounding may cross the integer
                near += 1
                assert abs(got[y, c] - float(e)) < 1.0
            else:
                assert got[y, c] == fl, (y, c, float(e))
    assert near < x.size // 4


def test_u8_impulse_response_drops_the_fraction():
    """A single bright pixel: each blurred value is the integer part of
    255 * float(w_i * w_j) at the mirrored offset (not its rounded value)."""
    w = oracle.gauss_weights(5, 1.0)
    x = np.zeros((1, 11, 13), dtype=np.uint8)
    x[0, 5, 6] = 255
    got = oracle.preprocess_u8(x, w, median=False)[0]
    want = np.zeros((11, 13), dtype=np.uint8)
    for i in range(5):
        for j in range(5):
            v = 255.0 * float(np.float32(w[i] * w[j]))
            want[5 + 2 - i, 6 + 2 - j] = int(np.floor(v))
    assert np.array_equal(got, want)
    # the rounding rule matters here: some products have a fraction >= 1/2
    fr = [255.0 * float(np.float32(w[i] * w[j])) % 1 for i in range(5) for j in range(5)]
    assert max(fr) >= 0.5


def test_u8_median_brute_force_and_identity():
    """Without a blur the 8-bit pipeline is the 3 x 3 median of the frame,
    checked against numpy's median of each clamped neighbourhood; without
    either it is the identity."""
    rng = np.random.default_rng(7)
    x = rng.integers(0, 256, size=(2, 7, 9), dtype=np.uint8)
    got = oracle.preprocess_u8(x, None, median=True)
    for t in range(2):
        for y in range(7):
            for c in range(9):
                nb = [x[t, min(max(y + dy, 0), 6), min(max(c + dx, 0), 8)]
                      for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
                assert got[t, y, c] == int(np.median(nb))
    assert np.array_equal(oracle.preprocess_u8(x, None, median=False), x)


def test_u8_blur_then_median_and_constant_frames():
    """The median runs on the blurred 8-bit image; a constant frame c blurs to
    c or c - 1 (the single-precision weights sum to 1 within a few ulp) and
    stays constant."""
    w = oracle.gauss_weights(5, 1.0)
    rng = np.random.default_rng(8)
    x = rng.integers(0, 256, size=(1, 8, 10), dtype=np.uint8)
    b = oracle.preprocess_u8(x, w, median=False)
    assert np.array_equal(oracle.preprocess_u8(x, w, median=True),
                          oracle.preprocess_u8(b, None, median=True))
    for c in (0, 1, 17, 128, 254, 255):
        out = oracle.preprocess_u8(np.full((1, 6, 7), c, np.uint8), w, median=True)
        assert out.min() == out.max() and out[0, 0, 0] in (c, max(c - 1, 0))
