"""Pins of the motion-compensation oracle (the model warped by the camera
homography before the update; Sec. 2.2 and 2.4): identities, exact integer
shifts, bilinear reproduction of linear fields, an independent library
implementation (scipy.ndimage.map_coordinates) and the uncovered-pixel rule."""
import numpy as np
import pytest

import oracle
import synth

from scipy import ndimage

P = oracle.default_params(2.0)


def _state(seed, H, W):
    return synth.state(seed, H, W, "f64", 30)


def _frame(seed, H, W):
    return synth.uniform(seed, 0, np.arange(H * W), "f64")


def test_identity_copies_exactly():
    H, W = 9, 13
    st = _state(1, H, W)
    out = oracle.warp_state(st, _frame(1, H, W), np.eye(3), P, H, W)
    for k in st:
        assert np.array_equal(out[k], np.asarray(st[k]).astype(out[k].dtype)), k


@pytest.mark.parametrize("dx,dy", [(2, 0), (0, -3), (-1, 2), (4, 5)])
def test_integer_shift_is_exact_and_resets_the_uncovered_band(dx, dy):
    """map: current (c, y) <- previous (c - dx, y - dy): the scene moved by (dx, dy)."""
    H, W = 10, 12
    st = _state(2, H, W)
    fr = _frame(2, H, W)
    m = np.array([[1, 0, -dx], [0, 1, -dy], [0, 0, 1]], dtype=float)
    out = oracle.warp_state(st, fr, m, P, H, W)
    for y in range(H):
        for c in range(W):
            i = y * W + c
            sy, sc = y - dy, c - dx
            if 0 <= sy < H and 0 <= sc < W:
                j = sy * W + sc
                for k in st:
                    assert out[k][i] == st[k][j], (k, y, c)
            else:
                assert out["mean_a"][i] == fr[i] and out["mean_c"][i] == fr[i]
                assert out["var_a"][i] == P.var_init and out["age_a"][i] == 1
                assert out["age_c"][i] == 1


def test_bilinear_reproduces_a_linear_field():
    """Bilinear interpolation is exact on f = a*x + b*y + c (up to rounding)."""
    H, W = 16, 20
    yy, xx = np.mgrid[0:H, 0:W]
    f = (0.25 * xx - 0.125 * yy + 0.5).ravel()
    st = {"mean_a": f, "var_a": f + 2, "mean_c": -f, "var_c": f + 3,
          "age_a": np.ones(H * W, np.int32), "age_c": np.ones(H * W, np.int32)}
    th = 0.1
    m = np.array([[np.cos(th), -np.sin(th), 1.3], [np.sin(th), np.cos(th), -0.7], [0, 0, 1.0]])
    out = oracle.warp_state(st, np.zeros(H * W), m, P, H, W)
    qx = m[0, 0] * xx + m[0, 1] * yy + m[0, 2]
    qy = m[1, 0] * xx + m[1, 1] * yy + m[1, 2]
    cov = ((qx >= 0) & (qx <= W - 1) & (qy >= 0) & (qy <= H - 1)).ravel()
    assert cov.sum() > H * W // 2
    want = (0.25 * qx - 0.125 * qy + 0.5).ravel()
    assert np.max(np.abs(out["mean_a"][cov] - want[cov])) <= 1e-13
    assert np.max(np.abs(out["mean_c"][cov] + want[cov])) <= 1e-13


def test_matches_scipy_map_coordinates():
    H, W = 24, 31
    st = _state(3, H, W)
    rng = np.random.default_rng(3)
    m = np.array([[1.02, 0.03, -1.1], [-0.02, 0.98, 0.6], [1e-4, -2e-4, 1.0]])
    out = oracle.warp_state(st, _frame(3, H, W), m, P, H, W)
    yy, xx = np.mgrid[0:H, 0:W]
    den = m[2, 0] * xx + m[2, 1] * yy + m[2, 2]
    qx = (m[0, 0] * xx + m[0, 1] * yy + m[0, 2]) / den
    qy = (m[1, 0] * xx + m[1, 1] * yy + m[1, 2]) / den
    cov = ((qx >= 0) & (qx <= W - 1) & (qy >= 0) & (qy <= H - 1)).ravel()
    for k in ("mean_a", "var_a", "mean_c", "var_c"):
        ref = ndimage.map_coordinates(np.asarray(st[k]).reshape(H, W), [qy, qx], order=1,
                                      mode="nearest").ravel()
        assert np.max(np.abs(out[k][cov] - ref[cov])) <= 1e-14, k
    # nearest ages, away from half-way ties
    frac_ok = ((np.abs(qx - np.floor(qx) - 0.5) > 1e-6) & (np.abs(qy - np.floor(qy) - 0.5) > 1e-6)).ravel()
    sel = cov & frac_ok
    for k in ("age_a", "age_c"):
        ref = ndimage.map_coordinates(np.asarray(st[k]).reshape(H, W).astype(float), [qy, qx],
                                      order=0, mode="nearest").ravel()
        assert np.array_equal(out[k][sel], ref[sel].astype(np.int32)), k
    assert (~cov).sum() > 0   # some pixels uncovered, restarted
    assert np.all(out["age_a"][~cov] == 1)


def test_points_behind_the_camera_are_uncovered():
    H, W = 4, 5
    st = _state(4, H, W)
    fr = _frame(4, H, W)
    m = np.array([[1, 0, 0], [0, 1, 0], [0, 0, -1.0]])   # den < 0 everywhere
    out = oracle.warp_state(st, fr, m, P, H, W)
    assert np.array_equal(out["mean_a"], fr) and np.all(out["var_c"] == P.var_init)
