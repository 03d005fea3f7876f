"""The seeded input generator (host side): known answers and value maps."""
import numpy as np

import synth


def test_splitmix64_known_answers():
    # SplitMix64 seeded with 0: the first outputs of the published generator
    # (mix(k * gamma) for k = 1, 2, ...), as listed for Vigna's splitmix64.c.
    expected = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F,
                0xF88BB8A8724C81EC, 0x1B39896A51A8749B]
    k = np.arange(1, 6, dtype=np.uint64)
    with np.errstate(over="ignore"):
        got = synth.mix64(k * synth.GAMMA)
    assert [int(v) for v in got] == expected


def test_draws_are_counter_based():
    a = synth.draws(7, 3, np.arange(100))
    b = synth.draws(7, 3, np.arange(50, 150))
    assert np.array_equal(a[50:], b[:50])
    assert not np.array_equal(synth.draws(7, 4, np.arange(100)), a)
    assert not np.array_equal(synth.draws(8, 3, np.arange(100)), a)


def test_uniform_grids_exact():
    idx = np.arange(200000)
    for dt, bits in (("f64", 52), ("f32", 23), ("bf16", 7)):
        u = synth.uniform(1, 0, idx, dt)
        assert u.min() >= -1.0 and u.max() < 1.0
        n = (u + 1.0) * 2.0 ** bits
        assert np.array_equal(n, np.round(n)), dt
        assert abs(u.mean()) < 0.01 and abs(u.var() - 1.0 / 3.0) < 0.01
    u32 = synth.uniform(1, 0, idx, "f32")
    assert np.array_equal(u32.astype(np.float32).astype(np.float64), u32)


def test_ages_uniform():
    a = synth.ages(5, synth.STREAM_AGE_A, np.arange(300000), 30)
    assert a.min() == 1 and a.max() == 30
    counts = np.bincount(a, minlength=31)[1:]
    assert counts.min() > 0.9 * 10000 and counts.max() < 1.1 * 10000


def test_normal_moments_and_exactness():
    g = synth.normal(2, synth.STREAM_GRAD_BG, np.arange(200000))
    assert abs(g.mean()) < 0.01 and abs(g.var() - 1.0) < 0.02
    assert np.array_equal(g.astype(np.float32).astype(np.float64), g)


def test_logical_index_layout():
    T, H, W = 3, 4, 5
    full = synth.frames(0, T, H, W, "f64")
    part = synth.frames(0, T, H, W, "f64", t=[2], pix=[7, 19])
    assert full.shape == (T, H * W)
    assert np.array_equal(part[0], full[2, [7, 19]])


def test_video_levels_and_slices():
    """The structured video: 8-bit levels, consistent when evaluated on a
    subset of frames and pixels, noise centred with ~3 levels of spread."""
    T, H, W = 20, 16, 24
    q = synth.video_levels(4, T, H, W)
    assert q.min() >= -128 and q.max() <= 127
    assert np.array_equal(synth.video(4, T, H, W), q / 128.0)
    t = np.array([0, 7, 19])
    pix = np.array([0, 5, 100, H * W - 1])
    assert np.array_equal(synth.video_levels(4, T, H, W, t=t, pix=pix), q[t][:, pix])
    s = synth.irwin_hall_sum(4, synth.STREAM_VIDEO_NOISE, np.arange(200000))
    n = ((s - 393210) * 3 + 32768) >> 16
    assert abs(n.mean()) < 0.05 and 2.9 < n.std() < 3.1
    r = synth.video_rects(4, H, W)
    assert r.shape == (synth.VIDEO_RECTS, 7)
    assert np.all((r[:, 2] >= H // 16) & (r[:, 2] <= H // 16 + H // 8))
    assert np.all((r[:, 4] >= -3) & (r[:, 4] <= 3) & (r[:, 5] >= -4) & (r[:, 5] <= 4))


def test_video_rectangle_moves():
    """A pixel covered by the last rectangle at frame t shows that rectangle's
    level up to the noise, at the position its velocity gives."""
    T, H, W = 12, 64, 80
    q = synth.video_levels(6, T, H, W)
    top0, left0, rh, rw, vy, vx, lq = synth.video_rects(6, H, W)[-1]
    for t in (0, 5, 11):
        h = (top0 + vy * t) % H
        w = (left0 + vx * t) % W
        assert abs(int(q[t, h * W + w]) - int(np.clip(lq, -128, 127))) <= 18
