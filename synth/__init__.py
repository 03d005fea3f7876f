"""Seeded synthetic inputs: a counter-based SplitMix64 generator (host side).

This module is shared by the CPU oracle's tests and by the GPU path's tests and
benchmark.  It holds none of the background-model arithmetic: it only turns
(seed, stream, index) into numbers.  The device twin in ``synth/synth.hip``
implements the same definitions independently, so a GPU buffer filled there is
bit-identical to what the functions below return for the same logical indices.

Definition (SplitMix64, Steele, Lea and Flood, OOPSLA 2014; the constants of
Vigna's reference splitmix64.c):

    mix(z)  = z3 where z1 = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
                       z2 = (z1 ^ (z1 >> 27)) * 0x94D049BB133111EB
                       z3 = z2 ^ (z2 >> 31)                 (all mod 2**64)
    gamma   = 0x9E3779B97F4A7C15
    output number i (0-based) of a generator seeded with s = mix(s + (i+1)*gamma)

Streams:   key(seed, stream) = mix(mix(seed + gamma) + (stream + 1) * gamma)
           draw(seed, stream, i) = mix(key + (i + 1) * gamma)

Value maps (all exact, no rounding anywhere):
  uniform, f64 : (k >> 11) * 2**-52 - 1        53-bit grid on [-1, 1)
  uniform, f32 : (k >> 40) * 2**-23 - 1        24-bit grid on [-1, 1)
  uniform, bf16: (k >> 56) * 2**-7  - 1        8-bit grid on [-1, 1) (like 8-bit video)
  age in {1..A}: 1 + (((k >> 32) * A) >> 32)
  normal       : Irwin-Hall sum of 12 16-bit uniforms from draws 3i, 3i+1, 3i+2
                 (four 16-bit chunks each, low chunk first):
                 (sum_chunks - 393210) * 2**-16, mean 0, variance ~1, exact in f32.
  below(k, n)  : ((k >> 32) * n) >> 32, an integer in [0, n)

Structured video (``video``): 8-bit-like levels q in [-128, 127], value q/128
(exact in f64, f32 and bf16), all in integer arithmetic:
  background  bq(p) = below(draw(seed, 11, p), 161) - 80, static per pixel
  lighting    + 4 levels from frame T//2 on (a global exposure step)
  objects     6 rectangles, parameters from draws 8r..8r+6 of stream 13:
              top0 = below(k0, H), left0 = below(k1, W),
              height = H//16 + below(k2, H//8 + 1), width = W//16 + below(k3, W//8 + 1),
              vy = below(k4, 7) - 3, vx = below(k5, 9) - 4, level = below(k6, 256) - 128;
              at frame t the rectangle starts at ((top0 + vy*t) mod H, (left0 + vx*t) mod W)
              and wraps around the frame edges; a later rectangle covers an earlier one
  noise       n = floor((3 * (S - 393210) + 2**15) / 2**16), S the Irwin-Hall sum of
              stream 12 at the element's logical index (mean 0, standard deviation ~3 levels)
  value       clamp(level + n, -128, 127) / 128 with level = the covering rectangle's
              level, else bq + lighting.

The logical index of element (t, h, w) of a T x H x W array is t*H*W + h*W + w,
whatever the strides of the buffer it is stored in.
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# stream numbers used by the workloads
STREAM_FRAMES = 0
STREAM_MEAN_A = 1
STREAM_MEAN_C = 2
STREAM_VAR_A = 3
STREAM_VAR_C = 4
STREAM_AGE_A = 5
STREAM_AGE_C = 6
STREAM_GRAD_BG = 7
STREAM_GRAD_STATE = 8
STREAM_DIRECTION = 9
STREAM_BATCH_SIZES = 10
STREAM_VIDEO_BG = 11
STREAM_VIDEO_NOISE = 12
STREAM_VIDEO_RECTS = 13
VIDEO_RECTS = 6
VIDEO_LIGHT_STEP = 4

DTYPES = ("f64", "f32", "bf16")


def mix64(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def stream_key(seed: int, stream: int) -> np.uint64:
    with np.errstate(over="ignore"):
        k0 = mix64(np.array([np.uint64(seed % 2**64) + GAMMA], dtype=np.uint64))[0]
        s = np.uint64(stream + 1) * GAMMA
        return mix64(np.array([k0 + s], dtype=np.uint64))[0]


def draws(seed: int, stream: int, index) -> np.ndarray:
    """Raw 64-bit draws at the given logical indices (any integer array)."""
    idx = np.asarray(index, dtype=np.uint64)
    key = stream_key(seed, stream)
    with np.errstate(over="ignore"):
        return mix64(key + (idx + np.uint64(1)) * GAMMA)


def uniform(seed: int, stream: int, index, dtype: str = "f64") -> np.ndarray:
    """U[-1, 1) on the dtype's exact grid, returned as float64 (exact values)."""
    k = draws(seed, stream, index)
    if dtype == "f64":
        return (k >> np.uint64(11)).astype(np.float64) * 2.0 ** -52 - 1.0
    if dtype == "f32":
        return (k >> np.uint64(40)).astype(np.float64) * 2.0 ** -23 - 1.0
    if dtype == "bf16":
        return (k >> np.uint64(56)).astype(np.float64) * 2.0 ** -7 - 1.0
    raise ValueError(f"unknown dtype {dtype!r}")


def abs_uniform(seed: int, stream: int, index, dtype: str = "f64") -> np.ndarray:
    return np.abs(uniform(seed, stream, index, dtype))


def ages(seed: int, stream: int, index, age_max: int) -> np.ndarray:
    k = draws(seed, stream, index)
    hi = k >> np.uint64(32)
    with np.errstate(over="ignore"):
        a = (hi * np.uint64(age_max)) >> np.uint64(32)
    return (a + np.uint64(1)).astype(np.int32)


def normal(seed: int, stream: int, index) -> np.ndarray:
    """Approximately N(0,1): Irwin-Hall sum of 12 16-bit uniforms (exact in f32)."""
    return (irwin_hall_sum(seed, stream, index) - 393210).astype(np.float64) * 2.0 ** -16


def below(k: np.ndarray, n: int) -> np.ndarray:
    """Map 64-bit draws to integers in [0, n) (n < 2**32), as int64."""
    with np.errstate(over="ignore"):
        return ((np.asarray(k, dtype=np.uint64) >> np.uint64(32)) * np.uint64(n) >> np.uint64(32)).astype(np.int64)


def irwin_hall_sum(seed: int, stream: int, index) -> np.ndarray:
    """The integer Irwin-Hall sum S of ``normal`` (so normal = (S - 393210) * 2**-16)."""
    idx = np.asarray(index, dtype=np.uint64)
    total = np.zeros(idx.shape, dtype=np.int64)
    mask16 = np.uint64(0xFFFF)
    for j in range(3):
        with np.errstate(over="ignore"):
            k = draws(seed, stream, idx * np.uint64(3) + np.uint64(j))
        for c in range(4):
            total += ((k >> np.uint64(16 * c)) & mask16).astype(np.int64)
    return total


def video_rects(seed: int, H: int, W: int) -> np.ndarray:
    """The six rectangles of ``video``: rows (top0, left0, height, width, vy, vx, level)."""
    k = draws(seed, STREAM_VIDEO_RECTS, np.arange(8 * VIDEO_RECTS, dtype=np.uint64)).reshape(VIDEO_RECTS, 8)
    out = np.empty((VIDEO_RECTS, 7), dtype=np.int64)
    out[:, 0] = below(k[:, 0], H)
    out[:, 1] = below(k[:, 1], W)
    out[:, 2] = H // 16 + below(k[:, 2], H // 8 + 1)
    out[:, 3] = W // 16 + below(k[:, 3], W // 8 + 1)
    out[:, 4] = below(k[:, 4], 7) - 3
    out[:, 5] = below(k[:, 5], 9) - 4
    out[:, 6] = below(k[:, 6], 256) - 128
    return out


def video_levels(seed: int, T: int, H: int, W: int, t=None, pix=None) -> np.ndarray:
    """Integer levels q in [-128, 127] of the structured video, shape (len(t), len(pix))."""
    t = np.arange(T, dtype=np.int64) if t is None else np.asarray(t, dtype=np.int64)
    pix = np.arange(H * W, dtype=np.int64) if pix is None else np.asarray(pix, dtype=np.int64)
    h = (pix // W)[None, :]
    w = (pix % W)[None, :]
    tt = t[:, None]
    level = (below(draws(seed, STREAM_VIDEO_BG, pix.astype(np.uint64)), 161) - 80)[None, :] \
        + np.where(tt >= T // 2, VIDEO_LIGHT_STEP, 0)
    level = np.broadcast_to(level, (len(t), len(pix))).copy()
    for top0, left0, rh, rw, vy, vx, lq in video_rects(seed, H, W):
        top = (top0 + vy * tt) % H
        left = (left0 + vx * tt) % W
        inside = ((h - top) % H < rh) & ((w - left) % W < rw)
        level = np.where(inside, lq, level)
    idx = (tt.astype(np.uint64) * np.uint64(H * W) + pix.astype(np.uint64)[None, :])
    noise = ((irwin_hall_sum(seed, STREAM_VIDEO_NOISE, idx) - 393210) * 3 + 32768) >> 16
    return np.clip(level + noise, -128, 127)


def video(seed: int, T: int, H: int, W: int, t=None, pix=None) -> np.ndarray:
    """Structured video frames as float64 values q/128, shape (len(t), len(pix))."""
    return video_levels(seed, T, H, W, t, pix).astype(np.float64) / 128.0


# ---------------------------------------------------------------- workloads
def logical_index(T: int, H: int, W: int, t=None, pix=None) -> np.ndarray:
    """Logical indices of frames [t] x pixels [pix] (flat pixel p = h*W + w).

    Returns an array of shape (len(t), len(pix)).
    """
    t = np.arange(T, dtype=np.uint64) if t is None else np.asarray(t, dtype=np.uint64)
    pix = np.arange(H * W, dtype=np.uint64) if pix is None else np.asarray(pix, dtype=np.uint64)
    return t[:, None] * np.uint64(H * W) + pix[None, :]


def frames(seed: int, T: int, H: int, W: int, dtype: str, t=None, pix=None) -> np.ndarray:
    """Frames as float64 values, shape (len(t), len(pix))."""
    return uniform(seed, STREAM_FRAMES, logical_index(T, H, W, t, pix), dtype)


def state(seed: int, H: int, W: int, acc: str, age_max: int, pix=None) -> dict:
    """Random mid-run model state for the given flat pixels (all, by default)."""
    pix = np.arange(H * W, dtype=np.uint64) if pix is None else np.asarray(pix, dtype=np.uint64)
    g = "f64" if acc == "f64" else "f32"
    return {
        "mean_a": uniform(seed, STREAM_MEAN_A, pix, g),
        "mean_c": uniform(seed, STREAM_MEAN_C, pix, g),
        "var_a": abs_uniform(seed, STREAM_VAR_A, pix, g),
        "var_c": abs_uniform(seed, STREAM_VAR_C, pix, g),
        "age_a": ages(seed, STREAM_AGE_A, pix, age_max),
        "age_c": ages(seed, STREAM_AGE_C, pix, age_max),
    }


def grad_bg(seed: int, T: int, H: int, W: int, t=None, pix=None) -> np.ndarray:
    return normal(seed, STREAM_GRAD_BG, logical_index(T, H, W, t, pix))


def grad_state(seed: int, H: int, W: int, pix=None) -> np.ndarray:
    """Upstream gradient of the final (mean_a, var_a, mean_c, var_c); shape (4, npix)."""
    pix = np.arange(H * W, dtype=np.uint64) if pix is None else np.asarray(pix, dtype=np.uint64)
    idx = np.arange(4, dtype=np.uint64)[:, None] * np.uint64(H * W) + pix[None, :]
    return normal(seed, STREAM_GRAD_STATE, idx)
