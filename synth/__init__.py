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
    idx = np.asarray(index, dtype=np.uint64)
    total = np.zeros(idx.shape, dtype=np.int64)
    mask16 = np.uint64(0xFFFF)
    for j in range(3):
        with np.errstate(over="ignore"):
            k = draws(seed, stream, idx * np.uint64(3) + np.uint64(j))
        for c in range(4):
            total += ((k >> np.uint64(16 * c)) & mask16).astype(np.int64)
    return (total - 393210).astype(np.float64) * 2.0 ** -16


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
