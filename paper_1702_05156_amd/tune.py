"""Launch-shape autotuner for the DSGM kernels.

The forward kernels have two free launch parameters that do not change any
result (the tests check bit-identical outputs across them): the workgroup size
(64, 128 or 256 threads) and the number of horizontally adjacent pixels each
lane owns (1, 2 or 4: wider means wider loads and stores but more registers and
fewer waves per SIMD).  The tuner times every legal candidate on the caller's
own buffers with HIP events (the model state is cloned for every trial, so the
caller's state is left as it was), keeps the fastest, and caches it in a JSON
file keyed by the problem's types, output set and sizes:

    $DSGM_TUNE_CACHE, else ~/.cache/dsgm_tune.json

``tuned(key)`` is a context manager that applies a cached shape through
``dsgm_set_launch`` for the calls inside it (the setting is per process).

``tune_batched`` does the same for a batch of uneven instances over two
dimensions: the tile width (pixels per lane: 1, 2, 4), with which it plans the
batch, and the number of persistent workgroups (the planner's device-filling
count, three quarters and half of it).  It times one launch of each pair and
returns (and caches) the fastest; ``Batch(items, vector=best["vector"],
grid=best["grid"])`` then plans with it.
"""
from __future__ import annotations

import contextlib
import json
import os
import threading

import torch

from . import dsgm

BLOCKS = (64, 128, 192, 256)
VECTORS = (1, 2, 4)
GRID_FRACTIONS = (1.0, 0.75, 0.5)  # of the planner's device-filling persistent grid
_lock = threading.Lock()


def cache_path() -> str:
    return os.environ.get("DSGM_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "dsgm_tune.json"))


def _load() -> dict:
    try:
        with open(cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(cache: dict) -> None:
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + f".tmp{os.getpid()}"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def forward_key(frames: torch.Tensor, state: "dsgm.State", *, bg=False, ckpt_every=0,
                mask_rule=0) -> str:
    T, H, W = frames.shape
    return (f"fwd/{str(frames.dtype)[6:]}/{str(state.mean_a.dtype)[6:]}/bg{int(bool(bg))}/"
            f"ck{int(ckpt_every > 0)}/m{mask_rule}/{H}x{W}")


def lookup(key: str):
    return _load().get(key)


@contextlib.contextmanager
def tuned(key: str):
    """Apply the cached launch shape for `key` (if any) to the calls inside."""
    best = lookup(key)
    if best is None:
        yield None
        return
    with _lock:
        dsgm.dsgm_set_launch(best["block"], best["vector"])
        try:
            yield best
        finally:
            dsgm.dsgm_set_launch(0, 0)


def tune_forward(frames: torch.Tensor, state: "dsgm.State", params: "dsgm.Params", *,
                 bg: bool = False, ckpt_every: int = 0, reps: int = 3, frames_limit: int = 64,
                 store: bool = True) -> dict:
    """Time every (block, vector) candidate of dsgm_forward on these buffers.

    Only the first `frames_limit` frames are used for timing (the cost per frame
    does not depend on T once T is a few dozen).  Returns and caches
    {"block", "vector", "ms_per_frame", "candidates": [...]}.
    """
    fr = frames[: max(1, min(frames.shape[0], frames_limit))]
    T, H, W = fr.shape
    masks = torch.empty_strided(fr.shape, fr.stride(), dtype=torch.uint8, device=fr.device)
    bgt = (torch.empty_strided(fr.shape, fr.stride(), dtype=state.mean_a.dtype, device=fr.device)
           if bg else None)
    ck = None
    if ckpt_every:
        ck = torch.empty(max(dsgm.dsgm_ckpt_bytes(T, H, W, state.acc, ckpt_every), 1),
                         dtype=torch.uint8, device=fr.device)
    results = []
    stream = torch.cuda.current_stream()
    with _lock:
        try:
            for block in BLOCKS:
                for vec in VECTORS:
                    if W % vec:
                        continue
                    dsgm.dsgm_set_launch(block, vec)
                    st = state.clone()
                    dsgm.dsgm_forward(fr, st, params, masks, bgt, ck, ckpt_every)  # warm
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    for _ in range(reps):
                        dsgm.dsgm_forward(fr, st, params, masks, bgt, ck, ckpt_every)
                    e1.record(stream)
                    torch.cuda.synchronize()
                    ms = e0.elapsed_time(e1) / reps / T
                    results.append({"block": block, "vector": vec, "ms_per_frame": ms})
        finally:
            dsgm.dsgm_set_launch(0, 0)
    best = min(results, key=lambda r: r["ms_per_frame"])
    out = dict(best, candidates=results)
    if store:
        key = forward_key(frames, state, bg=bg, ckpt_every=ckpt_every, mask_rule=params.mask_rule)
        with _lock:
            cache = _load()
            cache[key] = {"block": best["block"], "vector": best["vector"],
                          "ms_per_frame": best["ms_per_frame"]}
            _store(cache)
    return out


def batched_key(items) -> str:
    fr0, st0 = items[0][0], items[0][1]
    total = sum(int(fr.numel()) for fr, *_ in items)
    return (f"batched/{str(fr0.dtype)[6:]}/{str(st0.mean_a.dtype)[6:]}/n{len(items)}/"
            f"e{total}")


def tune_batched(items, params: "dsgm.Params", *, reps: int = 2, store: bool = True) -> dict:
    """Time one persistent batched launch per (tile width, persistent grid) pair
    on these instances.

    The instances' states advance with every launch (the timing does not
    depend on the values).  Returns and caches {"vector", "grid",
    "grid_fraction", "ms", "candidates"}.
    """
    results = []
    stream = torch.cuda.current_stream()
    with _lock:
        for vec in VECTORS:
            try:
                b = dsgm.Batch(items, vector=vec)
            except dsgm.DSGMError:
                continue
            if b.plan.vector != vec:
                continue  # a layout the instances do not allow
            full = int(b.plan.grid)
            for frac in GRID_FRACTIONS:
                grid = max(1, int(round(full * frac)))
                b.plan.grid = grid
                b.run(params)  # warm
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for _ in range(reps):
                    b.run(params)
                e1.record(stream)
                torch.cuda.synchronize()
                results.append({"vector": vec, "grid": grid, "grid_fraction": frac,
                                "ms": e0.elapsed_time(e1) / reps,
                                "work_items": int(b.plan.n_items)})
            del b
    if not results:
        raise RuntimeError("no tile width is allowed by these instances")
    best = min(results, key=lambda r: r["ms"])
    out = dict(best, candidates=results)
    if store:
        key = batched_key(items)
        with _lock:
            cache = _load()
            cache[key] = {"vector": best["vector"], "grid": best["grid"],
                          "grid_fraction": best["grid_fraction"], "ms": best["ms"]}
            _store(cache)
    return out
