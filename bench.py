#!/usr/bin/env python3
"""Throughput of the DSGM hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Workload: the plain method in FP64, one instance of 1920 x 2560 pixels x 500
frames (64x the paper's 320 x 240 x 500 sequence), frames i.i.d. U[-1,1) and a
random mid-run model state from seed 1, generated on the device.  One step is
one call of dsgm_forward over all 500 frames of every pixel (masks out, state
updated in place; the next step continues from that state, so every step does
identical work).  Inputs are resident in HBM before the timed region starts.

Prints one JSON line with the throughput in elements/s (element = one
pixel-frame update), the roofline of the forward kernel (HBM bound; bytes per
launch over the kernel's HIP-event duration) and the oracle's CPU throughput on
a bounded sample.  Parity of this exact launch configuration against the oracle
is checked by tests/test_gpu_forward.py::test_full_size_f64_sampled_bit_exact.
"""
from __future__ import annotations

import argparse
import hashlib
import glob
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def source_hash() -> str:
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1702_05156_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode() + fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str):
    """HBM traffic per launch from committed counter runs, if they were taken on
    the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("source_hash") != source_hash():
        return None
    return d.get("traffic_bytes_per_launch")


def cpu_baseline(T, H, W, seed, target_s=12.0):
    """The FP64 oracle on a bounded sample of the same workload: whole rows of
    pixels, all T frames (pixels are independent, so a row sample is the same
    per-element work)."""
    import numpy as np
    import oracle
    import synth

    p = oracle.default_params(2.0)

    def run(rows):
        pix = np.arange(rows * W)
        x = synth.frames(seed, T, H, W, "f64", pix=pix)
        st = synth.state(seed, H, W, "f64", 30, pix=pix)
        t0 = time.perf_counter()
        oracle.forward(x, st, p, bg=False, codes=False)
        return time.perf_counter() - t0, rows * W * T

    dt, n = run(4)
    rows = int(min(H, max(4, 4 * target_s / max(dt, 1e-6))))
    dt, n = run(rows)
    return {"value": n / dt, "unit": "elements/s", "cores": oracle.max_threads(), "kind": "oracle",
            "sample": f"{rows} of {H} rows x {W} columns x {T} frames = {n} elements, "
                      f"FP64 scalar C, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter scale)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the DSGM update is independent per pixel, so "
              "several GPUs would each run this same kernel on their own band of rows with no "
              "exchange; run it with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    torch.cuda.set_device(0)
    if args.copy_probe:
        n = args.copy_probe * (1 << 20)
        a = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n}))
        return

    from paper_1702_05156_amd import dsgm
    from synth import device as sdev

    T, H, W, seed = 500, 1920, 2560, 1
    p = dsgm.dsgm_params_default(2.0)
    fr = sdev.frames(seed, T, H, W, torch.float64)
    st = dsgm.State(*sdev.state(seed, H, W, torch.float64))
    masks = torch.empty((T, H, W), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        dsgm.dsgm_forward(fr, st, p, masks)
    torch.cuda.synchronize()

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    start.record(stream)
    for i in range(args.steps):
        ev[i][0].record(stream)
        dsgm.dsgm_forward(fr, st, p, masks)
        ev[i][1].record(stream)
    stop.record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    total_ms = start.elapsed_time(stop)
    kern_ms = [a.elapsed_time(b) for a, b in ev]
    ms_step = total_ms / args.steps
    elems = T * H * W
    value = elems / (ms_step * 1e-3)

    px = H * W
    alg_bytes = elems * (8 + 1) + px * (4 * 8 + 2) * 2
    k_avg = float(np.mean(kern_ms))
    achieved = alg_bytes / (k_avg * 1e-3) / 1e9
    kernel = "fwd_kernel_f64_f64_p4"
    traffic = load_traffic(kernel)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": kernel, "kernel_ms_avg": round(k_avg, 4),
            "alg_bytes_per_launch": alg_bytes, "alg_bytes_per_element": round(alg_bytes / elems, 4)}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(T, H, W, seed)

    out = {
        "metric": "hot-path elements/s and % roofline (fwd+adjoint), mixed vs FP64 at tol",
        "value": round(value, 1), "unit": "elements/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "dsgm_forward_fp64_1920x2560x500", "T": T, "H": H, "W": W,
                   "frames": "f64", "state": "f64", "outputs": "masks", "seed": seed,
                   "element": "one pixel-frame update"},
        "roofline": roof, "cpu_baseline": cpu,
        "wall_s_timed": round(t_wall, 3),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
