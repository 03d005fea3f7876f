#!/usr/bin/env python3
"""Throughput of the DSGM hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
                    [--legs main,mixed,video,filtered,warped,grid,streaming,attainable,adjoint,
                            batched,largest]
                    [--no-cpu-baseline]

Main workload (the `value`): the plain method in FP64, one instance of
1920 x 2560 pixels x 500 frames (64x the paper's 320 x 240 x 500 sequence),
frames i.i.d. U[-1,1) and a random mid-run model state from seed 1, generated
on the device.  One step is one call of dsgm_forward over all 500 frames of
every pixel (masks out, state updated in place; the next step continues from
that state, so every step does identical work).  Inputs are resident in HBM
before the timed region starts.  Element = one pixel-frame update.

Secondary legs, reported under "legs" (same timing method):
  mixed    BF16 frames (8-bit grid) with FP32 state vs the FP64 path on the same
           frames: throughput of both, and how far the FP32 results are from the
           FP64 ones (which the parity tests prove bit-identical to the oracle)
  video    the same size on a structured video (static background, exposure step,
           moving rectangles, 8-bit levels) from a state initialised from frame 0:
           FP64 and BF16/FP32 throughput on a realistic decision mix
  filtered the main workload with the paper's preprocessing (Gaussian blur, 3x3
           median) fused into the forward, FP64 and BF16/FP32
  warped   motion-compensated update: 100 frames, one launch per frame, each with
           its own camera homography (the model is gathered through it), FP64
  grid     Yi et al.'s grid model (4x4-pixel blocks) on the main workload's frames
  streaming  one call per frame (T = 1): FP64 against the appendix's 8-bit as-run
           model, whose state is 6 bytes per pixel instead of 68
  attainable  the same bytes as the forward and backward kernels moved by kernels
           with no model arithmetic: the attainable HBM rate of each access pattern
  adjoint  FP32 frames and state, bg on, checkpoints every 32 frames, upstream
           gradients ~N(0,1) (seed 2): forward and dsgm_backward throughput
  batched  512 instances of log-uniform size (seed 3), BF16 frames, FP32 state,
           one graph-captured persistent launch per step, against the plain FP64
           form (FP64 frames of the same values, FP64 state) on the same instances
  largest  one 2160x3840x1344 instance (~200 GB resident), FP32 frames, FP64
           state and arithmetic, FP32 bg and gradients: forward and backward

Prints one JSON line: throughput, the roofline of the main kernel (HBM bound;
algorithmic bytes per launch over the kernel's HIP-event duration), the
oracle's CPU throughput on a bounded sample, and the legs.  Parity of each
timed launch configuration against the oracle is checked by the test suite
(test_full_size_f64_sampled_bit_exact, test_full_size_f32_forward_and_adjoint_sampled,
test_full_size_batched_sampled, test_full_size_io32_forward_and_adjoint_sampled).
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
# VALU lane-ops/s, an FMA counted as one op.  FP64: the published 78.6 TFLOP/s
# vector peak -> 39.3 T, i.e. 64 lanes per CU per clock at 2.4 GHz on 256 CUs.
# FP32: the published 157.3 TFLOP/s vector peak -> 78.6 T.  That figure is
# quoted for packed FP32, which the library does not emit; it is still the
# ceiling used, because 32-bit VALU instructions measurably retire faster than
# 64 lanes per CU per clock here: the BF16/FP32 forward's counters give 39.3
# VALU wavefront instructions x 64 lanes per element over 2.4576 G elements in
# 2.0108 ms, i.e. 48.0 T lane-ops/s, above the 39.3 T that a 64-lane issue
# limit allows (profiles/counters_all_kernels.md, row `fwd_kernel<dsgm::bf16_t,
# float, float, 4, 4, 0>`).  With the 39.3 T figure that kernel would run at
# 122 % of its ceiling.
VALU_PEAK_F64 = 256 * 64 * 2.4e9
VALU_PEAK_F32 = 256 * 128 * 2.4e9

# Algorithmic VALU ops per element (one pixel-frame), counted from the update
# equations on the executed branch with the i.i.d. input's mix (A-match 40 %,
# C-match 15 %, reset 45 %): A test 5, C test 5 when A misses, update 10
# (8 flops, 2 integer) when a model matches, reset 3 moves, exchange test 1,
# mask 6 -> about 22.  The other paths add their own arithmetic to that.
OPS_STEP = 22
OPS_ADJOINT = 36    # replay of the step (22) + reverse sweep of the matched update (14)
OPS_PRE = 22 + 18 + 14   # + 5-tap row and column passes (9 each) + 3 x 3 median (14 min/max)
OPS_WARP = 22 + 32 + 6 + 28 + 4   # + homography (2 divisions) + weights + 4 bilinear planes + nearest
OPS_GRID4 = 10 + 22 / 16   # per pixel: block sum 1, V 3, mask 6; the step once per 16 pixels
OPS_U8 = 22 + 12    # + the 8-bit storage rule on 4 values
OPS_PRE_U8 = OPS_U8 + 50 + 14 + 2   # + the 5 x 5 window (25 products, 25 sums), median, store rule


# the sources a kernel is compiled from: its translation unit and the headers
# that unit includes (a change anywhere else does not change the kernel)
KERNEL_SOURCES = {
    "fwd_kernel_f64_f64_p2": ["dsgm_fwd_f64_f64.hip", "dsgm_fwd_impl.h", "dsgm_internal.h",
                              "dsgm_device.h", "dsgm_f32x2.h", "dsgm_geom.h"],
}


def source_hash(kernel: str) -> str:
    h = hashlib.sha256()
    for name in sorted(KERNEL_SOURCES[kernel]):
        with open(os.path.join(ROOT, "paper_1702_05156_amd", "csrc", name), "rb") as fh:
            h.update(name.encode() + fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str):
    """HBM traffic per launch from committed counter runs, if they were taken on
    the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("source_hash") != source_hash(kernel):
        return None
    return d.get("traffic_bytes_per_launch")


def cpu_baseline(T, H, W, seed, target_s=10.0, chunk_rows=32):
    """The FP64 oracle on a bounded sample of the same workload: whole rows of
    pixels over all T frames (pixels are independent, so a row sample is the
    same per-element work), generated and run in chunks of rows until about
    `target_s` seconds of oracle time have accumulated or the rows run out.
    Only the oracle's own time is counted."""
    import numpy as np
    import oracle
    import synth

    p = oracle.default_params(2.0)
    cores = oracle.max_threads()  # read first: a thread count passed to the oracle sticks
    done_rows, n, dt = 0, 0, 0.0
    while done_rows < H and dt < target_s:
        rows = min(chunk_rows, H - done_rows)
        pix = np.arange(done_rows * W, (done_rows + rows) * W)
        x = synth.frames(seed, T, H, W, "f64", pix=pix)
        st = synth.state(seed, H, W, "f64", 30, pix=pix)
        t0 = time.perf_counter()
        oracle.forward(x, st, p, bg=False, codes=False, nthreads=cores)
        dt += time.perf_counter() - t0
        n += rows * W * T
        done_rows += rows
        del x, st
    # the same oracle on one thread, over the first chunk of rows
    rows = min(chunk_rows, H)
    pix = np.arange(0, rows * W)
    x = synth.frames(seed, T, H, W, "f64", pix=pix)
    st = synth.state(seed, H, W, "f64", 30, pix=pix)
    t0 = time.perf_counter()
    oracle.forward(x, st, p, bg=False, codes=False, nthreads=1)
    dt1 = time.perf_counter() - t0
    n1 = rows * W * T
    return {"value": n / dt, "unit": "elements/s", "cores": cores, "kind": "oracle",
            "sample": f"rows 0-{done_rows - 1} of {H} x {W} columns x {T} frames = {n} elements "
                      f"(FP64 scalar C, OpenMP over pixel chunks), {dt:.2f} s of oracle time",
            "cpu_model": cpu_model(),
            "single_thread": {"value": n1 / dt1, "unit": "elements/s",
                              "sample": f"rows 0-{rows - 1}: {n1} elements, {dt1:.2f} s"}}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# The paper's own figures, quoted as context: it prints no kernel-only rate for
# this step, only whole-program times and speed-ups on its 2012-era GPUs, with
# OpenCV preprocessing and per-frame display included.
PAPER_CONTEXT = {
    "note": "whole-program figures on the paper's hardware (no kernel-only rate is printed); "
            "context, not a target",
    "sequence": "320x240 pixels x 500 frames = 38.4 M pixel-frames (Sec. 4.2.1)",
    "gt650m_opencv_filters_cuda_dsgm_s": 9.35,
    "gt650m_derived_elements_per_s": round(38.4e6 / 9.35, -3),
    "gt650m_own_filters_serial_cuda_dsgm_s": 50.74,
    "gt650m_cuda_separable_gaussian_cuda_median_s": 13.03,
    "gt650m_hardware": "GeForce GT 650M (Kepler) + Core i7 2.6 GHz, 121 threads per block, mean of "
                       "20 runs (Sec. 4.3.2, the preprocessing comparison table)",
    "gt650m_speedup_vs_serial": 2.5,
    "gtx570_speedup_vs_serial": 2.7,
    "speedup_source": "whole program incl. OpenCV filters and frame display; GT 650M Sec. 4.3.3, "
                      "GTX 570 (Fermi) Sec. 4.3.4",
}


def progress(msg: str) -> None:
    """One progress line on stderr (stdout carries only the result line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def timed(fn, steps, warmup, stream):
    """Run fn `warmup` times, then time `steps` calls: (ms per step over the whole
    region, per-call HIP-event durations in ms), events on `stream`."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for i in range(steps):
        ev[i][0].record(stream)
        fn()
        ev[i][1].record(stream)
    stop.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / steps, [a.elapsed_time(b) for a, b in ev]


def timed_launches(call, n, steps, warmup, stream):
    """For paths of n launches per step, call(i) making the i-th: (ms per step
    over the whole region, mean duration of one launch in ms).  The durations
    come from a second pass with HIP events around every launch, so that the
    events' own host cost does not enter the wall-clock figure."""
    import torch
    for _ in range(warmup):
        for i in range(n):
            call(i)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(steps):
        for i in range(n):
            call(i)
    stop.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / steps
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(n)]
    durs = []
    for _ in range(steps):
        for i in range(n):
            ev[i][0].record(stream)
            call(i)
            ev[i][1].record(stream)
        torch.cuda.synchronize()
        durs += [a.elapsed_time(b) for a, b in ev]
    return ms, sum(durs) / len(durs)


def roof(alg_bytes, k_ms, elems=None, ops=None, fp32=False):
    """Roofline of one launch: algorithmic bytes over its duration against the
    HBM peak; with the launch's elements and the algorithmic VALU ops per
    element (in FP32 or FP64 arithmetic), also both ceilings in elements/s.
    `bound` names the binding ceiling: "hbm" (achieved in GB/s) or "alu"
    (achieved in algorithmic lane-ops/s against the VALU peak, the HBM figures
    kept under "hbm")."""
    gbs = alg_bytes / (k_ms * 1e-3) / 1e9
    out = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(gbs / HBM_PEAK_GBS, 4)}
    if elems and ops:
        rate = elems / (k_ms * 1e-3)
        hbm_c = HBM_PEAK_GBS * 1e9 * elems / alg_bytes
        valu_peak = VALU_PEAK_F32 if fp32 else VALU_PEAK_F64
        valu_c = valu_peak / ops
        binding = "hbm" if hbm_c <= valu_c else "valu"
        if binding == "valu":
            out = {"bound": "alu", "achieved": round(rate * ops / 1e12, 3),
                   "peak": round(valu_peak / 1e12, 3), "unit": "T lane-ops/s",
                   "frac": round(rate / valu_c, 4), "hbm": out}
        out["ceilings"] = {"bytes_per_element": round(alg_bytes / elems, 4), "ops_per_element": ops,
                           "arithmetic": "f32" if fp32 else "f64",
                           "hbm_elements_per_s": round(hbm_c, 1),
                           "valu_elements_per_s": round(valu_c, 1),
                           "binding": binding,
                           "frac_of_binding": round(rate / min(hbm_c, valu_c), 4)}
    return out


def fp64_error(dsgm, torch, run, fr, st_lo, var_init):
    """Error of one reduced-precision pass against the FP64 pass on the same
    frames from the same start (the FP64 state holds the reduced state's
    values, so both see identical inputs; the FP64 GPU path is the oracle's
    arithmetic bit for bit).  run(state, masks, codes) makes one pass; with
    codes=None it is the launch the leg times, and every error below is
    measured on that launch's masks and state.  The same pass is made once
    more with decision codes (a one-pixel-per-lane variant), which must give
    the same bits; its codes say which pixels diverged (any decision differs
    from the FP64 pass)."""
    T, H, W = fr.shape
    clone = lambda s: dsgm.State(*(t.clone() for t in s.planes()))
    a_lo, a_cd = clone(st_lo), clone(st_lo)
    a64 = dsgm.State(st_lo.mean_a.double(), st_lo.var_a.double(), st_lo.mean_c.double(),
                     st_lo.var_c.double(), st_lo.age_a.clone(), st_lo.age_c.clone())
    m_lo = torch.empty((T, H, W), dtype=torch.uint8, device="cuda")
    m_cd, m64 = torch.empty_like(m_lo), torch.empty_like(m_lo)
    c_lo, c64 = torch.empty_like(m_lo), torch.empty_like(m_lo)
    run(a_lo, m_lo, None)
    run(a_cd, m_cd, c_lo)
    run(a64, m64, c64)
    torch.cuda.synchronize()
    same_bits = bool(torch.equal(m_lo, m_cd)) and all(
        torch.equal(a, b) for a, b in zip(a_lo.planes(), a_cd.planes()))
    div = ((c_lo & 15) != (c64 & 15)).any(dim=0)
    del m_cd, c_lo, c64, a_cd
    same = ~div
    dm = (a_lo.mean_a.double() - a64.mean_a).abs()
    dv = (a_lo.var_a.double() - a64.var_a).abs() / torch.clamp(a64.var_a, min=var_init)
    out = {"measured_on": "the timed launch (no decision codes)",
           "timed_launch_equals_codes_variant": same_bits,
           "mask_elements_differing_frac": float((m_lo != m64).sum().item()) / (T * H * W),
           "pixels_with_any_mask_difference_frac":
               float((m_lo != m64).any(dim=0).sum().item()) / (H * W),
           "pixels_with_any_decision_difference_frac": float(div.sum().item()) / (H * W),
           "max_abs_mean_a_err_undiverged": float(dm[same].max().item()) if bool(same.any()) else None,
           "max_rel_var_a_err_undiverged": float(dv[same].max().item()) if bool(same.any()) else None}
    return out, same


# ---------------------------------------------------------------- legs
def leg_mixed(args, dsgm, sdev, torch):
    """BF16 frames: FP32 state vs FP64 state on the same frames."""
    T, H, W, seed = 500, 1920, 2560, 1
    p = dsgm.dsgm_params_default(2.0)
    fr = sdev.frames(seed, T, H, W, torch.bfloat16)
    st32 = dsgm.State(*sdev.state(seed, H, W, torch.float32))
    st64 = dsgm.State(*sdev.state(seed, H, W, torch.float64))
    m32 = torch.empty((T, H, W), dtype=torch.uint8, device="cuda")
    m64 = torch.empty_like(m32)
    stream = torch.cuda.current_stream()
    s32, s64 = st32.clone(), st64.clone()
    steps = max(3, args.steps // 2)
    ms32, k32 = timed(lambda: dsgm.dsgm_forward(fr, s32, p, m32), steps, 2, stream)
    ms64, k64 = timed(lambda: dsgm.dsgm_forward(fr, s64, p, m64), steps, 2, stream)
    err, _ = fp64_error(dsgm, torch, lambda s_, m_, c_: dsgm.dsgm_forward(fr, s_, p, m_, codes=c_),
                        fr, st32, p.var_init)
    elems = T * H * W
    out = {
        "workload": "bf16 frames 1920x2560x500 seed 1, masks only",
        "fp32_state": {"elements_per_s": round(elems / (ms32 * 1e-3), 1), "ms_per_step": round(ms32, 4),
                       "roofline": roof(elems * 3 + H * W * 36, float(sum(k32) / len(k32)), elems, OPS_STEP, True)},
        "fp64_state": {"elements_per_s": round(elems / (ms64 * 1e-3), 1), "ms_per_step": round(ms64, 4),
                       "roofline": roof(elems * 3 + H * W * 68, float(sum(k64) / len(k64)), elems, OPS_STEP)},
        "speedup_fp32_over_fp64": round(ms64 / ms32, 3),
        "error_vs_fp64": err,
    }
    del fr, st32, st64, m32, m64, s32, s64
    torch.cuda.empty_cache()
    return out


def leg_video(args, dsgm, sdev, torch):
    """The structured video (static background, exposure step at frame 250,
    six moving rectangles, ~3-level noise, 8-bit levels), 1920x2560x500, seed 1,
    state initialised from frame 0 before the first step; FP64 and BF16/FP32."""
    T, H, W, seed = 500, 1920, 2560, 1
    p = dsgm.dsgm_params_default(2.0)
    stream = torch.cuda.current_stream()
    elems, px = T * H * W, H * W
    steps = max(3, args.steps // 2)
    out = {"workload": "structured video 1920x2560x500 seed 1, masks only, state from frame 0"}
    for name, in_dt, acc_dt, in_b, st_b in (("fp64", torch.float64, torch.float64, 8, 68),
                                             ("bf16_fp32", torch.bfloat16, torch.float32, 2, 36)):
        fr = sdev.video(seed, T, H, W, in_dt)
        st = dsgm.State.empty(H, W, acc_dt)
        dsgm.dsgm_state_init_from_frame(fr[0], st, p)
        masks = torch.empty((T, H, W), dtype=torch.uint8, device="cuda")
        st0 = dsgm.State(*(t.clone() for t in st.planes()))
        ms, kk = timed(lambda: dsgm.dsgm_forward(fr, st, p, masks), steps, 1, stream)
        out[name] = {"elements_per_s": round(elems / (ms * 1e-3), 1), "ms_per_step": round(ms, 4),
                     "roofline": roof(elems * (in_b + 1) + px * st_b, float(sum(kk) / len(kk)),
                                      elems, OPS_STEP, acc_dt == torch.float32)}
        if acc_dt == torch.float32:
            out[name]["error_vs_fp64"], _ = fp64_error(
                dsgm, torch, lambda s_, m_, c_: dsgm.dsgm_forward(fr, s_, p, m_, codes=c_), fr, st0,
                p.var_init)
        del fr, st, masks
        torch.cuda.empty_cache()
    return out


def leg_filtered(args, dsgm, sdev, torch):
    """The forward with the paper's preprocessing fused in (5-tap Gaussian,
    sigma 1, then the 3x3 median): the main workload's frames and state (FP64),
    BF16 frames with FP32 state, and the appendix's 8-bit pipeline (U8 frames
    and state, its two-dimensional single-precision blur)."""
    T, H, W, seed = 500, 1920, 2560, 1
    p = dsgm.dsgm_params_default(2.0)
    filt = dsgm.gauss_filter(5, 1.0, True)
    stream = torch.cuda.current_stream()
    elems, px = T * H * W, H * W
    steps = max(3, args.steps // 2)
    out = {"workload": "1920x2560x500 seed 1, masks only, 5-tap Gaussian (sigma 1) + 3x3 median "
                       "fused into the forward"}
    for name, in_dt, acc_dt, in_b, st_b in (("fp64", torch.float64, torch.float64, 8, 68),
                                             ("bf16_fp32", torch.bfloat16, torch.float32, 2, 36)):
        fr = sdev.frames(seed, T, H, W, in_dt)
        st = dsgm.State(*sdev.state(seed, H, W, acc_dt))
        masks = torch.empty((T, H, W), dtype=torch.uint8, device="cuda")
        st0 = dsgm.State(*(t.clone() for t in st.planes()))
        ms, kk = timed(lambda: dsgm.dsgm_forward_filtered(fr, st, p, filt, masks), steps, 1, stream)
        if acc_dt == torch.float32:
            err, _ = fp64_error(
                dsgm, torch,
                lambda s_, m_, c_: dsgm.dsgm_forward_filtered(fr, s_, p, filt, m_, codes=c_),
                fr, st0, p.var_init)
        out[name] = {"elements_per_s": round(elems / (ms * 1e-3), 1), "ms_per_step": round(ms, 4),
                     "roofline": roof(elems * (in_b + 1) + px * st_b, float(sum(kk) / len(kk)),
                                      elems, OPS_PRE, acc_dt == torch.float32)}
        if acc_dt == torch.float32:
            out[name]["error_vs_fp64"] = err
        del fr, st, st0, masks
        torch.cuda.empty_cache()
    # the appendix's pipeline on 8-bit images: its two-dimensional single-
    # precision blur written back to 8 bits, the median of the 8-bit image and
    # the 8-bit as-run update, on the structured video at 8-bit levels
    fr = (sdev.video(seed, T, H, W, torch.float32) * 128 + 128).to(torch.uint8)
    p8 = dsgm.dsgm_params_default(255.0, dsgm.MASK_PRINTED)
    p8.weight_rule = dsgm.WEIGHT_APPENDIX
    st = dsgm.State.empty(H, W, torch.uint8)
    dsgm.dsgm_state_init_from_frame(fr[0], st, p8)
    masks = torch.empty((T, H, W), dtype=torch.uint8, device="cuda")
    ms, kk = timed(lambda: dsgm.dsgm_forward_filtered(fr, st, p8, filt, masks), steps, 1, stream)
    out["u8_as_run"] = {"workload": "structured video at 8-bit levels, 8-bit state, the appendix's "
                                    "weights and printed mask rule",
                        "elements_per_s": round(elems / (ms * 1e-3), 1), "ms_per_step": round(ms, 4),
                        "roofline": roof(elems * 2 + px * 12, float(sum(kk) / len(kk)), elems,
                                         OPS_PRE_U8)}
    del fr, st, masks
    torch.cuda.empty_cache()
    return out


def leg_warped(args, dsgm, sdev, torch):
    """Motion-compensated update: 100 frames of 1920x2560 (FP64 frames and state,
    seed 1), each with its own small camera homography (shift of up to 1.5
    pixels and a rotation of up to 0.01 rad, seed 5), one launch per frame
    ping-ponging two state buffers; element = one pixel-frame update."""
    import numpy as np
    T, H, W, seed = 100, 1920, 2560, 1
    p = dsgm.dsgm_params_default(2.0)
    stream = torch.cuda.current_stream()
    fr = sdev.frames(seed, T, H, W, torch.float64)
    a = dsgm.State(*sdev.state(seed, H, W, torch.float64))
    b = dsgm.State.empty(H, W)
    masks = torch.empty((H, W), dtype=torch.uint8, device="cuda")
    rng = np.random.default_rng(5)
    maps = []
    for _ in range(T):
        m = np.eye(3)
        m[0, 2], m[1, 2] = rng.uniform(-1.5, 1.5, size=2)
        m[0, 1], m[1, 0] = rng.uniform(-0.01, 0.01, size=2)
        maps.append(m)
    bufs = [a, b]

    def call(t):
        dsgm.dsgm_forward_warped(fr[t], bufs[t % 2], bufs[1 - t % 2], p, maps[t], masks)

    steps = max(2, args.steps // 4)
    ms, k_ms = timed_launches(call, T, steps, 1, stream)
    elems = T * H * W
    out = {"workload": "1920x2560 x 100 frames, fp64, one launch per frame, per-frame homography",
           "elements_per_s": round(elems / (ms * 1e-3), 1), "ms_per_step": round(ms, 4),
           "kernel_ms_avg": round(k_ms, 5),
           "roofline": roof(H * W * (8 + 1 + 34 + 34), k_ms, H * W, OPS_WARP)}
    del fr, a, b, masks, bufs
    torch.cuda.empty_cache()
    return out


def leg_grid(args, dsgm, sdev, torch):
    """Yi et al.'s grid model, blocks of 4 x 4 pixels, on the main workload's
    FP64 frames (1920x2560x500, seed 1) from a random block state; element =
    one pixel-frame (its mask bit), as for the pixel model."""
    T, H, W, seed, b = 500, 1920, 2560, 1, 4
    p = dsgm.dsgm_params_default(2.0)
    stream = torch.cuda.current_stream()
    fr = sdev.frames(seed, T, H, W, torch.float64)
    st = dsgm.State(*sdev.state(seed, H // b, W // b, torch.float64))
    masks = torch.empty((T, H, W), dtype=torch.uint8, device="cuda")
    steps = max(3, args.steps // 2)
    ms, kk = timed(lambda: dsgm.dsgm_forward_grid(fr, st, p, b, masks), steps, 1, stream)
    elems = T * H * W
    out = {"workload": "1920x2560x500 fp64, 4x4-pixel blocks, masks only",
           "elements_per_s": round(elems / (ms * 1e-3), 1), "ms_per_step": round(ms, 4),
           "roofline": roof(elems * 9 + (H // b) * (W // b) * 68, float(sum(kk) / len(kk)),
                       elems, OPS_GRID4)}
    del fr, st, masks
    torch.cuda.empty_cache()
    return out


def leg_streaming(args, dsgm, sdev, torch):
    """Streaming, one call per frame (T = 1), 1920x2560 x 50 frames: the model
    state goes through HBM every frame.  FP64 (68 bytes of state per pixel,
    read and written) against the appendix's 8-bit as-run model (6 bytes), on
    the structured video at 8-bit levels, seed 1."""
    import numpy as np
    T, H, W, seed = 50, 1920, 2560, 1
    stream = torch.cuda.current_stream()
    steps = max(2, args.steps // 4)
    elems, px = T * H * W, H * W
    out = {"workload": "1920x2560 x 50 frames, one dsgm_forward call per frame"}
    v = sdev.video(seed, T, H, W, torch.float64)                       # q/128, q in -128..127
    for name, frames, st_dtype, p, st_bytes, in_b in (
            ("fp64", v, torch.float64, dsgm.dsgm_params_default(2.0), 34, 8),
            ("u8_as_run", (v * 128 + 128).to(torch.uint8), torch.uint8,
             dsgm.dsgm_params_default(255.0, dsgm.MASK_PRINTED), 6, 1)):
        if name == "u8_as_run":
            p.weight_rule = dsgm.WEIGHT_APPENDIX
        st = dsgm.State.empty(H, W, st_dtype)
        dsgm.dsgm_state_init_from_frame(frames[0], st, p)
        masks = torch.empty((T, H, W), dtype=torch.uint8, device="cuda")

        ops = OPS_U8 if name == "u8_as_run" else OPS_STEP

        def call(t):
            dsgm.dsgm_forward(frames[t:t + 1], st, p, masks[t:t + 1])

        ms, k_ms = timed_launches(call, T, steps, 1, stream)
        out[name] = {"elements_per_s": round(elems / (ms * 1e-3), 1), "ms_per_step": round(ms, 4),
                     "kernel_ms_avg": round(k_ms, 5),
                     "roofline": roof(px * (in_b + 1 + 2 * st_bytes), k_ms, px, ops),
                     "bytes_per_element": in_b + 1 + 2 * st_bytes}
        del st, masks, frames
    del v
    torch.cuda.empty_cache()
    out["speedup_u8_over_fp64"] = round(out["u8_as_run"]["elements_per_s"] /
                                        out["fp64"]["elements_per_s"], 3)
    return out


def leg_attainable(args, dsgm, sdev, torch):
    """Attainable HBM rate of each kernel's access pattern: kernels that move the
    same bytes in the same order, widths and cache hints as the forward and
    backward kernels but do no model arithmetic (synth/probe.hip), at the size
    of the main and adjoint workloads.  The real kernels' rates are compared
    with these as well as with the published peak."""
    T, H, W = 500, 1920, 2560
    npx, elems = H * W, T * H * W
    stream = torch.cuda.current_stream()
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    out = {}
    masks = torch.empty((T, H, W), dtype=torch.uint8, device="cuda")
    for name, dt, P in (("forward_f64_frames_p2", torch.float64, 2),
                        ("forward_f32_frames_p2", torch.float32, 2),
                        ("forward_bf16_frames_p4", torch.bfloat16, 4)):
        fr = torch.zeros((T, H, W), dtype=dt, device="cuda")
        ms, kk = timed(lambda: sdev.probe_forward(fr, P, masks, sink), 5, 2, stream)
        k = float(sum(kk) / len(kk))
        out[name] = {"bytes_per_element": fr.element_size() + 1, "kernel_ms": round(k, 4),
                     "GB_per_s": round(elems * (fr.element_size() + 1) / (k * 1e-3) / 1e9, 1)}
        del fr
        torch.cuda.empty_cache()
    del masks
    for name, dt in (("backward_f32", torch.float32), ("backward_f64", torch.float64)):
        x = torch.zeros((T, H, W), dtype=dt, device="cuda")
        g = torch.zeros_like(x)
        gx = torch.empty_like(x)
        ms, kk = timed(lambda: sdev.probe_backward(x, g, gx), 5, 2, stream)
        k = float(sum(kk) / len(kk))
        out[name] = {"bytes_per_element": 3 * x.element_size(), "kernel_ms": round(k, 4),
                     "GB_per_s": round(elems * 3 * x.element_size() / (k * 1e-3) / 1e9, 1)}
        del x, g, gx
        torch.cuda.empty_cache()
    return out


def leg_adjoint(args, dsgm, sdev, torch):
    T, H, W, K, seed = 500, 1920, 2560, 32, 2
    p = dsgm.dsgm_params_default(2.0)
    fr = sdev.frames(seed, T, H, W, torch.float32)
    st = dsgm.State(*sdev.state(seed, H, W, torch.float32))
    masks = torch.empty((T, H, W), dtype=torch.uint8, device="cuda")
    bg = torch.empty((T, H, W), dtype=torch.float32, device="cuda")
    ck = torch.empty(dsgm.dsgm_ckpt_bytes(T, H, W, dsgm.ACC_F32, K), dtype=torch.uint8, device="cuda")
    gbg = sdev.grad_bg(seed + 100, T, H, W, torch.float32)
    gst = sdev.grad_state(seed + 100, H, W, torch.float32)
    gst = tuple(gst[i].contiguous() for i in range(4))
    gx = torch.empty((T, H, W), dtype=torch.float32, device="cuda")
    gs0 = tuple(torch.empty((H, W), dtype=torch.float32, device="cuda") for _ in range(4))
    gvi = torch.empty(1, dtype=torch.float64, device="cuda")
    ws = torch.empty(dsgm.dsgm_workspace_bytes(T, H, W, dsgm.ACC_F32), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    st0 = st.clone()
    steps = max(3, args.steps // 2)
    msf, kf = timed(lambda: dsgm.dsgm_forward(fr, st, p, masks, bg, ck, K), steps, 2, stream)
    # the backward of one forward pass from the initial state
    for a, b in zip(st.planes(), st0.planes()):
        a.copy_(b)
    dsgm.dsgm_forward(fr, st, p, masks, bg, ck, K)
    msb, kb = timed(lambda: dsgm.dsgm_backward(fr, p, ck, K, dsgm.ACC_F32, gbg, gst, gx, gs0, gvi, ws),
                    steps, 1, stream)
    # error against the FP64 forward and adjoint on the same inputs (upstream
    # gradients upcast); gradients compared on the pixels whose decisions agree
    def run_fwd(s_, m_, c_):
        # the timed launch's outputs (bg and checkpoints) in the state's own type
        acc_ = dsgm.ACC_F32 if s_.mean_a.dtype == torch.float32 else dsgm.ACC_F64
        bg_ = torch.empty((T, H, W), dtype=s_.mean_a.dtype, device="cuda")
        ck_ = torch.empty(dsgm.dsgm_ckpt_bytes(T, H, W, acc_, K), dtype=torch.uint8, device="cuda")
        dsgm.dsgm_forward(fr, s_, p, m_, bg_, ck_, K, codes=c_)

    ferr, same = fp64_error(dsgm, torch, run_fwd, fr, st0, p.var_init)
    s64 = dsgm.State(st0.mean_a.double(), st0.var_a.double(), st0.mean_c.double(),
                     st0.var_c.double(), st0.age_a.clone(), st0.age_c.clone())
    r64 = dsgm.backward(fr, p, dsgm.forward(fr, s64, p, ckpt_every=K)["ckpt"], K, dsgm.ACC_F64,
                        gbg.double(), tuple(g.double() for g in gst))
    torch.cuda.synchronize()
    keep = same.view(1, -1).double()  # 1 on undiverged pixels
    num = den = 0.0
    for t0 in range(0, T, 50):  # in frame chunks: no full-size FP64 temporaries
        g32 = gx[t0:t0 + 50].reshape(-1, H * W).double()
        g64 = r64["grad_frames"][t0:t0 + 50].reshape(-1, H * W)
        num += float((((g32 - g64) * keep) ** 2).sum())
        den += float(((g64 * keep) ** 2).sum())
    snum = sum(float((((a.reshape(1, -1).double() - b.reshape(1, -1)) * keep) ** 2).sum())
               for a, b in zip(gs0, r64["grad_state0"]))
    sden = sum(float(((b.reshape(1, -1) * keep) ** 2).sum()) for b in r64["grad_state0"])
    berr = {"grad_frames_rel_l2_undiverged": (num / den) ** 0.5,
            "grad_state0_rel_l2_undiverged": (snum / sden) ** 0.5}
    del s64, r64, g32, g64, same, keep
    elems, px = T * H * W, H * W
    ck_slots = (T + K - 1) // K
    fwd_bytes = elems * (4 + 1 + 4) + px * 36
    bwd_bytes = elems * 12 + px * (16 + 16 + 8)
    out = {
        "workload": "fp32 frames and state 1920x2560x500 seed 2, bg on, K=32",
        "forward": {"elements_per_s": round(elems / (msf * 1e-3), 1), "ms_per_step": round(msf, 4),
                    "roofline": roof(fwd_bytes, float(sum(kf) / len(kf)), elems, OPS_STEP, True),
                    "checkpoint_bytes_written": ck_slots * px * 18},
        "backward": {"elements_per_s": round(elems / (msb * 1e-3), 1), "ms_per_step": round(msb, 4),
                     "roofline": roof(bwd_bytes, float(sum(kb) / len(kb)), elems, OPS_ADJOINT, True),
                     "checkpoint_bytes_read": ck_slots * px * 18},
        "grad_var_init": float(gvi.item()),
        "error_vs_fp64": dict(ferr, **berr),
    }
    del fr, st, st0, masks, bg, ck, gbg, gst, gx, gs0, gvi, ws
    torch.cuda.empty_cache()
    return out


def leg_largest(args, dsgm, sdev, torch):
    """The largest single instance: 2160 x 3840 x 1344 (11.1 G elements, ~200 GB
    resident), FP32 frames, FP64 state and arithmetic, FP32 bg and gradient
    arrays (decisions and state those of the FP64 path, arrays rounded once),
    checkpoints every 32 frames, upstream gradients ~N(0,1), seed 4."""
    T, H, W, K, seed = 1344, 2160, 3840, 32, 4
    acc = dsgm.ACC_F64_IO32
    p = dsgm.dsgm_params_default(2.0)
    fr = sdev.frames(seed, T, H, W, torch.float32)
    st = dsgm.State(*sdev.state(seed, H, W, torch.float64))
    st0 = st.clone()
    masks = torch.empty((T, H, W), dtype=torch.uint8, device="cuda")
    bg = torch.empty((T, H, W), dtype=torch.float32, device="cuda")
    ck = torch.empty(dsgm.dsgm_ckpt_bytes(T, H, W, acc, K), dtype=torch.uint8, device="cuda")
    gbg = sdev.grad_bg(seed + 100, T, H, W, torch.float32)
    gst = sdev.grad_state(seed + 100, H, W, torch.float32)
    gst = tuple(gst[i].contiguous() for i in range(4))
    gx = torch.empty((T, H, W), dtype=torch.float32, device="cuda")
    gs0 = tuple(torch.empty((H, W), dtype=torch.float32, device="cuda") for _ in range(4))
    gvi = torch.empty(1, dtype=torch.float64, device="cuda")
    ws = torch.empty(dsgm.dsgm_workspace_bytes(T, H, W, acc), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    resident = torch.cuda.memory_allocated()
    stream = torch.cuda.current_stream()
    steps = max(2, args.steps // 8)
    msf, kf = timed(lambda: dsgm.dsgm_forward(fr, st, p, masks, bg, ck, K, acc=acc), steps, 1, stream)
    for a, b in zip(st.planes(), st0.planes()):
        a.copy_(b)
    dsgm.dsgm_forward(fr, st, p, masks, bg, ck, K, acc=acc)
    msb, kb = timed(lambda: dsgm.dsgm_backward(fr, p, ck, K, acc, gbg, gst, gx, gs0, gvi, ws),
                    steps, 1, stream)
    # error against FP64 arrays on a band of rows (pixels are independent, so
    # the band run alone is the full run's arithmetic for those pixels): the
    # FP32 bg and gradients must be the FP64 values rounded once
    R = 64
    # copies (a row slice of a dense plane is itself dense, and the forward
    # updates the state it is given in place)
    sb = dsgm.State(*(t[:R].clone() for t in st0.planes()))
    fb = fr[:, :R].contiguous()  # dense, so the outputs dsgm.forward allocates are too
    ob = dsgm.forward(fb, sb, p, bg=True, ckpt_every=K)
    rb = dsgm.backward(fb, p, ob["ckpt"], K, dsgm.ACC_F64, gbg[:, :R].double(),
                       tuple(g[:R].double() for g in gst))
    torch.cuda.synchronize()
    bg64, gx64 = ob["bg"], rb["grad_frames"]
    rel = lambda a, b: float(((a.double() - b).abs() / b.abs().clamp(min=1e-300)).max())
    err = {"band": f"rows 0-{R - 1}, all {T} frames",
           "masks_equal": bool(torch.equal(masks[:, :R], ob["masks"])),
           "bg_equals_fp64_rounded_once": bool(torch.equal(bg[:, :R], bg64.float())),
           "grad_frames_equal_fp64_rounded_once": bool(torch.equal(gx[:, :R], gx64.float())),
           "max_rel_err_bg": rel(bg[:, :R], bg64),
           "max_rel_err_grad_frames": rel(gx[:, :R], gx64)}
    gvi_io32 = float(gvi.item())
    del sb, ob, rb, bg64, gx64
    # the same instance in compensated single precision (F32X2: (hi, lo) float
    # pairs, FP32 instruction rates), from the pairs nearest to the FP64 start,
    # timed on the same buffers (the pair state has the FP64 state's size)
    x2 = dsgm.ACC_F32X2
    sx = dsgm.State(*(dsgm.x2_from_f64(t) if t.is_floating_point() else t.clone()
                      for t in st0.planes()))
    sx0 = sx.clone()
    msf2, kf2 = timed(lambda: dsgm.dsgm_forward(fr, sx, p, masks, bg, ck, K, acc=x2), steps, 1,
                      stream)
    for a, b in zip(sx.planes(), sx0.planes()):
        a.copy_(b)
    dsgm.dsgm_forward(fr, sx, p, masks, bg, ck, K, acc=x2)
    msb2, kb2 = timed(lambda: dsgm.dsgm_backward(fr, p, ck, K, x2, gbg, gst, gx, gs0, gvi, ws),
                      steps, 1, stream)
    gvi_x2 = float(gvi.item())
    # the band again in FP64 (GPU FP64 path = the oracle's arithmetic) from the
    # pair values, against the pair run's outputs on that band
    sb = dsgm.State(*(dsgm.x2_to_f64(t[:R]) if t.is_complex() else t[:R].clone()
                      for t in sx0.planes()))
    ob = dsgm.forward(fb, sb, p, bg=True, codes=True, ckpt_every=K)
    sxb = dsgm.State(*(t[:R].clone() for t in sx0.planes()))
    cb = torch.empty_like(ob["codes"])
    dsgm.dsgm_forward(fb, sxb, p, torch.empty_like(ob["masks"]), codes=cb)
    rb = dsgm.backward(fb, p, ob["ckpt"], K, dsgm.ACC_F64, gbg[:, :R].double(),
                       tuple(g[:R].double() for g in gst))
    torch.cuda.synchronize()
    def beyond(a, r):
        """largest |a - r| beyond half an FP32 ulp of r (<= 0: rounded once)"""
        f = r.float().abs()
        half_ulp = 0.5 * (torch.nextafter(f, torch.full_like(f, float("inf"))).double() - f.double())
        return float(((a.double() - r).abs() - half_ulp).max())
    fin = {k: float((dsgm.x2_to_f64(getattr(sx, k)[:R]) - getattr(sb, k)).abs().max())
           for k in ("mean_a", "var_a", "mean_c", "var_c")}
    err_x2 = {"band": f"rows 0-{R - 1}, all {T} frames, against the FP64 path from the same values",
              "decision_elements_differing": int((cb != ob["codes"]).sum().item()),
              "masks_equal": bool(torch.equal(masks[:, :R], ob["masks"])),
              "max_abs_err_final_state": max(fin.values()),
              "bg_beyond_half_ulp_of_fp64": beyond(bg[:, :R], ob["bg"]),
              "grad_frames_beyond_half_ulp_of_fp64": beyond(gx[:, :R], rb["grad_frames"]),
              "max_rel_err_grad_frames": rel(gx[:, :R], rb["grad_frames"])}
    del sb, fb, ob, rb, sxb, cb, sx, sx0
    elems, px = T * H * W, H * W
    ck_slots = (T + K - 1) // K
    out_x2 = {"workload": "the same instance with F32X2 state (compensated FP32 pairs), "
                          "fp32 bg/gradients",
              "forward": {"elements_per_s": round(elems / (msf2 * 1e-3), 1),
                          "ms_per_step": round(msf2, 3),
                          "roofline": roof(elems * 9 + px * 68, float(sum(kf2) / len(kf2)), elems,
                                           OPS_STEP, fp32=True)},
              "backward": {"elements_per_s": round(elems / (msb2 * 1e-3), 1),
                           "ms_per_step": round(msb2, 3),
                           "roofline": roof(elems * 12 + px * 40, float(sum(kb2) / len(kb2)), elems,
                                            OPS_ADJOINT, fp32=True)},
              "grad_var_init": gvi_x2,
              "time_ratio_over_f64_io32": {"forward": round(msf2 / msf, 3),
                                           "backward": round(msb2 / msb, 3)},
              "error_vs_fp64": err_x2}
    out = {"workload": "2160x3840x1344 fp32 frames, fp64 state, fp32 bg/gradients, K=32, seed 4",
           "resident_bytes": int(resident),
           "forward": {"elements_per_s": round(elems / (msf * 1e-3), 1), "ms_per_step": round(msf, 3),
                       "roofline": roof(elems * 9 + px * 68, float(sum(kf) / len(kf)), elems, OPS_STEP),
                       "checkpoint_bytes_written": ck_slots * px * 34},
           "backward": {"elements_per_s": round(elems / (msb * 1e-3), 1), "ms_per_step": round(msb, 3),
                        "roofline": roof(elems * 12 + px * 40, float(sum(kb) / len(kb)), elems, OPS_ADJOINT),
                        "checkpoint_bytes_read": ck_slots * px * 34},
           "grad_var_init": gvi_io32,
           "error_vs_fp64": err,
           "f32x2": out_x2}
    del fr, st, st0, masks, bg, ck, gbg, gst, gx, gs0, gvi, ws
    torch.cuda.empty_cache()
    return out


def batch_shapes(seed=3, n=512):
    """Instance sizes: m = 256^u with u ~ U[0,1) (synth stream 10), width
    8*round(40 m^(1/4)), height 8*round(30 m^(1/4)), frames round(32 m^(1/2)):
    elements ~ m * (320*240*32), log-uniform over 1x..256x of that unit."""
    import numpy as np
    import synth
    u = (synth.uniform(seed, 10, np.arange(n), "f64") + 1.0) / 2.0
    m = 256.0 ** u
    W = 8 * np.round(40 * m ** 0.25).astype(int)
    H = 8 * np.round(30 * m ** 0.25).astype(int)
    T = np.round(32 * m ** 0.5).astype(int)
    return [(int(t), int(h), int(w)) for t, h, w in zip(T, H, W)]


def batch_seed(i: int) -> int:
    return 3000 + i


def fp64_chunks(shapes, max_bytes=130e9):
    """The batch's FP64 form in launches that fit: consecutive instances while
    their FP64 frames stay within max_bytes."""
    chunks, cur, cur_bytes = [], [], 0
    for i, (T, H, W) in enumerate(shapes):
        b = T * H * W * 8
        if cur and cur_bytes + b > max_bytes:
            chunks.append(cur)
            cur, cur_bytes = [], 0
        cur.append(i)
        cur_bytes += b
    chunks.append(cur)
    return chunks


def _batch_items(shapes, idx, dsgm, sdev, torch, frames_dtype, state_dtype, st0):
    """Instances `idx` of the batch: BF16-grid frames stored as `frames_dtype`
    (exact upcast), the FP32 initial state `st0[i]` stored as `state_dtype`."""
    items = []
    for i in idx:
        T, H, W = shapes[i]
        fr = sdev.frames(batch_seed(i), T, H, W, torch.bfloat16)
        if frames_dtype != torch.bfloat16:
            fr = fr.to(frames_dtype)
        s = st0[i]
        cp = lambda t: t.to(dtype=state_dtype, copy=True)  # never the initial state itself
        st = dsgm.State(cp(s.mean_a), cp(s.var_a), cp(s.mean_c), cp(s.var_c), s.age_a.clone(),
                        s.age_c.clone())
        # every instance counts its foreground pixels per frame (the batched
        # launch's reduction: exact integer sums, one atomic per wavefront and frame)
        items.append((fr, st, torch.empty((T, H, W), dtype=torch.uint8, device="cuda"), None,
                      torch.empty((T,), dtype=torch.int32, device="cuda")))
    return items


def _counts_exact(items, torch):
    """every instance's counters equal the 255s of its masks, frame by frame"""
    for _, _, m, _, c in items:
        T = m.shape[0]
        if not torch.equal(c, (m.view(T, -1) == 255).sum(dim=1).to(torch.int32)):
            return False
    return True


def leg_batched(args, dsgm, sdev, torch):
    """The mixed-precision batched form (BF16 frames, FP32 state, one graph-
    captured persistent launch) against the plain FP64 form (FP64 frames holding
    the same values, FP64 state from the same initial values) on the same 512
    instances.  The FP64 form does not fit in HBM at once (481 GB of frames), so
    it runs as consecutive batched launches over chunks of the instance list and
    its time is the sum of the chunks'.  Accuracy: the masks of one pass from
    the common initial state, mixed vs FP64."""
    shapes = batch_shapes()
    p = dsgm.dsgm_params_default(2.0)
    stream = torch.cuda.current_stream()
    st0 = [dsgm.State(*sdev.state(batch_seed(i), H, W, torch.float32)) for i, (T, H, W) in
           enumerate(shapes)]
    items = _batch_items(shapes, range(len(shapes)), dsgm, sdev, torch, torch.bfloat16,
                         torch.float32, st0)
    # the tile width (pixels per lane) of the plan is picked by the autotuner
    from paper_1702_05156_amd import tune
    tuned = tune.tune_batched(items, p, store=False)
    batch = dsgm.Batch(items, vector=tuned["vector"], grid=tuned["grid"])
    batch.run(p)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(stream)
    with torch.cuda.graph(g, stream=s):
        batch.run(p)
    torch.cuda.synchronize()
    steps = max(3, args.steps // 4)
    ms, kk = timed(g.replay, steps, 1, stream)
    elems = batch.plan.total_elements
    px = sum(H * W for _, H, W in shapes)
    alg = elems * 3 + px * 36
    n_items, grid = int(batch.plan.n_items), int(batch.plan.grid)
    # one pass from the initial state for the accuracy comparison
    for (_, st, _, _, _), s0 in zip(items, st0):
        for a, b in zip(st.planes(), s0.planes()):
            a.copy_(b)
    batch.run(p)
    torch.cuda.synchronize()
    counts_ok = _counts_exact(items, torch)
    fg_total = sum(int(c.sum().item()) for *_, c in items)
    masks_mixed = [m for _, _, m, _, _ in items]
    del items, batch, g
    torch.cuda.empty_cache()

    # the FP64 form, chunked to fit
    chunks = fp64_chunks(shapes)
    ms64 = 0.0
    k64 = []
    diff_elems = 0
    diff_px = 0
    for idx in chunks:
        it = _batch_items(shapes, idx, dsgm, sdev, torch, torch.float64, torch.float64, st0)
        b64 = dsgm.Batch(it)
        b64.run(p)
        torch.cuda.synchronize()
        counts_ok = counts_ok and _counts_exact(it, torch)
        for i, (_, _, m, _, _) in zip(idx, it):
            d = m != masks_mixed[i]
            diff_elems += int(d.sum().item())
            diff_px += int(d.any(dim=0).sum().item())
        m_chunk, k_chunk = timed(lambda: b64.run(p), steps, 1, stream)
        ms64 += m_chunk
        k64.append(float(sum(k_chunk) / len(k_chunk)))
        del it, b64
        torch.cuda.empty_cache()
    del masks_mixed, st0
    torch.cuda.empty_cache()
    out = {"workload": "512 instances, log-uniform 1x..256x of 320x240x32, bf16 frames, fp32 state, "
                       "masks and per-frame foreground counts, seed 3",
           "fg_counts_equal_mask_sums": counts_ok,
           "foreground_fraction": fg_total / elems,
           "instances": len(shapes), "total_elements": int(elems), "work_items": n_items,
           "persistent_workgroups": grid,
           "autotuned_pixels_per_lane": tuned["vector"],
           "autotuned_grid_fraction": tuned["grid_fraction"],
           "autotune_candidates_ms": {f'{c["vector"]}px/{c["grid"]}wg': round(c["ms"], 3)
                                      for c in tuned["candidates"]},
           "elements_per_s": round(elems / (ms * 1e-3), 1), "ms_per_step": round(ms, 4),
           "roofline": roof(alg, float(sum(kk) / len(kk)), elems, OPS_STEP, True),
           "fp64_form": {"workload": "the same 512 instances, fp64 frames (same values) and fp64 "
                                     "state, batched launches over %d chunks" % len(chunks),
                         "elements_per_s": round(elems / (ms64 * 1e-3), 1),
                         "ms_per_step": round(ms64, 4),
                         "roofline": roof(elems * 9 + px * 68, sum(k64), elems, OPS_STEP)},
           "speedup_mixed_over_fp64": round(ms64 / ms, 3),
           "error_vs_fp64": {"mask_elements_differing_frac": diff_elems / elems,
                             "pixels_with_any_mask_difference_frac": diff_px / px}}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--legs",
                    default="main,mixed,video,filtered,warped,grid,streaming,attainable,adjoint,"
                            "batched,largest")
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

    legs = set(args.legs.split(","))
    T, H, W, seed = 500, 1920, 2560, 1
    p = dsgm.dsgm_params_default(2.0)
    fr = sdev.frames(seed, T, H, W, torch.float64)
    st = dsgm.State(*sdev.state(seed, H, W, torch.float64))
    masks = torch.empty((T, H, W), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    t_wall = time.perf_counter()
    ms_step, kern_ms = timed(lambda: dsgm.dsgm_forward(fr, st, p, masks), args.steps, args.warmup,
                             stream)
    t_wall = time.perf_counter() - t_wall
    elems = T * H * W
    value = elems / (ms_step * 1e-3)
    px = H * W
    alg_bytes = elems * (8 + 1) + px * (4 * 8 + 2) * 2
    k_avg = float(np.mean(kern_ms))
    kernel = "fwd_kernel_f64_f64_p2"
    rf = roof(alg_bytes, k_avg, elems, OPS_STEP)
    rf.update({"traffic": load_traffic(kernel), "kernel": kernel, "kernel_ms_avg": round(k_avg, 4),
               "alg_bytes_per_launch": alg_bytes,
               "alg_bytes_per_element": round(alg_bytes / elems, 4)})
    del fr, st, masks
    torch.cuda.empty_cache()

    out_legs = {}
    progress(f"main leg done: {value / 1e9:.1f} G elements/s")
    for name, fn in (("mixed", leg_mixed), ("video", leg_video), ("filtered", leg_filtered),
                     ("warped", leg_warped), ("grid", leg_grid), ("streaming", leg_streaming),
                     ("attainable", leg_attainable), ("adjoint", leg_adjoint),
                     ("batched", leg_batched), ("largest", leg_largest)):
        if name in legs:
            t0 = time.perf_counter()
            out_legs[name] = fn(args, dsgm, sdev, torch)
            progress(f"{name} leg done in {time.perf_counter() - t0:.1f} s")

    cpu = None if args.no_cpu_baseline else cpu_baseline(T, H, W, seed)
    if cpu is not None:
        progress("cpu baseline done")

    out = {
        "metric": "hot-path elements/s and % roofline (fwd+adjoint), mixed vs FP64 at tol",
        "value": round(value, 1), "unit": "elements/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "dsgm_forward_fp64_1920x2560x500", "T": T, "H": H, "W": W,
                   "frames": "f64", "state": "f64", "outputs": "masks", "seed": seed,
                   "element": "one pixel-frame update"},
        "roofline": rf, "cpu_baseline": cpu, "paper_context": PAPER_CONTEXT, "legs": out_legs,
        "wall_s_timed": round(t_wall, 3),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
