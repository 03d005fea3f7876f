/*
 * synth.h -- device-side seeded synthetic inputs (libsynth.so).
 *
 * Counter-based SplitMix64 (Steele, Lea and Flood, OOPSLA 2014); the exact
 * definitions of the streams and value maps are those of synth/__init__.py,
 * which produces bit-identical values on the host.  This library holds no
 * arithmetic of the background model.  Test and benchmark infrastructure.
 *
 * Destination arrays are T x H x W addressed as t*frame_stride + h*row_stride
 * + w (in elements); the value written there is the one of logical index
 * t*H*W + h*W + w.  All calls are asynchronous on `stream`; return 0 on
 * success, -1 on a bad argument, -6 on a HIP error.
 */
#ifndef SYNTH_H
#define SYNTH_H

#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { SYNTH_F64 = 0, SYNTH_F32 = 1, SYNTH_BF16 = 2 };
enum { SYNTH_UNIFORM = 0, SYNTH_ABS_UNIFORM = 1, SYNTH_NORMAL = 2 };

/* kind: SYNTH_UNIFORM (U[-1,1) on the dtype's exact grid), SYNTH_ABS_UNIFORM
 * (its absolute value), SYNTH_NORMAL (Irwin-Hall, f64/f32 only) */
int synth_fill(void* dst, int32_t dtype, int32_t kind, int64_t T, int64_t H, int64_t W,
               int64_t row_stride, int64_t frame_stride, uint64_t seed, uint64_t stream_id,
               hipStream_t stream);

/* ages in {1..age_max}, dense n bytes, logical index = position */
int synth_ages(uint8_t* dst, int64_t n, int32_t age_max, uint64_t seed, uint64_t stream_id,
               hipStream_t stream);

/* the structured video of synth.video (static background, a global lighting
 * exposure step at frame T/2, six moving rectangles, ~3-level noise; values q/128) */
int synth_video(void* dst, int32_t dtype, int64_t T, int64_t H, int64_t W, int64_t row_stride,
                int64_t frame_stride, uint64_t seed, hipStream_t stream);

/* Memory-access-pattern probes (probe.hip): the byte traffic of the forward
 * (pixels_per_lane adjacent elements of elem_bytes each per lane and frame,
 * nontemporal loads, one mask byte per element out) and of the backward (one
 * element per lane, frames walked backwards, x and g in, gx out), with no model
 * arithmetic.  Frames are dense (frame stride = npx elements); `sink` is one
 * word of scratch that is written only to keep the loads alive. */
int synth_probe_forward(const void* frames, int32_t elem_bytes, int32_t pixels_per_lane,
                        uint8_t* masks, uint32_t* sink, int64_t T, int64_t npx, hipStream_t stream);
int synth_probe_backward(const void* x, const void* g, void* gx, int32_t elem_bytes, int64_t T,
                         int64_t npx, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif
