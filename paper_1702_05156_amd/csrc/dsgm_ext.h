// dsgm_ext.h -- host/device interface of the kernels beyond the plain
// forward, adjoint and batched paths (internal; not installed): the 8-bit
// as-run model, the fused preprocessing, the motion-compensated update and the
// grid model.
#pragma once

#include "dsgm_internal.h"

namespace dsgm {

// The 8-bit as-run model (dsgm_u8.hip): U8 frames and U8 state planes, FwdArgs
// with var_init already in stored form; flags FWD_CODES and FWD_PRINTED only.
hipError_t launch_fwd_u8(const FwdArgs& a, int P, int flags, int block, hipStream_t stream);
hipError_t launch_init_u8(const FwdArgs& a, hipStream_t stream);

// Arguments of the forward with fused preprocessing (dsgm_pre.hip).
struct PreArgs {
  const void* frames;
  uint8_t* masks;
  void* bg;        // NULL: none
  void* filtered;  // NULL: none; the preprocessed frames, array type
  uint8_t* codes;  // NULL: none
  void* mean_a;
  void* var_a;
  void* mean_c;
  void* var_c;
  uint8_t* age_a;
  uint8_t* age_c;
  int64_t T, H, W, row_stride, frame_stride;
  int64_t tiles_x, tiles_y;
  double theta_s, theta_d, var_init, var_floor, mask_floor;
  int32_t age_max, weight_rule, mask_rule;
  double w[7];  // blur weights, 2*rg+1 of them
};

// rg: blur radius 0..3 (0: no blur); median: 3 x 3 median after the blur
hipError_t launch_pre(const PreArgs& a, int in_dtype, int acc, int rg, bool median,
                      hipStream_t stream);
// the 8-bit form (dsgm_u8.hip): U8 frames and state, var_init already stored,
// the appendix's two-dimensional single-precision blur written back to 8 bits
hipError_t launch_pre_u8(const PreArgs& a, int rg, bool median, hipStream_t stream);

// Arguments of one frame of the update on the motion-compensated model
// (dsgm_warp.hip).
struct WarpArgs {
  const void* frame;
  uint8_t* masks;
  void* bg;        // NULL: none
  uint8_t* codes;  // NULL: none
  const void* src_mean_a;
  const void* src_var_a;
  const void* src_mean_c;
  const void* src_var_c;
  const uint8_t* src_age_a;
  const uint8_t* src_age_c;
  void* dst_mean_a;
  void* dst_var_a;
  void* dst_mean_c;
  void* dst_var_c;
  uint8_t* dst_age_a;
  uint8_t* dst_age_c;
  int64_t H, W, row_stride;
  double map[9];  // current pixel (column, row, 1) -> previous frame, row-major
  double theta_s, theta_d, var_init, var_floor, mask_floor;
  int32_t age_max, weight_rule, mask_rule;
};

hipError_t launch_warp(const WarpArgs& a, int in_dtype, int acc, hipStream_t stream);

// Arguments of the grid-model forward (dsgm_grid.hip).
struct GridArgs {
  const void* frames;
  uint8_t* masks;  // T x H x W, strided like the frames
  void* bg;        // NULL or T x Hb x Wb dense: mean_A of each block after each frame
  uint8_t* codes;  // NULL or T x Hb x Wb dense
  void* mean_a;    // Hb x Wb planes
  void* var_a;
  void* mean_c;
  void* var_c;
  uint8_t* age_a;
  uint8_t* age_c;
  int64_t T, H, W, row_stride, frame_stride, Hb, Wb;
  int32_t vec_ok;  // whole blocks may use one vector access per row
  double theta_s, theta_d, var_init, var_floor, mask_floor;
  int32_t age_max, weight_rule, mask_rule;
};

hipError_t launch_grid(const GridArgs& a, int in_dtype, int acc, int b, hipStream_t stream);

// Fill n elements of the given frame type (0 F64, 1 F32, 2 BF16, 3 U8) with
// independent uniform intensities, a function of (seed, index) (dsgm_tune.hip).
hipError_t launch_tune_fill(void* out, int in_dtype, int64_t n, uint64_t seed,
                            hipStream_t stream);

// Count of the non-finite frame elements (dsgm_check.hip): clears *count,
// then adds the NaN and infinite elements of the T x H x W frames.
struct CountArgs {
  int64_t T, H, W, row_stride, frame_stride;
  unsigned long long* count;
};
hipError_t launch_count_nonfinite(const void* frames, int in_dtype, const CountArgs& a,
                                  hipStream_t stream);

// logical tile of workgroup b of nb, XCD-contiguous (dsgm_geom.h)
using geom::tile_of;

}  // namespace dsgm
