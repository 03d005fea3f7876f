// dsgm_internal.h -- host/device interface between the C ABI layer and the
// kernels of libdsgm.so (internal; not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dsgm_device.h"

namespace dsgm {

// Arguments of the forward kernels, passed by value as the kernel argument.
struct FwdArgs {
  const void* frames;
  uint8_t* masks;
  void* bg;
  uint8_t* codes;
  void* mean_a;
  void* var_a;
  void* mean_c;
  void* var_c;
  uint8_t* age_a;
  uint8_t* age_c;
  void* ckpt;             // NULL: no checkpoints
  int64_t ckpt_every;     // K
  int64_t ckpt_slot_bytes;// bytes of one checkpoint (4 float planes + 2 age planes)
  int64_t ckpt_fplane;    // bytes of one float plane, padded to 256
  int64_t ckpt_aplane;    // bytes of one age plane, padded to 256
  int64_t T, H, W, row_stride, frame_stride;
  int64_t groups_per_row; // W / P
  int64_t ngroups;        // H * W / P
  double theta_s, theta_d, var_init, var_floor, mask_floor;
  int32_t age_max, weight_rule, mask_rule;
};

// in_dtype: 0 f64, 1 f32, 2 bf16; acc: 0 f64, 1 f32; P in {1, 2, 4}
hipError_t launch_forward(const FwdArgs& a, int in_dtype, int acc, int P, int block,
                          hipStream_t stream);

// state = (x, var_init, 1) for both models from frame 0 (uses frames, the
// state planes, H, W, row_stride, var_init)
hipError_t launch_init(const FwdArgs& a, int in_dtype, int acc, hipStream_t stream);

}  // namespace dsgm
