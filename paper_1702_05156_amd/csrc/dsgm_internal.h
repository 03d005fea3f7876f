// dsgm_internal.h -- host/device interface between the C ABI layer and the
// kernels of libdsgm.so (internal; not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dsgm_device.h"
#include "dsgm_geom.h"

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

// Arguments of the backward kernels.
struct BwdArgs {
  const void* frames;
  const void* ckpt;
  const void* grad_bg;     // NULL: zero
  const void* gst_mean_a;  // upstream gradient of the final planes (all NULL: zero)
  const void* gst_var_a;
  const void* gst_mean_c;
  const void* gst_var_c;
  void* grad_frames;
  void* gs0_mean_a;
  void* gs0_var_a;
  void* gs0_mean_c;
  void* gs0_var_c;
  double* gvi_px;          // H*W per-pixel contributions (workspace)
  int64_t ckpt_every, ckpt_slot_bytes, ckpt_fplane, ckpt_aplane;
  int64_t T, H, W, row_stride, frame_stride;
  double theta_s, theta_d, var_init, var_floor, mask_floor;
  int32_t age_max, weight_rule, mask_rule;
};

hipError_t launch_backward(const BwdArgs& a, int in_dtype, int acc, hipStream_t stream);

// deterministic compensated sum of n doubles into out[0]; partial holds
// 2 * geom::REDUCE_BLOCKS doubles
hipError_t launch_reduce(const double* x, int64_t n, double* partial, double* out,
                         hipStream_t stream);

// Batched forward: device-side descriptors written by the host planner.
// The foreground counts of an instance are accumulated in COUNT_STRIPES
// copies (stripe = work item mod COUNT_STRIPES, each T counters) so that the
// wavefronts working on one instance at the same time add to different
// addresses; a last small kernel adds the stripes into the caller's counters.
constexpr int COUNT_STRIPES = int(geom::COUNT_STRIPES);

struct BatchInst {
  const void* frames;
  uint8_t* masks;
  void* bg;             // NULL: no bg for this instance
  uint32_t* fg_counts;  // NULL: no foreground counts for this instance
  uint32_t* stripes;    // with fg_counts: COUNT_STRIPES x T counters in the plan buffer
  void* state[6];
  int64_t T, H, W, row_stride, frame_stride, groups_per_row;
};

// one wavefront's work: `count` (<= 64) consecutive pixel groups of one instance
struct BatchItem {
  int32_t inst;
  int32_t first_group;
  int32_t count;
  int32_t pad;
};

static_assert(sizeof(BatchInst) == 136, "plan layout: instance descriptor size");
static_assert(sizeof(BatchItem) == 16, "plan layout: item size");

struct BatchArgs {
  unsigned long long* counter;  // next item; reset to 0 by each launch
  const BatchInst* inst;
  int64_t n_inst;
  const BatchItem* items;
  int64_t n_items;
  double theta_s, theta_d, var_init, var_floor, mask_floor;
  int32_t age_max, weight_rule, mask_rule;
};

// Variant flags of the forward kernels (see dsgm_fwd_impl.h).
enum : int { FWD_BG = 1, FWD_CODES = 2, FWD_CKPT = 4, FWD_PRINTED = 8 };

// flags: FWD_BG and FWD_PRINTED only
const void* batched_kernel_symbol(int in_dtype, int acc, int P, int flags);
// counts: some instance has foreground counters (cleared before the launch)
hipError_t launch_batched(const BatchArgs& a, int in_dtype, int acc, int P, int flags, int grid,
                          bool counts, hipStream_t stream);

// in_dtype: 0 f64, 1 f32, 2 bf16; acc: 0 f64, 1 f32, 2 f64 state with f32 bg and
// gradients, 4 f32x2 state with f32 bg and gradients; P in {1, 2, 4}; flags FWD_*
hipError_t launch_forward(const FwdArgs& a, int in_dtype, int acc, int P, int flags, int block,
                          hipStream_t stream);

// per (frames, state) type translation units
#define DSGM_FWD_DECLARE(NAME)                                                              \
  hipError_t launch_fwd_##NAME(const FwdArgs& a, int P, int flags, int block,               \
                               hipStream_t stream);                                         \
  const void* batched_sym_##NAME(int P, int flags);
DSGM_FWD_DECLARE(f64_f64)
DSGM_FWD_DECLARE(f32_f64)
DSGM_FWD_DECLARE(bf16_f64)
DSGM_FWD_DECLARE(f32_f32)
DSGM_FWD_DECLARE(bf16_f32)
DSGM_FWD_DECLARE(f32_f64io32)
DSGM_FWD_DECLARE(bf16_f64io32)
#undef DSGM_FWD_DECLARE
hipError_t launch_fwd_f32_f32x2(const FwdArgs& a, int P, int flags, int block, hipStream_t stream);
hipError_t launch_fwd_bf16_f32x2(const FwdArgs& a, int P, int flags, int block, hipStream_t stream);

// state = (x, var_init, 1) for both models from frame 0 (uses frames, the
// state planes, H, W, row_stride, var_init)
hipError_t launch_init(const FwdArgs& a, int in_dtype, int acc, hipStream_t stream);

}  // namespace dsgm
