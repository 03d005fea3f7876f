// dsgm_fwd_bf16_f32x2.hip -- forward kernels for bfloat16 frames, compensated
// single-precision (f32x2) state, float bg output (internal).
#include "dsgm_fwd_impl.h"

namespace dsgm {

DSGM_FWD_INSTANTIATE_SINGLE(bf16_t, f32x2, float, bf16_f32x2)

}  // namespace dsgm
