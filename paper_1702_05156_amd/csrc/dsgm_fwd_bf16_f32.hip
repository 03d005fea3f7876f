// dsgm_fwd_bf16_f32.hip -- forward kernels for bf16_t frames, float state (internal).
#include "dsgm_fwd_impl.h"

namespace dsgm {

DSGM_FWD_INSTANTIATE(bf16_t, float, float, bf16_f32)

}  // namespace dsgm
