// dsgm_fwd_f32_f32.hip -- forward kernels for float frames, float state (internal).
#include "dsgm_fwd_impl.h"

namespace dsgm {

DSGM_FWD_INSTANTIATE(float, float, float, f32_f32)

}  // namespace dsgm
