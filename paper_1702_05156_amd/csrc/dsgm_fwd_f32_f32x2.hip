// dsgm_fwd_f32_f32x2.hip -- forward kernels for float frames, compensated
// single-precision (f32x2) state, float bg output (internal).
#include "dsgm_fwd_impl.h"

namespace dsgm {

DSGM_FWD_INSTANTIATE_SINGLE(float, f32x2, float, f32_f32x2)

}  // namespace dsgm
