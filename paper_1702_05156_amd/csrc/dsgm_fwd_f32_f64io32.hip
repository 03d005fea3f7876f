// dsgm_fwd_f32_f64io32.hip -- forward kernels for float frames, double state,
// float bg output (internal).
#include "dsgm_fwd_impl.h"

namespace dsgm {

DSGM_FWD_INSTANTIATE(float, double, float, f32_f64io32)

}  // namespace dsgm
