// dsgm_fwd_f32_f64.hip -- forward kernels for float frames, double state (internal).
#include "dsgm_fwd_impl.h"

namespace dsgm {

DSGM_FWD_INSTANTIATE(float, double, double, f32_f64)

}  // namespace dsgm
