// dsgm_fwd_f64_f64.hip -- forward kernels for double frames, double state (internal).
#include "dsgm_fwd_impl.h"

namespace dsgm {

DSGM_FWD_INSTANTIATE(double, double, double, f64_f64)

}  // namespace dsgm
