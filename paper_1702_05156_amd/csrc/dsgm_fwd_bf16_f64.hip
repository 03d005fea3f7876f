// dsgm_fwd_bf16_f64.hip -- forward kernels for bf16_t frames, double state (internal).
#include "dsgm_fwd_impl.h"

namespace dsgm {

DSGM_FWD_INSTANTIATE(bf16_t, double, double, bf16_f64)

}  // namespace dsgm
