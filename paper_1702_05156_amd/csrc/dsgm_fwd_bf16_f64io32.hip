// dsgm_fwd_bf16_f64io32.hip -- forward kernels for bf16_t frames, double state,
// float bg output (internal).
#include "dsgm_fwd_impl.h"

namespace dsgm {

DSGM_FWD_INSTANTIATE(bf16_t, double, float, bf16_f64io32)

}  // namespace dsgm
