// dsgm_tune.hip -- the synthetic workload the launch-shape tuner times
// (internal).
//
// The tuner runs the forward on frames of independent intensities, uniform
// over the full range of the frame type; with the default parameters this is
// the workload where lanes of a wavefront disagree most often on the branch
// they take, i.e. the one that separates launch shapes most clearly.  The
// values come from a counter-based integer hash of (seed, index), so a fill is
// reproducible and needs no state.
#include <algorithm>

#include "dsgm_ext.h"

namespace dsgm {

namespace {

// 64-bit finaliser of a counter (xor-shift-multiply rounds), full avalanche
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 33)) * 0xff51afd7ed558ccdull;
  z = (z ^ (z >> 33)) * 0xc4ceb9fe1a85ec53ull;
  return z ^ (z >> 33);
}

__global__ void __launch_bounds__(256) tune_fill_kernel(void* out, int in_dtype, int64_t n,
                                                        uint64_t seed) {
  const int64_t step = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += step) {
    const uint64_t h = mix64(seed * 0x9e3779b97f4a7c15ull + uint64_t(i));
    const double u = double(h >> 11) * 0x1.0p-53;  // [0, 1)
    const double v = 2.0 * u - 1.0;                // [-1, 1)
    switch (in_dtype) {
      case 0: static_cast<double*>(out)[i] = v; break;
      case 1: static_cast<float*>(out)[i] = float(v); break;
      case 2:  // the float's upper half: a value in [-1, 1] as well
        static_cast<bf16_t*>(out)[i] = bf16_t{uint16_t(__float_as_uint(float(v)) >> 16)};
        break;
      default: static_cast<uint8_t*>(out)[i] = uint8_t(h >> 56); break;
    }
  }
}

}  // namespace

hipError_t launch_tune_fill(void* out, int in_dtype, int64_t n, uint64_t seed,
                            hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(tune_fill_kernel, dim3(uint32_t(blocks)), dim3(256), 0, stream, out,
                     in_dtype, n, seed);
  return hipGetLastError();
}

}  // namespace dsgm
