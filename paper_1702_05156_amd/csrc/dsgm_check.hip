// dsgm_check.hip -- counting the non-finite intensities of a frame sequence
// (internal).
//
// The update is defined for finite intensities only (with a NaN or an
// infinity the IEEE comparisons decide the branches).  This pass lets a
// caller check its input first: every lane counts the NaN and infinite
// elements of the rows it visits, the wavefront sums its lanes' counts with
// butterfly shuffles, and one lane per wavefront adds the sum to a 64-bit
// counter.  The counter is cleared by a one-lane kernel in the same stream (no
// memset), so the pair can be captured into a graph; integer addition makes
// the count exact and independent of the order.
#include <algorithm>

#include "dsgm_ext.h"

namespace dsgm {

namespace {

__device__ __forceinline__ bool nonfinite(double v) { return !__builtin_isfinite(v); }
__device__ __forceinline__ bool nonfinite(float v) { return !__builtin_isfinite(v); }
__device__ __forceinline__ bool nonfinite(bf16_t v) { return (v.bits & 0x7F80u) == 0x7F80u; }
__device__ __forceinline__ bool nonfinite(uint8_t) { return false; }

__global__ void count_clear(unsigned long long* count) {
  if (threadIdx.x == 0) count[0] = 0ull;
}

// rows (t, h) of the sequence, grid-stride over rows, lanes over columns
template <typename In>
__global__ void __launch_bounds__(256) count_nonfinite_kernel(const In* frames, int64_t T, int64_t H,
                                                             int64_t W, int64_t row_stride,
                                                             int64_t frame_stride,
                                                             unsigned long long* count) {
  unsigned n = 0;
  const int64_t rows = T * H;
  for (int64_t row = blockIdx.x; row < rows; row += gridDim.x) {
    const int64_t t = row / H, h = row - t * H;
    const In* p = frames + t * frame_stride + h * row_stride;
    for (int64_t c = threadIdx.x; c < W; c += blockDim.x) n += nonfinite(p[c]) ? 1u : 0u;
  }
  for (int off = 32; off > 0; off >>= 1) n += __shfl_xor(n, off, 64);
  if ((threadIdx.x & 63) == 0 && n) atomicAdd(count, (unsigned long long)n);
}

template <typename In>
hipError_t launch_t(const void* frames, const CountArgs& a, hipStream_t stream) {
  const int64_t rows = a.T * a.H;
  hipLaunchKernelGGL(count_clear, dim3(1), dim3(64), 0, stream, a.count);
  if (rows == 0 || a.W == 0) return hipGetLastError();
  const dim3 grid{uint32_t(std::min<int64_t>(rows, 8192)), 1, 1}, block{256, 1, 1};
  hipLaunchKernelGGL((count_nonfinite_kernel<In>), grid, block, 0, stream,
                     static_cast<const In*>(frames), a.T, a.H, a.W, a.row_stride, a.frame_stride,
                     a.count);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_count_nonfinite(const void* frames, int in_dtype, const CountArgs& a,
                                  hipStream_t stream) {
  switch (in_dtype) {
    case 0: return launch_t<double>(frames, a, stream);
    case 1: return launch_t<float>(frames, a, stream);
    case 2: return launch_t<bf16_t>(frames, a, stream);
    case 3: return launch_t<uint8_t>(frames, a, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace dsgm
