// synth.hip -- device twin of synth/__init__.py (counter-based SplitMix64).
#include <stdint.h>

#include <hip/hip_runtime.h>

#include "synth.h"

namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

__host__ __device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

uint64_t stream_key(uint64_t seed, uint64_t stream_id) {
  const uint64_t k0 = mix64(seed + kGamma);
  return mix64(k0 + (stream_id + 1) * kGamma);
}

__device__ inline uint64_t draw(uint64_t key, uint64_t i) { return mix64(key + (i + 1) * kGamma); }

struct FillArgs {
  void* dst;
  int64_t T, H, W, rs, fs, n;
  uint64_t key;
  int32_t dtype, kind;
};

__device__ inline double uniform_value(uint64_t k, int dtype) {
  if (dtype == SYNTH_F64) return double(k >> 11) * 0x1p-52 - 1.0;
  if (dtype == SYNTH_F32) return double(k >> 40) * 0x1p-23 - 1.0;
  return double(k >> 56) * 0x1p-7 - 1.0;
}

__global__ void fill_kernel(const FillArgs a) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < a.n; i += stride) {
    double v;
    if (a.kind == SYNTH_NORMAL) {
      int64_t s = 0;
      for (int j = 0; j < 3; ++j) {
        const uint64_t k = draw(a.key, uint64_t(i) * 3 + j);
        for (int c = 0; c < 4; ++c) s += int64_t((k >> (16 * c)) & 0xFFFF);
      }
      v = double(s - 393210) * 0x1p-16;
    } else {
      v = uniform_value(draw(a.key, uint64_t(i)), a.dtype);
      if (a.kind == SYNTH_ABS_UNIFORM) v = v < 0 ? -v : v;
    }
    const int64_t hw = a.H * a.W;
    const int64_t t = i / hw, r = i - t * hw, h = r / a.W, w = r - h * a.W;
    const int64_t o = t * a.fs + h * a.rs + w;
    if (a.dtype == SYNTH_F64) {
      static_cast<double*>(a.dst)[o] = v;
    } else if (a.dtype == SYNTH_F32) {
      static_cast<float*>(a.dst)[o] = float(v);  // exact: v lies on the 24-bit grid
    } else {
      static_cast<uint16_t*>(a.dst)[o] = uint16_t(__float_as_uint(float(v)) >> 16);  // exact
    }
  }
}

struct AgeArgs {
  uint8_t* dst;
  int64_t n;
  uint64_t key;
  uint32_t age_max;
};

__global__ void ages_kernel(const AgeArgs a) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < a.n; i += stride) {
    const uint64_t hi = draw(a.key, uint64_t(i)) >> 32;
    a.dst[i] = uint8_t(((hi * a.age_max) >> 32) + 1);
  }
}

int grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  return int(g < 65536 ? (g > 0 ? g : 1) : 65536);
}

}  // namespace

extern "C" {

int synth_fill(void* dst, int32_t dtype, int32_t kind, int64_t T, int64_t H, int64_t W,
               int64_t row_stride, int64_t frame_stride, uint64_t seed, uint64_t stream_id,
               hipStream_t stream) {
  if (T < 0 || H < 0 || W < 0 || row_stride < W || (T > 1 && frame_stride < (H - 1) * row_stride + W))
    return -1;
  if (dtype < SYNTH_F64 || dtype > SYNTH_BF16 || kind < SYNTH_UNIFORM || kind > SYNTH_NORMAL) return -1;
  if (kind == SYNTH_NORMAL && dtype == SYNTH_BF16) return -1;
  const int64_t n = T * H * W;
  if (n == 0) return 0;
  if (!dst) return -1;
  FillArgs a{dst, T, H, W, row_stride, frame_stride, n, stream_key(seed, stream_id), dtype, kind};
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n)), dim3(256), 0, stream, a);
  return hipGetLastError() == hipSuccess ? 0 : -6;
}

int synth_ages(uint8_t* dst, int64_t n, int32_t age_max, uint64_t seed, uint64_t stream_id,
               hipStream_t stream) {
  if (n < 0 || age_max < 1 || age_max > 255) return -1;
  if (n == 0) return 0;
  if (!dst) return -1;
  AgeArgs a{dst, n, stream_key(seed, stream_id), uint32_t(age_max)};
  hipLaunchKernelGGL(ages_kernel, dim3(grid_for(n)), dim3(256), 0, stream, a);
  return hipGetLastError() == hipSuccess ? 0 : -6;
}

}  // extern "C"
