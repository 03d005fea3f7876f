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

// ---------------------------------------------------------------- structured video
constexpr int kRects = 6;
constexpr uint64_t kStreamVideoBg = 11, kStreamVideoNoise = 12, kStreamVideoRects = 13;
constexpr int64_t kLightStep = 4;

__host__ __device__ inline int64_t below(uint64_t k, uint64_t n) {
  return int64_t(((k >> 32) * n) >> 32);
}

__device__ inline int64_t pmod(int64_t a, int64_t m) {
  const int64_t r = a % m;
  return r < 0 ? r + m : r;
}

struct VideoArgs {
  void* dst;
  int64_t T, H, W, rs, fs, n;
  uint64_t key_bg, key_noise;
  int64_t rect[kRects][7];  // top0, left0, height, width, vy, vx, level
  int32_t dtype;
};

__global__ void video_kernel(const VideoArgs a) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  const int64_t hw = a.H * a.W;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < a.n; i += stride) {
    const int64_t t = i / hw, p = i - t * hw, h = p / a.W, w = p - h * a.W;
    int64_t level = below(draw(a.key_bg, uint64_t(p)), 161) - 80 + (t >= a.T / 2 ? kLightStep : 0);
    for (int r = 0; r < kRects; ++r) {
      const int64_t top = pmod(a.rect[r][0] + a.rect[r][4] * t, a.H);
      const int64_t left = pmod(a.rect[r][1] + a.rect[r][5] * t, a.W);
      if (pmod(h - top, a.H) < a.rect[r][2] && pmod(w - left, a.W) < a.rect[r][3]) level = a.rect[r][6];
    }
    int64_t s = 0;
    for (int j = 0; j < 3; ++j) {
      const uint64_t k = draw(a.key_noise, uint64_t(i) * 3 + j);
      for (int c = 0; c < 4; ++c) s += int64_t((k >> (16 * c)) & 0xFFFF);
    }
    int64_t q = level + (((s - 393210) * 3 + 32768) >> 16);
    q = q < -128 ? -128 : (q > 127 ? 127 : q);
    const int64_t o = t * a.fs + h * a.rs + w;
    const float v = float(q) * 0x1p-7f;  // exact: at most 8 significant bits
    if (a.dtype == SYNTH_F64)
      static_cast<double*>(a.dst)[o] = double(v);
    else if (a.dtype == SYNTH_F32)
      static_cast<float*>(a.dst)[o] = v;
    else
      static_cast<uint16_t*>(a.dst)[o] = uint16_t(__float_as_uint(v) >> 16);
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

int synth_video(void* dst, int32_t dtype, int64_t T, int64_t H, int64_t W, int64_t row_stride,
                int64_t frame_stride, uint64_t seed, hipStream_t stream) {
  if (T < 0 || H < 0 || W < 0 || row_stride < W || (T > 1 && frame_stride < (H - 1) * row_stride + W))
    return -1;
  if (dtype < SYNTH_F64 || dtype > SYNTH_BF16 || H >= (int64_t(1) << 31) || W >= (int64_t(1) << 31))
    return -1;
  const int64_t n = T * H * W;
  if (n == 0) return 0;
  if (!dst) return -1;
  VideoArgs a{};
  a.dst = dst;
  a.T = T;
  a.H = H;
  a.W = W;
  a.rs = row_stride;
  a.fs = frame_stride;
  a.n = n;
  a.key_bg = stream_key(seed, kStreamVideoBg);
  a.key_noise = stream_key(seed, kStreamVideoNoise);
  const uint64_t kr = stream_key(seed, kStreamVideoRects);
  for (int r = 0; r < kRects; ++r) {
    uint64_t k[7];
    for (int j = 0; j < 7; ++j) k[j] = mix64(kr + (uint64_t(8 * r + j) + 1) * kGamma);
    a.rect[r][0] = below(k[0], uint64_t(H));
    a.rect[r][1] = below(k[1], uint64_t(W));
    a.rect[r][2] = H / 16 + below(k[2], uint64_t(H / 8 + 1));
    a.rect[r][3] = W / 16 + below(k[3], uint64_t(W / 8 + 1));
    a.rect[r][4] = below(k[4], 7) - 3;
    a.rect[r][5] = below(k[5], 9) - 4;
    a.rect[r][6] = below(k[6], 256) - 128;
  }
  a.dtype = dtype;
  hipLaunchKernelGGL(video_kernel, dim3(grid_for(n)), dim3(256), 0, stream, a);
  return hipGetLastError() == hipSuccess ? 0 : -6;
}

}  // extern "C"
