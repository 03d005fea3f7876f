// dsgm_fwd.hip -- dispatch of the forward kernels, the state initialisation
// kernel and the batched launch (internal).  The kernels themselves are in
// dsgm_fwd_impl.h, instantiated by dsgm_fwd_<frames>_<state>.hip.
#include "dsgm_fwd_impl.h"

namespace dsgm {

namespace {

__global__ void counter_reset(unsigned long long* counter) {
  if (threadIdx.x == 0) *counter = 0ull;
}

// clears the count stripes of every instance that has foreground counters
// (one block per instance); a kernel rather than a memset so that the launch
// sequence can be captured into a graph and replayed
__global__ void __launch_bounds__(256) counts_reset(const BatchInst* inst) {
  const BatchInst& I = inst[blockIdx.x];
  if (I.fg_counts == nullptr) return;
  const int64_t n = I.T * COUNT_STRIPES;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) I.stripes[i] = 0u;
}

// adds each instance's stripes into its counters (one block per instance;
// integer sums, exact in any order)
__global__ void __launch_bounds__(256) counts_sum(const BatchInst* inst) {
  const BatchInst& I = inst[blockIdx.x];
  if (I.fg_counts == nullptr) return;
  for (int64_t t = threadIdx.x; t < I.T; t += blockDim.x) {
    uint32_t c = 0u;
    for (int s = 0; s < COUNT_STRIPES; ++s) c += I.stripes[int64_t(s) * I.T + t];
    I.fg_counts[t] = c;
  }
}

template <typename In, typename Acc>
__global__ void __launch_bounds__(256) init_kernel(const FwdArgs a) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.H * a.W) return;
  const int64_t h = i / a.W, w = i - h * a.W;
  const Acc x = to_acc<In, Acc>(static_cast<const In*>(a.frames)[h * a.row_stride + w]);
  static_cast<Acc*>(a.mean_a)[i] = x;
  static_cast<Acc*>(a.mean_c)[i] = x;
  static_cast<Acc*>(a.var_a)[i] = Acc(a.var_init);
  static_cast<Acc*>(a.var_c)[i] = Acc(a.var_init);
  a.age_a[i] = 1;
  a.age_c[i] = 1;
}

template <typename In, typename Acc>
hipError_t launch_init_t(const FwdArgs& a, hipStream_t stream) {
  const int64_t grid = (a.H * a.W + 255) / 256;
  hipLaunchKernelGGL((init_kernel<In, Acc>), dim3(uint32_t(grid)), dim3(256), 0, stream, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_init(const FwdArgs& a, int in_dtype, int acc, hipStream_t stream) {
  if (acc == 0 || acc == 2) {
    if (in_dtype == 0) return launch_init_t<double, double>(a, stream);
    if (in_dtype == 1) return launch_init_t<float, double>(a, stream);
    if (in_dtype == 2) return launch_init_t<bf16_t, double>(a, stream);
  } else if (acc == 1) {
    if (in_dtype == 1) return launch_init_t<float, float>(a, stream);
    if (in_dtype == 2) return launch_init_t<bf16_t, float>(a, stream);
  } else if (acc == 4) {
    if (in_dtype == 1) return launch_init_t<float, f32x2>(a, stream);
    if (in_dtype == 2) return launch_init_t<bf16_t, f32x2>(a, stream);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_forward(const FwdArgs& a, int in_dtype, int acc, int P, int flags, int block,
                          hipStream_t stream) {
  if (acc == 0) {
    if (in_dtype == 0) return launch_fwd_f64_f64(a, P, flags, block, stream);
    if (in_dtype == 1) return launch_fwd_f32_f64(a, P, flags, block, stream);
    if (in_dtype == 2) return launch_fwd_bf16_f64(a, P, flags, block, stream);
  } else if (acc == 1) {
    if (in_dtype == 1) return launch_fwd_f32_f32(a, P, flags, block, stream);
    if (in_dtype == 2) return launch_fwd_bf16_f32(a, P, flags, block, stream);
  } else if (acc == 2) {
    if (in_dtype == 1) return launch_fwd_f32_f64io32(a, P, flags, block, stream);
    if (in_dtype == 2) return launch_fwd_bf16_f64io32(a, P, flags, block, stream);
  } else if (acc == 4) {
    if (in_dtype == 1) return launch_fwd_f32_f32x2(a, P, flags, block, stream);
    if (in_dtype == 2) return launch_fwd_bf16_f32x2(a, P, flags, block, stream);
  }
  return hipErrorInvalidValue;
}

const void* batched_kernel_symbol(int in_dtype, int acc, int P, int flags) {
  if (acc == 0) {
    if (in_dtype == 0) return batched_sym_f64_f64(P, flags);
    if (in_dtype == 1) return batched_sym_f32_f64(P, flags);
    if (in_dtype == 2) return batched_sym_bf16_f64(P, flags);
  } else if (acc == 1) {
    if (in_dtype == 1) return batched_sym_f32_f32(P, flags);
    if (in_dtype == 2) return batched_sym_bf16_f32(P, flags);
  } else if (acc == 2) {
    if (in_dtype == 1) return batched_sym_f32_f64io32(P, flags);
    if (in_dtype == 2) return batched_sym_bf16_f64io32(P, flags);
  }
  return nullptr;
}

hipError_t launch_batched(const BatchArgs& a, int in_dtype, int acc, int P, int flags, int grid,
                          bool counts, hipStream_t stream) {
  const void* fn = batched_kernel_symbol(in_dtype, acc, P, flags);
  if (!fn) return hipErrorInvalidValue;
  hipLaunchKernelGGL(counter_reset, dim3(1), dim3(64), 0, stream, a.counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (counts) {
    hipLaunchKernelGGL(counts_reset, dim3(uint32_t(a.n_inst)), dim3(256), 0, stream, a.inst);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  BatchArgs args = a;
  void* kargs[] = {&args};
  e = hipLaunchKernel(fn, dim3(uint32_t(grid)), dim3(256), kargs, 0, stream);
  if (e != hipSuccess || !counts) return e;
  hipLaunchKernelGGL(counts_sum, dim3(uint32_t(a.n_inst)), dim3(256), 0, stream, a.inst);
  return hipGetLastError();
}

}  // namespace dsgm
