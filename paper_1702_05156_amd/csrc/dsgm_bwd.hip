// dsgm_bwd.hip -- checkpointed adjoint of the DSGM update (internal).
//
// One lane owns one pixel.  The frames are cut into segments of K frames whose
// starting states the forward pass stored (checkpoints).  Segments are
// processed from the last to the first.  A segment is replayed in chunks of at
// most KC frames (KC is the compile-time tape length): for the last unprocessed
// chunk the lane reloads the segment's checkpoint, runs the forward step without
// outputs up to the chunk, then over the chunk while recording a tape in
// registers -- per frame the blend's d = m' - x and a 16-bit word holding the
// table slot, hitA and swap -- and finally sweeps the chunk backwards, reading
// the upstream gradient of bg and writing the gradient of the frame.  All of a
// chunk's frame loads are issued before its replay and its gradient loads
// before its sweep (with FP64 state during the replay, last frame first, the
// order the sweep reads them), so their HBM latency overlaps.  With K <= KC
// each frame is replayed once; longer segments replay a prefix per chunk.
//
// The per-pixel contribution to d/d(var_init) is accumulated in FP64 and
// written to the workspace; reduce_pass1/2 then add the H*W contributions in a
// fixed order with compensated (two-sum) arithmetic, so the scalar is
// reproducible run to run and independent of the backward's launch shape.
#include <type_traits>

#include "dsgm_internal.h"

namespace dsgm {

namespace {

// With FP32 state the kernel is compiled for at least 4 waves per SIMD (at most
// 128 VGPRs), which fits without spills once the upstream gradients are loaded
// in two halves (below): BF16 frames ran 4 % faster than at 3 waves, FP32
// frames the same.  FP64 state keeps the compiler's choice: its tape alone
// takes 64 VGPRs, and neither the split loads nor 3 waves per SIMD (which
// spill) were faster.
template <typename In, typename Acc, typename Io, int KC, bool HAS_GBG, bool HAS_GST>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(Acc) == 4 ? 4 : 1)))
bwd_kernel(const BwdArgs a) {
  __shared__ TableEntry<Acc> tbl[TABLE_SIZE];
  for (int i = threadIdx.x; i < TABLE_SIZE; i += blockDim.x)
    tbl[i] = make_entry<Acc>(i, a.weight_rule, a.age_max, Acc(a.var_init));
  __syncthreads();

  const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= a.H * a.W) return;
  const int64_t h = g / a.W;
  const int64_t w = g - h * a.W;
  const uint32_t foff = uint32_t(h * a.row_stride + w);  // < 2^31 elements (host check)
  const uint32_t off_in = foff * uint32_t(sizeof(In));
  const uint32_t off_io = foff * uint32_t(sizeof(Io));

  const StepConsts<Acc> k =
      step_consts<Acc>(a.theta_s, a.theta_d, a.var_init, a.var_floor, a.mask_floor);

  const char* __restrict__ frames = static_cast<const char*>(a.frames);
  const char* __restrict__ gbg = static_cast<const char*>(a.grad_bg);
  char* __restrict__ gfr = static_cast<char*>(a.grad_frames);
  const char* __restrict__ ck = static_cast<const char*>(a.ckpt);
  const int64_t fs_in = a.frame_stride * int64_t(sizeof(In));
  const int64_t fs_io = a.frame_stride * int64_t(sizeof(Io));

  auto x_at = [&](int64_t t) {
    return to_acc<In, Acc>(*reinterpret_cast<const In*>(frames + t * fs_in + off_in));
  };

  Adjoint<Acc> adj;
  adj.gvi = 0.0;
  if (HAS_GST) {
    adj.gmA = Acc(static_cast<const Io*>(a.gst_mean_a)[g]);
    adj.gvA = Acc(static_cast<const Io*>(a.gst_var_a)[g]);
    adj.gmC = Acc(static_cast<const Io*>(a.gst_mean_c)[g]);
    adj.gvC = Acc(static_cast<const Io*>(a.gst_var_c)[g]);
  } else {
    adj.gmA = adj.gvA = adj.gmC = adj.gvC = Acc(0);
  }

  const int64_t T = a.T, K = a.ckpt_every;
  const int64_t nseg = geom::n_segments(T, K);

  // One chunk of `len` <= KC frames starting at c0, from state s: all of its
  // frame loads are issued before the taped replay, all of its upstream bg
  // gradient loads before the reverse sweep (FULL chunks need no per-frame
  // guard).
  auto chunk = [&](Model<Acc> s, const int64_t c0, const int len, auto full_tag) {
    constexpr bool FULL = decltype(full_tag)::value;
    // frames and upstream gradients are held in their storage types (half the
    // registers of FP64 when the arrays are FP32) and widened at use
    In xs[KC];
    Io gb[KC];
#pragma unroll
    for (int i = 0; i < KC; ++i)
      if (FULL || i < len) xs[i] = *reinterpret_cast<const In*>(frames + (c0 + i) * fs_in + off_in);
    // the upstream gradients are requested in the order the sweep uses them,
    // last frame first; with FP32 state those of frames [LATE, KC) after the
    // replay and [0, LATE) once the sweep reaches frame LATE - 1 (fewer
    // registers live)
    constexpr int LATE = sizeof(Acc) == 4 ? KC / 2 : 0;
    auto load_gb = [&](const int j) {
      gb[j] = Io(0);
      if (HAS_GBG && (FULL || j < len))
        gb[j] = *reinterpret_cast<const Io*>(gbg + (c0 + j) * fs_io + off_io);
    };
    Acc tape_d[KC];
    uint32_t tape_m[(KC + 1) / 2];
#pragma unroll
    for (int i = 0; i < KC; ++i) {
      if (FULL || i < len) {
        const StepRecord<Acc> r = step_rec<Acc, false>(s, to_acc<In, Acc>(xs[i]), k, tbl);
        tape_d[i] = r.d;
        const uint32_t m = uint32_t(r.idx) | (r.hitA ? 0x200u : 0u) | (r.swap ? 0x400u : 0u);
        if (i % 2 == 0)
          tape_m[i / 2] = m;
        else
          tape_m[i / 2] |= m << 16;
      }
      // FP64 state: frame i's value is dead now and the gradient the sweep
      // needs i-th goes out, so the loads overlap the rest of the replay
      if constexpr (LATE == 0) load_gb(KC - 1 - i);
    }
    if constexpr (LATE > 0) {
#pragma unroll
      for (int j = KC - 1; j >= LATE; --j) load_gb(j);
    }
#pragma unroll
    for (int i = KC - 1; i >= 0; --i) {
      if constexpr (LATE > 0) {
        if (i == LATE - 1) {
#pragma unroll
          for (int j = LATE - 1; j >= 0; --j) load_gb(j);
        }
      }
      if (FULL || i < len) {
        const uint32_t m = (tape_m[i / 2] >> (16 * (i % 2))) & 0xFFFFu;
        const Acc gx = reverse_step<Acc, HAS_GBG>(adj, Acc(gb[i]), tape_d[i], int(m & 0x1FFu),
                                                  (m & 0x200u) != 0, (m & 0x400u) != 0, tbl);
        *reinterpret_cast<Io*>(gfr + (c0 + i) * fs_io + off_io) = Io(gx);  // rounded once
      }
    }
  };

  for (int64_t seg = nseg - 1; seg >= 0; --seg) {
    const geom::Range sg = geom::segment(seg, T, K);
    const int64_t s0 = sg.lo;
    const char* base = ck + seg * a.ckpt_slot_bytes;
    const int64_t nchunk = geom::n_chunks(sg, KC);
    for (int64_t c = nchunk - 1; c >= 0; --c) {
      const geom::Range ch = geom::chunk(sg, c, KC);
      const int64_t c0 = ch.lo, c1 = ch.hi;
      Model<Acc> s;
      s.mA = reinterpret_cast<const Acc*>(base + 0 * a.ckpt_fplane)[g];
      s.vA = reinterpret_cast<const Acc*>(base + 1 * a.ckpt_fplane)[g];
      s.mC = reinterpret_cast<const Acc*>(base + 2 * a.ckpt_fplane)[g];
      s.vC = reinterpret_cast<const Acc*>(base + 3 * a.ckpt_fplane)[g];
      s.aA = reinterpret_cast<const uint8_t*>(base + 4 * a.ckpt_fplane)[g];
      s.aC = reinterpret_cast<const uint8_t*>(base + 4 * a.ckpt_fplane + a.ckpt_aplane)[g];
      // replay up to the chunk (only when segments are longer than the tape),
      // eight frames of loads at a time
      int64_t t = s0;
      for (; t + 8 <= c0; t += 8) {
        Acc xr[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) xr[i] = x_at(t + i);
#pragma unroll
        for (int i = 0; i < 8; ++i) (void)step_rec<Acc, false>(s, xr[i], k, tbl);
      }
      for (; t < c0; ++t) (void)step_rec<Acc, false>(s, x_at(t), k, tbl);
      const int len = int(c1 - c0);
      if (len == KC)
        chunk(s, c0, len, std::true_type{});
      else
        chunk(s, c0, len, std::false_type{});
    }
  }
  static_cast<Io*>(a.gs0_mean_a)[g] = Io(adj.gmA);
  static_cast<Io*>(a.gs0_var_a)[g] = Io(adj.gvA);
  static_cast<Io*>(a.gs0_mean_c)[g] = Io(adj.gmC);
  static_cast<Io*>(a.gs0_var_c)[g] = Io(adj.gvC);
  a.gvi_px[g] = adj.gvi;
}

// ------------------------------------------------------------ compensated sum
// Sum2 of Ogita, Rump and Oishi (2005): every addition is an error-free
// two-sum, the rounding errors are summed separately, and (s, c) pairs are
// combined the same way; the result is as accurate as if computed in twice the
// working precision.  Fixed order throughout: deterministic.
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

struct Pair {
  double s, c;
};

__device__ __forceinline__ Pair pair_add(Pair x, Pair y) {
  Pair r;
  double e;
  two_sum(x.s, y.s, r.s, e);
  r.c = (x.c + y.c) + e;
  return r;
}

constexpr int RED_THREADS = 256;
constexpr int RED_BLOCKS = geom::REDUCE_BLOCKS;
static_assert(RED_BLOCKS == RED_THREADS, "pass 2 gives one pair to each thread");

// pass 1: block b sums the contiguous chunk b of the input; thread i takes
// elements i, i + 256, ... of the chunk; then a fixed binary tree in LDS
__global__ void __launch_bounds__(RED_THREADS) reduce_pass1(const double* __restrict__ x, int64_t n,
                                                             double* __restrict__ partial) {
  __shared__ Pair sh[RED_THREADS];
  const int64_t chunk = (n + RED_BLOCKS - 1) / RED_BLOCKS;
  const int64_t lo = int64_t(blockIdx.x) * chunk;
  const int64_t hi = lo + chunk < n ? lo + chunk : n;
  Pair p{0.0, 0.0};
  for (int64_t i = lo + threadIdx.x; i < hi; i += RED_THREADS) {
    double e;
    two_sum(p.s, x[i], p.s, e);
    p.c += e;
  }
  sh[threadIdx.x] = p;
  __syncthreads();
  for (int w = RED_THREADS / 2; w > 0; w /= 2) {
    if (int(threadIdx.x) < w) sh[threadIdx.x] = pair_add(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = sh[0].s;
    partial[2 * blockIdx.x + 1] = sh[0].c;
  }
}

// pass 2: one block combines the RED_BLOCKS pairs in the same fixed tree
__global__ void __launch_bounds__(RED_THREADS) reduce_pass2(const double* __restrict__ partial,
                                                             double* __restrict__ out) {
  __shared__ Pair sh[RED_THREADS];
  sh[threadIdx.x] = Pair{partial[2 * threadIdx.x], partial[2 * threadIdx.x + 1]};
  __syncthreads();
  for (int w = RED_THREADS / 2; w > 0; w /= 2) {
    if (int(threadIdx.x) < w) sh[threadIdx.x] = pair_add(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0].s + sh[0].c;
}

template <typename In, typename Acc, typename Io, int KC>
hipError_t launch_bwd_k(const BwdArgs& a, hipStream_t stream) {
  const int block = 256;
  const int64_t grid = (a.H * a.W + block - 1) / block;
  const bool gb = a.grad_bg != nullptr, gs = a.gst_mean_a != nullptr;
  if (gb && gs)
    hipLaunchKernelGGL((bwd_kernel<In, Acc, Io, KC, true, true>), dim3(uint32_t(grid)), dim3(block), 0, stream, a);
  else if (gb)
    hipLaunchKernelGGL((bwd_kernel<In, Acc, Io, KC, true, false>), dim3(uint32_t(grid)), dim3(block), 0, stream, a);
  else if (gs)
    hipLaunchKernelGGL((bwd_kernel<In, Acc, Io, KC, false, true>), dim3(uint32_t(grid)), dim3(block), 0, stream, a);
  else
    hipLaunchKernelGGL((bwd_kernel<In, Acc, Io, KC, false, false>), dim3(uint32_t(grid)), dim3(block), 0, stream, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_reduce(const double* x, int64_t n, double* partial, double* out,
                         hipStream_t stream) {
  hipLaunchKernelGGL(reduce_pass1, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, stream, x, n, partial);
  hipLaunchKernelGGL(reduce_pass2, dim3(1), dim3(RED_THREADS), 0, stream, partial, out);
  return hipGetLastError();
}

hipError_t launch_backward(const BwdArgs& a, int in_dtype, int acc, hipStream_t stream) {
  if (acc == 0) {
    if (in_dtype == 0) return launch_bwd_k<double, double, double, 16>(a, stream);
    if (in_dtype == 1) return launch_bwd_k<float, double, double, 16>(a, stream);
    if (in_dtype == 2) return launch_bwd_k<bf16_t, double, double, 16>(a, stream);
  } else if (acc == 1) {
    if (in_dtype == 1) return launch_bwd_k<float, float, float, 32>(a, stream);
    if (in_dtype == 2) return launch_bwd_k<bf16_t, float, float, 32>(a, stream);
  } else if (acc == 2) {
    if (in_dtype == 1) return launch_bwd_k<float, double, float, 32>(a, stream);
    if (in_dtype == 2) return launch_bwd_k<bf16_t, double, float, 32>(a, stream);
  } else if (acc == 4) {
    if (in_dtype == 1) return launch_bwd_k<float, f32x2, float, 32>(a, stream);
    if (in_dtype == 2) return launch_bwd_k<bf16_t, f32x2, float, 32>(a, stream);
  }
  return hipErrorInvalidValue;
}

}  // namespace dsgm
