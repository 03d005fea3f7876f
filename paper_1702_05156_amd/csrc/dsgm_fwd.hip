// dsgm_fwd.hip -- time-fused forward kernel of the DSGM update (internal).
//
// Decomposition (the paper's Sec. 3.4 assigns one thread per pixel; here one
// lane owns P horizontally adjacent pixels of one row for the whole sequence):
// the lane loads its pixels' six state values once, keeps them in registers,
// walks the T frames, and stores the state once at the end.  Per frame it reads
// P intensities (one aligned vector load; a wavefront reads 64*P consecutive
// pixels) and writes P mask bytes (one aligned store), optionally bg (the
// apparent mean) and the decision codes.  Every wavefront touches contiguous
// memory; nothing is shared between lanes, so there is no LDS traffic except
// the 257-entry update table.
#include "dsgm_internal.h"

namespace dsgm {

namespace {

template <int B>
struct Raw;
template <>
struct Raw<1> { using type = uint8_t; };
template <>
struct Raw<2> { using type = uint16_t; };
template <>
struct Raw<4> { using type = uint32_t; };
template <>
struct Raw<8> { using type = uint32_t __attribute__((ext_vector_type(2))); };
template <>
struct Raw<16> { using type = uint32_t __attribute__((ext_vector_type(4))); };

// streaming (nontemporal) vector load/store of P elements; 32-byte vectors are
// moved as two 16-byte halves
template <typename X, int P>
__device__ __forceinline__ Vec<X, P> ld_stream(const X* p) {
  constexpr int B = int(sizeof(X)) * P;
  if constexpr (B <= 16) {
    using R = typename Raw<B>::type;
    return __builtin_bit_cast(Vec<X, P>, __builtin_nontemporal_load(reinterpret_cast<const R*>(p)));
  } else {
    using R = typename Raw<16>::type;
    struct Two { R lo, hi; } t;
    t.lo = __builtin_nontemporal_load(reinterpret_cast<const R*>(p));
    t.hi = __builtin_nontemporal_load(reinterpret_cast<const R*>(p) + 1);
    return __builtin_bit_cast(Vec<X, P>, t);
  }
}

template <typename X, int P>
__device__ __forceinline__ void st_stream(X* p, const Vec<X, P>& v) {
  constexpr int B = int(sizeof(X)) * P;
  if constexpr (B <= 16) {
    using R = typename Raw<B>::type;
    __builtin_nontemporal_store(__builtin_bit_cast(R, v), reinterpret_cast<R*>(p));
  } else {
    using R = typename Raw<16>::type;
    struct Two { R lo, hi; };
    const Two t = __builtin_bit_cast(Two, v);
    __builtin_nontemporal_store(t.lo, reinterpret_cast<R*>(p));
    __builtin_nontemporal_store(t.hi, reinterpret_cast<R*>(p) + 1);
  }
}

template <typename In, typename Acc, int P, int U, bool BG, bool CODES>
__global__ void __launch_bounds__(256) fwd_kernel(const FwdArgs a) {
  __shared__ TableEntry<Acc> tbl[TABLE_SIZE];
  for (int i = threadIdx.x; i < TABLE_SIZE; i += blockDim.x)
    tbl[i] = make_entry<Acc>(i, a.weight_rule, a.age_max, Acc(a.var_init));
  __syncthreads();

  const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= a.ngroups) return;
  const int64_t h = g / a.groups_per_row;
  const int64_t w0 = (g - h * a.groups_per_row) * P;
  const uint32_t foff = uint32_t(h * a.row_stride + w0);  // < 2^31 elements (host check)
  const int64_t soff = h * a.W + w0;

  StepConsts<Acc> k;
  k.theta_s = Acc(a.theta_s);
  k.theta_d = Acc(a.theta_d);
  k.var_init = Acc(a.var_init);
  k.ts_vf = k.theta_s * Acc(a.var_floor);
  k.td_mf = k.theta_d * Acc(a.mask_floor);
  k.printed = a.mask_rule == 1;

  Acc* mA_p = static_cast<Acc*>(a.mean_a) + soff;
  Acc* vA_p = static_cast<Acc*>(a.var_a) + soff;
  Acc* mC_p = static_cast<Acc*>(a.mean_c) + soff;
  Acc* vC_p = static_cast<Acc*>(a.var_c) + soff;
  uint8_t* aA_p = a.age_a + soff;
  uint8_t* aC_p = a.age_c + soff;

  Model<Acc> s[P];
  {
    const Vec<Acc, P> mA = *reinterpret_cast<const Vec<Acc, P>*>(mA_p);
    const Vec<Acc, P> vA = *reinterpret_cast<const Vec<Acc, P>*>(vA_p);
    const Vec<Acc, P> mC = *reinterpret_cast<const Vec<Acc, P>*>(mC_p);
    const Vec<Acc, P> vC = *reinterpret_cast<const Vec<Acc, P>*>(vC_p);
    const Vec<uint8_t, P> aA = *reinterpret_cast<const Vec<uint8_t, P>*>(aA_p);
    const Vec<uint8_t, P> aC = *reinterpret_cast<const Vec<uint8_t, P>*>(aC_p);
#pragma unroll
    for (int j = 0; j < P; ++j) {
      s[j].mA = mA.v[j];
      s[j].vA = vA.v[j];
      s[j].mC = mC.v[j];
      s[j].vC = vC.v[j];
      s[j].aA = aA.v[j];
      s[j].aC = aC.v[j];
    }
  }

  // per frame: a uniform base pointer (scalar registers) plus a 32-bit
  // per-lane byte offset, so loads and stores use the saddr+voffset form
  const char* __restrict__ frames = static_cast<const char*>(a.frames);
  char* __restrict__ masks = reinterpret_cast<char*>(a.masks);
  char* __restrict__ bg = static_cast<char*>(a.bg);
  char* __restrict__ codes = reinterpret_cast<char*>(a.codes);
  const int64_t T = a.T, fs = a.frame_stride;
  const uint32_t off_in = foff * uint32_t(sizeof(In));
  const uint32_t off_acc = foff * uint32_t(sizeof(Acc));

  // checkpoints: state before frames 0, K, 2K, ...
  char* ck = static_cast<char*>(a.ckpt);
  int ck_left = 0;

  auto do_frame = [&](const Vec<In, P>& xin, int64_t t) {
    if (ck != nullptr) {
      if (ck_left == 0) {
        char* base = ck + (t / a.ckpt_every) * a.ckpt_slot_bytes;
        Vec<Acc, P> mA, vA, mC, vC;
        Vec<uint8_t, P> aA, aC;
#pragma unroll
        for (int j = 0; j < P; ++j) {
          mA.v[j] = s[j].mA;
          vA.v[j] = s[j].vA;
          mC.v[j] = s[j].mC;
          vC.v[j] = s[j].vC;
          aA.v[j] = uint8_t(s[j].aA);
          aC.v[j] = uint8_t(s[j].aC);
        }
        *reinterpret_cast<Vec<Acc, P>*>(base + 0 * a.ckpt_fplane + soff * sizeof(Acc)) = mA;
        *reinterpret_cast<Vec<Acc, P>*>(base + 1 * a.ckpt_fplane + soff * sizeof(Acc)) = vA;
        *reinterpret_cast<Vec<Acc, P>*>(base + 2 * a.ckpt_fplane + soff * sizeof(Acc)) = mC;
        *reinterpret_cast<Vec<Acc, P>*>(base + 3 * a.ckpt_fplane + soff * sizeof(Acc)) = vC;
        *reinterpret_cast<Vec<uint8_t, P>*>(base + 4 * a.ckpt_fplane + soff) = aA;
        *reinterpret_cast<Vec<uint8_t, P>*>(base + 4 * a.ckpt_fplane + a.ckpt_aplane + soff) = aC;
        ck_left = a.ckpt_every;
      }
      --ck_left;
    }
    Vec<uint8_t, P> mk;
    Vec<Acc, P> bgv;
    Vec<uint8_t, P> cd;
#pragma unroll
    for (int j = 0; j < P; ++j) {
      unsigned c = 0;
      const bool fg = step<Acc, CODES>(s[j], to_acc<In, Acc>(xin.v[j]), k, tbl, &c);
      mk.v[j] = fg ? uint8_t(255) : uint8_t(0);
      if (BG) bgv.v[j] = s[j].mA;
      if (CODES) cd.v[j] = uint8_t(c);
    }
    const int64_t o = t * fs;
    st_stream<uint8_t, P>(reinterpret_cast<uint8_t*>(masks + o + foff), mk);
    if (BG) st_stream<Acc, P>(reinterpret_cast<Acc*>(bg + o * int64_t(sizeof(Acc)) + off_acc), bgv);
    if (CODES) *reinterpret_cast<Vec<uint8_t, P>*>(codes + o + foff) = cd;
  };

  int64_t t = 0;
  // full batches of U frames: U loads in flight, then U steps
  for (; t + U <= T; t += U) {
    Vec<In, P> xb[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
      xb[u] = ld_stream<In, P>(
          reinterpret_cast<const In*>(frames + (t + u) * fs * int64_t(sizeof(In)) + off_in));
#pragma unroll
    for (int u = 0; u < U; ++u) do_frame(xb[u], t + u);
  }
  for (; t < T; ++t)
    do_frame(ld_stream<In, P>(reinterpret_cast<const In*>(frames + t * fs * int64_t(sizeof(In)) + off_in)), t);

  {
    Vec<Acc, P> mA, vA, mC, vC;
    Vec<uint8_t, P> aA, aC;
#pragma unroll
    for (int j = 0; j < P; ++j) {
      mA.v[j] = s[j].mA;
      vA.v[j] = s[j].vA;
      mC.v[j] = s[j].mC;
      vC.v[j] = s[j].vC;
      aA.v[j] = uint8_t(s[j].aA);
      aC.v[j] = uint8_t(s[j].aC);
    }
    *reinterpret_cast<Vec<Acc, P>*>(mA_p) = mA;
    *reinterpret_cast<Vec<Acc, P>*>(vA_p) = vA;
    *reinterpret_cast<Vec<Acc, P>*>(mC_p) = mC;
    *reinterpret_cast<Vec<Acc, P>*>(vC_p) = vC;
    *reinterpret_cast<Vec<uint8_t, P>*>(aA_p) = aA;
    *reinterpret_cast<Vec<uint8_t, P>*>(aC_p) = aC;
  }
}

template <typename In, typename Acc, int P, bool BG, bool CODES>
hipError_t launch_p(const FwdArgs& a, int block, hipStream_t stream) {
  constexpr int U = 4;
  const int64_t grid = (a.ngroups + block - 1) / block;
  hipLaunchKernelGGL((fwd_kernel<In, Acc, P, U, BG, CODES>), dim3(uint32_t(grid)), dim3(block), 0,
                     stream, a);
  return hipGetLastError();
}

template <typename In, typename Acc>
hipError_t launch_t(const FwdArgs& a, int P, int block, hipStream_t stream) {
  const bool bg = a.bg != nullptr, cd = a.codes != nullptr;
#define DSGM_FWD_CASE(PP)                                                   \
  if (P == PP) {                                                            \
    if (bg && cd) return launch_p<In, Acc, PP, true, true>(a, block, stream);   \
    if (bg) return launch_p<In, Acc, PP, true, false>(a, block, stream);        \
    if (cd) return launch_p<In, Acc, PP, false, true>(a, block, stream);        \
    return launch_p<In, Acc, PP, false, false>(a, block, stream);               \
  }
  DSGM_FWD_CASE(1)
  DSGM_FWD_CASE(2)
  DSGM_FWD_CASE(4)
#undef DSGM_FWD_CASE
  return hipErrorInvalidValue;
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
  if (acc == 0) {
    if (in_dtype == 0) return launch_init_t<double, double>(a, stream);
    if (in_dtype == 1) return launch_init_t<float, double>(a, stream);
    if (in_dtype == 2) return launch_init_t<bf16_t, double>(a, stream);
  } else if (acc == 1) {
    if (in_dtype == 1) return launch_init_t<float, float>(a, stream);
    if (in_dtype == 2) return launch_init_t<bf16_t, float>(a, stream);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_forward(const FwdArgs& a, int in_dtype, int acc, int P, int block,
                          hipStream_t stream) {
  if (acc == 0) {
    if (in_dtype == 0) return launch_t<double, double>(a, P, block, stream);
    if (in_dtype == 1) return launch_t<float, double>(a, P, block, stream);
    if (in_dtype == 2) return launch_t<bf16_t, double>(a, P, block, stream);
  } else if (acc == 1) {
    if (in_dtype == 1) return launch_t<float, float>(a, P, block, stream);
    if (in_dtype == 2) return launch_t<bf16_t, float>(a, P, block, stream);
  }
  return hipErrorInvalidValue;
}

}  // namespace dsgm
