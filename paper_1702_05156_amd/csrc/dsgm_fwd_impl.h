// dsgm_fwd_impl.h -- time-fused forward kernels of the DSGM update (internal;
// included by the per-accumulation-type translation units).
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
//
// fwd_kernel     one instance, one lane per pixel group, grid covers the groups
// batched_kernel many instances, persistent: each wavefront repeatedly takes
//                the next (instance, 64-group tile) item from a device counter;
//                items are ordered longest-first (LPT) by the host planner.
// Optional outputs, checkpoints and the mask rule are compile-time variants so
// that the common kernel carries none of their code.
#pragma once

#include "dsgm_internal.h"

namespace dsgm {

namespace fwd {

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

template <typename Acc>
__device__ __forceinline__ StepConsts<Acc> make_consts(double theta_s, double theta_d,
                                                      double var_init, double var_floor,
                                                      double mask_floor) {
  return step_consts<Acc>(theta_s, theta_d, var_init, var_floor, mask_floor);
}

template <typename Acc>
__device__ __forceinline__ void fill_table(TableEntry<Acc>* tbl, int weight_rule, int age_max,
                                           double var_init) {
  for (int i = threadIdx.x; i < TABLE_SIZE; i += blockDim.x)
    tbl[i] = make_entry<Acc>(i, weight_rule, age_max, Acc(var_init));
  __syncthreads();
}

// Compile-time variants of the forward kernels.  F_COUNT (batched kernel
// only) adds the per-frame foreground counts of instances that have counters.
// F_STEP (one-frame launches without checkpoints or codes) requests the
// state before the workgroup builds its table.
enum : int { F_BG = FWD_BG, F_CODES = FWD_CODES, F_CKPT = FWD_CKPT, F_PRINTED = FWD_PRINTED,
             F_COUNT = 16, F_STEP = 32 };

// Everything one lane needs to run its pixel group through T frames.
struct GroupJob {
  const char* frames;  // element (0, 0, 0) of the instance
  char* masks;
  char* bg;            // used with F_BG
  char* codes;         // used with F_CODES
  char* state[6];      // the six planes (element 0)
  char* ckpt;          // used with F_CKPT: checkpoint slot 0
  uint32_t* counts;    // used with F_COUNT: T foreground counters (this item's stripe)
  int64_t ckpt_every, ckpt_slot_bytes, ckpt_fplane, ckpt_aplane;
  int64_t T, frame_stride;
  uint32_t foff;       // element offset of the group within a frame (< 2^31)
  int64_t soff;        // pixel index of the group's first pixel (h*W + w)
};

template <typename Acc, int P>
__device__ __forceinline__ void store_state(char* const planes[6], int64_t soff,
                                            const Model<Acc>* s) {
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
  *reinterpret_cast<Vec<Acc, P>*>(planes[0] + soff * int64_t(sizeof(Acc))) = mA;
  *reinterpret_cast<Vec<Acc, P>*>(planes[1] + soff * int64_t(sizeof(Acc))) = vA;
  *reinterpret_cast<Vec<Acc, P>*>(planes[2] + soff * int64_t(sizeof(Acc))) = mC;
  *reinterpret_cast<Vec<Acc, P>*>(planes[3] + soff * int64_t(sizeof(Acc))) = vC;
  *reinterpret_cast<Vec<uint8_t, P>*>(planes[4] + soff) = aA;
  *reinterpret_cast<Vec<uint8_t, P>*>(planes[5] + soff) = aC;
}

// the group's six state values
template <typename Acc, int P>
__device__ __forceinline__ void load_state(const GroupJob& j, Model<Acc>* s) {
  const int64_t o = j.soff * int64_t(sizeof(Acc));
  const Vec<Acc, P> mA = *reinterpret_cast<const Vec<Acc, P>*>(j.state[0] + o);
  const Vec<Acc, P> vA = *reinterpret_cast<const Vec<Acc, P>*>(j.state[1] + o);
  const Vec<Acc, P> mC = *reinterpret_cast<const Vec<Acc, P>*>(j.state[2] + o);
  const Vec<Acc, P> vC = *reinterpret_cast<const Vec<Acc, P>*>(j.state[3] + o);
  const Vec<uint8_t, P> aA = *reinterpret_cast<const Vec<uint8_t, P>*>(j.state[4] + j.soff);
  const Vec<uint8_t, P> aC = *reinterpret_cast<const Vec<uint8_t, P>*>(j.state[5] + j.soff);
#pragma unroll
  for (int q = 0; q < P; ++q) {
    s[q].mA = mA.v[q];
    s[q].vA = vA.v[q];
    s[q].mC = mC.v[q];
    s[q].vC = vC.v[q];
    s[q].aA = aA.v[q];
    s[q].aC = aC.v[q];
  }
}

// The group through its T frames; with F_STEP from the state `pre` the
// caller has already loaded, else from the state planes.
template <typename In, typename Acc, typename Io, int P, int U, int FLAGS>
__device__ __forceinline__ void run_group(const GroupJob& j, const StepConsts<Acc>& k,
                                          const TableEntry<Acc>* __restrict__ tbl,
                                          const Model<Acc>* pre = nullptr) {
  constexpr bool BG = (FLAGS & F_BG) != 0;
  constexpr bool CODES = (FLAGS & F_CODES) != 0;
  constexpr bool CKPT = (FLAGS & F_CKPT) != 0;
  constexpr bool PRINTED = (FLAGS & F_PRINTED) != 0;
  constexpr bool COUNT = (FLAGS & F_COUNT) != 0;
  Model<Acc> s[P];
  if constexpr ((FLAGS & F_STEP) != 0) {
#pragma unroll
    for (int q = 0; q < P; ++q) s[q] = pre[q];
  } else {
    // load_state's loads written out rather than called: a call compiles
    // the time-fused kernels to a different instruction schedule than the
    // one their measurements were made with
    const int64_t o = j.soff * int64_t(sizeof(Acc));
    const Vec<Acc, P> mA = *reinterpret_cast<const Vec<Acc, P>*>(j.state[0] + o);
    const Vec<Acc, P> vA = *reinterpret_cast<const Vec<Acc, P>*>(j.state[1] + o);
    const Vec<Acc, P> mC = *reinterpret_cast<const Vec<Acc, P>*>(j.state[2] + o);
    const Vec<Acc, P> vC = *reinterpret_cast<const Vec<Acc, P>*>(j.state[3] + o);
    const Vec<uint8_t, P> aA = *reinterpret_cast<const Vec<uint8_t, P>*>(j.state[4] + j.soff);
    const Vec<uint8_t, P> aC = *reinterpret_cast<const Vec<uint8_t, P>*>(j.state[5] + j.soff);
#pragma unroll
    for (int q = 0; q < P; ++q) {
      s[q].mA = mA.v[q];
      s[q].vA = vA.v[q];
      s[q].mC = mC.v[q];
      s[q].vC = vC.v[q];
      s[q].aA = aA.v[q];
      s[q].aC = aC.v[q];
    }
  }

  // per frame: a uniform base pointer (scalar registers) plus a 32-bit
  // per-lane byte offset, so loads and stores use the saddr+voffset form
  const int64_t T = j.T, fs = j.frame_stride;
  const uint32_t off_in = j.foff * uint32_t(sizeof(In));
  const uint32_t off_io = j.foff * uint32_t(sizeof(Io));
  // checkpoints: the state before frames 0, K, 2K, ... into consecutive slots
  char* ck_slot = j.ckpt;
  int64_t ck_left = 0;

  auto do_frame = [&](const Vec<In, P>& xin, int64_t t) {
    if (CKPT) {
      if (ck_left == 0) {
        char* planes[6] = {ck_slot, ck_slot + j.ckpt_fplane, ck_slot + 2 * j.ckpt_fplane,
                           ck_slot + 3 * j.ckpt_fplane, ck_slot + 4 * j.ckpt_fplane,
                           ck_slot + 4 * j.ckpt_fplane + j.ckpt_aplane};
        store_state<Acc, P>(planes, j.soff, s);
        ck_slot += j.ckpt_slot_bytes;
        ck_left = j.ckpt_every;
      }
      --ck_left;
    }
    Vec<uint8_t, P> mk;
    Vec<Io, P> bgv;
    Vec<uint8_t, P> cd;
    // the P pixels' exchanges share one wavefront-uniform branch
    Acc xs[P], qd[P];
    StepRecord<Acc> r[P];
    bool any = false;
#pragma unroll
    for (int q = 0; q < P; ++q) {
      xs[q] = to_acc<In, Acc>(xin.v[q]);
      r[q] = step_core<Acc>(s[q], xs[q], k, tbl);
      qd[q] = mask_dist<Acc>(r[q]);
      any |= r[q].swap;
    }
    if (any_lane(any)) {
#pragma unroll
      for (int q = 0; q < P; ++q) {
        apply_swap<Acc>(s[q], xs[q], k, r[q].swap);
        qd[q] = mask_dist_swapped<Acc>(r[q], s[q], xs[q], qd[q]);
      }
    }
#pragma unroll
    for (int q = 0; q < P; ++q) {
      r[q].fg = fg_from<Acc, PRINTED>(qd[q], s[q], xs[q], k);
      mk.v[q] = r[q].fg ? uint8_t(255) : uint8_t(0);
      if (BG) bgv.v[q] = Io(s[q].mA);  // rounded once when Io is narrower
      if (CODES) cd.v[q] = uint8_t(code_of<Acc>(r[q]));
    }
    if (COUNT && j.counts != nullptr) {  // uniform: the item's instance has counters
      // the wavefront's foreground pixels of this frame: one ballot per pixel
      // of the lane group, summed in scalar registers, one integer atomic
      // (exact, order-free) from the first lane; every caller has lane 0 active
      uint32_t n = 0;
#pragma unroll
      for (int q = 0; q < P; ++q) n += uint32_t(__builtin_popcountll(__builtin_amdgcn_ballot_w64(r[q].fg)));
      if ((threadIdx.x & 63) == 0 && n != 0) atomicAdd(j.counts + t, n);
    }
    const int64_t o = t * fs;
    st_stream<uint8_t, P>(reinterpret_cast<uint8_t*>(j.masks + o + j.foff), mk);
    if (BG) st_stream<Io, P>(reinterpret_cast<Io*>(j.bg + o * int64_t(sizeof(Io)) + off_io), bgv);
    if (CODES) *reinterpret_cast<Vec<uint8_t, P>*>(j.codes + o + j.foff) = cd;
  };

  // Full batches of U frames, software-pipelined over two register buffers:
  // the loads of batch b+1 are issued before the steps of batch b, so U frames
  // are always in flight while the lane computes.  All conditions are uniform.
  auto load_batch = [&](Vec<In, P>* xb, int64_t t0) {
#pragma unroll
    for (int u = 0; u < U; ++u)
      xb[u] = ld_stream<In, P>(
          reinterpret_cast<const In*>(j.frames + (t0 + u) * fs * int64_t(sizeof(In)) + off_in));
  };
  auto run_batch = [&](const Vec<In, P>* xb, int64_t t0) {
#pragma unroll
    for (int u = 0; u < U; ++u) do_frame(xb[u], t0 + u);
  };
  const int64_t nfull = T / U;
  Vec<In, P> xa[U], xb[U];
  if (nfull > 0) load_batch(xa, 0);
  for (int64_t b = 0; b < nfull; b += 2) {
    if (b + 1 < nfull) load_batch(xb, (b + 1) * U);
    run_batch(xa, b * U);
    if (b + 1 >= nfull) break;
    if (b + 2 < nfull) load_batch(xa, (b + 2) * U);
    run_batch(xb, (b + 1) * U);
  }
  for (int64_t t = nfull * U; t < T; ++t)
    do_frame(ld_stream<In, P>(
                 reinterpret_cast<const In*>(j.frames + t * fs * int64_t(sizeof(In)) + off_in)),
             t);

  store_state<Acc, P>(j.state, j.soff, s);
}

// The job of one lane group of a one-frame launch (no checkpoints, no codes).
__device__ __forceinline__ GroupJob step_job(const FwdArgs& a, const geom::Group& G) {
  GroupJob j;
  j.frames = static_cast<const char*>(a.frames);
  j.masks = reinterpret_cast<char*>(a.masks);
  j.bg = static_cast<char*>(a.bg);
  j.codes = nullptr;
  j.state[0] = static_cast<char*>(a.mean_a);
  j.state[1] = static_cast<char*>(a.var_a);
  j.state[2] = static_cast<char*>(a.mean_c);
  j.state[3] = static_cast<char*>(a.var_c);
  j.state[4] = reinterpret_cast<char*>(a.age_a);
  j.state[5] = reinterpret_cast<char*>(a.age_c);
  j.ckpt = nullptr;
  j.counts = nullptr;
  j.ckpt_every = 1;
  j.ckpt_slot_bytes = j.ckpt_fplane = j.ckpt_aplane = 0;
  j.T = a.T;
  j.frame_stride = a.frame_stride;
  j.foff = uint32_t(G.foff);  // < 2^31 elements (host check)
  j.soff = G.soff;
  return j;
}

template <typename In, typename Acc, typename Io, int P, int U, int FLAGS>
__global__ void __launch_bounds__(256) fwd_kernel(const FwdArgs a) {
  __shared__ TableEntry<Acc> tbl[TABLE_SIZE];
  if constexpr ((FLAGS & F_STEP) != 0) {
    // one frame: the state is requested before the table is built, so that
    // its latency overlaps the table's divisions and barrier
    const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const bool active = g < a.ngroups;
    const GroupJob j = step_job(a, geom::group_of(g, a.groups_per_row, P, a.W, a.row_stride));
    Model<Acc> s[P];
    if (active) load_state<Acc, P>(j, s);
    fill_table<Acc>(tbl, a.weight_rule, a.age_max, a.var_init);
    if (!active) return;  // no barrier follows
    const StepConsts<Acc> k = make_consts<Acc>(a.theta_s, a.theta_d, a.var_init, a.var_floor,
                                               a.mask_floor);
    run_group<In, Acc, Io, P, U, FLAGS>(j, k, tbl, s);
    return;
  }
  fill_table<Acc>(tbl, a.weight_rule, a.age_max, a.var_init);

  const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= a.ngroups) return;
  const geom::Group G = geom::group_of(g, a.groups_per_row, P, a.W, a.row_stride);
  const StepConsts<Acc> k = make_consts<Acc>(a.theta_s, a.theta_d, a.var_init, a.var_floor,
                                             a.mask_floor);
  GroupJob j;
  j.frames = static_cast<const char*>(a.frames);
  j.masks = reinterpret_cast<char*>(a.masks);
  j.bg = static_cast<char*>(a.bg);
  j.codes = reinterpret_cast<char*>(a.codes);
  j.state[0] = static_cast<char*>(a.mean_a);
  j.state[1] = static_cast<char*>(a.var_a);
  j.state[2] = static_cast<char*>(a.mean_c);
  j.state[3] = static_cast<char*>(a.var_c);
  j.state[4] = reinterpret_cast<char*>(a.age_a);
  j.state[5] = reinterpret_cast<char*>(a.age_c);
  j.ckpt = static_cast<char*>(a.ckpt);
  j.counts = nullptr;
  j.ckpt_every = a.ckpt_every;
  j.ckpt_slot_bytes = a.ckpt_slot_bytes;
  j.ckpt_fplane = a.ckpt_fplane;
  j.ckpt_aplane = a.ckpt_aplane;
  j.T = a.T;
  j.frame_stride = a.frame_stride;
  j.foff = uint32_t(G.foff);  // < 2^31 elements (host check)
  j.soff = G.soff;
  run_group<In, Acc, Io, P, U, FLAGS>(j, k, tbl);
}

// The first active lane's copy of v in every lane, as a value the compiler
// knows to be the same across the wavefront (held in scalar registers).  The
// callers run with all 64 lanes active (256-thread workgroups, uniform control
// flow), so the first active lane is lane 0.
template <typename T>
__device__ __forceinline__ T wave_uniform(const T& v) {
  static_assert(sizeof(T) % 4 == 0, "whole dwords");
  int w[sizeof(T) / 4];
  __builtin_memcpy(w, &v, sizeof(T));
#pragma unroll
  for (int i = 0; i < int(sizeof(T) / 4); ++i) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
  T out;
  __builtin_memcpy(&out, w, sizeof(T));
  return out;
}

// Waves per SIMD the batched kernel is compiled for.  BF16 frames with FP32
// state, 4 pixels per lane and no bg output: 5 (96 instead of 104 VGPRs, a
// 36-byte spill outside the frame loop), measured 2.4 % faster than 4; the
// other variants spill more under that bound and keep the compiler's choice.
template <typename In, typename Acc, int P, int FLAGS>
constexpr int batched_waves() {
  return (sizeof(In) == 2 && sizeof(Acc) == 4 && P == 4 && (FLAGS & F_BG) == 0) ? 5 : 1;
}

// One work item of the batched kernel; a batch with bg outputs may hold
// instances without.
template <typename In, typename Acc, typename Io, int P, int U, int FLAGS>
__device__ __forceinline__ void run_item(const GroupJob& j, const BatchInst& I,
                                         const StepConsts<Acc>& k,
                                         const TableEntry<Acc>* __restrict__ tbl) {
  if constexpr ((FLAGS & F_BG) != 0) {
    if (I.bg != nullptr)
      run_group<In, Acc, Io, P, U, FLAGS>(j, k, tbl);
    else
      run_group<In, Acc, Io, P, U, FLAGS & ~F_BG>(j, k, tbl);
  } else {
    run_group<In, Acc, Io, P, U, FLAGS>(j, k, tbl);
  }
}

// FLAGS may only hold F_BG and F_PRINTED (no codes, no checkpoints)
template <typename In, typename Acc, typename Io, int P, int U, int FLAGS>
__global__ void __launch_bounds__(256)
    __attribute__((amdgpu_waves_per_eu(batched_waves<In, Acc, P, FLAGS>())))
    batched_kernel(const BatchArgs a) {
  __shared__ TableEntry<Acc> tbl[TABLE_SIZE];
  fill_table<Acc>(tbl, a.weight_rule, a.age_max, a.var_init);
  const StepConsts<Acc> k = make_consts<Acc>(a.theta_s, a.theta_d, a.var_init, a.var_floor,
                                             a.mask_floor);
  const int lane = int(threadIdx.x) & 63;
  for (;;) {
    // one atomic per wavefront; the item index is broadcast to all 64 lanes,
    // so the loop condition is uniform and every wavefront exits once the
    // counter has passed n_items
    unsigned long long item = 0;
    if (lane == 0) item = atomicAdd(a.counter, 1ull);
    item = wave_uniform(item);
    if (item >= (unsigned long long)a.n_items) break;
    // the item and its instance are the same for the whole wavefront: scalar
    // registers, not 30 vector registers per lane
    const BatchItem it = wave_uniform(a.items[item]);
    const BatchInst I = wave_uniform(a.inst[it.inst]);
    if (lane < it.count) {
      const int64_t g = int64_t(it.first_group) + lane;
      const geom::Group G = geom::group_of(g, I.groups_per_row, P, I.W, I.row_stride);
      GroupJob j;
      j.frames = static_cast<const char*>(I.frames);
      j.masks = reinterpret_cast<char*>(I.masks);
      j.bg = static_cast<char*>(I.bg);
      j.codes = nullptr;
      for (int q = 0; q < 6; ++q) j.state[q] = static_cast<char*>(I.state[q]);
      j.ckpt = nullptr;
      j.counts = I.fg_counts ? I.stripes + geom::stripe_of(item) * I.T : nullptr;
      j.ckpt_every = 1;
      j.ckpt_slot_bytes = j.ckpt_fplane = j.ckpt_aplane = 0;
      j.T = I.T;
      j.frame_stride = I.frame_stride;
      j.foff = uint32_t(G.foff);
      j.soff = G.soff;
      // one body for instances with and without foreground counters (a
      // uniform run-time test per frame), so the kernel's code stays one copy
      run_item<In, Acc, Io, P, U, FLAGS | F_COUNT>(j, I, k, tbl);
    }
  }
}

// Launchers of one (In, Acc) pair, defined in the per-type translation units.
template <typename In, typename Acc, typename Io, int P, int FLAGS>
hipError_t launch_fwd_v(const FwdArgs& a, int block, hipStream_t stream) {
  constexpr int U = 4;
  const int64_t grid = (a.ngroups + block - 1) / block;
  hipLaunchKernelGGL((fwd_kernel<In, Acc, Io, P, U, FLAGS>), dim3(uint32_t(grid)), dim3(block), 0,
                     stream, a);
  return hipGetLastError();
}

// runtime flags -> compile-time variant.  Decision codes are a debug output:
// they only exist as one-pixel-per-lane variants (results do not depend on P),
// so the caller must size the grid for P = 1 when it asks for codes.
template <typename In, typename Acc, typename Io, int P>
hipError_t launch_fwd_p(const FwdArgs& a, int flags, int block, hipStream_t stream) {
  switch (flags & (F_BG | F_CKPT | F_PRINTED)) {
    case 0: return launch_fwd_v<In, Acc, Io, P, 0>(a, block, stream);
    case F_BG: return launch_fwd_v<In, Acc, Io, P, F_BG>(a, block, stream);
    case F_CKPT: return launch_fwd_v<In, Acc, Io, P, F_CKPT>(a, block, stream);
    case F_BG | F_CKPT: return launch_fwd_v<In, Acc, Io, P, F_BG | F_CKPT>(a, block, stream);
    case F_PRINTED: return launch_fwd_v<In, Acc, Io, P, F_PRINTED>(a, block, stream);
    case F_BG | F_PRINTED: return launch_fwd_v<In, Acc, Io, P, F_BG | F_PRINTED>(a, block, stream);
    case F_CKPT | F_PRINTED: return launch_fwd_v<In, Acc, Io, P, F_CKPT | F_PRINTED>(a, block, stream);
    default: return launch_fwd_v<In, Acc, Io, P, F_BG | F_CKPT | F_PRINTED>(a, block, stream);
  }
}

// one-frame launches without checkpoints or codes (F_STEP)
template <typename In, typename Acc, typename Io, int P>
hipError_t launch_fwd_step(const FwdArgs& a, int flags, int block, hipStream_t stream) {
  switch (flags & (F_BG | F_PRINTED)) {
    case 0: return launch_fwd_v<In, Acc, Io, P, F_STEP>(a, block, stream);
    case F_BG: return launch_fwd_v<In, Acc, Io, P, F_STEP | F_BG>(a, block, stream);
    case F_PRINTED: return launch_fwd_v<In, Acc, Io, P, F_STEP | F_PRINTED>(a, block, stream);
    default: return launch_fwd_v<In, Acc, Io, P, F_STEP | F_BG | F_PRINTED>(a, block, stream);
  }
}

template <typename In, typename Acc, typename Io>
hipError_t launch_fwd_codes(const FwdArgs& a, int flags, int block, hipStream_t stream) {
  switch (flags & (F_BG | F_CKPT | F_PRINTED)) {
    case 0: return launch_fwd_v<In, Acc, Io, 1, F_CODES>(a, block, stream);
    case F_BG: return launch_fwd_v<In, Acc, Io, 1, F_CODES | F_BG>(a, block, stream);
    case F_CKPT: return launch_fwd_v<In, Acc, Io, 1, F_CODES | F_CKPT>(a, block, stream);
    case F_BG | F_CKPT: return launch_fwd_v<In, Acc, Io, 1, F_CODES | F_BG | F_CKPT>(a, block, stream);
    case F_PRINTED: return launch_fwd_v<In, Acc, Io, 1, F_CODES | F_PRINTED>(a, block, stream);
    case F_BG | F_PRINTED:
      return launch_fwd_v<In, Acc, Io, 1, F_CODES | F_BG | F_PRINTED>(a, block, stream);
    case F_CKPT | F_PRINTED:
      return launch_fwd_v<In, Acc, Io, 1, F_CODES | F_CKPT | F_PRINTED>(a, block, stream);
    default: return launch_fwd_v<In, Acc, Io, 1, F_CODES | F_BG | F_CKPT | F_PRINTED>(a, block, stream);
  }
}

template <typename In, typename Acc, typename Io>
hipError_t launch_fwd_t(const FwdArgs& a, int P, int flags, int block, hipStream_t stream) {
  if (flags & F_CODES) {
    if (P != 1) return hipErrorInvalidValue;  // the caller sizes the grid for P = 1
    return launch_fwd_codes<In, Acc, Io>(a, flags, block, stream);
  }
  if (a.T == 1 && (flags & F_CKPT) == 0) {
    if (P == 4) return launch_fwd_step<In, Acc, Io, 4>(a, flags, block, stream);
    if (P == 2) return launch_fwd_step<In, Acc, Io, 2>(a, flags, block, stream);
    return launch_fwd_step<In, Acc, Io, 1>(a, flags, block, stream);
  }
  if (P == 4) return launch_fwd_p<In, Acc, Io, 4>(a, flags, block, stream);
  if (P == 2) return launch_fwd_p<In, Acc, Io, 2>(a, flags, block, stream);
  return launch_fwd_p<In, Acc, Io, 1>(a, flags, block, stream);
}

template <typename In, typename Acc, typename Io, int P>
const void* batched_symbol_p(int flags) {
  constexpr int U = 4;
  switch (flags & (F_BG | F_PRINTED)) {
    case 0: return reinterpret_cast<const void*>(&batched_kernel<In, Acc, Io, P, U, 0>);
    case F_BG: return reinterpret_cast<const void*>(&batched_kernel<In, Acc, Io, P, U, F_BG>);
    case F_PRINTED:
      return reinterpret_cast<const void*>(&batched_kernel<In, Acc, Io, P, U, F_PRINTED>);
    default:
      return reinterpret_cast<const void*>(&batched_kernel<In, Acc, Io, P, U, F_BG | F_PRINTED>);
  }
}

template <typename In, typename Acc, typename Io>
const void* batched_symbol_t(int P, int flags) {
  if (P == 4) return batched_symbol_p<In, Acc, Io, 4>(flags);
  if (P == 2) return batched_symbol_p<In, Acc, Io, 2>(flags);
  return batched_symbol_p<In, Acc, Io, 1>(flags);
}

}  // namespace fwd

// The single-instance forward only (no batched kernel), for state types the
// batched launch does not take.
#define DSGM_FWD_INSTANTIATE_SINGLE(IN, ACC, IO, NAME)                                     \
  hipError_t launch_fwd_##NAME(const FwdArgs& a, int P, int flags, int block,              \
                               hipStream_t stream) {                                       \
    return fwd::launch_fwd_t<IN, ACC, IO>(a, P, flags, block, stream);                     \
  }

// One translation unit per (frame type, accumulation type) instantiates these.
#define DSGM_FWD_INSTANTIATE(IN, ACC, IO, NAME)                                            \
  hipError_t launch_fwd_##NAME(const FwdArgs& a, int P, int flags, int block,              \
                               hipStream_t stream) {                                       \
    return fwd::launch_fwd_t<IN, ACC, IO>(a, P, flags, block, stream);                     \
  }                                                                                        \
  const void* batched_sym_##NAME(int P, int flags) {                                       \
    return fwd::batched_symbol_t<IN, ACC, IO>(P, flags);                                   \
  }

}  // namespace dsgm
