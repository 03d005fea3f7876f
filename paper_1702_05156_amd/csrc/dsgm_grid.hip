// dsgm_grid.hip -- Yi et al.'s grid model (internal).
//
// Sec. 2.2 gives the update of Yi et al.'s model, where one dual Gaussian
// model covers a block G of b x b pixels: the block's mean intensity M is the
// value the tests, the blend and the reset use, and the variance term V is the
// largest squared distance of the updated mean from the block's intensities.
// The paper itself uses b = 1.  The foreground mask stays per pixel: pixel j
// of the block is background iff (mean_A - I_j)^2 <= theta_d * max(floor, ref).
//
// Decomposition: one lane per block for all T frames, the block's models in
// registers; per frame the lane reads the block's b rows (one vector load per
// row when the block is whole and aligned), keeps the b*b intensities in
// registers for the V and mask passes, and writes b mask rows; with FP64
// state the next frame's rows are loaded while the current one is processed
// (FP32 state relies on occupancy instead).  Neighbouring
// lanes own neighbouring blocks, so every row access is contiguous across the
// wavefront.  With FP64 state the block sum (row-major from 0), the division
// by |G| and the update follow the order of a scalar evaluation.
#include "dsgm_ext.h"
#include "dsgm_fwd_impl.h"

namespace dsgm {

namespace grid {

using fwd::fill_table;
using fwd::make_consts;

template <typename In, typename Acc, typename Io, int B>
__global__ void __launch_bounds__(256) grid_kernel(const GridArgs a) {
  __shared__ TableEntry<Acc> tbl[TABLE_SIZE];
  fill_table<Acc>(tbl, a.weight_rule, a.age_max, a.var_init);
  const StepConsts<Acc> k =
      make_consts<Acc>(a.theta_s, a.theta_d, a.var_init, a.var_floor, a.mask_floor);
  const bool printed = a.mask_rule != 0;

  const int64_t blk = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (blk >= a.Hb * a.Wb) return;  // no barrier follows
  const geom::GridBlock gb = geom::grid_block(blk, a.Wb, B, a.H, a.W);
  const int64_t y0 = gb.y0, x0 = gb.x0;
  const int rows = gb.rows, cols = gb.cols;
  const bool whole = rows == B && cols == B;
  const bool vec = whole && a.vec_ok;
  const Acc n = Acc(rows * cols);

  Model<Acc> s;
  s.mA = static_cast<const Acc*>(a.mean_a)[blk];
  s.vA = static_cast<const Acc*>(a.var_a)[blk];
  s.mC = static_cast<const Acc*>(a.mean_c)[blk];
  s.vC = static_cast<const Acc*>(a.var_c)[blk];
  s.aA = a.age_a[blk];
  s.aC = a.age_c[blk];

  const In* frames = static_cast<const In*>(a.frames);
  const int64_t base = y0 * a.row_stride + x0;
  // the block's b x b intensities of frame t
  auto load = [&](int64_t t, Acc (&I)[B][B]) {
    const int64_t o = t * a.frame_stride + base;
    if (vec) {
#pragma unroll
      for (int r = 0; r < B; ++r) {
        const Vec<In, B> v = fwd::ld_stream<In, B>(frames + o + r * a.row_stride);
#pragma unroll
        for (int c = 0; c < B; ++c) I[r][c] = to_acc<In, Acc>(v.v[c]);
      }
    } else {
#pragma unroll
      for (int r = 0; r < B; ++r)
#pragma unroll
        for (int c = 0; c < B; ++c)
          I[r][c] = (r < rows && c < cols) ? to_acc<In, Acc>(frames[o + r * a.row_stride + c])
                                           : Acc(0);
    }
  };
  auto frame = [&](int64_t t, const Acc (&I)[B][B]) {
    const int64_t o = t * a.frame_stride + base;
    // block mean, row-major from 0 (missing pixels of an edge block are skipped)
    Acc sum = Acc(0);
#pragma unroll
    for (int r = 0; r < B; ++r)
#pragma unroll
      for (int c = 0; c < B; ++c)
        if (whole || (r < rows && c < cols)) sum = sum + I[r][c];
    const Acc M = sum / n;

    // Sec. 2.3 decisions on M, the Sec. 2.2 blend of the matched model with M
    const Acc dA = M - s.mA;
    const Acc dC = M - s.mC;
    const bool hitA = (dA * dA < k.theta_s * s.vA) | (dA * dA < k.ts_vf);
    const bool hitC = (dC * dC < k.theta_s * s.vC) | (dC * dC < k.ts_vf);
    const int idx = hitA ? s.aA : (hitC ? s.aC : RESET_SLOT);
    const Acc m = hitA ? s.mA : s.mC;
    const Acc v = hitA ? s.vA : s.vC;
    const TableEntry<Acc> e = tbl[idx];
    const Acc mn = blend(e.u, m, e.w, M);
    // V: the block's largest squared distance from the updated mean; a reset
    // candidate has no V (its variance is var_init)
    Acc V = Acc(0);
#pragma unroll
    for (int r = 0; r < B; ++r)
#pragma unroll
      for (int c = 0; c < B; ++c)
        if (whole || (r < rows && c < cols)) {
          const Acc d = mn - I[r][c];
          const Acc q = d * d;
          V = V < q ? q : V;
        }
    V = idx == RESET_SLOT ? Acc(0) : V;
    const Acc vn = blend(e.u, v, e.w, V) + e.r;
    const int an = e.next;
    s.mA = hitA ? mn : s.mA;
    s.vA = hitA ? vn : s.vA;
    s.aA = hitA ? an : s.aA;
    s.mC = hitA ? s.mC : mn;
    s.vC = hitA ? s.vC : vn;
    s.aC = hitA ? s.aC : an;
    const bool swap = s.aC > s.aA;
    if (any_lane(swap)) apply_swap<Acc>(s, M, k, swap);

    // per-pixel mask against the block's apparent model
#pragma unroll
    for (int r = 0; r < B; ++r) {
      Vec<uint8_t, B> mk;
#pragma unroll
      for (int c = 0; c < B; ++c) {
        const Acc d = s.mA - I[r][c];
        const Acc qd = d * d;
        const Acc ref = printed ? I[r][c] : s.vA;
        const bool fg = !((qd <= k.theta_d * ref) | (qd <= k.td_mf));
        mk.v[c] = fg ? uint8_t(255) : uint8_t(0);
      }
      if (vec) {
        *reinterpret_cast<Vec<uint8_t, B>*>(a.masks + o + r * a.row_stride) = mk;
      } else if (r < rows) {
#pragma unroll
        for (int c = 0; c < B; ++c)
          if (c < cols) a.masks[o + r * a.row_stride + c] = mk.v[c];
      }
    }
    if (a.codes) {
      const unsigned code = (hitA ? CODE_HIT_A : (hitC ? CODE_HIT_C : CODE_RESET)) |
                            (swap ? CODE_SWAP : 0u);
      a.codes[t * a.Hb * a.Wb + blk] = uint8_t(code);
    }
    if (a.bg) static_cast<Io*>(a.bg)[t * a.Hb * a.Wb + blk] = Io(s.mA);
  };
  if constexpr (sizeof(Acc) == 4) {
    // FP32 state: one frame buffer.  The registers it frees (76 instead of
    // 120 VGPRs at b = 4, 6 waves per SIMD instead of 4) hide the load latency
    // better than a second buffer: 8 % faster.  With FP64 state a single
    // buffer measured 3.5 % slower, so FP64 keeps two.
    Acc I0[B][B];
    for (int64_t t = 0; t < a.T; ++t) {
      load(t, I0);
      frame(t, I0);
    }
  } else {
    // two frame buffers: the next frame's loads are in flight while this one
    // is processed
    Acc I0[B][B], I1[B][B];
    const int64_t T = a.T;
    if (T > 0) load(0, I0);
    int64_t t = 0;
    for (; t + 1 < T; t += 2) {
      load(t + 1, I1);
      frame(t, I0);
      if (t + 2 < T) load(t + 2, I0);
      frame(t + 1, I1);
    }
    if (t < T) frame(t, I0);
  }
  static_cast<Acc*>(a.mean_a)[blk] = s.mA;
  static_cast<Acc*>(a.var_a)[blk] = s.vA;
  static_cast<Acc*>(a.mean_c)[blk] = s.mC;
  static_cast<Acc*>(a.var_c)[blk] = s.vC;
  a.age_a[blk] = uint8_t(s.aA);
  a.age_c[blk] = uint8_t(s.aC);
}

template <typename In, typename Acc, typename Io>
hipError_t launch_t(const GridArgs& a, int b, hipStream_t stream) {
  const int64_t nb = a.Hb * a.Wb;
  const dim3 grid{uint32_t((nb + 255) / 256), 1, 1}, block{256, 1, 1};
  switch (b) {
    case 1: hipLaunchKernelGGL((grid_kernel<In, Acc, Io, 1>), grid, block, 0, stream, a); break;
    case 2: hipLaunchKernelGGL((grid_kernel<In, Acc, Io, 2>), grid, block, 0, stream, a); break;
    case 4: hipLaunchKernelGGL((grid_kernel<In, Acc, Io, 4>), grid, block, 0, stream, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace grid

hipError_t launch_grid(const GridArgs& a, int in_dtype, int acc, int b, hipStream_t stream) {
  if (acc == 0) {
    if (in_dtype == 0) return grid::launch_t<double, double, double>(a, b, stream);
    if (in_dtype == 1) return grid::launch_t<float, double, double>(a, b, stream);
    if (in_dtype == 2) return grid::launch_t<bf16_t, double, double>(a, b, stream);
  } else if (acc == 1) {
    if (in_dtype == 1) return grid::launch_t<float, float, float>(a, b, stream);
    if (in_dtype == 2) return grid::launch_t<bf16_t, float, float>(a, b, stream);
  } else if (acc == 2) {
    if (in_dtype == 1) return grid::launch_t<float, double, float>(a, b, stream);
    if (in_dtype == 2) return grid::launch_t<bf16_t, double, float>(a, b, stream);
  }
  return hipErrorInvalidValue;
}

}  // namespace dsgm
