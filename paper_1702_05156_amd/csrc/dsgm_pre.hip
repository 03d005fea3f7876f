// dsgm_pre.hip -- the forward with the paper's frame preprocessing fused in
// (internal).
//
// Sec. 2.1 and the preprocessing of Sec. 3.1.1 / 3.3.1: every frame is blurred
// with a separable kernel (along rows, then along columns; a sampled,
// normalised Gaussian by default) and then median-filtered over 3 x 3
// neighbourhoods, borders clamped to the nearest valid row and column; the
// background update of Sec. 2.2-2.3 then runs on the filtered frame.  Here all
// three happen in one pass over the sequence: the filtered frame never goes
// to memory unless the caller asks for it.
//
// Decomposition: a workgroup of 256 lanes owns a TH x TW = 16 x 64 tile of
// pixels for all T frames, each lane four horizontally adjacent pixels of one
// row, with their model state in registers.  Per frame the workgroup stages
// the tile plus a halo of R = RG (+1 with the median) rows and columns of the
// raw frame in LDS (indices clamped to the frame), runs the row pass and the
// column pass of the blur in LDS, then each lane takes the median of its
// pixels' 3 x 3 neighbourhoods and updates its models.  The next frame's tile
// is loaded into registers while the current one is filtered, so its HBM
// latency overlaps the arithmetic.  Tiles are dealt so that each XCD gets a
// contiguous range of them: neighbouring tiles, whose halos overlap, run on
// the same L2.
//
// Median of nine: sort each of the three columns of the neighbourhood; the
// median is then the median of (largest column minimum, median of the column
// medians, smallest column maximum).  Four adjacent pixels share their column
// sorts (six columns), so a pixel costs about 21 min/max.  All selections
// are exact.
//
// The blur sums run from 0 in index order with every product and sum rounded
// (no contraction) for FP64 state, the order the oracle uses.
#include "dsgm_ext.h"
#include "dsgm_fwd_impl.h"

namespace dsgm {

namespace pre {

using fwd::fill_table;
using fwd::make_consts;

// tile shape and every tile cell index: dsgm_geom.h
using geom::pre::TH;
using geom::pre::TW;
using geom::pre::PX;
using geom::pre::NT;
template <int RG, bool MED>
using Geo = geom::pre::Geo<RG, MED>;

// min and max of finite values (v_min/v_max; a zero's sign may differ from a
// sort's when +0 and -0 tie, which leaves every value unchanged)
__device__ __forceinline__ double mn(double a, double b) { return __builtin_fmin(a, b); }
__device__ __forceinline__ double mx(double a, double b) { return __builtin_fmax(a, b); }
__device__ __forceinline__ float mn(float a, float b) { return __builtin_fminf(a, b); }
__device__ __forceinline__ float mx(float a, float b) { return __builtin_fmaxf(a, b); }

// median of three
template <typename Acc>
__device__ __forceinline__ Acc med3(Acc a, Acc b, Acc c) {
  return mx(mn(a, b), mn(mx(a, b), c));
}

// blur sum over n taps from 0 in index order (no contraction for double)
template <typename Acc>
__device__ __forceinline__ Acc tap(Acc acc, Acc w, Acc x) { return acc + w * x; }
template <>
__device__ __forceinline__ float tap<float>(float acc, float w, float x) {
  return __builtin_fmaf(w, x, acc);
}

template <typename In, typename Acc, typename Io, int RG, bool MED, bool PRINTED>
__global__ void __launch_bounds__(NT) pre_kernel(const PreArgs a) {
  using G = Geo<RG, MED>;
  // raw, row-blurred and blurred tiles each have their own storage, so a frame
  // needs three barriers: the next frame's raw tile can be staged while slow
  // lanes still read this frame's blurred tile (without a blur the raw tile is
  // the blurred tile and a fourth barrier guards it)
  __shared__ Acc buf_raw[G::RAW_N];
  __shared__ Acc buf_hb[RG > 0 ? G::HB_N : 1];
  __shared__ Acc buf_gb[RG > 0 ? G::GB_N : 1];
  __shared__ TableEntry<Acc> tbl[TABLE_SIZE];
  fill_table<Acc>(tbl, a.weight_rule, a.age_max, a.var_init);  // ends with a barrier
  const StepConsts<Acc> k =
      make_consts<Acc>(a.theta_s, a.theta_d, a.var_init, a.var_floor, a.mask_floor);

  Acc wt[2 * RG + 1];
#pragma unroll
  for (int i = 0; i < 2 * RG + 1; ++i) wt[i] = Acc(a.w[i]);

  const int64_t tile = tile_of(blockIdx.x, gridDim.x);
  const int64_t y0 = (tile / a.tiles_x) * TH, x0 = (tile % a.tiles_x) * TW;
  const int tid = threadIdx.x;
  const int ty = G::lane_row(tid), tx = G::lane_col(tid);  // this lane's row and first column
  const int64_t gy = y0 + ty;

  // this lane's raw-tile elements: LDS slot and frame offset (both fixed per frame)
  uint32_t roff[G::LOADS];
#pragma unroll
  for (int l = 0; l < G::LOADS; ++l) {
    const int i = G::raw_cell(tid, l);
    roff[l] = i < G::RAW_N ? uint32_t(G::raw_source(i, y0, x0, a.H, a.W, a.row_stride))
                           : 0u;  // < 2^31 (host check)
  }
  // the median's rows and columns in the blurred tile, clamped to the frame
  int gr[3], gc[PX + 2];
#pragma unroll
  for (int d = 0; d < 3; ++d) gr[d] = G::med_row(gy, d, y0, a.H);
#pragma unroll
  for (int d = 0; d < PX + 2; ++d) gc[d] = G::med_col(x0 + tx, d, x0, a.W);

  bool valid[PX];
  bool all_valid = gy < a.H;
#pragma unroll
  for (int q = 0; q < PX; ++q) {
    valid[q] = gy < a.H && x0 + tx + q < a.W;
    all_valid = all_valid && valid[q];
  }
  const int64_t pix = gy * a.W + x0 + tx;          // state index of pixel 0
  const int64_t foff = gy * a.row_stride + x0 + tx; // frame offset of pixel 0
  const bool vec_ok = all_valid && (a.row_stride % PX) == 0 && (a.frame_stride % PX) == 0 &&
                      (a.W % PX) == 0;

  Model<Acc> s[PX];
#pragma unroll
  for (int q = 0; q < PX; ++q) {
    if (valid[q]) {
      s[q].mA = static_cast<const Acc*>(a.mean_a)[pix + q];
      s[q].vA = static_cast<const Acc*>(a.var_a)[pix + q];
      s[q].mC = static_cast<const Acc*>(a.mean_c)[pix + q];
      s[q].vC = static_cast<const Acc*>(a.var_c)[pix + q];
      s[q].aA = a.age_a[pix + q];
      s[q].aC = a.age_c[pix + q];
    } else {
      s[q].mA = s[q].vA = s[q].mC = s[q].vC = Acc(0);
      s[q].aA = s[q].aC = 1;
    }
  }

  // this lane's outputs of the row and column passes (pairs of adjacent
  // outputs, lane-strided) and the row pass's window start in the raw tile:
  // the same every frame
  constexpr int ROW_IT = G::ROW_IT, COL_IT = G::COL_IT;
  uint32_t row_src[ROW_IT];
#pragma unroll
  for (int it = 0; it < ROW_IT; ++it) row_src[it] = uint32_t(G::row_window(G::row_pair(tid, it)));

  const In* frames = static_cast<const In*>(a.frames);
  In nxt[G::LOADS];
  auto load_frame = [&](int64_t t) {
    const In* f = frames + t * a.frame_stride;
#pragma unroll
    for (int l = 0; l < G::LOADS; ++l)
      if (G::raw_active(tid, l)) nxt[l] = f[roff[l]];
  };
  if (a.T > 0) load_frame(0);

  for (int64_t t = 0; t < a.T; ++t) {
    // 1. stage the raw tile, then start loading the next frame's
#pragma unroll
    for (int l = 0; l < G::LOADS; ++l)
      if (G::raw_active(tid, l)) buf_raw[G::raw_cell(tid, l)] = to_acc<In, Acc>(nxt[l]);
    __syncthreads();
    if (t + 1 < a.T) load_frame(t + 1);

    const Acc* gbp;  // the blurred tile, GB_H x GB_W
    if constexpr (RG > 0) {
      // 2. row pass: hb[r][v] = sum_j w_j raw[r][v + j], v in [0, HB_W).  A
      // lane makes two horizontally adjacent outputs per step from one window
      // of 2*RG + 2 values (HB_W is even, so a pair never straddles rows)
      static_assert(G::HB_W % 2 == 0 && G::GB_W % 2 == 0, "output pairs stay in one row");
#pragma unroll
      for (int it = 0; it < ROW_IT; ++it) {
        const int pi = G::row_pair(tid, it);
        if (G::row_active(tid, it)) {
          const Acc* src = buf_raw + row_src[it];
          Acc win[2 * RG + 2];
#pragma unroll
          for (int j = 0; j < 2 * RG + 2; ++j) win[j] = src[j];
          Acc a0 = Acc(0), a1 = Acc(0);
#pragma unroll
          for (int j = 0; j < 2 * RG + 1; ++j) {
            a0 = tap(a0, wt[j], win[j]);
            a1 = tap(a1, wt[j], win[j + 1]);
          }
          buf_hb[2 * pi] = a0;
          buf_hb[2 * pi + 1] = a1;
        }
      }
      __syncthreads();
      // 3. column pass: gb[r][v] = sum_i w_i hb[r + i][v], r in [0, GB_H); the
      // two tiles have the same width, so gb's row-major index is hb's
      static_assert(G::HB_W == G::GB_W, "row-blurred and blurred tiles share a width");
#pragma unroll
      for (int it = 0; it < COL_IT; ++it) {
        const int pi = G::col_pair(tid, it);
        if (G::col_active(tid, it)) {
          const Acc* src = buf_hb + 2 * pi;
          Acc a0 = Acc(0), a1 = Acc(0);
#pragma unroll
          for (int j = 0; j < 2 * RG + 1; ++j) {
            a0 = tap(a0, wt[j], src[j * G::HB_W]);
            a1 = tap(a1, wt[j], src[j * G::HB_W + 1]);
          }
          buf_gb[2 * pi] = a0;
          buf_gb[2 * pi + 1] = a1;
        }
      }
      __syncthreads();
      gbp = buf_gb;
    } else {
      gbp = buf_raw;  // no blur: the raw tile (R = RM) is the blurred tile
    }

    // 4. median of each pixel's 3 x 3 neighbourhood, then the model update
    Acc xs[PX];
    if constexpr (MED) {
      Acc lo[PX + 2], md[PX + 2], hi[PX + 2];
#pragma unroll
      for (int d = 0; d < PX + 2; ++d) {
        const Acc p0 = gbp[gr[0] * G::GB_W + gc[d]];
        const Acc p1 = gbp[gr[1] * G::GB_W + gc[d]];
        const Acc p2 = gbp[gr[2] * G::GB_W + gc[d]];
        const Acc l01 = mn(p0, p1), h01 = mx(p0, p1);
        lo[d] = mn(l01, p2);
        const Acc h = mx(l01, p2);
        hi[d] = mx(h01, h);
        md[d] = mn(h01, h);
      }
#pragma unroll
      for (int q = 0; q < PX; ++q) {
        const Acc a0 = mx(mx(lo[q], lo[q + 1]), lo[q + 2]);
        const Acc b0 = med3(md[q], md[q + 1], md[q + 2]);
        const Acc c0 = mn(mn(hi[q], hi[q + 1]), hi[q + 2]);
        xs[q] = med3(a0, b0, c0);
      }
    } else {
#pragma unroll
      for (int q = 0; q < PX; ++q) xs[q] = gbp[gr[1] * G::GB_W + gc[q + 1]];
    }

    StepRecord<Acc> rec[PX];
    bool any = false;
#pragma unroll
    for (int q = 0; q < PX; ++q) {
      rec[q] = step_core<Acc>(s[q], xs[q], k, tbl);
      any |= rec[q].swap;
    }
    if (any_lane(any)) {
#pragma unroll
      for (int q = 0; q < PX; ++q) apply_swap<Acc>(s[q], xs[q], k, rec[q].swap);
    }
    Vec<uint8_t, PX> mk, cd;
    Vec<Io, PX> bgv;
    Vec<Io, PX> fv;  // the filtered frame in the array type
#pragma unroll
    for (int q = 0; q < PX; ++q) {
      rec[q].fg = fg_of<Acc, PRINTED>(s[q], xs[q], k);
      mk.v[q] = rec[q].fg ? uint8_t(255) : uint8_t(0);
      cd.v[q] = uint8_t(code_of<Acc>(rec[q]));
      bgv.v[q] = Io(s[q].mA);
      fv.v[q] = Io(xs[q]);
    }
    const int64_t o = t * a.frame_stride + foff;
    if (vec_ok) {
      *reinterpret_cast<Vec<uint8_t, PX>*>(a.masks + o) = mk;
      if (a.bg) *reinterpret_cast<Vec<Io, PX>*>(static_cast<Io*>(a.bg) + o) = bgv;
      if (a.filtered) *reinterpret_cast<Vec<Io, PX>*>(static_cast<Io*>(a.filtered) + o) = fv;
      if (a.codes) *reinterpret_cast<Vec<uint8_t, PX>*>(a.codes + o) = cd;
    } else {
#pragma unroll
      for (int q = 0; q < PX; ++q) {
        if (!valid[q]) continue;
        a.masks[o + q] = mk.v[q];
        if (a.bg) static_cast<Io*>(a.bg)[o + q] = bgv.v[q];
        if (a.filtered) static_cast<Io*>(a.filtered)[o + q] = fv.v[q];
        if (a.codes) a.codes[o + q] = cd.v[q];
      }
    }
    if constexpr (RG == 0) __syncthreads();  // the next frame overwrites the raw tile
  }

#pragma unroll
  for (int q = 0; q < PX; ++q) {
    if (!valid[q]) continue;
    static_cast<Acc*>(a.mean_a)[pix + q] = s[q].mA;
    static_cast<Acc*>(a.var_a)[pix + q] = s[q].vA;
    static_cast<Acc*>(a.mean_c)[pix + q] = s[q].mC;
    static_cast<Acc*>(a.var_c)[pix + q] = s[q].vC;
    a.age_a[pix + q] = uint8_t(s[q].aA);
    a.age_c[pix + q] = uint8_t(s[q].aC);
  }
}

template <typename In, typename Acc, typename Io, bool MED, bool PRINTED>
hipError_t launch_rg(const PreArgs& a, int rg, hipStream_t stream) {
  const int64_t nb = a.tiles_x * a.tiles_y;
  const dim3 grid{uint32_t(nb), 1, 1}, block{NT, 1, 1};
  switch (rg) {
    case 0: hipLaunchKernelGGL((pre_kernel<In, Acc, Io, 0, MED, PRINTED>), grid, block, 0, stream, a); break;
    case 1: hipLaunchKernelGGL((pre_kernel<In, Acc, Io, 1, MED, PRINTED>), grid, block, 0, stream, a); break;
    case 2: hipLaunchKernelGGL((pre_kernel<In, Acc, Io, 2, MED, PRINTED>), grid, block, 0, stream, a); break;
    case 3: hipLaunchKernelGGL((pre_kernel<In, Acc, Io, 3, MED, PRINTED>), grid, block, 0, stream, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename In, typename Acc, typename Io>
hipError_t launch_t(const PreArgs& a, int rg, bool median, hipStream_t stream) {
  const bool printed = a.mask_rule != 0;
  if (median)
    return printed ? launch_rg<In, Acc, Io, true, true>(a, rg, stream)
                   : launch_rg<In, Acc, Io, true, false>(a, rg, stream);
  return printed ? launch_rg<In, Acc, Io, false, true>(a, rg, stream)
                 : launch_rg<In, Acc, Io, false, false>(a, rg, stream);
}

}  // namespace pre

hipError_t launch_pre(const PreArgs& a, int in_dtype, int acc, int rg, bool median,
                      hipStream_t stream) {
  if (acc == 0) {
    if (in_dtype == 0) return pre::launch_t<double, double, double>(a, rg, median, stream);
    if (in_dtype == 1) return pre::launch_t<float, double, double>(a, rg, median, stream);
    if (in_dtype == 2) return pre::launch_t<bf16_t, double, double>(a, rg, median, stream);
  } else if (acc == 1) {
    if (in_dtype == 1) return pre::launch_t<float, float, float>(a, rg, median, stream);
    if (in_dtype == 2) return pre::launch_t<bf16_t, float, float>(a, rg, median, stream);
  } else if (acc == 2) {
    if (in_dtype == 1) return pre::launch_t<float, double, float>(a, rg, median, stream);
    if (in_dtype == 2) return pre::launch_t<bf16_t, double, float>(a, rg, median, stream);
  }
  return hipErrorInvalidValue;
}

}  // namespace dsgm
