// dsgm_warp.hip -- one frame of the update on the motion-compensated model
// (internal).
//
// Sec. 2.2 updates the model from its previous values "after motion
// compensation"; Sec. 2.4 notes that with a per-pixel model the camera's
// homography simply maps the model values to the pixels they now belong to.
// This kernel does both steps of one frame in one pass: each lane takes one
// pixel of the current frame, maps it through the caller's 3 x 3 matrix to
// its position in the previous frame, gathers the previous model there
// (bilinear means and variances from the four surrounding pixels, the
// nearest pixel's ages; a pixel mapped outside the previous frame restarts
// from the current intensity), then runs the update and writes the mask and
// the new model to a second set of planes.  The gathers of neighbouring lanes
// hit neighbouring addresses, so they coalesce when the motion is smooth.
//
// With FP64 state the coordinates, weights and blends are evaluated with
// every product and sum rounded in the order of a scalar evaluation.
#include "dsgm_ext.h"
#include "dsgm_fwd_impl.h"

namespace dsgm {

namespace warp {

using fwd::fill_table;
using fwd::make_consts;

// weighted sum of four values in the stated order (no contraction for double)
__device__ __forceinline__ double bilin(double w00, double a, double w10, double b, double w01,
                                        double c, double w11, double d) {
  return ((w00 * a + w10 * b) + w01 * c) + w11 * d;
}
__device__ __forceinline__ float bilin(float w00, float a, float w10, float b, float w01, float c,
                                       float w11, float d) {
  return __builtin_fmaf(w11, d, __builtin_fmaf(w01, c, __builtin_fmaf(w10, b, w00 * a)));
}

// two adjacent elements from one load; the address needs only element
// alignment (the hardware serves multi-dword loads at dword alignment)
template <typename Acc>
struct Pair {
  Acc x, y;
};
template <typename Acc>
__device__ __forceinline__ Pair<Acc> ld_pair(const Acc* p) {
  typedef Acc V __attribute__((ext_vector_type(2), aligned(sizeof(Acc))));
  const V v = *reinterpret_cast<const V*>(p);
  return Pair<Acc>{v.x, v.y};
}

template <typename In, typename Acc, typename Io>
__global__ void __launch_bounds__(256) warp_kernel(const WarpArgs a) {
  __shared__ TableEntry<Acc> tbl[TABLE_SIZE];

  // consecutive rows go to the same XCD, whose L2 then serves the source rows
  // that neighbouring output rows share
  const int64_t i = tile_of(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const bool active = i < a.H * a.W;
  const int64_t y = active ? i / a.W : 0, c = active ? i - y * a.W : 0;
  const int64_t fo = y * a.row_stride + c;  // frame / output offset

  // The frame value, the source position (dsgm_geom.h) and the gathers are
  // requested before the table is built, so that their latency overlaps the
  // table's divisions and barrier.  Per state plane, the top and bottom
  // source rows' two neighbours: one pair load per row at columns xa, xa + 1
  // (xa = x0 except on the last column, where both neighbours are x0); a
  // one-column frame loads its single neighbour into both halves.
  In xin = In();
  geom::WarpSrc src;
  src.covered = false;
  Pair<Acc> top[4], bot[4];
  bool lo = true;
  uint8_t age_a = 1, age_c = 1;
  const Acc* const planes[4] = {static_cast<const Acc*>(a.src_mean_a),
                                static_cast<const Acc*>(a.src_var_a),
                                static_cast<const Acc*>(a.src_mean_c),
                                static_cast<const Acc*>(a.src_var_c)};
  if (active) {
    xin = static_cast<const In*>(a.frame)[fo];
    src = geom::warp_source(c, y, a.map, a.H, a.W);
    if (src.covered) {
      if (a.W >= 2) {
        lo = src.xa == src.x0;
        const int64_t r0 = src.y0 * a.W + src.xa, r1 = src.y1 * a.W + src.xa;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          top[j] = ld_pair(planes[j] + r0);
          bot[j] = ld_pair(planes[j] + r1);
        }
      } else {
        const int64_t r0 = src.y0, r1 = src.y1;  // W = 1: x0 = x1 = 0
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const Acc t = planes[j][r0], b = planes[j][r1];
          top[j] = Pair<Acc>{t, t};
          bot[j] = Pair<Acc>{b, b};
        }
      }
      age_a = a.src_age_a[src.yn * a.W + src.xn];
      age_c = a.src_age_c[src.yn * a.W + src.xn];
    }
  }
  fill_table<Acc>(tbl, a.weight_rule, a.age_max, a.var_init);
  const StepConsts<Acc> k =
      make_consts<Acc>(a.theta_s, a.theta_d, a.var_init, a.var_floor, a.mask_floor);
  if (!active) return;  // no barrier follows
  const Acc x = to_acc<In, Acc>(xin);

  Model<Acc> s;
  if (src.covered) {
    const double fx = src.fx, fy = src.fy;
    const Acc w00 = Acc((1.0 - fx) * (1.0 - fy)), w10 = Acc(fx * (1.0 - fy));
    const Acc w01 = Acc((1.0 - fx) * fy), w11 = Acc(fx * fy);
    Acc g[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const Pair<Acc> t = top[j], b = bot[j];
      g[j] = bilin(w00, lo ? t.x : t.y, w10, t.y, w01, lo ? b.x : b.y, w11, b.y);
    }
    s.mA = g[0];
    s.vA = g[1];
    s.mC = g[2];
    s.vC = g[3];
    s.aA = age_a;
    s.aC = age_c;
  } else {
    s.mA = s.mC = x;
    s.vA = s.vC = k.var_init;
    s.aA = s.aC = 1;
  }

  StepRecord<Acc> r = step_core<Acc>(s, x, k, tbl);
  if (any_lane(r.swap)) apply_swap<Acc>(s, x, k, r.swap);
  r.fg = a.mask_rule != 0 ? fg_of<Acc, true>(s, x, k) : fg_of<Acc, false>(s, x, k);

  a.masks[fo] = r.fg ? uint8_t(255) : uint8_t(0);
  if (a.bg) static_cast<Io*>(a.bg)[fo] = Io(s.mA);
  if (a.codes) a.codes[fo] = uint8_t(code_of<Acc>(r));
  static_cast<Acc*>(a.dst_mean_a)[i] = s.mA;
  static_cast<Acc*>(a.dst_var_a)[i] = s.vA;
  static_cast<Acc*>(a.dst_mean_c)[i] = s.mC;
  static_cast<Acc*>(a.dst_var_c)[i] = s.vC;
  a.dst_age_a[i] = uint8_t(s.aA);
  a.dst_age_c[i] = uint8_t(s.aC);
}

template <typename In, typename Acc, typename Io>
hipError_t launch_t(const WarpArgs& a, hipStream_t stream) {
  const int64_t n = a.H * a.W;
  const dim3 grid{uint32_t((n + 255) / 256), 1, 1}, block{256, 1, 1};
  hipLaunchKernelGGL((warp_kernel<In, Acc, Io>), grid, block, 0, stream, a);
  return hipGetLastError();
}

}  // namespace warp

hipError_t launch_warp(const WarpArgs& a, int in_dtype, int acc, hipStream_t stream) {
  if (acc == 0) {
    if (in_dtype == 0) return warp::launch_t<double, double, double>(a, stream);
    if (in_dtype == 1) return warp::launch_t<float, double, double>(a, stream);
    if (in_dtype == 2) return warp::launch_t<bf16_t, double, double>(a, stream);
  } else if (acc == 1) {
    if (in_dtype == 1) return warp::launch_t<float, float, float>(a, stream);
    if (in_dtype == 2) return warp::launch_t<bf16_t, float, float>(a, stream);
  } else if (acc == 2) {
    if (in_dtype == 1) return warp::launch_t<float, double, float>(a, stream);
    if (in_dtype == 2) return warp::launch_t<bf16_t, double, float>(a, stream);
  }
  return hipErrorInvalidValue;
}

}  // namespace dsgm
