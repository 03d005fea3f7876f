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
  fill_table<Acc>(tbl, a.weight_rule, a.age_max, a.var_init);
  const StepConsts<Acc> k =
      make_consts<Acc>(a.theta_s, a.theta_d, a.var_init, a.var_floor, a.mask_floor);

  // consecutive rows go to the same XCD, whose L2 then serves the source rows
  // that neighbouring output rows share
  const int64_t i = tile_of(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (i >= a.H * a.W) return;  // no barrier follows
  const int64_t y = i / a.W, c = i - y * a.W;
  const int64_t fo = y * a.row_stride + c;  // frame / output offset
  const Acc x = to_acc<In, Acc>(static_cast<const In*>(a.frame)[fo]);

  // the source position and its neighbours (dsgm_geom.h)
  const geom::WarpSrc src = geom::warp_source(c, y, a.map, a.H, a.W);
  Model<Acc> s;
  if (src.covered) {
    const double fx = src.fx, fy = src.fy;
    const int64_t x0 = src.x0, y0 = src.y0, x1 = src.x1, y1 = src.y1;
    const Acc w00 = Acc((1.0 - fx) * (1.0 - fy)), w10 = Acc(fx * (1.0 - fy));
    const Acc w01 = Acc((1.0 - fx) * fy), w11 = Acc(fx * fy);
    const Acc* mA = static_cast<const Acc*>(a.src_mean_a);
    const Acc* vA = static_cast<const Acc*>(a.src_var_a);
    const Acc* mC = static_cast<const Acc*>(a.src_mean_c);
    const Acc* vC = static_cast<const Acc*>(a.src_var_c);
    if (a.W >= 2) {
      // each row's two neighbours come from one pair load at columns xa, xa+1
      // (xa = x0 except on the last column, where both neighbours are x0)
      const int64_t xa = src.xa;
      const bool lo = xa == x0;
      const int64_t r0 = y0 * a.W + xa, r1 = y1 * a.W + xa;
      auto gather = [&](const Acc* p) {
        const Pair<Acc> t = ld_pair(p + r0), b = ld_pair(p + r1);
        return bilin(w00, lo ? t.x : t.y, w10, t.y, w01, lo ? b.x : b.y, w11, b.y);
      };
      s.mA = gather(mA);
      s.vA = gather(vA);
      s.mC = gather(mC);
      s.vC = gather(vC);
    } else {
      const int64_t i00 = y0 * a.W + x0, i10 = y0 * a.W + x1, i01 = y1 * a.W + x0,
                    i11 = y1 * a.W + x1;
      s.mA = bilin(w00, mA[i00], w10, mA[i10], w01, mA[i01], w11, mA[i11]);
      s.vA = bilin(w00, vA[i00], w10, vA[i10], w01, vA[i01], w11, vA[i11]);
      s.mC = bilin(w00, mC[i00], w10, mC[i10], w01, mC[i01], w11, mC[i11]);
      s.vC = bilin(w00, vC[i00], w10, vC[i10], w01, vC[i01], w11, vC[i11]);
    }
    s.aA = a.src_age_a[src.yn * a.W + src.xn];
    s.aC = a.src_age_c[src.yn * a.W + src.xn];
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
