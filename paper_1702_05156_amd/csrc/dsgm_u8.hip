// dsgm_u8.hip -- the 8-bit as-run model of the appendix (internal).
//
// The appendix's inner update reads 8-bit frames and keeps each model's mean
// and variance in 8-bit images: the arithmetic is double precision, and every
// value written back is converted to an integer, the fraction dropped (here
// also limited to [0, 255], where the conversion has no defined result).  The
// tests, the swap and the mask then see the stored values.  This kernel runs
// that model time-fused like fwd_kernel: one lane owns P adjacent pixels of a
// row for all T frames with their models in registers (as doubles holding the
// stored integers), and per frame reads P frame bytes and writes P mask bytes.
// The state is 6 bytes per pixel instead of 68, which is what a T = 1
// streaming caller moves per frame; such calls run u8_step_kernel below.
#include "dsgm_ext.h"
#include "dsgm_fwd_impl.h"

namespace dsgm {

namespace u8 {

using fwd::fill_table;
using fwd::ld_stream;
using fwd::make_consts;
using fwd::st_stream;

// the storage rule of an 8-bit image: drop the fraction, limit to [0, 255]
__device__ __forceinline__ double stored(double v) {
  return __builtin_fmin(255.0, __builtin_fmax(0.0, __builtin_trunc(v)));
}

template <int P, bool CODES, bool PRINTED>
__global__ void __launch_bounds__(256) u8_kernel(const FwdArgs a) {
  __shared__ TableEntry<double> tbl[TABLE_SIZE];
  fill_table<double>(tbl, a.weight_rule, a.age_max, a.var_init);  // var_init already stored
  const StepConsts<double> k =
      make_consts<double>(a.theta_s, a.theta_d, a.var_init, a.var_floor, a.mask_floor);

  const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= a.ngroups) return;  // no barrier follows
  const geom::Group G = geom::group_of(g, a.groups_per_row, P, a.W, a.row_stride);
  const int64_t pix = G.soff, foff = G.foff;

  Model<double> s[P];
  {
    const Vec<uint8_t, P> mA = *reinterpret_cast<const Vec<uint8_t, P>*>(
        static_cast<const uint8_t*>(a.mean_a) + pix);
    const Vec<uint8_t, P> vA = *reinterpret_cast<const Vec<uint8_t, P>*>(
        static_cast<const uint8_t*>(a.var_a) + pix);
    const Vec<uint8_t, P> mC = *reinterpret_cast<const Vec<uint8_t, P>*>(
        static_cast<const uint8_t*>(a.mean_c) + pix);
    const Vec<uint8_t, P> vC = *reinterpret_cast<const Vec<uint8_t, P>*>(
        static_cast<const uint8_t*>(a.var_c) + pix);
    const Vec<uint8_t, P> aA = *reinterpret_cast<const Vec<uint8_t, P>*>(a.age_a + pix);
    const Vec<uint8_t, P> aC = *reinterpret_cast<const Vec<uint8_t, P>*>(a.age_c + pix);
#pragma unroll
    for (int q = 0; q < P; ++q) {
      s[q].mA = double(mA.v[q]);
      s[q].vA = double(vA.v[q]);
      s[q].mC = double(mC.v[q]);
      s[q].vC = double(vC.v[q]);
      s[q].aA = aA.v[q];
      s[q].aC = aC.v[q];
    }
  }

  const uint8_t* frames = static_cast<const uint8_t*>(a.frames);
  constexpr int U = 8;  // frames in flight
  auto frame_at = [&](int64_t t) { return ld_stream<uint8_t, P>(frames + t * a.frame_stride + foff); };
  auto do_frame = [&](const Vec<uint8_t, P>& xv, int64_t t) {
    double xs[P];
    StepRecord<double> r[P];
    bool any = false;
#pragma unroll
    for (int q = 0; q < P; ++q) {
      xs[q] = double(xv.v[q]);
      r[q] = step_core<double>(s[q], xs[q], k, tbl);
      // the matched model (or the reset candidate) is written to 8-bit storage;
      // the other models hold stored values already, which the rule keeps
      s[q].mA = stored(s[q].mA);
      s[q].vA = stored(s[q].vA);
      s[q].mC = stored(s[q].mC);
      s[q].vC = stored(s[q].vC);
      any |= r[q].swap;
    }
    if (any_lane(any)) {
#pragma unroll
      for (int q = 0; q < P; ++q) apply_swap<double>(s[q], xs[q], k, r[q].swap);
    }
    Vec<uint8_t, P> mk, cd;
#pragma unroll
    for (int q = 0; q < P; ++q) {
      r[q].fg = fg_of<double, PRINTED>(s[q], xs[q], k);
      mk.v[q] = r[q].fg ? uint8_t(255) : uint8_t(0);
      cd.v[q] = uint8_t(code_of<double>(r[q]));
    }
    const int64_t o = t * a.frame_stride + foff;
    st_stream<uint8_t, P>(a.masks + o, mk);
    if (CODES) *reinterpret_cast<Vec<uint8_t, P>*>(a.codes + o) = cd;
  };
  const int64_t T = a.T;
  int64_t t = 0;
  for (; t + U <= T; t += U) {
    Vec<uint8_t, P> xb[U];
#pragma unroll
    for (int u = 0; u < U; ++u) xb[u] = frame_at(t + u);
#pragma unroll
    for (int u = 0; u < U; ++u) do_frame(xb[u], t + u);
  }
  for (; t < T; ++t) do_frame(frame_at(t), t);

  Vec<uint8_t, P> mA, vA, mC, vC, aA, aC;
#pragma unroll
  for (int q = 0; q < P; ++q) {
    mA.v[q] = uint8_t(s[q].mA);
    vA.v[q] = uint8_t(s[q].vA);
    mC.v[q] = uint8_t(s[q].mC);
    vC.v[q] = uint8_t(s[q].vC);
    aA.v[q] = uint8_t(s[q].aA);
    aC.v[q] = uint8_t(s[q].aC);
  }
  *reinterpret_cast<Vec<uint8_t, P>*>(static_cast<uint8_t*>(a.mean_a) + pix) = mA;
  *reinterpret_cast<Vec<uint8_t, P>*>(static_cast<uint8_t*>(a.var_a) + pix) = vA;
  *reinterpret_cast<Vec<uint8_t, P>*>(static_cast<uint8_t*>(a.mean_c) + pix) = mC;
  *reinterpret_cast<Vec<uint8_t, P>*>(static_cast<uint8_t*>(a.var_c) + pix) = vC;
  *reinterpret_cast<Vec<uint8_t, P>*>(a.age_a + pix) = aA;
  *reinterpret_cast<Vec<uint8_t, P>*>(a.age_c + pix) = aC;
}

// One frame per call (T = 1, the streaming step): a persistent grid whose
// lanes walk pixel groups, each lane loading the next group's frame and state
// bytes before it updates the current group, so the loads of one group overlap
// the arithmetic of the previous one (with one frame per launch there is no
// frame loop to hide them behind).  The table is built once per workgroup,
// while the first group's bytes are on their way.  Bounded to 128 VGPRs, so
// that the whole persistent grid (four workgroups per CU) is resident at once.
template <int P, bool CODES, bool PRINTED>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
u8_step_kernel(const FwdArgs a) {
  __shared__ TableEntry<double> tbl[TABLE_SIZE];
  using V = Vec<uint8_t, P>;
  const uint8_t* frame = static_cast<const uint8_t*>(a.frames);
  uint8_t* const planes[4] = {static_cast<uint8_t*>(a.mean_a), static_cast<uint8_t*>(a.var_a),
                              static_cast<uint8_t*>(a.mean_c), static_cast<uint8_t*>(a.var_c)};
  struct Bytes {
    V x, p[4], aA, aC;
  };
  // group g: row h, first column w (pixel index h*W + w, frame offset h*row_stride + w)
  auto offsets = [&](int64_t g, int64_t& pix, int64_t& foff) {
    const geom::Group G = geom::group_of(g, a.groups_per_row, P, a.W, a.row_stride);
    pix = G.soff;
    foff = G.foff;
  };
  auto load = [&](int64_t g, Bytes& b) {
    int64_t pix, foff;
    offsets(g, pix, foff);
    b.x = ld_stream<uint8_t, P>(frame + foff);
#pragma unroll
    for (int i = 0; i < 4; ++i) b.p[i] = *reinterpret_cast<const V*>(planes[i] + pix);
    b.aA = *reinterpret_cast<const V*>(a.age_a + pix);
    b.aC = *reinterpret_cast<const V*>(a.age_c + pix);
  };
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  Bytes cur, nxt;
  // the first group's bytes are requested before the table is built, so their
  // latency overlaps the table's divisions and its barrier
  if (g < a.ngroups) load(g, cur);
  fill_table<double>(tbl, a.weight_rule, a.age_max, a.var_init);
  const StepConsts<double> k =
      make_consts<double>(a.theta_s, a.theta_d, a.var_init, a.var_floor, a.mask_floor);
  if (g >= a.ngroups) return;  // no barrier follows
  for (; g < a.ngroups; g += stride) {
    const bool more = g + stride < a.ngroups;
    if (more) load(g + stride, nxt);
    Model<double> s[P];
    double xs[P];
    StepRecord<double> r[P];
    bool any = false;
#pragma unroll
    for (int q = 0; q < P; ++q) {
      s[q].mA = double(cur.p[0].v[q]);
      s[q].vA = double(cur.p[1].v[q]);
      s[q].mC = double(cur.p[2].v[q]);
      s[q].vC = double(cur.p[3].v[q]);
      s[q].aA = cur.aA.v[q];
      s[q].aC = cur.aC.v[q];
      xs[q] = double(cur.x.v[q]);
      r[q] = step_core<double>(s[q], xs[q], k, tbl);
      s[q].mA = stored(s[q].mA);
      s[q].vA = stored(s[q].vA);
      s[q].mC = stored(s[q].mC);
      s[q].vC = stored(s[q].vC);
      any |= r[q].swap;
    }
    if (any_lane(any)) {
#pragma unroll
      for (int q = 0; q < P; ++q) apply_swap<double>(s[q], xs[q], k, r[q].swap);
    }
    V mk, cd, o[4], oA, oC;
#pragma unroll
    for (int q = 0; q < P; ++q) {
      r[q].fg = fg_of<double, PRINTED>(s[q], xs[q], k);
      mk.v[q] = r[q].fg ? uint8_t(255) : uint8_t(0);
      cd.v[q] = uint8_t(code_of<double>(r[q]));
      o[0].v[q] = uint8_t(s[q].mA);
      o[1].v[q] = uint8_t(s[q].vA);
      o[2].v[q] = uint8_t(s[q].mC);
      o[3].v[q] = uint8_t(s[q].vC);
      oA.v[q] = uint8_t(s[q].aA);
      oC.v[q] = uint8_t(s[q].aC);
    }
    int64_t pix, foff;
    offsets(g, pix, foff);
    st_stream<uint8_t, P>(a.masks + foff, mk);
    if (CODES) *reinterpret_cast<V*>(a.codes + foff) = cd;
#pragma unroll
    for (int i = 0; i < 4; ++i) *reinterpret_cast<V*>(planes[i] + pix) = o[i];
    *reinterpret_cast<V*>(a.age_a + pix) = oA;
    *reinterpret_cast<V*>(a.age_c + pix) = oC;
    if (more) cur = nxt;
  }
}

// persistent grid of the one-frame kernel: four 256-lane workgroups per CU
// (measured against eight and sixteen on 1920 x 2560 frames: 22.1 us per
// frame against 22.7 and 23.2; a grid of one group per lane took 23.7)
constexpr int64_t kStepGrid = 1024;

template <int P, bool CODES, bool PRINTED>
hipError_t launch_step(const FwdArgs& a, int block, hipStream_t stream) {
  const int64_t need = (a.ngroups + block - 1) / block;
  const dim3 grid{uint32_t(need < kStepGrid ? need : kStepGrid), 1, 1}, blk{uint32_t(block), 1, 1};
  hipLaunchKernelGGL((u8_step_kernel<P, CODES, PRINTED>), grid, blk, 0, stream, a);
  return hipGetLastError();
}

template <int P>
hipError_t launch_p(const FwdArgs& a, int flags, int block, hipStream_t stream) {
  const dim3 grid{uint32_t((a.ngroups + block - 1) / block), 1, 1}, blk{uint32_t(block), 1, 1};
  const bool codes = (flags & FWD_CODES) != 0, printed = (flags & FWD_PRINTED) != 0;
  if (a.T == 1) {
    if (codes && printed) return launch_step<P, true, true>(a, block, stream);
    if (codes) return launch_step<P, true, false>(a, block, stream);
    if (printed) return launch_step<P, false, true>(a, block, stream);
    return launch_step<P, false, false>(a, block, stream);
  }
  if (codes && printed) hipLaunchKernelGGL((u8_kernel<P, true, true>), grid, blk, 0, stream, a);
  else if (codes) hipLaunchKernelGGL((u8_kernel<P, true, false>), grid, blk, 0, stream, a);
  else if (printed) hipLaunchKernelGGL((u8_kernel<P, false, true>), grid, blk, 0, stream, a);
  else hipLaunchKernelGGL((u8_kernel<P, false, false>), grid, blk, 0, stream, a);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256) u8_init_kernel(const FwdArgs a) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.H * a.W) return;
  const int64_t h = i / a.W, w = i - h * a.W;
  const uint8_t x = static_cast<const uint8_t*>(a.frames)[h * a.row_stride + w];
  const uint8_t v = uint8_t(stored(a.var_init));
  static_cast<uint8_t*>(a.mean_a)[i] = x;
  static_cast<uint8_t*>(a.mean_c)[i] = x;
  static_cast<uint8_t*>(a.var_a)[i] = v;
  static_cast<uint8_t*>(a.var_c)[i] = v;
  a.age_a[i] = 1;
  a.age_c[i] = 1;
}

// The appendix's preprocessing as it runs on 8-bit frames, fused into the
// 8-bit update (one pass over the sequence, like pre_kernel): a workgroup owns
// a 16 x 64 tile for all frames, each lane four adjacent pixels of one row
// with their models in registers.  Per frame it stages the tile's raw bytes
// plus a halo of RG + 1 rows and columns in LDS (indices clamped to the frame),
// computes every blurred byte of the tile and of the median's halo with the
// two-dimensional single-precision sum of the appendix's blur (window rows
// outer, columns inner, weights float(w_i * w_j), every product and sum
// rounded, no fused multiply-add), drops its fraction (limited to 255), takes
// each pixel's median of the nine blurred bytes around it and runs the 8-bit
// update on it.  Two barriers per frame: after the raw bytes are staged and
// after the blurred bytes are written; the next frame's bytes are loaded into
// registers while the current one is filtered.  All tile cell indices come
// from geom::pre::Geo.
template <int RG, bool MED, bool PRINTED>
__global__ void __launch_bounds__(geom::pre::NT) pre_u8_kernel(const PreArgs a) {
  using G = geom::pre::Geo<RG, MED>;
  constexpr int PX = geom::pre::PX, TH = geom::pre::TH, TW = geom::pre::TW;
  constexpr int N = 2 * RG + 1;  // taps per window row
  __shared__ float buf_raw[G::RAW_N];
  __shared__ float buf_gb[RG > 0 ? G::GB_N : 1];
  __shared__ TableEntry<double> tbl[TABLE_SIZE];
  fill_table<double>(tbl, a.weight_rule, a.age_max, a.var_init);  // var_init already stored
  const StepConsts<double> k =
      make_consts<double>(a.theta_s, a.theta_d, a.var_init, a.var_floor, a.mask_floor);
  float w2[N * N];  // the window's weights, row-major, rounded once
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) w2[i * N + j] = float(a.w[i] * a.w[j]);

  const int64_t tile = tile_of(blockIdx.x, gridDim.x);
  const int64_t y0 = (tile / a.tiles_x) * TH, x0 = (tile % a.tiles_x) * TW;
  const int tid = threadIdx.x;
  const int ty = G::lane_row(tid), tx = G::lane_col(tid);
  const int64_t gy = y0 + ty;

  uint32_t roff[G::LOADS];  // frame offsets of this lane's raw cells (fixed per frame)
#pragma unroll
  for (int l = 0; l < G::LOADS; ++l) {
    const int i = G::raw_cell(tid, l);
    roff[l] = i < G::RAW_N ? uint32_t(G::raw_source(i, y0, x0, a.H, a.W, a.row_stride)) : 0u;
  }
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
  const int64_t pix = gy * a.W + x0 + tx;
  const int64_t foff = gy * a.row_stride + x0 + tx;
  const bool vec_ok = all_valid && (a.row_stride % PX) == 0 && (a.frame_stride % PX) == 0 &&
                      (a.W % PX) == 0;

  const uint8_t* const planes_in[4] = {static_cast<const uint8_t*>(a.mean_a),
                                       static_cast<const uint8_t*>(a.var_a),
                                       static_cast<const uint8_t*>(a.mean_c),
                                       static_cast<const uint8_t*>(a.var_c)};
  Model<double> s[PX];
#pragma unroll
  for (int q = 0; q < PX; ++q) {
    if (valid[q]) {
      s[q].mA = double(planes_in[0][pix + q]);
      s[q].vA = double(planes_in[1][pix + q]);
      s[q].mC = double(planes_in[2][pix + q]);
      s[q].vC = double(planes_in[3][pix + q]);
      s[q].aA = a.age_a[pix + q];
      s[q].aC = a.age_c[pix + q];
    } else {
      s[q].mA = s[q].vA = s[q].mC = s[q].vC = 0.0;
      s[q].aA = s[q].aC = 1;
    }
  }

  const uint8_t* frames = static_cast<const uint8_t*>(a.frames);
  uint8_t nxt[G::LOADS];
  auto load_frame = [&](int64_t t) {
    const uint8_t* f = frames + t * a.frame_stride;
#pragma unroll
    for (int l = 0; l < G::LOADS; ++l)
      if (G::raw_active(tid, l)) nxt[l] = f[roff[l]];
  };
  if (a.T > 0) load_frame(0);

  for (int64_t t = 0; t < a.T; ++t) {
    // 1. stage the raw bytes, then start loading the next frame's
#pragma unroll
    for (int l = 0; l < G::LOADS; ++l)
      if (G::raw_active(tid, l)) buf_raw[G::raw_cell(tid, l)] = float(nxt[l]);
    __syncthreads();
    if (t + 1 < a.T) load_frame(t + 1);

    const float* gbp;
    if constexpr (RG > 0) {
      // 2. the blurred bytes of the tile and the median's halo
#pragma unroll
      for (int it = 0; it < G::GB_IT; ++it) {
        if (G::gb_active(tid, it)) {
          const int cell = G::gb_cell(tid, it);
          const float* win = buf_raw + G::blur_window(cell);
          float blur = 0.0f;
#pragma unroll
          for (int i = 0; i < N; ++i)
#pragma unroll
            for (int j = 0; j < N; ++j) {
              const float prod = win[i * G::RAW_W + j] * w2[i * N + j];
              blur = blur + prod;
            }
          buf_gb[cell] = __builtin_fminf(255.0f, __builtin_fmaxf(0.0f, __builtin_truncf(blur)));
        }
      }
      __syncthreads();
      gbp = buf_gb;
    } else {
      gbp = buf_raw;  // no blur: the raw bytes are the blurred ones (R = RM)
    }
    constexpr int GW = RG > 0 ? G::GB_W : G::RAW_W;

    // 3. each pixel's median of the nine blurred bytes (exact in single
    // precision: the values are integers), then the 8-bit update
    double xs[PX];
    if constexpr (MED) {
      float lo[PX + 2], md[PX + 2], hi[PX + 2];
#pragma unroll
      for (int d = 0; d < PX + 2; ++d) {
        const float p0 = gbp[gr[0] * GW + gc[d]];
        const float p1 = gbp[gr[1] * GW + gc[d]];
        const float p2 = gbp[gr[2] * GW + gc[d]];
        const float l01 = __builtin_fminf(p0, p1), h01 = __builtin_fmaxf(p0, p1);
        lo[d] = __builtin_fminf(l01, p2);
        const float h = __builtin_fmaxf(l01, p2);
        hi[d] = __builtin_fmaxf(h01, h);
        md[d] = __builtin_fminf(h01, h);
      }
#pragma unroll
      for (int q = 0; q < PX; ++q) {
        const float a0 = __builtin_fmaxf(__builtin_fmaxf(lo[q], lo[q + 1]), lo[q + 2]);
        const float b0 = __builtin_fmaxf(__builtin_fminf(md[q], md[q + 1]),
                                         __builtin_fminf(__builtin_fmaxf(md[q], md[q + 1]), md[q + 2]));
        const float c0 = __builtin_fminf(__builtin_fminf(hi[q], hi[q + 1]), hi[q + 2]);
        xs[q] = double(__builtin_fmaxf(__builtin_fminf(a0, b0),
                                       __builtin_fminf(__builtin_fmaxf(a0, b0), c0)));
      }
    } else {
#pragma unroll
      for (int q = 0; q < PX; ++q) xs[q] = double(gbp[gr[1] * GW + gc[q + 1]]);
    }

    StepRecord<double> r[PX];
    bool any = false;
#pragma unroll
    for (int q = 0; q < PX; ++q) {
      r[q] = step_core<double>(s[q], xs[q], k, tbl);
      s[q].mA = stored(s[q].mA);
      s[q].vA = stored(s[q].vA);
      s[q].mC = stored(s[q].mC);
      s[q].vC = stored(s[q].vC);
      any |= r[q].swap;
    }
    if (any_lane(any)) {
#pragma unroll
      for (int q = 0; q < PX; ++q) apply_swap<double>(s[q], xs[q], k, r[q].swap);
    }
    Vec<uint8_t, PX> mk, cd, fv;
#pragma unroll
    for (int q = 0; q < PX; ++q) {
      r[q].fg = fg_of<double, PRINTED>(s[q], xs[q], k);
      mk.v[q] = r[q].fg ? uint8_t(255) : uint8_t(0);
      cd.v[q] = uint8_t(code_of<double>(r[q]));
      fv.v[q] = uint8_t(xs[q]);
    }
    uint8_t* const filt = static_cast<uint8_t*>(a.filtered);
    const int64_t o = t * a.frame_stride + foff;
    if (vec_ok) {
      *reinterpret_cast<Vec<uint8_t, PX>*>(a.masks + o) = mk;
      if (filt) *reinterpret_cast<Vec<uint8_t, PX>*>(filt + o) = fv;
      if (a.codes) *reinterpret_cast<Vec<uint8_t, PX>*>(a.codes + o) = cd;
    } else {
#pragma unroll
      for (int q = 0; q < PX; ++q) {
        if (!valid[q]) continue;
        a.masks[o + q] = mk.v[q];
        if (filt) filt[o + q] = fv.v[q];
        if (a.codes) a.codes[o + q] = cd.v[q];
      }
    }
    if constexpr (RG == 0) __syncthreads();  // the next frame overwrites the raw bytes
  }

#pragma unroll
  for (int q = 0; q < PX; ++q) {
    if (!valid[q]) continue;
    static_cast<uint8_t*>(a.mean_a)[pix + q] = uint8_t(s[q].mA);
    static_cast<uint8_t*>(a.var_a)[pix + q] = uint8_t(s[q].vA);
    static_cast<uint8_t*>(a.mean_c)[pix + q] = uint8_t(s[q].mC);
    static_cast<uint8_t*>(a.var_c)[pix + q] = uint8_t(s[q].vC);
    a.age_a[pix + q] = uint8_t(s[q].aA);
    a.age_c[pix + q] = uint8_t(s[q].aC);
  }
}

template <bool MED, bool PRINTED>
hipError_t launch_pre_rg(const PreArgs& a, int rg, hipStream_t stream) {
  const dim3 grid{uint32_t(a.tiles_x * a.tiles_y), 1, 1}, block{geom::pre::NT, 1, 1};
  switch (rg) {
    case 0: hipLaunchKernelGGL((pre_u8_kernel<0, MED, PRINTED>), grid, block, 0, stream, a); break;
    case 1: hipLaunchKernelGGL((pre_u8_kernel<1, MED, PRINTED>), grid, block, 0, stream, a); break;
    case 2: hipLaunchKernelGGL((pre_u8_kernel<2, MED, PRINTED>), grid, block, 0, stream, a); break;
    case 3: hipLaunchKernelGGL((pre_u8_kernel<3, MED, PRINTED>), grid, block, 0, stream, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace u8

hipError_t launch_fwd_u8(const FwdArgs& a, int P, int flags, int block, hipStream_t stream) {
  if (flags & (FWD_BG | FWD_CKPT)) return hipErrorInvalidValue;
  if (P == 4) return u8::launch_p<4>(a, flags, block, stream);
  if (P == 2) return u8::launch_p<2>(a, flags, block, stream);
  if (P == 1) return u8::launch_p<1>(a, flags, block, stream);
  return hipErrorInvalidValue;
}

hipError_t launch_pre_u8(const PreArgs& a, int rg, bool median, hipStream_t stream) {
  const bool printed = a.mask_rule != 0;
  if (median)
    return printed ? u8::launch_pre_rg<true, true>(a, rg, stream)
                   : u8::launch_pre_rg<true, false>(a, rg, stream);
  return printed ? u8::launch_pre_rg<false, true>(a, rg, stream)
                 : u8::launch_pre_rg<false, false>(a, rg, stream);
}

hipError_t launch_init_u8(const FwdArgs& a, hipStream_t stream) {
  const int64_t n = a.H * a.W;
  hipLaunchKernelGGL(u8::u8_init_kernel, dim3(uint32_t((n + 255) / 256)), dim3(256), 0, stream, a);
  return hipGetLastError();
}

}  // namespace dsgm
