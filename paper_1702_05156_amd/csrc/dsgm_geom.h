// dsgm_geom.h -- launch geometry of the kernels (internal).
//
// Which pixels a lane owns, and which frame elements, checkpoint slots,
// tile cells and source pixels it touches, as functions of its workgroup and
// lane indices.  The kernels compute their indices with these functions, and
// the host-side extent checker of the test suite walks every lane of a launch
// through the same functions to show that each access stays inside its buffer
// and that each pixel is owned by exactly one lane.  Everything here is plain
// integer (and, for the motion-compensated update's source position, IEEE
// double) arithmetic that gives the same results on the host and the device.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dsgm {
namespace geom {

#define DSGM_HD __host__ __device__ __forceinline__

DSGM_HD int64_t pad_to(int64_t b, int64_t a) { return (b + a - 1) / a * a; }
DSGM_HD int64_t pad256(int64_t b) { return pad_to(b, 256); }
DSGM_HD int64_t min64(int64_t a, int64_t b) { return a < b ? a : b; }
DSGM_HD int64_t clamp64(int64_t v, int64_t hi) { return v < 0 ? 0 : (v > hi ? hi : v); }

// Logical tile of workgroup b of nb: the hardware deals workgroups to the 8
// XCDs round-robin (b mod 8), each XCD with its own L2; this bijection gives
// XCD k the k-th contiguous share of the tiles, so tiles that share input rows
// (stencil halos, the source rows of a warp) meet in the same L2.
DSGM_HD int64_t tile_of(int64_t b, int64_t nb) {
  const int64_t k = b % 8, i = b / 8, q = nb / 8, rem = nb % 8;
  return k < rem ? k * (q + 1) + i : rem * (q + 1) + (k - rem) * q + i;
}

// ------------------------------------------------- lane groups (time-fused)
// Group g of a frame cut into groups of P horizontally adjacent pixels
// (W is a multiple of P): its row, first column, pixel index of its first
// pixel in the dense state planes and element offset within a frame.
struct Group {
  int64_t h, w0, soff, foff;
};
DSGM_HD Group group_of(int64_t g, int64_t groups_per_row, int P, int64_t W, int64_t row_stride) {
  Group r;
  r.h = g / groups_per_row;
  r.w0 = (g - r.h * groups_per_row) * P;
  r.soff = r.h * W + r.w0;
  r.foff = r.h * row_stride + r.w0;
  return r;
}

// ------------------------------------------------------------- checkpoints
// One slot holds the state of every pixel before frame s*K: four float planes
// and two age planes, each padded to 256 bytes.  The forward writes slots
// 0 .. ckpt_slots(T, K) - 1; the backward reads them.
struct CkptLayout {
  int64_t fplane, aplane, slot;
};
DSGM_HD CkptLayout ckpt_layout(int64_t px, int64_t acc_bytes) {
  CkptLayout c;
  c.fplane = pad256(px * acc_bytes);
  c.aplane = pad256(px);
  c.slot = 4 * c.fplane + 2 * c.aplane;
  return c;
}
DSGM_HD int64_t ckpt_slots(int64_t T, int64_t K) { return (T + K - 1) / K; }

// -------------------------------------------------- backward segments/chunks
// The reverse sweep takes the segments [seg*K, min((seg+1)*K, T)) from last
// to first and, within one, chunks of at most KC frames from last to first.
struct Range {
  int64_t lo, hi;
};
DSGM_HD int64_t n_segments(int64_t T, int64_t K) { return (T + K - 1) / K; }
DSGM_HD Range segment(int64_t seg, int64_t T, int64_t K) {
  Range r;
  r.lo = seg * K;
  r.hi = min64(r.lo + K, T);
  return r;
}
DSGM_HD int64_t n_chunks(Range s, int KC) { return (s.hi - s.lo + KC - 1) / KC; }
DSGM_HD Range chunk(Range s, int64_t c, int KC) {
  Range r;
  r.lo = s.lo + c * KC;
  r.hi = min64(r.lo + KC, s.hi);
  return r;
}

// The backward's workspace: one FP64 term per pixel for d/d var_init, then
// the reduction's per-block (sum, compensation) pairs.
constexpr int REDUCE_BLOCKS = 256;
DSGM_HD int64_t ws_partial_offset(int64_t px) { return pad256(px * 8); }
DSGM_HD int64_t ws_bytes(int64_t px) { return ws_partial_offset(px) + 2 * REDUCE_BLOCKS * 8; }

// ------------------------------------------------------------ batched items
// An item is up to 64 consecutive lane groups of one instance (one
// wavefront's work); its foreground counts go to one of COUNT_STRIPES
// stripes of T counters, chosen by the item's position in the queue.
constexpr int64_t ITEM_GROUPS = 64;
constexpr int64_t COUNT_STRIPES = 256;
DSGM_HD int64_t stripe_of(uint64_t item) { return int64_t(item % uint64_t(COUNT_STRIPES)); }

// ------------------------------------------------ fused preprocessing tiles
// A workgroup of NT lanes owns a TH x TW tile for all frames, each lane PX
// horizontally adjacent pixels of one row.  Per frame it stages the tile plus
// a halo of R = RG + RM raw rows and columns (indices clamped to the frame),
// blurs rows into HB (all raw rows, the median's halo columns), then columns
// into GB (the median's halo rows and columns), and takes each pixel's 3 x 3
// median from GB.  Every tile cell index below is into one of those arrays.
namespace pre {
constexpr int TH = 16;   // tile rows
constexpr int TW = 64;   // tile columns
constexpr int PX = 4;    // pixels per lane (one row)
constexpr int NT = 256;  // lanes per workgroup
static_assert(TH * TW == NT * PX, "tile = lanes x pixels");

template <int RG, bool MED>
struct Geo {
  static constexpr int RM = MED ? 1 : 0;       // median radius
  static constexpr int R = RG + RM;            // halo of the raw tile
  static constexpr int RAW_H = TH + 2 * R, RAW_W = TW + 2 * R;
  static constexpr int HB_W = TW + 2 * RM;     // row-blurred: all raw rows, median halo columns
  static constexpr int GB_H = TH + 2 * RM, GB_W = TW + 2 * RM;
  static constexpr int RAW_N = RAW_H * RAW_W;
  static constexpr int HB_N = RAW_H * HB_W;
  static constexpr int GB_N = GB_H * GB_W;
  static constexpr int LOADS = (RAW_N + NT - 1) / NT;  // raw elements per lane
  static constexpr int ROW_IT = (HB_N / 2 + NT - 1) / NT;  // row-pass output pairs per lane
  static constexpr int COL_IT = (GB_N / 2 + NT - 1) / NT;  // column-pass output pairs per lane
  static constexpr int GB_IT = (GB_N + NT - 1) / NT;  // 2-D blur cells per lane (8-bit form)

  // the raw cell a lane stages in its l-th load, and whether it has one
  DSGM_HD static int raw_cell(int tid, int l) { return tid + l * NT; }
  DSGM_HD static bool raw_active(int tid, int l) { return l + 1 < LOADS || raw_cell(tid, l) < RAW_N; }
  // the frame element of raw cell i of the tile at (y0, x0), clamped
  DSGM_HD static int64_t raw_source(int i, int64_t y0, int64_t x0, int64_t H, int64_t W,
                                    int64_t row_stride) {
    const int r = i / RAW_W, c = i - r * RAW_W;
    const int64_t yy = clamp64(y0 - R + r, H - 1), xx = clamp64(x0 - R + c, W - 1);
    return yy * row_stride + xx;
  }
  // the it-th output pair of the row pass: HB cells 2*pair, 2*pair + 1 from
  // the raw window starting at row_window (2*RG + 2 cells)
  DSGM_HD static int row_pair(int tid, int it) { return tid + it * NT; }
  DSGM_HD static bool row_active(int tid, int it) {
    return it + 1 < ROW_IT || row_pair(tid, it) < HB_N / 2;
  }
  DSGM_HD static int row_window(int pair) {
    const int r = pair / (HB_W / 2), v = 2 * (pair - r * (HB_W / 2));
    return r * RAW_W + v;
  }
  // the it-th output pair of the column pass: GB cells 2*pair, 2*pair + 1 from
  // HB cells 2*pair + j*HB_W (+1), j < 2*RG + 1 (the two arrays share a width)
  DSGM_HD static int col_pair(int tid, int it) { return tid + it * NT; }
  DSGM_HD static bool col_active(int tid, int it) {
    return it + 1 < COL_IT || col_pair(tid, it) < GB_N / 2;
  }
  // the it-th cell of the two-dimensional blur (the 8-bit form): GB cell
  // `cell` from the (2*RG + 1) x (2*RG + 1) raw window whose top-left cell is
  // blur_window(cell) (GB cell (r, c) is frame pixel (y0 - RM + r, x0 - RM + c),
  // whose window starts at raw cell (r, c))
  DSGM_HD static int gb_cell(int tid, int it) { return tid + it * NT; }
  DSGM_HD static bool gb_active(int tid, int it) { return it + 1 < GB_IT || gb_cell(tid, it) < GB_N; }
  DSGM_HD static int blur_window(int cell) {
    const int r = cell / GB_W, c = cell - r * GB_W;
    return r * RAW_W + c;
  }
  // the lane's row and first column in the tile
  DSGM_HD static int lane_row(int tid) { return tid / (TW / PX); }
  DSGM_HD static int lane_col(int tid) { return (tid % (TW / PX)) * PX; }
  // the median's rows (d < 3) and columns (d < PX + 2) in GB for the lane at
  // frame row gy, first column gx, clamped to the frame
  DSGM_HD static int med_row(int64_t gy, int d, int64_t y0, int64_t H) {
    return int(clamp64(gy + d - 1, H - 1) - (y0 - RM));
  }
  DSGM_HD static int med_col(int64_t gx, int d, int64_t x0, int64_t W) {
    return int(clamp64(gx + d - 1, W - 1) - (x0 - RM));
  }
};
}  // namespace pre

// ------------------------------------------- motion-compensated source pixel
// Where output pixel (c, y) of an H x W frame reads the previous state under
// the 3 x 3 homography `map` (row-major, output -> source): the bilinear
// neighbours (x0|x1, y0|y1), the column xa of the pair load that serves both
// columns of a row, and the nearest pixel (xn, yn) for the ages.  Outside
// the source frame (or behind the camera) nothing is read.
struct WarpSrc {
  bool covered;
  double fx, fy;  // bilinear fractions
  int64_t x0, y0, x1, y1, xa, xn, yn;
};
DSGM_HD WarpSrc warp_source(int64_t c, int64_t y, const double* map, int64_t H, int64_t W) {
  WarpSrc s;
  const double xd = double(c), yd = double(y);
  const double den = (map[6] * xd + map[7] * yd) + map[8];
  const double qx = ((map[0] * xd + map[1] * yd) + map[2]) / den;
  const double qy = ((map[3] * xd + map[4] * yd) + map[5]) / den;
  s.covered = den > 0.0 && qx >= 0.0 && qx <= double(W - 1) && qy >= 0.0 && qy <= double(H - 1);
  s.fx = s.fy = 0.0;
  s.x0 = s.y0 = s.x1 = s.y1 = s.xa = s.xn = s.yn = 0;
  if (s.covered) {
    const double fx0 = floor(qx), fy0 = floor(qy);
    s.fx = qx - fx0;
    s.fy = qy - fy0;
    s.x0 = int64_t(fx0);
    s.y0 = int64_t(fy0);
    s.x1 = s.x0 + 1 < W ? s.x0 + 1 : W - 1;
    s.y1 = s.y0 + 1 < H ? s.y0 + 1 : H - 1;
    s.xa = s.x0 < W - 1 ? s.x0 : W - 2;  // used when W >= 2
    s.xn = int64_t(floor(qx + 0.5));
    s.yn = int64_t(floor(qy + 0.5));
    s.xn = s.xn > W - 1 ? W - 1 : s.xn;
    s.yn = s.yn > H - 1 ? H - 1 : s.yn;
  }
  return s;
}

// ------------------------------------------------------- grid model blocks
// Block blk of the B x B grid over an H x W frame (Wb blocks per row): its
// top-left pixel and its rows and columns (fewer on the bottom and right
// edges).
struct GridBlock {
  int64_t y0, x0;
  int rows, cols;
};
DSGM_HD GridBlock grid_block(int64_t blk, int64_t Wb, int B, int64_t H, int64_t W) {
  GridBlock b;
  const int64_t by = blk / Wb, bx = blk - by * Wb;
  b.y0 = by * B;
  b.x0 = bx * B;
  b.rows = int(H - b.y0 < B ? H - b.y0 : B);
  b.cols = int(W - b.x0 < B ? W - b.x0 : B);
  return b;
}

#undef DSGM_HD

}  // namespace geom
}  // namespace dsgm
