// Host-side extent checker of the kernels' launch geometry (built and run by
// tests/test_geometry.py on the CPU; no GPU call is made).
//
// Every kernel of libdsgm.so computes which pixels a lane owns and which
// elements, checkpoint slots, tile cells and source pixels it touches with
// the functions of csrc/dsgm_geom.h.  This program walks every workgroup and
// lane of each launch, as the launchers size it, through the same functions
// for many shapes (ragged, strided, smaller than one tile, one row, one
// column, frame counts that are not multiples of the tape or the checkpoint
// interval), and checks:
//   * each access stays inside the buffer the library's own size rules give
//     (frame extent, state planes, dsgm_ckpt_bytes, dsgm_workspace_bytes,
//     dsgm_batch_plan_bytes, the LDS arrays of a tile);
//   * each pixel (or block, or work group) is owned by exactly one lane;
//   * the reverse sweep's segments and chunks partition the frames;
//   * the batch planner's items cover every lane group once, in LPT order.
// Prints "ok" and exits 0, or prints the first violations and exits 1.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "dsgm.h"
#include "dsgm_geom.h"
#include "dsgm_internal.h"
#include "dsgm_plan.h"

namespace g = dsgm::geom;

static long failures = 0;
#define CHECK(cond, ...)                                   \
  do {                                                     \
    if (!(cond)) {                                         \
      if (failures < 20) {                                 \
        printf("line %d: %s: ", __LINE__, #cond);          \
        printf(__VA_ARGS__);                               \
        printf("\n");                                      \
      }                                                    \
      ++failures;                                          \
    }                                                      \
  } while (0)

struct Shape {
  int64_t T, H, W, rs, fs;
};
// elements a T x H x W strided array spans
static int64_t extent(const Shape& s) {
  if (s.T == 0 || s.H == 0 || s.W == 0) return 0;
  return (s.T - 1) * s.fs + (s.H - 1) * s.rs + s.W;
}
static dsgm_shape abi(const Shape& s) { return dsgm_shape{s.T, s.H, s.W, s.rs, s.fs}; }

static std::vector<Shape> shapes() {
  std::vector<Shape> v;
  const int64_t dims[][3] = {{1, 1, 1},   {3, 1, 4},    {5, 4, 1},    {7, 2, 8},     {33, 16, 64},
                             {40, 17, 65}, {9, 15, 63}, {64, 31, 132}, {100, 48, 192}, {17, 3, 520},
                             {2, 130, 12}, {65, 20, 36}, {31, 7, 4}};
  for (auto& d : dims) {
    const int64_t T = d[0], H = d[1], W = d[2];
    v.push_back({T, H, W, W, H * W});                         // dense
    v.push_back({T, H, W, W + 4, (H * (W + 4)) + 8});         // padded rows and frames
    v.push_back({T, H, W, W + 12, (H - 1) * (W + 12) + W});   // frames packed tight
  }
  return v;
}

// ---------------------------------------------------------------- tile_of
static void check_tile_of() {
  for (int64_t nb = 1; nb <= 4200; nb += (nb < 300 ? 1 : 97)) {
    std::vector<char> seen(static_cast<size_t>(nb), 0);
    for (int64_t b = 0; b < nb; ++b) {
      const int64_t t = g::tile_of(b, nb);
      CHECK(t >= 0 && t < nb, "nb %lld b %lld -> %lld", (long long)nb, (long long)b, (long long)t);
      if (t >= 0 && t < nb) {
        CHECK(!seen[size_t(t)], "nb %lld: tile %lld twice", (long long)nb, (long long)t);
        seen[size_t(t)] = 1;
      }
    }
  }
}

// ------------------------------------------- time-fused forward and backward
static void check_groups(const Shape& s, int P, int block, std::vector<int>& owner) {
  const int64_t gpr = s.W / P, ng = s.H * gpr;
  const int64_t grid = (ng + block - 1) / block;
  const int64_t fext = extent(s);
  std::fill(owner.begin(), owner.end(), 0);
  for (int64_t b = 0; b < grid; ++b)
    for (int tid = 0; tid < block; ++tid) {
      const int64_t gi = b * block + tid;
      if (gi >= ng) continue;  // the kernel returns
      const g::Group G = g::group_of(gi, gpr, P, s.W, s.rs);
      CHECK(G.soff >= 0 && G.soff + P <= s.H * s.W, "state offset %lld", (long long)G.soff);
      CHECK(G.foff >= 0 && G.foff < (int64_t(1) << 31), "frame offset %lld", (long long)G.foff);
      // first and last frame of the sequence: every t in between lies between them
      CHECK((s.T - 1) * s.fs + G.foff + P <= fext, "frame access past the extent");
      CHECK(G.foff % P == 0 || s.rs % P != 0, "group not aligned to its width");
      for (int q = 0; q < P; ++q) {
        const int64_t pix = G.h * s.W + G.w0 + q;
        CHECK(G.w0 + q < s.W && pix == G.soff + q, "pixel outside its row");
        if (pix >= 0 && pix < int64_t(owner.size())) ++owner[size_t(pix)];
      }
    }
  for (int64_t p = 0; p < s.H * s.W; ++p)
    CHECK(owner[size_t(p)] == 1, "pixel %lld owned %d times (P %d)", (long long)p,
          owner[size_t(p)], P);
}

static void check_forward(const Shape& s, std::vector<int>& owner) {
  for (int P : {1, 2, 4}) {
    if (s.W % P) continue;
    for (int block : {64, 128, 192, 256}) check_groups(s, P, block, owner);
  }
  // checkpoints: slots 0 .. ckpt_slots-1, each plane's bytes inside the slot
  for (int acc : {DSGM_ACC_F64, DSGM_ACC_F32, DSGM_ACC_F64_IO32, DSGM_ACC_F32X2}) {
    const int64_t ae = acc == DSGM_ACC_F64 ? 8 : acc == DSGM_ACC_F32 ? 4 : 8;
    for (int K : {1, 7, 16, 32, 40}) {
      const size_t bytes = dsgm_ckpt_bytes(abi(s), dsgm_acc(acc), K);
      const int64_t px = s.H * s.W;
      const g::CkptLayout c = g::ckpt_layout(px, ae);
      const int64_t slots = g::ckpt_slots(s.T, K);
      int64_t written = 0;
      for (int64_t t = 0; t < s.T; ++t) written += (t % K == 0);  // the forward's slot cadence
      CHECK(written == slots, "slots %lld written %lld", (long long)slots, (long long)written);
      CHECK(c.fplane >= px * ae && c.aplane >= px && c.fplane % 256 == 0 && c.aplane % 256 == 0,
            "plane sizes");
      CHECK(int64_t(bytes) >= slots * c.slot, "ckpt bytes %zu < %lld slots", bytes,
            (long long)slots);
      // the last byte the last slot's last plane holds
      if (slots > 0 && px > 0)
        CHECK((slots - 1) * c.slot + 4 * c.fplane + c.aplane + px <= int64_t(bytes),
              "last age plane past the buffer");
    }
  }
}

static void check_backward(const Shape& s, std::vector<int>& owner) {
  const int64_t px = s.H * s.W;
  for (int acc : {DSGM_ACC_F64, DSGM_ACC_F32, DSGM_ACC_F64_IO32, DSGM_ACC_F32X2}) {
    CHECK(int64_t(dsgm_workspace_bytes(abi(s), dsgm_acc(acc))) == g::ws_bytes(px),
          "workspace size");
  }
  CHECK(g::ws_partial_offset(px) >= px * 8 && g::ws_partial_offset(px) % 256 == 0,
        "partial sums overlap the per-pixel terms");
  // one lane per pixel, 256-thread workgroups
  const int64_t grid = (px + 255) / 256;
  std::fill(owner.begin(), owner.end(), 0);
  for (int64_t gi = 0; gi < grid * 256; ++gi) {
    if (gi >= px) continue;
    const int64_t h = gi / s.W, w = gi - h * s.W;
    const int64_t foff = h * s.rs + w;
    CHECK((s.T - 1) * s.fs + foff + 1 <= extent(s), "backward frame access");
    ++owner[size_t(gi)];
  }
  for (int64_t p = 0; p < px; ++p) CHECK(owner[size_t(p)] == 1, "backward pixel %lld", (long long)p);
  // segments and chunks partition [0, T), chunks fit the tape, slots exist
  for (int K : {1, 5, 16, 32, 33, 100}) {
    for (int KC : {16, 32}) {
      std::vector<int> hit(size_t(s.T), 0);
      const int64_t nseg = g::n_segments(s.T, K);
      CHECK(nseg == g::ckpt_slots(s.T, K), "segments != checkpoint slots");
      int64_t prev_lo = s.T;
      for (int64_t seg = nseg - 1; seg >= 0; --seg) {
        const g::Range sg = g::segment(seg, s.T, K);
        CHECK(sg.lo >= 0 && sg.lo < sg.hi && sg.hi <= s.T && sg.hi == prev_lo,
              "segment %lld [%lld, %lld)", (long long)seg, (long long)sg.lo, (long long)sg.hi);
        prev_lo = sg.lo;
        int64_t cprev = sg.hi;
        for (int64_t c = g::n_chunks(sg, KC) - 1; c >= 0; --c) {
          const g::Range ch = g::chunk(sg, c, KC);
          CHECK(ch.lo >= sg.lo && ch.lo < ch.hi && ch.hi == cprev && ch.hi - ch.lo <= KC,
                "chunk [%lld, %lld)", (long long)ch.lo, (long long)ch.hi);
          cprev = ch.lo;
          for (int64_t t = ch.lo; t < ch.hi && t >= 0 && t < s.T; ++t) ++hit[size_t(t)];
        }
        CHECK(cprev == sg.lo, "chunks do not reach the segment start");
      }
      CHECK(prev_lo == 0 || s.T == 0, "segments do not reach frame 0");
      for (int64_t t = 0; t < s.T; ++t) CHECK(hit[size_t(t)] == 1, "frame %lld swept %d times",
                                             (long long)t, hit[size_t(t)]);
    }
  }
}

// ----------------------------------------------------------------- batched
static uint64_t lcg(uint64_t& x) {
  x = x * 6364136223846793005ull + 1442695040888963407ull;
  return x >> 33;
}

static void check_batched() {
  uint64_t seed = 12345;
  char* const base = reinterpret_cast<char*>(uintptr_t(1) << 40);  // a fake, aligned address
  for (int trial = 0; trial < 40; ++trial) {
    const int n = 1 + int(lcg(seed) % 24);
    std::vector<dsgm_instance> inst(static_cast<size_t>(n));
    std::vector<Shape> sh(static_cast<size_t>(n));
    int64_t at = 0;
    auto take = [&](int64_t bytes) {
      char* p = base + at;
      at += g::pad256(bytes + 1);
      return p;
    };
    for (int i = 0; i < n; ++i) {
      const int64_t W = 4 * (1 + int64_t(lcg(seed) % 40)) + (lcg(seed) % 4 == 0 ? 2 : 0);
      const int64_t H = int64_t(lcg(seed) % 30) + (lcg(seed) % 9 == 0 ? 0 : 1);
      const int64_t T = int64_t(lcg(seed) % 50) + (lcg(seed) % 11 == 0 ? 0 : 1);
      const int64_t rs = W + 4 * int64_t(lcg(seed) % 3);
      Shape s{T, H, W, rs, H * rs + 8 * int64_t(lcg(seed) % 2)};
      sh[size_t(i)] = s;
      dsgm_instance& I = inst[size_t(i)];
      memset(&I, 0, sizeof(I));
      I.shape = abi(s);
      const int64_t ext = std::max<int64_t>(extent(s), 1), px = std::max<int64_t>(H * W, 1);
      I.frames = take(ext * 2);
      I.masks = reinterpret_cast<uint8_t*>(take(ext));
      I.bg = (trial % 3 == 0 && i % 2 == 0) ? take(ext * 4) : nullptr;
      I.fg_counts = (i % 3 != 1) ? reinterpret_cast<uint32_t*>(take(std::max<int64_t>(T, 1) * 4)) : nullptr;
      I.state.mean_a = take(px * 4);
      I.state.var_a = take(px * 4);
      I.state.mean_c = take(px * 4);
      I.state.var_c = take(px * 4);
      I.state.age_a = reinterpret_cast<uint8_t*>(take(px));
      I.state.age_c = reinterpret_cast<uint8_t*>(take(px));
    }
    dsgm::PlanImage img;
    const int rc = dsgm::plan_image(inst.data(), n, DSGM_IN_BF16, DSGM_ACC_F32, base, &img);
    CHECK(rc == DSGM_OK, "plan_image rc %d: %s", rc, dsgm_last_error());
    if (rc != DSGM_OK) continue;
    CHECK(int64_t(dsgm_batch_plan_bytes(inst.data(), n, DSGM_IN_BF16, DSGM_ACC_F32)) == img.bytes,
          "plan bytes");
    CHECK(int64_t(img.host.size()) == img.bytes, "image size");
    CHECK(img.inst_off >= 8 && img.inst_off + n * int64_t(sizeof(dsgm::BatchInst)) <= img.items_off &&
              img.items_off + img.n_items * int64_t(sizeof(dsgm::BatchItem)) <= img.stripes_off &&
              img.stripes_off <= img.bytes,
          "plan regions overlap");
    const auto* desc = reinterpret_cast<const dsgm::BatchInst*>(img.host.data() + img.inst_off);
    const auto* items = reinterpret_cast<const dsgm::BatchItem*>(img.host.data() + img.items_off);
    const int P = img.P;
    // stripes: inside the plan's stripe region, disjoint, 256-byte aligned
    std::vector<std::pair<int64_t, int64_t>> spans;
    for (int i = 0; i < n; ++i) {
      const dsgm::BatchInst& d = desc[i];
      const bool work = sh[size_t(i)].T > 0 && sh[size_t(i)].H * sh[size_t(i)].W > 0;
      CHECK(d.groups_per_row == sh[size_t(i)].W / P, "groups per row");
      if (d.fg_counts) {
        CHECK(work, "counters kept for an empty instance");
        const int64_t off = reinterpret_cast<const char*>(d.stripes) - base;
        CHECK(off >= img.stripes_off && off % 256 == 0 &&
                  off + g::COUNT_STRIPES * d.T * 4 <= img.bytes,
              "stripes of instance %d at %lld", i, (long long)off);
        spans.push_back({off, off + g::COUNT_STRIPES * d.T * 4});
      }
    }
    std::sort(spans.begin(), spans.end());
    for (size_t k = 1; k < spans.size(); ++k) CHECK(spans[k].first >= spans[k - 1].second, "stripes overlap");
    // items: every lane group of every instance exactly once, LPT order
    std::vector<std::vector<int>> seen(static_cast<size_t>(n));
    for (int i = 0; i < n; ++i)  // an instance with no frames or no pixels has no items
      seen[size_t(i)].assign(sh[size_t(i)].T > 0 ? size_t(sh[size_t(i)].H * (sh[size_t(i)].W / P)) : 0, 0);
    std::vector<int> owner;
    int64_t prev_cost = INT64_MAX;
    for (int64_t k = 0; k < img.n_items; ++k) {
      const dsgm::BatchItem& it = items[k];
      CHECK(it.inst >= 0 && it.inst < n, "item %lld instance %d", (long long)k, it.inst);
      if (it.inst < 0 || it.inst >= n) continue;
      const dsgm::BatchInst& d = desc[it.inst];
      const Shape& s = sh[size_t(it.inst)];
      const int64_t ng = s.H * (s.W / P);
      CHECK(it.count >= 1 && it.count <= g::ITEM_GROUPS && it.first_group >= 0 &&
                it.first_group + it.count <= ng,
            "item %lld groups [%d, +%d) of %lld", (long long)k, it.first_group, it.count,
            (long long)ng);
      const int64_t cost = d.T * it.count;
      CHECK(cost <= prev_cost, "items not in LPT order");
      prev_cost = cost;
      CHECK(g::stripe_of(uint64_t(k)) * d.T + (d.T - 1) < g::COUNT_STRIPES * d.T, "stripe index");
      for (int lane = 0; lane < 64; ++lane) {
        if (lane >= it.count) continue;  // the kernel skips these lanes
        const int64_t gi = int64_t(it.first_group) + lane;
        const g::Group G = g::group_of(gi, d.groups_per_row, P, d.W, d.row_stride);
        CHECK(G.soff + P <= s.H * s.W && (s.T - 1) * s.fs + G.foff + P <= extent(s),
              "batched access past instance %d", it.inst);
        if (gi >= 0 && gi < ng) ++seen[size_t(it.inst)][size_t(gi)];
      }
    }
    for (int i = 0; i < n; ++i)
      for (size_t gi = 0; gi < seen[size_t(i)].size(); ++gi)
        CHECK(seen[size_t(i)][gi] == 1, "instance %d group %zu taken %d times", i, gi,
              seen[size_t(i)][gi]);
  }
}

// --------------------------------------------------- fused preprocessing
template <int RG, bool MED>
static void check_pre_rg(const Shape& s) {
  using G = g::pre::Geo<RG, MED>;
  const int64_t tiles_x = (s.W + g::pre::TW - 1) / g::pre::TW;
  const int64_t tiles_y = (s.H + g::pre::TH - 1) / g::pre::TH;
  const int64_t nb = tiles_x * tiles_y;
  const int64_t fext = extent(s);
  std::vector<int> owner(size_t(s.H * s.W), 0);
  for (int64_t b = 0; b < nb; ++b) {
    const int64_t tile = g::tile_of(b, nb);
    const int64_t y0 = (tile / tiles_x) * g::pre::TH, x0 = (tile % tiles_x) * g::pre::TW;
    for (int tid = 0; tid < g::pre::NT; ++tid) {
      for (int l = 0; l < G::LOADS; ++l) {
        if (!G::raw_active(tid, l)) continue;
        const int i = G::raw_cell(tid, l);
        CHECK(i >= 0 && i < G::RAW_N, "raw cell %d of %d", i, G::RAW_N);
        const int64_t o = G::raw_source(i, y0, x0, s.H, s.W, s.rs);
        CHECK(o >= 0 && (s.T - 1) * s.fs + o < fext, "raw source %lld", (long long)o);
      }
      if (RG > 0) {
        for (int it = 0; it < G::ROW_IT; ++it) {
          if (!G::row_active(tid, it)) continue;
          const int pi = G::row_pair(tid, it), w0 = G::row_window(pi);
          CHECK(2 * pi + 1 < G::HB_N, "row pass writes HB cell %d", 2 * pi + 1);
          // the window of 2*RG + 2 raw cells stays inside one raw row
          CHECK(w0 >= 0 && w0 % G::RAW_W + 2 * RG + 1 < G::RAW_W && w0 + 2 * RG + 1 < G::RAW_N,
                "row window %d", w0);
          // output pair (r, v), (r, v+1) reads raw columns v .. v + 2*RG + 1 of row r
          CHECK(w0 / G::RAW_W == (2 * pi) / G::HB_W && w0 % G::RAW_W == (2 * pi) % G::HB_W,
                "row window not aligned with its outputs");
        }
        // the two-dimensional blur of the 8-bit form: every GB cell's window
        // lies in the raw tile, centred on the cell's frame pixel
        for (int it = 0; it < G::GB_IT; ++it) {
          if (!G::gb_active(tid, it)) continue;
          const int cell = G::gb_cell(tid, it), win = G::blur_window(cell);
          CHECK(cell >= 0 && cell < G::GB_N, "2-D blur cell %d", cell);
          const int wr = win / G::RAW_W, wc = win % G::RAW_W;
          CHECK(wr + 2 * RG < G::RAW_H && wc + 2 * RG < G::RAW_W, "2-D window (%d, %d)", wr, wc);
          // frame offsets from the tile origin: the window's centre raw cell
          // (wr + RG - R) and the cell's pixel (its GB index - RM) coincide
          CHECK(wr + RG - G::R == cell / G::GB_W - G::RM && wc + RG - G::R == cell % G::GB_W - G::RM,
                "2-D window not centred on its cell");
        }
        for (int it = 0; it < G::COL_IT; ++it) {
          if (!G::col_active(tid, it)) continue;
          const int pi = G::col_pair(tid, it);
          CHECK(2 * pi + 1 < G::GB_N, "column pass writes GB cell %d", 2 * pi + 1);
          CHECK(2 * pi + 2 * RG * G::HB_W + 1 < G::HB_N, "column pass reads past HB");
          CHECK((2 * pi) % G::GB_W + 1 < G::GB_W, "column pair straddles a row");
        }
      }
      // every lane takes its medians, also one whose pixels lie outside the frame
      const int ty = G::lane_row(tid), tx = G::lane_col(tid);
      const int64_t gy = y0 + ty;
      const int gbw = RG > 0 ? G::GB_W : G::RAW_W, gbn = RG > 0 ? G::GB_N : G::RAW_N;
      CHECK(RG > 0 || (G::RAW_W == G::GB_W && G::RAW_N == G::GB_N), "raw tile is not the blurred tile");
      // the median reads rows d < 3 and columns e < PX + 2 of the lane's
      // neighbourhoods; without it only the centre row and the lane's own columns
      for (int d = MED ? 0 : 1; d < (MED ? 3 : 2); ++d) {
        const int r = G::med_row(gy, d, y0, s.H);
        for (int e = MED ? 0 : 1; e < (MED ? g::pre::PX + 2 : g::pre::PX + 1); ++e) {
          const int c = G::med_col(x0 + tx, e, x0, s.W);
          CHECK(r >= 0 && r < G::GB_H && c >= 0 && c < gbw && r * gbw + c < gbn,
                "median cell (%d, %d)", r, c);
          // and it is the blurred value of an in-frame pixel (borders clamp)
          CHECK(y0 - G::RM + r >= 0 && y0 - G::RM + r < s.H && x0 - G::RM + c >= 0 &&
                    x0 - G::RM + c < s.W,
                "median reads frame pixel (%lld, %lld)", (long long)(y0 - G::RM + r),
                (long long)(x0 - G::RM + c));
        }
      }
      for (int q = 0; q < g::pre::PX; ++q) {
        const int64_t x = x0 + tx + q;
        if (gy < s.H && x < s.W) {
          ++owner[size_t(gy * s.W + x)];
          CHECK((s.T - 1) * s.fs + gy * s.rs + x < fext, "pre output past the extent");
        }
      }
    }
  }
  for (size_t p = 0; p < owner.size(); ++p)
    CHECK(owner[p] == 1, "pre: pixel %zu owned %d times (RG %d MED %d)", p, owner[p], RG, int(MED));
}

static void check_pre(const Shape& s) {
  check_pre_rg<0, true>(s);
  check_pre_rg<1, true>(s);
  check_pre_rg<2, true>(s);
  check_pre_rg<3, true>(s);
  check_pre_rg<1, false>(s);
  check_pre_rg<2, false>(s);
  check_pre_rg<3, false>(s);
}

// -------------------------------------------- motion-compensated update
static void check_warp(int64_t H, int64_t W) {
  const double c = std::cos(0.3), sn = std::sin(0.3);
  const double maps[][9] = {
      {1, 0, 0, 0, 1, 0, 0, 0, 1},                                   // identity
      {1, 0, 2.5, 0, 1, -1.25, 0, 0, 1},                             // shift
      {1, 0, -double(W), 0, 1, double(H), 0, 0, 1},                  // all outside
      {c, -sn, 3, sn, c, -2, 0, 0, 1},                               // rotation
      {1.7, 0.1, -4, -0.2, 0.6, 5, 0, 0, 1},                         // affine
      {1, 0, 0, 0, 1, 0, 0.002, -0.003, 1},                          // perspective
      {1, 0, 0, 0, 1, 0, -0.5, 0, 1},                                // den <= 0 on part
      {1, 0, double(W - 1), 0, 1, double(H - 1), 0, 0, 1},           // corner only
      {0, 0, double(W - 1), 0, 0, double(H - 1), 0, 0, 1},           // every pixel -> last
      {1e-9, 0, 0, 0, 1e-9, 0, 0, 0, 1},                             // every pixel -> first
  };
  const int64_t n = H * W, grid = (n + 255) / 256;
  for (const auto& map : maps) {
    std::vector<int> owner(size_t(n), 0);
    for (int64_t b = 0; b < grid; ++b)
      for (int tid = 0; tid < 256; ++tid) {
        const int64_t i = g::tile_of(b, grid) * 256 + tid;
        if (i >= n) continue;
        ++owner[size_t(i)];
        const int64_t y = i / W, x = i - y * W;
        const g::WarpSrc s = g::warp_source(x, y, map, H, W);
        if (!s.covered) continue;
        CHECK(s.x0 >= 0 && s.x0 < W && s.y0 >= 0 && s.y0 < H && s.x1 >= s.x0 && s.x1 < W &&
                  s.y1 >= s.y0 && s.y1 < H,
              "bilinear neighbours (%lld, %lld)", (long long)s.x0, (long long)s.y0);
        if (W >= 2) {
          CHECK(s.xa >= 0 && s.xa + 1 < W && (s.xa == s.x0 || s.xa + 1 == s.x0),
                "pair column %lld", (long long)s.xa);
          CHECK(s.y1 * W + s.xa + 1 < n, "pair load past the plane");
        }
        CHECK(s.xn >= 0 && s.xn < W && s.yn >= 0 && s.yn < H, "nearest (%lld, %lld)",
              (long long)s.xn, (long long)s.yn);
        CHECK(s.fx >= 0 && s.fx < 1 && s.fy >= 0 && s.fy < 1, "fractions");
      }
    for (int64_t p = 0; p < n; ++p) CHECK(owner[size_t(p)] == 1, "warp pixel %lld", (long long)p);
  }
}

// ------------------------------------------------------------- grid model
static void check_grid(const Shape& s) {
  for (int B : {1, 2, 4}) {
    const int64_t Hb = (s.H + B - 1) / B, Wb = (s.W + B - 1) / B, nb = Hb * Wb;
    std::vector<int> owner(size_t(s.H * s.W), 0);
    const int64_t grid = (nb + 255) / 256;
    for (int64_t blk = 0; blk < grid * 256; ++blk) {
      if (blk >= nb) continue;
      const g::GridBlock gb = g::grid_block(blk, Wb, B, s.H, s.W);
      CHECK(gb.rows >= 1 && gb.rows <= B && gb.cols >= 1 && gb.cols <= B, "block size");
      CHECK(gb.y0 + gb.rows <= s.H && gb.x0 + gb.cols <= s.W, "block past the frame");
      const bool whole = gb.rows == B && gb.cols == B;
      const int64_t o_last = (s.T - 1) * s.fs + gb.y0 * s.rs + gb.x0;
      // whole blocks read and write B elements of each of B rows, edge blocks rows x cols
      CHECK(o_last + (gb.rows - 1) * s.rs + (whole ? B : gb.cols) <= extent(s), "grid access");
      for (int r = 0; r < gb.rows; ++r)
        for (int c = 0; c < gb.cols; ++c) ++owner[size_t((gb.y0 + r) * s.W + gb.x0 + c)];
    }
    for (size_t p = 0; p < owner.size(); ++p) CHECK(owner[p] == 1, "grid pixel %zu (B %d)", p, B);
  }
}

// ------------------------------------------ 8-bit one-frame persistent walk
static void check_u8_step(const Shape& s) {
  for (int P : {1, 2, 4}) {
    if (s.W % P) continue;
    const int64_t gpr = s.W / P, ng = s.H * gpr;
    const int block = 256;
    const int64_t need = (ng + block - 1) / block, grid = std::min<int64_t>(need, 1024);
    const int64_t stride = grid * block;
    std::vector<int> owner(size_t(ng), 0);
    for (int64_t b = 0; b < grid; ++b)
      for (int tid = 0; tid < block; ++tid)
        for (int64_t gi = b * block + tid; gi < ng; gi += stride) {
          const g::Group G = g::group_of(gi, gpr, P, s.W, s.rs);
          CHECK(G.soff + P <= s.H * s.W && G.foff + P <= (s.H - 1) * s.rs + s.W, "u8 access");
          ++owner[size_t(gi)];
        }
    for (int64_t gi = 0; gi < ng; ++gi) CHECK(owner[size_t(gi)] == 1, "u8 group %lld", (long long)gi);
  }
}

int main() {
  check_tile_of();
  std::vector<int> owner;
  for (const Shape& s : shapes()) {
    owner.assign(size_t(std::max<int64_t>(s.H * s.W, 1)), 0);
    check_forward(s, owner);
    check_backward(s, owner);
    check_pre(s);
    check_grid(s);
    check_u8_step({1, s.H, s.W, s.rs, s.fs});
  }
  // a frame larger than one tile in both directions, at the paper's size
  check_pre({2, 240, 320, 320, 240 * 320});
  for (auto hw : {std::pair<int64_t, int64_t>{1, 1}, {1, 7}, {6, 1}, {17, 33}, {48, 64}, {240, 320}})
    check_warp(hw.first, hw.second);
  check_batched();
  if (failures) {
    printf("%ld failures\n", failures);
    return 1;
  }
  printf("ok\n");
  return 0;
}
