// dsgm_api.hip -- the extern "C" entry points of libdsgm.so declared in
// include/dsgm.h: argument validation (host only, before any HIP call), launch
// configuration and dispatch to the kernels.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "dsgm.h"
#include "dsgm_ext.h"
#include "dsgm_internal.h"
#include "dsgm_plan.h"

namespace {

thread_local char g_last_error[512] = "";

int fail(int status, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
  va_end(ap);
  return status;
}

int ok() {
  g_last_error[0] = '\0';
  return DSGM_OK;
}

int hip_fail(hipError_t e, const char* where) {
  return fail(DSGM_E_HIP, "%s: %s", where, hipGetErrorString(e));
}

size_t in_size(int d) {
  return d == DSGM_IN_F64 ? 8 : d == DSGM_IN_F32 ? 4 : d == DSGM_IN_BF16 ? 2 : 1;
}
// element size of the model state (and of every arithmetic operation)
size_t acc_size(int a) { return a == DSGM_ACC_F32 ? 4 : a == DSGM_ACC_U8 ? 1 : 8; }
// element size of bg and of every gradient array
size_t io_size(int a) { return a == DSGM_ACC_F64 ? 8 : 4; }

bool aligned(const void* p, size_t n) { return (reinterpret_cast<uintptr_t>(p) % n) == 0; }

int64_t pad256(int64_t b) { return dsgm::geom::pad256(b); }

int check_params(const dsgm_params* p) {
  if (!p) return fail(DSGM_E_ARG, "params is NULL");
  const double v[5] = {p->theta_s, p->theta_d, p->var_init, p->var_floor, p->mask_floor};
  const char* n[5] = {"theta_s", "theta_d", "var_init", "var_floor", "mask_floor"};
  for (int i = 0; i < 5; ++i) {
    if (std::isnan(v[i])) return fail(DSGM_E_ARG, "params.%s is NaN", n[i]);
    if (i != 4 && v[i] < 0) return fail(DSGM_E_ARG, "params.%s < 0", n[i]);
  }
  if (std::isinf(p->var_init) || std::isinf(p->var_floor) || std::isinf(p->mask_floor))
    return fail(DSGM_E_ARG, "params: var_init and the floors must be finite");
  if (p->age_max < 1 || p->age_max > 255)
    return fail(DSGM_E_ARG, "params.age_max = %d outside 1..255", p->age_max);
  if (p->weight_rule != DSGM_WEIGHT_EQ && p->weight_rule != DSGM_WEIGHT_APPENDIX)
    return fail(DSGM_E_ARG, "params.weight_rule = %d invalid", p->weight_rule);
  if (p->mask_rule != DSGM_MASK_VARIANCE && p->mask_rule != DSGM_MASK_PRINTED)
    return fail(DSGM_E_ARG, "params.mask_rule = %d invalid", p->mask_rule);
  return DSGM_OK;
}

int check_types(int in_dtype, int acc) {
  if (in_dtype < DSGM_IN_F64 || in_dtype > DSGM_IN_BF16)
    return fail(DSGM_E_DTYPE, "in_dtype = %d invalid", in_dtype);
  if (acc == DSGM_ACC_F32X2)
    return fail(DSGM_E_DTYPE, "F32X2 state: dsgm_forward, dsgm_backward and the state "
                              "initialisation only");
  if (acc != DSGM_ACC_F64 && acc != DSGM_ACC_F32 && acc != DSGM_ACC_F64_IO32)
    return fail(DSGM_E_DTYPE, "acc = %d invalid", acc);
  if (acc != DSGM_ACC_F64 && in_dtype == DSGM_IN_F64)
    return fail(DSGM_E_DTYPE, "F64 frames need ACC_F64");
  return DSGM_OK;
}

// as check_types, and also the compensated pair state (F32X2, with F32 or BF16
// frames), which dsgm_forward, dsgm_backward and the state initialisation
// implement
int check_types_x2(int in_dtype, int acc) {
  if (acc == DSGM_ACC_F32X2) {
    if (in_dtype != DSGM_IN_F32 && in_dtype != DSGM_IN_BF16)
      return fail(DSGM_E_DTYPE, "F32X2 state needs F32 or BF16 frames");
    return DSGM_OK;
  }
  return check_types(in_dtype, acc);
}

// as check_types_x2, and also the 8-bit as-run pair (U8 frames with U8 state),
// which only dsgm_forward and dsgm_state_init_from_frame implement
int check_types_u8(int in_dtype, int acc) {
  if (in_dtype == DSGM_IN_U8 && acc == DSGM_ACC_U8) return DSGM_OK;
  if (in_dtype == DSGM_IN_U8 || acc == DSGM_ACC_U8)
    return fail(DSGM_E_DTYPE, "U8 frames and U8 state go together");
  return check_types_x2(in_dtype, acc);
}

// the 8-bit storage rule applied to a parameter (var_init of a reset model)
double stored_u8(double v) { return v > 0.0 ? (v >= 255.0 ? 255.0 : std::trunc(v)) : 0.0; }

// frames-like arrays: per-frame extent must fit 31 bits of elements and bytes
int check_shape(const dsgm_shape& s, size_t max_elem_bytes) {
  if (s.T < 0 || s.H < 0 || s.W < 0)
    return fail(DSGM_E_SHAPE, "negative size T=%lld H=%lld W=%lld", (long long)s.T,
                (long long)s.H, (long long)s.W);
  if (s.row_stride < s.W)
    return fail(DSGM_E_SHAPE, "row_stride %lld < W %lld", (long long)s.row_stride, (long long)s.W);
  const int64_t extent = s.H > 0 ? (s.H - 1) * s.row_stride + s.W : 0;
  if (s.T > 1 && s.frame_stride < extent)
    return fail(DSGM_E_SHAPE, "frame_stride %lld < frame extent %lld", (long long)s.frame_stride,
                (long long)extent);
  if (s.frame_stride < 0) return fail(DSGM_E_SHAPE, "negative frame_stride");
  if (double(extent) * double(max_elem_bytes) >= 2147483648.0)
    return fail(DSGM_E_SHAPE, "one frame spans %lld elements: more than 2^31 bytes",
                (long long)extent);
  if (s.H > 0 && s.W > 0 && double(s.H) * double(s.W) >= 2147483648.0)
    return fail(DSGM_E_SHAPE, "H*W >= 2^31");
  return DSGM_OK;
}

// set by dsgm_set_launch (tuning) while other threads may be launching:
// atomics, read once per call
std::atomic<int> g_block_override{0};
std::atomic<int> g_vector_override{0};

// Launch shapes chosen by dsgm_autotune, per (frame type, state type, H, W,
// output flags); dsgm_forward looks its arguments up here.
struct TuneKey {
  int in_dtype, acc;
  int64_t H, W;
  int flags;
  bool operator<(const TuneKey& o) const {
    return std::tie(in_dtype, acc, H, W, flags) < std::tie(o.in_dtype, o.acc, o.H, o.W, o.flags);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, std::pair<int, int>> g_tune;  // -> (block, pixels per lane)

bool tune_lookup(const TuneKey& k, int* block, int* vector) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  const auto it = g_tune.find(k);
  if (it == g_tune.end()) return false;
  *block = it->second.first;
  *vector = it->second.second;
  return true;
}

constexpr int kTuneFlags = DSGM_TUNE_BG | DSGM_TUNE_CKPT | DSGM_TUNE_PRINTED;
constexpr int kTuneFrames = 64;  // frames per timed call: the cost per frame is flat beyond
constexpr int kTuneCkptEvery = 32;

// Preferred pixels per lane, measured on MI355X at 1920x2560x500: FP64 and
// FP32 state run fastest with 2 (more waves per SIMD), BF16 frames with 4
// (wider loads of the narrow frames).
int preferred_vector(int in_dtype, int acc) {
  if (in_dtype == DSGM_IN_BF16) return 4;
  (void)acc;
  return 2;
}

// widest per-lane pixel count (up to `cap`) allowed by the sizes, strides and
// alignments
int pick_vector(const dsgm_shape& s, const void* const* ptrs, const size_t* elem, int n,
                int cap = 4) {
  const int cand[3] = {4, 2, 1};
  for (int c : cand) {
    if (c > cap) continue;
    if (s.W % c || s.row_stride % c || (s.T > 1 && s.frame_stride % c)) continue;
    bool good = true;
    for (int i = 0; i < n && good; ++i)
      if (ptrs[i] && !aligned(ptrs[i], elem[i] * c)) good = false;
    if (good) return c;
  }
  return 1;
}

// ---------------------------------------------------------------- batching
constexpr int64_t kPlanHeader = 256;  // the item counter lives here

int64_t pad_to(int64_t b, int64_t a) { return dsgm::geom::pad_to(b, a); }

struct PlanLayout {
  int P = 4;
  int64_t n_items = 0, total = 0, inst_off = 0, items_off = 0, stripes_off = 0, bytes = 0;
  bool bg = false, counts = false;
};

// validate the instances and lay out the device plan; no HIP call
int plan_layout(const dsgm_instance* inst, int32_t n, int in_dtype, int acc, PlanLayout* L) {
  int rc;
  if ((rc = check_types(in_dtype, acc))) return rc;
  if (n < 0 || (n > 0 && !inst)) return fail(DSGM_E_ARG, "instances: NULL or negative count");
  const size_t ie = in_size(in_dtype), ae = acc_size(acc), oe = io_size(acc);
  int P = 4;
  L->bg = false;
  L->counts = false;
  for (int32_t i = 0; i < n; ++i) {
    const dsgm_instance& I = inst[i];
    if ((rc = check_shape(I.shape, ie > oe ? ie : oe)))
      return fail(rc, "instance %d: %s", i, g_last_error);
    const int64_t px = I.shape.H * I.shape.W;
    if (px == 0 || I.shape.T == 0) continue;
    if (!I.frames || !I.masks || !I.state.mean_a || !I.state.var_a || !I.state.mean_c ||
        !I.state.var_c || !I.state.age_a || !I.state.age_c)
      return fail(DSGM_E_ARG, "instance %d: a required pointer is NULL", i);
    const void* ptrs[10] = {I.frames, I.masks, I.bg, I.state.mean_a, I.state.var_a,
                            I.state.mean_c, I.state.var_c, I.state.age_a, I.state.age_c,
                            I.fg_counts};
    const size_t elem[10] = {ie, 1, oe, ae, ae, ae, ae, 1, 1, 4};
    for (int k = 0; k < 10; ++k)
      if (ptrs[k] && !aligned(ptrs[k], elem[k]))
        return fail(DSGM_E_ALIGN, "instance %d: pointer %d not aligned to %zu bytes", i, k, elem[k]);
    P = std::min(P, pick_vector(I.shape, ptrs, elem, 9));  // the counters do not limit P
    if (I.bg) L->bg = true;
    if (I.fg_counts) L->counts = true;
  }
  const int widest = P;
  P = std::min(P, preferred_vector(in_dtype, acc));
  const int vo = g_vector_override.load(std::memory_order_relaxed);
  if (vo && widest % vo == 0) P = vo;
  int64_t items = 0, total = 0, stripes = 0;
  for (int32_t i = 0; i < n; ++i) {
    const dsgm_shape& s = inst[i].shape;
    if (s.H * s.W == 0 || s.T == 0) continue;
    items += (s.H * (s.W / P) + dsgm::geom::ITEM_GROUPS - 1) / dsgm::geom::ITEM_GROUPS;
    total += s.T * s.H * s.W;
    if (inst[i].fg_counts) stripes += pad_to(s.T * dsgm::COUNT_STRIPES * 4, 256);
  }
  L->P = P;
  L->n_items = items;
  L->total = total;
  L->inst_off = kPlanHeader;
  L->items_off = kPlanHeader + pad_to(int64_t(n) * int64_t(sizeof(dsgm::BatchInst)), 256);
  L->stripes_off = L->items_off + pad_to(items * int64_t(sizeof(dsgm::BatchItem)), 256);
  L->bytes = L->stripes_off + stripes;
  return DSGM_OK;
}


}  // namespace

extern "C" {

int dsgm_version(void) { return 100; }

const char* dsgm_status_string(int status) {
  switch (status) {
    case DSGM_OK: return "DSGM_OK";
    case DSGM_E_ARG: return "DSGM_E_ARG";
    case DSGM_E_SHAPE: return "DSGM_E_SHAPE";
    case DSGM_E_DTYPE: return "DSGM_E_DTYPE";
    case DSGM_E_ALIGN: return "DSGM_E_ALIGN";
    case DSGM_E_WORKSPACE: return "DSGM_E_WORKSPACE";
    case DSGM_E_HIP: return "DSGM_E_HIP";
    case DSGM_E_UNSUPPORTED: return "DSGM_E_UNSUPPORTED";
    default: return "DSGM_UNKNOWN";
  }
}

const char* dsgm_last_error(void) { return g_last_error; }

int dsgm_params_default(dsgm_params* p, double intensity_range, int32_t mask_rule) {
  if (!p) return fail(DSGM_E_ARG, "params is NULL");
  if (!(intensity_range > 0) || std::isinf(intensity_range))
    return fail(DSGM_E_ARG, "intensity_range must be positive and finite");
  if (mask_rule != DSGM_MASK_VARIANCE && mask_rule != DSGM_MASK_PRINTED)
    return fail(DSGM_E_ARG, "mask_rule = %d invalid", mask_rule);
  const double s = intensity_range / 255.0;
  p->theta_s = 2.0;
  p->theta_d = 4.0;
  p->var_init = 255.0 * s * s;
  p->var_floor = 0.1 * s * s;
  p->mask_floor = mask_rule == DSGM_MASK_VARIANCE ? 0.25 * s * s : 0.25 * s;
  p->age_max = 30;
  p->weight_rule = DSGM_WEIGHT_EQ;
  p->mask_rule = mask_rule;
  return ok();
}

size_t dsgm_ckpt_bytes(dsgm_shape shape, dsgm_acc acc, int32_t ckpt_every) {
  if (acc != DSGM_ACC_F64 && acc != DSGM_ACC_F32 && acc != DSGM_ACC_F64_IO32 &&
      acc != DSGM_ACC_F32X2)
    return 0;
  if (ckpt_every < 1 || shape.T < 0 || shape.H < 0 || shape.W < 0) return 0;
  const int64_t n = dsgm::geom::ckpt_slots(shape.T, ckpt_every);
  const int64_t px = shape.H * shape.W;
  return size_t(n * dsgm::geom::ckpt_layout(px, int64_t(acc_size(acc))).slot);
}

int dsgm_state_init_from_frame(const void* frame0, dsgm_in_dtype in_dtype, dsgm_shape shape,
                               dsgm_acc acc, const dsgm_params* params, dsgm_state* state,
                               hipStream_t stream) {
  int rc;
  if ((rc = check_types_u8(in_dtype, acc))) return rc;
  if ((rc = check_params(params))) return rc;
  dsgm_shape one = shape;
  one.T = 1;
  const size_t ie = in_size(in_dtype), ae = acc_size(acc);
  if ((rc = check_shape(one, ie > ae ? ie : ae))) return rc;
  if (!state) return fail(DSGM_E_ARG, "state is NULL");
  const int64_t px = shape.H * shape.W;
  if (px == 0) return ok();
  if (!frame0) return fail(DSGM_E_ARG, "frame0 is NULL");
  if (!state->mean_a || !state->var_a || !state->mean_c || !state->var_c || !state->age_a ||
      !state->age_c)
    return fail(DSGM_E_ARG, "a state plane is NULL");
  const void* ptrs[5] = {frame0, state->mean_a, state->var_a, state->mean_c, state->var_c};
  const size_t elem[5] = {ie, ae, ae, ae, ae};
  for (int i = 0; i < 5; ++i)
    if (!aligned(ptrs[i], elem[i]))
      return fail(DSGM_E_ALIGN, "pointer argument %d is not aligned to %zu bytes", i, elem[i]);
  dsgm::FwdArgs a;
  memset(&a, 0, sizeof(a));
  a.frames = frame0;
  a.mean_a = state->mean_a;
  a.var_a = state->var_a;
  a.mean_c = state->mean_c;
  a.var_c = state->var_c;
  a.age_a = state->age_a;
  a.age_c = state->age_c;
  a.H = shape.H;
  a.W = shape.W;
  a.row_stride = shape.row_stride;
  a.var_init = params->var_init;
  hipError_t e = acc == DSGM_ACC_U8 ? dsgm::launch_init_u8(a, stream)
                                    : dsgm::launch_init(a, in_dtype, acc, stream);
  if (e != hipSuccess) return hip_fail(e, "dsgm_state_init_from_frame launch");
  return ok();
}

}  // extern "C"

namespace {

// dsgm_forward with an optional forced launch shape (block, pixels per lane;
// 0 = the usual choice), which the tuner uses to time its candidates
int forward_impl(const void* frames, dsgm_in_dtype in_dtype, dsgm_shape shape, dsgm_acc acc,
                 const dsgm_params* params, dsgm_state* state, uint8_t* masks, void* bg,
                 void* ckpt, size_t ckpt_bytes, int32_t ckpt_every, uint8_t* codes,
                 hipStream_t stream, int force_block, int force_vector) {
  int rc;
  if ((rc = check_types_u8(in_dtype, acc))) return rc;
  if ((rc = check_params(params))) return rc;
  const bool as_run = acc == DSGM_ACC_U8;
  if (as_run && (bg || ckpt))
    return fail(DSGM_E_UNSUPPORTED, "the 8-bit as-run model has no bg or checkpoint output");
  const size_t ie = in_size(in_dtype), ae = acc_size(acc), oe = io_size(acc);
  if ((rc = check_shape(shape, ie > oe ? ie : oe))) return rc;
  if (!state) return fail(DSGM_E_ARG, "state is NULL");
  const int64_t px = shape.H * shape.W;
  if (px == 0 || shape.T == 0) return ok();
  if (!frames) return fail(DSGM_E_ARG, "frames is NULL");
  if (!masks) return fail(DSGM_E_ARG, "masks is NULL");
  if (!state->mean_a || !state->var_a || !state->mean_c || !state->var_c || !state->age_a ||
      !state->age_c)
    return fail(DSGM_E_ARG, "a state plane is NULL");
  if (ckpt && ckpt_every < 1) return fail(DSGM_E_ARG, "ckpt_every = %d < 1", ckpt_every);
  if (ckpt && ckpt_bytes < dsgm_ckpt_bytes(shape, acc, ckpt_every))
    return fail(DSGM_E_WORKSPACE, "checkpoint buffer of %zu bytes, %zu needed", ckpt_bytes,
                dsgm_ckpt_bytes(shape, acc, ckpt_every));
  const void* ptrs[11] = {frames, masks, bg, codes, state->mean_a, state->var_a,
                          state->mean_c, state->var_c, state->age_a, state->age_c, ckpt};
  const size_t elem[11] = {ie, 1, oe, 1, ae, ae, ae, ae, 1, 1, 256};
  for (int i = 0; i < 11; ++i) {
    const size_t need = i == 10 ? 16 : elem[i];
    if (ptrs[i] && !aligned(ptrs[i], need))
      return fail(DSGM_E_ALIGN, "pointer argument %d is not aligned to %zu bytes", i, need);
  }
  const int widest = pick_vector(shape, ptrs, elem, 10);
  // pixels per lane the layout allows: sizes, strides and every base pointer,
  // the checkpoint's included
  auto legal = [&](int v) { return widest % v == 0 && (!ckpt || aligned(ckpt, ae * v)); };
  int P = std::min(widest, preferred_vector(in_dtype, acc));
  if (!legal(P)) P = 1;
  if (as_run) P = widest;  // four one-byte pixels per lane when the layout allows
  // 192-thread workgroups for the time-fused FP64 forward at two pixels per
  // lane: 0.8-1.3 % faster than 256 on 1920 x 2560 x 500 on two machines
  // (interleaved runs; 64 and 128 were not faster); 256 elsewhere
  int block = (in_dtype == DSGM_IN_F64 && acc == DSGM_ACC_F64 && P == 2 && shape.T > 1) ? 192 : 256;
  const int tflags = (bg ? DSGM_TUNE_BG : 0) | (ckpt ? DSGM_TUNE_CKPT : 0) |
                     (params->mask_rule == DSGM_MASK_PRINTED ? DSGM_TUNE_PRINTED : 0);
  int tb = force_block, tv = force_vector;
  const int bo = g_block_override.load(std::memory_order_relaxed);
  const int vo = g_vector_override.load(std::memory_order_relaxed);
  if (!tb && !bo && !vo) tune_lookup(TuneKey{in_dtype, acc, shape.H, shape.W, tflags}, &tb, &tv);
  if (tb) block = tb;
  if (tv && legal(tv)) P = tv;
  if (vo && legal(vo)) P = vo;
  if (bo) block = bo;
  if (codes && !as_run) P = 1;  // the decision-code (debug) variants run one pixel per lane

  dsgm::FwdArgs a;
  memset(&a, 0, sizeof(a));
  a.frames = frames;
  a.masks = masks;
  a.bg = bg;
  a.codes = codes;
  a.mean_a = state->mean_a;
  a.var_a = state->var_a;
  a.mean_c = state->mean_c;
  a.var_c = state->var_c;
  a.age_a = state->age_a;
  a.age_c = state->age_c;
  a.ckpt = ckpt;
  a.ckpt_every = ckpt ? ckpt_every : 1;
  const dsgm::geom::CkptLayout cl = dsgm::geom::ckpt_layout(px, int64_t(ae));
  a.ckpt_fplane = cl.fplane;
  a.ckpt_aplane = cl.aplane;
  a.ckpt_slot_bytes = cl.slot;
  a.T = shape.T;
  a.H = shape.H;
  a.W = shape.W;
  a.row_stride = shape.row_stride;
  a.frame_stride = shape.frame_stride;
  a.groups_per_row = shape.W / P;
  a.ngroups = shape.H * (shape.W / P);
  a.theta_s = params->theta_s;
  a.theta_d = params->theta_d;
  a.var_init = as_run ? stored_u8(params->var_init) : params->var_init;
  a.var_floor = params->var_floor;
  a.mask_floor = params->mask_floor;
  a.age_max = params->age_max;
  a.weight_rule = params->weight_rule;
  a.mask_rule = params->mask_rule;
  const int flags = (bg ? dsgm::FWD_BG : 0) | (codes ? dsgm::FWD_CODES : 0) |
                    (ckpt ? dsgm::FWD_CKPT : 0) |
                    (params->mask_rule == DSGM_MASK_PRINTED ? dsgm::FWD_PRINTED : 0);
  hipError_t e = as_run ? dsgm::launch_fwd_u8(a, P, flags, block, stream)
                        : dsgm::launch_forward(a, in_dtype, acc, P, flags, block, stream);
  if (e != hipSuccess) return hip_fail(e, "dsgm_forward launch");
  return ok();
}

// the tuner's buffers, carved from one workspace in 256-byte-aligned pieces
struct TuneLayout {
  dsgm_shape shape;
  int64_t frames = 0, masks = 0, bg = 0, ckpt = 0, planes = 0, ages = 0, bytes = 0;
  size_t ckpt_bytes = 0;
};

TuneLayout tune_layout(int in_dtype, int acc, const dsgm_shape& s, int flags) {
  TuneLayout L;
  const int64_t T = std::min<int64_t>(s.T, kTuneFrames), px = s.H * s.W;
  L.shape = dsgm_shape{T, s.H, s.W, s.W, px};
  const int64_t n = T * px;
  int64_t off = 0;
  auto take = [&](int64_t b) { const int64_t o = off; off += pad256(b); return o; };
  L.frames = take(n * int64_t(in_size(in_dtype)));
  L.masks = take(n);
  if (flags & DSGM_TUNE_BG) L.bg = take(n * int64_t(io_size(acc)));
  if (flags & DSGM_TUNE_CKPT) {
    L.ckpt_bytes = dsgm_ckpt_bytes(L.shape, dsgm_acc(acc), kTuneCkptEvery);
    L.ckpt = take(int64_t(L.ckpt_bytes));
  }
  L.planes = take(4 * pad256(px * int64_t(acc_size(acc))));
  L.ages = take(2 * pad256(px));
  L.bytes = off;
  return L;
}

int check_tune_args(int in_dtype, int acc, const dsgm_shape& shape, int flags) {
  int rc;
  if ((rc = check_types_u8(in_dtype, acc))) return rc;
  if (flags & ~kTuneFlags) return fail(DSGM_E_ARG, "flags = %d: unknown bits", flags);
  if (acc == DSGM_ACC_U8 && (flags & (DSGM_TUNE_BG | DSGM_TUNE_CKPT)))
    return fail(DSGM_E_UNSUPPORTED, "the 8-bit as-run model has no bg or checkpoint output");
  const size_t ie = in_size(in_dtype), oe = io_size(acc);
  const dsgm_shape dense{std::min<int64_t>(shape.T, kTuneFrames), shape.H, shape.W, shape.W,
                         shape.H * shape.W};
  if (shape.T < 0 || shape.H < 0 || shape.W < 0)
    return fail(DSGM_E_SHAPE, "negative size T=%lld H=%lld W=%lld", (long long)shape.T,
                (long long)shape.H, (long long)shape.W);
  return check_shape(dense, ie > oe ? ie : oe);
}

}  // namespace

extern "C" {

int dsgm_forward(const void* frames, dsgm_in_dtype in_dtype, dsgm_shape shape, dsgm_acc acc,
                 const dsgm_params* params, dsgm_state* state, uint8_t* masks, void* bg,
                 void* ckpt, size_t ckpt_bytes, int32_t ckpt_every, uint8_t* codes,
                 hipStream_t stream) {
  return forward_impl(frames, in_dtype, shape, acc, params, state, masks, bg, ckpt, ckpt_bytes,
                      ckpt_every, codes, stream, 0, 0);
}

size_t dsgm_autotune_bytes(dsgm_in_dtype in_dtype, dsgm_acc acc, dsgm_shape shape,
                           int32_t flags) {
  if (check_tune_args(in_dtype, acc, shape, flags)) return 0;
  if (shape.T == 0 || shape.H * shape.W == 0) return 0;
  return size_t(tune_layout(in_dtype, acc, shape, flags).bytes);
}

int dsgm_autotune(dsgm_in_dtype in_dtype, dsgm_acc acc, dsgm_shape shape, int32_t flags,
                  void* workspace, size_t ws_bytes, int32_t* chosen, hipStream_t stream) {
  int rc;
  if (chosen) chosen[0] = chosen[1] = 0;
  if ((rc = check_tune_args(in_dtype, acc, shape, flags))) return rc;
  if (shape.T == 0 || shape.H * shape.W == 0) return ok();
  const TuneLayout L = tune_layout(in_dtype, acc, shape, flags);
  if (!workspace) return fail(DSGM_E_ARG, "workspace is NULL");
  if (!aligned(workspace, 256)) return fail(DSGM_E_ALIGN, "workspace is not 256-byte aligned");
  if (ws_bytes < size_t(L.bytes))
    return fail(DSGM_E_WORKSPACE, "workspace of %zu bytes, %lld needed", ws_bytes,
                (long long)L.bytes);
  char* w = static_cast<char*>(workspace);
  const int64_t px = shape.H * shape.W;
  void* frames = w + L.frames;
  uint8_t* masks = reinterpret_cast<uint8_t*>(w + L.masks);
  void* bg = (flags & DSGM_TUNE_BG) ? w + L.bg : nullptr;
  void* ckpt = (flags & DSGM_TUNE_CKPT) ? w + L.ckpt : nullptr;
  const int64_t fplane = pad256(px * int64_t(acc_size(acc)));
  dsgm_state st;
  st.mean_a = w + L.planes;
  st.var_a = w + L.planes + fplane;
  st.mean_c = w + L.planes + 2 * fplane;
  st.var_c = w + L.planes + 3 * fplane;
  st.age_a = reinterpret_cast<uint8_t*>(w + L.ages);
  st.age_c = reinterpret_cast<uint8_t*>(w + L.ages + pad256(px));
  dsgm_params p;
  dsgm_params_default(&p, in_dtype == DSGM_IN_U8 ? 255.0 : 2.0,
                      (flags & DSGM_TUNE_PRINTED) ? DSGM_MASK_PRINTED : DSGM_MASK_VARIANCE);

  hipError_t e = dsgm::launch_tune_fill(frames, in_dtype, L.shape.T * px, 1, stream);
  if (e != hipSuccess) return hip_fail(e, "dsgm_autotune fill");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if ((e = hipEventCreate(&e0)) != hipSuccess) return hip_fail(e, "dsgm_autotune event");
  if ((e = hipEventCreate(&e1)) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_fail(e, "dsgm_autotune event");
  }
  // two rounds over the candidates, each candidate's time the better of its
  // two (interleaving keeps clock and cache drift from favouring one)
  // (192 is the FP64 forward's default: the table must be able to hold it)
  constexpr int kBlocks = 4, kVectors = 3, kCand = kBlocks * kVectors;
  const int blocks[kBlocks] = {64, 128, 192, 256}, vectors[kVectors] = {1, 2, 4};
  constexpr int kReps = 4, kRounds = 2;
  float best_ms[kCand];
  for (int c = 0; c < kCand; ++c) best_ms[c] = -1.f;
  rc = DSGM_OK;
  for (int round = 0; round < kRounds && rc == DSGM_OK; ++round) {
    for (int c = 0; c < kCand && rc == DSGM_OK; ++c) {
      const int b = blocks[c / kVectors], v = vectors[c % kVectors];
      if (shape.W % v) continue;
      // every candidate starts from the same state; one untimed call warms up
      if ((rc = dsgm_state_init_from_frame(frames, in_dtype, L.shape, acc, &p, &st, stream)))
        break;
      for (int r = 0; r <= kReps && rc == DSGM_OK; ++r) {
        if (r == 1 && (e = hipEventRecord(e0, stream)) != hipSuccess) {
          rc = hip_fail(e, "dsgm_autotune event record");
          break;
        }
        rc = forward_impl(frames, in_dtype, L.shape, acc, &p, &st, masks, bg, ckpt, L.ckpt_bytes,
                          kTuneCkptEvery, nullptr, stream, b, v);
      }
      if (rc != DSGM_OK) break;
      float ms = 0.f;
      if ((e = hipEventRecord(e1, stream)) != hipSuccess ||
          (e = hipEventSynchronize(e1)) != hipSuccess ||
          (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) {
        rc = hip_fail(e, "dsgm_autotune timing");
        break;
      }
      if (best_ms[c] < 0.f || ms < best_ms[c]) best_ms[c] = ms;
    }
  }
  int best = -1;
  for (int c = 0; c < kCand; ++c)
    if (best_ms[c] >= 0.f && (best < 0 || best_ms[c] < best_ms[best])) best = c;
  const int best_block = best >= 0 ? blocks[best / kVectors] : 256;
  const int best_vector = best >= 0 ? vectors[best % kVectors] : 1;
  (void)hipEventDestroy(e0);  // release failures change nothing for the caller
  (void)hipEventDestroy(e1);
  if (rc != DSGM_OK) return rc;
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune[TuneKey{in_dtype, acc, shape.H, shape.W, flags}] = {best_block, best_vector};
  }
  if (chosen) {
    chosen[0] = best_block;
    chosen[1] = best_vector;
  }
  return ok();
}

int dsgm_autotune_lookup(dsgm_in_dtype in_dtype, dsgm_acc acc, dsgm_shape shape, int32_t flags,
                         int32_t* chosen) {
  int rc;
  if (!chosen) return fail(DSGM_E_ARG, "chosen is NULL");
  chosen[0] = chosen[1] = 0;
  if ((rc = check_tune_args(in_dtype, acc, shape, flags))) return rc;
  int b = 0, v = 0;
  if (tune_lookup(TuneKey{in_dtype, acc, shape.H, shape.W, flags}, &b, &v)) {
    chosen[0] = b;
    chosen[1] = v;
  }
  return ok();
}

int dsgm_autotune_clear(void) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune.clear();
  return ok();
}

int dsgm_count_nonfinite(const void* frames, dsgm_in_dtype in_dtype, dsgm_shape shape,
                         uint64_t* count, hipStream_t stream) {
  int rc;
  if (in_dtype < DSGM_IN_F64 || in_dtype > DSGM_IN_U8)
    return fail(DSGM_E_DTYPE, "in_dtype = %d invalid", in_dtype);
  if ((rc = check_shape(shape, in_size(in_dtype)))) return rc;
  if (!count) return fail(DSGM_E_ARG, "count is NULL");
  if (!aligned(count, 8)) return fail(DSGM_E_ALIGN, "count is not 8-byte aligned");
  if (shape.T * shape.H * shape.W > 0 && !frames) return fail(DSGM_E_ARG, "frames is NULL");
  if (frames && !aligned(frames, in_size(in_dtype)))
    return fail(DSGM_E_ALIGN, "frames not aligned to %zu bytes", in_size(in_dtype));
  dsgm::CountArgs a{shape.T, shape.H, shape.W, shape.row_stride, shape.frame_stride,
                    reinterpret_cast<unsigned long long*>(count)};
  const hipError_t e = dsgm::launch_count_nonfinite(frames, in_dtype, a, stream);
  if (e != hipSuccess) return hip_fail(e, "dsgm_count_nonfinite launch");
  return ok();
}

int dsgm_gauss_weights(int32_t n, double sigma, double* weights) {
  if (n < 1 || n > 7 || n % 2 == 0) return fail(DSGM_E_ARG, "blur taps n = %d (odd, 1..7)", n);
  if (!(sigma > 0.0) || !std::isfinite(sigma)) return fail(DSGM_E_ARG, "sigma must be > 0");
  if (!weights) return fail(DSGM_E_ARG, "weights is NULL");
  const int32_t r = (n - 1) / 2;
  double sum = 0.0;
  for (int32_t i = 0; i < n; ++i) {
    const double d = double(i - r);
    weights[i] = std::exp(-(d * d) / (2.0 * sigma * sigma));
    sum += weights[i];
  }
  for (int32_t i = 0; i < n; ++i) weights[i] = weights[i] / sum;
  return ok();
}

int dsgm_forward_filtered(const void* frames, dsgm_in_dtype in_dtype, dsgm_shape shape,
                          dsgm_acc acc, const dsgm_params* params, const dsgm_filter* filter,
                          dsgm_state* state, uint8_t* masks, void* bg, void* filtered,
                          uint8_t* codes, hipStream_t stream) {
  int rc;
  // the 8-bit pair runs the appendix's 8-bit preprocessing and update
  const bool as_run = in_dtype == DSGM_IN_U8 || acc == DSGM_ACC_U8;
  if (as_run) {
    if (in_dtype != DSGM_IN_U8 || acc != DSGM_ACC_U8)
      return fail(DSGM_E_DTYPE, "U8 frames and U8 state go together");
  } else if ((rc = check_types(in_dtype, acc))) {
    return rc;
  }
  if ((rc = check_params(params))) return rc;
  if (as_run && bg) return fail(DSGM_E_UNSUPPORTED, "the 8-bit as-run model has no bg output");
  if (!filter) return fail(DSGM_E_ARG, "filter is NULL");
  if (filter->n < 0 || (filter->n > 0 && filter->n % 2 == 0))
    return fail(DSGM_E_ARG, "blur taps n = %d (0 or odd)", filter->n);
  if (filter->n > 7) return fail(DSGM_E_UNSUPPORTED, "blur taps n = %d > 7", filter->n);
  if (filter->n == 1 && filter->weights[0] != 1.0)
    return fail(DSGM_E_UNSUPPORTED, "a one-tap blur must have weight 1");
  if (filter->median != 0 && filter->median != 1)
    return fail(DSGM_E_ARG, "median = %d (0 or 1)", filter->median);
  for (int i = 0; i < filter->n; ++i)
    if (!std::isfinite(filter->weights[i])) return fail(DSGM_E_ARG, "blur weight %d not finite", i);
  const size_t ie = in_size(in_dtype), ae = acc_size(acc), oe = as_run ? 1 : io_size(acc);
  if ((rc = check_shape(shape, ie > oe ? ie : oe))) return rc;
  if (!state) return fail(DSGM_E_ARG, "state is NULL");
  if (shape.H * shape.W == 0 || shape.T == 0) return ok();
  if (!frames) return fail(DSGM_E_ARG, "frames is NULL");
  if (!masks) return fail(DSGM_E_ARG, "masks is NULL");
  if (!state->mean_a || !state->var_a || !state->mean_c || !state->var_c || !state->age_a ||
      !state->age_c)
    return fail(DSGM_E_ARG, "a state plane is NULL");
  const void* ptrs[10] = {frames, masks, bg, codes, filtered, state->mean_a, state->var_a,
                          state->mean_c, state->var_c, nullptr};
  const size_t elem[10] = {ie, 1, oe, 1, oe, ae, ae, ae, ae, 1};
  for (int i = 0; i < 9; ++i)
    if (ptrs[i] && !aligned(ptrs[i], elem[i]))
      return fail(DSGM_E_ALIGN, "pointer argument %d is not aligned to %zu bytes", i, elem[i]);
  // the kernel writes four adjacent pixels with one vector store when the row
  // and frame strides and W are multiples of four; the bases must allow it
  const void* vec_ptrs[4] = {masks, bg, codes, filtered};
  const size_t vec_elem[4] = {1, oe, 1, oe};
  for (int i = 0; i < 4; ++i)
    if (vec_ptrs[i] && !aligned(vec_ptrs[i], 4 * vec_elem[i]))
      return fail(DSGM_E_ALIGN, "output %d is not aligned to %zu bytes", i, 4 * vec_elem[i]);

  dsgm::PreArgs a;
  memset(&a, 0, sizeof(a));
  a.frames = frames;
  a.masks = masks;
  a.bg = bg;
  a.filtered = filtered;
  a.codes = codes;
  a.mean_a = state->mean_a;
  a.var_a = state->var_a;
  a.mean_c = state->mean_c;
  a.var_c = state->var_c;
  a.age_a = state->age_a;
  a.age_c = state->age_c;
  a.T = shape.T;
  a.H = shape.H;
  a.W = shape.W;
  a.row_stride = shape.row_stride;
  a.frame_stride = shape.frame_stride;
  a.tiles_x = (shape.W + dsgm::geom::pre::TW - 1) / dsgm::geom::pre::TW;
  a.tiles_y = (shape.H + dsgm::geom::pre::TH - 1) / dsgm::geom::pre::TH;
  if (a.tiles_x * a.tiles_y >= (int64_t(1) << 31))
    return fail(DSGM_E_SHAPE, "too many tiles");
  a.theta_s = params->theta_s;
  a.theta_d = params->theta_d;
  a.var_init = as_run ? stored_u8(params->var_init) : params->var_init;
  a.var_floor = params->var_floor;
  a.mask_floor = params->mask_floor;
  a.age_max = params->age_max;
  a.weight_rule = params->weight_rule;
  a.mask_rule = params->mask_rule;
  for (int i = 0; i < filter->n; ++i) a.w[i] = filter->weights[i];
  const int rg = filter->n > 0 ? (filter->n - 1) / 2 : 0;  // n = 1 (weight 1) is no blur
  hipError_t e = as_run ? dsgm::launch_pre_u8(a, rg, filter->median != 0, stream)
                        : dsgm::launch_pre(a, in_dtype, acc, rg, filter->median != 0, stream);
  if (e != hipSuccess) return hip_fail(e, "dsgm_forward_filtered launch");
  return ok();
}

int dsgm_forward_warped(const void* frame, dsgm_in_dtype in_dtype, dsgm_shape shape,
                        dsgm_acc acc, const dsgm_params* params, const double* inv_map,
                        const dsgm_state* src, dsgm_state* dst, uint8_t* masks, void* bg,
                        uint8_t* codes, hipStream_t stream) {
  int rc;
  if ((rc = check_types(in_dtype, acc))) return rc;
  if ((rc = check_params(params))) return rc;
  if (!inv_map) return fail(DSGM_E_ARG, "inv_map is NULL");
  for (int i = 0; i < 9; ++i)
    if (!std::isfinite(inv_map[i])) return fail(DSGM_E_ARG, "inv_map[%d] is not finite", i);
  const size_t ie = in_size(in_dtype), ae = acc_size(acc), oe = io_size(acc);
  if ((rc = check_shape(shape, ie > oe ? ie : oe))) return rc;
  if (shape.T != 1) return fail(DSGM_E_SHAPE, "T = %lld, need one frame per call",
                                (long long)shape.T);
  if (!src || !dst) return fail(DSGM_E_ARG, "src or dst is NULL");
  const int64_t px = shape.H * shape.W;
  if (px == 0) return ok();
  if (!frame) return fail(DSGM_E_ARG, "frame is NULL");
  if (!masks) return fail(DSGM_E_ARG, "masks is NULL");
  const void* sp[6] = {src->mean_a, src->var_a, src->mean_c, src->var_c, src->age_a, src->age_c};
  void* dp[6] = {dst->mean_a, dst->var_a, dst->mean_c, dst->var_c, dst->age_a, dst->age_c};
  const size_t pe[6] = {ae, ae, ae, ae, 1, 1};
  for (int i = 0; i < 6; ++i) {
    if (!sp[i] || !dp[i]) return fail(DSGM_E_ARG, "a state plane is NULL");
    if (!aligned(sp[i], pe[i]) || !aligned(dp[i], pe[i]))
      return fail(DSGM_E_ALIGN, "state plane %d is not aligned to %zu bytes", i, pe[i]);
  }
  // the gathers read src while dst is written: no dst plane may overlap a src plane
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) {
      const uintptr_t d0 = reinterpret_cast<uintptr_t>(dp[i]), d1 = d0 + size_t(px) * pe[i];
      const uintptr_t s0 = reinterpret_cast<uintptr_t>(sp[j]), s1 = s0 + size_t(px) * pe[j];
      if (d0 < s1 && s0 < d1) return fail(DSGM_E_ARG, "dst plane %d overlaps src plane %d", i, j);
    }
  const void* ptrs[4] = {frame, masks, bg, codes};
  const size_t elem[4] = {ie, 1, oe, 1};
  for (int i = 0; i < 4; ++i)
    if (ptrs[i] && !aligned(ptrs[i], elem[i]))
      return fail(DSGM_E_ALIGN, "pointer argument %d is not aligned to %zu bytes", i, elem[i]);

  dsgm::WarpArgs a;
  memset(&a, 0, sizeof(a));
  a.frame = frame;
  a.masks = masks;
  a.bg = bg;
  a.codes = codes;
  a.src_mean_a = src->mean_a;
  a.src_var_a = src->var_a;
  a.src_mean_c = src->mean_c;
  a.src_var_c = src->var_c;
  a.src_age_a = src->age_a;
  a.src_age_c = src->age_c;
  a.dst_mean_a = dst->mean_a;
  a.dst_var_a = dst->var_a;
  a.dst_mean_c = dst->mean_c;
  a.dst_var_c = dst->var_c;
  a.dst_age_a = dst->age_a;
  a.dst_age_c = dst->age_c;
  a.H = shape.H;
  a.W = shape.W;
  a.row_stride = shape.row_stride;
  for (int i = 0; i < 9; ++i) a.map[i] = inv_map[i];
  a.theta_s = params->theta_s;
  a.theta_d = params->theta_d;
  a.var_init = params->var_init;
  a.var_floor = params->var_floor;
  a.mask_floor = params->mask_floor;
  a.age_max = params->age_max;
  a.weight_rule = params->weight_rule;
  a.mask_rule = params->mask_rule;
  if ((px + 255) / 256 >= (int64_t(1) << 31)) return fail(DSGM_E_SHAPE, "frame too large");
  hipError_t e = dsgm::launch_warp(a, in_dtype, acc, stream);
  if (e != hipSuccess) return hip_fail(e, "dsgm_forward_warped launch");
  return ok();
}

int dsgm_forward_grid(const void* frames, dsgm_in_dtype in_dtype, dsgm_shape shape, dsgm_acc acc,
                      const dsgm_params* params, int32_t b, dsgm_state* state, uint8_t* masks,
                      void* bg, uint8_t* codes, hipStream_t stream) {
  int rc;
  if ((rc = check_types(in_dtype, acc))) return rc;
  if ((rc = check_params(params))) return rc;
  if (b != 1 && b != 2 && b != 4) return fail(DSGM_E_UNSUPPORTED, "block size %d (1, 2 or 4)", b);
  const size_t ie = in_size(in_dtype), ae = acc_size(acc), oe = io_size(acc);
  if ((rc = check_shape(shape, ie))) return rc;
  if (!state) return fail(DSGM_E_ARG, "state is NULL");
  if (shape.H * shape.W == 0 || shape.T == 0) return ok();
  if (!frames) return fail(DSGM_E_ARG, "frames is NULL");
  if (!masks) return fail(DSGM_E_ARG, "masks is NULL");
  if (!state->mean_a || !state->var_a || !state->mean_c || !state->var_c || !state->age_a ||
      !state->age_c)
    return fail(DSGM_E_ARG, "a state plane is NULL");
  const void* ptrs[8] = {frames, masks, bg, codes, state->mean_a, state->var_a, state->mean_c,
                         state->var_c};
  const size_t elem[8] = {ie, 1, oe, 1, ae, ae, ae, ae};
  for (int i = 0; i < 8; ++i)
    if (ptrs[i] && !aligned(ptrs[i], elem[i]))
      return fail(DSGM_E_ALIGN, "pointer argument %d is not aligned to %zu bytes", i, elem[i]);
  dsgm::GridArgs a;
  memset(&a, 0, sizeof(a));
  a.frames = frames;
  a.masks = masks;
  a.bg = bg;
  a.codes = codes;
  a.mean_a = state->mean_a;
  a.var_a = state->var_a;
  a.mean_c = state->mean_c;
  a.var_c = state->var_c;
  a.age_a = state->age_a;
  a.age_c = state->age_c;
  a.T = shape.T;
  a.H = shape.H;
  a.W = shape.W;
  a.row_stride = shape.row_stride;
  a.frame_stride = shape.frame_stride;
  a.Hb = (shape.H + b - 1) / b;
  a.Wb = (shape.W + b - 1) / b;
  a.vec_ok = shape.row_stride % b == 0 && (shape.T <= 1 || shape.frame_stride % b == 0) &&
             aligned(frames, ie * b) && aligned(masks, size_t(b));
  a.theta_s = params->theta_s;
  a.theta_d = params->theta_d;
  a.var_init = params->var_init;
  a.var_floor = params->var_floor;
  a.mask_floor = params->mask_floor;
  a.age_max = params->age_max;
  a.weight_rule = params->weight_rule;
  a.mask_rule = params->mask_rule;
  hipError_t e = dsgm::launch_grid(a, in_dtype, acc, b, stream);
  if (e != hipSuccess) return hip_fail(e, "dsgm_forward_grid launch");
  return ok();
}

size_t dsgm_workspace_bytes(dsgm_shape shape, dsgm_acc acc) {
  if (acc != DSGM_ACC_F64 && acc != DSGM_ACC_F32 && acc != DSGM_ACC_F64_IO32 &&
      acc != DSGM_ACC_F32X2)
    return 0;
  if (shape.T < 0 || shape.H < 0 || shape.W < 0) return 0;
  return size_t(dsgm::geom::ws_bytes(shape.H * shape.W));
}

namespace {

// Argument checks of both adjoint entry points, all before any HIP call.
// `workspace` is the caller's buffer (dsgm_backward) or NULL when the library
// brings its own (dsgm_backward_noalloc).
int backward_validate(const void* frames, dsgm_in_dtype in_dtype, dsgm_shape shape,
                      dsgm_acc acc, const dsgm_params* params, const void* ckpt,
                      size_t ckpt_bytes, int32_t ckpt_every, const void* grad_bg,
                      const dsgm_grad_state* grad_state_T, const void* grad_frames,
                      const dsgm_grad_state* grad_state0, const double* grad_var_init,
                      const void* workspace) {
  int rc;
  if ((rc = check_types_x2(in_dtype, acc))) return rc;
  if ((rc = check_params(params))) return rc;
  const size_t ie = in_size(in_dtype), oe = io_size(acc);
  if ((rc = check_shape(shape, ie > oe ? ie : oe))) return rc;
  const int64_t px = shape.H * shape.W;
  const int64_t n = shape.T * px;
  if (!grad_var_init) return fail(DSGM_E_ARG, "grad_var_init is NULL");
  if (px > 0) {
    if (!grad_state0 || !grad_state0->mean_a || !grad_state0->var_a || !grad_state0->mean_c ||
        !grad_state0->var_c)
      return fail(DSGM_E_ARG, "grad_state0 or one of its planes is NULL");
    if (grad_state_T && (!grad_state_T->mean_a || !grad_state_T->var_a ||
                         !grad_state_T->mean_c || !grad_state_T->var_c))
      return fail(DSGM_E_ARG, "a plane of grad_state_T is NULL");
  }
  if (n > 0) {
    if (!frames) return fail(DSGM_E_ARG, "frames is NULL");
    if (!grad_frames) return fail(DSGM_E_ARG, "grad_frames is NULL");
    if (!ckpt) return fail(DSGM_E_ARG, "ckpt is NULL");
    if (ckpt_every < 1) return fail(DSGM_E_ARG, "ckpt_every = %d < 1", ckpt_every);
    if (ckpt_bytes < dsgm_ckpt_bytes(shape, acc, ckpt_every))
      return fail(DSGM_E_WORKSPACE, "checkpoint buffer of %zu bytes, %zu needed", ckpt_bytes,
                  dsgm_ckpt_bytes(shape, acc, ckpt_every));
  }
  const void* ptrs[14] = {frames, grad_bg, grad_frames, workspace, grad_var_init, ckpt,
                          grad_state0 ? grad_state0->mean_a : nullptr,
                          grad_state0 ? grad_state0->var_a : nullptr,
                          grad_state0 ? grad_state0->mean_c : nullptr,
                          grad_state0 ? grad_state0->var_c : nullptr,
                          grad_state_T ? grad_state_T->mean_a : nullptr,
                          grad_state_T ? grad_state_T->var_a : nullptr,
                          grad_state_T ? grad_state_T->mean_c : nullptr,
                          grad_state_T ? grad_state_T->var_c : nullptr};
  const size_t elem[14] = {ie, oe, oe, 8, 8, 16, oe, oe, oe, oe, oe, oe, oe, oe};
  for (int i = 0; i < 14; ++i)
    if (ptrs[i] && !aligned(ptrs[i], elem[i]))
      return fail(DSGM_E_ALIGN, "pointer argument %d is not aligned to %zu bytes", i, elem[i]);
  return DSGM_OK;
}

// The launches of the adjoint (arguments already validated), with the
// per-pixel d/d(var_init) terms at gvi_px (H*W doubles, device) and the
// reduction's partial sums at partial (2 * geom::REDUCE_BLOCKS doubles,
// device).  Every pixel's term is written by the adjoint kernel and every
// partial by the reduction, so neither buffer needs clearing.
int backward_launch(const char* fn, const void* frames, dsgm_in_dtype in_dtype, dsgm_shape shape,
                    dsgm_acc acc, const dsgm_params* params, const void* ckpt,
                    int32_t ckpt_every, const void* grad_bg, const dsgm_grad_state* grad_state_T,
                    void* grad_frames, dsgm_grad_state* grad_state0, double* grad_var_init,
                    double* gvi_px, double* partial, hipStream_t stream) {
  const size_t ae = acc_size(acc);
  const int64_t px = shape.H * shape.W;
  hipError_t e;
  if (px > 0) {
    dsgm::BwdArgs a;
    memset(&a, 0, sizeof(a));
    a.frames = frames;
    a.ckpt = ckpt;
    a.grad_bg = grad_bg;
    if (grad_state_T) {
      a.gst_mean_a = grad_state_T->mean_a;
      a.gst_var_a = grad_state_T->var_a;
      a.gst_mean_c = grad_state_T->mean_c;
      a.gst_var_c = grad_state_T->var_c;
    }
    a.grad_frames = grad_frames;
    a.gs0_mean_a = grad_state0->mean_a;
    a.gs0_var_a = grad_state0->var_a;
    a.gs0_mean_c = grad_state0->mean_c;
    a.gs0_var_c = grad_state0->var_c;
    a.gvi_px = gvi_px;
    a.ckpt_every = ckpt_every >= 1 ? ckpt_every : 1;
    const dsgm::geom::CkptLayout cl = dsgm::geom::ckpt_layout(px, int64_t(ae));
    a.ckpt_fplane = cl.fplane;
    a.ckpt_aplane = cl.aplane;
    a.ckpt_slot_bytes = cl.slot;
    a.T = shape.T;
    a.H = shape.H;
    a.W = shape.W;
    a.row_stride = shape.row_stride;
    a.frame_stride = shape.frame_stride;
    a.theta_s = params->theta_s;
    a.theta_d = params->theta_d;
    a.var_init = params->var_init;
    a.var_floor = params->var_floor;
    a.mask_floor = params->mask_floor;
    a.age_max = params->age_max;
    a.weight_rule = params->weight_rule;
    a.mask_rule = params->mask_rule;
    e = dsgm::launch_backward(a, in_dtype, acc, stream);
    if (e != hipSuccess) return hip_fail(e, fn);
  }
  e = dsgm::launch_reduce(gvi_px, px, partial, grad_var_init, stream);
  if (e != hipSuccess) return hip_fail(e, fn);
  return ok();
}

// The library's own buffer for the adjoint entry point that allocates
// nothing: room for DSGM_NOALLOC_MAX_PIXELS per-pixel terms and the
// reduction's partial sums.  Each device that runs the library holds one copy
// until the process ends.  Host code never passes this name to a kernel: it
// stands for a host-side shadow, not the device address; scratch_ptr() returns
// the device address of the current device's copy.
constexpr int64_t kScratchDoubles = int64_t(DSGM_NOALLOC_MAX_PIXELS) + 512;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The current device's copy of `scratch`, looked up once per device (with that
// device current) and kept.
int scratch_ptr(double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "dsgm_backward_noalloc: hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices)
    return fail(DSGM_E_UNSUPPORTED, "dsgm_backward_noalloc: device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "dsgm_backward_noalloc: hipGetSymbolAddress");
    if (!p) return fail(DSGM_E_HIP, "dsgm_backward_noalloc: no device address for the scratch");
    g_scratch_ptr[dev] = p;
  }
  *out = static_cast<double*>(g_scratch_ptr[dev]);
  return DSGM_OK;
}

}  // namespace

int dsgm_backward(const void* frames, dsgm_in_dtype in_dtype, dsgm_shape shape, dsgm_acc acc,
                  const dsgm_params* params, const void* ckpt, size_t ckpt_bytes,
                  int32_t ckpt_every, const void* grad_bg, const dsgm_grad_state* grad_state_T, void* grad_frames,
                  dsgm_grad_state* grad_state0, double* grad_var_init, void* workspace,
                  size_t workspace_bytes, hipStream_t stream) {
  int rc;
  if ((rc = backward_validate(frames, in_dtype, shape, acc, params, ckpt, ckpt_bytes, ckpt_every,
                              grad_bg, grad_state_T, grad_frames, grad_state0, grad_var_init,
                              workspace)))
    return rc;
  if (!workspace) return fail(DSGM_E_ARG, "workspace is NULL");
  const size_t need = dsgm_workspace_bytes(shape, acc);
  if (workspace_bytes < need)
    return fail(DSGM_E_WORKSPACE, "workspace of %zu bytes, %zu needed", workspace_bytes, need);
  const int64_t px = shape.H * shape.W;
  double* gvi_px = static_cast<double*>(workspace);
  double* partial =
      reinterpret_cast<double*>(static_cast<char*>(workspace) + dsgm::geom::ws_partial_offset(px));
  return backward_launch("dsgm_backward launch", frames, in_dtype, shape, acc, params, ckpt,
                         ckpt_every, grad_bg, grad_state_T, grad_frames, grad_state0,
                         grad_var_init, gvi_px, partial, stream);
}

int dsgm_backward_noalloc(const void* frames, dsgm_in_dtype in_dtype, dsgm_shape shape,
                          dsgm_acc acc, const dsgm_params* params, const void* ckpt,
                          size_t ckpt_bytes, int32_t ckpt_every, const void* grad_bg,
                          const dsgm_grad_state* grad_state_T, void* grad_frames,
                          dsgm_grad_state* grad_state0, double* grad_var_init,
                          hipStream_t stream) {
  int rc;
  if ((rc = backward_validate(frames, in_dtype, shape, acc, params, ckpt, ckpt_bytes, ckpt_every,
                              grad_bg, grad_state_T, grad_frames, grad_state0, grad_var_init,
                              nullptr)))
    return rc;
  const int64_t px = shape.H * shape.W;
  if (px > int64_t(DSGM_NOALLOC_MAX_PIXELS))
    return fail(DSGM_E_WORKSPACE, "dsgm_backward_noalloc: H*W = %lld pixels, at most %lld",
                (long long)px, (long long)DSGM_NOALLOC_MAX_PIXELS);
  double* base = nullptr;
  if ((rc = scratch_ptr(&base))) return rc;
  return backward_launch("dsgm_backward_noalloc launch", frames, in_dtype, shape, acc, params,
                         ckpt, ckpt_every, grad_bg, grad_state_T, grad_frames, grad_state0,
                         grad_var_init, base, base + int64_t(DSGM_NOALLOC_MAX_PIXELS), stream);
}

size_t dsgm_batch_plan_bytes(const dsgm_instance* instances, int32_t n, dsgm_in_dtype in_dtype,
                             dsgm_acc acc) {
  PlanLayout L;
  if (plan_layout(instances, n, in_dtype, acc, &L)) return 0;
  return size_t(L.bytes);
}

}  // extern "C"

namespace dsgm {

int plan_image(const dsgm_instance* instances, int32_t n, int in_dtype, int acc, void* plan_buffer,
               PlanImage* img) {
  PlanLayout L;
  int rc = plan_layout(instances, n, in_dtype, acc, &L);
  if (rc) return rc;
  if (!img) return fail(DSGM_E_ARG, "plan image is NULL");
  const int P = L.P;
  std::vector<char>& host = img->host;
  host.assign(size_t(L.bytes), 0);
  auto* desc = reinterpret_cast<dsgm::BatchInst*>(host.data() + L.inst_off);
  auto* items = reinterpret_cast<dsgm::BatchItem*>(host.data() + L.items_off);
  int64_t k = 0;
  int64_t stripe_at = L.stripes_off;
  for (int32_t i = 0; i < n; ++i) {
    const dsgm_instance& I = instances[i];
    dsgm::BatchInst& d = desc[i];
    d.frames = I.frames;
    d.masks = I.masks;
    d.bg = I.bg;
    // counters of an instance with no work are never cleared: none are kept
    d.fg_counts = (I.shape.H * I.shape.W == 0 || I.shape.T == 0) ? nullptr : I.fg_counts;
    d.stripes = nullptr;
    if (d.fg_counts) {
      d.stripes = reinterpret_cast<uint32_t*>(static_cast<char*>(plan_buffer) + stripe_at);
      stripe_at += pad_to(I.shape.T * dsgm::COUNT_STRIPES * 4, 256);
    }
    d.state[0] = I.state.mean_a;
    d.state[1] = I.state.var_a;
    d.state[2] = I.state.mean_c;
    d.state[3] = I.state.var_c;
    d.state[4] = I.state.age_a;
    d.state[5] = I.state.age_c;
    d.T = I.shape.T;
    d.H = I.shape.H;
    d.W = I.shape.W;
    d.row_stride = I.shape.row_stride;
    d.frame_stride = I.shape.frame_stride;
    d.groups_per_row = I.shape.W / P;
    if (I.shape.H * I.shape.W == 0 || I.shape.T == 0) continue;
    const int64_t ng = I.shape.H * (I.shape.W / P);
    for (int64_t g = 0; g < ng; g += dsgm::geom::ITEM_GROUPS) {
      items[k].inst = i;
      items[k].first_group = int32_t(g);
      items[k].count = int32_t(std::min<int64_t>(dsgm::geom::ITEM_GROUPS, ng - g));
      items[k].pad = 0;
      ++k;
    }
  }
  // longest processing time first: cost = frames x groups; ties keep instance order
  std::stable_sort(items, items + k, [&](const dsgm::BatchItem& x, const dsgm::BatchItem& y) {
    return desc[x.inst].T * x.count > desc[y.inst].T * y.count;
  });
  img->P = P;
  img->n_items = L.n_items;
  img->total = L.total;
  img->inst_off = L.inst_off;
  img->items_off = L.items_off;
  img->stripes_off = L.stripes_off;
  img->bytes = L.bytes;
  img->bg = L.bg;
  img->counts = L.counts;
  return DSGM_OK;
}

}  // namespace dsgm

extern "C" {

int dsgm_plan_batched(const dsgm_instance* instances, int32_t n, dsgm_in_dtype in_dtype,
                      dsgm_acc acc, void* plan_buffer, size_t plan_bytes, dsgm_batch_plan* plan,
                      hipStream_t stream) {
  PlanLayout L;
  int rc = plan_layout(instances, n, in_dtype, acc, &L);
  if (rc) return rc;
  if (!plan) return fail(DSGM_E_ARG, "plan is NULL");
  if (!plan_buffer) return fail(DSGM_E_ARG, "plan_buffer is NULL");
  if (!aligned(plan_buffer, 256)) return fail(DSGM_E_ALIGN, "plan_buffer is not 256-byte aligned");
  if (plan_bytes < size_t(L.bytes))
    return fail(DSGM_E_WORKSPACE, "plan buffer of %zu bytes, %lld needed", plan_bytes,
                (long long)L.bytes);
  dsgm::PlanImage img;
  if ((rc = dsgm::plan_image(instances, n, in_dtype, acc, plan_buffer, &img))) return rc;
  // persistent grid: as many 256-thread blocks as fit on the device at once
  int dev = 0, ncu = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  const void* fn = dsgm::batched_kernel_symbol(in_dtype, acc, img.P, img.bg ? dsgm::FWD_BG : 0);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, 0);
  if (e != hipSuccess) return hip_fail(e, "dsgm_plan_batched: device query");
  e = hipMemcpyAsync(plan_buffer, img.host.data(), size_t(img.bytes), hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "dsgm_plan_batched: copy");
  plan->device_plan = plan_buffer;
  plan->n_items = img.n_items;
  plan->total_elements = img.total;
  plan->n_instances = n;
  plan->in_dtype = in_dtype;
  plan->acc = acc;
  plan->vector = img.P;
  plan->grid = std::max(1, per_cu) * std::max(1, ncu);
  plan->has_bg = img.bg ? 1 : 0;
  plan->has_counts = img.counts ? 1 : 0;
  return ok();
}

int dsgm_forward_batched(const dsgm_batch_plan* plan, const dsgm_params* params,
                         hipStream_t stream) {
  int rc;
  if (!plan || !plan->device_plan) return fail(DSGM_E_ARG, "plan is NULL or not planned");
  if ((rc = check_types(plan->in_dtype, plan->acc))) return rc;
  if ((rc = check_params(params))) return rc;
  if (plan->vector != 1 && plan->vector != 2 && plan->vector != 4)
    return fail(DSGM_E_ARG, "plan.vector = %d invalid", plan->vector);
  if (plan->grid < 1) return fail(DSGM_E_ARG, "plan.grid = %d: at least one workgroup", plan->grid);
  if (plan->n_items == 0) return ok();
  char* base = static_cast<char*>(plan->device_plan);
  dsgm::BatchArgs a;
  memset(&a, 0, sizeof(a));
  a.counter = reinterpret_cast<unsigned long long*>(base);
  a.inst = reinterpret_cast<const dsgm::BatchInst*>(base + kPlanHeader);
  a.n_inst = plan->n_instances;
  a.items = reinterpret_cast<const dsgm::BatchItem*>(
      base + kPlanHeader + pad_to(int64_t(plan->n_instances) * int64_t(sizeof(dsgm::BatchInst)), 256));
  a.n_items = plan->n_items;
  a.theta_s = params->theta_s;
  a.theta_d = params->theta_d;
  a.var_init = params->var_init;
  a.var_floor = params->var_floor;
  a.mask_floor = params->mask_floor;
  a.age_max = params->age_max;
  a.weight_rule = params->weight_rule;
  a.mask_rule = params->mask_rule;
  const int flags = (plan->has_bg ? dsgm::FWD_BG : 0) |
                    (params->mask_rule == DSGM_MASK_PRINTED ? dsgm::FWD_PRINTED : 0);
  hipError_t e = dsgm::launch_batched(a, plan->in_dtype, plan->acc, plan->vector, flags,
                                      plan->grid, plan->has_counts != 0, stream);
  if (e != hipSuccess) return hip_fail(e, "dsgm_forward_batched launch");
  return ok();
}

// Launch-shape override used by the tuner and the tests: block size (64..256,
// multiple of 64, 0 = default) and pixels per lane (1, 2, 4; 0 = widest legal).
int dsgm_set_launch(int32_t block, int32_t vector) {
  if (block != 0 && (block < 64 || block > 256 || block % 64))
    return fail(DSGM_E_ARG, "block = %d: must be 0 or a multiple of 64 in 64..256", block);
  if (vector != 0 && vector != 1 && vector != 2 && vector != 4)
    return fail(DSGM_E_ARG, "vector = %d: must be 0, 1, 2 or 4", vector);
  g_block_override.store(block, std::memory_order_relaxed);
  g_vector_override.store(vector, std::memory_order_relaxed);
  return ok();
}

}  // extern "C"
