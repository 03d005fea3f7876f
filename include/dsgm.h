/*
 * dsgm.h -- C ABI of libdsgm.so: the Dual-Mode Single Gaussian Model (DSGM)
 * background update and foreground mask on an MI355X (gfx950) GPU.
 *
 * Method: Henderson & Vertescher, "An Analysis of Parallelized Motion Masking
 * Using Dual-Mode Single Gaussian Models" (arXiv:1702.05156):
 *   Sec. 2.2  Single Gaussian Model: per pixel, the mean and the variance are
 *             blended with the new intensity at an age-dependent rate and the
 *             age grows by one up to a cap of 30 (grid of one pixel, so the
 *             block mean is the pixel's intensity).
 *   Sec. 2.3  Dual-mode SGM: an apparent model A and a candidate model C; test
 *             A, then C, update the one that matches, else reset C; promote C
 *             to A when it is older.
 *   Appendix  "Dual-mode SGM Inner Update Code Snippet": the variance floor in
 *             the match tests and the 0/255 foreground rule.
 *   Sec. 3.4  the parallel decomposition: pixels are independent.
 *
 * Conventions
 *   - Every pointer argument is a DEVICE pointer unless marked (host).  The
 *     caller owns all memory; no call allocates device memory.
 *   - Element strides: frames and every per-frame output (masks, bg, codes,
 *     gradients of frames and of bg) are T x H x W arrays addressed as
 *     t*frame_stride + h*row_stride + w, in elements of their own type.  State
 *     planes and their gradients are dense H x W (pitch W).
 *   - "accumulation type" below means the state type of dsgm_acc; "array type"
 *     the type of bg and of the gradient arrays (FP32 for F64_IO32).
 *   - Every call is asynchronous on `stream` (NULL = the null stream) and never
 *     synchronizes, except the set-up calls dsgm_plan_batched and
 *     dsgm_autotune, which say so.  Arguments are validated on the host before any HIP call; a
 *     kernel fault surfaces as a HIP error of a later call or synchronization.
 *   - Every call returns a dsgm_status; nothing is thrown across the ABI.  On
 *     failure dsgm_last_error() (per thread) describes it.
 *   - Calls are reentrant; concurrent calls on different streams that touch
 *     disjoint memory are independent.
 *   - NaN or infinite intensities are not supported: results are whatever the
 *     IEEE comparisons make of them (memory safety is unaffected);
 *     dsgm_count_nonfinite checks a sequence for them.
 */
#ifndef DSGM_H
#define DSGM_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DSGM_OK = 0,
  DSGM_E_ARG = -1,         /* null pointer, bad enum or bad parameter value   */
  DSGM_E_SHAPE = -2,       /* negative size, stride too small, too large      */
  DSGM_E_DTYPE = -3,       /* unsupported storage/accumulation combination    */
  DSGM_E_ALIGN = -4,       /* pointer not aligned to its element size         */
  DSGM_E_WORKSPACE = -5,   /* workspace/checkpoint buffer too small           */
  DSGM_E_HIP = -6,         /* the HIP runtime reported an error               */
  DSGM_E_UNSUPPORTED = -7  /* valid but not implemented                       */
} dsgm_status;

/* storage type of the frames (U8: 8-bit frames, 0..255, for the as-run model) */
/* The _RANGE_ members of this and the next enum are not valid arguments: they
 * make every int32 value a value of the type, so that any integer a caller
 * passes can be read and rejected (DSGM_E_DTYPE) without undefined behaviour. */
typedef enum { DSGM_IN_F64 = 0, DSGM_IN_F32 = 1, DSGM_IN_BF16 = 2, DSGM_IN_U8 = 3,
               DSGM_IN_RANGE_MIN_ = -2147483647 - 1, DSGM_IN_RANGE_MAX_ = 2147483647 } dsgm_in_dtype;

/* type of the model state and of every arithmetic operation, and of the bulk
 * output arrays (bg and every gradient array):
 *   F64       state, arithmetic and arrays in FP64 (F64/F32/BF16 frames)
 *   F32       state, arithmetic and arrays in FP32 (F32/BF16 frames)
 *   F64_IO32  state and arithmetic in FP64, bg and gradient arrays in FP32
 *             (F32/BF16 frames): decisions and state are those of the FP64
 *             path, the arrays are its values rounded once to FP32, at the
 *             memory cost of FP32 (the state is per pixel, not per frame)
 *   U8        the appendix's as-run model (U8 frames only): means and
 *             variances kept as uint8 planes, FP64 arithmetic, every stored
 *             value converted to an integer with its fraction dropped and
 *             limited to [0, 255] (var_init too); the tests, the swap and the
 *             mask see the stored values.  dsgm_forward (masks, codes),
 *             dsgm_forward_filtered (the appendix's 8-bit preprocessing first)
 *             and dsgm_state_init_from_frame only; other calls return
 *             DSGM_E_DTYPE
 *   F32X2     compensated single precision (F32/BF16 frames): each state value
 *             is an unevaluated sum hi + lo of two floats (|lo| <= ulp(hi)/2),
 *             stored as interleaved (hi, lo) pairs, 8 bytes per value; every
 *             operation is formed from error-free FP32 transformations (about
 *             48 significant bits), so state and decisions follow the FP64
 *             evaluation to about 1e-13, at FP32 instruction rates; bg and
 *             gradient arrays are FP32 (hi + lo rounded once).
 *             dsgm_forward, dsgm_backward(_noalloc), dsgm_state_init_from_frame
 *             and the tuner; other calls return DSGM_E_DTYPE */
typedef enum { DSGM_ACC_F64 = 0, DSGM_ACC_F32 = 1, DSGM_ACC_F64_IO32 = 2, DSGM_ACC_U8 = 3,
               DSGM_ACC_F32X2 = 4,
               DSGM_ACC_RANGE_MIN_ = -2147483647 - 1, DSGM_ACC_RANGE_MAX_ = 2147483647 } dsgm_acc;

/* learning weight of a model of age a: Sec. 2.2 gives 1/(a+1); the appendix
 * computes 1/a.  The complementary weight is 1 - w in the accumulation type. */
typedef enum { DSGM_WEIGHT_EQ = 0, DSGM_WEIGHT_APPENDIX = 1 } dsgm_weight_rule;

/* background rule (appendix): (mean_A - x)^2 <= theta_d * max(mask_floor, ref)
 * with ref = var_A (VARIANCE) or ref = x as printed (PRINTED). */
typedef enum { DSGM_MASK_VARIANCE = 0, DSGM_MASK_PRINTED = 1 } dsgm_mask_rule;

/* decision-code bits written per pixel and frame by dsgm_forward(codes != NULL) */
enum { DSGM_CODE_HIT_A = 1, DSGM_CODE_HIT_C = 2, DSGM_CODE_RESET = 4, DSGM_CODE_SWAP = 8,
       DSGM_CODE_FG = 16 };

typedef struct {
  double theta_s;     /* match: (x - mean)^2 < theta_s * max(var, var_floor), >= 0 */
  double theta_d;     /* background threshold, >= 0                               */
  double var_init;    /* variance of a reset candidate (255 on 8-bit data), >= 0  */
  double var_floor;   /* appendix floor inside the match tests (0.1 on 8-bit)     */
  double mask_floor;  /* appendix floor inside the background rule (0.25)         */
  int32_t age_max;    /* age cap, 1..255 (30 in Sec. 2.2)                         */
  int32_t weight_rule;/* dsgm_weight_rule                                         */
  int32_t mask_rule;  /* dsgm_mask_rule                                           */
} dsgm_params;

typedef struct {
  int64_t T, H, W;      /* frames, rows, columns (each >= 0)                       */
  int64_t row_stride;   /* elements between rows, >= W                             */
  int64_t frame_stride; /* elements between frames, >= (H-1)*row_stride + W        */
} dsgm_shape;

/* model state: four H x W planes of the accumulation type and two H x W uint8
 * age planes; ages must lie in [1, age_max] */
typedef struct {
  void* mean_a;
  void* var_a;
  void* mean_c;
  void* var_c;
  uint8_t* age_a;
  uint8_t* age_c;
} dsgm_state;

/* gradients of the four float state planes (H x W each, array type) */
typedef struct {
  void* mean_a;
  void* var_a;
  void* mean_c;
  void* var_c;
} dsgm_grad_state;

/*
 * The paper's constants on an intensity scale of width `intensity_range`
 * (255 for 8-bit data, 2 for data in [-1, 1)): var_init = 255 s^2 (Sec. 2.3),
 * age_max = 30 (Sec. 2.2), var_floor = 0.1 s^2 and mask_floor = 0.25 s^2 for
 * the VARIANCE rule or 0.25 s for the PRINTED rule (appendix), s = range/255.
 * theta_s = 2 and theta_d = 4 (not printed in the paper).  `p` is a host
 * pointer.  Returns DSGM_E_ARG for a NULL p, a non-positive range or a bad rule.
 */
int dsgm_params_default(dsgm_params* p /* host */, double intensity_range, int32_t mask_rule);

/*
 * Initial model from one frame (the paper states none): mean_a = mean_c = x,
 * var_a = var_c = var_init, age_a = age_c = 1.  `frame0` is an H x W frame
 * addressed with shape.row_stride (shape.T and frame_stride are ignored).
 */
int dsgm_state_init_from_frame(const void* frame0, dsgm_in_dtype in_dtype, dsgm_shape shape,
                               dsgm_acc acc, const dsgm_params* params /* host */,
                               dsgm_state* state /* host struct of device pointers */,
                               hipStream_t stream);

/*
 * Run T frames of the DSGM update (Sec. 2.2-2.3, appendix) over every pixel,
 * updating `state` in place.  T == 1 is the per-frame streaming step; T > 1
 * fuses the frames, keeping each pixel's model in registers, with results
 * bit-identical to T calls with T == 1.
 *   masks      T x H x W uint8, 0 = background, 255 = foreground (required)
 *   bg         T x H x W of the array type: mean_A after each frame
 *              (optional, NULL to skip)
 *   ckpt       checkpoint buffer of ckpt_bytes >= dsgm_ckpt_bytes(shape, acc,
 *              ckpt_every) bytes (else DSGM_E_WORKSPACE): the state before
 *              frames 0, K, 2K, ... (K = ckpt_every), used by dsgm_backward
 *              (optional, NULL to skip)
 *   codes      T x H x W uint8 decision codes (DSGM_CODE_* bits; optional)
 * With ACC_F64 the arithmetic is IEEE binary64, rounded after every operation
 * (no fused multiply-add), and the results are bit-identical to a scalar FP64
 * evaluation of the same steps.
 */
int dsgm_forward(const void* frames, dsgm_in_dtype in_dtype, dsgm_shape shape, dsgm_acc acc,
                 const dsgm_params* params /* host */, dsgm_state* state /* host struct */,
                 uint8_t* masks, void* bg, void* ckpt, size_t ckpt_bytes, int32_t ckpt_every,
                 uint8_t* codes, hipStream_t stream);

/* bytes of the checkpoint buffer for dsgm_forward/dsgm_backward (0 on bad args) */
size_t dsgm_ckpt_bytes(dsgm_shape shape, dsgm_acc acc, int32_t ckpt_every);

/* bytes of the workspace dsgm_backward needs: H*W doubles (per-pixel
 * contributions to d/d(var_init), padded to 256 B) plus 4 KiB of partial sums
 * (0 on bad arguments) */
size_t dsgm_workspace_bytes(dsgm_shape shape, dsgm_acc acc);

/*
 * Reverse-mode derivative of the differentiable outputs -- bg after every frame
 * and the final mean_a, var_a, mean_c, var_c -- with respect to the frames,
 * the initial four float planes and var_init, with every decision (match,
 * reset, swap) held at the value the forward pass took.  The paper has no
 * derivative; this is the chain rule through the Sec. 2.2 update and the
 * Sec. 2.3 reset and swap (the foreground mask has no derivative).  Segments of
 * ckpt_every frames are recomputed from `ckpt`, which dsgm_forward wrote with
 * the same frames, params, shape and ckpt_every, and swept backwards.
 *   frames         as given to dsgm_forward
 *   ckpt           ckpt_bytes >= dsgm_ckpt_bytes(shape, acc, ckpt_every) bytes
 *                  (device; smaller returns DSGM_E_WORKSPACE)
 *   grad_bg        T x H x W, array type, strided like the frames (NULL = zero)
 *   grad_state_T   upstream gradient of the final planes, array type (host
 *                  struct or NULL = zero)
 *   grad_frames    T x H x W, array type, strided like the frames (out)
 *   grad_state0    gradient of the initial planes, array type (host struct of
 *                  device planes, out)
 *   grad_var_init  one double on the device (out): the H*W per-pixel terms are
 *                  accumulated in FP64 and added in a fixed order with
 *                  compensated (error-free two-sum) arithmetic, so it is
 *                  reproducible and independent of the launch shape
 *   workspace      dsgm_workspace_bytes(shape, acc) bytes of device memory;
 *                  smaller returns DSGM_E_WORKSPACE
 * With ACC_F64, grad_frames and grad_state0 are bit-identical to a scalar FP64
 * evaluation of the same chain rule in the same order.
 */
int dsgm_backward(const void* frames, dsgm_in_dtype in_dtype, dsgm_shape shape, dsgm_acc acc,
                  const dsgm_params* params /* host */, const void* ckpt, size_t ckpt_bytes,
                  int32_t ckpt_every, const void* grad_bg,
                  const dsgm_grad_state* grad_state_T /* host, or NULL */,
                  void* grad_frames, dsgm_grad_state* grad_state0 /* host */,
                  double* grad_var_init, void* workspace, size_t workspace_bytes,
                  hipStream_t stream);

/*
 * dsgm_backward for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops, harnesses that forbid hipMalloc): the same
 * arguments without the workspace, the same kernels and bit-identical results.
 * The per-pixel terms and partial sums live in a buffer of the library's own,
 * 8 * (DSGM_NOALLOC_MAX_PIXELS + 512) bytes (64 MiB + 4 KiB) on each device
 * the function runs on, held until the process ends; its device address is
 * looked up on the first call on a device (with that device current).
 *   H * W > DSGM_NOALLOC_MAX_PIXELS returns DSGM_E_WORKSPACE (before any HIP
 *   call); every other argument and error is as for dsgm_backward.
 * Nothing is allocated by the call.  Every call on one device shares that
 * device's buffer: calls that may overlap on one device (different streams,
 * or host threads without ordering) race and must be serialised by the
 * caller; calls ordered on one stream are safe.
 */
#define DSGM_NOALLOC_MAX_PIXELS (1LL << 23) /* 8,388,608 pixels: 2160 x 3840 fits */
int dsgm_backward_noalloc(const void* frames, dsgm_in_dtype in_dtype, dsgm_shape shape,
                          dsgm_acc acc, const dsgm_params* params /* host */, const void* ckpt,
                          size_t ckpt_bytes, int32_t ckpt_every, const void* grad_bg,
                          const dsgm_grad_state* grad_state_T /* host, or NULL */,
                          void* grad_frames, dsgm_grad_state* grad_state0 /* host */,
                          double* grad_var_init, hipStream_t stream);

/*
 * Frame preprocessing (Sec. 2.1; serial and GPU versions in Sec. 3.1.1 and
 * 3.3.1): a separable blur -- the n-tap kernel applied along rows, then along
 * columns of the row-blurred frame, each sum taken from 0 in tap order -- then
 * the median of every 3 x 3 neighbourhood of the blurred frame.  Indices
 * outside the frame are clamped to the nearest valid row or column (the
 * appendix clamps one past the last index; the last index is used).
 */
typedef struct {
  int32_t n;           /* blur taps: 0 (no blur) or odd, 1..7 (n = 1: weight 1)   */
  int32_t median;      /* 1: 3 x 3 median after the blur; 0: none                  */
  double weights[7];   /* the n taps (host values), weights[(n-1)/2] the centre    */
} dsgm_filter;

/*
 * The Sec. 2.1 Gaussian density sampled at the integer offsets d = i - (n-1)/2,
 * e_i = exp(-(d*d) / (2*sigma*sigma)), normalised by their sum (taken in index
 * order): w_i = e_i / sum.  n odd in 1..7, sigma > 0; writes n doubles to
 * `weights` (host).  Returns DSGM_E_ARG on bad arguments.
 */
int dsgm_gauss_weights(int32_t n, double sigma, double* weights /* host, n */);

/*
 * dsgm_forward on the preprocessed frames, in one pass: the frames are read
 * once per halo tile, filtered in LDS and fed to the update; the filtered
 * frames are written only if `filtered` is not NULL (T x H x W, array type,
 * strided like the frames).  masks, bg and codes as for dsgm_forward; no
 * checkpoints (the adjoint does not run through the filters).  `filter` is a
 * host struct; n > 7 returns DSGM_E_UNSUPPORTED.  With ACC_F64 the results are
 * bit-identical to a scalar FP64 evaluation of the blur sums, the median and
 * the update in the stated order.
 *
 * U8 frames with U8 state run the pipeline as the appendix runs it on 8-bit
 * images (its blur, median and update snippets): the blur is two-dimensional,
 * a single-precision sum over the window's rows (outer) and columns (inner) of
 * each byte times the weight float(weights[i] * weights[j]) (product in
 * double, rounded once), every product and sum rounded, written back to 8
 * bits by dropping the fraction (limited to 255); the median takes the nine
 * blurred bytes of each clamped 3 x 3 neighbourhood; the update is the 8-bit
 * as-run model of dsgm_forward.  `filtered` (optional) receives the median's
 * bytes; bg must be NULL (DSGM_E_UNSUPPORTED).  Bit-identical to a scalar
 * evaluation in that order.
 */
int dsgm_forward_filtered(const void* frames, dsgm_in_dtype in_dtype, dsgm_shape shape,
                          dsgm_acc acc, const dsgm_params* params /* host */,
                          const dsgm_filter* filter /* host */, dsgm_state* state /* host struct */,
                          uint8_t* masks, void* bg, void* filtered, uint8_t* codes,
                          hipStream_t stream);

/*
 * One frame of the update on the motion-compensated model (Sec. 2.2 uses the
 * previous values "after motion compensation"; Sec. 2.4 maps the per-pixel
 * model through the camera's homography).  The homography is an input (its
 * estimation, KLT tracking and RANSAC in the paper, is the caller's):
 *   inv_map   host, 9 doubles, row-major: takes a pixel (column c, row y, 1)
 *             of the current frame to the previous frame,
 *             den = (m6*c + m7*y) + m8, qx = ((m0*c + m1*y) + m2) / den,
 *             qy = ((m3*c + m4*y) + m5) / den
 * A pixel with den > 0 and (qx, qy) inside [0, W-1] x [0, H-1] takes from
 * `src` the bilinear blend of the four surrounding means and variances
 * (weights (1-fx)(1-fy), fx(1-fy), (1-fx)fy, fx*fy, fx = qx - floor(qx), in
 * that order; an index past the last row or column is clamped, its weight is
 * 0) and the nearest pixel's ages (floor(q + 0.5)); any other pixel restarts
 * from the frame, (x, var_init, 1) for both models.  The update then runs on
 * that model and writes the mask (and bg, codes) of the frame and the new
 * model to `dst`.  shape.T must be 1 (one call per frame); frame, masks, bg
 * and codes are H x W with shape.row_stride; the state planes are dense
 * H x W; no plane of `dst` may overlap a plane of `src` (DSGM_E_ARG).  With
 * ACC_F64 the results are bit-identical to a scalar FP64 evaluation in the
 * stated order.
 */
int dsgm_forward_warped(const void* frame, dsgm_in_dtype in_dtype, dsgm_shape shape,
                        dsgm_acc acc, const dsgm_params* params /* host */,
                        const double* inv_map /* host, 9 */, const dsgm_state* src /* host struct */,
                        dsgm_state* dst /* host struct */, uint8_t* masks, void* bg,
                        uint8_t* codes, hipStream_t stream);

/*
 * Yi et al.'s grid model, which Sec. 2.2 describes and the paper reduces to
 * one pixel: one dual model per block of b x b pixels (b = 1, 2 or 4; edge
 * blocks keep the pixels that exist).  Per frame and block the tests, the
 * blend and the reset use the block mean M = (row-major sum from 0) / |G|,
 * and the matched model's variance term is the largest squared distance of
 * the updated mean from the block's intensities; each pixel's mask bit uses
 * the block's apparent model.  b = 1 is exactly dsgm_forward.
 *   state    Hb x Wb planes (Hb = ceil(H/b), Wb = ceil(W/b)), updated in place
 *   masks    T x H x W, strided like the frames
 *   bg       NULL or T x Hb x Wb dense, array type: the block's mean_A after
 *            each frame
 *   codes    NULL or T x Hb x Wb dense (CODE_* bits without CODE_FG)
 * b outside {1, 2, 4} returns DSGM_E_UNSUPPORTED.
 */
int dsgm_forward_grid(const void* frames, dsgm_in_dtype in_dtype, dsgm_shape shape, dsgm_acc acc,
                      const dsgm_params* params /* host */, int32_t b,
                      dsgm_state* state /* host struct */, uint8_t* masks, void* bg,
                      uint8_t* codes, hipStream_t stream);

/* one instance of a batch: its own sizes, strides, frames, state and outputs */
typedef struct {
  dsgm_shape shape;
  const void* frames;
  dsgm_state state;
  uint8_t* masks;
  void* bg;             /* NULL: no bg output */
  uint32_t* fg_counts;  /* NULL, or T counters (device, 4-byte aligned): after the
                           launch, entry t holds the number of foreground pixels of
                           frame t (mask 255), an exact integer sum; each launch
                           clears them first */
} dsgm_instance;

/* host-side handle of a planned batch (plain data, owned by the caller) */
typedef struct {
  void* device_plan;      /* the caller's plan buffer (device)                 */
  int64_t n_items;        /* work items: (instance, up to 64 pixel groups)     */
  int64_t total_elements; /* sum over instances of T*H*W                      */
  int32_t n_instances;
  int32_t in_dtype, acc;
  int32_t vector;         /* pixels per lane, common to all instances         */
  int32_t grid;           /* persistent workgroups: the planner sets the count
                             that fills the device; the caller may lower it to
                             any value >= 1 (results do not depend on it)     */
  int32_t has_bg;
  int32_t has_counts;     /* some instance has foreground counters            */
} dsgm_batch_plan;

/* bytes of the device plan buffer for these instances (0 on bad arguments) */
size_t dsgm_batch_plan_bytes(const dsgm_instance* instances /* host */, int32_t n,
                             dsgm_in_dtype in_dtype, dsgm_acc acc);

/*
 * Plan many independent instances (different sizes, frame counts, strides) for
 * one persistent launch.  Each instance is cut into work items of up to 64
 * pixel groups (one wavefront's work over all of the instance's frames); the
 * items are ordered longest-first (frames x groups, LPT) and written, with the
 * instance descriptors, to `plan_buffer` (device, 256-byte aligned,
 * dsgm_batch_plan_bytes bytes, owned by the caller, which keeps it and every
 * instance buffer alive while the plan is used).  The pixels-per-lane width is
 * the widest every instance allows.  This call copies the plan to the device
 * and synchronizes `stream`; it is not meant for the hot loop.
 */
int dsgm_plan_batched(const dsgm_instance* instances /* host */, int32_t n, dsgm_in_dtype in_dtype,
                      dsgm_acc acc, void* plan_buffer, size_t plan_bytes,
                      dsgm_batch_plan* plan /* host, out */, hipStream_t stream);

/*
 * Run every instance of a plan through all of its frames (the per-instance
 * results are those of dsgm_forward on that instance alone): one small kernel
 * resets the plan's work counter, a second clears the foreground counters
 * when some instance has them (plan.has_counts), then one persistent kernel
 * whose wavefronts take items from it until none are left; each wavefront adds
 * its foreground pixels of each frame to the instance's counter with one
 * integer atomic, so the counts are exact and do not depend on the schedule.
 * Enqueues exactly these kernels and nothing else (no allocation, no copy, no
 * memset, no synchronization), so the call can be captured into a HIP graph
 * and replayed.  Launches of one plan must not overlap (they share the
 * counters).
 */
int dsgm_forward_batched(const dsgm_batch_plan* plan /* host */, const dsgm_params* params /* host */,
                         hipStream_t stream);

/* human-readable name of a status code (static string) */
const char* dsgm_status_string(int status);

/* description of the last failure of a call on this thread ("" if none) */
const char* dsgm_last_error(void);

/* ABI version: major*10000 + minor*100 + patch */
int dsgm_version(void);

/*
 * Count the NaN and infinite intensities of T x H x W frames (addressed with
 * the shape's strides, like every frames argument) into *count (device, one
 * uint64, overwritten).  The update is defined for finite intensities; with
 * others its branches are whatever the IEEE comparisons decide, so this is the
 * check a caller can run on its input first.  Enqueues two kernels (one
 * clears the counter) and nothing else, so it can be captured into a graph;
 * the count is exact.  U8 frames always count 0.
 */
int dsgm_count_nonfinite(const void* frames, dsgm_in_dtype in_dtype, dsgm_shape shape,
                         uint64_t* count, hipStream_t stream);

/* Flags of the launch-shape tuner: the optional outputs of the calls to tune */
typedef enum {
  DSGM_TUNE_BG = 1,      /* bg written */
  DSGM_TUNE_CKPT = 2,    /* checkpoints written */
  DSGM_TUNE_PRINTED = 4  /* params.mask_rule = DSGM_MASK_PRINTED */
} dsgm_tune_flags;

/* bytes of the workspace dsgm_autotune needs for these arguments (0 on bad
 * arguments or an empty problem) */
size_t dsgm_autotune_bytes(dsgm_in_dtype in_dtype, dsgm_acc acc, dsgm_shape shape,
                           int32_t flags);

/*
 * Launch-shape tuner of dsgm_forward (a set-up call, not for the hot loop).
 * Sec. 3.4 measures how the threads per block change the GPU time; this call
 * makes that measurement for the caller's problem: it times dsgm_forward on
 * min(T, 64) frames of H x W independent uniform intensities (dense layout,
 * default parameters for the frame type's range, the outputs that `flags`
 * names) for every workgroup size 64, 128, 192, 256 and every pixels-per-lane width
 * 1, 2, 4 that W allows, each from the same initial state, and keeps the
 * fastest in a process-wide table under the key (in_dtype, acc, H, W, flags).
 * Later dsgm_forward calls whose arguments have that key launch with the
 * chosen shape (a width their strides or alignments do not allow is replaced
 * as usual); dsgm_set_launch overrides the table.  Results never depend on the
 * launch shape.
 *   workspace  device, 256-byte aligned, dsgm_autotune_bytes bytes, owned by
 *              the caller (free to reuse once the call returns)
 *   chosen     NULL or (host) 2 int32: the chosen block size and width
 *              ({0, 0} for an empty problem, which tunes nothing)
 * Runs its kernels on `stream` and synchronizes it.  The 8-bit as-run pair
 * accepts DSGM_TUNE_PRINTED only (DSGM_E_UNSUPPORTED otherwise).
 */
int dsgm_autotune(dsgm_in_dtype in_dtype, dsgm_acc acc, dsgm_shape shape, int32_t flags,
                  void* workspace, size_t ws_bytes, int32_t* chosen /* host */, hipStream_t stream);

/* the tuner's table entry for these arguments: chosen (host, 2 int32) =
 * {block, width}, or {0, 0} if they were not tuned; no HIP call */
int dsgm_autotune_lookup(dsgm_in_dtype in_dtype, dsgm_acc acc, dsgm_shape shape, int32_t flags,
                         int32_t* chosen /* host */);

/* empty the tuner's table (later calls use the default launch shapes) */
int dsgm_autotune_clear(void);

/*
 * Launch-shape override for tuning and tests (process-wide): `block` threads
 * per workgroup (0 = default, else a multiple of 64 in 64..256) and `vector`
 * pixels per lane (0 = the widest that sizes, strides and alignments allow,
 * else 1, 2 or 4; a value the arguments do not allow is ignored).  Results do
 * not depend on either.  Returns DSGM_E_ARG for other values.
 */
int dsgm_set_launch(int32_t block, int32_t vector);

#ifdef __cplusplus
}
#endif

#endif /* DSGM_H */
