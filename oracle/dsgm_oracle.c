/*
 * dsgm_oracle.c -- plain, slow FP64 reference of the Dual-Mode Single Gaussian
 * Model (DSGM) background update and foreground mask.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code, no
 * header and no table with the GPU library, and the product path never calls it.
 *
 * Sources (Henderson & Vertescher, "An Analysis of Parallelized Motion Masking
 * Using Dual-Mode Single Gaussian Models", arXiv:1702.05156):
 *   - Sec. 2.2 (Single Gaussian Model): the mean, variance and age equations.
 *     The mean is an age-weighted blend of the previous mean and the pixel
 *     intensity; the variance blends the previous variance with the squared
 *     distance of the *updated* mean from the intensity; the age grows by one and
 *     is capped at 30.  The grid has one pixel, so the block mean M is the pixel
 *     intensity and the block-max squared deviation is that pixel's own.
 *   - Sec. 2.3 (Dual-mode SGM): the apparent model is tested first, the candidate
 *     only if the apparent one did not match; if neither matches the candidate is
 *     reset to (intensity, initial variance, age 1); when the candidate's age
 *     exceeds the apparent one's, the candidate becomes the apparent model and the
 *     candidate is reset.
 *   - Appendix "Dual-mode SGM Inner Update Code Snippet": the variance floor
 *     inside the match tests, the age cap as "increment while below the cap",
 *     the strict comparisons of the tests and the swap, and the background rule
 *     "squared distance of the apparent mean <= theta_d times a floored reference".
 *
 * Readings of points the paper leaves open (each one is a parameter here):
 *   - weight rule: the equations' 1/(a+1) (WEIGHT_EQ, default) or the appendix's
 *     1/a (WEIGHT_APPENDIX); in both cases the complementary weight is 1 - w,
 *     rounded in FP64, as the appendix computes it.
 *   - the match tests use the model before this frame's update (the appendix
 *     computes the differences first; the superscript (t) in the text is a slip).
 *   - mask reference: the apparent variance (MASK_VARIANCE, default) or the
 *     intensity as printed in the appendix (MASK_PRINTED).
 *   - ages are capped as min(a + 1, age_max); ages stay in [1, age_max].
 *   - every product and sum is rounded separately (no fused multiply-add):
 *     build with -ffp-contract=off.
 *
 * All arrays are dense: frames and per-frame outputs are T x N (frame-major),
 * per-pixel state arrays have N entries.  Return value 0 on success, -1 on a
 * bad argument.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
  double theta_s;    /* match threshold on squared distance / variance   */
  double theta_d;    /* background threshold                             */
  double var_init;   /* variance of a freshly reset candidate model      */
  double var_floor;  /* floor on the variance inside the match tests     */
  double mask_floor; /* floor on the reference inside the background rule*/
  int32_t age_max;   /* age cap                                          */
  int32_t weight_rule;
  int32_t mask_rule;
} orc_params;

enum { ORC_WEIGHT_EQ = 0, ORC_WEIGHT_APPENDIX = 1 };
enum { ORC_MASK_VARIANCE = 0, ORC_MASK_PRINTED = 1 };

/* decision-code bits, one byte per pixel and frame */
enum { ORC_HIT_A = 1, ORC_HIT_C = 2, ORC_RESET = 4, ORC_SWAP = 8, ORC_FG = 16 };

typedef struct {
  double mean, var;
  int32_t age;
} orc_model;

/* what one frame's update of one pixel leaves for the reverse sweep */
typedef struct {
  uint8_t code;
  double u, w; /* weights of the matched model (0 if none matched) */
  double d;    /* updated mean minus intensity (0 if none matched)  */
} orc_tape;

static double orc_max(double a, double b) { return a < b ? b : a; }

static double orc_sq(double a) { return a * a; }

/* Learning weight of a model of age a (Sec. 2.2 equations, or the appendix). */
static double orc_weight(int32_t a, const orc_params* p) {
  if (p->weight_rule == ORC_WEIGHT_APPENDIX) return 1.0 / (double)a;
  return 1.0 / ((double)a + 1.0);
}

/* Sec. 2.2: update one model with intensity x; returns the tape entries. */
static void orc_sgm_update(orc_model* m, double x, const orc_params* p, orc_tape* tp) {
  double w = orc_weight(m->age, p);
  double u = 1.0 - w;
  double mean = u * m->mean + w * x; /* mean equation                    */
  double d = mean - x;               /* uses the updated mean            */
  double V = d * d;                  /* per-pixel V: squared deviation   */
  double var = u * m->var + w * V;   /* variance equation                */
  m->mean = mean;
  m->var = var;
  m->age = m->age < p->age_max ? m->age + 1 : p->age_max; /* age, capped */
  tp->u = u;
  tp->w = w;
  tp->d = d;
}

static void orc_reset(orc_model* m, double x, const orc_params* p) {
  m->mean = x;
  m->var = p->var_init;
  m->age = 1;
}

/*
 * One frame of one pixel (Sec. 2.3 and the appendix).  If `forced` is
 * non-negative its HIT_A/HIT_C/SWAP bits replace the model's own decisions (the
 * foreground bit is always recomputed).  Writes the three signed decision
 * margins (lhs - rhs of the A test, the C test and the background test) when
 * `margins` is not NULL.  Returns the decision code.
 */
/* The appendix keeps means and variances in 8-bit images: every value written
 * to one is converted to an integer (the fraction dropped), and here limited
 * to [0, 255] (a conversion outside that range has no defined result). */
static double orc_u8(double v) {
  if (!(v > 0.0)) return 0.0;
  if (v >= 255.0) return 255.0;
  return trunc(v);
}

static void orc_quantize(orc_model* m) {
  m->mean = orc_u8(m->mean);
  m->var = orc_u8(m->var);
}

static uint8_t orc_step_q(orc_model* A, orc_model* C, double x, const orc_params* p, int forced,
                          orc_tape* tp, double* margins, int quant);

static uint8_t orc_step(orc_model* A, orc_model* C, double x, const orc_params* p, int forced,
                        orc_tape* tp, double* margins) {
  return orc_step_q(A, C, x, p, forced, tp, margins, 0);
}

/* `quant`: the 8-bit as-run model of the appendix -- the matched model (or the
 * reset candidate) is stored through orc_u8 before the swap test and the
 * mask, which therefore see the stored values. */
static uint8_t orc_step_q(orc_model* A, orc_model* C, double x, const orc_params* p, int forced,
                          orc_tape* tp, double* margins, int quant) {
  uint8_t code = 0;
  double qa = orc_sq(x - A->mean);
  double ta = p->theta_s * orc_max(A->var, p->var_floor);
  double qc = orc_sq(x - C->mean);
  double tc = p->theta_s * orc_max(C->var, p->var_floor);
  int hit_a, hit_c, swap;

  if (forced >= 0) {
    hit_a = (forced & ORC_HIT_A) != 0;
    hit_c = !hit_a && (forced & ORC_HIT_C) != 0;
  } else {
    hit_a = qa < ta;              /* apparent model first             */
    hit_c = !hit_a && (qc < tc);  /* candidate only if A did not match */
  }
  tp->u = tp->w = tp->d = 0.0;
  if (hit_a) {
    code |= ORC_HIT_A;
    orc_sgm_update(A, x, p, tp);
  } else if (hit_c) {
    code |= ORC_HIT_C;
    orc_sgm_update(C, x, p, tp);
  } else {
    code |= ORC_RESET;
    orc_reset(C, x, p);
  }
  if (quant) {
    orc_quantize(A);
    orc_quantize(C);
  }

  swap = (forced >= 0) ? ((forced & ORC_SWAP) != 0) : (C->age > A->age);
  if (swap) {
    code |= ORC_SWAP;
    *A = *C;
    orc_reset(C, x, p);
    if (quant) orc_quantize(C);
  }

  {
    double qd = orc_sq(A->mean - x);
    double ref = p->mask_rule == ORC_MASK_PRINTED ? x : A->var;
    double td = p->theta_d * orc_max(p->mask_floor, ref);
    if (!(qd <= td)) code |= ORC_FG;
    if (margins) {
      margins[0] = qa - ta;
      margins[1] = qc - tc;
      margins[2] = qd - td;
    }
  }
  tp->code = code;
  return code;
}

static int orc_check(const orc_params* p) {
  if (!p) return -1;
  if (p->age_max < 1) return -1;
  if (p->weight_rule != ORC_WEIGHT_EQ && p->weight_rule != ORC_WEIGHT_APPENDIX) return -1;
  if (p->mask_rule != ORC_MASK_VARIANCE && p->mask_rule != ORC_MASK_PRINTED) return -1;
  return 0;
}

static void orc_set_threads(int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
}

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

#define ORC_CHUNK 1024

/*
 * Forward pass over T frames of N pixels, frame by frame as in the paper's
 * serial loop.  State arrays are updated in place.  masks (0 = background,
 * 255 = foreground), bg (the apparent mean after each frame), codes, and
 * margins (T x N x 3) are optional outputs; forced (T x N) optionally supplies
 * the decisions.  Pixels are split into chunks across OpenMP threads; every
 * pixel is computed by the same scalar code whatever the thread count.
 */
int orc_forward(int64_t T, int64_t N, const double* frames, double* mean_a, double* var_a,
                int32_t* age_a, double* mean_c, double* var_c, int32_t* age_c,
                const orc_params* p, uint8_t* masks, double* bg, uint8_t* codes,
                const uint8_t* forced, double* margins, int nthreads) {
  int64_t nchunk, c;
  if (orc_check(p) || T < 0 || N < 0) return -1;
  if (T > 0 && N > 0 && (!frames || !mean_a || !var_a || !age_a || !mean_c || !var_c || !age_c))
    return -1;
  orc_set_threads(nthreads);
  nchunk = (N + ORC_CHUNK - 1) / ORC_CHUNK;
#pragma omp parallel for schedule(static)
  for (c = 0; c < nchunk; ++c) {
    int64_t p0 = c * ORC_CHUNK, p1 = p0 + ORC_CHUNK < N ? p0 + ORC_CHUNK : N;
    int64_t t, i;
    for (t = 0; t < T; ++t) {
      for (i = p0; i < p1; ++i) {
        int64_t e = t * N + i;
        orc_model A = {mean_a[i], var_a[i], age_a[i]};
        orc_model C = {mean_c[i], var_c[i], age_c[i]};
        orc_tape tp;
        uint8_t code = orc_step(&A, &C, frames[e], p, forced ? (int)forced[e] : -1, &tp,
                                margins ? margins + 3 * e : NULL);
        mean_a[i] = A.mean; var_a[i] = A.var; age_a[i] = A.age;
        mean_c[i] = C.mean; var_c[i] = C.var; age_c[i] = C.age;
        if (masks) masks[e] = (code & ORC_FG) ? 255 : 0;
        if (bg) bg[e] = A.mean;
        if (codes) codes[e] = code;
      }
    }
  }
  return 0;
}

/*
 * Reverse-mode derivative of the differentiable outputs (bg after every frame
 * and the final mean_a, var_a, mean_c, var_c) with the decisions held fixed.
 * The paper has no derivative; this is the chain rule through the Sec. 2.2
 * update, the Sec. 2.3 reset and swap, one pixel at a time, on a full tape.
 *   grad_bg       T x N upstream gradient of bg (NULL = zero)
 *   grad_state_T  4 x N upstream gradient of the final (mean_a, var_a, mean_c, var_c) (NULL = zero)
 *   grad_frames   T x N output
 *   grad_state0   4 x N output, same plane order
 *   grad_var_init N outputs: each pixel's contribution (the caller sums them)
 */
int orc_backward(int64_t T, int64_t N, const double* frames, const double* mean_a0,
                 const double* var_a0, const int32_t* age_a0, const double* mean_c0,
                 const double* var_c0, const int32_t* age_c0, const orc_params* p,
                 const uint8_t* forced, const double* grad_bg, const double* grad_state_T,
                 double* grad_frames, double* grad_state0, double* grad_var_init, int nthreads) {
  int64_t i;
  if (orc_check(p) || T < 0 || N < 0) return -1;
  if (N > 0 && (!mean_a0 || !var_a0 || !age_a0 || !mean_c0 || !var_c0 || !age_c0 ||
                !grad_state0 || !grad_var_init))
    return -1;
  if (T > 0 && N > 0 && (!frames || !grad_frames)) return -1;
  orc_set_threads(nthreads);
#pragma omp parallel for schedule(static)
  for (i = 0; i < N; ++i) {
    orc_tape* tape = (orc_tape*)malloc(sizeof(orc_tape) * (size_t)(T > 0 ? T : 1));
    orc_model A = {mean_a0[i], var_a0[i], age_a0[i]};
    orc_model C = {mean_c0[i], var_c0[i], age_c0[i]};
    double gmA = 0, gvA = 0, gmC = 0, gvC = 0, gvi = 0;
    int64_t t;
    for (t = 0; t < T; ++t) {
      int64_t e = t * N + i;
      orc_step(&A, &C, frames[e], p, forced ? (int)forced[e] : -1, &tape[t], NULL);
    }
    if (grad_state_T) {
      gmA = grad_state_T[0 * N + i];
      gvA = grad_state_T[1 * N + i];
      gmC = grad_state_T[2 * N + i];
      gvC = grad_state_T[3 * N + i];
    }
    for (t = T - 1; t >= 0; --t) {
      int64_t e = t * N + i;
      const orc_tape* tp = &tape[t];
      double gx = 0.0;
      if (grad_bg) gmA += grad_bg[e]; /* bg[t] is the apparent mean after the swap */
      if (tp->code & ORC_SWAP) {
        /* after the swap: A holds the pre-swap C, C holds (x, var_init) */
        gx += gmC;
        gvi += gvC;
        gmC = gmA;
        gvC = gvA;
        gmA = 0.0;
        gvA = 0.0;
      }
      if (tp->code & (ORC_HIT_A | ORC_HIT_C)) {
        double* gm = (tp->code & ORC_HIT_A) ? &gmA : &gmC;
        double* gv = (tp->code & ORC_HIT_A) ? &gvA : &gvC;
        double gV = tp->w * *gv;          /* var' = u*var + w*V        */
        double gd = 2.0 * tp->d * gV;     /* V = d*d                   */
        double gmn = *gm + gd;            /* d = mean' - x             */
        gx += tp->w * gmn - gd;           /* mean' = u*mean + w*x      */
        *gv = tp->u * *gv;
        *gm = tp->u * gmn;
      } else {
        /* reset: C = (x, var_init) */
        gx += gmC;
        gvi += gvC;
        gmC = 0.0;
        gvC = 0.0;
      }
      grad_frames[e] = gx;
    }
    grad_state0[0 * N + i] = gmA;
    grad_state0[1 * N + i] = gvA;
    grad_state0[2 * N + i] = gmC;
    grad_state0[3 * N + i] = gvC;
    grad_var_init[i] = gvi;
    free(tape);
  }
  return 0;
}

/*
 * Forward-mode derivative (tangent) with the decisions held fixed: given
 * tangents of the frames (T x N), of the initial (mean_a, var_a, mean_c, var_c)
 * (4 x N) and of var_init, returns the tangents of bg (T x N, optional) and of
 * the final four float planes (4 x N).
 */
int orc_jvp(int64_t T, int64_t N, const double* frames, const double* mean_a0,
            const double* var_a0, const int32_t* age_a0, const double* mean_c0,
            const double* var_c0, const int32_t* age_c0, const orc_params* p,
            const uint8_t* forced, const double* dframes, const double* dstate0,
            double dvar_init, double* dbg, double* dstate_T, int nthreads) {
  int64_t i;
  if (orc_check(p) || T < 0 || N < 0) return -1;
  if (N > 0 && (!mean_a0 || !var_a0 || !age_a0 || !mean_c0 || !var_c0 || !age_c0 ||
                !dstate0 || !dstate_T))
    return -1;
  if (T > 0 && N > 0 && (!frames || !dframes)) return -1;
  orc_set_threads(nthreads);
#pragma omp parallel for schedule(static)
  for (i = 0; i < N; ++i) {
    orc_model A = {mean_a0[i], var_a0[i], age_a0[i]};
    orc_model C = {mean_c0[i], var_c0[i], age_c0[i]};
    double dmA = dstate0[0 * N + i], dvA = dstate0[1 * N + i];
    double dmC = dstate0[2 * N + i], dvC = dstate0[3 * N + i];
    int64_t t;
    for (t = 0; t < T; ++t) {
      int64_t e = t * N + i;
      double dx = dframes[e];
      orc_tape tp;
      orc_step(&A, &C, frames[e], p, forced ? (int)forced[e] : -1, &tp, NULL);
      if (tp.code & (ORC_HIT_A | ORC_HIT_C)) {
        double* dm = (tp.code & ORC_HIT_A) ? &dmA : &dmC;
        double* dv = (tp.code & ORC_HIT_A) ? &dvA : &dvC;
        double dmn = tp.u * *dm + tp.w * dx;
        double dd = dmn - dx;
        double dV = 2.0 * tp.d * dd;
        *dv = tp.u * *dv + tp.w * dV;
        *dm = dmn;
      } else {
        dmC = dx;
        dvC = dvar_init;
      }
      if (tp.code & ORC_SWAP) {
        dmA = dmC;
        dvA = dvC;
        dmC = dx;
        dvC = dvar_init;
      }
      if (dbg) dbg[e] = dmA;
    }
    dstate_T[0 * N + i] = dmA;
    dstate_T[1 * N + i] = dvA;
    dstate_T[2 * N + i] = dmC;
    dstate_T[3 * N + i] = dvC;
  }
  return 0;
}

/*
 * Motion compensation of the model (Sec. 2.2: the update uses the previous
 * mean, variance and age "after motion compensation"; Sec. 2.4: with a
 * per-pixel model the homography of the camera motion maps the model values to
 * the pixels they now belong to).  The homography itself (KLT features and
 * RANSAC in the paper) is an input: `map` (row-major 3 x 3) takes a pixel
 * (c, y) of the current frame to its position in the previous one,
 *   den = (map[6]*c + map[7]*y) + map[8],
 *   qx  = ((map[0]*c + map[1]*y) + map[2]) / den,  qy likewise with map[3..5].
 * Readings: a pixel is covered when den > 0 and (qx, qy) lies in
 * [0, W-1] x [0, H-1]; its means and variances are the bilinear blend of the
 * four surrounding pixels, weights (1-fx)(1-fy), fx(1-fy), (1-fx)fy, fx*fy with
 * fx = qx - floor(qx), fy likewise, summed in that order (a neighbour index
 * past the last row or column is clamped; its weight is then 0); its ages are
 * the nearest pixel's, floor(q + 0.5), clamped.  An uncovered pixel has no
 * history: both of its models start from the current intensity x, as in a
 * state initialised from a frame, (x, var_init, 1).  src and dst are distinct
 * H x W planes; `frame` is the current frame (H x W).
 */
int orc_warp_state(int64_t H, int64_t W, const double* map, const double* frame,
                   const double* mean_a, const double* var_a, const int32_t* age_a,
                   const double* mean_c, const double* var_c, const int32_t* age_c,
                   const orc_params* p, double* o_mean_a, double* o_var_a, int32_t* o_age_a,
                   double* o_mean_c, double* o_var_c, int32_t* o_age_c, int nthreads) {
  int64_t y;
  if (orc_check(p) || H < 0 || W < 0 || !map) return -1;
  if (H == 0 || W == 0) return 0;
  if (!frame || !mean_a || !var_a || !age_a || !mean_c || !var_c || !age_c || !o_mean_a ||
      !o_var_a || !o_age_a || !o_mean_c || !o_var_c || !o_age_c)
    return -1;
  orc_set_threads(nthreads);
#pragma omp parallel for schedule(static)
  for (y = 0; y < H; ++y) {
    int64_t c;
    for (c = 0; c < W; ++c) {
      const int64_t i = y * W + c;
      const double xd = (double)c, yd = (double)y;
      const double den = (map[6] * xd + map[7] * yd) + map[8];
      const double qx = ((map[0] * xd + map[1] * yd) + map[2]) / den;
      const double qy = ((map[3] * xd + map[4] * yd) + map[5]) / den;
      if (!(den > 0.0) || !(qx >= 0.0) || !(qx <= (double)(W - 1)) || !(qy >= 0.0) ||
          !(qy <= (double)(H - 1))) {
        o_mean_a[i] = frame[i];
        o_mean_c[i] = frame[i];
        o_var_a[i] = p->var_init;
        o_var_c[i] = p->var_init;
        o_age_a[i] = 1;
        o_age_c[i] = 1;
        continue;
      }
      {
        const double fx0 = floor(qx), fy0 = floor(qy);
        const double fx = qx - fx0, fy = qy - fy0;
        const int64_t x0 = (int64_t)fx0, y0 = (int64_t)fy0;
        const int64_t x1 = x0 + 1 < W ? x0 + 1 : W - 1, y1 = y0 + 1 < H ? y0 + 1 : H - 1;
        const double w00 = (1.0 - fx) * (1.0 - fy), w10 = fx * (1.0 - fy);
        const double w01 = (1.0 - fx) * fy, w11 = fx * fy;
        const int64_t i00 = y0 * W + x0, i10 = y0 * W + x1, i01 = y1 * W + x0, i11 = y1 * W + x1;
        int64_t xn = (int64_t)floor(qx + 0.5), yn = (int64_t)floor(qy + 0.5);
        if (xn > W - 1) xn = W - 1;
        if (yn > H - 1) yn = H - 1;
        o_mean_a[i] = ((w00 * mean_a[i00] + w10 * mean_a[i10]) + w01 * mean_a[i01]) + w11 * mean_a[i11];
        o_var_a[i] = ((w00 * var_a[i00] + w10 * var_a[i10]) + w01 * var_a[i01]) + w11 * var_a[i11];
        o_mean_c[i] = ((w00 * mean_c[i00] + w10 * mean_c[i10]) + w01 * mean_c[i01]) + w11 * mean_c[i11];
        o_var_c[i] = ((w00 * var_c[i00] + w10 * var_c[i10]) + w01 * var_c[i01]) + w11 * var_c[i11];
        o_age_a[i] = age_a[yn * W + xn];
        o_age_c[i] = age_c[yn * W + xn];
      }
    }
  }
  return 0;
}

/*
 * Yi et al.'s grid model, which the paper describes (Sec. 2.2) and reduces to
 * one pixel per grid: the frame is cut into blocks G of b x b pixels (blocks on
 * the right and bottom edges keep the pixels that exist), one dual model per
 * block.  Per frame and block:
 *   M = (sum of the block's intensities, row-major from 0) / |G|
 *   the match tests, reset and swap of Sec. 2.3 use M for the intensity;
 *   the matched model's mean is blended with M; its V is the largest squared
 *   distance of the updated mean from the block's intensities,
 *   V = max over j in G of (mean' - I_j)^2 (instead of (mean' - M)^2);
 *   a pixel is background iff (mean_A - I_j)^2 <= theta_d * max(mask floor, ref),
 *   ref = var_A or I_j (the per-pixel rule of the appendix with the block's A).
 * With b = 1 this is exactly orc_forward.  State arrays hold Hb x Wb blocks
 * (Hb = ceil(H/b), Wb = ceil(W/b)); frames and masks are T x H x W; codes
 * (optional) T x Hb x Wb.
 */
int orc_forward_grid(int64_t T, int64_t H, int64_t W, int32_t b, const double* frames,
                     double* mean_a, double* var_a, int32_t* age_a, double* mean_c, double* var_c,
                     int32_t* age_c, const orc_params* p, uint8_t* masks, uint8_t* codes,
                     int nthreads) {
  int64_t Hb, Wb, nb, k;
  if (orc_check(p) || T < 0 || H < 0 || W < 0 || b < 1) return -1;
  if (T == 0 || H == 0 || W == 0) return 0;
  if (!frames || !mean_a || !var_a || !age_a || !mean_c || !var_c || !age_c || !masks) return -1;
  Hb = (H + b - 1) / b;
  Wb = (W + b - 1) / b;
  nb = Hb * Wb;
  orc_set_threads(nthreads);
#pragma omp parallel for schedule(static)
  for (k = 0; k < nb; ++k) {
    const int64_t by = k / Wb, bx = k % Wb;
    const int64_t y0 = by * b, x0 = bx * b;
    const int64_t y1 = y0 + b < H ? y0 + b : H, x1 = x0 + b < W ? x0 + b : W;
    const double n = (double)((y1 - y0) * (x1 - x0));
    orc_model A = {mean_a[k], var_a[k], age_a[k]};
    orc_model C = {mean_c[k], var_c[k], age_c[k]};
    int64_t t, y, x;
    for (t = 0; t < T; ++t) {
      const double* f = frames + t * H * W;
      double sum = 0.0, M;
      int hit_a, hit_c;
      uint8_t code = 0;
      orc_model* U = NULL;
      for (y = y0; y < y1; ++y)
        for (x = x0; x < x1; ++x) sum += f[y * W + x];
      M = sum / n;
      hit_a = orc_sq(M - A.mean) < p->theta_s * orc_max(A.var, p->var_floor);
      hit_c = !hit_a && orc_sq(M - C.mean) < p->theta_s * orc_max(C.var, p->var_floor);
      if (hit_a) {
        code |= ORC_HIT_A;
        U = &A;
      } else if (hit_c) {
        code |= ORC_HIT_C;
        U = &C;
      } else {
        code |= ORC_RESET;
        orc_reset(&C, M, p);
      }
      if (U) {
        const double w = orc_weight(U->age, p);
        const double u = 1.0 - w;
        const double mean = u * U->mean + w * M;
        double V = 0.0;
        for (y = y0; y < y1; ++y)
          for (x = x0; x < x1; ++x) V = orc_max(V, orc_sq(mean - f[y * W + x]));
        U->var = u * U->var + w * V;
        U->mean = mean;
        U->age = U->age < p->age_max ? U->age + 1 : p->age_max;
      }
      if (C.age > A.age) {
        code |= ORC_SWAP;
        A = C;
        orc_reset(&C, M, p);
      }
      for (y = y0; y < y1; ++y)
        for (x = x0; x < x1; ++x) {
          const double I = f[y * W + x];
          const double ref = p->mask_rule == ORC_MASK_PRINTED ? I : A.var;
          const int fg = !(orc_sq(A.mean - I) <= p->theta_d * orc_max(p->mask_floor, ref));
          masks[t * H * W + y * W + x] = fg ? 255 : 0;
        }
      if (codes) codes[t * nb + k] = code;
    }
    mean_a[k] = A.mean; var_a[k] = A.var; age_a[k] = A.age;
    mean_c[k] = C.mean; var_c[k] = C.var; age_c[k] = C.age;
  }
  return 0;
}

/*
 * The 8-bit as-run model of the appendix: 8-bit frames, means and variances
 * stored in 8-bit images (orc_u8 on every write), FP64 arithmetic in between.
 * Same decisions and order as orc_forward; frames, means and variances are
 * uint8 arrays here.
 */
int orc_forward_u8(int64_t T, int64_t N, const uint8_t* frames, uint8_t* mean_a, uint8_t* var_a,
                   int32_t* age_a, uint8_t* mean_c, uint8_t* var_c, int32_t* age_c,
                   const orc_params* p, uint8_t* masks, uint8_t* codes, int nthreads) {
  int64_t nchunk, c;
  if (orc_check(p) || T < 0 || N < 0) return -1;
  if (T > 0 && N > 0 && (!frames || !mean_a || !var_a || !age_a || !mean_c || !var_c || !age_c))
    return -1;
  orc_set_threads(nthreads);
  nchunk = (N + ORC_CHUNK - 1) / ORC_CHUNK;
#pragma omp parallel for schedule(static)
  for (c = 0; c < nchunk; ++c) {
    int64_t p0 = c * ORC_CHUNK, p1 = p0 + ORC_CHUNK < N ? p0 + ORC_CHUNK : N;
    int64_t t, i;
    for (t = 0; t < T; ++t) {
      for (i = p0; i < p1; ++i) {
        int64_t e = t * N + i;
        orc_model A = {(double)mean_a[i], (double)var_a[i], age_a[i]};
        orc_model C = {(double)mean_c[i], (double)var_c[i], age_c[i]};
        orc_tape tp;
        uint8_t code = orc_step_q(&A, &C, (double)frames[e], p, -1, &tp, NULL, 1);
        mean_a[i] = (uint8_t)A.mean; var_a[i] = (uint8_t)A.var; age_a[i] = A.age;
        mean_c[i] = (uint8_t)C.mean; var_c[i] = (uint8_t)C.var; age_c[i] = C.age;
        if (masks) masks[e] = (code & ORC_FG) ? 255 : 0;
        if (codes) codes[e] = code;
      }
    }
  }
  return 0;
}
