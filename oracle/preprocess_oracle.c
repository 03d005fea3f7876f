/*
 * preprocess_oracle.c -- plain FP64 reference of the frame preprocessing the
 * paper applies before the background update: a Gaussian blur, then a 3 x 3
 * median filter (Henderson & Vertescher, arXiv:1702.05156, Sec. 2.1, the
 * serial and CUDA preprocessing of Sec. 3.1.1 and 3.3.1, and the appendix
 * snippets of both filters).
 *
 * TEST INFRASTRUCTURE ONLY, like dsgm_oracle.c: only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg may load this library.
 *
 * Readings (the paper gives no kernel size, sigma, filter order or border rule
 * that can be used as printed):
 *   - Gaussian weights: the Sec. 2.1 density sampled at integer offsets
 *     d = i - r (i = 0..n-1, r = (n-1)/2, mean 0), e_i = exp(-(d*d) / (2*sigma*sigma))
 *     evaluated in that order, then normalised by their sum taken in index
 *     order, w_i = e_i / sum (the density's constant factor cancels).
 *   - the blur is separable, as in the paper's CUDA version (Sec. 3.3.1): a
 *     pass along rows, then a pass along columns of the row-blurred image,
 *     each sum accumulated from 0 in index order i = 0..n-1.
 *   - borders: an index outside the frame is clamped to the nearest row or
 *     column inside it (the appendix clamps to the height and width, one past
 *     the last valid index; the last valid index is used instead).
 *   - order: Gaussian first, then the median of the 3 x 3 neighbourhood of the
 *     blurred frame (same border clamping).  n = 0 skips the blur, median = 0
 *     skips the median.
 *
 * Frames are dense T x H x W (frame-major), FP64.
 *
 * orc_preprocess_u8 is the same pipeline as the appendix runs it on 8-bit
 * frames (its blur and median snippets read and write 8-bit images), with
 * these readings:
 *   - the blur is the appendix's two-dimensional one: for each pixel a
 *     single-precision sum, started at 0 and taken over the window's rows
 *     (outer) and columns (inner), of the 8-bit value times the window's
 *     weight, each product and sum rounded to single precision (no fused
 *     multiply-add);
 *   - the window's weights are the products w_i * w_j of the normalised
 *     one-dimensional weights above (the two-dimensional Gaussian density
 *     factors into them), each product taken in double precision and rounded
 *     once to single precision;
 *   - the blurred value is written to the 8-bit image by dropping its fraction
 *     (limited to [0, 255], where the conversion has no defined result);
 *   - the median then sorts the nine 8-bit values of each clamped 3 x 3
 *     neighbourhood of the blurred image and takes the middle one.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#ifdef _OPENMP
#include <omp.h>
#endif

static int64_t pre_clamp(int64_t v, int64_t hi) { return v < 0 ? 0 : (v > hi ? hi : v); }

int orc_gauss_weights(int32_t n, double sigma, double* w) {
  if (n < 1 || n > 31 || (n % 2) == 0 || !(sigma > 0.0) || !w) return -1;
  const int32_t r = (n - 1) / 2;
  double s = 0.0;
  for (int32_t i = 0; i < n; ++i) {
    const double d = (double)(i - r);
    w[i] = exp(-(d * d) / (2.0 * sigma * sigma));
    s += w[i];
  }
  for (int32_t i = 0; i < n; ++i) w[i] = w[i] / s;
  return 0;
}

/* median of nine values: sort ascending (insertion sort), take the middle */
static double pre_median9(double v[9]) {
  for (int i = 1; i < 9; ++i) {
    const double x = v[i];
    int j = i - 1;
    while (j >= 0 && v[j] > x) {
      v[j + 1] = v[j];
      --j;
    }
    v[j + 1] = x;
  }
  return v[4];
}

int orc_preprocess(int64_t T, int64_t H, int64_t W, const double* in, double* out, int32_t n,
                   const double* w, int32_t median, int nthreads) {
  if (T < 0 || H < 0 || W < 0 || (n != 0 && (n < 1 || (n % 2) == 0 || !w))) return -1;
  if (T == 0 || H == 0 || W == 0) return 0;
  if (!in || !out) return -1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
  const int64_t HW = H * W;
  const int32_t r = n > 0 ? (n - 1) / 2 : 0;
  int rc = 0;
#pragma omp parallel
  {
    double* hb = (double*)malloc(sizeof(double) * (size_t)HW);
    double* gb = (double*)malloc(sizeof(double) * (size_t)HW);
    if (!hb || !gb) {
#pragma omp atomic write
      rc = -1;
    }
#pragma omp for schedule(static)
    for (int64_t t = 0; t < T; ++t) {
      if (!hb || !gb) continue;
      const double* x = in + t * HW;
      if (n > 0) {
        for (int64_t y = 0; y < H; ++y)
          for (int64_t c = 0; c < W; ++c) {
            double acc = 0.0;
            for (int32_t j = 0; j < n; ++j) acc += w[j] * x[y * W + pre_clamp(c + j - r, W - 1)];
            hb[y * W + c] = acc;
          }
        for (int64_t y = 0; y < H; ++y)
          for (int64_t c = 0; c < W; ++c) {
            double acc = 0.0;
            for (int32_t i = 0; i < n; ++i) acc += w[i] * hb[pre_clamp(y + i - r, H - 1) * W + c];
            gb[y * W + c] = acc;
          }
      } else {
        for (int64_t k = 0; k < HW; ++k) gb[k] = x[k];
      }
      double* o = out + t * HW;
      if (median) {
        for (int64_t y = 0; y < H; ++y)
          for (int64_t c = 0; c < W; ++c) {
            double v[9];
            int k = 0;
            for (int dy = -1; dy <= 1; ++dy)
              for (int dx = -1; dx <= 1; ++dx)
                v[k++] = gb[pre_clamp(y + dy, H - 1) * W + pre_clamp(c + dx, W - 1)];
            o[y * W + c] = pre_median9(v);
          }
      } else {
        for (int64_t k = 0; k < HW; ++k) o[k] = gb[k];
      }
    }
    free(hb);
    free(gb);
  }
  return rc;
}

/* median of nine 8-bit values: insertion sort ascending, take the middle */
static uint8_t pre_median9_u8(uint8_t v[9]) {
  for (int i = 1; i < 9; ++i) {
    const uint8_t x = v[i];
    int j = i - 1;
    while (j >= 0 && v[j] > x) {
      v[j + 1] = v[j];
      --j;
    }
    v[j + 1] = x;
  }
  return v[4];
}

int orc_preprocess_u8(int64_t T, int64_t H, int64_t W, const uint8_t* in, uint8_t* out, int32_t n,
                      const double* w, int32_t median, int nthreads) {
  if (T < 0 || H < 0 || W < 0 || (n != 0 && (n < 1 || n > 31 || (n % 2) == 0 || !w))) return -1;
  if (T == 0 || H == 0 || W == 0) return 0;
  if (!in || !out) return -1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
  const int64_t HW = H * W;
  const int32_t r = n > 0 ? (n - 1) / 2 : 0;
  /* the window's single-precision weights, row-major */
  float w2[31 * 31];
  for (int32_t i = 0; i < n; ++i)
    for (int32_t j = 0; j < n; ++j) w2[i * n + j] = (float)(w[i] * w[j]);
  int rc = 0;
#pragma omp parallel
  {
    uint8_t* gb = (uint8_t*)malloc((size_t)HW);
    if (!gb) {
#pragma omp atomic write
      rc = -1;
    }
#pragma omp for schedule(static)
    for (int64_t t = 0; t < T; ++t) {
      if (!gb) continue;
      const uint8_t* x = in + t * HW;
      if (n > 0) {
        for (int64_t y = 0; y < H; ++y)
          for (int64_t c = 0; c < W; ++c) {
            float blur = 0.0f;
            for (int32_t i = 0; i < n; ++i)
              for (int32_t j = 0; j < n; ++j) {
                const float pixel = (float)x[pre_clamp(y + i - r, H - 1) * W + pre_clamp(c + j - r, W - 1)];
                const float prod = pixel * w2[i * n + j];
                blur = blur + prod;
              }
            const float f = truncf(blur);
            gb[y * W + c] = (uint8_t)(f < 0.0f ? 0.0f : (f > 255.0f ? 255.0f : f));
          }
      } else {
        for (int64_t k = 0; k < HW; ++k) gb[k] = x[k];
      }
      uint8_t* o = out + t * HW;
      if (median) {
        for (int64_t y = 0; y < H; ++y)
          for (int64_t c = 0; c < W; ++c) {
            uint8_t v[9];
            int k = 0;
            for (int dy = -1; dy <= 1; ++dy)
              for (int dx = -1; dx <= 1; ++dx)
                v[k++] = gb[pre_clamp(y + dy, H - 1) * W + pre_clamp(c + dx, W - 1)];
            o[y * W + c] = pre_median9_u8(v);
          }
      } else {
        for (int64_t k = 0; k < HW; ++k) o[k] = gb[k];
      }
    }
    free(gb);
  }
  return rc;
}
