/* Drives every entry point of the CPU oracle on small, ragged and empty
 * problems, with every optional output, for a build under AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_oracle_sanitizers.py).  The oracle's
 * sources are included so that its types are visible; the preprocessing
 * oracle is linked as its own translation unit. */
#include "../oracle/dsgm_oracle.c"

#include <stdio.h>

int orc_gauss_weights(int32_t n, double sigma, double* w);
int orc_preprocess(int64_t T, int64_t H, int64_t W, const double* in, double* out, int32_t n,
                   const double* w, int32_t median, int nthreads);
int orc_preprocess_u8(int64_t T, int64_t H, int64_t W, const uint8_t* in, uint8_t* out,
                      int32_t n, const double* w, int32_t median, int nthreads);

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static double urand(void) { /* xorshift64*, uniform in [-1, 1) */
  rng_state ^= rng_state >> 12;
  rng_state ^= rng_state << 25;
  rng_state ^= rng_state >> 27;
  return (double)((rng_state * 2685821657736338717ull) >> 11) * 0x1.0p-52 - 1.0;
}

#define CHECK(x)                                                     \
  do {                                                               \
    if ((x) != 0) {                                                  \
      fprintf(stderr, "FAILED %s at line %d\n", #x, __LINE__);       \
      return 1;                                                      \
    }                                                                \
  } while (0)

static int run(int64_t T, int64_t H, int64_t W, int32_t rule, int32_t mrule) {
  const int64_t N = H * W, TN = T * N;
  const size_t nT = (size_t)(TN > 0 ? TN : 1), nN = (size_t)(N > 0 ? N : 1);
  orc_params p = {2.0, 4.0, 255.0 * (2.0 / 255) * (2.0 / 255), 0.1 * (2.0 / 255) * (2.0 / 255),
                  0.25 * (2.0 / 255) * (2.0 / 255), 30, rule, mrule};
  double* x = malloc(nT * sizeof(double));
  double *mA = malloc(nN * 8), *vA = malloc(nN * 8), *mC = malloc(nN * 8), *vC = malloc(nN * 8);
  int32_t *aA = malloc(nN * 4), *aC = malloc(nN * 4);
  double *m0 = malloc(nN * 8), *v0 = malloc(nN * 8), *c0 = malloc(nN * 8), *w0 = malloc(nN * 8);
  int32_t *a0 = malloc(nN * 4), *b0 = malloc(nN * 4);
  uint8_t *masks = malloc(nT), *codes = malloc(nT);
  double *bg = malloc(nT * 8), *marg = malloc(nT * 3 * 8);
  double *gbg = malloc(nT * 8), *gst = malloc(4 * nN * 8), *gx = malloc(nT * 8),
         *gs0 = malloc(4 * nN * 8), *gvi = malloc(nN * 8);
  double *dx = malloc(nT * 8), *ds0 = malloc(4 * nN * 8), *dbg = malloc(nT * 8),
         *dsT = malloc(4 * nN * 8);
  double *f1 = malloc(nT * 8), w[7], map[9] = {1, 0.01, 0.4, -0.01, 1, -0.7, 0, 0, 1};
  double *omA = malloc(nN * 8), *ovA = malloc(nN * 8), *omC = malloc(nN * 8), *ovC = malloc(nN * 8);
  int32_t *oaA = malloc(nN * 4), *oaC = malloc(nN * 4);
  uint8_t *u8x = malloc(nT), *u8m[4];
  int64_t i;
  for (i = 0; i < 4; ++i) u8m[i] = malloc(nN);
  for (i = 0; i < TN; ++i) {
    x[i] = urand();
    gbg[i] = urand();
    dx[i] = urand();
    u8x[i] = (uint8_t)(128 + 127 * urand());
  }
  for (i = 0; i < N; ++i) {
    m0[i] = urand();
    v0[i] = fabs(urand());
    c0[i] = urand();
    w0[i] = fabs(urand());
    a0[i] = 1 + (int32_t)(15 * (urand() + 1));
    b0[i] = 1 + (int32_t)(15 * (urand() + 1));
  }
  for (i = 0; i < 4 * N; ++i) {
    gst[i] = urand();
    ds0[i] = urand();
  }
  memcpy(mA, m0, nN * 8); memcpy(vA, v0, nN * 8); memcpy(mC, c0, nN * 8); memcpy(vC, w0, nN * 8);
  memcpy(aA, a0, nN * 4); memcpy(aC, b0, nN * 4);
  CHECK(orc_forward(T, N, x, mA, vA, aA, mC, vC, aC, &p, masks, bg, codes, NULL, marg, 0));
  CHECK(orc_forward(T, N, x, mA, vA, aA, mC, vC, aC, &p, NULL, NULL, NULL, codes, NULL, 0));
  CHECK(orc_backward(T, N, x, m0, v0, a0, c0, w0, b0, &p, codes, gbg, gst, gx, gs0, gvi, 0));
  CHECK(orc_backward(T, N, x, m0, v0, a0, c0, w0, b0, &p, NULL, NULL, NULL, gx, gs0, gvi, 0));
  CHECK(orc_jvp(T, N, x, m0, v0, a0, c0, w0, b0, &p, codes, dx, ds0, 0.5, dbg, dsT, 0));
  if (T > 0) /* the warp reads one whole frame */
    CHECK(orc_warp_state(H, W, map, x, m0, v0, a0, c0, w0, b0, &p, omA, ovA, oaA, omC, ovC, oaC, 0));
  {
    const int32_t b = 2;
    const int64_t nb = ((H + b - 1) / b) * ((W + b - 1) / b);
    double *gm = calloc((size_t)(nb > 0 ? nb : 1) * 4, 8);
    int32_t* ga = calloc((size_t)(nb > 0 ? nb : 1) * 2, 4);
    for (i = 0; i < nb; ++i) { ga[i] = 1; ga[nb + i] = 1; gm[nb + i] = 0.1; gm[3 * nb + i] = 0.1; }
    CHECK(orc_forward_grid(T, H, W, b, x, gm, gm + nb, ga, gm + 2 * nb, gm + 3 * nb, ga + nb, &p,
                           masks, codes, 0));
    free(gm);
    free(ga);
  }
  for (i = 0; i < N; ++i) {
    int k;
    for (k = 0; k < 4; ++k) u8m[k][i] = (uint8_t)(128 + 127 * urand());
    aA[i] = a0[i];
    aC[i] = b0[i];
  }
  CHECK(orc_forward_u8(T, N, u8x, u8m[0], u8m[1], aA, u8m[2], u8m[3], aC, &p, masks, codes, 0));
  CHECK(orc_gauss_weights(5, 1.0, w));
  CHECK(orc_preprocess(T, H, W, x, f1, 5, w, 1, 0));
  CHECK(orc_preprocess(T, H, W, x, f1, 0, NULL, 1, 0));
  CHECK(orc_gauss_weights(7, 2.0, w));
  CHECK(orc_preprocess(T, H, W, x, f1, 7, w, 0, 0));
  {
    uint8_t* pu = (uint8_t*)malloc((size_t)(T * H * W) + 1);
    CHECK(orc_preprocess_u8(T, H, W, u8x, pu, 7, w, 1, 0));
    CHECK(orc_gauss_weights(3, 0.8, w));
    CHECK(orc_preprocess_u8(T, H, W, u8x, pu, 3, w, 0, 0));
    CHECK(orc_preprocess_u8(T, H, W, u8x, pu, 0, NULL, 1, 0));
    free(pu);
  }
  free(x); free(mA); free(vA); free(mC); free(vC); free(aA); free(aC);
  free(m0); free(v0); free(c0); free(w0); free(a0); free(b0);
  free(masks); free(codes); free(bg); free(marg); free(gbg); free(gst); free(gx); free(gs0);
  free(gvi); free(dx); free(ds0); free(dbg); free(dsT); free(f1);
  free(omA); free(ovA); free(omC); free(ovC); free(oaA); free(oaC); free(u8x);
  for (i = 0; i < 4; ++i) free(u8m[i]);
  return 0;
}

int main(void) {
  const int64_t shapes[][3] = {{13, 5, 7}, {40, 1, 1}, {1, 9, 2}, {0, 4, 4}, {3, 0, 5}, {7, 1, 33}};
  int s, rule, mrule;
  for (s = 0; s < (int)(sizeof(shapes) / sizeof(shapes[0])); ++s)
    for (rule = 0; rule < 2; ++rule)
      for (mrule = 0; mrule < 2; ++mrule)
        if (run(shapes[s][0], shapes[s][1], shapes[s][2], rule, mrule)) return 1;
  printf("ok\n");
  return 0;
}
