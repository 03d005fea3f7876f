// Drives the host side of libdsgm.so -- argument validation, plan layout and
// ordering, the tuner table, status strings -- for a build whose host code is
// instrumented with AddressSanitizer and UndefinedBehaviorSanitizer
// (tests/test_api_sanitizers.py).  Runs without a GPU: every call either fails
// validation before its first HIP call, has nothing to do, or reaches a HIP
// call that reports the missing device (DSGM_E_HIP), which is what is
// expected then.  Device pointers are fake addresses that are never
// dereferenced on the host.
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <thread>
#include <vector>

#include "dsgm.h"

static int failures = 0;

#define EXPECT(call, want)                                                                  \
  do {                                                                                      \
    const int rc_ = (call);                                                                 \
    if (rc_ != (want)) {                                                                    \
      fprintf(stderr, "line %d: %s returned %d, expected %d (%s)\n", __LINE__, #call, rc_,   \
              (want), dsgm_last_error());                                                   \
      ++failures;                                                                           \
    }                                                                                       \
  } while (0)

// any status but success (a HIP call without a device fails one way or another)
#define EXPECT_FAIL(call)                                                                   \
  do {                                                                                      \
    const int rc_ = (call);                                                                 \
    if (rc_ == DSGM_OK) {                                                                   \
      fprintf(stderr, "line %d: %s succeeded without a device\n", __LINE__, #call);         \
      ++failures;                                                                           \
    }                                                                                       \
  } while (0)

static void* fake(uintptr_t a) { return reinterpret_cast<void*>(a); }

static const uintptr_t F = uintptr_t(1) << 20;  // aligned to every element size

static dsgm_state state_at(uintptr_t a) {
  dsgm_state s;
  s.mean_a = fake(a);
  s.var_a = fake(a + 0x100000);
  s.mean_c = fake(a + 0x200000);
  s.var_c = fake(a + 0x300000);
  s.age_a = static_cast<uint8_t*>(fake(a + 0x400000));
  s.age_c = static_cast<uint8_t*>(fake(a + 0x500000));
  return s;
}

static dsgm_shape shape(int64_t T, int64_t H, int64_t W) {
  dsgm_shape s = {T, H, W, W, H * W};
  return s;
}

static void params_and_strings() {
  dsgm_params p;
  EXPECT(dsgm_params_default(&p, 2.0, DSGM_MASK_VARIANCE), DSGM_OK);
  EXPECT(dsgm_params_default(nullptr, 2.0, 0), DSGM_E_ARG);
  EXPECT(dsgm_params_default(&p, -1.0, 0), DSGM_E_ARG);
  EXPECT(dsgm_params_default(&p, 2.0, 9), DSGM_E_ARG);
  for (int s = -9; s <= 2; ++s) {
    const char* n = dsgm_status_string(s);
    if (!n || !n[0]) ++failures;
  }
  if (dsgm_version() < 100) ++failures;
  if (strlen(dsgm_last_error()) > 511) ++failures;
}

static void forward_paths() {
  dsgm_params p;
  dsgm_params_default(&p, 2.0, 0);
  dsgm_state st = state_at(F);
  uint8_t* m = static_cast<uint8_t*>(fake(F));
  // nothing to do: no HIP call
  EXPECT(dsgm_forward(nullptr, DSGM_IN_F64, shape(0, 8, 8), DSGM_ACC_F64, &p, &st, nullptr,
                      nullptr, nullptr, 0, 0, nullptr, nullptr),
         DSGM_OK);
  EXPECT(dsgm_forward(fake(F), DSGM_IN_F32, shape(5, 0, 8), DSGM_ACC_F32, &p, &st, m, nullptr,
                      nullptr, 0, 0, nullptr, nullptr),
         DSGM_OK);
  // every kind of rejection
  EXPECT(dsgm_forward(fake(F), dsgm_in_dtype(7), shape(4, 8, 8), DSGM_ACC_F64, &p, &st, m, nullptr,
                      nullptr, 0, 0, nullptr, nullptr),
         DSGM_E_DTYPE);
  EXPECT(dsgm_forward(fake(F), DSGM_IN_F64, shape(4, 8, 8), dsgm_acc(9), &p, &st, m, nullptr,
                      nullptr, 0, 0, nullptr, nullptr),
         DSGM_E_DTYPE);
  EXPECT(dsgm_forward(fake(F), DSGM_IN_F64, shape(4, 8, 8), DSGM_ACC_F32X2, &p, &st, m, nullptr,
                      nullptr, 0, 0, nullptr, nullptr),
         DSGM_E_DTYPE);
  EXPECT(dsgm_forward(fake(F), DSGM_IN_F64, shape(4, 8, 8), DSGM_ACC_F64, nullptr, &st, m,
                      nullptr, nullptr, 0, 0, nullptr, nullptr),
         DSGM_E_ARG);
  EXPECT(dsgm_forward(fake(F), DSGM_IN_F64, shape(4, 8, 8), DSGM_ACC_F64, &p, nullptr, m,
                      nullptr, nullptr, 0, 0, nullptr, nullptr),
         DSGM_E_ARG);
  EXPECT(dsgm_forward(fake(F), DSGM_IN_F64, shape(-1, 8, 8), DSGM_ACC_F64, &p, &st, m, nullptr,
                      nullptr, 0, 0, nullptr, nullptr),
         DSGM_E_SHAPE);
  dsgm_shape bad = shape(4, 8, 8);
  bad.row_stride = 3;
  EXPECT(dsgm_forward(fake(F), DSGM_IN_F64, bad, DSGM_ACC_F64, &p, &st, m, nullptr, nullptr, 0, 0,
                      nullptr, nullptr),
         DSGM_E_SHAPE);
  EXPECT(dsgm_forward(fake(F), DSGM_IN_F64, shape(1, 1 << 17, 1 << 15), DSGM_ACC_F64, &p, &st, m,
                      nullptr, nullptr, 0, 0, nullptr, nullptr),
         DSGM_E_SHAPE);
  EXPECT(dsgm_forward(fake(F + 4), DSGM_IN_F64, shape(4, 8, 8), DSGM_ACC_F64, &p, &st, m, nullptr,
                      nullptr, 0, 0, nullptr, nullptr),
         DSGM_E_ALIGN);
  EXPECT(dsgm_forward(fake(F), DSGM_IN_F64, shape(4, 8, 8), DSGM_ACC_F64, &p, &st, m, nullptr,
                      fake(F), 10, 2, nullptr, nullptr),
         DSGM_E_WORKSPACE);
  EXPECT(dsgm_forward(fake(F), DSGM_IN_F64, shape(4, 8, 8), DSGM_ACC_F64, &p, &st, m, nullptr,
                      fake(F), 1 << 20, 0, nullptr, nullptr),
         DSGM_E_ARG);
  dsgm_params q = p;
  q.age_max = 0;
  EXPECT(dsgm_forward(fake(F), DSGM_IN_F64, shape(4, 8, 8), DSGM_ACC_F64, &q, &st, m, nullptr,
                      nullptr, 0, 0, nullptr, nullptr),
         DSGM_E_ARG);
  q = p;
  q.theta_s = -1.0;
  EXPECT(dsgm_forward(fake(F), DSGM_IN_F64, shape(4, 8, 8), DSGM_ACC_F64, &q, &st, m, nullptr,
                      nullptr, 0, 0, nullptr, nullptr),
         DSGM_E_ARG);
  // valid arguments reach the launch, which fails without a device
  EXPECT_FAIL(dsgm_forward(fake(F), DSGM_IN_BF16, shape(3, 5, 12), DSGM_ACC_F32, &p, &st, m,
                           nullptr, nullptr, 0, 0, nullptr, nullptr));
  EXPECT_FAIL(dsgm_state_init_from_frame(fake(F), DSGM_IN_F32, shape(1, 4, 4), DSGM_ACC_F32X2, &p,
                                         &st, nullptr));
  // sizes
  if (dsgm_ckpt_bytes(shape(100, 3, 5), DSGM_ACC_F64, 32) != size_t(4 * (4 * 256 + 2 * 256)))
    ++failures;
  if (dsgm_ckpt_bytes(shape(100, 3, 5), DSGM_ACC_F64, 0) != 0) ++failures;
  if (dsgm_workspace_bytes(shape(4, 8, 8), dsgm_acc(9)) != 0) ++failures;
}

static void backward_paths() {
  dsgm_params p;
  dsgm_params_default(&p, 2.0, 0);
  dsgm_grad_state g = {fake(F), fake(F + 0x10000), fake(F + 0x20000), fake(F + 0x30000)};
  double* gvi = static_cast<double*>(fake(F));
  const dsgm_shape sh = shape(4, 8, 8);
  EXPECT(dsgm_backward(fake(F), DSGM_IN_F64, sh, DSGM_ACC_F64, &p, fake(F), 1 << 30, 2, nullptr,
                       nullptr, fake(F), &g, gvi, fake(F), 16, nullptr),
         DSGM_E_WORKSPACE);
  EXPECT(dsgm_backward(fake(F), DSGM_IN_F64, sh, DSGM_ACC_F64, &p, fake(F), 1 << 30, 2, nullptr,
                       nullptr, fake(F), &g, gvi, nullptr, 1 << 20, nullptr),
         DSGM_E_ARG);
  EXPECT(dsgm_backward(fake(F), DSGM_IN_F64, sh, DSGM_ACC_F64, &p, nullptr, 0, 2, nullptr, nullptr,
                       fake(F), &g, gvi, fake(F), 1 << 20, nullptr),
         DSGM_E_ARG);
  EXPECT(dsgm_backward_noalloc(fake(F), DSGM_IN_F64, sh, DSGM_ACC_F64, &p, fake(F), 1 << 30, 0,
                               nullptr, nullptr, fake(F), &g, gvi, nullptr),
         DSGM_E_ARG);
  EXPECT(dsgm_backward_noalloc(fake(F), DSGM_IN_F32, shape(1, 3, 2796203), DSGM_ACC_F32,
                               &p, fake(F), size_t(1) << 40, 1, nullptr, nullptr, fake(F), &g, gvi,
                               nullptr),
         DSGM_E_WORKSPACE);
  EXPECT_FAIL(dsgm_backward(fake(F), DSGM_IN_F32, sh, DSGM_ACC_F32X2, &p, fake(F), 1 << 30, 2,
                            nullptr, &g, fake(F), &g, gvi, fake(F), 1 << 20, nullptr));
  EXPECT_FAIL(dsgm_backward_noalloc(fake(F), DSGM_IN_F32, sh, DSGM_ACC_F32, &p, fake(F), 1 << 30,
                                    2, nullptr, nullptr, fake(F), &g, gvi, nullptr));
}

static void batch_paths() {
  dsgm_params p;
  dsgm_params_default(&p, 2.0, 0);
  // many uneven instances, some empty, some with bg or counters
  std::vector<dsgm_instance> inst;
  uint64_t r = 12345;
  for (int i = 0; i < 300; ++i) {
    r = r * 6364136223846793005ull + 1442695040888963407ull;
    const int64_t T = int64_t(r >> 58), H = int64_t((r >> 40) & 63), W = 4 * int64_t((r >> 20) & 31);
    dsgm_instance d;
    memset(&d, 0, sizeof(d));
    d.shape = shape(T, H, W);
    d.frames = fake(F * (i + 1));
    d.state = state_at(F * (i + 1));
    d.masks = static_cast<uint8_t*>(fake(F * (i + 1)));
    d.bg = (i % 5 == 0) ? fake(F * (i + 1)) : nullptr;
    d.fg_counts = (i % 3 == 0) ? static_cast<uint32_t*>(fake(F * (i + 1))) : nullptr;
    inst.push_back(d);
  }
  const int32_t n = int32_t(inst.size());
  const size_t bytes = dsgm_batch_plan_bytes(inst.data(), n, DSGM_IN_BF16, DSGM_ACC_F32);
  if (bytes == 0) ++failures;
  if (dsgm_batch_plan_bytes(inst.data(), n, DSGM_IN_BF16, DSGM_ACC_F32X2) != 0) ++failures;
  if (dsgm_batch_plan_bytes(nullptr, 3, DSGM_IN_F32, DSGM_ACC_F32) != 0) ++failures;
  dsgm_batch_plan plan;
  memset(&plan, 0, sizeof(plan));
  EXPECT(dsgm_plan_batched(inst.data(), n, DSGM_IN_BF16, DSGM_ACC_F32, fake(F), bytes - 1, &plan,
                           nullptr),
         DSGM_E_WORKSPACE);
  EXPECT(dsgm_plan_batched(inst.data(), n, DSGM_IN_BF16, DSGM_ACC_F32, fake(F + 8), bytes, &plan,
                           nullptr),
         DSGM_E_ALIGN);
  EXPECT(dsgm_plan_batched(inst.data(), n, DSGM_IN_BF16, DSGM_ACC_F32, fake(F), bytes, nullptr,
                           nullptr),
         DSGM_E_ARG);
  // lays out, fills and orders the host copy, then fails at the device query
  EXPECT_FAIL(dsgm_plan_batched(inst.data(), n, DSGM_IN_BF16, DSGM_ACC_F32, fake(F), bytes, &plan,
                                nullptr));
  inst[7].frames = fake(F + 1);
  if (dsgm_batch_plan_bytes(inst.data(), n, DSGM_IN_BF16, DSGM_ACC_F32) != 0) ++failures;
  EXPECT(dsgm_forward_batched(nullptr, &p, nullptr), DSGM_E_ARG);
  plan.device_plan = fake(F);
  plan.in_dtype = DSGM_IN_F32;
  plan.acc = DSGM_ACC_F32;
  plan.vector = 3;
  EXPECT(dsgm_forward_batched(&plan, &p, nullptr), DSGM_E_ARG);
  plan.vector = 2;
  plan.n_items = 0;
  plan.grid = 0;
  EXPECT(dsgm_forward_batched(&plan, &p, nullptr), DSGM_E_ARG);
  plan.grid = 1;
  EXPECT(dsgm_forward_batched(&plan, &p, nullptr), DSGM_OK);
}

static void extension_paths() {
  dsgm_params p;
  dsgm_params_default(&p, 2.0, 0);
  dsgm_state st = state_at(F);
  dsgm_state st2 = state_at(F * 64);
  uint8_t* m = static_cast<uint8_t*>(fake(F));
  double w[7];
  EXPECT(dsgm_gauss_weights(5, 1.0, w), DSGM_OK);
  EXPECT(dsgm_gauss_weights(4, 1.0, w), DSGM_E_ARG);
  EXPECT(dsgm_gauss_weights(5, 0.0, w), DSGM_E_ARG);
  dsgm_filter f;
  memset(&f, 0, sizeof(f));
  f.n = 5;
  f.median = 1;
  memcpy(f.weights, w, sizeof(double) * 5);
  EXPECT(dsgm_forward_filtered(fake(F), DSGM_IN_F32, shape(2, 8, 8), DSGM_ACC_F32X2, &p, &f, &st,
                               m, nullptr, nullptr, nullptr, nullptr),
         DSGM_E_DTYPE);
  f.n = 8;
  EXPECT(dsgm_forward_filtered(fake(F), DSGM_IN_F32, shape(2, 8, 8), DSGM_ACC_F32, &p, &f, &st, m,
                               nullptr, nullptr, nullptr, nullptr),
         DSGM_E_ARG);
  const double id[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  EXPECT(dsgm_forward_warped(fake(F), DSGM_IN_F64, shape(2, 8, 8), DSGM_ACC_F64, &p, id, &st, &st2,
                             m, nullptr, nullptr, nullptr),
         DSGM_E_SHAPE);
  EXPECT(dsgm_forward_warped(fake(F), DSGM_IN_F64, shape(1, 8, 8), DSGM_ACC_F64, &p, id, &st, &st,
                             m, nullptr, nullptr, nullptr),
         DSGM_E_ARG);
  EXPECT(dsgm_forward_grid(fake(F), DSGM_IN_F64, shape(2, 8, 8), DSGM_ACC_F64, &p, 3, &st, m,
                           nullptr, nullptr, nullptr),
         DSGM_E_UNSUPPORTED);
  EXPECT(dsgm_count_nonfinite(nullptr, DSGM_IN_F64, shape(2, 8, 8),
                              static_cast<uint64_t*>(fake(F)), nullptr),
         DSGM_E_ARG);
}

static void tuner_paths() {
  int32_t chosen[2] = {7, 7};
  EXPECT(dsgm_autotune_clear(), DSGM_OK);
  const dsgm_shape sh = shape(500, 48, 64);
  if (dsgm_autotune_bytes(DSGM_IN_F64, DSGM_ACC_F64, sh, 0) == 0) ++failures;
  if (dsgm_autotune_bytes(DSGM_IN_F64, DSGM_ACC_F32, sh, 0) != 0) ++failures;
  EXPECT(dsgm_autotune(DSGM_IN_F64, DSGM_ACC_F64, sh, 64, fake(F), 1 << 30, chosen, nullptr),
         DSGM_E_ARG);
  EXPECT(dsgm_autotune(DSGM_IN_F64, DSGM_ACC_F64, sh, 0, fake(F), 16, chosen, nullptr),
         DSGM_E_WORKSPACE);
  EXPECT(dsgm_autotune(DSGM_IN_F64, DSGM_ACC_F64, sh, 0, fake(F + 8), 1 << 30, chosen, nullptr),
         DSGM_E_ALIGN);
  EXPECT(dsgm_autotune_lookup(DSGM_IN_F64, DSGM_ACC_F64, sh, 0, chosen), DSGM_OK);
  if (chosen[0] != 0 || chosen[1] != 0) ++failures;  // not tuned
  EXPECT(dsgm_autotune_lookup(DSGM_IN_F64, DSGM_ACC_F64, sh, 0, nullptr), DSGM_E_ARG);
  EXPECT(dsgm_set_launch(100, 0), DSGM_E_ARG);
  EXPECT(dsgm_set_launch(0, 3), DSGM_E_ARG);
  // the tables from several threads at once
  std::vector<std::thread> th;
  for (int t = 0; t < 8; ++t)
    th.emplace_back([t] {
      int32_t c[2];
      for (int i = 0; i < 200; ++i) {
        dsgm_autotune_lookup(DSGM_IN_F32, DSGM_ACC_F32, shape(10, 8 + t, 8 + i % 4), 0, c);
        if (i % 50 == 0) dsgm_autotune_clear();
        dsgm_set_launch(0, 0);
        dsgm_status_string(i % 9 - 8);
      }
    });
  for (auto& x : th) x.join();
  EXPECT(dsgm_set_launch(0, 0), DSGM_OK);
}

int main() {
  params_and_strings();
  forward_paths();
  backward_paths();
  batch_paths();
  extension_paths();
  tuner_paths();
  if (failures) {
    fprintf(stderr, "%d failures\n", failures);
    return 1;
  }
  printf("ok\n");
  return 0;
}
