// dsgm_device.h -- device-side pieces shared by the DSGM kernels (internal).
//
// One step of the Dual-Mode Single Gaussian Model for one pixel (Henderson &
// Vertescher, arXiv:1702.05156, Sec. 2.2-2.3 and the appendix's inner update),
// written branch-free for 64-wide wavefronts:
//
//   match tests   hitA = (x-mA)^2 < ts*max(vA, vf); hitC = (x-mC)^2 < ts*max(vC, vf)
//                 (evaluated as two comparisons, see step_core())
//                 (C only counts when A failed: the table index below gives A priority)
//   update        the matched model (A if hitA, else C) is blended with x using the
//                 weights of its age (Sec. 2.2): m' = u*m + w*x, V = (m'-x)^2,
//                 v' = u*v + w*V, age' = min(age+1, age_max)
//   reset         neither matched: C = (x, var_init, 1).  This is the same update
//                 with the table slot RESET_SLOT, whose weights are u = 0, w = 1,
//                 whose variance offset is var_init and whose next age is 1:
//                 0*m + 1*x = x, (x-x)^2 = 0, 0*v + 1*0 + var_init = var_init, all
//                 exact in IEEE arithmetic, so no extra select is needed.
//   exchange      if hitA the result goes to A, else to C
//   swap          C older than A: A = C, C = (x, var_init, 1) (rare: a branch
//                 that the whole wavefront skips when no lane swaps, any_lane())
//   mask          background iff (mA-x)^2 <= td*max(mf, ref), ref = vA or x
//
// With Acc = double every product and sum is rounded on its own (the library is
// built with -ffp-contract=off), so results are bit-identical to a scalar FP64
// evaluation in the paper's order.  With Acc = float the two blends use fused
// multiply-adds.  With Acc = f32x2 (compensated single precision, see
// dsgm_f32x2.h) the step has its own form, step_core_x2().
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dsgm_f32x2.h"

namespace dsgm {

constexpr int RESET_SLOT = 256;  // table slot used by the candidate reset
constexpr int TABLE_SIZE = 257;  // ages 0..255 plus the reset slot

enum : unsigned { CODE_HIT_A = 1, CODE_HIT_C = 2, CODE_RESET = 4, CODE_SWAP = 8, CODE_FG = 16 };

// Per-age update constants.  `r` is added to the blended variance (0 except in
// the reset slot); `next` is the age after the update.
template <typename Acc>
struct alignas(4 * sizeof(Acc)) TableEntry {
  Acc u, w, r;
  int32_t next;
};

template <typename Acc>
struct StepConsts {
  Acc theta_s, theta_d, var_init;
  Acc ts_vf;  // theta_s * var_floor
  Acc td_mf;  // theta_d * mask_floor
};

// Fill one table slot.  w = 1/(a+1) (Sec. 2.2) or 1/a (appendix), u = 1 - w,
// both rounded in the accumulation type; age 0 (never valid) maps to w = 1.
template <typename Acc>
__device__ inline TableEntry<Acc> make_entry(int i, int weight_rule, int age_max, Acc var_init) {
  if constexpr (is_f32x2<Acc>::value) {
    // the FP64 weights, each split into the nearest pair
    const TableEntry<double> d = make_entry<double>(i, weight_rule, age_max, double(var_init));
    TableEntry<f32x2> e;
    e.u = f32x2(d.u);
    e.w = f32x2(d.w);
    e.r = i == RESET_SLOT ? var_init : f32x2(0.f);
    e.next = d.next;
    return e;
  } else {
    TableEntry<Acc> e;
    if (i == RESET_SLOT) {
      e.u = Acc(0);
      e.w = Acc(1);
      e.r = var_init;
      e.next = 1;
      return e;
    }
    const Acc one = Acc(1);
    Acc w;
    if (weight_rule == 1)
      w = i == 0 ? one : one / Acc(i);
    else
      w = one / (Acc(i) + one);
    e.w = w;
    e.u = one - w;
    e.r = Acc(0);
    e.next = i + 1 < age_max ? i + 1 : age_max;
    return e;
  }
}

// The per-launch constants of the step.  The floor products are rounded once
// in the accumulation type (for f32x2: formed in FP64 and split), identically
// in the forward and the adjoint's replay, so both take the same decisions.
template <typename Acc>
__device__ __forceinline__ StepConsts<Acc> step_consts(double theta_s, double theta_d,
                                                       double var_init, double var_floor,
                                                       double mask_floor) {
  StepConsts<Acc> k;
  if constexpr (is_f32x2<Acc>::value) {
    k.theta_s = f32x2(theta_s);
    k.theta_d = f32x2(theta_d);
    k.var_init = f32x2(var_init);
    k.ts_vf = f32x2(theta_s * var_floor);
    k.td_mf = f32x2(theta_d * mask_floor);
  } else {
    k.theta_s = Acc(theta_s);
    k.theta_d = Acc(theta_d);
    k.var_init = Acc(var_init);
    k.ts_vf = k.theta_s * Acc(var_floor);
    k.td_mf = k.theta_d * Acc(mask_floor);
  }
  return k;
}

// blend u*a + w*b
__device__ __forceinline__ double blend(double u, double a, double w, double b) {
  return u * a + w * b;  // two roundings and a rounded sum (no contraction)
}
__device__ __forceinline__ float blend(float u, float a, float w, float b) {
  return __builtin_fmaf(u, a, w * b);
}

template <typename Acc>
struct Model {
  Acc mA, vA, mC, vC;
  int aA, aC;
};

// What one step decided, for the reverse sweep: the table slot used (the
// matched model's age, or RESET_SLOT), whether A matched, whether C was promoted,
// and d = (updated mean) - x of the blend.
template <typename Acc>
struct StepRecord {
  Acc d;
  int idx;
  bool hitA, hitC, swap, fg;
  // f32x2 only: the squared distances of the match tests and of the update
  // (d*d), which the background test reuses
  Acc qA, qC, V;
};

// True when the condition holds in any active lane of the wavefront.  Used to
// skip the rarely taken exchange as a whole: inside the branch every lane still
// applies it under its own condition, so results do not depend on the wavefront.
__device__ __forceinline__ bool any_lane(bool b) { return __builtin_amdgcn_ballot_w64(b) != 0; }

// The step in compensated single precision.  The frames are floats, so x is
// exact (x.lo = 0).  Same decisions and order as step_core() below, in the
// algebraically equal forms that need fewer pair operations:
//   m' = u*m + w*x = m + w*(x - m)     (u = 1 - w)
//   d  = m' - x    = -u*(x - m)
// with x - m taken from the match test, and the reset written as a select of
// (x, var_init) so that it stays exact.
__device__ __forceinline__ StepRecord<f32x2> step_core_x2(Model<f32x2>& s, const f32x2 xx,
                                                          const StepConsts<f32x2>& k,
                                                          const TableEntry<f32x2>* __restrict__ tbl) {
  using namespace x2;
  const float x = xx.hi;
  const f32x2 dA = sub(x, s.mA);
  const f32x2 qA = sqr(dA);
  const f32x2 dC = sub(x, s.mC);
  const f32x2 qC = sqr(dC);
  // both comparisons of each test are evaluated (no short circuit)
  const bool hA0 = lt(qA, mul(k.theta_s, s.vA)), hA1 = lt(qA, k.ts_vf);
  const bool hC0 = lt(qC, mul(k.theta_s, s.vC)), hC1 = lt(qC, k.ts_vf);
  const bool hitA = hA0 | hA1;
  const bool hitC = hC0 | hC1;
  const bool reset = !hitA && !hitC;

  const int idx = hitA ? s.aA : (hitC ? s.aC : RESET_SLOT);
  const f32x2 m = sel(hitA, s.mA, s.mC);
  const f32x2 v = sel(hitA, s.vA, s.vC);
  const f32x2 d0 = sel(hitA, dA, dC);
  const TableEntry<f32x2> e = tbl[idx];

  const f32x2 d = mul(f32x2(-e.u.hi, -e.u.lo), d0);  // 0 in the reset slot (u = 0)
  const f32x2 V = sqr(d);
  const f32x2 mn = sel(reset, f32x2(x), add(m, mul(e.w, d0)));
  const f32x2 vn = sel(reset, k.var_init, add(mul(e.u, v), mul(e.w, V)));
  const int an = e.next;

  s.mA = sel(hitA, mn, s.mA);
  s.vA = sel(hitA, vn, s.vA);
  s.aA = hitA ? an : s.aA;
  s.mC = sel(hitA, s.mC, mn);
  s.vC = sel(hitA, s.vC, vn);
  s.aC = hitA ? s.aC : an;

  StepRecord<f32x2> r;
  r.d = d;
  r.idx = idx;
  r.hitA = hitA;
  r.hitC = hitC && !hitA;
  r.swap = s.aC > s.aA;
  r.fg = false;
  r.qA = qA;
  r.qC = qC;
  r.V = V;
  return r;
}

// Match tests, update of the matched model and the exchange decision (not yet
// applied) for one frame of one pixel.  r.fg is left unset.
template <typename Acc>
__device__ __forceinline__ StepRecord<Acc> step_core(Model<Acc>& s, const Acc x,
                                                     const StepConsts<Acc>& k,
                                                     const TableEntry<Acc>* __restrict__ tbl) {
  if constexpr (is_f32x2<Acc>::value) {
    return step_core_x2(s, x, k, tbl);
  } else {
  // q < theta*max(v, f)  <=>  q < theta*v  or  q < theta*f  for theta >= 0:
  // rounding is monotone, so round(theta*max(v,f)) = max(round(theta*v),
  // round(theta*f)); the floor products are per-launch constants.
  const Acc dA = x - s.mA;
  const Acc qA = dA * dA;
  const Acc dC = x - s.mC;
  Acc qC = dC * dC;
  Acc tC = k.theta_s * s.vC;
  // With double state the empty asm makes both operands of the C test opaque,
  // so the compiler evaluates it in every lane instead of making it depend on
  // the A test; that schedule measured faster in the double backward (about
  // 8%) and equal in the double forward.
  if constexpr (sizeof(Acc) == 8) asm volatile("" : "+v"(qC), "+v"(tC));
  const bool hitA = (qA < k.theta_s * s.vA) | (qA < k.ts_vf);
  const bool hitC = (qC < tC) | (qC < k.ts_vf);

  const int idx = hitA ? s.aA : (hitC ? s.aC : RESET_SLOT);
  const Acc m = hitA ? s.mA : s.mC;
  const Acc v = hitA ? s.vA : s.vC;
  const TableEntry<Acc> e = tbl[idx];

  const Acc mn = blend(e.u, m, e.w, x);
  const Acc d = mn - x;
  const Acc V = d * d;
  const Acc vn = blend(e.u, v, e.w, V) + e.r;
  const int an = e.next;

  // the result replaces A if A matched, else C (update or reset)
  s.mA = hitA ? mn : s.mA;
  s.vA = hitA ? vn : s.vA;
  s.aA = hitA ? an : s.aA;
  s.mC = hitA ? s.mC : mn;
  s.vC = hitA ? s.vC : vn;
  s.aC = hitA ? s.aC : an;

  StepRecord<Acc> r;
  r.d = d;
  r.idx = idx;
  r.hitA = hitA;
  r.hitC = hitC && !hitA;
  r.swap = s.aC > s.aA;
  r.fg = false;
  r.qA = qA;
  r.V = V;
  return r;
  }
}

// The exchange: C older than A makes C the new A and resets C to (x, var_init, 1).
template <typename Acc>
__device__ __forceinline__ void apply_swap(Model<Acc>& s, const Acc x, const StepConsts<Acc>& k,
                                           const bool swap) {
  s.mA = swap ? s.mC : s.mA;
  s.vA = swap ? s.vC : s.vA;
  s.aA = swap ? s.aC : s.aA;
  s.mC = swap ? x : s.mC;
  s.vC = swap ? k.var_init : s.vC;
  s.aC = swap ? 1 : s.aC;
}

// The mask of the step (on the state after the exchange).  PRINTED selects the
// rule's reference: the intensity (as printed) or var_A.
template <typename Acc, bool PRINTED>
__device__ __forceinline__ bool fg_of(const Model<Acc>& s, const Acc x, const StepConsts<Acc>& k) {
  const Acc dd = s.mA - x;
  const Acc qd = dd * dd;
  const Acc ref = PRINTED ? x : s.vA;
  return !((qd <= k.theta_d * ref) | (qd <= k.td_mf));
}

// The squared distance (mA - x)^2 of the background test, taken from the
// step where it already formed it: mA after the step is the updated model if
// A matched (its d*d), else the untouched A (the A test's distance: x - mA is
// the exact negation of mA - x, so the square is the same number).  An
// exchange changes mA; mask_dist_swapped() then gives the promoted model's.
template <typename Acc>
__device__ __forceinline__ Acc mask_dist(const StepRecord<Acc>& r) {
  if constexpr (is_f32x2<Acc>::value)
    return x2::sel(r.hitA, r.V, r.qA);
  else
    return r.hitA ? r.V : r.qA;
}

// after an exchange (swap true): mA is the promoted C, updated (d*d) if C
// matched; if A matched (possible only from a state whose C was older than A),
// the untouched C (its test distance)
template <typename Acc>
__device__ __forceinline__ Acc mask_dist_swapped(const StepRecord<Acc>& r, const Model<Acc>& s,
                                                 const Acc x, const Acc qd) {
  if constexpr (is_f32x2<Acc>::value) {
    return x2::sel(r.swap, x2::sel(r.hitA, r.qC, r.V), qd);
  } else {
    const Acc dd = s.mA - x;
    return r.swap ? dd * dd : qd;
  }
}

// The mask from the step's squared distance qd = (mA - x)^2 and the state
// after the exchange.
template <typename Acc, bool PRINTED>
__device__ __forceinline__ bool fg_from(const Acc qd, const Model<Acc>& s, const Acc x,
                                        const StepConsts<Acc>& k) {
  if constexpr (is_f32x2<Acc>::value) {
    using namespace x2;
    const f32x2 ref = PRINTED ? x : s.vA;
    const bool b0 = le(qd, mul(k.theta_d, ref)), b1 = le(qd, k.td_mf);
    return !(b0 | b1);
  } else {
    const Acc ref = PRINTED ? x : s.vA;
    return !((qd <= k.theta_d * ref) | (qd <= k.td_mf));
  }
}

// The mask of the step given its record (on the state after the exchange).
template <typename Acc, bool PRINTED>
__device__ __forceinline__ bool fg_of(const Model<Acc>& s, const Acc x, const StepConsts<Acc>& k,
                                      const StepRecord<Acc>& r) {
  const Acc qd = mask_dist_swapped<Acc>(r, s, x, mask_dist<Acc>(r));
  return fg_from<Acc, PRINTED>(qd, s, x, k);
}

// One whole frame of one pixel (state updated in place).
template <typename Acc, bool PRINTED>
__device__ __forceinline__ StepRecord<Acc> step_rec(Model<Acc>& s, const Acc x,
                                                    const StepConsts<Acc>& k,
                                                    const TableEntry<Acc>* __restrict__ tbl) {
  StepRecord<Acc> r = step_core<Acc>(s, x, k, tbl);
  if (any_lane(r.swap)) apply_swap<Acc>(s, x, k, r.swap);
  r.fg = fg_of<Acc, PRINTED>(s, x, k, r);
  return r;
}

// The decision code of a step (CODE_* bits).
template <typename Acc>
__device__ __forceinline__ unsigned code_of(const StepRecord<Acc>& r) {
  return (r.hitA ? CODE_HIT_A : (r.hitC ? CODE_HIT_C : CODE_RESET)) | (r.swap ? CODE_SWAP : 0u) |
         (r.fg ? CODE_FG : 0u);
}

// Adjoint of one step, decisions fixed (the chain rule through step_rec):
//   bg = mA after the step           gmA += gbg
//   swap: A <- C, C <- (x, var_init) gx += gmC, gvi += gvC, (gmC, gvC) <- (gmA, gvA), A's = 0
//   blend of the matched model M (with the reset as the slot u = 0, w = 1, d = 0):
//     gV = w*gv, gd = 2*d*gV, gmn = gm + gd, gx += w*gmn - gd, gv <- u*gv, gm <- u*gmn
//   reset slot: var_init enters the new variance with slope 1: gvi += gv
// The operation order is that of a scalar FP64 evaluation, so with Acc = double
// the per-element results are bit-identical to it.
template <typename Acc>
struct Adjoint {
  Acc gmA, gvA, gmC, gvC;
  double gvi;  // this pixel's contribution to d/d(var_init), in FP64
};

template <typename Acc, bool HAS_GBG>
__device__ __forceinline__ Acc reverse_step(Adjoint<Acc>& g, const Acc gbg, const Acc d,
                                            const int idx, const bool hitA, const bool swap,
                                            const TableEntry<Acc>* __restrict__ tbl) {
  if (HAS_GBG) g.gmA = g.gmA + gbg;
  Acc gx = Acc(0);
  if (any_lane(swap)) {
    gx = swap ? gx + g.gmC : gx;
    g.gvi = swap ? g.gvi + double(g.gvC) : g.gvi;
    g.gmC = swap ? g.gmA : g.gmC;
    g.gvC = swap ? g.gvA : g.gvC;
    g.gmA = swap ? Acc(0) : g.gmA;
    g.gvA = swap ? Acc(0) : g.gvA;
  }
  const TableEntry<Acc> e = tbl[idx];
  const Acc gm = hitA ? g.gmA : g.gmC;
  const Acc gv = hitA ? g.gvA : g.gvC;
  const Acc gV = e.w * gv;
  const Acc gd = (Acc(2) * d) * gV;
  const Acc gmn = gm + gd;
  gx = gx + (e.w * gmn - gd);
  const Acc gvn = e.u * gv;
  const Acc gmo = e.u * gmn;
  if (idx == RESET_SLOT) g.gvi += double(gv);
  g.gmA = hitA ? gmo : g.gmA;
  g.gvA = hitA ? gvn : g.gvA;
  g.gmC = hitA ? g.gmC : gmo;
  g.gvC = hitA ? g.gvC : gvn;
  return gx;
}

// ---------------------------------------------------------------- storage types
struct bf16_t {
  uint16_t bits;
};

template <typename In, typename Acc>
__device__ __forceinline__ Acc to_acc(In v) {
  return Acc(v);
}
template <>
__device__ __forceinline__ float to_acc<bf16_t, float>(bf16_t v) {
  return __uint_as_float(uint32_t(v.bits) << 16);
}
template <>
__device__ __forceinline__ double to_acc<bf16_t, double>(bf16_t v) {
  return double(__uint_as_float(uint32_t(v.bits) << 16));
}
template <>
__device__ __forceinline__ f32x2 to_acc<bf16_t, f32x2>(bf16_t v) {
  return f32x2(__uint_as_float(uint32_t(v.bits) << 16));
}

// P consecutive elements, aligned to their total size so that the compiler
// emits the widest loads and stores the alignment allows.
template <typename X, int P>
struct alignas(sizeof(X) * P) Vec {
  X v[P];
};

}  // namespace dsgm
