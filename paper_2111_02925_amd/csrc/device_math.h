// Per-point arithmetic of the compressor on the device: interpolation
// stencils, the linear-scaling quantizer and its inverse.
//
// Paper: SZ3 (arXiv 2111.02925).  Section 6.2 (SZ3-Interp: linear and cubic
// interpolation with constant coefficients, from reconstructed points);
// Section 3.2 "Quantizer" (equal bins of width 2*eb, the code is the bin of
// the prediction error, out-of-range errors are unpredictable and stored
// separately); Appendix A.3 (quantize / recover).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace szg {

__device__ __forceinline__ float fabs_t(float v) { return __builtin_fabsf(v); }
__device__ __forceinline__ double fabs_t(double v) { return __builtin_fabs(v); }
__device__ __forceinline__ float rint_t(float v) { return __builtin_rintf(v); }
__device__ __forceinline__ double rint_t(double v) { return __builtin_rint(v); }
__device__ __forceinline__ bool finite_t(float v) { return __builtin_isfinite(v); }
__device__ __forceinline__ bool finite_t(double v) { return __builtin_isfinite(v); }

template <typename T>
struct QuantParams {
  T eb, twoeb, inv2eb;
  uint32_t R;
  __device__ static QuantParams from_meta(const Meta* m, uint32_t R) {
    QuantParams q;
    q.eb = (T)m->eb;  // exact: the stored doubles hold T values
    q.twoeb = (T)m->twoeb;
    q.inv2eb = (T)m->inv2eb;
    q.R = R;
    return q;
  }
};

// Exact test of |x - r| <= eb.  s = fl(x - r) decides every case but
// |s| == eb (rounding is monotone and eb is representable); there the sign of
// the subtraction's rounding error, recovered exactly by the TwoSum
// error-free transformation, decides.
template <typename T>
__device__ __forceinline__ bool bound_tie(T x, T r, T s) {
  const T y = -r;
  const T sum_minus_y = s - y;
  const T y_part = s - sum_minus_y;
  const T err = (x - sum_minus_y) + (y - y_part);
  // |x - r| < |s| exactly when the rounding error is zero or of the other
  // sign (combined as integers: no short-circuit branch)
  const uint32_t zero = err == T(0) ? 1u : 0u;
  const uint32_t neg_err = err < T(0) ? 1u : 0u, neg_s = s < T(0) ? 1u : 0u;
  return (zero | (neg_err ^ neg_s)) != 0u;
}
template <typename T>
__device__ __forceinline__ bool bound_holds(T x, T r, T eb) {
  const T s = x - r;
  const T as = fabs_t(s);
  bool holds = as < eb;
  // the tie with the bound is rare: lanes take the exact test only then
  if (as == eb) holds = bound_tie(x, r, s);
  return holds;
}

// Linear-scaling quantizer.  k = rint(|x - pred| / (2 eb)) (multiplied by the
// precomputed reciprocal), signed like the error; the code is R + k when
// |k| < R and the reconstruction pred + 2eb*k meets the bound, else 0
// (unpredictable: the reconstruction is x itself).  eb == 0 codes only exact
// predictions.  The signed k is rounded directly from the signed product:
// multiplication and round-half-even are symmetric in the sign, so this is
// the same integer.  Written with selects rather than branches (the tie case
// of the bound test aside), so that a wavefront does not diverge on it.
template <typename T>
__device__ __forceinline__ uint32_t quantize(T x, T pred, const QuantParams<T>& q, T& rec) {
  const T diff = x - pred;
  if (q.eb == T(0)) {  // the same for every point
    const bool exact = diff == T(0);
    rec = exact ? pred + q.twoeb * T(0) : x;
    return exact ? q.R : 0u;
  }
  const T kf = rint_t(diff * q.inv2eb);
  const bool in_range = fabs_t(kf) < (T)q.R;  // false for NaN
  // k stays in T: an integer below R in magnitude, exact in T, so R + k is
  // too and converts to the code exactly (one conversion instead of two);
  // + 0 turns a rounded -0 into the +0 that an integer k would give
  const T k = in_range ? kf + T(0) : T(0);
  const T r = pred + q.twoeb * k;
  const bool holds = bound_holds(x, r, q.eb);  // evaluated for every lane: no branch on in_range
  const bool ok = in_range & holds;
  rec = ok ? r : x;
  return ok ? (uint32_t)(k + (T)q.R) : 0u;
}

template <typename T>
__device__ __forceinline__ T recover(T pred, T twoeb, uint32_t code, uint32_t R) {
  return pred + twoeb * (T)((int)code - (int)R);
}

// Interpolation at a point i along one dimension from a = v(i-3s), b = v(i-s),
// c = v(i+s), e = v(i+3s) (flags say which exist).  Linear: midpoint; at the
// high edge the line through (i-3s, i-s); with b alone, b.  Cubic: 4-point
// Lagrange midpoint weights (-1, 9, 9, -1)/16; with one outer point missing
// the quadratic through the three others; with both missing the midpoint; at
// the high edge the linear rules.
template <typename T, int PRED>
__device__ __forceinline__ T interp_predict(T a, T b, T c, T e, bool has_a, bool has_c,
                                            bool has_e) {
  if (!has_c) return has_a ? (T(3) * b - a) * T(0.5) : b;
  if (PRED == SZ_INTERP_LINEAR) return (b + c) * T(0.5);
  if (has_a && has_e) return (T(9) * (b + c) - (a + e)) * T(0.0625);
  if (has_e) return ((T(3) * b + T(6) * c) - e) * T(0.125);
  if (has_a) return ((T(6) * b + T(3) * c) - a) * T(0.125);
  return (b + c) * T(0.5);
}

// The same prediction with every rule evaluated and the right one selected
// (no branches; each rule's operations and order are those above, so the
// selected value is bitwise the same).  Operands of rules that do not apply
// may hold any value.
template <typename T, int PRED>
__device__ __forceinline__ T interp_predict_sel(T a, T b, T c, T e, bool has_a, bool has_c,
                                                bool has_e) {
  const T one_sided = has_a ? (T(3) * b - a) * T(0.5) : b;
  const T mid = (b + c) * T(0.5);
  if (PRED == SZ_INTERP_LINEAR) return has_c ? mid : one_sided;
  const T four = (T(9) * (b + c) - (a + e)) * T(0.0625);
  const T quad_e = ((T(3) * b + T(6) * c) - e) * T(0.125);
  const T quad_a = ((T(6) * b + T(3) * c) - a) * T(0.125);
  const T two_sided = has_a ? (has_e ? four : quad_a) : (has_e ? quad_e : mid);
  return has_c ? two_sided : one_sided;
}

}  // namespace szg
