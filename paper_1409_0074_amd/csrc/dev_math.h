// Device arithmetic shared by the kernels of the local GP library.
//
// Rounding is pinned down operation by operation (the library is compiled
// with -ffp-contract=off, so nothing is fused unless written as fma):
//  * squared distance: terms accumulated in dimension order from 0.0, one
//    fused multiply-add per dimension;
//  * every inner product that feeds the local inverse, the ray objective or
//    the prediction: terms accumulated in index order from 0.0 with one fused
//    multiply-add each;
//  * exp: Cody-Waite reduction by ln2 and a degree-13 Taylor polynomial
//    (below), results under 2^-1022 flushed to zero;
//  * division and square root: IEEE (gfx950 f64 div/sqrt are correctly
//    rounded).
// With these definitions the kernel values, the partitioned-inverse updates,
// the ray line searches and the final mean and scale are reproducible bit
// for bit by any IEEE implementation of the same steps.  Only the candidate
// scoring contraction (MFMA) sums in a different order.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lagp {

// Taylor coefficients of exp in Horner order: 1/m! for m = 13 .. 2 (i = 0 ..
// 11), each the correctly rounded quotient of exact integers.
__host__ __device__ constexpr double gexp_coef(int i) {
  switch (i) {
    case 0: return 1.0 / 6227020800.0;
    case 1: return 1.0 / 479001600.0;
    case 2: return 1.0 / 39916800.0;
    case 3: return 1.0 / 3628800.0;
    case 4: return 1.0 / 362880.0;
    case 5: return 1.0 / 40320.0;
    case 6: return 1.0 / 5040.0;
    case 7: return 1.0 / 720.0;
    case 8: return 1.0 / 120.0;
    case 9: return 1.0 / 24.0;
    case 10: return 1.0 / 6.0;
    default: return 0.5;
  }
}

// exp(x) = 2^k exp(r), k = rint(x / ln2), r = x - k ln2 computed with ln2 as
// the double nearest to it plus the remainder (two fused multiply-adds);
// exp(r), |r| <= ln2/2, by its Taylor polynomial to degree 13 in Horner form
// (truncation below 1e-17 relative).  Faithful (< 1 ulp) on [-708, 709].
// coef(i) supplies gexp_coef(i); a kernel short of registers may read the
// same values from LDS instead of holding them as constants.
template <class Coef>
__device__ __forceinline__ double gexp_with(double x, const Coef& coef) {
  // straight-line: the out-of-range cases are selected at the end (no
  // divergent branches around the polynomial)
  const double xc = x < -708.0 ? -708.0 : (x > 709.0 ? 709.0 : (x == x ? x : 0.0));
  const double L2H = 0x1.62e42fefa39efp-1;   // double nearest ln 2
  const double L2L = 0x1.abc9e3b39803fp-56;  // ln 2 - L2H
  const double IL2 = 0x1.71547652b82fep+0;   // double nearest 1/ln 2
  const double k = __builtin_rint(xc * IL2);
  double r = __builtin_fma(-k, L2H, xc);
  r = __builtin_fma(-k, L2L, r);
  double t = coef(0);
#pragma unroll
  for (int i = 1; i < 12; ++i) t = __builtin_fma(t, r, coef(i));
  t = __builtin_fma(t, r, 1.0);
  t = __builtin_fma(t, r, 1.0);
  const double e = __builtin_ldexp(t, (int)k);
  if (x != x) return x;
  return x < -708.0 ? 0.0 : (x > 709.0 ? __builtin_huge_val() : e);
}

// gexp_with on U arguments in lockstep: the same operations on each (the
// same values), interleaved so that the U dependent chains overlap.
// coef(i) supplies gexp_coef(i) as in gexp_with.
template <int U, class Coef>
__device__ __forceinline__ void gexp_lockstep_with(double (&x)[U], const Coef& coef) {
  const double L2H = 0x1.62e42fefa39efp-1;
  const double L2L = 0x1.abc9e3b39803fp-56;
  const double IL2 = 0x1.71547652b82fep+0;
  double xc[U], k[U], r[U], t[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    // (in range: x itself; outside it, and for NaN, the polynomial's value
    // is replaced below, so the clamp only keeps the scaling finite)
    xc[u] = __builtin_fmax(__builtin_fmin(x[u], 709.0), -708.0);
    k[u] = __builtin_rint(xc[u] * IL2);
  }
#pragma unroll
  for (int u = 0; u < U; ++u) r[u] = __builtin_fma(-k[u], L2H, xc[u]);
#pragma unroll
  for (int u = 0; u < U; ++u) {
    r[u] = __builtin_fma(-k[u], L2L, r[u]);
    t[u] = coef(0);
  }
#pragma unroll
  for (int i = 1; i < 12; ++i) {
    const double ci = coef(i);
#pragma unroll
    for (int u = 0; u < U; ++u) t[u] = __builtin_fma(t[u], r[u], ci);
  }
#pragma unroll
  for (int u = 0; u < U; ++u) t[u] = __builtin_fma(t[u], r[u], 1.0);
#pragma unroll
  for (int u = 0; u < U; ++u) t[u] = __builtin_fma(t[u], r[u], 1.0);
  // the final choice as arithmetic, so that the polynomial is always used
  // (no branch around it): fma(e, 1, 0) = e in range; fma(e, 0, c) = c with
  // c = 0 below it, +inf above it and x itself for NaN (e is finite)
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const double e = __builtin_ldexp(t[u], (int)k[u]);
    const bool in = x[u] >= -708.0 && x[u] <= 709.0;
    const double c = x[u] != x[u] ? x[u] : (x[u] > 709.0 ? __builtin_huge_val() : 0.0);
    x[u] = __builtin_fma(e, in ? 1.0 : 0.0, c);
  }
}

template <int U>
__device__ __forceinline__ void gexp_lockstep(double (&x)[U]) {
  gexp_lockstep_with(x, gexp_coef);
}

__device__ __forceinline__ void gexp4(double (&x)[4]) { gexp_lockstep<4>(x); }

// The same function with the out-of-range cases as early returns and the
// coefficients as constants (the form the partitioned-inverse kernels were
// tuned with; identical values).
__device__ __forceinline__ double gexp(double x) {
  if (x != x) return x;
  if (x < -708.0) return 0.0;
  if (x > 709.0) return __builtin_huge_val();
  const double L2H = 0x1.62e42fefa39efp-1;
  const double L2L = 0x1.abc9e3b39803fp-56;
  const double IL2 = 0x1.71547652b82fep+0;
  const double k = __builtin_rint(x * IL2);
  double r = __builtin_fma(-k, L2H, x);
  r = __builtin_fma(-k, L2L, r);
  double t = gexp_coef(0);
#pragma unroll
  for (int i = 1; i < 12; ++i) t = __builtin_fma(t, r, gexp_coef(i));
  t = __builtin_fma(t, r, 1.0);
  t = __builtin_fma(t, r, 1.0);
  return __builtin_ldexp(t, (int)k);
}

// Squared Euclidean distance with one fma per dimension, in order.
__device__ __forceinline__ double sqdist(const double* a, const double* b, int p) {
  double s = 0.0;
  for (int k = 0; k < p; ++k) {
    const double t = a[k] - b[k];
    s = __builtin_fma(t, t, s);
  }
  return s;
}

// Gaussian correlation exp(-sum_k (a_k-b_k)^2/d_k) from the reciprocal
// lengthscales w_k = 1/d_k: one value (isotropic, dlen == 1) gives
// exp(-(r^2 w)), one per dimension (separable) accumulates
// s <- fma(t_k t_k, w_k, s).  No nugget.
__device__ __forceinline__ double corr(const double* a, const double* b, int p, const double* w, int dlen) {
  if (dlen == 1) return gexp(-(sqdist(a, b, p) * w[0]));
  double s = 0.0;
  for (int k = 0; k < p; ++k) {
    const double t = a[k] - b[k];
    s = __builtin_fma(t * t, w[k], s);
  }
  return gexp(-s);
}

// The same with the isotropic reciprocal lengthscale passed by value (a
// location's own, or w[0]); the separable case reads w.
__device__ __forceinline__ double corr(const double* a, const double* b, int p, double w0, const double* w,
                                       int dlen) {
  if (dlen == 1) return gexp(-(sqdist(a, b, p) * w0));
  double s = 0.0;
  for (int k = 0; k < p; ++k) {
    const double t = a[k] - b[k];
    s = __builtin_fma(t * t, w[k], s);
  }
  return gexp(-s);
}

// (d2, row) strict order used for the nearest-candidate lists.
__device__ __forceinline__ bool key_less(double da, int ia, double db, int ib) {
  return da < db || (da == db && ia < ib);
}

}  // namespace lagp
