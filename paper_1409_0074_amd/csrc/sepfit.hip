// Global separable lengthscales from a subset of the design, and the
// pre-scaling of inputs by their square roots (Sec. 5.3: local designs
// searched on inputs divided by the square roots of global lengthscales
// estimated on data subsets).
//
// The likelihood is the local one's (Eq. gpk, nugget g fixed) on the n
// subset points with the separable kernel
//   K_ij = exp(-sum_q (x_iq - x_jq)^2 w_q) + g [i = j],  w_q = 1/theta_q,
// the exponent summed in q order with one fused multiply-add per term.  In
// theta_k, with a_ij = (x_ik - x_jk)^2 w_k and E_ij = K_ij - g [i = j]:
//   dK/dtheta_k = E a w_k,  d2K/dtheta_k^2 = E (a^2 - 2a) w_k^2,
// and l', l'' follow as for the isotropic local fit (mle.hip).  The
// maximisation runs one coordinate at a time: a sweep takes k = 0..p-1 in
// turn and runs the bracketed Newton iteration of the local fit on theta_k
// with the others fixed; sweeps repeat until one moves no theta_k by more
// than tol theta_k, or maxsweep sweeps.  Every sum runs in index order from
// 0.0 with one fused multiply-add per term, so the estimates are reproducible
// bit for bit by any IEEE implementation of the same steps.
//
// One workgroup of 1024 threads runs the whole fit; the n x n matrices live
// in a global-memory workspace (3 n^2 + 7 n doubles), the factor's current
// column and row of its inverse in LDS.
#include "dev_math.h"
#include "exact_gemm.h"
#include "lagp_internal.h"

namespace lagp {

namespace {

constexpr int SEP_THREADS = 1024;

struct SepShared {
  double colm[SEP_NMAX];  // column m of the factor, below the diagonal
  double rowm[SEP_NMAX];  // row m of the factor's inverse
  double th[LAGP_MAX_DIM];
  double w[LAGP_MAX_DIM];
  double sc[12];
};

struct SepView {
  const double* XS;
  const double* y;
  int n, p;
  double g;
  double *E, *A, *B;  // n x n: exp(-s); K, its factor, then K^{-1}; L^{-1}, then K^{-1} dK
  double *al, *be, *ga, *de, *r;
};

// dK/dtheta_k and d2K/dtheta_k^2 at (i, j), from E and the coordinates.
__device__ __forceinline__ double sep_kd(const SepView& v, int i, int j, int k, double wk) {
  const double t = v.XS[i * v.p + k] - v.XS[j * v.p + k];
  const double a = (t * t) * wk;
  return (v.E[i * v.n + j] * a) * wk;
}
__device__ __forceinline__ double sep_kdd(const SepView& v, int i, int j, int k, double wk) {
  const double t = v.XS[i * v.p + k] - v.XS[j * v.p + k];
  const double a = (t * t) * wk;
  return (v.E[i * v.n + j] * (a * a - 2.0 * a)) * (wk * wk);
}

__device__ __forceinline__ double sep_dot(const double* a, const double* b, int n) {
  double s = 0.0;
  for (int k = 0; k < n; ++k) s = __builtin_fma(a[k], b[k], s);
  return s;
}

// Cholesky factor of K (in A, lower triangle) fused with the inverse of the
// factor (B, which holds the identity on entry), right-looking: step m takes
// the pivot sqrt(s_mm), divides column m of L and row m of L^{-1} by it
// (copies of both in LDS), then subtracts L_im L_km from every trailing
// s_ik (m < k <= i) and L_im (L^{-1})_mc from every (i, c) with c <= m.
// Every element receives the terms of its defining sum in ascending m, one
// fused multiply-add each: the column-by-column algorithm's values.
__device__ bool sep_cholesky(const SepView& v, SepShared& S) {
  const int n = v.n, tid = threadIdx.x, T = blockDim.x;
  const int lane = tid & 63, wv = tid >> 6, nw = T >> 6;
  double *A = v.A, *B = v.B;
  for (int m = 0; m < n; ++m) {
    const double smm = A[m * n + m];
    if (!(smm > 0.0)) return false;  // (every thread reads the same value)
    const double piv = __builtin_sqrt(smm);
    const int nl = n - m - 1, nr = m + 1;
    for (int t = tid; t < nl + nr; t += T) {
      if (t < nl) {
        const int i = m + 1 + t;
        const double x = A[i * n + m] / piv;
        A[i * n + m] = x;
        S.colm[i] = x;
      } else {
        const int c = t - nl;
        const double x = B[m * n + c] / piv;
        B[m * n + c] = x;
        S.rowm[c] = x;
      }
    }
    __syncthreads();
    for (int rr = wv; rr < nl; rr += nw) {  // one row per wave, lanes along it
      const int i = m + 1 + rr;
      const double lim = S.colm[i];
      const int width = rr + 1 + nr;  // columns m+1..i of L, then 0..m of L^{-1}
      for (int q = lane; q < width; q += 64) {
        if (q <= rr) {
          const int k = m + 1 + q;
          A[i * n + k] = __builtin_fma(-lim, S.colm[k], A[i * n + k]);
        } else {
          const int c = q - rr - 1;
          B[i * n + c] = __builtin_fma(-lim, S.rowm[c], B[i * n + c]);
        }
      }
    }
    __syncthreads();
  }
  return true;
}

// l' and l'' in theta_k at the lengthscales in S.th (all threads; results in
// S.sc[0], S.sc[1]; false if K is not positive definite).
__device__ bool sep_eval(const SepView& v, SepShared& S, int k) {
  const int n = v.n, p = v.p, tid = threadIdx.x, T = blockDim.x;
  if (tid < p) S.w[tid] = 1.0 / S.th[tid];
  __syncthreads();
  for (int t = tid; t < n * n; t += T) {
    const int i = t / n, j = t - i * n;
    double s = 0.0;
    for (int q = 0; q < p; ++q) {
      const double d = v.XS[i * p + q] - v.XS[j * p + q];
      s = __builtin_fma(d * d, S.w[q], s);
    }
    const double e = gexp(-s);
    v.E[t] = e;
    v.A[t] = e + (i == j ? v.g : 0.0);
    v.B[t] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  if (!sep_cholesky(v, S)) return false;
  // K^{-1} = L^{-T} L^{-1} over the factor (the terms below max(i, j) are
  // exact zeros of the lower triangular L^{-1})
  {
    const double* Li = v.B;
    double* Ki = v.A;
    exact_gemm(
        n, [=](int i, int q) { return Li[q * n + i]; }, [=](int q, int j) { return Li[q * n + j]; },
        [=](int i, int j, double x) { Ki[i * n + j] = x; });
  }
  __syncthreads();
  const double* Ki = v.A;
  const double wk = S.w[k];
  for (int i = tid; i < n; i += T) v.al[i] = sep_dot(Ki + i * n, v.y, n);
  __syncthreads();
  for (int i = tid; i < n; i += T) {
    double b = 0.0, d = 0.0;
    for (int j = 0; j < n; ++j) {
      b = __builtin_fma(sep_kd(v, i, j, k, wk), v.al[j], b);
      d = __builtin_fma(sep_kdd(v, i, j, k, wk), v.al[j], d);
    }
    v.be[i] = b;
    v.de[i] = d;
  }
  __syncthreads();
  for (int i = tid; i < n; i += T) v.ga[i] = sep_dot(Ki + i * n, v.be, n);
  {  // P = K^{-1} dK/dtheta_k over L^{-1}, which is no longer needed
    double* P = v.B;
    const SepView vv = v;
    exact_gemm(
        n, [=](int i, int q) { return Ki[i * n + q]; }, [=](int q, int j) { return sep_kd(vv, q, j, k, wk); },
        [=](int i, int j, double x) { P[i * n + j] = x; });
  }
  __syncthreads();
  for (int i = tid; i < n; i += T) {
    double r1 = 0.0, r2 = 0.0, r3 = 0.0;
    for (int j = 0; j < n; ++j) {
      const double kij = Ki[i * n + j];
      r1 = __builtin_fma(kij, sep_kd(v, j, i, k, wk), r1);
      r2 = __builtin_fma(kij, sep_kdd(v, j, i, k, wk), r2);
      r3 = __builtin_fma(v.B[i * n + j], v.B[j * n + i], r3);
    }
    v.r[i] = r1;
    v.r[n + i] = r2;
    v.r[2 * n + i] = r3;
  }
  __syncthreads();
  {  // the seven scalar sums, each one in-order chain, on lanes of different waves
    const int job = (tid & 63) == 0 ? tid >> 6 : -1;
    if (job >= 0 && job < 7) {
      double x = 0.0;
      if (job == 0) x = sep_dot(v.y, v.al, n);   // psi
      if (job == 1) x = sep_dot(v.al, v.be, n);  // alpha^T Kd alpha
      if (job == 2) x = sep_dot(v.be, v.ga, n);  // beta^T K^{-1} beta
      if (job == 3) x = sep_dot(v.al, v.de, n);  // alpha^T Kdd alpha
      if (job >= 4) {
        const double* rr = v.r + (job - 4) * n;  // the traces: in-order sums of the row sums
        for (int i = 0; i < n; ++i) x = x + rr[i];
      }
      S.sc[2 + job] = x;
    }
  }
  __syncthreads();
  if (tid == 0) {
    const double psi = S.sc[2], ab = S.sc[3], bgb = S.sc[4], add = S.sc[5];
    const double t1 = S.sc[6], t2 = S.sc[7], t3 = S.sc[8];
    const double hn = 0.5 * (double)n;
    const double q = ab / psi;
    S.sc[0] = -0.5 * t1 + hn * q;
    S.sc[1] = -0.5 * (t2 - t3) + hn * ((add - 2.0 * bgb) / psi + q * q);
  }
  __syncthreads();
  return true;
}

__global__ __launch_bounds__(SEP_THREADS) void k_sepfit(SepArgs a) {
  __shared__ SepShared S;
  const int n = a.n, p = a.p, tid = threadIdx.x;
  SepView v;
  v.XS = a.XS;
  v.y = a.y;
  v.n = n;
  v.p = p;
  v.g = a.g;
  v.E = a.ws;
  v.A = v.E + (size_t)n * n;
  v.B = v.A + (size_t)n * n;
  v.al = v.B + (size_t)n * n;
  v.be = v.al + n;
  v.ga = v.be + n;
  v.de = v.ga + n;
  v.r = v.de + n;
  if (tid < p) S.th[tid] = a.theta[tid];
  __syncthreads();
  // every thread takes the same decisions from the same values
  int flags = 0, total = 0;
  bool conv = false;
  for (int sweep = 0; sweep < a.maxsweep && !conv; ++sweep) {
    bool moved = false;
    for (int k = 0; k < p; ++k) {
      const double before = S.th[k];
      double lo = a.dmin, hi = a.dmax;
      double theta = before < lo ? lo : (before > hi ? hi : before);
      int it = 0, fl = 0;
      bool cc = false;
      while (it < a.maxit) {
        __syncthreads();  // every thread has read th and sc
        if (tid == 0) S.th[k] = theta;
        __syncthreads();
        const bool ok = sep_eval(v, S, k);
        ++it;
        double d1 = -1.0, d2 = 0.0;
        if (ok) {
          d1 = S.sc[0];
          d2 = S.sc[1];
        } else {
          fl |= LAGP_STATUS_MLE_NOTPD;
        }
        if (d1 == 0.0) {
          cc = true;
          break;
        }
        if (d1 > 0.0)
          lo = theta;
        else
          hi = theta;
        double tn = (d2 < 0.0) ? theta - d1 / d2 : lo;
        if (!(tn > lo && tn < hi)) tn = __builtin_sqrt(lo * hi);
        const bool done = fabs(tn - theta) <= a.tol * theta;
        theta = tn;
        if (done) {
          cc = true;
          break;
        }
      }
      if (!cc) fl |= LAGP_STATUS_MLE_MAXIT;
      __syncthreads();
      if (tid == 0) S.th[k] = theta;
      __syncthreads();
      total += it;
      flags |= fl;
      if (fabs(theta - before) > a.tol * before) moved = true;
    }
    if (!moved) conv = true;
  }
  if (!conv) flags |= LAGP_STATUS_MLE_MAXIT;
  for (int k = 0; k < p; ++k)
    if (S.th[k] <= a.dmin * (1.0 + a.tol) || S.th[k] >= a.dmax * (1.0 - a.tol)) flags |= LAGP_STATUS_MLE_BOUND;
  if (tid < p) a.theta[tid] = S.th[tid];
  if (tid == 0) {
    *a.iters = total;
    *a.flags = flags;
  }
}

// out[i][k] = X[i][k] / sqrt(theta_k), one element per thread.
__global__ void k_prescale(const double* X, int64_t N, int p, PrescaleScales sc, double* out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N * p) return;
  const int k = (int)(t % p);
  out[t] = X[t] / __builtin_sqrt(sc.theta[k]);
}

}  // namespace

size_t sepfit_workspace_bytes(int n) { return sizeof(double) * (3 * (size_t)n * n + 7 * (size_t)n); }

hipError_t launch_sepfit(const SepArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_sepfit, dim3(1), dim3(SEP_THREADS), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_prescale(const double* X, int64_t N, int p, const double* theta, double* out, hipStream_t s) {
  if (N <= 0) return hipSuccess;
  PrescaleScales sc{};
  for (int k = 0; k < p; ++k) sc.theta[k] = theta[k];
  const int64_t total = N * p;
  const unsigned blocks = (unsigned)((total + 255) / 256);
  hipLaunchKernelGGL(k_prescale, dim3(blocks), dim3(256), 0, s, X, N, p, sc, out);
  return hipGetLastError();
}

}  // namespace lagp
