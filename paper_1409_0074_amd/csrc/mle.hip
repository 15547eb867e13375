// Local maximum likelihood of an isotropic lengthscale on each location's
// local design, and the prediction under the estimate (one workgroup per
// location).
//
// The local log-likelihood (Eq. gpk with the n local points, nugget g fixed)
//   l(theta) = -1/2 log|K| - n/2 log psi,  psi = y^T K^{-1} y,
//   K = E + g I,  E_ik = exp(-a_ik),  a_ik = D_ik w,  w = 1/theta,
// has, with Kd = dK/dtheta = E a w, Kdd = d2K/dtheta2 = E (a^2 - 2a) w^2,
// alpha = K^{-1} y and beta = Kd alpha,
//   l'  = -1/2 tr(K^{-1} Kd) + n/2 (alpha^T beta) / psi
//   l'' = -1/2 [tr(K^{-1} Kdd) - tr(K^{-1} Kd K^{-1} Kd)]
//         + n/2 [(alpha^T Kdd alpha - 2 beta^T K^{-1} beta) / psi + ((alpha^T beta) / psi)^2].
// Newton's method on l' = 0 runs inside a bracket [lo, hi] that starts at
// [dmin, dmax]: an iterate with l' > 0 raises lo, otherwise it lowers hi; the
// Newton step is taken when l'' < 0 and it lands strictly inside the
// bracket, else the geometric midpoint sqrt(lo hi); a K that is not positive
// definite counts as l' < 0.  The iteration stops when a step moves theta by
// at most tol theta (or l' = 0) or after maxit evaluations.  The prediction at
// the estimate goes through the Cholesky factor: w = L^{-1} k_x,
// z = L^{-1} y, mean = w^T z, scale psi ((1+g) - w^T w) / n with psi = z^T z.
//
// Every sum runs in index order from 0.0 with one fused multiply-add per
// term, a trace is the in-order sum of its row sums, and K^{-1} comes from
// the Cholesky factor as L^{-T} L^{-1}, so the estimates and predictions are
// reproducible bit for bit by any IEEE implementation of the same steps.
#include "dev_math.h"
#include "exact_gemm.h"
#include "lagp_internal.h"

namespace lagp {

namespace {

constexpr int MLE_THREADS = 256;
constexpr int MLE_NMAX_LDS = 50;  // designs whose matrices stay in LDS (two workgroups per CU)
static_assert(MLE_THREADS == 256, "the per-row loops deal rows to exactly 4 waves");
static_assert(LAGP_MAX_N <= MLE_THREADS, "a row per thread in the per-row loops");

// Row handled by thread tid in the per-row loops: rows dealt to the
// four waves in turn (i = 4 lane + wave), so all four SIMDs share them.
__device__ __forceinline__ int mle_row_of_thread(int tid) { return 4 * (tid & 63) + (tid >> 6); }

struct MleLds {
  double* XJ;   // n x p
  double* D;    // n (n+1) / 2: squared distances, packed lower triangle (exactly symmetric)
  double* E;    // n (n+1) / 2: exp(-a), packed likewise
  double* Lm;   // n x LD: K, then its Cholesky factor (lower triangle), then K^{-1}
  double* Li;   // n x LD: L^{-1} (lower), then K^{-1} Kd
  double* y;    // n
  double* al;   // n: K^{-1} y
  double* be;   // n: Kd alpha
  double* ga;   // n: K^{-1} beta
  double* de;   // n: Kdd alpha
  double* r;    // 3 n: row sums of the three traces
  double* dg;   // n: diagonal of the Cholesky factor
  double* x;    // LAGP_MAX_DIM
  double* sc;   // 12 scalars
};

// Position of (i, k) in a packed symmetric matrix (lower triangle by rows).
__device__ __forceinline__ int sym(int i, int k) { return i >= k ? i * (i + 1) / 2 + k : k * (k + 1) / 2 + i; }

// The two packed triangles and two full matrices stay under 80 KB at
// n = 50, so two workgroups share a CU; larger designs keep the same layout
// in a per-location slice of a device workspace.
__host__ __device__ inline size_t mle_lds_bytes_n(int n, int p) {
  const int LD = n + 1;
  return sizeof(double) * ((size_t)n * p + (size_t)n * (n + 1) + 2 * (size_t)n * LD + 9 * (size_t)n +
                           LAGP_MAX_DIM + 12);
}

__device__ inline MleLds mle_carve(unsigned char* s, int n, int p) {
  const int LD = n + 1;
  MleLds L;
  double* d = reinterpret_cast<double*>(s);
  L.XJ = d; d += n * p;
  L.D = d; d += n * (n + 1) / 2;
  L.E = d; d += n * (n + 1) / 2;
  L.Lm = d; d += n * LD;
  L.Li = d; d += n * LD;
  L.y = d; d += n;
  L.al = d; d += n;
  L.be = d; d += n;
  L.ga = d; d += n;
  L.de = d; d += n;
  L.r = d; d += 3 * n;
  L.dg = d; d += n;
  L.x = d; d += LAGP_MAX_DIM;
  L.sc = d;
  return L;
}

// Cholesky factor of the n x n matrix in Lm and, when Li is given, the
// inverse of the factor, both right-looking so that every step is parallel:
// step m takes the pivot L_mm = sqrt(s_mm) (kept in dg; Lm's diagonal is not
// overwritten), divides column m of L and row m of L^{-1} by it, then
// subtracts L_im L_km from every trailing s_ik (m < k <= i) and L_im
// (L^{-1})_mc from every s'_ic (m < i, c <= m).  Each element therefore
// receives exactly the terms of its defining sum
//   L_ik = (K_ik - sum_{m<k} L_im L_km) / L_kk,
//   (L^{-1})_ic = ([i = c] - sum_{c<=m<i} L_im (L^{-1})_mc) / L_ii
// in ascending m, one fused multiply-add each: the values of the
// column-by-column algorithm, bit for bit.  Li must hold the identity on and
// below the diagonal on entry.  Returns false if a pivot is not positive.
__device__ bool mle_cholesky(double* Lm, double* dg, double* Li, int n, int LD) {
  const int tid = threadIdx.x, T = blockDim.x;
  for (int m = 0; m < n; ++m) {
    const double smm = Lm[m * LD + m];
    if (!(smm > 0.0)) return false;  // (every thread reads the same value)
    const double piv = __builtin_sqrt(smm);
    const int nl = n - m - 1, nr = Li ? m + 1 : 0;
    for (int t = tid; t < nl + nr; t += T) {
      if (t < nl) {
        const int i = m + 1 + t;
        Lm[i * LD + m] = Lm[i * LD + m] / piv;
      } else {
        const int c = t - nl;
        Li[m * LD + c] = Li[m * LD + c] / piv;
      }
    }
    if (tid == 0) dg[m] = piv;
    __syncthreads();
    // trailing updates, rows dealt to the waves in turn, columns to the lanes
    // in chunks of 64: (i, k) with m < k <= i, and (i, c) with c <= m.
    // Column m of L and row m of L^{-1} are not written here, so each lane
    // reads its L_km and (L^{-1})_mc once per chunk, and every element still
    // receives one update per m.
    const int lane = tid & 63, wv = tid >> 6, nwv = T >> 6;
    const int ncol = nl > nr ? nl : nr;
    for (int c0 = 0; c0 < ncol; c0 += 64) {
      const int cl = c0 + lane, k = m + 1 + cl;
      const double lkm = cl < nl ? Lm[k * LD + m] : 0.0;
      const double lmc = cl < nr ? Li[m * LD + cl] : 0.0;
      for (int r = wv; r < nl; r += nwv) {
        const int i = m + 1 + r;
        const double lim = Lm[i * LD + m];
        if (cl <= r) Lm[i * LD + k] = __builtin_fma(-lim, lkm, Lm[i * LD + k]);
        if (cl < nr) Li[i * LD + cl] = __builtin_fma(-lim, lmc, Li[i * LD + cl]);
      }
    }
    __syncthreads();
  }
  return true;
}

// Index-order inner product (one thread).
__device__ __forceinline__ double mle_dot(const double* a, const double* b, int n) {
  double s = 0.0;
  for (int k = 0; k < n; ++k) s = __builtin_fma(a[k], b[k], s);
  return s;
}

// dK/dtheta and d2K/dtheta2 at (i, k) from the packed D and E (the same
// expressions, hence the same values, wherever they are needed).
__device__ __forceinline__ double mle_kd(const MleLds& L, int s, double w) {
  const double a = L.D[s] * w;
  return (L.E[s] * a) * w;
}
__device__ __forceinline__ double mle_kdd(const MleLds& L, int s, double w, double ww) {
  const double a = L.D[s] * w;
  return (L.E[s] * (a * a - 2.0 * a)) * ww;
}

// l' and l'' at theta (all threads; results in sc[0], sc[1]; returns false
// if K is not positive definite).
__device__ bool mle_eval(const MleLds& L, int n, double g, double theta) {
  const int tid = threadIdx.x, LD = n + 1, T = blockDim.x;
  const double w = 1.0 / theta;
  for (int t = tid; t < n * n; t += T) {
    const int i = t / n, k = t % n;
    if (k <= i) {  // the factorisation reads the lower triangle only
      const int s = sym(i, k);
      const double e = gexp(-(L.D[s] * w));
      L.E[s] = e;
      L.Lm[i * LD + k] = e + (i == k ? g : 0.0);
    }
    L.Li[i * LD + k] = (i == k) ? 1.0 : 0.0;
  }
  __syncthreads();
  if (!mle_cholesky(L.Lm, L.dg, L.Li, n, LD)) return false;
  // K^{-1} = L^{-T} L^{-1}: (K^{-1})_ik = sum_{m >= max(i,k)} (L^{-1})_mi (L^{-1})_mk,
  // the terms below max(i,k) being exact zeros of the lower triangular
  // factor; written over the factor, which is no longer needed
  {
    const double* Li = L.Li;
    double* Ki = L.Lm;
    exact_gemm(
        n, [=](int i, int k) { return Li[k * LD + i]; }, [=](int k, int j) { return Li[k * LD + j]; },
        [=](int i, int j, double v) { Ki[i * LD + j] = v; });
  }
  __syncthreads();
  const double* Ki = L.Lm;
  const int ri = mle_row_of_thread(tid);
  if (ri < n) L.al[ri] = mle_dot(Ki + ri * LD, L.y, n);
  __syncthreads();
  const double ww = w * w;
  if (ri < n) {
    const int i = ri;
    double b = 0.0, d = 0.0;
    for (int k = 0; k < n; ++k) {
      const int s = sym(i, k);
      b = __builtin_fma(mle_kd(L, s, w), L.al[k], b);
      d = __builtin_fma(mle_kdd(L, s, w, ww), L.al[k], d);
    }
    L.be[i] = b;
    L.de[i] = d;
  }
  __syncthreads();
  if (ri < n) L.ga[ri] = mle_dot(Ki + ri * LD, L.be, n);
  // P = K^{-1} Kd into the L^{-1} buffer (no longer needed)
  {
    double* P = L.Li;
    const MleLds& LL = L;
    exact_gemm(
        n, [=](int i, int k) { return Ki[i * LD + k]; }, [&](int k, int j) { return mle_kd(LL, sym(k, j), w); },
        [=](int i, int j, double v) { P[i * LD + j] = v; });
  }
  __syncthreads();
  if (ri < n) {
    const int i = ri;
    double r1 = 0.0, r2 = 0.0, r3 = 0.0;
    for (int k = 0; k < n; ++k) {
      const double kik = Ki[i * LD + k];
      const int s = sym(k, i);
      r1 = __builtin_fma(kik, mle_kd(L, s, w), r1);
      r2 = __builtin_fma(kik, mle_kdd(L, s, w, ww), r2);
      r3 = __builtin_fma(L.Li[i * LD + k], L.Li[k * LD + i], r3);
    }
    L.r[i] = r1;
    L.r[n + i] = r2;
    L.r[2 * n + i] = r3;
  }
  __syncthreads();
  // the seven scalar sums, each one in-order chain, on lanes of different waves
  {
    const int job = (tid & 63) == 0 ? tid >> 6 : -1;
    const int nw = T >> 6;
    for (int q = job; q >= 0 && q < 7; q += nw) {
      double v = 0.0;
      if (q == 0) v = mle_dot(L.y, L.al, n);   // psi
      if (q == 1) v = mle_dot(L.al, L.be, n);  // alpha^T Kd alpha
      if (q == 2) v = mle_dot(L.be, L.ga, n);  // beta^T K^{-1} beta
      if (q == 3) v = mle_dot(L.al, L.de, n);  // alpha^T Kdd alpha
      if (q >= 4) {
        const double* rr = L.r + (q - 4) * n;  // the traces: in-order sums of the row sums
        for (int i = 0; i < n; ++i) v = v + rr[i];
      }
      L.sc[2 + q] = v;
    }
  }
  __syncthreads();
  if (tid == 0) {
    const double psi = L.sc[2], ab = L.sc[3], bgb = L.sc[4], add = L.sc[5];
    const double t1 = L.sc[6], t2 = L.sc[7], t3 = L.sc[8];
    const double hn = 0.5 * (double)n;
    const double q = ab / psi;
    L.sc[0] = -0.5 * t1 + hn * q;
    L.sc[1] = -0.5 * (t2 - t3) + hn * ((add - 2.0 * bgb) / psi + q * q);
  }
  __syncthreads();
  return true;
}

// WS: the location's matrices in its slice of a.ws (designs past the LDS
// sizes), else in LDS.
template <bool WS>
__global__ __launch_bounds__(MLE_THREADS) void k_mle(MleArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int n = a.n, p = a.p, LD = n + 1, tid = threadIdx.x, T = blockDim.x;
  const int64_t m = blockIdx.x;
  unsigned char* base = smem;
  if constexpr (WS) base = reinterpret_cast<unsigned char*>(a.ws) + (size_t)m * ((mle_lds_bytes_n(n, p) + 255) & ~size_t(255));
  const MleLds L = mle_carve(base, n, p);
  const int32_t* J = a.sel + m * n;
  const int st_in = a.status_in ? a.status_in[m] : 0;
  const int fl_prev = a.flags_prev ? a.flags_prev[m] : 0;
  const int it_prev = a.iters_prev ? a.iters_prev[m] : 0;
  const double th0 = a.theta0 ? a.theta0[m] : a.d0;
  const bool skip = !(th0 > 0.0) || (st_in & (LAGP_STATUS_NOTPD | LAGP_STATUS_NONFINITE));
  if (skip) {  // the design stage failed (here or in an earlier stage): nothing to fit
    if (tid == 0) {
      a.theta_out[m] = a.nan_on_skip ? __builtin_nan("") : (th0 > 0.0 ? th0 : a.d0);
      a.status_out[m] = st_in | fl_prev;
      a.iters_out[m] = it_prev;
      if (a.mean) {
        a.mean[m] = __builtin_nan("");
        a.s2[m] = __builtin_nan("");
        a.df[m] = (double)n;
      }
    }
    return;
  }
  for (int t = tid; t < n * p; t += T) L.XJ[t] = a.X[(int64_t)J[t / p] * p + (t % p)];
  for (int i = tid; i < n; i += T) L.y[i] = a.y[J[i]];
  for (int k = tid; k < LAGP_MAX_DIM; k += T) L.x[k] = k < p ? a.XX[m * p + k] : 0.0;
  __syncthreads();
  for (int t = tid; t < n * n; t += T) {
    const int i = t / n, k = t % n;
    if (k <= i) L.D[sym(i, k)] = sqdist(L.XJ + i * p, L.XJ + k * p, p);
  }
  __syncthreads();

  // safeguarded Newton iteration (thread 0 decides, everyone evaluates)
  double lo = a.dmin, hi = a.dmax;
  double theta = th0 < lo ? lo : (th0 > hi ? hi : th0);
  int it = 0, conv = 0, flags = 0;
  while (it < a.maxit) {
    const bool ok = mle_eval(L, n, a.g, theta);
    ++it;
    double d1 = -1.0, d2 = 0.0;
    if (ok) {
      d1 = L.sc[0];
      d2 = L.sc[1];
    } else {
      flags |= LAGP_STATUS_MLE_NOTPD;
    }
    __syncthreads();  // every thread has read sc before the next evaluation writes it
    if (d1 == 0.0) {
      conv = 1;
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
      conv = 1;
      break;
    }
  }
  if (!conv) flags |= LAGP_STATUS_MLE_MAXIT;
  if (theta <= a.dmin * (1.0 + a.tol) || theta >= a.dmax * (1.0 - a.tol)) flags |= LAGP_STATUS_MLE_BOUND;

  int st = st_in | fl_prev | flags;
  if (a.mean) {
    // prediction at the estimate through the Cholesky factor
    const double w = 1.0 / theta;
    for (int t = tid; t < n * n; t += T) {
      const int i = t / n, k = t % n;
      if (k <= i) L.Lm[i * LD + k] = gexp(-(L.D[sym(i, k)] * w)) + (i == k ? a.g : 0.0);
    }
    __syncthreads();
    const bool pd = mle_cholesky(L.Lm, L.dg, nullptr, n, LD);
    for (int i = tid; i < n; i += T) L.be[i] = gexp(-(sqdist(L.XJ + i * p, L.x, p) * w));  // k_x
    __syncthreads();
    if (tid == 0) {
      double mu = __builtin_nan(""), sc = __builtin_nan("");
      if (pd) {
        for (int i = 0; i < n; ++i) {  // w = L^{-1} k_x into ga, z = L^{-1} y into de
          double u = L.be[i], v = L.y[i];
          for (int k = 0; k < i; ++k) {
            u = __builtin_fma(-L.Lm[i * LD + k], L.ga[k], u);
            v = __builtin_fma(-L.Lm[i * LD + k], L.de[k], v);
          }
          L.ga[i] = u / L.dg[i];
          L.de[i] = v / L.dg[i];
        }
        mu = mle_dot(L.ga, L.de, n);
        const double psi = mle_dot(L.de, L.de, n);
        sc = psi * ((1.0 + a.g) - mle_dot(L.ga, L.ga, n)) / (double)n;
      } else {
        st |= LAGP_STATUS_NOTPD;
      }
      if (!(fabs(mu) <= 1.7976931348623157e308 && fabs(sc) <= 1.7976931348623157e308)) st |= LAGP_STATUS_NONFINITE;
      a.mean[m] = mu;
      a.s2[m] = sc;
      a.df[m] = (double)n;
    }
  }
  if (tid == 0) {
    a.theta_out[m] = theta;
    a.status_out[m] = st;
    a.iters_out[m] = it_prev + it;
  }
}

}  // namespace

size_t mle_lds_bytes(int n, int p) { return mle_lds_bytes_n(n, p); }

bool mle_supported(int n, int p, size_t lds_max) { return n <= LAGP_MAX_N && p <= LAGP_MAX_DIM && lds_max > 0; }

static bool mle_in_lds(int n, int p, size_t lds_max) { return n <= MLE_NMAX_LDS && mle_lds_bytes_n(n, p) <= lds_max; }

size_t mle_workspace_bytes_per_location(int n, int p, size_t lds_max) {
  return mle_in_lds(n, p, lds_max) ? 0 : ((mle_lds_bytes_n(n, p) + 255) & ~size_t(255));
}

hipError_t launch_mle(const MleArgs& a, hipStream_t s, size_t lds_max) {
  if (a.M <= 0) return hipSuccess;
  if (!mle_in_lds(a.n, a.p, lds_max)) {
    hipLaunchKernelGGL(k_mle<true>, dim3(a.M), dim3(MLE_THREADS), 0, s, a);
    return hipGetLastError();
  }
  const size_t lds = mle_lds_bytes_n(a.n, a.p);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mle<false>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mle<false>, dim3(a.M), dim3(MLE_THREADS), lds, s, a);
  return hipGetLastError();
}

}  // namespace lagp
