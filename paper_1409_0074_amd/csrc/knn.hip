// Exact nearest-candidate lists: for each location, the ncand design rows
// with the smallest (squared distance, row) keys, in that order (the N'
// nearest neighbours the local search is restricted to, Sec. 2.2).
//
// One workgroup serves KNN_QB locations and streams the whole design once.
// Each thread takes one design row per pass, computes its squared distance to
// every location of the group (one fma per dimension, in order) and appends
// (d2, row) to that location's buffer when it beats the location's current
// threshold key.  A buffer that could overflow on the next pass is compacted:
// the workgroup sorts it in LDS (bitonic network) and keeps the ncand
// smallest, whose largest key becomes the new threshold.  After the last pass
// every buffer is sorted once more and its first ncand entries written out.
// Because the threshold is always the ncand-th smallest key seen so far, no
// row of the final answer is ever dropped, and the result is exact.
#include "dev_math.h"
#include "lagp_internal.h"

namespace lagp {

int knn_sort_size(int ncand) {
  int S = 512;
  while (S < ncand + 512) S <<= 1;
  return S;
}

size_t knn_lds_bytes(int S, int p) {
  return (size_t)S * (sizeof(double) + sizeof(int)) + (size_t)KNN_QB * p * sizeof(double) +
         KNN_QB * (sizeof(double) + 2 * sizeof(int));
}

// Bitonic sort of S = 2^k (key, row) pairs in LDS, ascending.
__device__ void lds_bitonic_sort(double* kd, int* ki, int S) {
  for (int size = 2; size <= S; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < (S >> 1); t += blockDim.x) {
        const int lo = 2 * stride * (t / stride) + (t % stride);
        const int hi = lo + stride;
        const bool up = (lo & size) == 0;
        const double a = kd[lo], b = kd[hi];
        const int ia = ki[lo], ib = ki[hi];
        const bool sw = up ? key_less(b, ib, a, ia) : key_less(a, ia, b, ib);
        if (sw) {
          kd[lo] = b;
          kd[hi] = a;
          ki[lo] = ib;
          ki[hi] = ia;
        }
      }
      __syncthreads();
    }
  }
}

// Load `count` buffered pairs into LDS, pad to S with +inf keys, sort.
__device__ void load_and_sort(const double* bd, const int32_t* bi, int count, double* kd, int* ki, int S) {
  for (int t = threadIdx.x; t < S; t += blockDim.x) {
    if (t < count) {
      kd[t] = bd[t];
      ki[t] = bi[t];
    } else {
      kd[t] = __builtin_huge_val();
      ki[t] = 0x7fffffff;
    }
  }
  __syncthreads();
  lds_bitonic_sort(kd, ki, S);
}

template <int P>
__global__ __launch_bounds__(KNN_THREADS) void k_knn(KnnArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int S = a.S;
  const int p = P > 0 ? P : a.p;
  double* kd = reinterpret_cast<double*>(smem);
  double* qx = kd + S;                       // KNN_QB x p
  double* thr_d = qx + KNN_QB * p;           // KNN_QB
  int* ki = reinterpret_cast<int*>(thr_d + KNN_QB);  // S
  int* thr_i = ki + S;                       // KNN_QB
  int* cnt = thr_i + KNN_QB;                 // KNN_QB

  const int m0 = blockIdx.x * KNN_QB;
  const int nq = min(KNN_QB, a.M - m0);
  for (int t = threadIdx.x; t < KNN_QB * p; t += blockDim.x) {
    const int q = t / p;
    qx[t] = (q < nq) ? a.XX[(int64_t)(m0 + q) * p + (t % p)] : 0.0;
  }
  if (threadIdx.x < KNN_QB) {
    thr_d[threadIdx.x] = __builtin_huge_val();
    thr_i[threadIdx.x] = 0x7fffffff;
    cnt[threadIdx.x] = 0;
  }
  __syncthreads();

  double* bd = a.buf_d2 + (int64_t)m0 * S;
  int32_t* bi = a.buf_idx + (int64_t)m0 * S;

  for (int64_t base = 0; base < a.N; base += KNN_THREADS) {
    const int64_t i = base + threadIdx.x;
    if (i < a.N) {
      double xi[P > 0 ? P : LAGP_MAX_DIM];
      const double* src = a.X + i * p;
#pragma unroll
      for (int k = 0; k < (P > 0 ? P : LAGP_MAX_DIM); ++k)
        if (P > 0 || k < p) xi[k] = src[k];
      for (int q = 0; q < nq; ++q) {
        const double* xq = qx + q * p;
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < (P > 0 ? P : LAGP_MAX_DIM); ++k) {
          if (P > 0 || k < p) {
            const double t = xi[k] - xq[k];
            s = __builtin_fma(t, t, s);
          }
        }
        if (key_less(s, (int)i, thr_d[q], thr_i[q])) {
          const int pos = atomicAdd(&cnt[q], 1);
          bd[(int64_t)q * S + pos] = s;
          bi[(int64_t)q * S + pos] = (int32_t)i;
        }
      }
    }
    __syncthreads();
    // compact every buffer that the next pass could overflow
    for (int q = 0; q < nq; ++q) {
      const int c = cnt[q];
      if (c > S - KNN_THREADS) {
        load_and_sort(bd + (int64_t)q * S, bi + (int64_t)q * S, c, kd, ki, S);
        for (int t = threadIdx.x; t < a.ncand; t += blockDim.x) {
          bd[(int64_t)q * S + t] = kd[t];
          bi[(int64_t)q * S + t] = ki[t];
        }
        if (threadIdx.x == 0) {
          thr_d[q] = kd[a.ncand - 1];
          thr_i[q] = ki[a.ncand - 1];
          cnt[q] = a.ncand;
        }
        __syncthreads();
      }
    }
  }
  // final exact order
  for (int q = 0; q < nq; ++q) {
    const int c = cnt[q];
    load_and_sort(bd + (int64_t)q * S, bi + (int64_t)q * S, c, kd, ki, S);
    const int64_t m = m0 + q;
    for (int t = threadIdx.x; t < a.ncand; t += blockDim.x) {
      a.out_idx[m * a.ncand + t] = ki[t];
      if (a.out_d2) a.out_d2[m * a.ncand + t] = kd[t];
    }
    __syncthreads();
  }
}

hipError_t launch_knn(const KnnArgs& a, hipStream_t s) {
  if (a.M <= 0) return hipSuccess;
  const size_t lds = knn_lds_bytes(a.S, a.p);
  const dim3 grid((a.M + KNN_QB - 1) / KNN_QB);
#define LAGP_KNN_CASE(PP)                                                                          \
  case PP: {                                                                                       \
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_knn<PP>),                   \
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);       \
    if (e != hipSuccess) return e;                                                                 \
    hipLaunchKernelGGL(k_knn<PP>, grid, dim3(KNN_THREADS), lds, s, a);                             \
    break;                                                                                         \
  }
  switch (a.p) {
    LAGP_KNN_CASE(1)
    LAGP_KNN_CASE(2)
    LAGP_KNN_CASE(3)
    LAGP_KNN_CASE(4)
    LAGP_KNN_CASE(8)
    default: {
      hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_knn<0>),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k_knn<0>, grid, dim3(KNN_THREADS), lds, s, a);
    }
  }
#undef LAGP_KNN_CASE
  return hipGetLastError();
}

// Per-dimension min and max of the design (bounding box that cuts rays).
__global__ __launch_bounds__(256) void k_bbox(const double* X, int64_t N, int p, double* lo, double* hi) {
  __shared__ double slo[256], shi[256];
  const int k = blockIdx.x;
  double a = __builtin_huge_val(), b = -__builtin_huge_val();
  for (int64_t i = threadIdx.x; i < N; i += blockDim.x) {
    const double v = X[i * p + k];
    a = fmin(a, v);
    b = fmax(b, v);
  }
  slo[threadIdx.x] = a;
  shi[threadIdx.x] = b;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      slo[threadIdx.x] = fmin(slo[threadIdx.x], slo[threadIdx.x + w]);
      shi[threadIdx.x] = fmax(shi[threadIdx.x], shi[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    lo[k] = slo[0];
    hi[k] = shi[0];
  }
}

hipError_t launch_bbox(const double* X, int64_t N, int p, double* lo, double* hi, hipStream_t s) {
  hipLaunchKernelGGL(k_bbox, dim3(p), dim3(256), 0, s, X, N, p, lo, hi);
  return hipGetLastError();
}

}  // namespace lagp
