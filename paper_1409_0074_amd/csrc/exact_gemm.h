// C = A B on the f64 matrix cores with every element summed exactly in
// index order (shared by the likelihood kernels).
#pragma once

#include <hip/hip_runtime.h>

namespace lagp {

typedef double v4d_t __attribute__((ext_vector_type(4)));

// C = A B for n x n operands on f64 MFMA: 16 x 16 tiles, one per wave at a
// time, k in chunks of 4 in ascending order.  v_mfma_f64_16x16x4f64 adds
// sum_k A[i][k] B[k][j] to its accumulator as fused multiply-adds in
// ascending k, so every element is the index-order fma chain from 0.0 (the
// padding past n adds exact zeros).  Lane layout: A[i][k] from lane
// 16k + i, B[k][j] from lane 16k + j, C[i][j] in register i/4 of lane
// 16(i%4) + j.
template <class FA, class FB, class ST>
__device__ __forceinline__ void exact_gemm(int n, const FA& fa, const FB& fb, const ST& st) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int nt = (n + 15) / 16, nk = (n + 3) / 4;
  for (int t = wv; t < nt * nt; t += nw) {
    const int ti = t / nt, tj = t % nt;
    const int ai = 16 * ti + (lane & 15), bj = 16 * tj + (lane & 15), kl = lane >> 4;
    v4d_t acc = {0.0, 0.0, 0.0, 0.0};
    for (int kc = 0; kc < nk; ++kc) {
      const int k = 4 * kc + kl;
      const double av = (ai < n && k < n) ? fa(ai, k) : 0.0;
      const double bv = (k < n && bj < n) ? fb(k, bj) : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * ti + 4 * r + kl;
      if (i < n && bj < n) st(i, bj, acc[r]);
    }
  }
}

}  // namespace lagp
