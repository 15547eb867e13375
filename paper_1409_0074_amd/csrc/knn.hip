// Exact nearest-candidate lists: for each location, the ncand design rows
// with the smallest (squared distance, row) keys, in that order (the N'
// nearest neighbours the local search is restricted to, Sec. 2.2).
// Squared distances accumulate the dimensions in order, one fma each.
#include "dev_math.h"
#include "lagp_internal.h"

namespace lagp {

int knn_sort_size(int ncand) {
  int S = 512;
  while (S < ncand + 512) S <<= 1;
  return S;
}

// Bitonic sort of S = 2^k (key, row) pairs in LDS, ascending.
__device__ void lds_bitonic_sort(double* kd, int* ki, int S) {
  for (int size = 2; size <= S; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      const int ls = __builtin_ctz(stride);  // strides are powers of two
      for (int t = threadIdx.x; t < (S >> 1); t += blockDim.x) {
        const int lo = ((t >> ls) << (ls + 1)) + (t & (stride - 1));
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

// ------------------------------------------------ threshold-first kNN ---
//
// For large designs the lists come from three passes:
//  1. threshold: one lane per location; the KSEL-th smallest squared
//     distance over a subsample of the design (rows t*A mod N, t < Ns, A
//     coprime with N, gathered once per call).  Ns = N / r with
//     r = 2 n_t / KSEL (n_t = N', or a quarter of the sort size when that is
//     larger), so that about 2 n_t >= 2 N' rows of the full design fall below
//     that value (relative spread 1/sqrt(KSEL): fewer than N' with
//     probability ~3e-5).
//  2. scan: each wave takes 64 locations and one slice of the design, screens
//     16 rows at a time with MFMA inner products, and appends the rows with
//     d2 <= threshold to the location's buffer (capacity CAP) through a
//     per-location atomic.
//  3. merge: one workgroup per location keeps the exact ncand smallest
//     (d2, row) keys of its buffer (LDS bitonic sorts, streaming when the
//     buffer exceeds the sort size).  If the threshold caught fewer than
//     ncand rows, or more than CAP, the workgroup falls back to the exact
//     single-pass compaction scan of the whole design for that location.
// Every key and order is exact; the threshold only decides how much work is
// done, never which rows are returned.

constexpr int KT = 4;               // per-part list length of the threshold pass
constexpr int KSEL = 64;            // subsample order statistic taken as the threshold
constexpr int KPARTS = 256 / KT;    // most parts: the reduce sorts at most 256 values per location
static_assert(KSEL <= KT * KPARTS, "the partial lists must hold KSEL values");

// The design never changes while these kernels run: reading it through the
// constant address space lets wave-uniform row reads become scalar loads
// into SGPRs (one 64-byte row feeds the 64 lanes' fmas directly).
typedef const double __attribute__((address_space(4))) cdouble;
__device__ __forceinline__ const cdouble* as_const(const double* p) { return (const cdouble*)p; }

// Subsample gather: row t of the subsample is design row t*A mod N (A coprime
// with N, so structured designs such as grids are sampled without a regular
// pattern); stored contiguously so the threshold pass streams it.
__global__ __launch_bounds__(256) void k_knn_gather_sub(Knn2Args a) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.sub_count * a.p) return;
  const int64_t row = t / a.p, k = t - row * a.p;
  const int64_t src = (row * a.sub_stride) % a.N;  // row, stride < 2^31: no overflow
  a.sub[t] = a.X[src * a.p + k];
}

// Threshold pass, part 1: wave (w, group) takes subsample rows
// t = w*Ns/parts .. (w+1)*Ns/parts - 1 and leaves, per location, its KT
// smallest squared distances in the location's buffer (scratch until the
// scan).
template <int P>
__global__ __launch_bounds__(64) void k_knn_tau(Knn2Args a) {
  constexpr int PD = P > 0 ? P : LAGP_MAX_DIM;
  const int q = blockIdx.y * 64 + threadIdx.x;
  const bool live = q < a.M;
  const int p = P > 0 ? P : a.p;
  double xq[PD];
#pragma unroll
  for (int k = 0; k < PD; ++k)
    if (P > 0 || k < p) xq[k] = live ? a.XX[(int64_t)q * p + k] : 0.0;
  double best[KT];
#pragma unroll
  for (int k = 0; k < KT; ++k) best[k] = __builtin_huge_val();
  double cur = __builtin_huge_val();
  const int64_t t0 = (a.sub_count * blockIdx.x) / gridDim.x;
  const int64_t t1 = (a.sub_count * (blockIdx.x + 1)) / gridDim.x;
  const cdouble* X = as_const(a.sub);
  constexpr int U = 4;  // rows per iteration, their loads issued together
  for (int64_t t = t0; t < t1; t += U) {
    double s[U];
#pragma unroll
    for (int r = 0; r < U; ++r) {
      const int64_t row = t + r < t1 ? t + r : t1 - 1;
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < PD; ++k) {
        if (P > 0 || k < p) {
          const double u = xq[k] - X[row * p + k];
          acc = __builtin_fma(u, u, acc);
        }
      }
      s[r] = t + r < t1 ? acc : __builtin_huge_val();
    }
#pragma unroll
    for (int r = 0; r < U; ++r) {
      if (s[r] < cur) {
        bool done = false;
        double mx = 0.0;
#pragma unroll
        for (int k = 0; k < KT; ++k) {
          if (!done && best[k] == cur) {
            best[k] = s[r];
            done = true;
          }
          mx = fmax(mx, best[k]);
        }
        cur = mx;
      }
    }
  }
  if (live) {
    double* dst = a.buf_d2 + (int64_t)q * a.CAP + blockIdx.x * KT;
#pragma unroll
    for (int k = 0; k < KT; ++k) dst[k] = best[k];
  }
}

// Threshold pass, part 2: the KSEL-th smallest over the partial lists (the
// KSEL-th smallest of the subsample unless one part held more than KT of the
// KSEL smallest; either way only the amount of work depends on it).  One
// 64-thread block per location sorts the parts * KT <= 256 values in LDS.
__global__ __launch_bounds__(64) void k_knn_tau_reduce(Knn2Args a, int parts) {
  __shared__ double v[256];
  const int q = blockIdx.x;
  const double* src = a.buf_d2 + (int64_t)q * a.CAP;
  const int nv = parts * KT;
  for (int t = threadIdx.x; t < 256; t += 64) v[t] = t < nv ? src[t] : __builtin_huge_val();
  __syncthreads();
  for (int size = 2; size <= 256; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      const int ls = __builtin_ctz(stride);
      for (int t = threadIdx.x; t < 128; t += 64) {
        const int lo = ((t >> ls) << (ls + 1)) + (t & (stride - 1));
        const int hi = lo + stride;
        const bool up = (lo & size) == 0;
        const double x = v[lo], y = v[hi];
        if (up ? (y < x) : (x < y)) {
          v[lo] = y;
          v[hi] = x;
        }
      }
      __syncthreads();
    }
  }
  if (threadIdx.x == 0) {
    a.tau[q] = a.force_fallback ? -1.0 : v[KSEL - 1];
    a.cnt[q] = 0;
  }
}

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Scan with an MFMA distance screen.  For 64 locations (four sets of 16) and
// a tile of 16 design rows, 16x16x4 FP64 MFMAs give the inner products
// <x_q, x_i>; t = ||x_i||^2 - 2 <x_q, x_i> then approximates d2 - ||x_q||^2.
// With u = 2^-53, the defined squared distance (an fma chain over the
// dimensions) is within (p+2)u d2 of the true one, and t within
// (2p+6)u (||x_q||^2 + 2 max_i ||x_i||^2) of its true value, so the screen
// t <= tau (1 + 2(p+2)u) - ||x_q||^2 + 4(p+4)u (||x_q||^2 + 2 max ||x_i||^2)
// (twice each bound) passes every row whose defined squared distance is
// <= tau.  Passing rows get the defined squared distance and are appended
// only if it is <= tau: the rows collected are exactly those of a plain scan
// (in another order, which the merge's sort by (d2, row) removes).
// MFMA operands: A[i][k] from lane 16k + i (location 16s + i, dimension
// 4c + k), B[k][n] from lane 16k + n (row n of the tile, dimension 4c + k),
// D[i][n] in register i/4 of lane 16(i%4) + n.
template <int P>
__global__ __launch_bounds__(64) void k_knn_scan(Knn2Args a) {
  constexpr int PD = P > 0 ? P : LAGP_MAX_DIM;
  constexpr int NCH = (PD + 3) / 4;  // K-chunks of 4 dimensions
  const int p = P > 0 ? P : a.p;
  const int lane = threadIdx.x, g = lane >> 4, n = lane & 15;
  const int q0 = blockIdx.x * 64;
  double af[4][NCH];
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      const int q = q0 + 16 * s + n, d = 4 * c + g;
      af[s][c] = (q < a.M && d < p) ? a.XX[(int64_t)q * p + d] : 0.0;
    }
  // screen bounds of this lane's outputs: set s, register r -> location
  // q0 + 16 s + 4 r + g
  const double u = 0x1p-53;
  double th[4][4];
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int q = q0 + 16 * s + 4 * r + g;
      double t = -__builtin_huge_val();
      if (q < a.M) {
        const double tau = a.tau[q];
        double qn = 0.0;
        for (int k = 0; k < p; ++k) qn = __builtin_fma(a.XX[(int64_t)q * p + k], a.XX[(int64_t)q * p + k], qn);
        if (tau >= 0.0)
          t = tau * (1.0 + 2.0 * (p + 2) * u) - qn + 4.0 * (p + 4) * u * (qn + 2.0 * a.rn_max);
      }
      th[s][r] = t;
    }
  const int64_t i0 = (int64_t)blockIdx.y * a.slice;
  const int64_t i1 = i0 + a.slice < a.N ? i0 + a.slice : a.N;
  // Screened pairs are staged in LDS and settled in batches (one lane per
  // pair): the defined squared distance, and for d2 <= tau an append to the
  // location's buffer.
  constexpr int STG = 2048;
  __shared__ int32_t st_row[STG];
  __shared__ uint8_t st_q[STG];
  __shared__ int st_n;
  if (lane == 0) st_n = 0;
  __syncthreads();
  auto flush = [&]() {
    __syncthreads();
    const int tot = st_n;
    for (int e = lane; e < tot; e += 64) {
      const int64_t row = st_row[e];
      const int q = q0 + st_q[e];
      const double* xq = a.XX + (int64_t)q * p;
      const double* xr = a.X + row * p;
      double acc = 0.0;
      for (int k = 0; k < p; ++k) {
        const double d = xq[k] - xr[k];
        acc = __builtin_fma(d, d, acc);
      }
      if (acc <= a.tau[q]) {
        const int pos = atomicAdd(&a.cnt[q], 1);
        if (pos < a.CAP) {
          a.buf_d2[(int64_t)q * a.CAP + pos] = acc;
          a.buf_idx[(int64_t)q * a.CAP + pos] = (int32_t)row;
        }
      }
    }
    __syncthreads();
    if (lane == 0) st_n = 0;
    __syncthreads();
  };
  // the next tile's rows are loaded while the current one is screened
  double bn[NCH], rnn;
  auto load_tile = [&](int64_t i, double (&bf)[NCH], double& rn) {
    const int64_t rr = i + n;
    const int64_t rl = rr < i1 ? rr : i1 - 1;  // in bounds
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      const int d = 4 * c + g;
      bf[c] = d < p ? a.X[rl * p + d] : 0.0;
    }
    rn = rr < i1 ? a.rn[rl] : __builtin_huge_val();
  };
  if (i0 < i1) load_tile(i0, bn, rnn);
  for (int64_t i = i0; i < i1; i += 16) {
    const int64_t rr = i + n;
    const bool valid = rr < i1;
    double bf[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) bf[c] = bn[c];
    const double rn = rnn;
    if (i + 16 < i1) load_tile(i + 16, bn, rnn);
    unsigned hit = 0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int c = 0; c < NCH; ++c) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(af[s][c], bf[c], acc, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (__builtin_fma(-2.0, acc[r], rn) <= th[s][r]) hit |= 1u << (4 * s + r);
    }
    if (!valid) hit = 0;  // (t = inf passes an infinite bound)
    if (!__builtin_expect(__any(hit), 0)) continue;
    // stage the screened pairs: (row, location within the wave's 64)
    const int nh = __builtin_popcount(hit);
    const int base = nh ? atomicAdd(&st_n, nh) : 0;
    for (int k = 0; hit; ++k) {
      const int b = __builtin_ctz(hit);  // b = 4 s + r: location 16 s + 4 r + g
      hit &= hit - 1;
      st_row[base + k] = (int32_t)rr;
      st_q[base + k] = (uint8_t)(4 * b + g);
    }
    __syncthreads();
    if (st_n > STG - 1024) flush();  // a tile stages at most 64 x 16
  }
  flush();
}

// The same scan with the screen on the FP32 matrix cores (twice the FP64
// rate), for designs whose squared norms stay far inside FP32's range.  The
// accumulator starts at rn_i - th_q (one FP32 addition per entry) and the
// product adds -2 x_q . x_i over the coordinates alone, so it ends at
// t - th_q itself and a pair passes when its sign bit is set (no per-pair
// conversion, fma or comparison; a byte permute gathers four sign bits at
// once), with no K chunk spent on the two constant terms.
// Error: operands are rounded to FP32 (u32 = 2^-24; th_q upward, which only
// widens the screen); the start value is rounded once and the product's
// 4 NCC terms are summed into it with at most 4 NCC + 1 roundings, so with
// K = 4 NCC + 4 the accumulator is within
// (K + 3) u32 (2 ||x_q||^2 + 3 max ||x_i||^2 + tau) (1 + 1e-3) of
// t - th_q (the terms: the rounded coordinates, 2 u32 (||x_q||^2 + ||x_i||^2);
// rn_i, u32 ||x_i||^2; the start value, u32 (||x_i||^2 + |th_q|); the
// summation, (4 NCC + 1) u32 times the sum of the magnitudes, which is at
// most 2 ||x_q||^2 + 2 ||x_i||^2 + tau + |rn_i - th_q|).
// th_q adds 4 (K + 4) u32 (2 ||x_q||^2 + 3 max ||x_i||^2 + tau) + 2^-100
// (flushed subnormals) to the FP64 bound of the other scan, so every row
// whose defined squared distance is <= tau gives a negative accumulator, and
// the defined squared distance (FP64, from the FP64 coordinates) still
// decides.  Infinite bounds stay exact: th = -inf (no row) gives +inf, th = +inf
// (every row) -inf, and a row past the slice (rn = +inf) is masked.
// MFMA operands as in the FP64 scan; the FP32 16x16x4 result D[i][n] (and
// the start value C[i][n]) sits in register i % 4 of lane 16 (i / 4) + n.
// Six waves per SIMD with three tiles in flight each (the scan waits on the
// design stream): registers capped to fit, which also keeps the MFMA results
// out of the accumulation registers.
constexpr int SCAN32_WAVES = 6;  // per SIMD (registers of SD = 3 tiles in flight)

template <int P>
__global__ __launch_bounds__(64, SCAN32_WAVES) void k_knn_scan32(Knn2Args a) {
  constexpr int SD = 3;  // tiles in flight per wave
  constexpr int PD = P > 0 ? P : LAGP_MAX_DIM;
  constexpr int NCC = (PD + 3) / 4;  // K-chunks of 4 coordinates
  constexpr int K = 4 * NCC + 4;     // (the bound's constant)
  const int p = P > 0 ? P : a.p;
  const int lane = threadIdx.x, g = lane >> 4, n = lane & 15;
  const int q0 = blockIdx.x * 64;
  const double u = 0x1p-53, u32 = 0x1p-24;
  // A operand: set s, row n -> location q0 + 16 s + n; nth_l[s][i]: -th of
  // location q0 + 16 s + i (the start value's rows, read per tile: registers
  // are what limits the waves per SIMD)
  float af[4][NCC];
  __shared__ __align__(16) float nth_l[4][16];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int q = q0 + 16 * s + n;
    double th = -__builtin_huge_val();
    if (q < a.M) {
      const double tau = a.tau[q];
      double qn = 0.0;
      for (int k = 0; k < p; ++k) qn = __builtin_fma(a.XX[(int64_t)q * p + k], a.XX[(int64_t)q * p + k], qn);
      if (tau >= 0.0)
        th = tau * (1.0 + 2.0 * (p + 2) * u) - qn + 4.0 * (p + 4) * u * (qn + 2.0 * a.rn_max) +
             4.0 * (K + 4) * u32 * (2.0 * qn + 3.0 * a.rn_max + tau) + 0x1p-100;
      if (!(qn <= 1e30)) th = __builtin_huge_val();  // out of FP32's comfort: every row passes
    }
    const float nth = -__double2float_ru(th);
#pragma unroll
    for (int c = 0; c < NCC; ++c) {
      const int d = 4 * c + g;
      af[s][c] = (d < p && q < a.M) ? -2.0f * (float)a.XX[(int64_t)q * p + d] : 0.0f;
    }
    if (g == 0) nth_l[s][n] = nth;
  }
  // hit-mask bits of real locations: bit 8 r + s <-> location q0 + 16 s + 4 g + r
  unsigned locmask = 0;
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (q0 + 16 * s + 4 * g + r < a.M) locmask |= 1u << (8 * r + s);
  const int64_t i0 = (int64_t)blockIdx.y * a.slice;
  const int64_t i1 = i0 + a.slice < a.N ? i0 + a.slice : a.N;
  // Staging (the workgroup is one wave, so its count lives in a scalar
  // register): a lane whose tile has hits stages one entry, its design row
  // and its hit word with g in bits 28-29 (the locations are 16 s + 4 g + r
  // for the set bits 8 r + s); a tile adds at most 64 entries and the buffer
  // is settled once it holds more than STG - 64.
  constexpr int STG = 320;
  __shared__ int32_t st_row[STG];
  __shared__ uint32_t st_w[STG];
  int st_n = 0;
  auto flush = [&]() {
    __syncthreads();  // (the entries' LDS writes are complete)
    for (int e = lane; e < st_n; e += 64) {
      const int64_t row = st_row[e];
      const uint32_t w = st_w[e];
      const int gq = (int)(w >> 28);
      const double* xr = a.X + row * p;
      for (uint32_t m = w & 0x0F0F0F0Fu; m; m &= m - 1) {
        const int bb = __builtin_ctz(m);
        const int q = q0 + 16 * (bb & 7) + 4 * gq + (bb >> 3);
        const double* xq = a.XX + (int64_t)q * p;
        double acc = 0.0;
        for (int k = 0; k < p; ++k) {
          const double d = xq[k] - xr[k];
          acc = __builtin_fma(d, d, acc);
        }
        if (acc <= a.tau[q]) {
          const int pos = atomicAdd(&a.cnt[q], 1);
          if (pos < a.CAP) {
            a.buf_d2[(int64_t)q * a.CAP + pos] = acc;
            a.buf_idx[(int64_t)q * a.CAP + pos] = (int32_t)row;
          }
        }
      }
    }
    __syncthreads();  // (every entry read before the next tile's writes)
    st_n = 0;
  };
  // B operand: column n -> design row i + n.  Tiles are loaded SD tiles
  // ahead (SD register sets in a ring) into raw registers and converted only
  // when used: the scan waits on the design stream, not on its arithmetic.
  float xn[SD][NCC];
  double rnn[SD];
  auto load_tile = [&](int64_t i, float (&xr)[NCC], double& rr_n) {
    const int64_t rr = i + n;
    const int64_t rl = rr < i1 ? rr : i1 - 1;  // in bounds: every load is unconditional
    rr_n = a.rn[rl];
#pragma unroll
    for (int c = 0; c < NCC; ++c) {
      const int d = 4 * c + g;
      xr[c] = a.X32[rl * p + (d < p ? d : p - 1)];
    }
  };
  auto scan_tile = [&](int64_t i, const float (&xr)[NCC], double rr_n) {
    const int64_t rr = i + n;
    const bool valid = rr < i1;
    float bf[NCC];
    const float rn = valid ? (float)rr_n : __builtin_huge_valf();
#pragma unroll
    for (int c = 0; c < NCC; ++c) {
      const int d = 4 * c + g;
      bf[c] = (P > 0 && 4 * c + 3 < P) || d < p ? xr[c] : 0.0f;  // (chunks that may hold padding)
    }
    unsigned hit = 0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const float4 t4 = *reinterpret_cast<const float4*>(&nth_l[s][4 * g]);
      v4f acc = {rn + t4.x, rn + t4.y, rn + t4.z, rn + t4.w};
#pragma unroll
      for (int c = 0; c < NCC; ++c) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(af[s][c], bf[c], acc, 0, 0, 0);
      // the four sign bytes into one word (bits 7, 15, 23, 31), then bits 8 r + s
      const unsigned lo = __builtin_amdgcn_perm(__float_as_uint(acc[1]), __float_as_uint(acc[0]), 0x0c0c0703u);
      const unsigned hi = __builtin_amdgcn_perm(__float_as_uint(acc[3]), __float_as_uint(acc[2]), 0x07030c0cu);
      hit |= ((lo | hi) >> (7 - s)) & (0x01010101u << s);
    }
    hit &= locmask;
    if (!valid) hit = 0;
    const uint64_t bal = __ballot(hit != 0);
    if (!bal) return;
    if (hit) {
      const int pos = st_n + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                            __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
      st_row[pos] = (int32_t)rr;
      st_w[pos] = hit | ((uint32_t)g << 28);
    }
    st_n += __builtin_popcountll(bal);
    if (st_n > STG - 64) flush();
  };
#pragma unroll
  for (int d = 0; d < SD; ++d)
    if (i0 + 16 * d < i1) load_tile(i0 + 16 * d, xn[d], rnn[d]);
  for (int64_t ib = i0; ib < i1; ib += 16 * SD) {
#pragma unroll
    for (int d = 0; d < SD; ++d) {  // (static register sets)
      const int64_t i = ib + 16 * d;
      if (i < i1) {
        float xr[NCC];
#pragma unroll
        for (int c = 0; c < NCC; ++c) xr[c] = xn[d][c];
        const double rr_n = rnn[d];
        if (i + 16 * SD < i1) load_tile(i + 16 * SD, xn[d], rnn[d]);
        scan_tile(i, xr, rr_n);
      }
    }
  }
  flush();
}

// Squared row norms of the design and their maximum (for the scan's screen).
__global__ __launch_bounds__(256) void k_row_norms(const double* X, int64_t N, int p, double* rn,
                                                   unsigned long long* rmax_bits, float* X32) {
  double m = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int k = 0; k < p; ++k) {
      s = __builtin_fma(X[i * p + k], X[i * p + k], s);
      X32[i * p + k] = (float)X[i * p + k];
    }
    rn[i] = s;
    m = fmax(m, s);
  }
  for (int o = 32; o >= 1; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  // non-negative doubles order like their bit patterns
  if ((threadIdx.x & 63) == 0) atomicMax(rmax_bits, (unsigned long long)__builtin_bit_cast(long long, m));
}

hipError_t launch_row_norms(const double* X, int64_t N, int p, double* rn, double* rmax, float* X32,
                            hipStream_t s) {
  hipError_t e = hipMemsetAsync(rmax, 0, sizeof(double), s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_row_norms, dim3(1024), dim3(256), 0, s, X, N, p, rn,
                     reinterpret_cast<unsigned long long*>(rmax), X32);
  return hipGetLastError();
}

// Exact single-location scan with compaction (the fallback): the buffer
// (capacity >= S) receives rows beating the running threshold; whenever it
// could overflow it is sorted in LDS and cut back to the ncand best.
template <int P>
__device__ void knn_exact_one(const Knn2Args& a, int q, double* kd, int* ki, double* bd, int32_t* bi, double* sc,
                              int* si) {
  const int S = a.S;
  const int p = P > 0 ? P : a.p;
  const double* xq = a.XX + (int64_t)q * p;
  if (threadIdx.x == 0) {
    sc[0] = __builtin_huge_val();
    si[0] = 0x7fffffff;
    si[1] = 0;
  }
  __syncthreads();
  for (int64_t base = 0; base < a.N; base += blockDim.x) {
    const int64_t i = base + threadIdx.x;
    if (i < a.N) {
      const double* xr = a.X + i * p;
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < (P > 0 ? P : LAGP_MAX_DIM); ++k) {
        if (P > 0 || k < p) {
          const double u = xq[k] - xr[k];
          s = __builtin_fma(u, u, s);
        }
      }
      if (key_less(s, (int)i, sc[0], si[0])) {
        const int pos = atomicAdd(&si[1], 1);
        bd[pos] = s;
        bi[pos] = (int32_t)i;
      }
    }
    __syncthreads();
    const int c = si[1];
    if (c > S - (int)blockDim.x) {
      load_and_sort(bd, bi, c, kd, ki, S);
      for (int t = threadIdx.x; t < a.ncand; t += blockDim.x) {
        bd[t] = kd[t];
        bi[t] = ki[t];
      }
      if (threadIdx.x == 0) {
        sc[0] = kd[a.ncand - 1];
        si[0] = ki[a.ncand - 1];
        si[1] = a.ncand;
      }
      __syncthreads();
    }
  }
  load_and_sort(bd, bi, si[1], kd, ki, S);
}

// Bitonic sort of S = E * blockDim.x (key, row) pairs held E per thread in
// registers (thread t holds elements t E .. t E + E - 1), ascending by
// (key, row): the network of lds_bitonic_sort, with partners in the same
// thread compared in registers, partners in the same wave exchanged by
// shuffles, and only partners in other waves exchanged through LDS (kd, ki:
// S entries).  Same comparisons, same result.
template <int E, int ST>
__device__ __forceinline__ void bitonic_in_thread(double (&k)[E], int (&v)[E], int e0, int size) {
#pragma unroll
  for (int x = 0; x < E; ++x) {
    const int y = x ^ ST;
    if (y > x) {
      const bool up = ((e0 + x) & size) == 0;
      const bool sw = up ? key_less(k[y], v[y], k[x], v[x]) : key_less(k[x], v[x], k[y], v[y]);
      if (sw) {
        const double tk = k[x];
        k[x] = k[y];
        k[y] = tk;
        const int tv = v[x];
        v[x] = v[y];
        v[y] = tv;
      }
    }
  }
}

__device__ __forceinline__ void keep_of_pair(double& k, int& v, double pk, int pv, int e, int stride, int size) {
  const bool lower = (e & stride) == 0;  // e < e ^ stride
  const bool up = (e & size) == 0;
  const bool pk_less = key_less(pk, pv, k, v);
  // the lower position keeps the smaller when ascending, the larger otherwise
  const bool take = (lower == up) ? pk_less : !pk_less;
  if (take) {
    k = pk;
    v = pv;
  }
}

template <int E>
__device__ void reg_bitonic_sort(double (&k)[E], int (&v)[E], double* kd, int* ki) {
  const int t = threadIdx.x, S = E * blockDim.x;
  const int e0 = t * E;
  for (int size = 2; size <= S; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      if (stride < E) {
        if (stride == 1) bitonic_in_thread<E, 1>(k, v, e0, size);
        if constexpr (E > 2) if (stride == 2) bitonic_in_thread<E, 2>(k, v, e0, size);
        if constexpr (E > 4) if (stride == 4) bitonic_in_thread<E, 4>(k, v, e0, size);
        if constexpr (E > 8) if (stride == 8) bitonic_in_thread<E, 8>(k, v, e0, size);
      } else if (stride < 64 * E) {
        const int lx = stride / E;  // partner lane within the wave
#pragma unroll
        for (int x = 0; x < E; ++x) {
          const double pk = __shfl_xor(k[x], lx, 64);
          const int pv = __shfl_xor(v[x], lx, 64);
          keep_of_pair(k[x], v[x], pk, pv, e0 + x, stride, size);
        }
      } else {
#pragma unroll
        for (int x = 0; x < E; ++x) {
          kd[e0 + x] = k[x];
          ki[e0 + x] = v[x];
        }
        __syncthreads();
#pragma unroll
        for (int x = 0; x < E; ++x) {
          const int pe = (e0 + x) ^ stride;
          keep_of_pair(k[x], v[x], kd[pe], ki[pe], e0 + x, stride, size);
        }
        __syncthreads();
      }
    }
  }
}

// The merge with E pairs per thread in registers: sort the first S collected
// pairs, then stream the rest through positions ncand .. S-1 (as the LDS
// form below does), and write the ncand smallest.
template <int E>
__device__ void merge_regs(const Knn2Args& a, int q, double* kd, int* ki) {
  const int nc = a.ncand, t = threadIdx.x, e0 = t * E, S = E * blockDim.x;
  const double* bd = a.buf_d2 + (int64_t)q * a.CAP;
  const int32_t* bi = a.buf_idx + (int64_t)q * a.CAP;
  const int c = a.cnt[q];
  double k[E];
  int v[E];
  int taken = c < S ? c : S;
#pragma unroll
  for (int x = 0; x < E; ++x) {
    const int e = e0 + x;
    k[x] = e < taken ? bd[e] : __builtin_huge_val();
    v[x] = e < taken ? bi[e] : 0x7fffffff;
  }
  reg_bitonic_sort<E>(k, v, kd, ki);
  while (taken < c) {  // stream the rest through positions nc .. S-1
    const int add = (c - taken) < (S - nc) ? (c - taken) : (S - nc);
#pragma unroll
    for (int x = 0; x < E; ++x) {
      const int e = e0 + x;
      if (e >= nc) {
        const int src = e - nc;
        k[x] = src < add ? bd[taken + src] : __builtin_huge_val();
        v[x] = src < add ? bi[taken + src] : 0x7fffffff;
      }
    }
    reg_bitonic_sort<E>(k, v, kd, ki);
    taken += add;
  }
#pragma unroll
  for (int x = 0; x < E; ++x) {
    const int e = e0 + x;
    if (e < nc) {
      a.out_idx[(int64_t)q * nc + e] = v[x];
      if (a.out_d2) a.out_d2[(int64_t)q * nc + e] = k[x];
    }
  }
}

template <int P>
__global__ __launch_bounds__(KNN_THREADS) void k_knn_merge(Knn2Args a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int S = a.S;
  double* kd = reinterpret_cast<double*>(smem);
  double* sc = kd + S;
  int* ki = reinterpret_cast<int*>(sc + 2);
  int* si = ki + S;
  const int q = blockIdx.x;
  const int nc = a.ncand;
  double* bd = a.buf_d2 + (int64_t)q * a.CAP;
  int32_t* bi = a.buf_idx + (int64_t)q * a.CAP;
  const int c = a.cnt[q];
  if (c >= nc && c <= a.CAP && S == 8 * KNN_THREADS && blockDim.x == KNN_THREADS) {
    merge_regs<8>(a, q, kd, ki);
    return;
  }
  if (c >= nc && c <= a.CAP) {
    int taken = c < S ? c : S;
    load_and_sort(bd, bi, taken, kd, ki, S);
    while (taken < c) {
      const int add = (c - taken) < (S - nc) ? (c - taken) : (S - nc);
      for (int t = threadIdx.x; t < S - nc; t += blockDim.x) {
        if (t < add) {
          kd[nc + t] = bd[taken + t];
          ki[nc + t] = bi[taken + t];
        } else {
          kd[nc + t] = __builtin_huge_val();
          ki[nc + t] = 0x7fffffff;
        }
      }
      __syncthreads();
      lds_bitonic_sort(kd, ki, S);
      taken += add;
    }
  } else {
    knn_exact_one<P>(a, q, kd, ki, bd, bi, sc, si);
  }
  for (int t = threadIdx.x; t < nc; t += blockDim.x) {
    a.out_idx[(int64_t)q * nc + t] = ki[t];
    if (a.out_d2) a.out_d2[(int64_t)q * nc + t] = kd[t];
  }
}

static int64_t gcd64(int64_t x, int64_t y) {
  while (y) {
    const int64_t t = x % y;
    x = y;
    y = t;
  }
  return x;
}

// Rows the threshold aims to let through, about 2 n_t with n_t = ncand, or a
// quarter of the sort size for short lists (whose buffers hold at least the
// sort size anyway): a short list then still samples one row in eight or
// fewer instead of the whole design.
static int knn2_target(int ncand) {
  const int S4 = knn_sort_size(ncand) / 4;
  return ncand > S4 ? ncand : S4;
}

int64_t knn2_sub_rows(int64_t N, int ncand) {
  int64_t r = (2 * (int64_t)knn2_target(ncand)) / KSEL;
  if (r < 1) r = 1;
  return (N + r - 1) / r;
}

size_t knn2_shared_bytes(int64_t N, int p, int ncand) {
  return ((size_t)knn2_sub_rows(N, ncand) * p * sizeof(double) + 255) & ~size_t(255);
}

int knn2_capacity(int ncand) {
  const int S = knn_sort_size(ncand);
  return 4 * ncand > S ? 4 * ncand : S;
}

size_t knn2_bytes_per_location(int ncand) {
  return (size_t)knn2_capacity(ncand) * (sizeof(double) + sizeof(int32_t)) + sizeof(double) + sizeof(int32_t);
}

size_t knn2_merge_lds_bytes(int S) { return (size_t)S * (sizeof(double) + sizeof(int)) + 2 * sizeof(double) + 2 * sizeof(int); }

template <int P>
static hipError_t launch_knn2_p(Knn2Args a, hipStream_t s) {
  const int groups = (a.M + 63) / 64;
  // enough subsample parts for about 8192 waves (the pass is latency-bound;
  // short lists keep each wave's insertions cheap); KSEL <= KT * parts <= 256
  // <= CAP
  int parts = (8192 + groups - 1) / groups;
  if (parts > KPARTS) parts = KPARTS;
  if (parts < KSEL / KT) parts = KSEL / KT;
  if ((int64_t)parts > a.sub_count) parts = (int)a.sub_count;
  if (parts < 1) parts = 1;
  const int64_t gn = a.sub_count * a.p;
  hipLaunchKernelGGL(k_knn_gather_sub, dim3((unsigned)((gn + 255) / 256)), dim3(256), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_knn_tau<P>, dim3(parts, groups), dim3(64), 0, s, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_knn_tau_reduce, dim3(a.M), dim3(64), 0, s, a, parts);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // The FP32 screen when its slack (which grows with the squared norms) stays
  // under 5% of an estimate of the threshold (the squared radius holding
  // ncand of N points spread over the design's extent); designs far from the
  // origin relative to their extent keep the FP64 screen, whose slack is
  // 2^29 times smaller.  Either way the lists are exact.
  constexpr int K32 = 4 * (((P > 0 ? P : LAGP_MAX_DIM) + 3) / 4) + 4;  // k_knn_scan32's bound constant
  const double tau_est = a.spread2 * pow((double)a.ncand / (double)a.N, 2.0 / a.p);
  const double slack32 = 4.0 * (K32 + 4) * 0x1p-24 * (5.0 * a.rn_max + tau_est);
  const bool fp32 = a.X32 && a.rn_max <= 1e30 && slack32 <= 0.05 * tau_est;
  // scan: groups of 64 locations x slices of the design, three rounds of the
  // scan's resident waves (shorter slices hide the tail of the last round);
  // the groups vary fastest, so the waves that read one slice run together
  // and share it through L2
  const int sgroups = (a.M + 63) / 64;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                              hipSuccess || cus < 1)
    cus = 256;
  const int64_t waves = (int64_t)3 * 4 * cus * (fp32 ? SCAN32_WAVES : 7);  // (4 SIMDs per CU)
  int64_t nsl = (waves + sgroups - 1) / sgroups;
  const int64_t maxsl = (a.N + 1023) / 1024;
  if (nsl > maxsl) nsl = maxsl;
  if (nsl < 1) nsl = 1;
  a.slice = (a.N + nsl - 1) / nsl;
  if (fp32)
    hipLaunchKernelGGL(k_knn_scan32<P>, dim3(sgroups, (unsigned)((a.N + a.slice - 1) / a.slice)), dim3(64), 0, s, a);
  else
    hipLaunchKernelGGL(k_knn_scan<P>, dim3(sgroups, (unsigned)((a.N + a.slice - 1) / a.slice)), dim3(64), 0, s, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t lds = knn2_merge_lds_bytes(a.S);
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_knn_merge<P>), hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_knn_merge<P>, dim3(a.M), dim3(KNN_THREADS), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_knn2(Knn2Args a, hipStream_t s) {
  if (a.M <= 0) return hipSuccess;
  a.S = knn_sort_size(a.ncand);
  a.CAP = knn2_capacity(a.ncand);
  // subsample: one row in r, r = 2 n_t / KSEL, so that about 2 n_t >= 2 ncand
  // design rows fall under the KSEL-th smallest sampled distance
  a.sub_count = knn2_sub_rows(a.N, a.ncand);
  int64_t A = (int64_t)((double)a.N * 0.6180339887498949) | 1;
  if (A >= a.N) A = 1;
  while (gcd64(A, a.N) != 1) A += 2;
  a.sub_stride = A % a.N;
  if (a.N == 1) a.sub_stride = 0;
  switch (a.p) {
    case 1: return launch_knn2_p<1>(a, s);
    case 2: return launch_knn2_p<2>(a, s);
    case 3: return launch_knn2_p<3>(a, s);
    case 4: return launch_knn2_p<4>(a, s);
    case 8: return launch_knn2_p<8>(a, s);
    default: return launch_knn2_p<0>(a, s);
  }
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
