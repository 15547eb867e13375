// Exhaustive greedy local designs by incremental Cholesky columns for the
// shapes whose columns do not fit on chip (n up to LAGP_MAX_N, N' up to
// LAGP_MAX_NCAND): the same recursion as chol.hip, with every candidate's
// column u_c = L^{-1} k_J(x_c) kept in a workspace in device memory.
//
// With K_J + g I = L L^T, candidate c carries u_c and
//   v_c = (1 + g) - u_c^T u_c,  cov_c = K(x_c, x) - w_x^T u_c,  q_c = y_c - z^T u_c
// (w_x = L^{-1} k_J(x), z = L^{-1} y_J), and its criterion of Sec. 3.1 (the
// integrand of Eq. alc at x) is cov_c^2 / v_c.  Taking candidate t appends
// e_c = (K(x_t, x_c) - u_t^T u_c) (1 / sqrt(v_t)) to every other column and
// drops e_c^2, (cov_t / sqrt(v_t)) e_c and (q_t / sqrt(v_t)) e_c from v_c,
// cov_c and q_c.  After n points mean = w_x^T z and the scale is
// z^T z ((1 + g) - w_x^T w_x) / n (Eqs. predgp, preds2 with n local points).
//
// A step streams the j entries of every column once (the inner products
// u_t^T u_c) and appends one: Sum_j 8 j N' bytes per location, so the kernel
// is bound by device-memory bandwidth.  Layout: a workgroup owns a slice of
// the workspace, rows of ncw doubles (ncw = 4 x the workgroup size): n rows
// of u entries (row k holds entry k of every column) and p rows of candidate
// coordinates; thread t holds candidates CPT t .. CPT t + CPT - 1 (CPT = 4, or
// 8 past N' = 2048), so a row is read as CPT / 4 32-byte loads per thread,
// coalesced across the wave.  The grid is
// persistent (as many workgroups as fit on the device at once, each looping
// over locations), so the workspace does not grow with the number of
// locations.  Sums, the exp and the order of every operation are those of
// the on-chip kernel: results are the same bit for bit.
#include <atomic>
#include <cstdlib>

#include "dev_math.h"
#include "lagp_internal.h"

namespace lagp {

namespace {

constexpr int CW_MAXT = 512;      // largest workgroup (8 candidates per thread: N' <= 4096)
constexpr int CW_MAXW = CW_MAXT / 64;

typedef double d4 __attribute__((ext_vector_type(4)));

struct CwLds {
  double slotv[CW_MAXW];    // per wave: its best criterion
  double slot2[CW_MAXW];    // per wave: its runner-up
  double slotd[CW_MAXW][3]; // per wave: v, cov, q of its best
  int sloti[CW_MAXW];       // per wave: rank of its best (-1: none)
  double uw[LAGP_MAX_N];    // the chosen candidate's column
  double xw[LAGP_MAX_DIM];  // its coordinates
  double x[LAGP_MAX_DIM];   // the location
  double w[LAGP_MAX_DIM];   // reciprocal lengthscales (separable), 1 (isotropic)
  double ec[12];            // Taylor coefficients of exp (read per use, not held in registers)
  int J[LAGP_MAX_N];        // design ranks in selection order
};

// DPP move of a 32-bit key; rows outside ROWMASK keep v.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ uint32_t cw_dpp_u(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWMASK, 0xF, false);
}

__device__ __forceinline__ uint32_t cw_wave_max_u(uint32_t v) {
  v = max(v, cw_dpp_u<0xB1, 0xF>(v));   // quad_perm [1,0,3,2]
  v = max(v, cw_dpp_u<0x4E, 0xF>(v));   // quad_perm [2,3,0,1]
  v = max(v, cw_dpp_u<0x141, 0xF>(v));  // row_half_mirror
  v = max(v, cw_dpp_u<0x140, 0xF>(v));  // row_mirror
  v = max(v, cw_dpp_u<0x142, 0xA>(v));  // row_bcast:15
  v = max(v, cw_dpp_u<0x143, 0xC>(v));  // row_bcast:31
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Ballot of the lanes holding the wave's largest criterion (>= 0; anything
// else, NaN included, offers nothing): non-negative doubles order like
// their bit patterns, so the maximum is taken on the high words, then on the
// low words of the lanes tied there.
__device__ __forceinline__ uint64_t cw_wave_argmax(double sc) {
  const uint64_t b = __builtin_bit_cast(uint64_t, sc);
  const bool ok = sc >= 0.0;
  const uint32_t hi = ok ? (uint32_t)(b >> 32) | 0x80000000u : 0u;
  const uint32_t lo = (uint32_t)b;
  const uint32_t mhi = cw_wave_max_u(hi);
  const uint32_t mlo = cw_wave_max_u(hi == mhi ? lo : 0u);
  return __ballot(ok && hi == mhi && lo == mlo);
}

__device__ __forceinline__ double cw_readlane(double v, int l) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Maximum of a non-negative-or-negative double over the wave (every lane).
__device__ __forceinline__ double cw_wave_max(double v) {
  for (int m = 32; m >= 1; m >>= 1) v = fmax(v, __shfl_xor(v, m, 64));
  return v;
}

__device__ __forceinline__ double cw_score(double v, double cov, bool act, int& vflag) {
  if (!act) return -1.0;
  double sc;
  if (v > 0.0) {
    sc = cov * cov / v;
  } else {
    sc = 0.0;
    vflag = 1;
  }
  return sc >= 0.0 ? sc : -1.0;  // NaN: never chosen
}

// CPT: candidates per thread (4 or 8, consecutive ranks), read as CPT / 4
// 32-byte pieces per row.
template <int CPT, bool DIAG>
__global__ __launch_bounds__(CW_MAXT) void k_cholw(LocalArgs a) {
  constexpr int CW_CPT = CPT;
  constexpr int NV = CPT / 4;
  constexpr int CW_ROWS = 16 / CPT;  // column rows loaded ahead in the inner products (128 bytes a thread)
  __shared__ CwLds L;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nwv = blockDim.x >> 6;
  const int ncw = CW_CPT * blockDim.x;  // row length of this workgroup's slice
  const int p = a.p, n = a.n, n0 = a.n0, nc = a.ncand;
  const int c0 = CW_CPT * tid;
  double* U = a.cw + (size_t)blockIdx.x * (size_t)(n + p) * ncw;  // n rows of u entries
  double* Xs = U + (size_t)n * ncw;                               // p rows of coordinates
  if (tid < 12) L.ec[tid] = gexp_coef(tid);
  if (tid < LAGP_MAX_DIM) L.w[tid] = (a.dlen == 1 || tid >= p) ? 1.0 : a.w[tid];
  const auto coef = [&](int i) { return L.ec[i]; };

  for (int m = blockIdx.x; m < a.M; m += gridDim.x) {  // persistent: every workgroup reaches M
    double w0 = a.w[0];
    if (a.dloc) {
      const double dl = a.dloc[m];
      if (!(dl > 0.0)) {  // a location without a usable lengthscale is skipped
        if (tid == 0) a.status[m] = 0;
        continue;  // (uniform over the workgroup)
      }
      w0 = 1.0 / dl;
    }
    const int32_t* C = a.cand + (int64_t)m * nc;
    if (tid < LAGP_MAX_DIM) L.x[tid] = tid < p ? a.XX[(int64_t)m * p + tid] : 0.0;
    __syncthreads();
    // prologue: coordinates into the slice, the starting v, cov, q
    double v[CW_CPT], cov[CW_CPT], q[CW_CPT];
    bool act[CW_CPT];
    int vflag = 0;
#pragma unroll
    for (int i = 0; i < CW_CPT; ++i) {
      const int c = c0 + i;
      act[i] = c < nc;
      v[i] = 1.0 + a.g;
      cov[i] = 0.0;
      q[i] = 0.0;
      if (act[i]) {  // K(x_c, x): candidate first, dimensions in order
        const int64_t row = C[c];
        double s = 0.0;
        for (int k = 0; k < p; ++k) {
          const double xk = a.X[row * p + k];
          Xs[(size_t)k * ncw + c] = xk;
          const double t = xk - L.x[k];
          s = a.dlen == 1 ? __builtin_fma(t, t, s) : __builtin_fma(t * t, L.w[k], s);
        }
        cov[i] = gexp_with(a.dlen == 1 ? -(s * w0) : -s, coef);
        q[i] = a.y[row];
      } else {
        for (int k = 0; k < p; ++k) Xs[(size_t)k * ncw + c] = 0.0;
      }
    }
    double mu = 0.0, psi = 0.0, qq = 0.0;  // (meaningful in thread 0)
    bool pd = true;
    int done = 0;
    for (int j = 0; j < n; ++j) {
      // 1. each wave's best: forced to rank j while j < n0, else the largest
      //    criterion, lowest rank on ties
      double sc[CW_CPT];
#pragma unroll
      for (int i = 0; i < CW_CPT; ++i)
        sc[i] = j < n0 ? (c0 + i == j ? 0.0 : -1.0) : cw_score(v[i], cov[i], act[i], vflag);
      int pk = 0;
      double pb = sc[0];
#pragma unroll
      for (int i = 1; i < CW_CPT; ++i)
        if (sc[i] > pb) {
          pb = sc[i];
          pk = i;
        }
      double p2 = -1.0;  // the thread's runner-up
#pragma unroll
      for (int i = 0; i < CW_CPT; ++i)
        if (i != pk) p2 = fmax(p2, sc[i]);
      const uint64_t hit = cw_wave_argmax(pb);
      const int wl = hit ? __builtin_ctzll(hit) : -1;
      if (lane == wl) {
        L.slotv[wv] = pb;
        L.sloti[wv] = c0 + pk;
        double vv = v[0], cc = cov[0], qv = q[0];
#pragma unroll
        for (int i = 1; i < CW_CPT; ++i)
          if (pk == i) {
            vv = v[i];
            cc = cov[i];
            qv = q[i];
          }
        L.slotd[wv][0] = vv;
        L.slotd[wv][1] = cc;
        L.slotd[wv][2] = qv;
      }
      if (DIAG) {
        const double s2w = cw_wave_max(lane == wl ? p2 : pb);
        if (lane == 0) L.slot2[wv] = s2w;
      }
      if (wl < 0 && lane == 0) L.sloti[wv] = -1;
      __syncthreads();
      // 2. the best over waves (the earliest wave, lowest ranks, on ties)
      double cv = -1.0, c2 = -1.0;
      int ci = -1;
      if (lane < nwv) {
        ci = L.sloti[lane];
        cv = ci >= 0 ? L.slotv[lane] : -1.0;
        if (DIAG) c2 = L.slot2[lane];
      }
      const uint64_t gh = cw_wave_argmax(cv);
      if (!gh) break;  // no finite criterion anywhere: no prediction (uniform)
      const int ql = __builtin_ctzll(gh);
      const int w = __builtin_amdgcn_readlane(ci, ql);
      const double b1 = cw_readlane(cv, ql);
      double b2 = 0.0;
      if (DIAG) b2 = cw_wave_max(lane == ql ? c2 : fmax(cv, c2));
      const double vw = L.slotd[ql][0], covw = L.slotd[ql][1], qw = L.slotd[ql][2];
      if (j < n0 && !(vw > 0.0)) {  // the starting covariance is not positive definite
        pd = false;
        break;
      }
      if (!(vw > 0.0)) vflag = 1;
      const double li = 1.0 / __builtin_sqrt(vw);
      const double wj = covw * li, zj = qw * li;
      if (tid == 0) {
        L.J[j] = w;
        mu = __builtin_fma(wj, zj, mu);
        psi = __builtin_fma(zj, zj, psi);
        qq = __builtin_fma(wj, wj, qq);
        if (DIAG && j >= n0 && a.diag) {
          double* dg = a.diag + ((int64_t)m * (n - n0) + (j - n0)) * 2;
          dg[0] = b1;
          dg[1] = b2 < 0.0 ? -__builtin_huge_val() : b2;
        }
        if (j >= n0 && a.counts) {
          int32_t* ct = a.counts + ((int64_t)m * (n - n0) + (j - n0)) * 2;
          ct[0] = nc - j;
          ct[1] = 0;
        }
      }
#pragma unroll
      for (int i = 0; i < CW_CPT; ++i)
        if (c0 + i == w) act[i] = false;
      done = j + 1;
      if (j + 1 == n) break;
      // 3. the chosen column and coordinates to LDS
      for (int k = tid; k < j; k += blockDim.x) L.uw[k] = U[(size_t)k * ncw + w];
      if (tid < p) L.xw[tid] = Xs[(size_t)tid * ncw + w];
      __syncthreads();
      // 4. extend every column: kernel value, inner product, new entry
      // K(x_t, x_c): the chosen point first, dimensions in order
      double kv[CW_CPT];
#pragma unroll
      for (int i = 0; i < CW_CPT; ++i) kv[i] = 0.0;
      for (int k = 0; k < p; ++k) {
        d4 r[NV];
#pragma unroll
        for (int h = 0; h < NV; ++h) r[h] = *reinterpret_cast<const d4*>(Xs + (size_t)k * ncw + c0 + 4 * h);
        const double xk = L.xw[k];
        const double wk = L.w[k];
#pragma unroll
        for (int i = 0; i < CW_CPT; ++i) {
          const double t = xk - r[i / 4][i % 4];
          kv[i] = a.dlen == 1 ? __builtin_fma(t, t, kv[i]) : __builtin_fma(t * t, wk, kv[i]);
        }
      }
#pragma unroll
      for (int i = 0; i < CW_CPT; ++i) kv[i] = gexp_with(a.dlen == 1 ? -(kv[i] * w0) : -kv[i], coef);
      double d[CW_CPT];
#pragma unroll
      for (int i = 0; i < CW_CPT; ++i) d[i] = 0.0;
      const double* up = U + c0;
      int k = 0;
      for (; k + CW_ROWS <= j; k += CW_ROWS) {  // CW_ROWS rows in flight, summed in row order
        d4 r[CW_ROWS][NV];
#pragma unroll
        for (int h = 0; h < CW_ROWS; ++h)
#pragma unroll
          for (int g = 0; g < NV; ++g) r[h][g] = *reinterpret_cast<const d4*>(up + (size_t)(k + h) * ncw + 4 * g);
#pragma unroll
        for (int h = 0; h < CW_ROWS; ++h) {
          const double uk = L.uw[k + h];
#pragma unroll
          for (int i = 0; i < CW_CPT; ++i) d[i] = __builtin_fma(uk, r[h][i / 4][i % 4], d[i]);
        }
      }
      for (; k < j; ++k) {
        d4 r[NV];
#pragma unroll
        for (int g = 0; g < NV; ++g) r[g] = *reinterpret_cast<const d4*>(up + (size_t)k * ncw + 4 * g);
        const double uk = L.uw[k];
#pragma unroll
        for (int i = 0; i < CW_CPT; ++i) d[i] = __builtin_fma(uk, r[i / 4][i % 4], d[i]);
      }
      d4 e[NV];
#pragma unroll
      for (int i = 0; i < CW_CPT; ++i) {
        const double ei = (kv[i] - d[i]) * li;
        e[i / 4][i % 4] = ei;
        v[i] = __builtin_fma(-ei, ei, v[i]);
        cov[i] = __builtin_fma(-wj, ei, cov[i]);
        q[i] = __builtin_fma(-zj, ei, q[i]);
      }
#pragma unroll
      for (int g = 0; g < NV; ++g) *reinterpret_cast<d4*>(U + (size_t)j * ncw + c0 + 4 * g) = e[g];
      __syncthreads();  // the slots and the chosen column are rewritten by the next step
    }
    const int vf = __syncthreads_or(vflag);
    if (tid == 0) {
      const bool ok = pd && done == n;
      double mean = __builtin_nan(""), sc = __builtin_nan("");
      if (ok) {
        mean = mu;
        sc = psi * ((1.0 + a.g) - qq) / (double)n;
      }
      int st = 0;
      if (!pd) st |= LAGP_STATUS_NOTPD;
      if (vf) st |= LAGP_STATUS_VNONPOS;
      if (!(fabs(mean) <= 1.7976931348623157e308 && fabs(sc) <= 1.7976931348623157e308)) st |= LAGP_STATUS_NONFINITE;
      a.mean[m] = mean;
      a.s2[m] = sc;
      a.df[m] = (double)n;
      a.status[m] = st;
    }
    if (a.sel) {
      const int dn = pd ? done : n0;  // not positive definite: report the n0 nearest
      for (int i = tid; i < n; i += blockDim.x) a.sel[(int64_t)m * n + i] = i < dn ? C[pd ? L.J[i] : i] : -1;
    }
    __syncthreads();  // L.J and L.x are rewritten by the next location
  }
}

// Candidates per thread and workgroup size for a candidate count.
int cw_cpt(int ncand) { return ncand <= 4 * CW_MAXT ? 4 : 8; }
int cw_threads(int ncand) {
  const int c = cw_cpt(ncand);
  return 64 * ((ncand + 64 * c - 1) / (64 * c));
}

}  // namespace

size_t chol_stream_slot_bytes(int n, int ncand, int p) {
  return sizeof(double) * (size_t)(n + p) * (size_t)(cw_cpt(ncand) * cw_threads(ncand));
}

int chol_stream_max_slots(int ncand) {
  // resident workgroups per device, per kernel variant (cached: admission
  // control asks for it per request)
  static std::atomic<int> cached[2][64] = {};
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  const int v = cw_cpt(ncand) == 4 ? 0 : 1;
  if (dev >= 0 && dev < 64 && cached[v][dev].load() > 0) return cached[v][dev].load();
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
  const void* fn = cw_cpt(ncand) == 4 ? reinterpret_cast<const void*>(&k_cholw<4, true>)
                                      : reinterpret_cast<const void*>(&k_cholw<8, true>);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, cw_threads(ncand), 0) != hipSuccess || per < 1)
    per = 1;
  if (dev >= 0 && dev < 64) cached[v][dev].store(cus * per);
  return cus * per;
}

bool chol_stream_forced() {
  const char* s = std::getenv("LAGP_CHOL_FORCE_STREAM");
  return s && s[0] == '1';
}

hipError_t launch_chol_stream(const LocalArgs& a, int slots, hipStream_t s) {
  if (a.M <= 0) return hipSuccess;
  const int grid = a.M < slots ? a.M : slots;
  const int T = cw_threads(a.ncand);
  if (cw_cpt(a.ncand) == 4) {
    if (a.diag)
      hipLaunchKernelGGL((k_cholw<4, true>), dim3(grid), dim3(T), 0, s, a);
    else
      hipLaunchKernelGGL((k_cholw<4, false>), dim3(grid), dim3(T), 0, s, a);
  } else {
    if (a.diag)
      hipLaunchKernelGGL((k_cholw<8, true>), dim3(grid), dim3(T), 0, s, a);
    else
      hipLaunchKernelGGL((k_cholw<8, false>), dim3(grid), dim3(T), 0, s, a);
  }
  return hipGetLastError();
}

}  // namespace lagp
