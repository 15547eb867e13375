// Exhaustive greedy local designs by incremental Cholesky columns, one
// workgroup per location and one thread per candidate.
//
// With K_J + g I = L L^T for the design J chosen so far, candidate c carries
// u_c = L^{-1} k_J(x_c) and three scalars
//   v_c   = (1 + g) - u_c^T u_c          the Schur complement v_j of Eq. (alc)
//   cov_c = K(x_c, x) - w_x^T u_c         with w_x = L^{-1} k_J(x)
//   q_c   = y_c - z^T u_c                 with z   = L^{-1} y_J
// since k_J(x_c)^T K_J^{-1} k_J(x) = u_c^T w_x, the criterion of Sec. 3.1
// (the integrand of Eq. (alc) at the location itself) is cov_c^2 / v_c.
// Adding candidate w appends the row (u_w^T, l) to L with l = sqrt(v_w).
// Every other candidate gains the entry
//   e_c = (K(x_w, x_c) - u_w^T u_c) / l
// and v_c -= e_c^2, cov_c -= (cov_w / l) e_c, q_c -= (q_w / l) e_c; the new
// entries of w_x and z are cov_w / l and q_w / l.  After n points
//   mean = w_x^T z,  psi = z^T z,  k_x^T K^{-1} k_x = w_x^T w_x
// give Eqs. (predgp), (preds2) with n local points.  The starting design
// (the n0 nearest, Sec. 2.2) is the same recursion with the choice forced.
//
// A step costs one length-j inner product per candidate instead of the
// j x j contraction of the partitioned-inverse form, and a location's whole
// state (u_c in registers, candidate coordinates in LDS) stays on chip, so
// the search reads nothing from memory after its prologue.  It computes the
// same criterion and prediction in a different rounding order: results agree
// with the partitioned-inverse definition to rounding, not bit for bit.
#include "dev_math.h"
#include "lagp_internal.h"

namespace lagp {

namespace {

constexpr int CH_CHUNK = 8;  // u entries per statically indexed block

// NU: u entries kept per candidate (designs up to NU + 1 points); PM:
// coordinate rows (p <= PM, rows p .. PM-1 zero); TS: LDS row stride and
// largest workgroup (N' <= TS).
template <int NU, int PM, int TS>
struct ChCfg {
  // the first UL entries of every u_c live in LDS (ul[k * TS + c]), the rest
  // in registers
  static constexpr int UL = NU > 32 ? CH_CHUNK : 0;
  static constexpr int NUP = (NU + CH_CHUNK - 1) / CH_CHUNK * CH_CHUNK;
  static constexpr int SS = NUP + 4;  // slot: u (zero padded), v, cov, q, pad
  static constexpr int NCH = NU / CH_CHUNK + 1;  // step blocks: j = 0 .. NU
  static constexpr int NWV = TS / 64;
};

// LDS: coordinates by dimension (PM x TS), the leading u entries (UL x TS),
// two parities of per-wave slots and reduction words, the location, the
// design ranks.
struct ChLds {
  double* xs;
  double* ul;
  double* slot;  // 2 x NWV x SS
  double* redv;  // 2 x NWV: best criterion of each wave
  double* red2;  // 2 x NWV: runner-up of each wave
  double* x;     // LAGP_MAX_DIM
  double* ec;    // 12: the Taylor coefficients of exp (read per use, not held in registers)
  int* redi;     // 2 x NWV: rank of each wave's best
  int* J;        // n
};

__host__ __device__ constexpr size_t ch_lds_bytes(int PM, int TS, int UL, int SS, int n) {
  return sizeof(double) * ((size_t)(PM + UL) * TS + 2 * (size_t)(TS / 64) * SS + 4 * (size_t)(TS / 64) +
                           LAGP_MAX_DIM + 12) +
         sizeof(int) * (2 * (size_t)(TS / 64) + (size_t)n);
}

template <int NU, int PM, int TS>
__device__ inline ChLds ch_carve(unsigned char* s) {
  using C = ChCfg<NU, PM, TS>;
  ChLds L;
  L.xs = reinterpret_cast<double*>(s);
  L.ul = L.xs + PM * TS;
  L.slot = L.ul + C::UL * TS;
  L.redv = L.slot + 2 * C::NWV * C::SS;
  L.red2 = L.redv + 2 * C::NWV;
  L.x = L.red2 + 2 * C::NWV;
  L.ec = L.x + LAGP_MAX_DIM;
  L.redi = reinterpret_cast<int*>(L.ec + 12);
  L.J = L.redi + 2 * C::NWV;
  return L;
}

// Gaussian correlation between candidates ca and cb (columns of xs) in the
// rounding of corr(): dimension order, one fused multiply-add per term (the
// zero rows past p add exact zeros).
template <int PM, int TS>
__device__ __forceinline__ double ch_corr(const double* xs, const double* ec, int ca, int cb, const LocalArgs& A) {
  const auto coef = [ec](int i) { return ec[i]; };
  double s = 0.0;
  if (A.dlen == 1) {
#pragma unroll
    for (int k = 0; k < PM; ++k) {
      const double t = xs[k * TS + ca] - xs[k * TS + cb];
      s = __builtin_fma(t, t, s);
    }
    return gexp_with(-(s * A.w[0]), coef);
  }
#pragma unroll
  for (int k = 0; k < PM; ++k) {
    const double t = xs[k * TS + ca] - xs[k * TS + cb];
    s = __builtin_fma(t * t, A.w[k], s);
  }
  return gexp_with(-s, coef);
}

// Per-thread state of one candidate (u entries below UL are in LDS).
template <int NU>
struct ChState {
  double u[NU];
  double v, cov, q;
  bool act;
  int vflag;
};

// Per-location running results (meaningful in thread 0).
struct ChRun {
  double mu, psi, qq;
  int done;
  bool pd, stop;
};

template <int NU, int PM, int TS, int B>
__device__ __forceinline__ void ch_write_slot(double* sl, const ChState<NU>& S, const ChLds& L) {
  using C = ChCfg<NU, PM, TS>;
  constexpr int KE = (B + 1) * CH_CHUNK < NU ? (B + 1) * CH_CHUNK : NU;
#pragma unroll
  for (int k = 0; k < KE; ++k) sl[k] = k < C::UL ? L.ul[k * TS + threadIdx.x] : S.u[k];
  sl[C::NUP] = S.v;
  sl[C::NUP + 1] = S.cov;
  sl[C::NUP + 2] = S.q;
}

// Steps j = B*CH_CHUNK .. B*CH_CHUNK + CH_CHUNK - 1: choose design point j
// (forced to rank j while j < n0, else the largest criterion, lowest rank on
// ties), publish its column, extend every other candidate's.
template <int NU, int PM, int TS, bool DIAG, int B>
__device__ __forceinline__ void ch_block(const LocalArgs& a, const ChLds& L, ChState<NU>& S, ChRun& R, int64_t m) {
  using C = ChCfg<NU, PM, TS>;
  constexpr int NUP = C::NUP, SS = C::SS, UL = C::UL, NWV = C::NWV;
  constexpr int KE = (B + 1) * CH_CHUNK < NU ? (B + 1) * CH_CHUNK : NU;  // u entries in use up to this block
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nwv = blockDim.x >> 6;
  const int n = a.n, n0 = a.n0;
  for (int jj = 0; jj < CH_CHUNK; ++jj) {
    const int j = B * CH_CHUNK + jj;
    if (j >= n || R.stop) return;
    const int par = j & 1;
    double* sl = L.slot + par * NWV * SS;
    if (j < n0) {
      if (tid == j) ch_write_slot<NU, PM, TS, B>(sl + wv * SS, S, L);
    } else {
      double sc = -1.0;
      if (S.act) {
        if (S.v > 0.0) {
          sc = S.cov * S.cov / S.v;
        } else {
          sc = 0.0;
          S.vflag = 1;
        }
        if (!(sc >= 0.0)) sc = -1.0;  // NaN: never chosen
      }
      // wave maximum, then its lowest lane
      double wmax = sc;
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) wmax = fmax(wmax, __shfl_xor(wmax, o, 64));
      const uint64_t hit = __ballot(sc == wmax && wmax >= 0.0);
      const int wl = hit ? __builtin_ctzll(hit) : -1;
      if (lane == wl) ch_write_slot<NU, PM, TS, B>(sl + wv * SS, S, L);
      if constexpr (DIAG) {
        double s2 = lane == wl ? -1.0 : sc;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) s2 = fmax(s2, __shfl_xor(s2, o, 64));
        if (lane == 0) L.red2[par * NWV + wv] = s2;
      }
      if (lane == 0) {
        L.redv[par * NWV + wv] = wl >= 0 ? wmax : -1.0;
        L.redi[par * NWV + wv] = wl >= 0 ? (wv << 6) + wl : -1;
      }
    }
    __syncthreads();
    int w = j;
    double b1 = 0.0, b2 = 0.0;
    if (j >= n0) {
      // earliest wave wins ties: rank order
      b1 = -1.0;
      b2 = -1.0;
      w = -1;
      for (int qw = 0; qw < nwv; ++qw) {
        const double cv = L.redv[par * NWV + qw];
        const int ci = L.redi[par * NWV + qw];
        const double c2 = DIAG ? L.red2[par * NWV + qw] : -1.0;
        if (ci >= 0 && cv > b1) {
          b2 = fmax(b1, c2);
          b1 = cv;
          w = ci;
        } else {
          b2 = fmax(b2, ci >= 0 ? cv : -1.0);
          if (DIAG) b2 = fmax(b2, c2);
        }
      }
      if (w < 0) {  // no finite criterion anywhere: give up on x
        R.stop = true;
        return;
      }
    }
    w = __builtin_amdgcn_readfirstlane(w);
    const double* ws = sl + (w >> 6) * SS;
    const double vw = ws[NUP], covw = ws[NUP + 1], qw = ws[NUP + 2];
    if (j < n0 && !(vw > 0.0)) {  // the starting covariance is not positive definite
      R.pd = false;
      R.stop = true;
      return;
    }
    if (!(vw > 0.0)) S.vflag = 1;
    const double l = __builtin_sqrt(vw);
    const double wxj = covw / l, zj = qw / l;
    if (tid == 0) {
      L.J[j] = w;
      R.mu = __builtin_fma(wxj, zj, R.mu);
      R.psi = __builtin_fma(zj, zj, R.psi);
      R.qq = __builtin_fma(wxj, wxj, R.qq);
      if (DIAG && j >= n0 && a.diag) {
        double* dg = a.diag + (m * (n - n0) + (j - n0)) * 2;
        dg[0] = b1;
        dg[1] = b2 < 0.0 ? -__builtin_huge_val() : b2;
      }
    }
    if (tid == w) S.act = false;
    R.done = j + 1;
    if (j + 1 < n && S.act) {
      const double kv = ch_corr<PM, TS>(L.xs, L.ec, w, tid, a);
      double dot = 0.0;
#pragma unroll
      for (int k = 0; k < KE; ++k) dot = __builtin_fma(ws[k], k < UL ? L.ul[k * TS + tid] : S.u[k], dot);
      const double e = (kv - dot) / l;
#pragma unroll
      for (int kk = 0; kk < CH_CHUNK; ++kk) {
        constexpr int K0 = B * CH_CHUNK;
        if (K0 + kk < NU && kk == jj) {
          if (K0 + kk < UL)
            L.ul[(K0 + kk) * TS + tid] = e;
          else
            S.u[K0 + kk < NU ? K0 + kk : 0] = e;
        }
      }
      S.v = __builtin_fma(-e, e, S.v);
      S.cov = __builtin_fma(-wxj, e, S.cov);
      S.q = __builtin_fma(-zj, e, S.q);
    }
  }
}

template <int NU, int PM, int TS, bool DIAG, int B>
__device__ __forceinline__ void ch_blocks(const LocalArgs& a, const ChLds& L, ChState<NU>& S, ChRun& R, int64_t m) {
  if constexpr (B < ChCfg<NU, PM, TS>::NCH) {
    ch_block<NU, PM, TS, DIAG, B>(a, L, S, R, m);
    if (!R.stop && (B + 1) * CH_CHUNK < a.n) ch_blocks<NU, PM, TS, DIAG, B + 1>(a, L, S, R, m);
  }
}

// One workgroup of 64 ceil(N'/64) <= TS threads per location, thread c for
// the candidate of rank c.
template <int NU, int PM, int TS, bool DIAG>
__global__ __launch_bounds__(TS) __attribute__((amdgpu_waves_per_eu(4))) void k_chol(LocalArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  using Cf = ChCfg<NU, PM, TS>;
  const ChLds L = ch_carve<NU, PM, TS>(smem);
  const int tid = threadIdx.x;
  const int64_t m = blockIdx.x;
  const int p = a.p, n = a.n, nc = a.ncand;
  const int32_t* C = a.cand + m * nc;

  if (tid < LAGP_MAX_DIM) L.x[tid] = tid < p ? a.XX[m * p + tid] : 0.0;
  if (tid < 12) L.ec[tid] = gexp_coef(tid);
  ChState<NU> S;
#pragma unroll
  for (int k = 0; k < NU; ++k) S.u[k] = 0.0;
#pragma unroll
  for (int k = 0; k < Cf::UL; ++k) L.ul[k * TS + tid] = 0.0;
  S.act = tid < nc;
  S.vflag = 0;
  double yc = 0.0;
  if (S.act) {
    const int64_t row = C[tid];
#pragma unroll
    for (int k = 0; k < PM; ++k) L.xs[k * TS + tid] = k < p ? a.X[row * p + k] : 0.0;
    yc = a.y[row];
  } else {
#pragma unroll
    for (int k = 0; k < PM; ++k) L.xs[k * TS + tid] = 0.0;
  }
  __syncthreads();
  double kx = 0.0;
  if (S.act) {
    double s = 0.0;
    if (a.dlen == 1) {
#pragma unroll
      for (int k = 0; k < PM; ++k) {
        const double t = L.xs[k * TS + tid] - L.x[k];
        s = __builtin_fma(t, t, s);
      }
      kx = gexp(-(s * a.w[0]));
    } else {
#pragma unroll
      for (int k = 0; k < PM; ++k) {
        const double t = L.xs[k * TS + tid] - L.x[k];
        s = __builtin_fma(t * t, a.w[k], s);
      }
      kx = gexp(-s);
    }
  }
  S.v = 1.0 + a.g;
  S.cov = kx;
  S.q = yc;

  ChRun R{0.0, 0.0, 0.0, 0, true, false};
  ch_blocks<NU, PM, TS, DIAG, 0>(a, L, S, R, m);

  const int vf = __syncthreads_or(S.vflag);
  const bool ok = R.pd && R.done == n;
  if (tid == 0) {
    double mu = __builtin_nan(""), sc = __builtin_nan("");
    if (ok) {
      mu = R.mu;
      sc = R.psi * ((1.0 + a.g) - R.qq) / (double)n;
    }
    int st = 0;
    if (!R.pd) st |= LAGP_STATUS_NOTPD;
    if (vf) st |= LAGP_STATUS_VNONPOS;
    if (!(fabs(mu) <= 1.7976931348623157e308 && fabs(sc) <= 1.7976931348623157e308)) st |= LAGP_STATUS_NONFINITE;
    a.mean[m] = mu;
    a.s2[m] = sc;
    a.df[m] = (double)n;
    a.status[m] = st;
  }
  if (a.sel) {
    const int done = R.pd ? R.done : a.n0;  // not positive definite: report the n0 nearest
    for (int i = tid; i < n; i += blockDim.x) a.sel[m * n + i] = i < done ? C[R.pd ? L.J[i] : i] : -1;
  }
}

constexpr int CH_NU_SMALL = 31;  // n <= 32
constexpr int CH_NU_LARGE = 49;  // n <= 50

template <int NU, int PM, int TS>
constexpr size_t ch_bytes(int n) {
  using C = ChCfg<NU, PM, TS>;
  return ch_lds_bytes(PM, TS, C::UL, C::SS, n);
}

struct ChPick {
  int nu, pm, ts;
  size_t lds;
};

ChPick ch_pick(int n, int ncand, int p) {
  ChPick k;
  k.nu = n <= CH_NU_SMALL + 1 ? CH_NU_SMALL : CH_NU_LARGE;
  k.pm = p <= 8 ? 8 : LAGP_MAX_DIM;
  k.ts = ncand <= 512 ? 512 : 1024;
  const bool small = k.nu == CH_NU_SMALL, p8 = k.pm == 8, t5 = k.ts == 512;
  if (small)
    k.lds = p8 ? (t5 ? ch_bytes<CH_NU_SMALL, 8, 512>(n) : ch_bytes<CH_NU_SMALL, 8, 1024>(n))
               : (t5 ? ch_bytes<CH_NU_SMALL, LAGP_MAX_DIM, 512>(n) : ch_bytes<CH_NU_SMALL, LAGP_MAX_DIM, 1024>(n));
  else
    k.lds = p8 ? (t5 ? ch_bytes<CH_NU_LARGE, 8, 512>(n) : ch_bytes<CH_NU_LARGE, 8, 1024>(n))
               : (t5 ? ch_bytes<CH_NU_LARGE, LAGP_MAX_DIM, 512>(n) : ch_bytes<CH_NU_LARGE, LAGP_MAX_DIM, 1024>(n));
  return k;
}

template <int NU, int PM, int TS, bool DIAG>
hipError_t launch_chol_t(const LocalArgs& a, size_t lds, hipStream_t s) {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_chol<NU, PM, TS, DIAG>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int T = (a.ncand + 63) / 64 * 64;
  hipLaunchKernelGGL((k_chol<NU, PM, TS, DIAG>), dim3(a.M), dim3(T), lds, s, a);
  return hipGetLastError();
}

template <int NU, int PM, int TS>
hipError_t launch_chol_d(const LocalArgs& a, size_t lds, hipStream_t s) {
  return a.diag ? launch_chol_t<NU, PM, TS, true>(a, lds, s) : launch_chol_t<NU, PM, TS, false>(a, lds, s);
}

template <int NU, int PM>
hipError_t launch_chol_ts(const LocalArgs& a, int ts, size_t lds, hipStream_t s) {
  return ts == 512 ? launch_chol_d<NU, PM, 512>(a, lds, s) : launch_chol_d<NU, PM, 1024>(a, lds, s);
}

template <int NU>
hipError_t launch_chol_pm(const LocalArgs& a, const ChPick& k, hipStream_t s) {
  return k.pm == 8 ? launch_chol_ts<NU, 8>(a, k.ts, k.lds, s) : launch_chol_ts<NU, LAGP_MAX_DIM>(a, k.ts, k.lds, s);
}

}  // namespace

bool chol_supported(int n, int ncand, int p, size_t lds_max) {
  return n <= CH_NU_LARGE + 1 && ncand <= 1024 && p <= LAGP_MAX_DIM && ch_pick(n, ncand, p).lds <= lds_max;
}

hipError_t launch_chol(const LocalArgs& a, hipStream_t s) {
  if (a.M <= 0) return hipSuccess;
  const ChPick k = ch_pick(a.n, a.ncand, a.p);
  return k.nu == CH_NU_SMALL ? launch_chol_pm<CH_NU_SMALL>(a, k, s) : launch_chol_pm<CH_NU_LARGE>(a, k, s);
}

}  // namespace lagp
