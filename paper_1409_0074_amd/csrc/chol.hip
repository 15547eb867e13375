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
//   e_c = (K(x_w, x_c) - u_w^T u_c) (1 / l)
// and v_c -= e_c^2, cov_c -= (cov_w / l) e_c, q_c -= (q_w / l) e_c; the new
// entries of w_x and z are cov_w (1 / l) and q_w (1 / l).  After n points
//   mean = w_x^T z,  psi = z^T z,  k_x^T K^{-1} k_x = w_x^T w_x
// give Eqs. (predgp), (preds2) with n local points.  The starting design
// (the n0 nearest, Sec. 2.2) is the same recursion with the choice forced.
//
// A step costs one length-j inner product per candidate instead of the
// j x j contraction of the partitioned-inverse form, and a location's whole
// state (u_c in registers, candidate coordinates in LDS) stays on chip, so
// the search reads nothing from memory after its prologue.  Each thread
// holds two neighbouring candidates (2t, 2t+1): the per-step work that does
// not depend on the candidate (the winner's column read from LDS, the
// reductions, the barrier) is shared by two, and the two inner products
// are independent chains.  It computes the
// same criterion and prediction in a different rounding order: results agree
// with the partitioned-inverse definition to rounding, not bit for bit.
#include "dev_math.h"
#include "lagp_internal.h"

namespace lagp {

namespace {

constexpr int CH_CHUNK = 8;  // u entries per statically indexed block

typedef double v8d __attribute__((ext_vector_type(8)));

// NB: blocks of CH_CHUNK u entries kept per candidate.  The entry a step
// appends is read by later steps only, so designs of up to 8 NB + 2 points
// fit.  PM: coordinate rows (p <= PM, rows p .. PM-1 zero); CS: candidate
// slots, the LDS row stride (N' <= CS), two per thread.
template <int NB, int PM, int CS>
struct ChCfg {
  // the first NR blocks of every u_c live in registers, one 8-vector each
  // (an entry is appended at a run-time position with one indexed register
  // move), the last BL in LDS (entry RE + k of candidate c at ul[k * CS + c]):
  // the steps before entry RE is appended read no u entry from LDS
  static constexpr int BL = NB > 4 ? 1 : 0;
  static constexpr int UL = BL * CH_CHUNK;
  static constexpr int NR = NB - BL;
  static constexpr int RE = NR * CH_CHUNK;
  static constexpr int NUP = NB * CH_CHUNK;
  static constexpr int SS = NUP + 4;  // slot: u, then v, cov, q (and one unused word)
  static constexpr int NCH = NB + 1;  // step blocks: j = 0 .. 8 NB + 1
  static constexpr int NT = CS / 2;   // largest workgroup
  static constexpr int NWV = NT / 64;
};

// LDS: coordinates by dimension (PM x CS), the trailing u entries (UL x CS),
// two parities of per-wave slots and reduction words, the location, the exp
// coefficients, the design ranks.
struct ChLds {
  double* xs;
  double* ul;
  double* slot;  // 2 x NWV x SS
  double* redv;  // 2 x NWV: best criterion of each wave
  double* red2;  // 2 x NWV: runner-up of each wave
  double* x;     // LAGP_MAX_DIM
  double* ec;    // 12: Taylor coefficients of exp (read per use, not held in registers)
  int* redi;     // 2 x NWV: rank of each wave's best
  int* J;        // n
};

__host__ __device__ constexpr size_t ch_lds_bytes(int PM, int CS, int UL, int SS, int n) {
  return sizeof(double) * ((size_t)(PM + UL) * CS + 2 * (size_t)(CS / 128) * SS + 4 * (size_t)(CS / 128) +
                           LAGP_MAX_DIM + 12) +
         sizeof(int) * (2 * (size_t)(CS / 128) + (size_t)n);
}

template <int NB, int PM, int CS>
__device__ inline ChLds ch_carve(unsigned char* s) {
  using C = ChCfg<NB, PM, CS>;
  ChLds L;
  L.xs = reinterpret_cast<double*>(s);
  L.ul = L.xs + PM * CS;
  L.slot = L.ul + C::UL * CS;
  L.redv = L.slot + 2 * C::NWV * C::SS;
  L.red2 = L.redv + 2 * C::NWV;
  L.x = L.red2 + 2 * C::NWV;
  L.ec = L.x + LAGP_MAX_DIM;
  L.redi = reinterpret_cast<int*>(L.ec + 12);
  L.J = L.redi + 2 * C::NWV;
  return L;
}

// DPP lane move of a double (both halves), rows outside ROWMASK keep v.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double ch_dpp(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const int lo = (int)(uint32_t)b, hi = (int)(uint32_t)(b >> 32);
  const int lo2 = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROWMASK, 0xF, false);
  const int hi2 = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROWMASK, 0xF, false);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi2 << 32) | (uint64_t)(uint32_t)lo2);
}

__device__ __forceinline__ double ch_readlane(double v, int l) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Maximum over the wave (a value in every lane): quad swaps, half-row and
// row mirrors, then the row broadcasts; lane 63 ends with the maximum.
__device__ __forceinline__ double ch_wave_max(double v) {
  v = fmax(v, ch_dpp<0xB1, 0xF>(v));   // quad_perm [1,0,3,2]
  v = fmax(v, ch_dpp<0x4E, 0xF>(v));   // quad_perm [2,3,0,1]
  v = fmax(v, ch_dpp<0x141, 0xF>(v));  // row_half_mirror
  v = fmax(v, ch_dpp<0x140, 0xF>(v));  // row_mirror
  v = fmax(v, ch_dpp<0x142, 0xA>(v));  // row_bcast:15 into rows 1 and 3
  v = fmax(v, ch_dpp<0x143, 0xC>(v));  // row_bcast:31 into rows 2 and 3
  return ch_readlane(v, 63);
}

// Wave maximum of a 32-bit unsigned key (every lane): the same DPP pattern
// with the moves fused into the maximum (0 is the identity).
template <int CTRL, int ROWMASK>
__device__ __forceinline__ uint32_t ch_dpp_u(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWMASK, 0xF, false);
}

__device__ __forceinline__ uint32_t ch_wave_max_u(uint32_t v) {
  v = max(v, ch_dpp_u<0xB1, 0xF>(v));
  v = max(v, ch_dpp_u<0x4E, 0xF>(v));
  v = max(v, ch_dpp_u<0x141, 0xF>(v));
  v = max(v, ch_dpp_u<0x140, 0xF>(v));
  v = max(v, ch_dpp_u<0x142, 0xA>(v));
  v = max(v, ch_dpp_u<0x143, 0xC>(v));
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Lanes holding the largest criterion of the wave.  A criterion is >= 0
// (or -1: nothing to offer); for non-negative doubles the bit patterns order
// like the values, so the maximum is found on the high words, then on the
// low words of the lanes that tie there: two 32-bit reductions instead of a
// 64-bit one.  Returns the ballot of the lanes equal to the maximum (0 if
// no lane offers anything).
__device__ __forceinline__ uint64_t ch_wave_argmax(double sc) {
  const uint64_t b = __builtin_bit_cast(uint64_t, sc);
  const bool ok = sc >= 0.0;
  const uint32_t hi = ok ? (uint32_t)(b >> 32) | 0x80000000u : 0u;
  const uint32_t lo = (uint32_t)b;
  const uint32_t mhi = ch_wave_max_u(hi);
  const uint32_t mlo = ch_wave_max_u(hi == mhi ? lo : 0u);
  return __ballot(ok && hi == mhi && lo == mlo);
}

// Per-thread state of the candidate pair (2t, 2t+1); u block i < NR in
// r0[i] / r1[i], the later ones in LDS.
template <int NR>
struct ChPair {
  v8d r0[NR > 0 ? NR : 1], r1[NR > 0 ? NR : 1];
  double v[2], cov[2], q[2];
  bool act[2];
  int vflag;
};

// Per-location running results (meaningful in thread 0).
struct ChRun {
  double mu, psi, qq;
  int done;
  bool pd, stop;
  int n;  // this location's design size (<= a.n, the stride of the per-location outputs)
};

// Gaussian correlation between the winner w and candidate c in the rounding
// of corr(): dimension order, one fused multiply-add per term (the zero rows
// past p add exact zeros).  The coordinates of c come in a (c, c+1) pair;
// every coordinate is loaded before any is used, and the two exps run in
// lockstep.
template <int PM, bool ISO, int G>
__device__ __forceinline__ void ch_dist2(const double* xs, int CS, int w, int c0, const LocalArgs& A, double (&e)[2]) {
#pragma unroll
  for (int k0 = 0; k0 < PM; k0 += G) {
    double xw[G];
    double2 xc[G];
#pragma unroll
    for (int k = 0; k < G; ++k) {
      xw[k] = xs[(k0 + k) * CS + w];
      xc[k] = *reinterpret_cast<const double2*>(xs + (k0 + k) * CS + c0);
    }
#pragma unroll
    for (int k = 0; k < G; ++k) {
      const double t0 = xw[k] - xc[k].x, t1 = xw[k] - xc[k].y;
      if constexpr (ISO) {
        e[0] = __builtin_fma(t0, t0, e[0]);
        e[1] = __builtin_fma(t1, t1, e[1]);
      } else {
        e[0] = __builtin_fma(t0 * t0, A.w[k0 + k], e[0]);
        e[1] = __builtin_fma(t1 * t1, A.w[k0 + k], e[1]);
      }
    }
  }
}

template <int PM>
__device__ __forceinline__ void ch_corr2(const double* xs, int CS, int w, int c0, const double* ec,
                                         const LocalArgs& A, double w0, double& k0, double& k1) {
  // dimensions whose coordinates are in flight together (fewer where the
  // wide coordinate rows leave fewer registers)
  constexpr int G = PM > 8 ? 2 : 4;
  static_assert(PM % G == 0, "coordinate rows come in whole groups");
  double e[2] = {0.0, 0.0};
  if (A.dlen == 1) {
    ch_dist2<PM, true, G>(xs, CS, w, c0, A, e);
    e[0] = -(e[0] * w0);
    e[1] = -(e[1] * w0);
  } else {
    ch_dist2<PM, false, G>(xs, CS, w, c0, A, e);
    e[0] = -e[0];
    e[1] = -e[1];
  }
  gexp_lockstep_with(e, [ec](int i) { return ec[i]; });
  k0 = e[0];
  k1 = e[1];
}

// u entries in use during step block B (whole blocks; entries not yet
// appended are zero)
template <int NB, int B>
constexpr int ch_ke() { return (B + 1 < NB ? B + 1 : NB) * CH_CHUNK; }

// Publish candidate 2t + W: its u (whole blocks), v, cov, q.  (W is a
// template argument: a run-time choice between the two register sets would
// turn them into memory.)
template <int NB, int PM, int CS, int B, int W>
__device__ __forceinline__ void ch_write_slot(double* sl, const ChPair<ChCfg<NB, PM, CS>::NR>& S, const ChLds& L) {
  using C = ChCfg<NB, PM, CS>;
  constexpr int KE = ch_ke<NB, B>();
  const int c = 2 * threadIdx.x + W;
#pragma unroll
  for (int k = 0; k < KE; ++k) {
    if (k >= C::RE) {
      sl[k] = L.ul[(k - C::RE) * CS + c];
    } else {
      sl[k] = W == 0 ? S.r0[k / CH_CHUNK][k % CH_CHUNK] : S.r1[k / CH_CHUNK][k % CH_CHUNK];
    }
  }
  sl[C::NUP] = S.v[W];
  sl[C::NUP + 1] = S.cov[W];
  sl[C::NUP + 2] = S.q[W];
}

// The criterion of an available candidate (-1 for a taken one, never
// chosen; v <= 0 scores 0 and raises the flag; NaN scores -1).  Straight
// line: the quotient is formed whatever v is and selected afterwards.
__device__ __forceinline__ double ch_score(const double v, const double cov, bool act, int& vflag) {
  const double qt = (cov * cov) / v;
  const bool pos = v > 0.0;
  const double sc = pos ? qt : 0.0;
  vflag |= (act && !pos) ? 1 : 0;
  return (act && sc >= 0.0) ? sc : -1.0;
}

// Maximum of a 32-bit key over lanes 0 .. 7 (the other lanes hold 0): quad
// swaps and the half-row mirror leave it in lane 0.
__device__ __forceinline__ uint32_t ch_max8_u(uint32_t v) {
  v = max(v, ch_dpp_u<0xB1, 0xF>(v));
  v = max(v, ch_dpp_u<0x4E, 0xF>(v));
  v = max(v, ch_dpp_u<0x141, 0xF>(v));
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 0);
}

// ch_wave_argmax for criteria held by lanes 0 .. 7 only (-1 elsewhere).
__device__ __forceinline__ uint64_t ch_argmax8(double sc) {
  const uint64_t b = __builtin_bit_cast(uint64_t, sc);
  const bool ok = sc >= 0.0;
  const uint32_t hi = ok ? (uint32_t)(b >> 32) | 0x80000000u : 0u;
  const uint32_t lo = (uint32_t)b;
  const uint32_t mhi = ch_max8_u(hi);
  const uint32_t mlo = ch_max8_u(hi == mhi ? lo : 0u);
  return __ballot(ok && hi == mhi && lo == mlo);
}

// Steps j = B*CH_CHUNK .. B*CH_CHUNK + CH_CHUNK - 1: choose design point j
// (forced to rank j while j < n0, else the largest criterion, lowest rank on
// ties), publish its column, extend every other candidate's.
template <int NB, int PM, int CS, bool DIAG, int B>
__device__ __forceinline__ void ch_block(const LocalArgs& a, const ChLds& L, ChPair<ChCfg<NB, PM, CS>::NR>& S,
                                         ChRun& R, int64_t m, double w0) {
  using C = ChCfg<NB, PM, CS>;
  constexpr int NUP = C::NUP, SS = C::SS, NWV = C::NWV, NR = C::NR, RE = C::RE;
  constexpr int KE = ch_ke<NB, B>();
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nwv = blockDim.x >> 6;
  const int c0 = 2 * tid;
  const int n = R.n, n0 = a.n0, nst = a.n - a.n0;  // (nst: stride of the per-step outputs)
  for (int jj = 0; jj < CH_CHUNK; ++jj) {
    const int j = B * CH_CHUNK + jj;
    if (j >= n || R.stop) return;
    const int par = j & 1;
    double* sl = L.slot + par * NWV * SS;
    if (j < n0) {
      if ((j >> 1) == tid) {
        if ((j & 1) == 0) ch_write_slot<NB, PM, CS, B, 0>(sl + wv * SS, S, L);
        if ((j & 1) == 1) ch_write_slot<NB, PM, CS, B, 1>(sl + wv * SS, S, L);
      }
    } else {
      const double s0 = ch_score(S.v[0], S.cov[0], S.act[0], S.vflag);
      const double s1 = ch_score(S.v[1], S.cov[1], S.act[1], S.vflag);
      const int pick = s1 > s0 ? 1 : 0;  // the lower rank on ties
      const double pb = pick ? s1 : s0;
      const uint64_t hit = ch_wave_argmax(pb);
      const int wl = hit ? __builtin_ctzll(hit) : -1;
      const double wmax = wl >= 0 ? ch_readlane(pb, wl) : -1.0;
      if (lane == wl && pick == 0) ch_write_slot<NB, PM, CS, B, 0>(sl + wv * SS, S, L);
      if (lane == wl && pick == 1) ch_write_slot<NB, PM, CS, B, 1>(sl + wv * SS, S, L);
      if (lane == (wl >= 0 ? wl : 0)) {
        L.redv[par * NWV + wv] = wl >= 0 ? wmax : -1.0;
        L.redi[par * NWV + wv] = wl >= 0 ? c0 + pick : -1;
      }
      if constexpr (DIAG) {
        const double s2 = ch_wave_max(lane == wl ? (pick ? s0 : s1) : fmax(s0, s1));
        if (lane == 0) L.red2[par * NWV + wv] = s2;
      }
    }
    __syncthreads();
    int w = j;
    double b1 = 0.0, b2 = 0.0;
    if (j >= n0) {
      // the best over waves; the earliest wave (lowest ranks) wins ties
      double cv = -1.0, c2 = -1.0;
      int ci = -1;
      if (lane < nwv) {
        ci = L.redi[par * NWV + lane];
        const double rv = L.redv[par * NWV + lane];
        cv = ci >= 0 ? rv : -1.0;
        if constexpr (DIAG) c2 = L.red2[par * NWV + lane];
      }
      static_assert(NWV <= 8, "the cross-wave reduction covers eight waves");
      const uint64_t gh = ch_argmax8(cv);
      if (!gh) {  // no finite criterion anywhere: give up on x
        R.stop = true;
        return;
      }
      const int ql = __builtin_ctzll(gh);
      w = __builtin_amdgcn_readlane(ci, ql);
      b1 = ch_readlane(cv, ql);
      if constexpr (DIAG) b2 = ch_wave_max(lane == ql ? c2 : fmax(cv, c2));
    }
    const double* ws = sl + (w >> 7) * SS;
    const double vw = ws[NUP];
    // the winner's new diagonal entry sqrt(v) and the new entries of w_x
    // and z, formed by every wave (off the path to the next scores)
    const double li = 1.0 / __builtin_sqrt(vw), wxj = ws[NUP + 1] * li, zj = ws[NUP + 2] * li;
    if (j < n0 && !(vw > 0.0)) {  // the starting covariance is not positive definite
      R.pd = false;
      R.stop = true;
      return;
    }
    if (!(vw > 0.0)) S.vflag = 1;
    if (tid == 0) {
      L.J[j] = w;
      R.mu = __builtin_fma(wxj, zj, R.mu);
      R.psi = __builtin_fma(zj, zj, R.psi);
      R.qq = __builtin_fma(wxj, wxj, R.qq);
      if (DIAG && j >= n0 && a.diag) {
        double* dg = a.diag + (m * nst + (j - n0)) * 2;
        dg[0] = b1;
        dg[1] = b2 < 0.0 ? -__builtin_huge_val() : b2;
      }
      if (j >= n0 && a.counts) {  // every free candidate is scored
        int32_t* ct = a.counts + (m * nst + (j - n0)) * 2;
        ct[0] = a.ncand - j;
        ct[1] = 0;
      }
    }
    if (w == c0) S.act[0] = false;
    if (w == c0 + 1) S.act[1] = false;
    R.done = j + 1;
    if (j + 1 < n) {
      // both candidates of the pair, taken or not (a taken one is never read again)
      double kv0, kv1;
      ch_corr2<PM>(L.xs, CS, w, c0, L.ec, a, w0, kv0, kv1);
      double d0 = 0.0, d1 = 0.0;
#pragma unroll
      for (int k = 0; k < KE; ++k) {
        const double wk = ws[k];
        if (k >= RE) {
          const double2 uu = *reinterpret_cast<const double2*>(L.ul + (k - RE) * CS + c0);
          d0 = __builtin_fma(wk, uu.x, d0);
          d1 = __builtin_fma(wk, uu.y, d1);
        } else {
          d0 = __builtin_fma(wk, S.r0[k / CH_CHUNK][k % CH_CHUNK], d0);
          d1 = __builtin_fma(wk, S.r1[k / CH_CHUNK][k % CH_CHUNK], d1);
        }
      }
      const double e0 = (kv0 - d0) * li, e1 = (kv1 - d1) * li;
      // append u[j] (the entry of the last update, j = 8 NB, is never read)
      if constexpr (B < NR) {
        S.r0[B][jj] = e0;
        S.r1[B][jj] = e1;
      } else if constexpr (B < NB) {
        *reinterpret_cast<double2*>(L.ul + (j - RE) * CS + c0) = make_double2(e0, e1);
      }
      S.v[0] = __builtin_fma(-e0, e0, S.v[0]);
      S.v[1] = __builtin_fma(-e1, e1, S.v[1]);
      S.cov[0] = __builtin_fma(-wxj, e0, S.cov[0]);
      S.cov[1] = __builtin_fma(-wxj, e1, S.cov[1]);
      S.q[0] = __builtin_fma(-zj, e0, S.q[0]);
      S.q[1] = __builtin_fma(-zj, e1, S.q[1]);
    }
  }
}

template <int NB, int PM, int CS, bool DIAG, int B>
__device__ __forceinline__ void ch_blocks(const LocalArgs& a, const ChLds& L, ChPair<ChCfg<NB, PM, CS>::NR>& S,
                                          ChRun& R, int64_t m, double w0) {
  if constexpr (B < ChCfg<NB, PM, CS>::NCH) {
    ch_block<NB, PM, CS, DIAG, B>(a, L, S, R, m, w0);
    if (!R.stop && (B + 1) * CH_CHUNK < R.n) ch_blocks<NB, PM, CS, DIAG, B + 1>(a, L, S, R, m, w0);
  }
}

// One location on one workgroup of 64 ceil(N'/128) threads; thread t holds
// the candidates of ranks 2t and 2t+1.  Its design size, lengthscale and
// nugget are the location's own when the per-location arrays are given.
template <int NB, int PM, int CS, bool DIAG, bool PL>
__device__ __forceinline__ void ch_location(const LocalArgs& a, const ChLds& L, int64_t m) {
  using Cf = ChCfg<NB, PM, CS>;
  const int tid = threadIdx.x;
  const int p = a.p, nc = a.ncand, nmax = a.n;
  const int n = PL ? a.nloc[m] : a.n;
  const double g = PL ? a.gloc[m] : a.g;
  const int32_t* C = a.cand + m * nc;
  const int c0 = 2 * tid;
  // isotropic reciprocal lengthscale: per location when given (a location
  // without one is skipped), else the call's
  double w0 = a.w[0];
  if (a.dloc) {
    const double dl = a.dloc[m];
    if (!(dl > 0.0)) {
      if (tid == 0) a.status[m] = 0;
      return;
    }
    w0 = 1.0 / dl;
  }

  if (tid < LAGP_MAX_DIM) L.x[tid] = tid < p ? a.XX[m * p + tid] : 0.0;
  if (tid < 12) L.ec[tid] = gexp_coef(tid);
  ChPair<Cf::NR> S;
#pragma unroll
  for (int b = 0; b < (Cf::NR > 0 ? Cf::NR : 1); ++b) {
    S.r0[b] = v8d{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    S.r1[b] = S.r0[b];
  }
#pragma unroll
  for (int k = 0; k < Cf::UL; ++k) *reinterpret_cast<double2*>(L.ul + k * CS + c0) = make_double2(0.0, 0.0);
  S.vflag = 0;
  double yc[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int c = c0 + i;
    S.act[i] = c < nc;
    yc[i] = 0.0;
    if (S.act[i]) {
      const int64_t row = C[c];
#pragma unroll
      for (int k = 0; k < PM; ++k) L.xs[k * CS + c] = k < p ? a.X[row * p + k] : 0.0;
      yc[i] = a.y[row];
    } else {
#pragma unroll
      for (int k = 0; k < PM; ++k) L.xs[k * CS + c] = 0.0;
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    double kx = 0.0;
    if (S.act[i]) {
      double s = 0.0;
      if (a.dlen == 1) {
#pragma unroll
        for (int k = 0; k < PM; ++k) {
          const double t = L.xs[k * CS + c0 + i] - L.x[k];
          s = __builtin_fma(t, t, s);
        }
        kx = gexp(-(s * w0));
      } else {
#pragma unroll
        for (int k = 0; k < PM; ++k) {
          const double t = L.xs[k * CS + c0 + i] - L.x[k];
          s = __builtin_fma(t * t, a.w[k], s);
        }
        kx = gexp(-s);
      }
    }
    S.v[i] = 1.0 + g;
    S.cov[i] = kx;
    S.q[i] = yc[i];
  }

  ChRun R{0.0, 0.0, 0.0, 0, true, false, n};
  ch_blocks<NB, PM, CS, DIAG, 0>(a, L, S, R, m, w0);

  const int vf = __syncthreads_or(S.vflag);
  const bool ok = R.pd && R.done == n;
  if (tid == 0) {
    double mu = __builtin_nan(""), sc = __builtin_nan("");
    if (ok) {
      mu = R.mu;
      sc = R.psi * ((1.0 + g) - R.qq) / (double)n;
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
  if (a.sel) {  // rows of nmax entries, -1 past this location's design
    const int done = R.pd ? R.done : a.n0;  // not positive definite: report the n0 nearest
    for (int i = tid; i < nmax; i += blockDim.x) a.sel[m * nmax + i] = i < done ? C[R.pd ? L.J[i] : i] : -1;
  }
}

// The search kernel: one workgroup per location.  PL: the call carries
// per-location design sizes and nuggets (a merged batch of requests).
template <int NB, int PM, int CS, bool DIAG, bool PL>
__global__ __launch_bounds__(CS / 2) __attribute__((amdgpu_waves_per_eu(2))) void k_chol(LocalArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const ChLds L = ch_carve<NB, PM, CS>(smem);
  ch_location<NB, PM, CS, DIAG, PL>(a, L, blockIdx.x);
}

constexpr int CH_NB_SMALL = 4;  // n <= 34
constexpr int CH_NB_LARGE = 6;  // n <= 50
constexpr int CH_N_MAX = 8 * CH_NB_LARGE + 2;

template <int NB, int PM, int CS>
constexpr size_t ch_bytes(int n) {
  using C = ChCfg<NB, PM, CS>;
  return ch_lds_bytes(PM, CS, C::UL, C::SS, n);
}

struct ChPick {
  int nb, pm, cs;
  size_t lds;
};

ChPick ch_pick(int n, int ncand, int p) {
  ChPick k;
  k.nb = n <= 8 * CH_NB_SMALL + 2 ? CH_NB_SMALL : CH_NB_LARGE;
  k.pm = p <= 8 ? 8 : LAGP_MAX_DIM;
  k.cs = ncand <= 512 ? 512 : 1024;
  const bool small = k.nb == CH_NB_SMALL, p8 = k.pm == 8, c5 = k.cs == 512;
  if (small)
    k.lds = p8 ? (c5 ? ch_bytes<CH_NB_SMALL, 8, 512>(n) : ch_bytes<CH_NB_SMALL, 8, 1024>(n))
               : (c5 ? ch_bytes<CH_NB_SMALL, LAGP_MAX_DIM, 512>(n) : ch_bytes<CH_NB_SMALL, LAGP_MAX_DIM, 1024>(n));
  else
    k.lds = p8 ? (c5 ? ch_bytes<CH_NB_LARGE, 8, 512>(n) : ch_bytes<CH_NB_LARGE, 8, 1024>(n))
               : (c5 ? ch_bytes<CH_NB_LARGE, LAGP_MAX_DIM, 512>(n) : ch_bytes<CH_NB_LARGE, LAGP_MAX_DIM, 1024>(n));
  return k;
}

template <int NB, int PM, int CS, bool DIAG, bool PL>
hipError_t launch_chol_t(const LocalArgs& a, size_t lds, hipStream_t s) {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_chol<NB, PM, CS, DIAG, PL>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int T = (a.ncand + 127) / 128 * 64;
  hipLaunchKernelGGL((k_chol<NB, PM, CS, DIAG, PL>), dim3((unsigned)a.M), dim3(T), lds, s, a);
  return hipGetLastError();
}

template <int NB, int PM, int CS>
hipError_t launch_chol_d(const LocalArgs& a, size_t lds, hipStream_t s) {
  if (a.nloc) return a.diag ? launch_chol_t<NB, PM, CS, true, true>(a, lds, s) : launch_chol_t<NB, PM, CS, false, true>(a, lds, s);
  return a.diag ? launch_chol_t<NB, PM, CS, true, false>(a, lds, s) : launch_chol_t<NB, PM, CS, false, false>(a, lds, s);
}

template <int NB, int PM>
hipError_t launch_chol_cs(const LocalArgs& a, int cs, size_t lds, hipStream_t s) {
  return cs == 512 ? launch_chol_d<NB, PM, 512>(a, lds, s) : launch_chol_d<NB, PM, 1024>(a, lds, s);
}

template <int NB>
hipError_t launch_chol_pm(const LocalArgs& a, const ChPick& k, hipStream_t s) {
  return k.pm == 8 ? launch_chol_cs<NB, 8>(a, k.cs, k.lds, s) : launch_chol_cs<NB, LAGP_MAX_DIM>(a, k.cs, k.lds, s);
}

}  // namespace

bool chol_supported(int n, int ncand, int p, size_t lds_max) {
  return n <= CH_N_MAX && ncand <= 1024 && p <= LAGP_MAX_DIM && ch_pick(n, ncand, p).lds <= lds_max;
}

hipError_t launch_chol(const LocalArgs& a, hipStream_t s) {
  if (a.M <= 0) return hipSuccess;
  if (!a.nloc != !a.gloc) return hipErrorInvalidValue;
  const ChPick k = ch_pick(a.n, a.ncand, a.p);
  return k.nb == CH_NB_SMALL ? launch_chol_pm<CH_NB_SMALL>(a, k, s) : launch_chol_pm<CH_NB_LARGE>(a, k, s);
}

}  // namespace lagp
