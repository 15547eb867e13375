// Greedy local designs and local GP prediction, one workgroup per location.
//
// Per location x with candidate list C (nearest first):
//   start   J = the n0 nearest; K_J^{-1} by a Cholesky factorisation
//           (Sec. 2.2), or J = the n nearest in nearest-neighbour mode;
//   step j  choose the candidate maximising the reduction in variance at x,
//           the integrand of Eq. (alc):
//             ALC_c = (K(x_c,x) - k_c^T K^{-1} k_x)^2 / ((1+g) - k_c^T K^{-1} k_c)
//           - exhaustive (Sec. 3.1): every remaining candidate is scored; the
//             contraction W = K_J^{-1} [k_c]_c runs on f64 MFMA tiles of 16
//             candidates, its epilogue folds W into the quadratic form;
//           - ray (Sec. 4): p rays (or numrays) from round-robin starts among
//             the nearest remaining candidates, each a Brent line search on a
//             segment cut at the design's bounding box, an s = 0 check, the
//             best optimum snapped to the nearest allowed candidate;
//           then grow K_J^{-1} by the partitioned inverse (G_j, g_j, v_j under
//           Eq. (alc), with g_j = -K^{-1}k/v);
//   predict mean k^T K^{-1} y, scale psi ((1+g) - k^T K^{-1} k)/n, df n
//           (Eqs. predgp, preds2 with n local points).
// The kernel rows K(x_{J_i}, x_c) live in a per-location workspace (one row
// appended per step).  Everything except the MFMA scoring contraction uses
// index-order fma sums, so those values are reproducible bit for bit.
#include <cstdlib>

#include "dev_math.h"
#include "lagp_internal.h"

namespace lagp {

typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int NW = LOCAL_THREADS / 64;  // waves per workgroup
// Rays of one wave searched in lockstep: their objective evaluations share
// one pass (independent chains interleave), so a wave's step takes about the
// longest of its rays' Brent searches instead of their sum.
constexpr int RB = 3;

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double shfl_xor_d(double v, int m) { return __shfl_xor(v, m, 64); }
__device__ __forceinline__ int shfl_xor_i(int v, int m) { return __shfl_xor(v, m, 64); }

// LDS carve-up (all sizes decided on the host, see local_lds_bytes).
struct Lds {
  double* Ki;    // NR x LD, K_J^{-1}, zero outside the leading j x j block
  double* kx;    // NP: k_J(x)
  double* h;     // NP: K^{-1} k_x (scoring only)
  double* col;   // NP: kernel column of the chosen candidate
  double* wv;    // NP
  double* gv;    // NP: g_j
  double* yJ;    // NP
  double* x;     // LAGP_MAX_DIM: the location
  double w0;     // isotropic reciprocal lengthscale of this location (dlen = 1)
  double* xj;    // n x p: coordinates of the local design
  double* kzb;   // NW x RB x kzs: ray objective scratch, per wave and slot
  double* wvb;   // NW x RB x kzs
  double* ra;    // R x p: ray starts
  double* rdir;  // R x p: clipped segment directions
  double* rval;  // R: best ALC along each ray
  double* rs;    // R: its s*
  int* rev;      // R: Brent evaluations along each ray
  double* redv;  // 2 NW
  double* scal;  // 8 scalars
  int* redi;     // NW
  int* J;        // NP: ranks of the local design, selection order (ncand: a row outside the candidates)
  int* jrow;     // NP: design rows of the local design, selection order
  int* starts;   // R
  int* ints;     // 16 scalars
  int* shortlist;  // max(64, ncs/16): mixed form, the 16-candidate tiles re-scored in FP64
  double* tps;     // 16: tile ray form, each ray's parameter this round
  int* tpe;        // 16: tile ray form, whether the ray is evaluated this round
  int kzs;         // per-slot stride of kzb / wvb
  float* scr;      // ncs: mixed form, FP32 screened scores
  unsigned char* selm;  // ncs: 1 = not available (selected or padding)
};

__host__ __device__ inline size_t align16(size_t b) { return (b + 15) & ~size_t(15); }

// kzs = NP + 2: room for the zero-padded 8-wide blocks of the ray sums,
// 16-byte aligned but off the bank period, so the six MFMA inner-product
// chains, which read different slots' vectors at the same index, fall in
// different LDS banks.
struct LdsPlan {
  int NP, NR, LD, R, KZS;
  size_t off[28];
  size_t bytes;
};

// R > 0: ray scratch for R rays (tile: all rays of a step on one wave, no
// per-wave vectors); mixed: screened scores and shortlist.
__host__ __device__ inline LdsPlan plan_lds(int n, int ncs, int p, int R, bool mixed, bool tile = false) {
  LdsPlan P;
  // NP = 256 (n > 128): K_J^{-1} does not fit LDS and lives in a per-location
  // workspace (LocalArgs::kig)
  P.NP = n <= 64 ? 64 : (n <= 128 ? 128 : 256);
  // exact scoring and rays read rows below 4 ceil(j/4); the FP32 screen
  // reads whole 16-row blocks
  P.NR = mixed ? (n + 15) & ~15 : (n + 3) & ~3;
  // the ray sums read K^{-1} in 8-row blocks: whole blocks of (zeroed)
  // workspace rows past 128 points, where nothing else follows in memory
  if (P.NP == 256) P.NR = (n + 7) & ~7;
  P.KZS = P.NP + 2;
  // odd: the 16 rows of an MFMA operand fall in distinct banks (the tile ray
  // form, short of LDS, strides by the rows it uses)
  P.LD = (tile ? P.NR : P.NP) + 1;
  P.R = R < 1 ? 0 : R;
  const bool ray = R > 0 && !tile;
  size_t o = 0;
  int k = 0;
  auto take = [&](size_t b) { P.off[k++] = o; o = align16(o + b); };
  take(P.NP == 256 ? 0 : sizeof(double) * P.NR * P.LD);  // Ki
  for (int i = 0; i < 6; ++i) take(sizeof(double) * P.NP);  // kx h col wv gv yJ
  take(sizeof(double) * LAGP_MAX_DIM);     // x
  take(sizeof(double) * n * p);            // xj
  // kzb: per-wave ray vectors, or the tile form's kernel columns (16 chunks x 64 lanes)
  take(ray ? sizeof(double) * NW * RB * P.KZS : (tile && R > 0 ? sizeof(double) * 64 * (((n + 3) / 4 + 3) & ~3) : 0));
  take(ray ? sizeof(double) * NW * RB * P.KZS : 0);  // wvb
  take(sizeof(double) * P.R * p);          // ra
  take(sizeof(double) * P.R * p);          // rdir
  take(sizeof(double) * P.R);              // rval
  take(sizeof(double) * P.R);              // rs
  take(sizeof(int) * P.R);                 // rev
  take(sizeof(double) * 2 * NW);           // redv
  take(sizeof(double) * 8);                // scal
  take(sizeof(int) * NW);                  // redi
  take(sizeof(int) * P.NP);                // J
  take(sizeof(int) * P.NP);                // jrow
  take(sizeof(int) * P.R);                 // starts
  take(sizeof(int) * 16);                  // ints
  take(mixed ? sizeof(int) * (ncs / 16 > 64 ? ncs / 16 : 64) : 0);  // shortlist (tiles)
  take(tile ? sizeof(double) * 16 : 0);   // tps
  take(tile ? sizeof(int) * 16 : 0);      // tpe
  take(mixed ? sizeof(float) * ncs : 0);   // scr
  take(ncs);                               // selm
  P.bytes = o;
  return P;
}

__device__ inline Lds carve(unsigned char* s, const LdsPlan& P) {
  Lds L;
  int k = 0;
  auto D = [&]() { return reinterpret_cast<double*>(s + P.off[k++]); };
  L.Ki = D();
  L.kx = D(); L.h = D(); L.col = D(); L.wv = D(); L.gv = D(); L.yJ = D();
  L.x = D(); L.xj = D(); L.kzb = D(); L.wvb = D(); L.ra = D(); L.rdir = D();
  L.rval = D(); L.rs = D();
  L.rev = reinterpret_cast<int*>(s + P.off[k++]);
  L.redv = D(); L.scal = D();
  L.redi = reinterpret_cast<int*>(s + P.off[k++]);
  L.J = reinterpret_cast<int*>(s + P.off[k++]);
  L.jrow = reinterpret_cast<int*>(s + P.off[k++]);
  L.starts = reinterpret_cast<int*>(s + P.off[k++]);
  L.ints = reinterpret_cast<int*>(s + P.off[k++]);
  L.shortlist = reinterpret_cast<int*>(s + P.off[k++]);
  L.tps = reinterpret_cast<double*>(s + P.off[k++]);
  L.tpe = reinterpret_cast<int*>(s + P.off[k++]);
  L.scr = reinterpret_cast<float*>(s + P.off[k++]);
  L.selm = s + P.off[k++];
  L.kzs = P.KZS;
  return L;
}

// ------------------------------------------------------------ start ------

// K_J^{-1} of the starting design (J = ranks 0..n0-1), bit-compatible with a
// row-by-row Cholesky: L = chol(K_J + g I) computed column by column in LDS
// (each entry's sum runs over the same index order), L^{-1} by forward
// substitution (one thread per column, scratch in global memory), then
// K^{-1} = L^{-T} L^{-1}.  Returns false if a pivot is not positive.
__device__ __forceinline__ bool start_inverse(const LocalArgs& a, const Lds& L, int LD, const double* Kc, double* Li, int n0) {
  const int tid = threadIdx.x;
  const int ncs = a.ncs;
  for (int t = tid; t < n0 * n0; t += blockDim.x) {
    const int i = t / n0, k = t % n0;
    L.Ki[i * LD + k] = Kc[(int64_t)i * ncs + k] + (i == k ? a.g : 0.0);
  }
  if (tid == 0) L.ints[1] = 1;
  __syncthreads();
  for (int k = 0; k < n0; ++k) {
    if (tid == 0) {
      double s = L.Ki[k * LD + k];
      for (int m = 0; m < k; ++m) s = __builtin_fma(-L.Ki[k * LD + m], L.Ki[k * LD + m], s);
      if (!(s > 0.0)) L.ints[1] = 0;
      L.Ki[k * LD + k] = __builtin_sqrt(s);
    }
    __syncthreads();
    const double piv = L.Ki[k * LD + k];
    for (int i = k + 1 + tid; i < n0; i += blockDim.x) {
      double s = L.Ki[i * LD + k];
      for (int m = 0; m < k; ++m) s = __builtin_fma(-L.Ki[i * LD + m], L.Ki[k * LD + m], s);
      L.Ki[i * LD + k] = s / piv;
    }
    __syncthreads();
  }
  const bool ok = L.ints[1] != 0;
  // forward substitution: column c of L^{-1}
  for (int c = tid; c < n0; c += blockDim.x) {
    for (int i = c; i < n0; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int m = c; m < i; ++m) s = __builtin_fma(-L.Ki[i * LD + m], Li[m * n0 + c], s);
      Li[i * n0 + c] = s / L.Ki[i * LD + i];
    }
  }
  __syncthreads();
  for (int t = tid; t < n0 * n0; t += blockDim.x) {
    const int i = t / n0, k = t % n0;
    double s = 0.0;
    for (int m = (i > k ? i : k); m < n0; ++m) s = __builtin_fma(Li[m * n0 + i], Li[m * n0 + k], s);
    Li[n0 * n0 + t] = s;
  }
  __syncthreads();
  for (int t = tid; t < n0 * n0; t += blockDim.x) {
    const int i = t / n0, k = t % n0;
    L.Ki[i * LD + k] = Li[n0 * n0 + t];
  }
  __syncthreads();
  return ok;
}

// ------------------------------------------------------- exhaustive ------

// Gaussian correlation with the dimension loop unrolled to PM >= p (same
// arithmetic as corr(): t = u_k - v_k, first argument first).
template <int PM>
__device__ __forceinline__ double corr_pm(const double* u, const double* v, int p, double w0, const double* w,
                                          int dlen) {
  double acc = 0.0;
  if (dlen == 1) {
#pragma unroll
    for (int k = 0; k < PM; ++k)
      if (k < p) {
        const double t = u[k] - v[k];
        acc = __builtin_fma(t, t, acc);
      }
    return gexp(-(acc * w0));
  }
#pragma unroll
  for (int k = 0; k < PM; ++k)
    if (k < p) {
      const double t = u[k] - v[k];
      acc = __builtin_fma(t * t, w[k], acc);
    }
  return gexp(-acc);
}

// Candidates handled per thread and pass when gathering coordinates (their
// loads are all issued before the first use), by the unrolled dimension.
template <int PM>
constexpr int gather_width() { return PM <= 8 ? 4 : 1; }

// Prologue, one pass over the candidates (thread t takes c = t + k*blockDim):
// gather x_c into Xc, K(x_c, x) into kxc, and the n0 starting rows
// K(x_{J_i}, x_c) for c < kcols.  Rows past ncand hold zeros.
template <int PM>
__device__ __forceinline__ void gather_candidates(const LocalArgs& a, const Lds& L, const int32_t* C, double* Xc,
                                                  double* Kc, float* Kc32, double* kxc, int n0, int kcols) {
  constexpr int GATHER = gather_width<PM>();
  const int p = a.p, nc = a.ncand, ncs = a.ncs, nt = blockDim.x;
  for (int c0 = threadIdx.x; c0 < ncs; c0 += GATHER * nt) {
    int64_t row[GATHER];
#pragma unroll
    for (int u = 0; u < GATHER; ++u) {
      const int c = c0 + u * nt;
      row[u] = c < nc ? (int64_t)C[c] : 0;
    }
    double r[GATHER][PM];
#pragma unroll
    for (int u = 0; u < GATHER; ++u)
#pragma unroll
      for (int k = 0; k < PM; ++k) r[u][k] = a.X[row[u] * p + (k < p ? k : 0)];  // always in bounds
#pragma unroll
    for (int u = 0; u < GATHER; ++u) {
      const int c = c0 + u * nt;
      if (c >= ncs) break;
      const bool live = c < nc;
#pragma unroll
      for (int k = 0; k < PM; ++k) {
        if (!live) r[u][k] = 0.0;
        if (k < p) Xc[(int64_t)c * p + k] = r[u][k];
      }
      kxc[c] = live ? corr_pm<PM>(r[u], L.x, p, L.w0, a.w, a.dlen) : 0.0;
      if (c < kcols)
        for (int i = 0; i < n0; ++i) {
          const double kv = live ? corr_pm<PM>(L.xj + i * p, r[u], p, L.w0, a.w, a.dlen) : 0.0;
          Kc[(int64_t)i * ncs + c] = kv;
          if (Kc32) Kc32[(int64_t)i * ncs + c] = (float)kv;
        }
    }
  }
}

// New kernel row K(x_s, x_c) for every candidate from the gathered
// coordinates (each thread reads back the rows it gathered).
template <int PM>
__device__ __forceinline__ void kernel_row(const LocalArgs& a, double w0, const double* xs, const double* Xc, double* row,
                                           float* row32) {
  constexpr int GATHER = gather_width<PM>();
  const int p = a.p, nc = a.ncand, ncs = a.ncs, nt = blockDim.x;
  double s[PM];
#pragma unroll
  for (int k = 0; k < PM; ++k) s[k] = k < p ? xs[k] : 0.0;
  for (int c0 = threadIdx.x; c0 < ncs; c0 += GATHER * nt) {
    double r[GATHER][PM];
#pragma unroll
    for (int u = 0; u < GATHER; ++u) {
      const int c = c0 + u * nt < ncs ? c0 + u * nt : ncs - 1;  // in bounds
#pragma unroll
      for (int k = 0; k < PM; ++k) r[u][k] = Xc[(int64_t)c * p + (k < p ? k : 0)];
    }
#pragma unroll
    for (int u = 0; u < GATHER; ++u) {
      const int c = c0 + u * nt;
      if (c >= ncs) break;
      const double kv = c < nc ? corr_pm<PM>(s, r[u], p, w0, a.w, a.dlen) : 0.0;
      row[c] = kv;
      if (row32) row32[c] = (float)kv;
    }
  }
}

struct Best {
  double v1, v2;
  int i1;
};

__device__ __forceinline__ void best_push(Best& b, double v, int i) {
  if (v > b.v1 || (v == b.v1 && i < b.i1)) {
    b.v2 = b.v1;
    b.v1 = v;
    b.i1 = i;
  } else if (v > b.v2) {
    b.v2 = v;
  }
}

__device__ __forceinline__ Best best_merge(Best a, Best b) {
  Best r;
  if (b.v1 > a.v1 || (b.v1 == a.v1 && b.i1 < a.i1)) {
    r.v1 = b.v1; r.i1 = b.i1; r.v2 = fmax(a.v1, b.v2);
  } else {
    r.v1 = a.v1; r.i1 = a.i1; r.v2 = fmax(a.v2, b.v1);
  }
  return r;
}

// Block-wide argmax of the per-thread bests; result in L.ints[0], L.scal[1..2].
__device__ __forceinline__ void block_best(const Lds& L, Best b) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int m = 32; m >= 1; m >>= 1) {
    Best o;
    o.v1 = shfl_xor_d(b.v1, m);
    o.v2 = shfl_xor_d(b.v2, m);
    o.i1 = shfl_xor_i(b.i1, m);
    b = best_merge(b, o);
  }
  if (lane == 0) {
    L.redv[2 * wave] = b.v1;
    L.redv[2 * wave + 1] = b.v2;
    L.redi[wave] = b.i1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    Best r = {L.redv[0], L.redv[1], L.redi[0]};
    const int nw = blockDim.x >> 6;
    for (int w = 1; w < nw; ++w) {
      Best o = {L.redv[2 * w], L.redv[2 * w + 1], L.redi[w]};
      r = best_merge(r, o);
    }
    L.ints[0] = r.i1;
    L.scal[1] = r.v1;
    L.scal[2] = r.v2;
  }
  __syncthreads();
}

// Score every available candidate at design size j, exactly in the defined
// order, on f64 MFMA.  v_mfma_f64_16x16x4f64 and v_mfma_f64_4x4x4f64 both
// compute D = C + sum_k A[.][k] B[k][.] as a chain of fused multiply-adds in
// ascending k (checked bit for bit on gfx950), so chaining them over K-chunks
// in ascending order gives the sequential sums of the definitions:
//   W[i][c]  = sum_k fma(Kinv[i][k], k_c[k])        (A = Kinv rows, B = k_c chunk)
//   v_c      = (1+g) - sum_i fma(k_c[i], W[i][c])  (A = k_c chunk^T, B = W chunk;
//                                                   the diagonal of D)
//   cov_c    = K(x_c,x) - sum_i fma(W[i][c], k_x[i]) (A = k_x broadcast, B = W chunk)
// Lane layout (gfx950): A[i][k] from lane 16k + i, B[k][n] from lane 16k + n,
// D[i][n] in register i/4 of lane 16(i%4) + n.  With chunk q = rows
// 4q..4q+3, lane quarter g holds row 4q + g of a B operand, and register r
// of row block I holds W rows 16I + 4r + g: exactly the B operand of chunk
// 4I + r, and the loaded k_c chunk is exactly the A operand of the v chain.
// Rows and columns past j are zero, and fma(0, 0, s) = s, so the padding
// leaves every sum unchanged (up to the sign of a zero sum, which no later
// step can see: the scores square cov and subtract v from 1 + g).
// Buffer resource over one location's candidate-row block (gfx9 word 3).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t kc_rsrc(const LocalArgs& a, const double* Kc) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(Kc), (short)0, a.kc_rows * a.ncs * 8, 0x00020000);
}

// Column block of the candidate rows K(x_J, x_c), rows 4q + g4 of the
// 16-column tile at `col`; rows at or past j read as zero.  The block has
// kc_rows >= 4 ceil(j/4) rows (padded on the host), so every load is in
// bounds; one lane offset plus a wave-uniform row offset per chunk.
template <int NQ>
__device__ __forceinline__ void load_tile_b(const LocalArgs& a, __amdgpu_buffer_rsrc_t rs, int j, int col,
                                            double (&b)[NQ]) {
  const int g4 = (threadIdx.x & 63) >> 4;
  const int ncs = a.ncs;
  const int voff = (g4 * ncs + col) * 8;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const double v = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, q * 32 * ncs, 0));
    b[q] = 4 * q + g4 < j ? v : 0.0;
  }
}

// Exact ALC of one tile of 16 candidate columns (lane column cl holds
// candidate `col`) at a design size j with NQ = ceil(j/4) K-chunks, from the
// tile's candidate rows b; the value is valid in lanes 0..15.  PRE: a row
// block's K_J^{-1} fragments are all loaded before its chain starts (one
// tile per call: the chain then runs at the matrix cores' pace instead of
// waiting on LDS every other step).
template <int NP, int NQ, bool PRE = false>
__device__ __forceinline__ double alc_tile_exact_q(const LocalArgs& a, const Lds& L, int LD, const double (&b)[NQ],
                                                   double kxcol, int* vflag) {
  const int lane = threadIdx.x & 63;
  const int g4 = lane >> 4, cl = lane & 15;
  // An opaque offset keeps the K_J^{-1} fragments in LDS: hoisted out of the
  // tile loop they would need about NQ * NQ / 4 register pairs.
  int aoff = cl * LD + g4;
  asm volatile("" : "+v"(aoff));
  const double* arow = L.Ki + aoff;
  // Row block by row block: the W chain of a block (NQ accumulations into one
  // register set) is consumed at once by the v and cov chains, whose chunks
  // 4I .. 4I+3 are exactly that block's rows, so the chunk order stays
  // ascending and only one block of W is live.
  // The v and cov chains run on the four-block 4x4x4 FP64 MFMA (a quarter of
  // the work of a 16x16x4 step): block b covers candidates 4b .. 4b+3, its
  // operands A[b][i][k] (lane 16k + 4b + i) and B[b][k][n] (lane 16k + 4b + n)
  // are exactly the loaded kernel-row chunk and a W register, and
  // D[b][i][n] lands in lane 16i + 4b + n.
  //
  // Whole 16-row blocks of W run on 16x16x4; the last NQ % 4 chunks of rows
  // run on 4x4x4, four rows at a time (A[b][i][k] = K^{-1}[4q'+i][4q+k] in
  // every block b, B = the loaded chunk), at the same cost per row, so rows
  // are padded to a multiple of 4 rather than 16.  Its output
  // D[b][i][n] = W[4q'+i][4b+n] sits in lane 16i + 4b + n: the B operand of
  // chunk q' of the v and cov chains, like register r of a 16-row block.
  constexpr int NFULL = NQ / 4;
  double accv = 0.0, accc = 0.0;
#pragma unroll
  for (int I = 0; I < NFULL; ++I) {
    v4d acc = {0.0, 0.0, 0.0, 0.0};
    if constexpr (PRE) {
      double af[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) af[q] = arow[16 * I * LD + 4 * q];
      __builtin_amdgcn_sched_barrier(0);  // (the loads stay ahead of the chain)
#pragma unroll
      for (int q = 0; q < NQ; ++q) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(af[q], b[q], acc, 0, 0, 0);
    } else {
#pragma unroll
      for (int q = 0; q < NQ; ++q)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(arow[16 * I * LD + 4 * q], b[q], acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int q = 4 * I + r;
      accv = __builtin_amdgcn_mfma_f64_4x4x4f64(b[q], acc[r], accv, 0, 0, 0);
      accc = __builtin_amdgcn_mfma_f64_4x4x4f64(L.kx[4 * q + g4], acc[r], accc, 0, 0, 0);
    }
  }
  int aoff4 = (cl & 3) * LD + g4;
  asm volatile("" : "+v"(aoff4));
  const double* a4 = L.Ki + aoff4;
#pragma unroll
  for (int qr = 4 * NFULL; qr < NQ; ++qr) {
    double w4 = 0.0;
    if constexpr (PRE) {
      double af[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) af[q] = a4[4 * qr * LD + 4 * q];
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int q = 0; q < NQ; ++q) w4 = __builtin_amdgcn_mfma_f64_4x4x4f64(af[q], b[q], w4, 0, 0, 0);
    } else {
#pragma unroll
      for (int q = 0; q < NQ; ++q)
        w4 = __builtin_amdgcn_mfma_f64_4x4x4f64(a4[4 * qr * LD + 4 * q], b[q], w4, 0, 0, 0);
    }
    accv = __builtin_amdgcn_mfma_f64_4x4x4f64(b[qr], w4, accv, 0, 0, 0);
    accc = __builtin_amdgcn_mfma_f64_4x4x4f64(L.kx[4 * qr + g4], w4, accc, 0, 0, 0);
  }
  // v_c is the diagonal entry of candidate c = 4b + i: lane 16(c%4) + c; the
  // rows of the cov product are all equal, so every lane holds its column's.
  const double vsum = __shfl(accv, 16 * (cl & 3) + cl, 64);
  const double v = (1.0 + a.g) - vsum;
  const double cov = kxcol - accc;
  if (v > 0.0) return cov * cov / v;
  if (g4 == 0) *vflag = 1;
  return 0.0;
}

// Exhaustive scoring of one step: the waves take tiles round robin; the
// candidate rows of a wave's next tile are loaded while it works on the
// current one.
template <int NP, int NQ>
__device__ __forceinline__ Best score_exact_q(const LocalArgs& a, const Lds& L, int LD, const double* Kc,
                                           const double* kxc, int j, int* vflag) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int cl = lane & 15;
  const int ntiles = a.ncs >> 4;
  Best best = {-__builtin_huge_val(), -__builtin_huge_val(), 0x7fffffff};
  const __amdgpu_buffer_rsrc_t rs = kc_rsrc(a, Kc);
  // Double buffering costs 2 NQ more registers: only for the shorter chains.
  // K(x_c, x) of the tile travels with its rows: a load issued before the
  // next tile's prefetch is waited for without waiting for that prefetch.
  constexpr bool PREFETCH = NQ <= 16;
  double bn[NQ];
  double kxn = 0.0;
  if (PREFETCH && wave < ntiles) {
    kxn = kxc[(wave << 4) + cl];
    load_tile_b<NQ>(a, rs, j, (wave << 4) + cl, bn);
  }
  for (int t = wave; t < ntiles; t += NW) {
    double b[NQ];
    double kxcol;
    if constexpr (PREFETCH) {
#pragma unroll
      for (int q = 0; q < NQ; ++q) b[q] = bn[q];
      kxcol = kxn;
      if (t + NW < ntiles) {
        kxn = kxc[((t + NW) << 4) + cl];
        load_tile_b<NQ>(a, rs, j, ((t + NW) << 4) + cl, bn);
      }
    } else {
      kxcol = kxc[(t << 4) + cl];
      load_tile_b<NQ>(a, rs, j, (t << 4) + cl, b);
    }
    const int c = (t << 4) + cl;
    const double alc = alc_tile_exact_q<NP, NQ>(a, L, LD, b, kxcol, vflag);
    if (lane < 16 && !L.selm[c]) best_push(best, alc, c);
  }
  return best;
}

// Exact tile for a shortlist (mixed form): one tile, dispatched on NQ.
template <int NP, int NQ>
__device__ __forceinline__ double alc_tile_exact_n(const LocalArgs& a, const Lds& L, int LD, const double* Kc,
                                                const double* kxc, int j, int col, int* vflag) {
  double b[NQ];
  const double kxcol = kxc[col];
  load_tile_b<NQ>(a, kc_rsrc(a, Kc), j, col, b);
  return alc_tile_exact_q<NP, NQ>(a, L, LD, b, kxcol, vflag);
}

#define LAGP_CASES_16(M) M(1) M(2) M(3) M(4) M(5) M(6) M(7) M(8) M(9) M(10) M(11) M(12) M(13) M(14) M(15) M(16)
#define LAGP_CASES_32(M) LAGP_CASES_16(M) M(17) M(18) M(19) M(20) M(21) M(22) M(23) M(24) M(25) M(26) M(27) \
  M(28) M(29) M(30) M(31) M(32)

template <int NP>
__device__ __forceinline__ Best score_exact(const LocalArgs& a, const Lds& L, int LD, const double* Kc, const double* kxc, int j,
                            int* vflag) {
  const int nq = (j + 3) >> 2;
#define LAGP_SCORE_CASE(Q) \
  case Q:                  \
    if constexpr (Q <= NP / 4) return score_exact_q<NP, Q>(a, L, LD, Kc, kxc, j, vflag); \
    break;
  switch (nq) { LAGP_CASES_32(LAGP_SCORE_CASE) default: break; }
#undef LAGP_SCORE_CASE
  return Best{-__builtin_huge_val(), -__builtin_huge_val(), 0x7fffffff};
}

template <int NP>
__device__ __forceinline__ double alc_tile_exact(const LocalArgs& a, const Lds& L, int LD, const double* Kc, const double* kxc, int j,
                                 int col, int* vflag) {
  const int nq = (j + 3) >> 2;
#define LAGP_TILE_CASE(Q) \
  case Q:                 \
    if constexpr (Q <= NP / 4) return alc_tile_exact_n<NP, Q>(a, L, LD, Kc, kxc, j, col, vflag); \
    break;
  switch (nq) { LAGP_CASES_32(LAGP_TILE_CASE) default: break; }
#undef LAGP_TILE_CASE
  return 0.0;
}

// --------------------------------------------------------- mixed form ----

typedef float v4f __attribute__((ext_vector_type(4)));

// One rounding in FP32 or FP64 (u32 + u64): the unit of the screen's bounds.
constexpr double SCREEN_U = 0x1.00002p-24;

// A float >= x for x >= 0 (finite or +inf): the nearest float, moved up one
// unit when it fell below x.
__device__ __forceinline__ float f32_up(double x) {
  float f = (float)x;
  if ((double)f < x) f = __uint_as_float(__float_as_uint(f) + 1u);
  return f;
}

// FP32 screen of every candidate at design size j on f32 MFMA (FP32
// products and accumulation) from FP32 copies of the kernel rows and of
// K^{-1}: v = (1+g) - k_c^T K^{-1} k_c, cov = K(x_c,x) - h^T k_c (h =
// K^{-1} k_x), and beside them S_c = sum_i r_i k_c[i] with r_i = sum_l
// |K^{-1}_il|.  Every kernel value lies in [0, 1], so k^T |K^{-1}| k,
// |h|^T k and the error terms of the FP64 scoring's own sums are all at most
// S_c; running-error analysis of the two FP32 contractions (inputs rounded
// once, at most 2j + 4 further roundings, each at most 2 units to allow for
// truncating hardware, subnormals flushed) gives
//   |v_FP32 - v_FP64|     <= (4j + 16) u S_c + 4 u (1 + g) + A
//   |cov_FP32 - cov_FP64| <= (4j + 16) u S_c + 2 u (|K(x_c,x)| + |cov|) + A
// with u one rounding of either precision and A = 2^-100 (1 + sum_i r_i)
// for flushed subnormals.  From these the screen writes an upper bound of the
// candidate's FP64 criterion to scr[c] (rounded up; +inf when v may be <= 0,
// -inf if unavailable) and returns, per thread, the two largest lower
// bounds.  A taken candidate whose v may be <= 0 also gets +inf, so that its
// tile is re-scored and the FP64 form's VNONPOS flag is reproduced.
// Lane layout of v_mfma_f32_16x16x4f32 (gfx950): A[i][k] from lane 16k + i,
// B[k][n] from lane 16k + n, D[i][n] in register i%4 of lane 16(i/4) + n.
// K-chunk (I', c) holds rows 16I' + 4g + c in lane quarter g, so register r
// of row block I (rows 16I + 4g + r) pairs with chunk (I, r) in the epilogue.
template <int NP>
__device__ __forceinline__ Best screen_f32(const LocalArgs& a, const Lds& L, int LD, const float* Kc32,
                                           const double* kxc, int j, float* scr) {
  constexpr int RBMAX = NP / 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g4 = lane >> 4, cl = lane & 15;
  const int nrb = (j + 15) >> 4;
  const int ncs = a.ncs;
  const int ntiles = ncs >> 4;
  const float one_g = (float)(1.0 + a.g);
  const double absl = L.scal[4];
  const double cterm = (4.0 * j + 16.0) * SCREEN_U;
  Best lo2 = {-__builtin_huge_val(), -__builtin_huge_val(), 0x7fffffff};
  for (int t = wave; t < ntiles; t += NW) {
    const int c = (t << 4) + cl;
    float b[RBMAX][4];
#pragma unroll
    for (int I = 0; I < RBMAX; ++I)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * I + 4 * g4 + r;
        b[I][r] = (I < nrb && row < j) ? Kc32[(int64_t)row * ncs + c] : 0.0f;
      }
    float qf = 0.0f, cv = 0.0f, sa = 0.0f;
#pragma unroll
    for (int I = 0; I < RBMAX; ++I) {
      if (I < nrb) {
        v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
        const double* arow = L.Ki + (16 * I + cl) * LD + 4 * g4;
#pragma unroll
        for (int I2 = 0; I2 < RBMAX; ++I2)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if (I2 < nrb && 16 * I2 + r < j)
              acc = __builtin_amdgcn_mfma_f32_16x16x4f32((float)arow[16 * I2 + r], b[I2][r], acc, 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * I + 4 * g4 + r;
          qf = __builtin_fmaf(b[I][r], acc[r], qf);
          cv = __builtin_fmaf((float)L.h[row], b[I][r], cv);
          sa = __builtin_fmaf((float)L.wv[row], b[I][r], sa);
        }
      }
    }
    qf += __shfl_xor(qf, 16, 64);
    qf += __shfl_xor(qf, 32, 64);
    cv += __shfl_xor(cv, 16, 64);
    cv += __shfl_xor(cv, 32, 64);
    sa += __shfl_xor(sa, 16, 64);
    sa += __shfl_xor(sa, 32, 64);
    if (g4 == 0) {
      float hi_f = -__builtin_huge_valf();
      if (c < a.ncand) {
        const double v = (double)(one_g - qf);
        const double kx = kxc[c];
        const double cov = (double)((float)kx - cv);
        // S_c from its FP32 value: at most j + 3 roundings low
        const double S = (double)sa * (1.0 + 0x1p-15);
        const double dv = cterm * S + 4.0 * SCREEN_U * (1.0 + a.g) + absl;
        const double dc = cterm * S + 2.0 * SCREEN_U * (fabs(kx) + fabs(cov)) + absl;
        const bool vpos = v - dv > 0.0;  // then the FP64 v is > 0 as well
        if (!L.selm[c]) {
          double hi = __builtin_huge_val(), lo = 0.0;
          if (vpos) {
            const double ch = fabs(cov) + dc, cm = fmax(fabs(cov) - dc, 0.0);
            hi = ch * ch / (v - dv) * (1.0 + 0x1p-40);
            lo = cm * cm / (v + dv) * (1.0 - 0x1p-40);
          }
          hi_f = hi == hi ? f32_up(hi) : __builtin_huge_valf();
          best_push(lo2, lo == lo ? lo : 0.0, c);
        } else if (!vpos) {
          hi_f = __builtin_huge_valf();
        }
      }
      scr[c] = hi_f;
    }
  }
  return lo2;
}

// Mixed step.  The FP32 screen bounds every available candidate's FP64
// criterion; let T be the second largest lower bound.  The candidates with
// the best and the runner-up FP64 values both have values >= T (the two
// candidates holding the two largest lower bounds reach T), hence upper
// bounds >= T, so re-scoring in FP64 every 16-candidate tile that holds an
// upper bound >= T finds the FP64 argmax (ties to the smaller rank among
// equal values, which are all re-scored) and the FP64 runner-up value; the
// other candidates of those tiles, pushed too, cannot displace either.  When
// half the tiles or more qualify, all are re-scored by the FP64 form's own
// loop (the same values).  L.ints[5] / L.ints[6] receive the candidates
// whose upper bound reached T and the tiles re-scored.  Conditioning only
// worsens as the design grows, so once the screen has failed to rule out
// half the tiles the caller passes screen = false for the location's later
// steps, which are then scored in FP64 directly (the same values again):
// `screen` is cleared here for every thread alike.
template <int NP>
__device__ __forceinline__ Best score_mixed(const LocalArgs& a, const Lds& L, int LD, const double* Kc, const float* Kc32,
                            const double* kxc, int j, bool& screen, int* vflag) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  float* scr = L.scr;
  if (!screen) {  // the screen ruled out too little at an earlier step: FP64 scoring of every tile
    if (tid == 0) {
      L.ints[5] = a.ncand - j;
      L.ints[6] = a.ncs >> 4;
    }
    return score_exact<NP>(a, L, LD, Kc, kxc, j, vflag);
  }
  // h = K^{-1} k_x for the screen's covariance term, r = row sums of |K^{-1}|
  for (int i = tid; i < j; i += blockDim.x) {
    double s = 0.0, r = 0.0;
    for (int k = 0; k < j; ++k) {
      const double kik = L.Ki[k * LD + i];
      s = __builtin_fma(kik, L.kx[k], s);
      r += fabs(kik);
    }
    L.h[i] = s;
    L.wv[i] = r * (1.0 + 0x1p-40);  // (j < 2^11 additions of non-negative terms)
  }
  __syncthreads();
  if (tid == 0) {
    double r1 = 0.0;
    for (int i = 0; i < j; ++i) r1 += L.wv[i];
    L.scal[4] = 0x1p-100 * (1.0 + 2.0 * r1);
    L.ints[5] = 0;
    L.ints[7] = 0;
  }
  __syncthreads();
  const Best lo2 = screen_f32<NP>(a, L, LD, Kc32, kxc, j, scr);
  block_best(L, lo2);  // L.scal[2]: the second largest lower bound
  const double T = L.scal[2];
  const int ntiles = a.ncs >> 4;
  for (int t = tid; t < ntiles; t += blockDim.x) {
    int hits = 0;
    bool flag = false;
    for (int u = 0; u < 16; ++u) {
      const float h = scr[16 * t + u];
      const bool in = h > -__builtin_huge_valf() && (double)h >= T;
      flag |= in;
      hits += (in && !L.selm[16 * t + u]) ? 1 : 0;
    }
    if (flag) L.shortlist[atomicAdd(&L.ints[7], 1)] = t;
    if (hits) atomicAdd(&L.ints[5], hits);
  }
  __syncthreads();
  const int nlist = L.ints[7];  // (read by every thread after the barrier)
  const bool all = 2 * nlist >= ntiles;
  screen = !all;
  if (tid == 0) L.ints[6] = all ? ntiles : nlist;
  if (all) return score_exact<NP>(a, L, LD, Kc, kxc, j, vflag);
  // the listed tiles in FP64, one per wave at a time (any order: the
  // arg-max merge orders by value, then rank)
  Best best = {-__builtin_huge_val(), -__builtin_huge_val(), 0x7fffffff};
  for (int t = wave; t < nlist; t += NW) {
    const int c = (L.shortlist[t] << 4) + (lane & 15);
    const double alc = alc_tile_exact<NP>(a, L, LD, Kc, kxc, j, c, vflag);
    if (lane < 16 && !L.selm[c]) best_push(best, alc, c);
  }
  return best;
}

// ------------------------------------------------------------ update -----

// Grow K^{-1} from j x j to (j+1) x (j+1) with candidate rank cs, design row
// `row` (the partitioned inverse of Sec. 3.1), append it to the design, and
// compute its kernel row against every candidate.  cs = ncand: a row that is
// not among the candidates (a ray snapped over the whole design).  Returns
// v_j of the added point.
template <bool KROWS>  // exhaustive forms keep every candidate's kernel row
__device__ __forceinline__ double add_point(const LocalArgs& a, const Lds& L, int LD, double* Kc, float* Kc32, const double* kxc,
                            const double* Xc, int j, int cs, int32_t row) {
  const int tid = threadIdx.x;
  const int ncs = a.ncs, p = a.p;
  const bool listed = cs < a.ncand;
  // the new point's coordinates (gathered in the prologue, or the design's
  // own) join the design's
  for (int k = tid; k < p; k += blockDim.x)
    L.xj[j * p + k] = listed ? Xc[(int64_t)cs * p + k] : a.X[(int64_t)row * p + k];
  __syncthreads();
  const double* xs = L.xj + j * p;
  // K(x_J, x_s): the same arguments, in the same order, as the stored rows
  // K(x_{J_i}, x_c) (design point first), hence the same bits
  for (int i = tid; i < j; i += blockDim.x) L.col[i] = corr(L.xj + i * p, xs, p, L.w0, a.w, a.dlen);
  __syncthreads();
  // Kinv is exactly symmetric (every update adds g_i g_k v with
  // g_i g_k == g_k g_i), so thread i reads column i: same values, same
  // order, and consecutive threads hit consecutive LDS banks
  for (int i = tid; i < j; i += blockDim.x) {
    double s = 0.0;
    for (int k = 0; k < j; ++k) s = __builtin_fma(L.Ki[k * LD + i], L.col[k], s);
    L.wv[i] = s;
  }
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int i = 0; i < j; ++i) s = __builtin_fma(L.col[i], L.wv[i], s);
    L.scal[0] = (1.0 + a.g) - s;
  }
  __syncthreads();
  const double v = L.scal[0];
  for (int i = tid; i < j; i += blockDim.x) L.gv[i] = -L.wv[i] / v;
  __syncthreads();
  for (int t = tid; t < j * j; t += blockDim.x) {
    const int i = t / j, k = t - i * j;
    L.Ki[i * LD + k] = __builtin_fma(L.gv[i] * L.gv[k], v, L.Ki[i * LD + k]);
  }
  for (int i = tid; i < j; i += blockDim.x) {
    L.Ki[i * LD + j] = L.gv[i];
    L.Ki[j * LD + i] = L.gv[i];
  }
  if (tid == 0) {
    L.Ki[j * LD + j] = 1.0 / v;
    L.J[j] = cs;
    L.jrow[j] = row;
    if (listed) {
      L.selm[cs] = 1;
      L.kx[j] = kxc[cs];
    } else {
      L.kx[j] = corr(xs, L.x, p, L.w0, a.w, a.dlen);  // K(x_s, x) as kxc holds it
    }
  }
  if (KROWS && j + 1 < a.n) {
    double* row = Kc + (int64_t)j * ncs;
    float* row32 = Kc32 ? Kc32 + (int64_t)j * ncs : nullptr;
    if (p <= 8) {
      kernel_row<8>(a, L.w0, xs, Xc, row, row32);
    } else {
      for (int c = tid; c < ncs; c += blockDim.x) {
        const double kv = c < a.ncand ? corr(xs, Xc + (int64_t)c * p, p, L.w0, a.w, a.dlen) : 0.0;
        row[c] = kv;
        if (row32) row32[c] = (float)kv;
      }
    }
  }
  __syncthreads();
  return v;
}

// ---------------------------------------------------------- ray search ---


// Gaussian correlation of two vectors unrolled to the compile-time dimension
// P (0: runtime p), first argument first (same arithmetic as corr()).
template <int P>
__device__ __forceinline__ double corr_regs(const double* u, const double* v, int p, double w0, const double* w,
                                            int dlen) {
  constexpr int PM = P > 0 ? P : LAGP_MAX_DIM;
  double acc = 0.0;
  if (dlen == 1) {
#pragma unroll
    for (int k = 0; k < PM; ++k)
      if (P > 0 || k < p) {
        const double t = u[k] - v[k];
        acc = __builtin_fma(t, t, acc);
      }
    return gexp(-(acc * w0));
  }
#pragma unroll
  for (int k = 0; k < PM; ++k)
    if (P > 0 || k < p) {
      const double t = u[k] - v[k];
      acc = __builtin_fma(t * t, w[k], acc);
    }
  return gexp(-acc);
}

// Point z = a + s dir of ray r (z = a exactly at the start), from the ray's
// start and clipped direction in LDS.
template <int P>
__device__ __forceinline__ void ray_point(const Lds& L, int p, int r, double s, bool at_start, double* z) {
  constexpr int PM = P > 0 ? P : LAGP_MAX_DIM;
#pragma unroll
  for (int k = 0; k < PM; ++k)
    if (P > 0 || k < p) z[k] = at_start ? L.ra[r * p + k] : __builtin_fma(s, L.rdir[r * p + k], L.ra[r * p + k]);
}

// Ray objective ALC for the wave's slots, one lane per slot: lane t (< RB)
// passes its slot's ray rid, parameter s and flag ev and receives the value.
// Kernel vectors k_z on the lanes; K^{-1} k_z one row per lane (column reads
// of the symmetric inverse), the slots' chains interleaved; the six inner
// products k_z.w and w.k_x (w = K^{-1} k_z) as chains of 4x4x4 FP64 MFMAs,
// which add their four terms in order: chain c = 2t (v) or 2t+1 (cov) is the
// diagonal entry i = c % 4 of block c / 4, its operands A[b][i][k] and
// B[b][k][i] both in lane 16k + c.  Sums run in index order; the LDS vectors
// are zero past j (as is K^{-1}), so padded terms add fma(0, 0, t) = t only.
// xi: the lane's design point J_lane (registers).
template <int P, int NH>
__device__ __forceinline__ double ray_alc_lanes(const LocalArgs& a, const Lds& L, int LD, int j, const double* xi,
                                                int rid, double s, bool ev, bool at_start, int* vflag) {
  static_assert(NH == 2 || NH == 4, "design rows in two or four 64-row halves");
  constexpr int PM = P > 0 ? P : LAGP_MAX_DIM;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int p = a.p;
  int rids[RB];
  double ss[RB];
  bool evs[RB];
#pragma unroll
  for (int t = 0; t < RB; ++t) {
    rids[t] = __shfl(rid, t, 64);
    ss[t] = __shfl(s, t, 64);
    evs[t] = __shfl((int)ev, t, 64) != 0;
  }
#pragma unroll
  for (int t = 0; t < RB; ++t) {
    if (!evs[t]) continue;
    double z[PM];
    ray_point<P>(L, p, rids[t], ss[t], at_start, z);
    double* kz = L.kzb + (wave * RB + t) * L.kzs;
    if (lane < j) kz[lane] = corr_regs<P>(xi, z, p, L.w0, a.w, a.dlen);
#pragma unroll
    for (int h = 1; h < NH; ++h)
      if (lane + 64 * h < j) kz[lane + 64 * h] = corr_regs<P>(L.xj + (lane + 64 * h) * p, z, p, L.w0, a.w, a.dlen);
  }
  // K(z_t, x) on lane t
  double kzx = 0.0;
  if (lane < RB && ev) {
    double z[PM];
    ray_point<P>(L, p, rid, s, at_start, z);
    kzx = corr_regs<P>(z, L.x, p, L.w0, a.w, a.dlen);
  }
  wave_sync();
  const int nb = (j + 7) >> 3;
  const int KZS = L.kzs;
  const double* kzw = L.kzb + wave * RB * KZS;
  double* wzw = L.wvb + wave * RB * KZS;
#pragma unroll
  for (int h = 0; h < NH; ++h) {
    const int i = lane + 64 * h;
    if (i < j) {
      double acc[RB];
#pragma unroll
      for (int t = 0; t < RB; ++t) acc[t] = 0.0;
      for (int b = 0; b < nb; ++b) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int k = 8 * b + u;
          const double kik = L.Ki[k * LD + i];  // column i == row i
#pragma unroll
          for (int t = 0; t < RB; ++t) acc[t] = __builtin_fma(kik, kzw[t * KZS + k], acc[t]);
        }
      }
#pragma unroll
      for (int t = 0; t < RB; ++t)
        if (evs[t]) wzw[t * KZS + i] = acc[t];
    }
  }
  wave_sync();
  // the inner products on 4x4x4 MFMA (chain c = lane % 16, term 4q + lane / 16)
  const int cc = lane & 15, k4 = lane >> 4;
  const bool on = cc < 2 * RB;
  const int tc = on ? cc >> 1 : 0;
  const double* pu = (cc & 1) ? wzw + tc * KZS : kzw + tc * KZS;
  const double* pv = (cc & 1) ? L.kx : wzw + tc * KZS;
  double dacc = 0.0;
  const int nq = (j + 3) >> 2;
  for (int q = 0; q < nq; ++q) {
    const double av = on ? pu[4 * q + k4] : 0.0;
    const double bv = on ? pv[4 * q + k4] : 0.0;
    dacc = __builtin_amdgcn_mfma_f64_4x4x4f64(av, bv, dacc, 0, 0, 0);
  }
  // chain c's sum sits in lane 16 (c % 4) + c
  const int cv = 2 * (lane < RB ? lane : 0), cw = cv + 1;
  const double sv = __shfl(dacc, 16 * (cv & 3) + cv, 64);
  const double sw = __shfl(dacc, 16 * (cw & 3) + cw, 64);
  double out = 0.0;
  if (lane < RB && ev) {
    const double v = (1.0 + a.g) - sv;
    const double cov = kzx - sw;
    if (v > 0.0) {
      out = cov * cov / v;
    } else {
      *vflag = 1;
    }
  }
  wave_sync();
  return out;
}

// Brent's (1973) minimiser of f(s) = -ALC on [0, 1], one slot per lane
// (lane t < RB runs slot t's scalar recurrence; the evaluations of all slots
// share one pass): golden-section steps, replaced by the parabola through
// the three best points when that step lands inside the bracket and is
// shorter than half the step before last; never closer than
// tol1 = 2^-26 |x| + tol/3 to the best point; a slot stops when its bracket
// half-width about the best point is within 2 tol1 (or after brent_maxit
// steps).  A parabolic step that would land within 2 tol1 of an end becomes
// tol1 towards the midpoint (downwards when x is at or above it), and a step
// shorter than tol1 becomes tol1 in its own direction (downwards when zero),
// the conventions of the Brent_fmin routine Sec. 4 names.  eval(s, ev)
// returns, on every lane t < nl with ev set, the objective's ALC at lane
// t's parameter s (one call serves every lane).  Returns the minimiser on
// lane t, its value in *fbest.
template <bool BLOCK, class Eval>
__device__ __forceinline__ double brent_lanes(const LocalArgs& a, int nl, bool live, const Eval& eval, double* fbest,
                                              int* nev) {
  const double gold = 0x1.8722191a02d60p-2;  // (3 - sqrt 5)/2
  const double sqeps = 0x1p-26;              // sqrt(2^-52)
  const double tol = a.brent_tol;
  const int lane = threadIdx.x & 63;
  double lo = 0.0, hi = 1.0;
  double x = lo + gold * (hi - lo);
  double w = x, v = x;
  bool run = live && lane < nl;
  double f0;
  if constexpr (BLOCK)
    f0 = eval(x, run, nullptr);  // (the first evaluation runs whatever the lanes hold)
  else
    f0 = eval(x, run);
  double fx = -f0, fw = fx, fv = fx;
  double step = 0.0, prev = 0.0;
  int it = 0;
  for (;;) {
    double u = x;
    bool ev = false;
    if (run) {
      const double mid = 0.5 * (lo + hi);
      const double tol1 = sqeps * fabs(x) + tol / 3.0;
      const double tol2 = 2.0 * tol1;
      if (it >= a.brent_maxit || fabs(x - mid) <= tol2 - 0.5 * (hi - lo)) {
        run = false;
      } else {
        bool para = false;
        if (fabs(prev) > tol1) {
          const double rr = (x - w) * (fx - fv);
          double q = (x - v) * (fx - fw);
          double num = (x - v) * q - (x - w) * rr;
          double den = 2.0 * (q - rr);
          if (den > 0.0) num = -num;
          den = fabs(den);
          const double older = prev;
          prev = step;
          if (fabs(num) < fabs(0.5 * den * older) && num > den * (lo - x) && num < den * (hi - x)) {
            step = num / den;
            const double uu = x + step;
            if (uu - lo < tol2 || hi - uu < tol2) step = (x >= mid) ? -tol1 : tol1;
            para = true;
          }
        }
        if (!para) {
          prev = (x >= mid) ? lo - x : hi - x;
          step = gold * prev;
        }
        u = (fabs(step) >= tol1) ? x + step : ((step > 0.0) ? x + tol1 : x - tol1);
        ev = true;
      }
    }
    // (BLOCK: the evaluations span the workgroup, so every wave leaves
    // together: the evaluation's first barrier also carries whether any lane
    // evaluates, and it returns at once when none does)
    double fu;
    if constexpr (BLOCK) {
      bool go = true;
      fu = -eval(u, ev, &go);
      if (!go) break;
    } else {
      if (!__any(ev)) break;
      fu = -eval(u, ev);
    }
    if (ev) {
      ++it;
      if (fu <= fx) {
        if (u >= x) lo = x; else hi = x;
        v = w; fv = fw;
        w = x; fw = fx;
        x = u; fx = fu;
      } else {
        if (u < x) lo = u; else hi = u;
        if (fu <= fw || w == x) {
          v = w; fv = fw;
          w = u; fw = fu;
        } else if (fu <= fv || v == x || v == w) {
          v = u; fv = fu;
        }
      }
    }
  }
  *fbest = fx;
  *nev = (live && lane < nl) ? it + 1 : 0;  // objective evaluations, the first included
  return x;
}

// Round-robin starts of a ray step (Sec. 4): the R remaining candidates from
// rank k0 = t mod floor(sqrt t) on, t = j - n0 + 1, i.e. the available ranks
// numbered k0 .. k0 + R - 1 among the available ones in rank order.  Wave 0
// numbers 64 ranks at a time by a ballot.  Leaves their number in L.ints[2]
// (fewer than R only when the list runs out).
__device__ __forceinline__ int ray_starts(const LocalArgs& a, const Lds& L, int j, int n0) {
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    const int t = j - n0 + 1;
    int rt = 0;
    while ((rt + 1) * (rt + 1) <= t) ++rt;
    const int k0 = rt > 0 ? t % rt : 0;
    int seen = 0;  // available ranks below c0 (uniform)
    for (int c0 = 0; c0 < a.ncand && seen < k0 + a.numrays; c0 += 64) {
      const int c = c0 + lane;
      const bool av = c < a.ncand && !L.selm[c];
      const uint64_t bal = __ballot(av);
      const int num = seen + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                            __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
      if (av && num >= k0 && num < k0 + a.numrays) L.starts[num - k0] = c;
      seen += __builtin_popcountll(bal);
    }
    const int got = seen - k0 < 0 ? 0 : (seen - k0 < a.numrays ? seen - k0 : a.numrays);
    if (lane == 0) L.ints[2] = got;
  }
  __syncthreads();
  return L.ints[2];
}

// Segment of ray r (Sec. 4): from its start a, away from x, ten times
// |a - x| long, cut at the design's bounding box; returns the cut fraction
// tau, and writes a and the clipped direction to L.ra, L.rdir when `write`.
// The start's coordinates come from the location's gathered candidate
// coordinates Xc (the same values as its design row).
template <int P>
__device__ __forceinline__ double ray_segment(const LocalArgs& a, const Lds& L, const double* Xc, int r, bool write) {
  constexpr int PM = P > 0 ? P : LAGP_MAX_DIM;
  const int p = a.p;
  const double* src = Xc + (int64_t)L.starts[r] * p;
  double ak[PM], dk[PM];
  double tt = 1.0;
#pragma unroll
  for (int k = 0; k < PM; ++k) {
    ak[k] = 0.0;
    dk[k] = 0.0;
    if (P > 0 || k < p) {
      ak[k] = src[k];
      dk[k] = 10.0 * (ak[k] - L.x[k]);
      if (dk[k] > 0.0) tt = fmin(tt, (a.hi[k] - ak[k]) / dk[k]);
      else if (dk[k] < 0.0) tt = fmin(tt, (a.lo[k] - ak[k]) / dk[k]);
    }
  }
  if (tt < 0.0) tt = 0.0;
  if (write)
#pragma unroll
    for (int k = 0; k < PM; ++k)
      if (P > 0 || k < p) {
        L.ra[r * p + k] = ak[k];
        L.rdir[r * p + k] = tt * dk[k];
      }
  return tt;
}

// Snap over the whole design (ray search not restricted to the N' nearest,
// Sec. 5): the nearest design row to z outside the design and the step's
// starts, in the order a candidate list of the whole design would give:
// (squared distance to z, squared distance to x, row), each squared
// distance in dimension order with one fma per term (equal distances to z
// go to the row of lower rank, the nearer to x).  The design's cell grid is
// searched in boxes of cells around z's cell, growing until every cell
// outside the box is provably farther than the best row found (a row in a
// cell r + 1 or more cells away along a grid coordinate lies at least
// (r - 1) narrowest cell widths away: one width of slack per side for the
// rounding of the cell assignment).  Returns the row's candidate rank when
// it is a candidate, else ncand with the row in L.ints[8]; -1 if no row is
// left.
struct Near {
  double dz, dx;  // squared distances to z and to x
  int row;
};

__device__ __forceinline__ bool near_before(const Near& a, const Near& b) {
  return a.dz < b.dz || (a.dz == b.dz && (a.dx < b.dx || (a.dx == b.dx && a.row < b.row)));
}

// Block-wide first of the per-thread Nears (result in every thread).
__device__ __forceinline__ Near block_near(const Lds& L, Near b) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int m = 32; m >= 1; m >>= 1) {
    Near o;
    o.dz = shfl_xor_d(b.dz, m);
    o.dx = shfl_xor_d(b.dx, m);
    o.row = shfl_xor_i(b.row, m);
    if (near_before(o, b)) b = o;
  }
  if (lane == 0) {
    L.redv[2 * wave] = b.dz;
    L.redv[2 * wave + 1] = b.dx;
    L.redi[wave] = b.row;
  }
  __syncthreads();
  Near r = {L.redv[0], L.redv[1], L.redi[0]};
  const int nw = blockDim.x >> 6;
  for (int w = 1; w < nw; ++w) {
    const Near o = {L.redv[2 * w], L.redv[2 * w + 1], L.redi[w]};
    if (near_before(o, r)) r = o;
  }
  __syncthreads();  // (the words are rewritten by the next reduction)
  return r;
}

__device__ int snap_design(const LocalArgs& a, const Lds& L, const int32_t* C, const double (&z)[LAGP_MAX_DIM], int j,
                           int ns) {
  const GridDev& g = a.grid;
  const int tid = threadIdx.x, nt = blockDim.x, p = a.p;
  int cz[GRID_Q] = {0, 0, 0};
  for (int k = 0; k < g.q; ++k) cz[k] = grid_coord(g, k, z[k]);
  // a row is excluded when it is in the design or a start of this step
  const auto excluded = [&](int32_t row) {
    for (int i = 0; i < j; ++i)
      if (L.jrow[i] == row) return true;
    for (int r = 0; r < ns; ++r)
      if (C[L.starts[r]] == row) return true;
    return false;
  };
  Near nb = {__builtin_huge_val(), __builtin_huge_val(), 0x7fffffff};
  Near best = nb;
  int rdone = -1;
  for (int r = 0;; r = r < 4 ? r + 1 : r + r / 3) {
    int b0[GRID_Q], bn[GRID_Q];
    bool all = true;
    for (int k = 0; k < GRID_Q; ++k) {
      const int lo = cz[k] - r > 0 ? cz[k] - r : 0;
      const int hi = cz[k] + r < g.G[k] - 1 ? cz[k] + r : g.G[k] - 1;
      b0[k] = lo;
      bn[k] = hi - lo + 1;
      all = all && lo == 0 && hi == g.G[k] - 1;
    }
    const int64_t total = (int64_t)bn[0] * bn[1] * bn[2];
    for (int64_t t = tid; t < total; t += nt) {
      int c[GRID_Q];
      c[0] = b0[0] + (int)(t % bn[0]);
      c[1] = b0[1] + (int)((t / bn[0]) % bn[1]);
      c[2] = b0[2] + (int)(t / ((int64_t)bn[0] * bn[1]));
      int cheb = 0;
      for (int k = 0; k < GRID_Q; ++k) {
        const int dk = c[k] > cz[k] ? c[k] - cz[k] : cz[k] - c[k];
        cheb = dk > cheb ? dk : cheb;
      }
      if (cheb <= rdone) continue;  // examined in an earlier box
      const int64_t cell = grid_cell(g, c);
      const int e1 = g.start[cell + 1];
      for (int e = g.start[cell]; e < e1; ++e) {
        const double* xe = g.Xs + (int64_t)e * p;
        double acc = 0.0;
        for (int k = 0; k < p; ++k) {
          const double dz = xe[k] - z[k];
          acc = __builtin_fma(dz, dz, acc);
        }
        if (!(acc <= nb.dz)) continue;  // farther than this thread's best (or NaN)
        double dxx = 0.0;  // the row's squared distance to x, as the candidate lists order it
        for (int k = 0; k < p; ++k) {
          const double dk = xe[k] - L.x[k];
          dxx = __builtin_fma(dk, dk, dxx);
        }
        const Near o = {acc, dxx, g.rows[e]};
        if (near_before(o, nb) && !excluded(o.row)) nb = o;
      }
    }
    best = block_near(L, nb);
    const double lb = (double)(r - 1) * g.wmin;
    if (all || (r >= 1 && best.dz < lb * lb * (1.0 - 0x1p-40))) break;
    rdone = r;
  }
  const int found = best.row;
  if (found == 0x7fffffff) return -1;
  // its rank among the candidates, if it is one
  if (tid == 0) L.ints[9] = -1;
  __syncthreads();
  for (int c = tid; c < a.ncand; c += nt)
    if (C[c] == found) L.ints[9] = c;
  __syncthreads();
  const int rk = L.ints[9];
  if (rk >= 0) return rk;
  if (tid == 0) L.ints[8] = found;
  __syncthreads();
  return a.ncand;
}

// The end of a ray step, once every ray's value and s* are in L.rval, L.rs:
// the best ray (lowest on ties), its start when s* = 0, else its optimum
// snapped to the nearest candidate outside the design and the starts.
// Returns the chosen rank; *b1, *b2 the best and runner-up ray values.
template <int P>
__device__ __forceinline__ int ray_finish(const LocalArgs& a, const Lds& L, const int32_t* C, const double* Xc, int j,
                                          int ns, double* b1, double* b2) {
  constexpr int PM = P > 0 ? P : LAGP_MAX_DIM;
  constexpr int G = PM <= 8 ? 4 : 1;  // candidates whose coordinates are loaded together
  const int tid = threadIdx.x, p = a.p;
  __syncthreads();
  if (tid == 0) {
    double bv = -__builtin_huge_val(), sv = -__builtin_huge_val();
    int br = 0, esum = 0, emax = 0;
    for (int r = 0; r < ns; ++r) {
      esum += L.rev[r];
      emax = L.rev[r] > emax ? L.rev[r] : emax;
      const double vr = L.rval[r];
      if (vr > bv) {
        sv = bv; bv = vr; br = r;
      } else if (vr > sv) {
        sv = vr;
      }
    }
    L.ints[3] = br;
    L.ints[5] = esum;
    L.ints[6] = emax;
    L.scal[1] = bv;
    L.scal[2] = sv;
    L.scal[3] = L.rs[br];
  }
  __syncthreads();
  const int br = L.ints[3];
  const double sw = L.scal[3];
  *b1 = L.scal[1];
  *b2 = L.scal[2];
  if (sw == 0.0) return L.starts[br];
  const double* ar = L.ra + br * p;
  const double* dr = L.rdir + br * p;
  // snap z* = a + s* dir to the nearest candidate outside J and the starts
  // (the starts are flagged unavailable for the scan, 2 = start, and
  // released after it); over the whole design, the same scan first
  for (int r = tid; r < ns; r += blockDim.x) L.selm[L.starts[r]] = 2;
  __syncthreads();
  double zs[PM];
#pragma unroll
  for (int k = 0; k < PM; ++k) zs[k] = (P > 0 || k < p) ? __builtin_fma(sw, dr[k], ar[k]) : 0.0;
  Best nb = {-__builtin_huge_val(), -__builtin_huge_val(), 0x7fffffff};  // maximise -d2
  const int nt = blockDim.x;
  for (int c0 = tid; c0 < a.ncand; c0 += G * nt) {
    // the coordinates of G candidates (gathered by this thread in the
    // prologue) are loaded before the first is used
    double xc[G][PM];
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const int c = c0 + u * nt < a.ncand ? c0 + u * nt : c0;
#pragma unroll
      for (int k = 0; k < PM; ++k) xc[u][k] = (P > 0 || k < p) ? Xc[(int64_t)c * p + k] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const int c = c0 + u * nt;
      if (c >= a.ncand || L.selm[c]) continue;
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < PM; ++k)
        if (P > 0 || k < p) {
          const double t = xc[u][k] - zs[k];
          acc = __builtin_fma(t, t, acc);
        }
      best_push(nb, -acc, c);
    }
  }
  block_best(L, nb);  // (its barriers order the scan before the release)
  for (int r = tid; r < ns; r += blockDim.x) L.selm[L.starts[r]] = 0;
  __syncthreads();
  if (!a.snap_full) return L.ints[0];
  // Whole design.  The list holds the ncand nearest rows to x (as the
  // candidate search writes them), so a row outside it lies at least
  // R = |x_last - x| from x and at least R - |z* - x| from z*: when that
  // exceeds the best candidate's distance delta (with a 2^-40 relative
  // margin for the roundings of the three distances), no other row can be
  // nearer or tie, and the candidate is the design's nearest allowed row
  // (equal distances among candidates already go to the lower rank, nearer
  // to x).  Otherwise the design's cell grid is searched.
  {
    const double* xl = Xc + (int64_t)(a.ncand - 1) * p;
    double r2 = 0.0, q2 = 0.0;
#pragma unroll
    for (int k = 0; k < PM; ++k)
      if (P > 0 || k < p) {
        const double t = xl[k] - L.x[k], u = zs[k] - L.x[k];
        r2 = __builtin_fma(t, t, r2);
        q2 = __builtin_fma(u, u, q2);
      }
    const double d2 = -L.scal[1];  // (+inf when no candidate is available)
    const double e = 0x1p-40;
    if (__builtin_sqrt(r2) * (1.0 - e) - __builtin_sqrt(q2) * (1.0 + e) > __builtin_sqrt(d2) * (1.0 + e))
      return L.ints[0];
  }
  double zf[LAGP_MAX_DIM];
#pragma unroll
  for (int k = 0; k < LAGP_MAX_DIM; ++k) zf[k] = k < p ? __builtin_fma(sw, dr[k], ar[k]) : 0.0;
  return snap_design(a, L, C, zf, j, ns);
}

// One ray-search step at design size j: returns the chosen candidate rank,
// the best and runner-up ray values in *b1, *b2.  NH: 64-row parts of the
// design (2 up to n = 128, 4 up to 256).
template <int P, int NH>
__device__ __forceinline__ int ray_step(const LocalArgs& a, const Lds& L, int LD, const int32_t* C, const double* Xc, int j,
                                       int n0, double* b1, double* b2, int* vflag) {
  constexpr int PM = P > 0 ? P : LAGP_MAX_DIM;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int p = a.p;
  const int ns = ray_starts(a, L, j, n0);
  double xi[PM];
#pragma unroll
  for (int k = 0; k < PM; ++k) xi[k] = ((P > 0 || k < p) && lane < j) ? L.xj[lane * p + k] : 0.0;
  // wave w takes rays w, w + NW, ...: RB of them at a time
  for (int r0 = wave; r0 < ns; r0 += NW * RB) {
    int rid[RB];
    bool valid[RB];
    double tau[RB];
#pragma unroll
    for (int t = 0; t < RB; ++t) {
      rid[t] = r0 + NW * t;
      valid[t] = rid[t] < ns;
      tau[t] = 0.0;
      if (!valid[t]) {
        rid[t] = r0;  // a valid index; the slot is never evaluated
        continue;
      }
      // (every lane computes the same values; lane 0 writes them)
      tau[t] = ray_segment<P>(a, L, Xc, rid[t], lane == 0);
    }
    wave_sync();
    // slot t on lane t from here on
    int my_rid = rid[0];
    bool my_valid = valid[0], my_live;
    double my_tau = tau[0];
#pragma unroll
    for (int t = 1; t < RB; ++t)
      if (lane == t) {
        my_rid = rid[t];
        my_valid = valid[t];
        my_tau = tau[t];
      }
    my_valid = my_valid && lane < RB;
    const double a0 = ray_alc_lanes<P, NH>(a, L, LD, j, xi, my_rid, 0.0, my_valid, true, vflag);
    my_live = my_valid && my_tau > 0.0;
    double fb = 0.0;
    int nev = 0;
    const auto eval = [&](double s, bool e) {
      return ray_alc_lanes<P, NH>(a, L, LD, j, xi, my_rid, s, e, false, vflag);
    };
    const double xb = brent_lanes<false>(a, RB, my_live, eval, &fb, &nev);
    if (my_valid) {
      L.rev[my_rid] = nev;
      double sst = 0.0, val = a0;
      if (my_live) {
        sst = xb;
        val = -fb;
        if (a0 >= val) {
          sst = 0.0;
          val = a0;
        }
      }
      L.rval[my_rid] = val;
      L.rs[my_rid] = sst;
    }
    wave_sync();
  }
  return ray_finish<P>(a, L, C, Xc, j, ns, b1, b2);
}

// ------------------------------------------------ ray search on one tile --
//
// All rays of a step (R <= 16) searched by one wave in lockstep: ray t's
// Brent recurrence runs on lane t, and each round evaluates the objective at
// every live ray's current point as one 16-column tile of the exact scoring
// above.  Column t of the tile is ray t's point z_t: its kernel column
// K(x_J, z_t) is computed straight into the MFMA B layout (lane 16k + t
// holds K(x_{4q+k}, z_t) for chunk q, zero past j) and K(z_t, x) beside it,
// and alc_tile_exact_q gives (K(z_t,x) - k_t^T K^{-1} k_x)^2 /
// ((1+g) - k_t^T K^{-1} k_t) with every sum in index order: the same value,
// bit for bit, as the per-ray form above.  Columns past R, and rays not
// evaluated this round, hold zero kernel columns (v = 1 + g, no flag).

// corr_regs with the straight-line exp (gexp_with: the same values, no
// branches), so that independent evaluations interleave.
template <int P>
__device__ __forceinline__ double corr_regs_bf(const double* u, const double* v, int p, double w0, const double* w,
                                               int dlen) {
  constexpr int PM = P > 0 ? P : LAGP_MAX_DIM;
  double acc = 0.0;
  if (dlen == 1) {
#pragma unroll
    for (int k = 0; k < PM; ++k)
      if (P > 0 || k < p) {
        const double t = u[k] - v[k];
        acc = __builtin_fma(t, t, acc);
      }
    return gexp_with(-(acc * w0), gexp_coef);
  }
#pragma unroll
  for (int k = 0; k < PM; ++k)
    if (P > 0 || k < p) {
      const double t = u[k] - v[k];
      acc = __builtin_fma(t * t, w[k], acc);
    }
  return gexp_with(-acc, gexp_coef);
}

// Kernel columns of the round's ray points into the B layout in LDS: lane
// 16k + t writes K(x_{4q+k}, z_t) to kcol[64 q + lane] for q < nq (zero past
// j, or when ray t is not evaluated), and returns K(z_t, x) in wave 0 (zero
// likewise).  Groups of four chunks go to the waves round robin, every lane
// alike (rows past j read a valid row and are masked after), their exps in
// lockstep; K(z, x) rides along as a fifth exp of wave 0's first group.  The
// arithmetic of corr() per value (ISO: the isotropic form; x - z squares to
// the same value as z - x).
template <int P, bool ISO>
__device__ __forceinline__ double ray_columns_t(const LocalArgs& a, const Lds& L, int j, int nq, bool et,
                                                const double* z, double* kcol) {
  constexpr int PM = P > 0 ? P : LAGP_MAX_DIM;
  const int lane = threadIdx.x & 63;
  const int g4 = lane >> 4;
  const int p = a.p;
  // (the wave index as a scalar: the branches below are whole-wave)
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), nwv = blockDim.x >> 6;
  auto d2 = [&](const double* xi) {
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < PM; ++k)
      if (P > 0 || k < p) {
        const double t = xi[k] - z[k];
        acc = ISO ? __builtin_fma(t, t, acc) : __builtin_fma(t * t, a.w[k], acc);
      }
    return ISO ? -(acc * L.w0) : -acc;
  };
  auto store = [&](int q0, const double* e) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {  // (kcol holds whole groups of four chunks)
      const int i = 4 * (q0 + u) + g4;
      kcol[64 * (q0 + u) + lane] = (et && i < j) ? e[u] : 0.0;
    }
  };
  double kx = 0.0;
  int q0 = 4 * wv;
  if (wv == 0) {  // (wave 0 always has a group: nq >= 1)
    double e[5];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = 4 * u + g4;
      e[u] = d2(L.xj + (i < j ? i : 0) * p);
    }
    e[4] = d2(L.x);
    gexp_lockstep<5>(e);
    store(0, e);
    kx = e[4];
    q0 += 4 * nwv;
  }
  for (; q0 < nq; q0 += 4 * nwv) {
    double e[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = 4 * (q0 + u) + g4;
      e[u] = d2(L.xj + (i < j ? i : 0) * p);
    }
    gexp4(e);
    store(q0, e);
  }
  return et ? kx : 0.0;
}

template <int P>
__device__ __forceinline__ double ray_columns(const LocalArgs& a, const Lds& L, int j, int nq, int R, bool at_start,
                                              double* kcol) {
  constexpr int PM = P > 0 ? P : LAGP_MAX_DIM;
  const int t = threadIdx.x & 15;
  const double st = L.tps[t];
  const bool et = L.tpe[t] != 0 && t < R;
  double z[PM];
  ray_point<P>(L, a.p, et ? t : 0, st, at_start, z);
  return a.dlen == 1 ? ray_columns_t<P, true>(a, L, j, nq, et, z, kcol)
                     : ray_columns_t<P, false>(a, L, j, nq, et, z, kcol);
}

template <int NP, int NQ>
__device__ __forceinline__ double ray_tile_q(const LocalArgs& a, const Lds& L, int LD, const double* kcol, double kxcol,
                                             int* vflag) {
  const int lane = threadIdx.x & 63;
  double b[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) b[q] = kcol[64 * q + lane];
  return alc_tile_exact_q<NP, NQ, true>(a, L, LD, b, kxcol, vflag);
}

// The objective at every evaluated ray's point, as one tile of the exact
// scoring: lane t < R receives ray t's value (0 if it is not evaluated).
// With `go`: *go = whether any ray is evaluated (the rays live on wave 0),
// and nothing else is done when none is.
template <int NP, int P>
__device__ __forceinline__ double ray_tile(const LocalArgs& a, const Lds& L, int LD, int j, int R, double s, bool ev,
                                           bool at_start, int* vflag, bool* go = nullptr) {
  const int tid = threadIdx.x;
  const int nq = (j + 3) >> 2;
  double* kcol = L.kzb;
  if (tid < 16) {  // ray t's parameter, from lane t of wave 0, for every wave
    L.tps[tid] = s;
    L.tpe[tid] = ev ? 1 : 0;
  }
  if (go && tid < 64) {
    const bool any = __any(ev);
    if (tid == 0) L.ints[10] = any ? 1 : 0;
  }
  __syncthreads();
  if (go) {
    *go = L.ints[10] != 0;
    if (!*go) return 0.0;
  }
  const double kxcol = ray_columns<P>(a, L, j, nq, R, at_start, kcol);
  __syncthreads();
  double out = 0.0;
  if (tid < 64) {
#define LAGP_RAY_CASE(Q) \
  case Q:                \
    if constexpr (Q <= NP / 4) out = ray_tile_q<NP, Q>(a, L, LD, kcol, kxcol, vflag); \
    break;
    switch (nq) { LAGP_CASES_16(LAGP_RAY_CASE) default: break; }
#undef LAGP_RAY_CASE
  }
  __syncthreads();  // kcol and the parameters are rewritten by the next round
  return tid < R && ev ? out : 0.0;
}

// One ray-search step with every ray on one lane of a single wave.
template <int NP, int P>
__device__ __forceinline__ int ray_step_tile(const LocalArgs& a, const Lds& L, int LD, const int32_t* C, const double* Xc,
                                            int j, int n0, double* b1, double* b2, int* vflag) {
  const int lane = threadIdx.x;  // (rays live on the lanes of wave 0)
  const int ns = ray_starts(a, L, j, n0);
  const bool valid = lane < ns;
  const double tau = valid ? ray_segment<P>(a, L, Xc, lane, true) : 0.0;
  __syncthreads();
  const double a0 = ray_tile<NP, P>(a, L, LD, j, ns, 0.0, valid, true, vflag);
  const bool live = valid && tau > 0.0;
  double fb = 0.0;
  int nev = 0;
  const auto eval = [&](double s, bool e, bool* go) { return ray_tile<NP, P>(a, L, LD, j, ns, s, e, false, vflag, go); };
  const double xb = brent_lanes<true>(a, ns, live, eval, &fb, &nev);
  if (valid) {
    L.rev[lane] = nev;
    double sst = 0.0, val = a0;
    if (live) {
      sst = xb;
      val = -fb;
      if (a0 >= val) {
        sst = 0.0;
        val = a0;
      }
    }
    L.rval[lane] = val;
    L.rs[lane] = sst;
  }
  return ray_finish<P>(a, L, C, Xc, j, ns, b1, b2);
}

// ------------------------------------------------------------ kernel -----

// Kernel variants: one instantiation per search / scoring form so each
// carries only its own register footprint.
// MODE_RAY spreads the rays over the workgroup's four waves (any n, up to
// LAGP_MAX_RAYS rays); MODE_RAY_TILE searches them all on one wave of a
// 64-thread workgroup (n <= 64, at most 16 rays).
enum Mode { MODE_EXACT = 0, MODE_MIXED = 1, MODE_RAY = 3, MODE_NN = 4, MODE_RAY_TILE = 5 };

// Register budget per form: the ray form is held to three waves per SIMD
// (its LDS admits three workgroups per CU); the exhaustive forms schedule
// for two and fit three at n <= 64 by themselves (asking the scheduler for
// three there measured slower).
template <int NP, int MODE>
constexpr int local_waves_per_eu() { return MODE == MODE_RAY ? 3 : 2; }

// One wave per location in the tile ray form (its search is one wave's
// work; the per-step phases loop over the workgroup).
constexpr bool local_tile_rays(int n, int R) { return n <= 64 && R >= 1 && R <= 16; }
// Its workgroup: wave 0 holds the rays' Brent recurrences and scores the
// tile; both waves compute the tile's kernel columns.
constexpr int TILE_THREADS = 128;

template <int NP, int MODE, int P>
__global__ __launch_bounds__(LOCAL_THREADS) __attribute__((amdgpu_waves_per_eu(local_waves_per_eu<NP, MODE>())))
void k_local(LocalArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int R = a.search == LAGP_SEARCH_RAY ? a.numrays : 0;
  const LdsPlan plan = plan_lds(a.n, a.ncs, a.p, R, MODE == MODE_MIXED, MODE == MODE_RAY_TILE);
  Lds L = carve(smem, plan);
  const int LD = plan.LD;
  const int tid = threadIdx.x;
  const int m = blockIdx.x;
  static_assert(NP != 256 || MODE == MODE_RAY || MODE == MODE_NN, "designs past 128 points: rays and neighbours");
  if constexpr (NP == 256) L.Ki = a.kig + (int64_t)m * plan.NR * LD;  // (not in LDS)
  const int p = a.p, n = a.n, nc = a.ncand, ncs = a.ncs;
  const int n0 = (a.search == LAGP_SEARCH_NN) ? n : a.n0;
  // a per-location lengthscale (isotropic) replaces the common one; a
  // location without a usable one (a failed earlier stage) is left alone
  const double dl = a.dloc ? a.dloc[m] : 1.0;
  if (!(dl > 0.0)) {
    if (tid == 0) a.status[m] = 0;
    return;
  }
  {  // uniform over the workgroup: held in scalar registers
    const double w0 = a.dloc ? 1.0 / dl : a.w[0];
    const unsigned long long b = (unsigned long long)__double_as_longlong(w0);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
    L.w0 = __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
  }
  const int32_t* C = a.cand + (int64_t)m * nc;
  double* Kc = a.Kc + (int64_t)m * a.kc_rows * ncs;
  float* Kc32 = a.Kc32 ? a.Kc32 + (int64_t)m * a.kc_rows * ncs : nullptr;
  double* kxc = a.kxc + (int64_t)m * ncs;
  double* Li = a.chol + (int64_t)m * 2 * n0 * n0;

  for (int k = tid; k < p; k += blockDim.x) L.x[k] = a.XX[(int64_t)m * p + k];
  for (int t = tid; t < plan.NR * LD; t += blockDim.x) L.Ki[t] = 0.0;
  for (int t = tid; t < plan.NP; t += blockDim.x) {
    L.kx[t] = 0.0; L.h[t] = 0.0; L.col[t] = 0.0; L.wv[t] = 0.0; L.gv[t] = 0.0; L.yJ[t] = 0.0;
  }
  for (int c = tid; c < ncs; c += blockDim.x) L.selm[c] = (c < nc) ? 0 : 1;
  if constexpr (MODE == MODE_RAY)
    for (int t = tid; t < NW * RB * plan.KZS; t += blockDim.x) {
      L.kzb[t] = 0.0;  // zero past j: the ray sums run in zero-padded blocks
      L.wvb[t] = 0.0;
    }
  __syncthreads();

  // kernel vector to x, and the starting rows of the kernel matrix
  // exhaustive search keeps whole kernel rows; otherwise only K_J is needed
  const int kcols = (a.search == LAGP_SEARCH_EXHAUSTIVE) ? ncs : n0;
  double* Xc = a.Xc + (int64_t)m * ncs * p;
  for (int i = tid; i < n0; i += blockDim.x) {
    L.J[i] = i;
    L.jrow[i] = C[i];
    L.selm[i] = 1;
  }
  for (int t = tid; t < n0 * p; t += blockDim.x) L.xj[t] = a.X[(int64_t)C[t / p] * p + (t % p)];
  if (tid == 0) L.ints[4] = 0;
  __syncthreads();
  if (p <= 8)
    gather_candidates<8>(a, L, C, Xc, Kc, Kc32, kxc, n0, kcols);
  else
    gather_candidates<LAGP_MAX_DIM>(a, L, C, Xc, Kc, Kc32, kxc, n0, kcols);
  __syncthreads();
  for (int i = tid; i < n0; i += blockDim.x) L.kx[i] = kxc[i];
  const bool pd = start_inverse(a, L, LD, Kc, Li, n0);

  int vflag = 0;
  int done = n0;  // design size reached
  bool screen = true;  // mixed form: the FP32 screen still rules out candidates
  if (pd) {
    for (int j = n0; j < n; ++j) {
      int cs;
      double b1, b2;
      if constexpr (MODE == MODE_RAY) {
        cs = ray_step<P, NP == 256 ? 4 : 2>(a, L, LD, C, Xc, j, n0, &b1, &b2, &vflag);
      } else if constexpr (MODE == MODE_RAY_TILE) {
        cs = ray_step_tile<NP, P>(a, L, LD, C, Xc, j, n0, &b1, &b2, &vflag);
      } else if constexpr (MODE == MODE_NN) {
        cs = -1;  // (the nearest neighbours fill the design: no step runs)
        b1 = b2 = 0.0;
      } else {
        Best b;
        if constexpr (MODE == MODE_MIXED) {
          b = score_mixed<NP>(a, L, LD, Kc, Kc32, kxc, j, screen, &vflag);
        } else
          b = score_exact<NP>(a, L, LD, Kc, kxc, j, &vflag);
        block_best(L, b);
        cs = L.ints[0];
        b1 = L.scal[1];
        b2 = L.scal[2];
      }
      // no finite score anywhere (or nothing left to snap to): give up on x
      if (cs < 0 || cs > nc || (cs == nc && !a.snap_full)) break;
      const int32_t row = cs < nc ? C[cs] : L.ints[8];
      const double v =
          add_point<MODE == MODE_EXACT || MODE == MODE_MIXED>(a, L, LD, Kc, Kc32, kxc, Xc, j, cs, row);
      done = j + 1;
      if (!(v > 0.0)) vflag = 1;
      if (tid == 0 && a.diag) {
        double* dg = a.diag + ((int64_t)m * (n - a.n0) + (j - n0)) * 2;
        dg[0] = b1;
        dg[1] = b2;
      }
      if (tid == 0 && a.counts) {  // the step's search work (see LocalArgs::counts)
        int32_t* ct = a.counts + ((int64_t)m * (n - a.n0) + (j - n0)) * 2;
        const bool kept = MODE == MODE_RAY || MODE == MODE_RAY_TILE || MODE == MODE_MIXED;
        ct[0] = kept ? L.ints[5] : nc - j;
        ct[1] = kept ? L.ints[6] : 0;
      }
    }
  }

  // prediction with the n local points
  const bool ok = pd && done == n;
  if (ok) {
    for (int i = tid; i < n; i += blockDim.x) L.yJ[i] = a.y[L.jrow[i]];
    __syncthreads();
    for (int i = tid; i < n; i += blockDim.x) {
      double s = 0.0, t = 0.0;
      for (int k = 0; k < n; ++k) {
        const double kik = L.Ki[k * LD + i];  // column i == row i
        s = __builtin_fma(kik, L.kx[k], s);
        t = __builtin_fma(kik, L.yJ[k], t);
      }
      L.h[i] = s;
      L.wv[i] = t;
    }
  }
  if (vflag) L.ints[4] = 1;
  __syncthreads();
  if (tid == 0) {
    double mu = __builtin_nan(""), sc = __builtin_nan("");
    if (ok) {
      mu = 0.0;
      double psi = 0.0, q = 0.0;
      for (int i = 0; i < n; ++i) mu = __builtin_fma(L.h[i], L.yJ[i], mu);
      for (int i = 0; i < n; ++i) psi = __builtin_fma(L.yJ[i], L.wv[i], psi);
      for (int i = 0; i < n; ++i) q = __builtin_fma(L.kx[i], L.h[i], q);
      sc = psi * ((1.0 + a.g) - q) / (double)n;
    }
    int st = 0;
    if (!pd) st |= LAGP_STATUS_NOTPD;
    if (L.ints[4] == 1) st |= LAGP_STATUS_VNONPOS;
    if (!(fabs(mu) <= 1.7976931348623157e308 && fabs(sc) <= 1.7976931348623157e308)) st |= LAGP_STATUS_NONFINITE;
    a.mean[m] = mu;
    a.s2[m] = sc;
    a.df[m] = (double)n;
    a.status[m] = st;
  }
  if (a.sel)
    for (int i = tid; i < n; i += blockDim.x) a.sel[(int64_t)m * n + i] = (i < done) ? L.jrow[i] : -1;
}

size_t local_lds_bytes(int n, int ncs, int p, int numrays, bool mixed) {
  return plan_lds(n, ncs, p, numrays, mixed).bytes;
}

// Test hook: LAGP_RAY_FORCE_WAVES=1 keeps every ray search on the four-wave form.
static bool ray_force_waves() {
  const char* s = std::getenv("LAGP_RAY_FORCE_WAVES");
  return s && s[0] == '1';
}

template <int NP, int MODE, int P = 0>
static hipError_t launch_mode(const LocalArgs& a, size_t lds, hipStream_t s, int threads = LOCAL_THREADS) {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_local<NP, MODE, P>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_local<NP, MODE, P>), dim3(a.M), dim3(threads), lds, s, a);
  return hipGetLastError();
}

// The scoring width NP matters to the exhaustive forms only; ray and
// nearest-neighbour kernels are instantiated once (their LDS plan is sized at
// run time either way).
template <int NP>
static hipError_t launch_exhaustive(const LocalArgs& a, size_t lds, hipStream_t s) {
  if (a.precision == LAGP_PREC_MIXED) return launch_mode<NP, MODE_MIXED>(a, lds, s);
  return launch_mode<NP, MODE_EXACT>(a, lds, s);
}

hipError_t launch_local(const LocalArgs& a, hipStream_t s) {
  if (a.M <= 0) return hipSuccess;
  const int R = a.search == LAGP_SEARCH_RAY ? a.numrays : 0;
  const size_t lds = local_lds_bytes(a.n, a.ncs, a.p, R, a.precision == LAGP_PREC_MIXED);
  if (a.search == LAGP_SEARCH_RAY && local_tile_rays(a.n, a.numrays) && !ray_force_waves()) {
    const size_t lt = plan_lds(a.n, a.ncs, a.p, R, false, true).bytes;
    switch (a.p) {
      case 1: return launch_mode<64, MODE_RAY_TILE, 1>(a, lt, s, TILE_THREADS);
      case 2: return launch_mode<64, MODE_RAY_TILE, 2>(a, lt, s, TILE_THREADS);
      case 3: return launch_mode<64, MODE_RAY_TILE, 3>(a, lt, s, TILE_THREADS);
      case 4: return launch_mode<64, MODE_RAY_TILE, 4>(a, lt, s, TILE_THREADS);
      case 8: return launch_mode<64, MODE_RAY_TILE, 8>(a, lt, s, TILE_THREADS);
      default: return launch_mode<64, MODE_RAY_TILE, 0>(a, lt, s, TILE_THREADS);
    }
  }
  if (a.search == LAGP_SEARCH_RAY && a.n > 128) {  // K^{-1} in the workspace
    switch (a.p) {
      case 2: return launch_mode<256, MODE_RAY, 2>(a, lds, s);
      default: return launch_mode<256, MODE_RAY, 0>(a, lds, s);
    }
  }
  if (a.search == LAGP_SEARCH_RAY) {
    switch (a.p) {
      case 1: return launch_mode<64, MODE_RAY, 1>(a, lds, s);
      case 2: return launch_mode<64, MODE_RAY, 2>(a, lds, s);
      case 3: return launch_mode<64, MODE_RAY, 3>(a, lds, s);
      case 4: return launch_mode<64, MODE_RAY, 4>(a, lds, s);
      case 8: return launch_mode<64, MODE_RAY, 8>(a, lds, s);
      default: return launch_mode<64, MODE_RAY, 0>(a, lds, s);
    }
  }
  if (a.search == LAGP_SEARCH_NN) return a.n > 128 ? launch_mode<256, MODE_NN>(a, lds, s) : launch_mode<64, MODE_NN>(a, lds, s);
  return a.n <= 64 ? launch_exhaustive<64>(a, lds, s) : launch_exhaustive<128>(a, lds, s);
}

}  // namespace lagp
