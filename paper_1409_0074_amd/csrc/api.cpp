// Host side of the C ABI: argument checks, device workspace, launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "lagp_internal.h"

namespace {

thread_local std::string g_err;

int32_t fail(int32_t code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define LAGP_HIP(call)                                                                             \
  do {                                                                                             \
    hipError_t e_ = (call);                                                                        \
    if (e_ != hipSuccess) return fail(LAGP_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

size_t workspace_budget() {
  const char* s = std::getenv("LAGP_WORKSPACE_MB");
  if (s) {
    const long mb = std::atol(s);
    if (mb > 0) return (size_t)mb << 20;
  }
  return (size_t)16 << 30;  // a small share of the 288 GB of HBM
}

int max_lds_per_block() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 65536;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 65536;
  return v;
}

// Largest round-robin offset k = t mod floor(sqrt t) over t = 1..steps (Sec. 4).
int max_ray_offset(int steps) {
  int best = 0;
  for (int t = 1; t <= steps; ++t) {
    int r = 0;
    while ((r + 1) * (r + 1) <= t) ++r;
    best = std::max(best, r > 0 ? t % r : 0);
  }
  return best;
}

int32_t check_params(const lagp_design* d, const lagp_params* P, int* rays) {
  if (!P) return fail(LAGP_EINVAL, "params is NULL");
  const int p = d->p;
  if (P->search < LAGP_SEARCH_EXHAUSTIVE || P->search > LAGP_SEARCH_NN)
    return fail(LAGP_EINVAL, "search must be LAGP_SEARCH_EXHAUSTIVE, _RAY or _NN");
  if (P->precision != LAGP_PREC_FP64 && P->precision != LAGP_PREC_MIXED)
    return fail(LAGP_EINVAL, "precision must be LAGP_PREC_FP64 or LAGP_PREC_MIXED");
  if (P->precision == LAGP_PREC_MIXED && P->search != LAGP_SEARCH_EXHAUSTIVE)
    return fail(LAGP_EINVAL, "the mixed precision form applies to exhaustive search only");
  if (P->precision == LAGP_PREC_MIXED && (P->rescore_k < 1 || P->rescore_k > 64))
    return fail(LAGP_EINVAL, "rescore_k must be in [1, 64]");
  if (P->scoring != LAGP_SCORING_PARTINV && P->scoring != LAGP_SCORING_CHOL)
    return fail(LAGP_EINVAL, "scoring must be LAGP_SCORING_PARTINV or LAGP_SCORING_CHOL");
  if (P->scoring == LAGP_SCORING_CHOL &&
      (P->search != LAGP_SEARCH_EXHAUSTIVE || P->precision != LAGP_PREC_FP64))
    return fail(LAGP_EINVAL, "Cholesky scoring applies to exhaustive search in FP64 only");
  if (P->n < 1 || P->n > LAGP_MAX_N) return fail(LAGP_EINVAL, "n must be in [1, LAGP_MAX_N]");
  if (P->n > 128 && P->search == LAGP_SEARCH_EXHAUSTIVE && P->scoring != LAGP_SCORING_CHOL)
    return fail(LAGP_EINVAL, "designs past 128 points: exhaustive search by Cholesky columns, rays or neighbours");
  if (P->search != LAGP_SEARCH_NN && (P->n0 < 1 || P->n0 > P->n)) return fail(LAGP_EINVAL, "n0 must be in [1, n]");
  if (P->ncand < P->n) return fail(LAGP_EINVAL, "ncand must be >= n");
  if ((int64_t)P->ncand > d->N) return fail(LAGP_EINVAL, "ncand must be <= N");
  if (P->ncand > LAGP_MAX_NCAND) return fail(LAGP_EINVAL, "ncand must be <= LAGP_MAX_NCAND");
  if (!(P->d_len == 1 || P->d_len == p)) return fail(LAGP_EINVAL, "d_len must be 1 or p");
  for (int k = 0; k < P->d_len; ++k)
    if (!(P->d[k] > 0.0) || !std::isfinite(P->d[k])) return fail(LAGP_EINVAL, "lengthscales must be finite and > 0");
  if (!(P->g >= 0.0) || !std::isfinite(P->g)) return fail(LAGP_EINVAL, "nugget g must be finite and >= 0");
  if (P->snap != LAGP_SNAP_CANDIDATES && P->snap != LAGP_SNAP_DESIGN)
    return fail(LAGP_EINVAL, "snap must be LAGP_SNAP_CANDIDATES or LAGP_SNAP_DESIGN");
  if (P->snap == LAGP_SNAP_DESIGN && P->search != LAGP_SEARCH_RAY)
    return fail(LAGP_EINVAL, "snap over the whole design applies to ray search only");
  *rays = 0;
  if (P->search == LAGP_SEARCH_RAY) {
    const int R = P->numrays > 0 ? P->numrays : p;
    if (R > LAGP_MAX_RAYS) return fail(LAGP_EINVAL, "numrays must be <= LAGP_MAX_RAYS");
    // at step j the starts are remaining ranks k0 .. k0+R-1 with j taken
    const int need = (P->n - 1) + R + max_ray_offset(P->n - P->n0);
    if (P->ncand < need)
      return fail(LAGP_EINVAL, "ncand too small for the ray starts: need n - 1 + numrays + max round-robin offset = " +
                                   std::to_string(need));
    if (P->brent_tol < 0.0 || !std::isfinite(P->brent_tol)) return fail(LAGP_EINVAL, "brent_tol must be finite");
    *rays = R;
  }
  return LAGP_OK;
}

bool force_knn_fallback() {
  const char* s = std::getenv("LAGP_KNN_FORCE_FALLBACK");
  return s && s[0] == '1';
}

// Threshold-first kNN arguments over a workspace laid out as
// [tau: chunk doubles][cnt: chunk ints][d2: chunk*CAP doubles][row: chunk*CAP ints].
// ws: per-location buffers for `chunk` locations; sub: the per-call
// subsample block (knn2_shared_bytes).
lagp::Knn2Args knn_args(const lagp_design* d, const double* XX, int32_t M, int ncand, void* ws, int64_t chunk,
                        void* sub, int32_t* out_idx, double* out_d2) {
  lagp::Knn2Args k{};
  k.sub = reinterpret_cast<double*>(sub);
  const size_t cap = (lagp::knn2_bytes_per_location(ncand) - sizeof(double) - sizeof(int32_t)) /
                     (sizeof(double) + sizeof(int32_t));
  char* b = reinterpret_cast<char*>(ws);
  k.tau = reinterpret_cast<double*>(b);
  k.cnt = reinterpret_cast<int32_t*>(b + sizeof(double) * chunk);
  const size_t o_d2 = ((sizeof(double) + sizeof(int32_t)) * chunk + 255) & ~size_t(255);
  k.buf_d2 = reinterpret_cast<double*>(b + o_d2);
  k.buf_idx = reinterpret_cast<int32_t*>(b + o_d2 + sizeof(double) * cap * chunk);
  k.X = d->X;
  k.rn = d->rn;
  k.X32 = d->X32;
  k.rn_max = d->rn_max;
  k.spread2 = d->spread2;
  k.XX = XX;
  k.out_idx = out_idx;
  k.out_d2 = out_d2;
  k.N = d->N;
  k.M = M;
  k.p = d->p;
  k.ncand = ncand;
  k.force_fallback = force_knn_fallback() ? 1 : 0;
  return k;
}

struct Workspace {
  void* ptr = nullptr;
  hipStream_t s = nullptr;
  ~Workspace() {
    if (ptr) (void)hipFreeAsync(ptr, s);
  }
};

}  // namespace

extern "C" {

int32_t lagp_version(void) { return 10000; }

const char* lagp_last_error(void) { return g_err.c_str(); }

int32_t lagp_design_create(const double* X, const double* y, int64_t N, int32_t p, void* stream,
                           lagp_design** out) {
  if (!out) return fail(LAGP_EINVAL, "out is NULL");
  *out = nullptr;
  if (!X || !y) return fail(LAGP_EINVAL, "X and y must not be NULL");
  if (N < 1 || N > INT32_MAX) return fail(LAGP_EINVAL, "N must be in [1, 2^31-1]");
  if (p < 1 || p > LAGP_MAX_DIM) return fail(LAGP_EINVAL, "p must be in [1, LAGP_MAX_DIM]");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  lagp_design* d = new (std::nothrow) lagp_design();
  if (!d) return fail(LAGP_ENOMEM, "host allocation failed");
  d->N = N;
  d->p = p;
  if (hipGetDevice(&d->device) != hipSuccess) {
    delete d;
    return fail(LAGP_EDEVICE, "hipGetDevice failed");
  }
  const size_t xb = sizeof(double) * (size_t)N * p, yb = sizeof(double) * (size_t)N;
  double* rmax = nullptr;
  if (hipMalloc(&d->X, xb) != hipSuccess || hipMalloc(&d->y, yb) != hipSuccess ||
      hipMalloc(&d->lo, sizeof(double) * p) != hipSuccess || hipMalloc(&d->hi, sizeof(double) * p) != hipSuccess ||
      hipMalloc(&d->rn, yb) != hipSuccess || hipMalloc(&d->X32, sizeof(float) * (size_t)N * p) != hipSuccess ||
      hipMalloc(&rmax, sizeof(double)) != hipSuccess) {
    if (rmax) (void)hipFree(rmax);
    lagp_design_destroy(d);
    return fail(LAGP_ENOMEM, "device allocation of the design failed");
  }
  hipError_t e = hipMemcpyAsync(d->X, X, xb, hipMemcpyDefault, s);
  if (e == hipSuccess) e = hipMemcpyAsync(d->y, y, yb, hipMemcpyDefault, s);
  if (e == hipSuccess) e = lagp::launch_bbox(d->X, N, p, d->lo, d->hi, s);
  if (e == hipSuccess) e = lagp::launch_row_norms(d->X, N, p, d->rn, rmax, d->X32, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&d->rn_max, rmax, sizeof(double), hipMemcpyDeviceToHost, s);
  double* lo = d->lo_h;
  double* hi = d->hi_h;
  if (e == hipSuccess) e = hipMemcpyAsync(lo, d->lo, sizeof(double) * p, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(hi, d->hi, sizeof(double) * p, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  d->spread2 = 0.0;
  if (e == hipSuccess)
    for (int k = 0; k < p; ++k) d->spread2 += (hi[k] - lo[k]) * (hi[k] - lo[k]);
  (void)hipFree(rmax);
  if (e != hipSuccess) {
    lagp_design_destroy(d);
    return fail(LAGP_EDEVICE, std::string("design upload: ") + hipGetErrorString(e));
  }
  *out = d;
  return LAGP_OK;
}

void lagp_design_destroy(lagp_design* d) {
  if (!d) return;
  (void)hipDeviceSynchronize();
  if (d->X) (void)hipFree(d->X);
  if (d->y) (void)hipFree(d->y);
  if (d->lo) (void)hipFree(d->lo);
  if (d->hi) (void)hipFree(d->hi);
  if (d->rn) (void)hipFree(d->rn);
  if (d->X32) (void)hipFree(d->X32);
  if (d->grid_Xs) (void)hipFree(d->grid_Xs);
  if (d->grid_rows) (void)hipFree(d->grid_rows);
  if (d->grid_start) (void)hipFree(d->grid_start);
  delete d;
}

int32_t lagp_design_build_grid(const lagp_design* dc, void* stream) {
  if (!dc) return fail(LAGP_EINVAL, "design is NULL");
  lagp_design* d = const_cast<lagp_design*>(dc);  // the grid is a cache: the design itself is unchanged
  std::lock_guard<std::mutex> lk(d->grid_mu);
  if (d->grid_built) return LAGP_OK;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  lagp::GridDev g = lagp::grid_plan(d->N, d->p, d->lo_h, d->hi_h);
  const int64_t cells = lagp::grid_cells(g);
  int32_t *cid = nullptr, *cnt = nullptr;
  auto release = [&]() {
    if (cid) (void)hipFree(cid);
    if (cnt) (void)hipFree(cnt);
  };
  if (hipMalloc(&d->grid_Xs, sizeof(double) * (size_t)d->N * d->p) != hipSuccess ||
      hipMalloc(&d->grid_rows, sizeof(int32_t) * (size_t)d->N) != hipSuccess ||
      hipMalloc(&d->grid_start, sizeof(int32_t) * (size_t)(cells + 1)) != hipSuccess ||
      hipMalloc(&cid, sizeof(int32_t) * (size_t)d->N) != hipSuccess ||
      hipMalloc(&cnt, sizeof(int32_t) * (size_t)cells) != hipSuccess) {
    release();
    return fail(LAGP_ENOMEM, "device allocation of the design grid failed");
  }
  hipError_t e = lagp::launch_grid_build(d->X, d->N, d->p, g, cid, cnt, d->grid_start, d->grid_Xs, d->grid_rows, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  release();
  if (e != hipSuccess) return fail(LAGP_EDEVICE, std::string("design grid: ") + hipGetErrorString(e));
  d->grid = g;
  d->grid_built = true;
  return LAGP_OK;
}

int32_t lagp_design_info(const lagp_design* d, int64_t* N, int32_t* p) {
  if (!d) return fail(LAGP_EINVAL, "design is NULL");
  if (N) *N = d->N;
  if (p) *p = d->p;
  return LAGP_OK;
}

int32_t lagp_candidates(const lagp_design* d, const double* XX, int64_t M, int32_t ncand, int32_t* cand_idx,
                        double* cand_d2, void* stream) {
  if (!d) return fail(LAGP_EINVAL, "design is NULL");
  if (M < 0) return fail(LAGP_EINVAL, "M must be >= 0");
  if (M == 0) return LAGP_OK;
  if (!XX || !cand_idx) return fail(LAGP_EINVAL, "XX and cand_idx must not be NULL");
  if (ncand < 1 || (int64_t)ncand > d->N || ncand > LAGP_MAX_NCAND)
    return fail(LAGP_EINVAL, "ncand must be in [1, min(N, LAGP_MAX_NCAND)]");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int S = lagp::knn_sort_size(ncand);
  if (lagp::knn2_merge_lds_bytes(S) > (size_t)max_lds_per_block()) return fail(LAGP_EINVAL, "ncand too large for LDS");
  const size_t per = lagp::knn2_bytes_per_location(ncand);
  const size_t shared = lagp::knn2_shared_bytes(d->N, d->p, ncand);
  int64_t chunk = std::max<int64_t>(64, (int64_t)(workspace_budget() / per));
  chunk = std::min<int64_t>(chunk, M);
  const size_t o_sub = (per * chunk + 1024 + 255) & ~size_t(255);
  Workspace ws;
  ws.s = s;
  LAGP_HIP(hipMallocAsync(&ws.ptr, o_sub + shared, s));
  char* base = reinterpret_cast<char*>(ws.ptr);
  for (int64_t m0 = 0; m0 < M; m0 += chunk) {
    const int32_t mc = (int32_t)std::min<int64_t>(chunk, M - m0);
    LAGP_HIP(lagp::launch_knn2(knn_args(d, XX + m0 * d->p, mc, ncand, base, chunk, base + o_sub,
                                        cand_idx + m0 * ncand, cand_d2 ? cand_d2 + m0 * ncand : nullptr),
                               s));
  }
  return LAGP_OK;
}

}  // extern "C"

namespace lagp {

// The search arguments every entry point shares: design, locations,
// candidates and the method's parameters (workspace and outputs are the
// caller's to fill in).
lagp::LocalArgs local_args(const lagp_design* d, const lagp_params* P, int rays, const double* XX, int32_t M,
                           const int32_t* cand) {
  lagp::LocalArgs a{};
  a.X = d->X;
  a.y = d->y;
  a.lo = d->lo;
  a.hi = d->hi;
  a.XX = XX;
  a.cand = cand;
  a.N = d->N;
  a.M = M;
  a.p = d->p;
  a.n = P->n;
  a.n0 = P->search == LAGP_SEARCH_NN ? P->n : P->n0;
  a.ncand = P->ncand;
  a.ncs = (P->ncand + 15) & ~15;
  a.kc_rows = P->search == LAGP_SEARCH_EXHAUSTIVE ? (P->n + 3) / 4 * 4 : a.n0;  // exact tiles read whole chunks
  a.numrays = rays;
  a.search = P->search;
  a.precision = P->precision;
  a.rescore_k = P->rescore_k;
  a.dlen = P->d_len;
  a.brent_maxit = P->brent_maxit > 0 ? P->brent_maxit : 100;
  a.brent_tol = P->brent_tol > 0.0 ? P->brent_tol : std::ldexp(1.0, -13);
  a.g = P->g;
  for (int q = 0; q < P->d_len; ++q) a.w[q] = 1.0 / P->d[q];
  if (P->snap == LAGP_SNAP_DESIGN) {  // (the grid is built: ensure_grid)
    a.snap_full = 1;
    a.grid = d->grid;
  }
  return a;
}

// A ray search that snaps over the whole design needs the design's cell
// grid: built here on first use, unless the caller must not allocate.
int32_t ensure_grid(const lagp_design* d, const lagp_params* P, void* stream, bool may_build) {
  if (P->snap != LAGP_SNAP_DESIGN) return LAGP_OK;
  {
    std::lock_guard<std::mutex> lk(const_cast<lagp_design*>(d)->grid_mu);
    if (d->grid_built) return LAGP_OK;
  }
  if (!may_build)
    return fail(LAGP_EINVAL, "snap over the whole design needs the design grid: build it first (lagp_design_build_grid)");
  return lagp_design_build_grid(d, stream);
}

// Cholesky scoring: the on-chip kernel where the columns fit in registers and
// LDS, else the streaming kernel, whose workspace is a fixed number of slots
// (one per resident workgroup of its persistent grid, at most half the
// budget) rather than a per-location size.  Returns the slots' bytes.
bool chol_onchip(const lagp_design* d, const lagp_params* P) {
  return chol_supported(P->n, P->ncand, d->p, (size_t)max_lds_per_block()) && !chol_stream_forced();
}

bool chol_onchip_shape(const lagp_design* d, int n, int ncand) {
  return chol_supported(n, ncand, d->p, (size_t)max_lds_per_block()) && !chol_stream_forced();
}

size_t chol_stream_fixed(const lagp_design* d, const lagp_params* P, size_t budget, int* slots) {
  *slots = 0;
  if (P->scoring != LAGP_SCORING_CHOL || chol_onchip(d, P)) return 0;
  const size_t sb = chol_stream_slot_bytes(P->n, P->ncand, d->p);
  const int64_t k = std::min<int64_t>(chol_stream_max_slots(P->ncand), std::max<int64_t>(1, (int64_t)(budget / 2 / sb)));
  *slots = (int)k;
  return (sb * (size_t)k + 255) & ~size_t(255);
}

// K_J^{-1} of a design past 128 points (ray and neighbour searches), which
// does not fit LDS: ceil8(n) rows of 257 doubles per location (the local
// kernel's plan for n > 128).
size_t kig_bytes(const lagp_params* P) {
  if (P->n <= 128 || P->scoring == LAGP_SCORING_CHOL) return 0;
  return sizeof(double) * (size_t)((P->n + 7) & ~7) * 257;
}

// Bytes run_predict allocates for M locations under a workspace cap, and the
// per-location figure (kNN buffers when candidates are not given, the kernel
// rows, k(x_c, x), the candidates' coordinates, the starting-inverse scratch
// and a status word).
size_t predict_per_location_bytes(const lagp_design* d, const lagp_params* P, bool have_cand) {
  const int n = P->n, nc = P->ncand;
  if (P->scoring == LAGP_SCORING_CHOL)  // the search state stays on chip
    return (have_cand ? 0 : knn2_bytes_per_location(nc) + 1024 + sizeof(int32_t) * (size_t)nc) + sizeof(int32_t);
  const int n0 = P->search == LAGP_SEARCH_NN ? n : P->n0;
  const int ncs = (nc + 15) & ~15;
  const int kc_rows = P->search == LAGP_SEARCH_EXHAUSTIVE ? (n + 3) / 4 * 4 : n0;  // exact tiles read whole chunks
  const size_t b_knn = have_cand ? 0 : knn2_bytes_per_location(nc) + 1024;
  const size_t b_cand = have_cand ? 0 : sizeof(int32_t) * (size_t)nc;
  const size_t b_kc32 = P->precision == LAGP_PREC_MIXED ? sizeof(float) * (size_t)kc_rows * ncs : 0;
  return b_knn + b_cand + sizeof(double) * (size_t)kc_rows * ncs + b_kc32 + sizeof(double) * (size_t)ncs +
         sizeof(double) * (size_t)ncs * d->p + sizeof(double) * 2 * (size_t)n0 * n0 + kig_bytes(P) +
         sizeof(int32_t);
}

int64_t predict_chunk(const lagp_design* d, const lagp_params* P, bool have_cand, int64_t M, size_t ws_budget) {
  const size_t per = predict_per_location_bytes(d, P, have_cand);
  int64_t chunk = std::max<int64_t>(KNN_QB, (int64_t)(ws_budget / per));
  return std::min<int64_t>(chunk, M);
}

size_t predict_workspace_bytes(const lagp_design* d, const lagp_params* P, bool have_cand, int64_t M,
                               size_t ws_budget) {
  if (M <= 0) return 0;
  const size_t shared = have_cand ? 0 : knn2_shared_bytes(d->N, d->p, P->ncand);
  int slots = 0;
  const size_t fixed = chol_stream_fixed(d, P, ws_budget, &slots);
  return predict_per_location_bytes(d, P, have_cand) *
             (size_t)predict_chunk(d, P, have_cand, M, ws_budget > fixed ? ws_budget - fixed : 0) +
         shared + fixed + 11 * 256;  // 11 aligned sections
}

int32_t run_predict(const lagp_design* d, const double* XX, int64_t M, const int32_t* cand_in,
                    const lagp_params* P, double* mean, double* s2, double* df, int32_t* sel_idx, double* diag,
                    int32_t* status, void* stream, size_t ws_budget, void* ext_ws, size_t ext_bytes,
                    int32_t* counts, const PerLocation* pl) {
  if (!d) return fail(LAGP_EINVAL, "design is NULL");
  if (M < 0) return fail(LAGP_EINVAL, "M must be >= 0");
  int rays = 0;
  int32_t rc = check_params(d, P, &rays);
  if (rc != LAGP_OK) return rc;
  if (M == 0) return LAGP_OK;
  if (!XX || !mean || !s2 || !df) return fail(LAGP_EINVAL, "XX, mean, s2 and df must not be NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int p = d->p, n = P->n, nc = P->ncand;
  const int n0 = P->search == LAGP_SEARCH_NN ? n : P->n0;
  const int ncs = (nc + 15) & ~15;
  const int S = lagp::knn_sort_size(nc);
  const int lds_max = max_lds_per_block();
  if (!cand_in && knn2_merge_lds_bytes(S) > (size_t)lds_max) return fail(LAGP_EINVAL, "ncand too large for LDS");
  const bool chol = P->scoring == LAGP_SCORING_CHOL;
  if ((rc = ensure_grid(d, P, stream, ext_ws == nullptr)) != LAGP_OK) return rc;
  if (!chol && lagp::local_lds_bytes(n, ncs, p, rays, P->precision == LAGP_PREC_MIXED) > (size_t)lds_max)
    return fail(LAGP_EINVAL, "local design too large for LDS (n, p, numrays)");
  const int kc_rows = P->search == LAGP_SEARCH_EXHAUSTIVE ? (n + 3) / 4 * 4 : n0;  // exact tiles read whole chunks
  // per-location workspace: kNN buffers and candidate list (unless given),
  // kernel rows, k(x_c, x), candidate coordinates, starting-inverse scratch,
  // status
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t b_knn = cand_in ? 0 : knn2_bytes_per_location(nc) + 1024;
  const size_t b_cand = cand_in ? 0 : sizeof(int32_t) * (size_t)nc;
  // (the Cholesky form keeps its search state on chip)
  const size_t b_kc = chol ? 0 : sizeof(double) * (size_t)kc_rows * ncs;
  const size_t b_kc32 = P->precision == LAGP_PREC_MIXED ? sizeof(float) * (size_t)kc_rows * ncs : 0;
  const size_t b_kxc = chol ? 0 : sizeof(double) * (size_t)ncs;
  const size_t b_xc = chol ? 0 : sizeof(double) * (size_t)ncs * p;
  const size_t b_chol = chol ? 0 : sizeof(double) * 2 * (size_t)n0 * n0;
  const size_t b_kig = kig_bytes(P);
  const size_t shared = cand_in ? 0 : knn2_shared_bytes(d->N, p, nc);
  int cw_slots = 0;
  const size_t b_cw = chol_stream_fixed(d, P, ext_ws ? ext_bytes : ws_budget, &cw_slots);
  if (pl && !(chol && cw_slots == 0 && chol_onchip(d, P)))
    return fail(LAGP_EINVAL, "internal: per-location parameters need the on-chip Cholesky form");
  int64_t chunk = predict_chunk(d, P, cand_in != nullptr, M, ws_budget > b_cw ? ws_budget - b_cw : 0);
  if (ext_ws) {  // as many locations as the given workspace holds (11 sections, each aligned)
    const size_t per = b_knn + b_cand + b_kc + b_kc32 + b_kxc + b_xc + b_chol + b_kig + sizeof(int32_t);
    const size_t fixed = shared + b_cw + 11 * 256;
    if (ext_bytes < fixed + per)
      return fail(LAGP_ENOMEM, "the workspace of one location (" + std::to_string(fixed + per) +
                                   " bytes) exceeds the " + std::to_string(ext_bytes) + "-byte scratch");
    chunk = std::min<int64_t>(M, (int64_t)((ext_bytes - fixed) / per));
  }
  Workspace ws;
  ws.s = s;
  const size_t o_knn = 0, o_cand = o_knn + al(b_knn * chunk), o_kc = o_cand + al(b_cand * chunk),
               o_kc32 = o_kc + al(b_kc * chunk), o_kxc = o_kc32 + al(b_kc32 * chunk),
               o_xc = o_kxc + al(b_kxc * chunk), o_chol = o_xc + al(b_xc * chunk),
               o_kig = o_chol + al(b_chol * chunk), o_st = o_kig + al(b_kig * chunk),
               o_sub = o_st + al(sizeof(int32_t) * chunk),
               o_cw = o_sub + al(shared), total = o_cw + b_cw;
  char* base = nullptr;
  if (ext_ws) {
    if (total > ext_bytes) return fail(LAGP_ENOMEM, "internal: workspace layout exceeds the scratch");
    base = reinterpret_cast<char*>(ext_ws);
  } else {
    LAGP_HIP(hipMallocAsync(&ws.ptr, total, s));
    base = reinterpret_cast<char*>(ws.ptr);
  }
  for (int64_t m0 = 0; m0 < M; m0 += chunk) {
    const int32_t mc = (int32_t)std::min<int64_t>(chunk, M - m0);
    const int32_t* cand = cand_in ? cand_in + m0 * nc : reinterpret_cast<const int32_t*>(base + o_cand);
    if (!cand_in)
      LAGP_HIP(launch_knn2(knn_args(d, XX + m0 * p, mc, nc, base + o_knn, chunk, base + o_sub,
                                    reinterpret_cast<int32_t*>(base + o_cand), nullptr),
                           s));
    lagp::LocalArgs a = local_args(d, P, rays, XX + m0 * p, mc, cand);
    a.Kc = reinterpret_cast<double*>(base + o_kc);
    a.Kc32 = b_kc32 ? reinterpret_cast<float*>(base + o_kc32) : nullptr;
    a.kxc = reinterpret_cast<double*>(base + o_kxc);
    a.Xc = reinterpret_cast<double*>(base + o_xc);
    a.chol = reinterpret_cast<double*>(base + o_chol);
    a.kig = b_kig ? reinterpret_cast<double*>(base + o_kig) : nullptr;
    a.cw = reinterpret_cast<double*>(base + o_cw);
    if (pl) {
      a.nloc = pl->n + m0;
      a.dloc = pl->d + m0;
      a.gloc = pl->g + m0;
    }
    a.mean = mean + m0;
    a.s2 = s2 + m0;
    a.df = df + m0;
    a.sel = sel_idx ? sel_idx + m0 * n : nullptr;
    a.diag = diag ? diag + m0 * (int64_t)(n - n0) * 2 : nullptr;
    a.counts = counts ? counts + m0 * (int64_t)(n - n0) * 2 : nullptr;
    a.status = status ? status + m0 : reinterpret_cast<int32_t*>(base + o_st);
    LAGP_HIP(!chol ? lagp::launch_local(a, s)
                   : cw_slots ? lagp::launch_chol_stream(a, cw_slots, s) : lagp::launch_chol(a, s));
  }
  return LAGP_OK;
}

int32_t check_predict_params(const lagp_design* d, const lagp_params* P) {
  int rays = 0;
  return check_params(d, P, &rays);
}

const char* set_error(const char* msg) {
  g_err = msg;
  return g_err.c_str();
}

}  // namespace lagp

extern "C" {

int32_t lagp_predict(const lagp_design* d, const double* XX, int64_t M, const lagp_params* P, double* mean,
                     double* s2, double* df, int32_t* sel_idx, double* diag, int32_t* status, void* stream) {
  return lagp::run_predict(d, XX, M, nullptr, P, mean, s2, df, sel_idx, diag, status, stream, workspace_budget());
}

int32_t lagp_predict_candidates(const lagp_design* d, const double* XX, int64_t M, const int32_t* cand_idx,
                                const lagp_params* P, double* mean, double* s2, double* df, int32_t* sel_idx,
                                double* diag, int32_t* status, void* stream) {
  if (M > 0 && !cand_idx) return fail(LAGP_EINVAL, "cand_idx must not be NULL");
  return lagp::run_predict(d, XX, M, cand_idx, P, mean, s2, df, sel_idx, diag, status, stream, workspace_budget());
}

int32_t lagp_predict_counts(const lagp_design* d, const double* XX, int64_t M, const int32_t* cand_idx,
                            const lagp_params* P, double* mean, double* s2, double* df, int32_t* sel_idx,
                            double* diag, int32_t* status, int32_t* counts, void* stream) {
  return lagp::run_predict(d, XX, M, cand_idx, P, mean, s2, df, sel_idx, diag, status, stream, workspace_budget(),
                           nullptr, 0, counts);
}

// ---- the entry point that allocates nothing --------------------------------
//
// Its workspace is this file-scope device array.  In host code the name
// `scratch` is only a host-side stand-in: the array's device address comes
// from hipGetSymbolAddress, taken once per device (with that device current)
// and kept; kernels and copies get that address, never the name.
static __device__ __align__(256) unsigned char scratch[LAGP_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};

// Device address of this device's copy of `scratch` (set up on first use).
int32_t scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return fail(LAGP_EDEVICE, "device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(LAGP_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return LAGP_OK;
}

}  // namespace

int32_t lagp_predict_noalloc(const lagp_design* d, const double* XX, int64_t M, const lagp_params* P, double* mean,
                             double* s2, double* df, int32_t* sel_idx, double* diag, int32_t* status, void* stream) {
  if (!d) return fail(LAGP_EINVAL, "design is NULL");
  int dev = -1;
  LAGP_HIP(hipGetDevice(&dev));
  if (dev != d->device) return fail(LAGP_EINVAL, "the current device is not the design's device");
  int32_t rc = lagp::check_predict_params(d, P);
  if (rc != LAGP_OK) return rc;
  if (M <= 0) return M < 0 ? fail(LAGP_EINVAL, "M must be >= 0") : LAGP_OK;
  void* ws = nullptr;
  rc = scratch_address(dev, &ws);
  if (rc != LAGP_OK) return rc;
  return lagp::run_predict(d, XX, M, nullptr, P, mean, s2, df, sel_idx, diag, status, stream, 0, ws,
                           (size_t)LAGP_NOALLOC_SCRATCH_BYTES);
}

// Local MLE (mle.hip) around a design search (the Cholesky form of
// chol.hip, or local.hip's exhaustive, ray or nearest-neighbour search):
// search under d0, estimate, [search under the estimate, estimate again],
// predict.
int32_t lagp_predict_mle(const lagp_design* d, const double* XX, int64_t M, const int32_t* cand_in,
                         const lagp_params* P, const lagp_mle_params* mle, double* mean, double* s2, double* df,
                         double* dhat, int32_t* sel_idx, int32_t* iters, int32_t* status, void* stream) {
  if (!d) return fail(LAGP_EINVAL, "design is NULL");
  if (M < 0) return fail(LAGP_EINVAL, "M must be >= 0");
  int rays = 0;
  int32_t rc = check_params(d, P, &rays);
  if (rc != LAGP_OK) return rc;
  if (!mle) return fail(LAGP_EINVAL, "mle is NULL");
  if (mle->mode != 1 && mle->mode != 2) return fail(LAGP_EINVAL, "mle->mode must be 1 or 2");
  if (P->precision != LAGP_PREC_FP64) return fail(LAGP_EINVAL, "local MLE runs in FP64 only");
  if (P->d_len != 1) return fail(LAGP_EINVAL, "local MLE estimates one isotropic lengthscale: d_len must be 1");
  if (M > 0 && (rc = lagp::ensure_grid(d, P, stream, true)) != LAGP_OK) return rc;
  const int p = d->p, n = P->n, nc = P->ncand;
  const bool chol = P->scoring == LAGP_SCORING_CHOL;  // else k_local's search (any mode)
  const double d0 = P->d[0];
  const double dmin = mle->dmin > 0.0 ? mle->dmin : d0 / 1000.0;
  const double dmax = mle->dmax > 0.0 ? mle->dmax : 100.0 * d0;
  const double tol = mle->tol > 0.0 ? mle->tol : 1e-8;
  const int maxit = mle->maxit > 0 ? mle->maxit : 100;
  if (!(dmin < dmax) || !std::isfinite(dmax)) return fail(LAGP_EINVAL, "need 0 < dmin < dmax (finite)");
  const int lds_max = max_lds_per_block();
  if (!lagp::mle_supported(n, p, (size_t)lds_max)) return fail(LAGP_EINVAL, "local MLE needs n <= LAGP_MAX_N");
  if (!chol && lagp::local_lds_bytes(n, (nc + 15) & ~15, p, rays, false) > (size_t)lds_max)
    return fail(LAGP_EINVAL, "local design too large for LDS (n, p, numrays)");
  if (M == 0) return LAGP_OK;
  if (!XX || !mean || !s2 || !df || !dhat) return fail(LAGP_EINVAL, "XX, mean, s2, df and dhat must not be NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int S = lagp::knn_sort_size(nc);
  if (!cand_in && lagp::knn2_merge_lds_bytes(S) > (size_t)lds_max) return fail(LAGP_EINVAL, "ncand too large for LDS");
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t b_knn = cand_in ? 0 : lagp::knn2_bytes_per_location(nc) + 1024;
  const size_t b_cand = cand_in ? 0 : sizeof(int32_t) * (size_t)nc;
  const size_t b_sel = sel_idx ? 0 : sizeof(int32_t) * (size_t)n;
  // stage scratch: status of each search, the stage-one estimate, flags and evaluations
  const size_t b_st = sizeof(int32_t) * 6, b_th = sizeof(double);
  // k_local's per-location buffers (kernel rows, k(x_c, x), coordinates,
  // starting-inverse scratch, status) for the ray and nearest-neighbour searches
  const size_t b_loc = chol ? 0 : lagp::predict_per_location_bytes(d, P, true);
  // the likelihood's matrices of designs past the LDS sizes
  const size_t b_mle = lagp::mle_workspace_bytes_per_location(n, p, (size_t)lds_max);
  const size_t per = b_knn + b_cand + b_sel + b_st + b_th + b_loc + b_mle;
  int cw_slots = 0;  // Cholesky scoring past the on-chip sizes: the streaming kernel's slots
  const size_t b_cw = lagp::chol_stream_fixed(d, P, workspace_budget(), &cw_slots);
  const size_t budget = workspace_budget() > b_cw ? workspace_budget() - b_cw : 0;
  const int64_t chunk = std::min<int64_t>(M, std::max<int64_t>(lagp::KNN_QB, (int64_t)(budget / per)));
  Workspace ws;
  ws.s = s;
  const size_t o_knn = 0, o_cand = o_knn + al(b_knn * chunk), o_sel = o_cand + al(b_cand * chunk),
               o_st = o_sel + al(b_sel * chunk), o_th = o_st + al(b_st * chunk), o_loc = o_th + al(b_th * chunk),
               o_mle = o_loc + al(b_loc * chunk) + 5 * 256, o_sub = o_mle + al(b_mle * chunk),
               o_cw = o_sub + al(cand_in ? 0 : lagp::knn2_shared_bytes(d->N, p, nc)), total = o_cw + b_cw;
  LAGP_HIP(hipMallocAsync(&ws.ptr, total, s));
  char* base = reinterpret_cast<char*>(ws.ptr);
  for (int64_t m0 = 0; m0 < M; m0 += chunk) {
    const int32_t mc = (int32_t)std::min<int64_t>(chunk, M - m0);
    const int32_t* cand = cand_in ? cand_in + m0 * nc : reinterpret_cast<const int32_t*>(base + o_cand);
    if (!cand_in)
      LAGP_HIP(lagp::launch_knn2(knn_args(d, XX + m0 * p, mc, nc, base + o_knn, chunk, base + o_sub,
                                          reinterpret_cast<int32_t*>(base + o_cand), nullptr),
                                 s));
    int32_t* sel = sel_idx ? sel_idx + m0 * n : reinterpret_cast<int32_t*>(base + o_sel);
    int32_t* stw = reinterpret_cast<int32_t*>(base + o_st);
    int32_t *st1 = stw, *fl1 = stw + chunk, *it1 = stw + 2 * chunk, *st2 = stw + 3 * chunk;
    int32_t* st_out = status ? status + m0 : stw + 4 * chunk;
    int32_t* it_out = iters ? iters + m0 : stw + 5 * chunk;
    double* th1 = reinterpret_cast<double*>(base + o_th);
    lagp::LocalArgs a = lagp::local_args(d, P, rays, XX + m0 * p, mc, cand);
    if (!chol) {  // [Kc: kc_rows x ncs][kxc: ncs][Xc: ncs x p][start scratch: 2 n0^2][K^{-1} past 128 points]
      const size_t ncs = (size_t)a.ncs, o_kxc = al(sizeof(double) * a.kc_rows * ncs * chunk),
                   o_xc = o_kxc + al(sizeof(double) * ncs * chunk), o_ch = o_xc + al(sizeof(double) * ncs * p * chunk),
                   o_ki = o_ch + al(sizeof(double) * 2 * (size_t)a.n0 * a.n0 * chunk);
      a.Kc = reinterpret_cast<double*>(base + o_loc);
      a.kxc = reinterpret_cast<double*>(base + o_loc + o_kxc);
      a.Xc = reinterpret_cast<double*>(base + o_loc + o_xc);
      a.chol = reinterpret_cast<double*>(base + o_loc + o_ch);
      a.kig = lagp::kig_bytes(P) ? reinterpret_cast<double*>(base + o_loc + o_ki) : nullptr;
    }
    a.mean = mean + m0;  // (overwritten by the prediction under the estimate)
    a.s2 = s2 + m0;
    a.df = df + m0;
    a.sel = sel;
    a.status = st1;
    a.cw = reinterpret_cast<double*>(base + o_cw);
    auto search = [&]() {
      return !chol ? lagp::launch_local(a, s) : cw_slots ? lagp::launch_chol_stream(a, cw_slots, s) : lagp::launch_chol(a, s);
    };
    LAGP_HIP(search());
    lagp::MleArgs e{};
    e.X = d->X;
    e.y = d->y;
    e.XX = XX + m0 * p;
    e.sel = sel;
    e.d0 = d0;
    e.dmin = dmin;
    e.dmax = dmax;
    e.tol = tol;
    e.g = P->g;
    e.maxit = maxit;
    e.n = n;
    e.p = p;
    e.M = mc;
    e.ws = b_mle ? reinterpret_cast<double*>(base + o_mle) : nullptr;
    e.status_in = st1;
    if (mle->mode == 1) {
      e.theta_out = dhat + m0;
      e.status_out = st_out;
      e.iters_out = it_out;
      e.mean = mean + m0;
      e.s2 = s2 + m0;
      e.df = df + m0;
      LAGP_HIP(lagp::launch_mle(e, s, (size_t)lds_max));
      continue;
    }
    e.theta_out = th1;
    e.status_out = fl1;
    e.iters_out = it1;
    e.nan_on_skip = 1;
    LAGP_HIP(lagp::launch_mle(e, s, (size_t)lds_max));
    a.dloc = th1;  // second stage: search under the estimate
    a.status = st2;
    LAGP_HIP(search());
    e.theta0 = th1;
    e.status_in = st2;
    e.flags_prev = fl1;
    e.iters_prev = it1;
    e.theta_out = dhat + m0;
    e.status_out = st_out;
    e.iters_out = it_out;
    e.mean = mean + m0;
    e.s2 = s2 + m0;
    e.df = df + m0;
    e.nan_on_skip = 0;
    LAGP_HIP(lagp::launch_mle(e, s, (size_t)lds_max));
  }
  return LAGP_OK;
}

// Global separable lengthscales on a subset (sepfit.hip), synchronous.
int32_t lagp_fit_separable(const double* XS, const double* yS, int32_t n, int32_t p, double g, double* theta,
                           double dmin, double dmax, double tol, int32_t maxit, int32_t maxsweep, int32_t* iters,
                           int32_t* status, void* stream) {
  if (n < 1 || n > lagp::SEP_NMAX) return fail(LAGP_EINVAL, "n must be in [1, 1024]");
  if (p < 1 || p > LAGP_MAX_DIM) return fail(LAGP_EINVAL, "p must be in [1, LAGP_MAX_DIM]");
  if (!XS || !yS || !theta) return fail(LAGP_EINVAL, "XS, yS and theta must not be NULL");
  if (!(g >= 0.0) || !std::isfinite(g)) return fail(LAGP_EINVAL, "nugget g must be finite and >= 0");
  if (!(dmin > 0.0) || !(dmin < dmax) || !std::isfinite(dmax)) return fail(LAGP_EINVAL, "need 0 < dmin < dmax (finite)");
  for (int k = 0; k < p; ++k)
    if (!(theta[k] > 0.0) || !std::isfinite(theta[k])) return fail(LAGP_EINVAL, "starting lengthscales must be finite and > 0");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  lagp::SepArgs a{};
  a.XS = XS;
  a.y = yS;
  a.n = n;
  a.p = p;
  a.g = g;
  a.dmin = dmin;
  a.dmax = dmax;
  a.tol = tol > 0.0 ? tol : 1e-8;
  a.maxit = maxit > 0 ? maxit : 100;
  a.maxsweep = maxsweep > 0 ? maxsweep : 20;
  // [theta: p][iters, flags][workspace]
  const size_t head = 256;
  Workspace ws;
  ws.s = s;
  LAGP_HIP(hipMallocAsync(&ws.ptr, head + lagp::sepfit_workspace_bytes(n), s));
  char* base = reinterpret_cast<char*>(ws.ptr);
  a.theta = reinterpret_cast<double*>(base);
  a.iters = reinterpret_cast<int32_t*>(base + 128);
  a.flags = a.iters + 1;
  a.ws = reinterpret_cast<double*>(base + head);
  LAGP_HIP(hipMemcpyAsync(a.theta, theta, sizeof(double) * p, hipMemcpyHostToDevice, s));
  LAGP_HIP(lagp::launch_sepfit(a, s));
  int32_t out2[2];
  LAGP_HIP(hipMemcpyAsync(theta, a.theta, sizeof(double) * p, hipMemcpyDeviceToHost, s));
  LAGP_HIP(hipMemcpyAsync(out2, a.iters, sizeof(int32_t) * 2, hipMemcpyDeviceToHost, s));
  LAGP_HIP(hipStreamSynchronize(s));
  if (iters) *iters = out2[0];
  if (status) *status = out2[1];
  return LAGP_OK;
}

// Inputs divided by the square roots of the lengthscales (sepfit.hip).
int32_t lagp_prescale(const double* X, int64_t N, int32_t p, const double* theta, double* out, void* stream) {
  if (N < 0) return fail(LAGP_EINVAL, "N must be >= 0");
  if (p < 1 || p > LAGP_MAX_DIM) return fail(LAGP_EINVAL, "p must be in [1, LAGP_MAX_DIM]");
  if (!theta) return fail(LAGP_EINVAL, "theta must not be NULL");
  for (int k = 0; k < p; ++k)
    if (!(theta[k] > 0.0) || !std::isfinite(theta[k])) return fail(LAGP_EINVAL, "lengthscales must be finite and > 0");
  if (N > 0 && (!X || !out)) return fail(LAGP_EINVAL, "X and out must not be NULL");
  LAGP_HIP(lagp::launch_prescale(X, N, p, theta, out, reinterpret_cast<hipStream_t>(stream)));
  return LAGP_OK;
}

}  // extern "C"
