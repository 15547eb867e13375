// Internal declarations of the local GP library (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "../../include/lagp.h"
#include "grid.h"

struct lagp_design {
  int64_t N;
  int32_t p;
  double* X;   // device, N x p row-major
  double* y;   // device, N
  double* lo;  // device, p: per-dimension minimum of X
  double* hi;  // device, p: per-dimension maximum of X
  double* rn;  // device, N: squared row norms of X (screening only)
  float* X32;  // device, N x p: X rounded to FP32 (screening only)
  double spread2;  // sum over dimensions of (max - min)^2 (chooses the kNN screen's precision)
  double rn_max;  // their maximum
  int device;
  double lo_h[LAGP_MAX_DIM], hi_h[LAGP_MAX_DIM];  // host copies of lo, hi
  // cell grid for snaps over the whole design (built on first use; the
  // device arrays belong to the handle)
  std::mutex grid_mu;
  bool grid_built = false;
  lagp::GridDev grid{};
  double* grid_Xs = nullptr;
  int32_t* grid_rows = nullptr;
  int32_t* grid_start = nullptr;
};

namespace lagp {

// Everything a local-design kernel needs for one chunk of locations.
struct LocalArgs {
  const double* X;
  const double* y;
  const double* lo;
  const double* hi;
  const double* XX;    // chunk locations, M x p
  const int32_t* cand; // M x ncand nearest rows, nearest first
  double* Kc;          // workspace, M x n x ncs: K(x_{J_i}, x_c) rows
  float* Kc32;         // workspace (mixed form only), the same rows in FP32
  double* kxc;         // workspace, M x ncs: K(x_c, x)
  double* Xc;          // workspace, M x ncs x p: candidate coordinates (rows past ncand zero)
  double* chol;        // workspace, M x n0 x n0 (starting inverse scratch)
  double* mean;
  double* s2;
  double* df;
  int32_t* sel;        // nullable, M x n
  double* diag;        // nullable, M x (n - n0) x 2
  int32_t* status;     // M
  int64_t N;
  int32_t M;
  int32_t p;
  int32_t n0, n, ncand, ncs, numrays;
  int32_t kc_rows;     // rows of Kc kept per location (n exhaustive, n0 otherwise)
  int32_t search, precision, rescore_k;
  int32_t dlen;
  int32_t brent_maxit;
  double brent_tol;
  double g;
  double w[LAGP_MAX_DIM];  // reciprocal lengthscales 1/d_k
  const double* dloc;      // nullable, M: per-location isotropic lengthscale (Cholesky form;
                           // a location whose entry is not > 0 is skipped, its status set to 0)
  double* cw;              // Cholesky form past the on-chip sizes: slots x chol_stream_slot_bytes
  int32_t* counts;         // nullable, M x (n - n0) x 2: per greedy step, the search's work:
                           // ray: Brent evaluations summed over the rays, the most of one ray;
                           // mixed: candidates whose FP32 upper bound reached the threshold,
                           // 16-candidate tiles re-scored in FP64; else: candidates scored, 0
  int32_t snap_full;       // ray search: snap over the whole design through `grid` (else the candidates)
  GridDev grid;
  double* kig;             // designs past 128 points (ray, nearest neighbours): M x NR x 257 K_J^{-1}
  // Cholesky form on chip: per-location design sizes (<= n, which then is the
  // stride of sel) and nuggets (both given or both null: n and g)
  const int32_t* nloc;
  const double* gloc;
};

// Per-location parameters of a merged batch (device arrays, M entries each):
// design size, isotropic lengthscale, nugget.
struct PerLocation {
  const int32_t* n;
  const double* d;
  const double* g;
};

// Arguments of the local MLE kernel (mle.hip) for one chunk of locations.
struct MleArgs {
  const double* X;
  const double* y;
  const double* XX;            // M x p
  const int32_t* sel;          // M x n design rows
  const double* theta0;        // nullable, M: starting lengthscales (else d0)
  double d0;
  const int32_t* status_in;    // nullable, M: status of the design stage
  const int32_t* flags_prev;   // nullable, M: status carried from an earlier stage
  const int32_t* iters_prev;   // nullable, M: evaluations carried from an earlier stage
  double* theta_out;           // M
  int32_t* status_out;         // M: status_in | flags_prev | this stage's flags
  int32_t* iters_out;          // M
  double* mean;                // nullable (then no prediction), M
  double* s2;
  double* df;
  double dmin, dmax, tol, g;
  int32_t maxit, n, p, M;
  int32_t nan_on_skip;         // a skipped location's theta_out: NaN (1) or its starting value (0)
  double* ws;                  // designs past the LDS sizes: M x mle_workspace_bytes_per_location
};

// Arguments of the threshold-first kNN (knn.hip).
struct Knn2Args {
  const double* X;
  const double* XX;   // M x p
  double* tau;        // workspace, M
  int32_t* cnt;       // workspace, M
  double* buf_d2;     // workspace, M x CAP
  int32_t* buf_idx;   // workspace, M x CAP
  int32_t* out_idx;   // M x ncand
  double* sub;        // workspace, sub_count x p: the threshold subsample
  const double* rn;   // N squared row norms of X
  const float* X32;   // nullable, N x p: X rounded to FP32 (the FP32 screen)
  double rn_max;
  double spread2;     // sum over dimensions of the design's squared extent
  double* out_d2;     // nullable, M x ncand
  int64_t N;
  int64_t sub_stride;
  int64_t sub_count;
  int64_t slice;
  int32_t M;
  int32_t p;
  int32_t ncand;
  int32_t S;
  int32_t CAP;
  int32_t force_fallback;  // test hook: every location takes the exact fallback scan
};

constexpr int KNN_QB = 8;        // smallest location chunk
constexpr int KNN_THREADS = 256;
constexpr int LOCAL_THREADS = 256;

int knn_sort_size(int ncand);
hipError_t launch_knn2(Knn2Args a, hipStream_t s);
hipError_t launch_row_norms(const double* X, int64_t N, int p, double* rn, double* rmax, float* X32, hipStream_t s);
int64_t knn2_sub_rows(int64_t N, int ncand);
size_t knn2_shared_bytes(int64_t N, int p, int ncand);  // per call, beside the per-location buffers
size_t knn2_bytes_per_location(int ncand);
size_t knn2_merge_lds_bytes(int S);

size_t local_lds_bytes(int n, int ncs, int p, int numrays, bool mixed);
hipError_t launch_local(const LocalArgs& a, hipStream_t s);

// Exhaustive search by incremental Cholesky columns (chol.hip): whether a
// shape fits its kernels, and the launch (no workspace beyond the arguments).
bool chol_supported(int n, int ncand, int p, size_t lds_max);
hipError_t launch_chol(const LocalArgs& a, hipStream_t s);
// The same search with the columns in a device workspace (cholws.hip), any
// n <= LAGP_MAX_N and ncand <= LAGP_MAX_NCAND: a persistent grid of at most
// `slots` workgroups, each owning chol_stream_slot_bytes of a.cw.
size_t chol_stream_slot_bytes(int n, int ncand, int p);
int chol_stream_max_slots(int ncand);
bool chol_stream_forced();  // test hook: LAGP_CHOL_FORCE_STREAM=1
hipError_t launch_chol_stream(const LocalArgs& a, int slots, hipStream_t s);

// Local MLE of the lengthscale and the prediction under it (mle.hip):
// n <= 50 in LDS, larger designs (n <= LAGP_MAX_N) in a per-location
// workspace slice.
size_t mle_lds_bytes(int n, int p);
bool mle_supported(int n, int p, size_t lds_max);
size_t mle_workspace_bytes_per_location(int n, int p, size_t lds_max);
hipError_t launch_mle(const MleArgs& a, hipStream_t s, size_t lds_max);

// Global separable fit on a subset (sepfit.hip): one workgroup, n <= SEP_NMAX.
constexpr int SEP_NMAX = 1024;
struct SepArgs {
  const double* XS;  // n x p subset coordinates
  const double* y;   // n
  int32_t n, p;
  double g, dmin, dmax, tol;
  int32_t maxit, maxsweep;
  double* theta;     // p: starting values in, estimates out
  int32_t* iters;    // 1: likelihood evaluations
  int32_t* flags;    // 1: LAGP_STATUS_MLE_* bits
  double* ws;        // sepfit_workspace_bytes(n)
};
struct PrescaleScales {
  double theta[LAGP_MAX_DIM];
};
size_t sepfit_workspace_bytes(int n);
hipError_t launch_sepfit(const SepArgs& a, hipStream_t s);
hipError_t launch_prescale(const double* X, int64_t N, int p, const double* theta, double* out, hipStream_t s);

hipError_t launch_bbox(const double* X, int64_t N, int p, double* lo, double* hi, hipStream_t s);

// The cell grid of a design (grid.hip): its shape from N, p and the bounding
// box; the build into caller-provided arrays (cid: N, cnt: cells scratch;
// start: cells + 1, Xs: N x p, rows: N), which fills g's pointers.
GridDev grid_plan(int64_t N, int p, const double* lo, const double* hi);
int64_t grid_cells(const GridDev& g);
hipError_t launch_grid_build(const double* X, int64_t N, int p, GridDev& g, int32_t* cid, int32_t* cnt,
                             int32_t* start, double* Xs, int32_t* rows, hipStream_t s);

// Shared by the C ABI and the server (api.cpp).
int32_t check_predict_params(const lagp_design* d, const lagp_params* P);
size_t predict_workspace_bytes(const lagp_design* d, const lagp_params* P, bool have_cand, int64_t M,
                               size_t ws_budget);
// ext_ws (nullable): a caller-provided device workspace of ext_bytes; the
// locations then run in chunks that fit it and nothing is allocated.
// pl (nullable): per-location n, d, g for exhaustive search by Cholesky
// columns on chip (P->n is then the largest n and the stride of sel_idx).
int32_t run_predict(const lagp_design* d, const double* XX, int64_t M, const int32_t* cand_in, const lagp_params* P,
                    double* mean, double* s2, double* df, int32_t* sel_idx, double* diag, int32_t* status,
                    void* stream, size_t ws_budget, void* ext_ws = nullptr, size_t ext_bytes = 0,
                    int32_t* counts = nullptr, const PerLocation* pl = nullptr);
bool chol_onchip_shape(const lagp_design* d, int n, int ncand);
const char* set_error(const char* msg);

}  // namespace lagp
