/*
 * lagp.h - C ABI of the MI355X local approximate Gaussian-process library.
 *
 * The library predicts, at every location x of a predictive set, with a GP
 * fitted to a small local design grown greedily from the design X_N
 * (Gramacy & Haaland, "Speeding up neighborhood search in local Gaussian
 * process prediction"):
 *   - candidates: the N' design rows nearest to x (Sec. 2.2, the restriction
 *     of the search to N' nearest neighbours);
 *   - start: the n0 nearest rows (Sec. 2.2);
 *   - greedy steps j = n0 .. n-1 add the candidate maximising the reduction
 *     in predictive variance at x, the integrand of Eq. (alc) (Sec. 3.1),
 *     found by exhaustive scoring of the remaining candidates or by the ray
 *     search of Sec. 4 (rays from x, Brent line search, snap to the nearest
 *     candidate); the local inverse grows by the partitioned-inverse update
 *     whose pieces G_j, g_j, v_j appear under Eq. (alc);
 *   - prediction: the Student-t mean and scale of Eqs. (predgp), (preds2)
 *     with the n local points in place of N, and n degrees of freedom.
 * Correlation K(a,b) = exp(-sum_k (a_k-b_k)^2 / d_k) (Sec. 2.1), one d
 * (isotropic) or one per dimension (separable); nugget g on the design
 * diagonal and in the prior variance 1 + g at candidates and at x.
 *
 * Conventions for every entry point:
 *   - arrays are row-major; X is N x p, XX is M x p, all FP64;
 *   - "device" pointers are HIP device memory (hipMalloc, or a torch CUDA
 *     tensor's data_ptr on ROCm); the caller owns every input and output;
 *   - stream is a hipStream_t passed as void* (NULL: the default stream);
 *     work is enqueued on it and outputs are valid once it is synchronised;
 *   - return codes: LAGP_OK (0) success, LAGP_EINVAL bad argument (checked
 *     on the host before anything is enqueued), LAGP_ENOMEM allocation
 *     failure, LAGP_EDEVICE a HIP error, LAGP_EAGAIN a full server queue,
 *     LAGP_WARN_NUMERIC success but some locations hit a numerical problem
 *     (their status word is non-zero).  lagp_last_error() gives the text of
 *     the last failure on the calling thread.  No C++ exception crosses the
 *     ABI.
 */
#ifndef LAGP_H
#define LAGP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LAGP_OK 0
#define LAGP_EINVAL (-1)
#define LAGP_ENOMEM (-2)
#define LAGP_EDEVICE (-3)
#define LAGP_EAGAIN (-4)
#define LAGP_WARN_NUMERIC 1

#define LAGP_MAX_DIM 16    /* largest input dimension p */
#define LAGP_MAX_N 256     /* largest local design size n */
#define LAGP_MAX_NCAND 4096 /* largest candidate count N' */
#define LAGP_MAX_RAYS 32   /* largest number of rays per greedy step */

/* search modes */
#define LAGP_SEARCH_EXHAUSTIVE 0 /* score every remaining candidate (Sec. 3.1) */
#define LAGP_SEARCH_RAY 1        /* rays + Brent + snap (Sec. 4) */
#define LAGP_SEARCH_NN 2         /* the n nearest neighbours, no search (Sec. 2.2) */

/* precision forms */
#define LAGP_PREC_FP64 0  /* everything in FP64, every sum in its defined order (bit-reproducible) */
#define LAGP_PREC_MIXED 1 /* candidate screening in FP32 on MFMA, shortlist re-scored in FP64 */

/* scoring forms of exhaustive search (both FP64) */
#define LAGP_SCORING_PARTINV 0 /* partitioned-inverse updates as the paper writes them; every sum in a
                                  defined order, bit-reproducible */
#define LAGP_SCORING_CHOL 1    /* incremental Cholesky columns: u_c = L^{-1} k_J(x_c) grows by one
                                  entry per step, so a step costs O(j) per candidate instead of
                                  O(j^2); the same criterion and prediction to rounding (not bit
                                  for bit), with smaller FP64 error at small nuggets.  Needs
                                  precision FP64 and exhaustive search.  Up to n = 50 and
                                  ncand = 1024 (512 when p > 8) the columns stay on chip; larger
                                  shapes keep them in a device workspace of about
                                  8 (n + p) ncand bytes per resident workgroup. */

/* snap scope of ray search (Sec. 4: the continuous optimum is snapped to a
 * design point; Sec. 5: ray searches are not restricted to the N' nearest) */
#define LAGP_SNAP_CANDIDATES 0 /* the nearest of the ncand candidates */
#define LAGP_SNAP_DESIGN 1     /* the nearest of the whole design, through a cell grid of the design
                                  built on first use (lagp_design_build_grid); ncand then only has to
                                  hold the ray starts */

/* per-location status bits */
#define LAGP_STATUS_VNONPOS 1   /* a Schur complement v <= 0 was met; scored as 0 */
#define LAGP_STATUS_NONFINITE 2 /* non-finite mean or scale */
#define LAGP_STATUS_NOTPD 4     /* the starting n0 x n0 covariance is not positive definite */
#define LAGP_STATUS_MLE_BOUND 16 /* local MLE: the lengthscale estimate sits at a bound of its range */
#define LAGP_STATUS_MLE_NOTPD 32 /* local MLE: K was not positive definite at some Newton iterate */
#define LAGP_STATUS_MLE_MAXIT 64 /* local MLE: the Newton iteration ran out of iterations */

typedef struct lagp_design lagp_design;
typedef struct lagp_server lagp_server;

/* Method parameters (laGP's start, end, close, numrays, d, g, method).
 *   n0: nearest neighbours in the starting design, 1 <= n0 <= n;
 *   n: final local design size, n <= LAGP_MAX_N;
 *   ncand: N', nearest candidates searched, n <= ncand <= min(N, LAGP_MAX_NCAND);
 *   numrays: rays per greedy step in ray search (<= 0 means p, Sec. 5's
 *     default); the candidate list must hold n - 1 + numrays + the largest
 *     round-robin offset (Sec. 4) entries;
 *   search: LAGP_SEARCH_*; precision: LAGP_PREC_*;
 *   d_len: 1 (isotropic) or p (separable); d[0..d_len-1] > 0;
 *   g: nugget >= 0;
 *   rescore_k: size of the FP64 re-scored shortlist in the mixed form (1..64);
 *   scoring: LAGP_SCORING_* (exhaustive search only; 0 otherwise);
 *   brent_maxit, brent_tol: Brent line-search budget (<= 0: 100) and
 *     tolerance (<= 0: 2^-13);
 *   snap: LAGP_SNAP_* (ray search only; 0 otherwise); reserved: 0. */
typedef struct {
  int32_t n0;
  int32_t n;
  int32_t ncand;
  int32_t numrays;
  int32_t search;
  int32_t precision;
  int32_t d_len;
  int32_t rescore_k;
  double d[LAGP_MAX_DIM];
  double g;
  int32_t brent_maxit;
  int32_t scoring;
  double brent_tol;
  int32_t snap;
  int32_t reserved;
} lagp_params;

/* Local maximum likelihood of an isotropic lengthscale (Sec. 5: every
 * local design is coupled with a Newton-like estimate of the lengthscale
 * from the local likelihood, Eq. gpk with the n local points; optionally a
 * second-stage re-design under that estimate).
 *   mode: 1 = estimate on the design searched under params->d[0], predict
 *         under the estimate on that design; 2 = two stages: search under
 *         d0, estimate, search again under the estimate, estimate again
 *         from it, predict on the second design;
 *   dmin, dmax: the range of the estimate (<= 0: d0/1000 and 100 d0);
 *   tol: stop when a Newton step moves the estimate by at most tol times it
 *        (<= 0: 1e-8); maxit: likelihood evaluations per stage (<= 0: 100). */
typedef struct {
  int32_t mode;
  int32_t maxit;
  double dmin;
  double dmax;
  double tol;
} lagp_mle_params;

/* Library version, major*10000 + minor*100 + patch. */
int32_t lagp_version(void);

/* Text of the last error on the calling thread ("" if none).  The pointer
 * stays valid until the next failing call on this thread. */
const char* lagp_last_error(void);

/* Upload a design (Sec. 2.1: the N x p inputs X_N and responses Y_N).
 * X (N x p) and y (N) are device pointers; the handle keeps its own device
 * copies and the bounding box of X (used to cut rays, Sec. 4), so the inputs
 * may be freed once the stream is synchronised.  1 <= p <= LAGP_MAX_DIM,
 * N >= 1.  *out receives the handle.  The handle is immutable: concurrent
 * lagp_predict calls on different streams may share it. */
int32_t lagp_design_create(const double* X, const double* y, int64_t N, int32_t p, void* stream,
                           lagp_design** out);

/* Release a design handle (NULL is ignored).  Synchronises the device. */
void lagp_design_destroy(lagp_design* design);

/* Build the design's cell grid for snaps over the whole design (ray search
 * with snap = LAGP_SNAP_DESIGN, Sec. 5) if it is not built yet: the first
 * min(p, 3) coordinates cut into about N / 2 cells (at most 2^22) between
 * their minimum and maximum, each row and its coordinates grouped by cell.
 * Device memory N (8 p + 4) + 4 (cells + 1) bytes, owned by the handle and
 * freed with it.  Synchronous (the stream is synchronised before return);
 * thread-safe.  The predict calls build it themselves on first use; callers
 * that must not allocate during them (lagp_predict_noalloc) call this
 * first.  LAGP_EINVAL on a NULL design, LAGP_ENOMEM, LAGP_EDEVICE. */
int32_t lagp_design_build_grid(const lagp_design* design, void* stream);

/* Dimensions of a design handle. */
int32_t lagp_design_info(const lagp_design* design, int64_t* N, int32_t* p);

/* The ncand design rows nearest to each location (Sec. 2.2): for location m,
 * cand_idx[m*ncand + r] is the row of rank r, ordered by squared distance
 * then row index, and cand_d2 (nullable) its squared distance (dimensions
 * summed in order with one fused multiply-add each).  XX (M x p),
 * cand_idx (M x ncand, int32) and cand_d2 (M x ncand) are device pointers.
 * 1 <= ncand <= min(N, LAGP_MAX_NCAND); M >= 0 (M == 0 is a no-op). */
int32_t lagp_candidates(const lagp_design* design, const double* XX, int64_t M, int32_t ncand,
                        int32_t* cand_idx, double* cand_d2, void* stream);

/* Local approximate GP prediction at the M rows of XX (device, M x p).
 * Outputs (device): mean, s2 (Student-t scale sigma^2 of Eq. preds2 with n
 * local points) and df (= n), each of length M; sel_idx (nullable, M x n
 * int32) the design rows of the local design in selection order; diag
 * (nullable, M x (n - n0) x 2) per greedy step the best and runner-up
 * criterion values the search saw (exhaustive: the two largest ALC; ray: the
 * two best ray optima); status (nullable, M int32) LAGP_STATUS_* bits.
 * Locations are independent; their results do not depend on M or on which
 * other locations share the call.  Workspace is allocated on the stream
 * (stream-ordered) and released on it; locations are processed in chunks
 * whose workspace fits a budget (16 GiB, or LAGP_WORKSPACE_MB from the
 * environment; about 0.5 MB per location at n = 50, N' = 1000, p = 8).
 * The call is asynchronous: it
 * returns LAGP_OK once the work is enqueued, and numerical trouble at a
 * location shows only in its status word. */
int32_t lagp_predict(const lagp_design* design, const double* XX, int64_t M, const lagp_params* params,
                     double* mean, double* s2, double* df, int32_t* sel_idx, double* diag, int32_t* status,
                     void* stream);

/* Local GP prediction from candidate lists already on the device, as
 * lagp_candidates writes them: cand_idx (M x params->ncand int32, nearest
 * first; with LAGP_SNAP_DESIGN the lists must be exactly the ncand nearest
 * rows, as the whole-design snap relies on every other row lying at least
 * as far from x as the list's last).  Everything else as lagp_predict.  Lets a caller keep candidate
 * lists resident and re-run the design search (another n, search mode or
 * precision) without repeating the neighbour search. */
int32_t lagp_predict_candidates(const lagp_design* design, const double* XX, int64_t M, const int32_t* cand_idx,
                                const lagp_params* params, double* mean, double* s2, double* df, int32_t* sel_idx,
                                double* diag, int32_t* status, void* stream);

/* lagp_predict_candidates (cand_idx nullable: NULL searches the candidates
 * here) with the work of each greedy step reported, for measurement (the
 * paper's Sec. 6 notes that ray searches vary in length: the slowest take
 * about twice the mean evaluations).  counts (device, nullable,
 * M x (n - n0) x 2 int32), per location and step:
 *   ray search (Sec. 4): [0] objective evaluations of the Brent line
 *     searches summed over the step's rays (each search's first evaluation
 *     included, the s = 0 checks not), [1] the most evaluations of one ray;
 *   mixed form: [0] candidates whose FP32 upper bound on the FP64 criterion
 *     reached the threshold (the certified shortlist), [1] 16-candidate
 *     tiles re-scored in FP64;
 *   FP64 exhaustive search (Sec. 3.1): [0] candidates scored (N' - j), [1] 0.
 * Nearest-neighbour search has no greedy step.  Results as lagp_predict. */
int32_t lagp_predict_counts(const lagp_design* design, const double* XX, int64_t M, const int32_t* cand_idx,
                            const lagp_params* params, double* mean, double* s2, double* df, int32_t* sel_idx,
                            double* diag, int32_t* status, int32_t* counts, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation and outputs as lagp_predict (bit for bit), with every
 * workspace taken from a fixed per-device scratch area of
 * LAGP_NOALLOC_SCRATCH_BYTES (64 MiB) that the library holds on each GPU it
 * runs on until the process ends.  Nothing is allocated or freed by this
 * call.  Locations run in chunks that fit the scratch (about 1,200 per
 * chunk at n = 50, N' = 1000 with Cholesky scoring and a 1e6-row design;
 * about 100 with the partitioned-inverse form, whose kernel rows are kept
 * in the workspace).  LAGP_ENOMEM when even one location's workspace plus
 * the per-call candidate-search subsample exceeds the scratch; LAGP_EINVAL
 * when the current device is not the design's or as lagp_predict.  Every
 * call on one GPU shares that GPU's scratch and leaves its contents behind
 * (nothing in it needs to start cleared: every kernel writes what it reads,
 * counters included): calls that overlap on one GPU, from several threads
 * or on several streams, race and must be serialised by the caller. */
#define LAGP_NOALLOC_SCRATCH_BYTES (64u << 20)
int32_t lagp_predict_noalloc(const lagp_design* design, const double* XX, int64_t M, const lagp_params* params,
                             double* mean, double* s2, double* df, int32_t* sel_idx, double* diag, int32_t* status,
                             void* stream);

/* Local GP prediction with local maximum likelihood of the lengthscale
 * (lagp_mle_params).  The estimate maximises the local likelihood
 * l(d) = -1/2 log|K| - n/2 log(y^T K^-1 y) of the n local points (Eq. gpk,
 * nugget fixed) by Newton's method on l'(d) = 0 from analytic first and
 * second derivatives, kept inside a bracket that shrinks from [dmin, dmax]
 * (geometric bisection when a Newton step would leave it); the prediction
 * (Eqs. predgp, preds2 with n local points) is taken under the estimate
 * through the Cholesky factor of K.  The design search is any of the three
 * (Sec. 5 couples each with local inference): exhaustive (either scoring),
 * rays, or nearest neighbours (whose design does not depend on d, so its
 * second stage repeats the first).  Needs n <= 50, an isotropic lengthscale
 * (d_len = 1) and precision FP64.  cand_idx (nullable, device, M x ncand int32) gives the
 * candidate lists as lagp_candidates writes them; NULL searches them here.
 * Outputs (device): mean, s2, df (M); dhat (M) the estimate used; sel_idx
 * (nullable, M x n) the final local design; iters (nullable, M) likelihood
 * evaluations over all stages; status (nullable, M) LAGP_STATUS_* bits of
 * every stage or'ed.  A location whose design search fails reports NaN mean
 * and scale and the lengthscale it was searched under.  Otherwise as
 * lagp_predict (asynchronous on the stream, workspace stream-ordered). */
int32_t lagp_predict_mle(const lagp_design* design, const double* XX, int64_t M, const int32_t* cand_idx,
                         const lagp_params* params, const lagp_mle_params* mle, double* mean, double* s2,
                         double* df, double* dhat, int32_t* sel_idx, int32_t* iters, int32_t* status,
                         void* stream);

/* ---- pre-scaling by global separable lengthscales (Sec. 5.3) ------------
 *
 * Local designs searched on inputs divided by the square roots of global
 * lengthscales estimated on a subset of the data align ray searches with
 * exhaustive ones on anisotropic responses (Sec. 5.3).  The two calls below
 * give the fit and the scaling; the caller draws the subset, scales the
 * design and the predictive locations with the same lengthscales, and runs
 * the local path on the scaled inputs (an isotropic lengthscale, typically
 * with local MLE). */

/* Global separable lengthscales theta_k of K(x, x') = exp(-sum_k
 * (x_k - x'_k)^2 / theta_k) + g [x = x'] by maximum likelihood (Eq. gpk on
 * the n subset points, nugget g fixed), one coordinate at a time: each sweep
 * runs, for k = 0..p-1, the bracketed Newton iteration of lagp_predict_mle
 * on theta_k within [dmin, dmax] with the others fixed; sweeps repeat until
 * one moves no theta_k by more than tol theta_k (tol <= 0: 1e-8), at most
 * maxsweep times (<= 0: 20), with at most maxit evaluations per coordinate
 * (<= 0: 100).  XS (device, n x p row-major FP64, 1 <= n <= 1024,
 * p <= LAGP_MAX_DIM) and yS (device, n) stay the caller's.  theta (host, p)
 * holds the starting values on entry and the estimates on return; iters
 * (host, nullable) the likelihood evaluations; status (host, nullable) the
 * LAGP_STATUS_MLE_* bits (BOUND: some theta_k at a bound; MAXIT: a
 * coordinate or the sweeps ran out; NOTPD: some K not positive definite).
 * Runs on the stream and waits for it (the results are host values).
 * Workspace: 3 n^2 + 7 n doubles, stream-ordered.  LAGP_EINVAL on bad sizes
 * or bounds. */
int32_t lagp_fit_separable(const double* XS, const double* yS, int32_t n, int32_t p, double g, double* theta,
                           double dmin, double dmax, double tol, int32_t maxit, int32_t maxsweep, int32_t* iters,
                           int32_t* status, void* stream);

/* out[i][k] = X[i][k] / sqrt(theta[k]) for N rows of p coordinates (device,
 * row-major FP64; out may equal X).  theta: host, p values, each finite and
 * > 0.  Asynchronous on the stream.  LAGP_EINVAL on bad sizes or values. */
int32_t lagp_prescale(const double* X, int64_t N, int32_t p, const double* theta, double* out, void* stream);

/* ---- serving: continuous batching over a resident design ---------------
 *
 * A server owns a worker thread and one device stream per in-flight slot.
 * Requests (host location arrays plus parameters) are admitted as long as
 * the device memory they need fits the budget; admitted requests run
 * concurrently on the device, results stay in server memory until fetched.
 * Waiting requests with identical parameters share a batch; exhaustive FP64
 * requests scored by Cholesky columns on chip (n <= 50, N' <= 1024, one
 * isotropic lengthscale, no snap) share one whatever their n, lengthscale
 * and nugget, which the batch then carries per location into a single
 * launch.  Each slot holds pinned host staging for its largest batch (4096
 * locations at n = 256 with their per-location parameters: (1072 + 8 p) x
 * 4096 bytes), allocated at creation and released by lagp_server_destroy;
 * submits and batches allocate no pinned memory. */

/* Create a server on a design.  hbm_budget_bytes bounds the device memory
 * the admitted requests may hold at once; max_inflight bounds how many run
 * together (1 ..= 64).  LAGP_EDEVICE when a stream or the pinned staging
 * cannot be created. */
int32_t lagp_server_create(const lagp_design* design, size_t hbm_budget_bytes, int32_t max_inflight,
                           lagp_server** out);

/* Submit a request: XX_host (M x p, host memory, copied before return),
 * params as for lagp_predict.  *ticket receives its id.  LAGP_EAGAIN when the
 * queue of waiting requests is full; LAGP_ENOMEM when the request alone can
 * never fit the budget. */
int32_t lagp_server_submit(lagp_server* server, const double* XX_host, int64_t M, const lagp_params* params,
                           uint64_t* ticket);

/* *done = 1 once the ticket's results are ready on the host, else 0. */
int32_t lagp_server_poll(lagp_server* server, uint64_t ticket, int32_t* done);

/* Block until the ticket is done, then copy its results into host arrays
 * (each nullable; mean/s2/df length M, sel_idx M x n, status M) and release
 * the ticket.  *latency_ms (nullable) receives submit-to-ready time. */
int32_t lagp_server_fetch(lagp_server* server, uint64_t ticket, double* mean, double* s2, double* df,
                          int32_t* sel_idx, int32_t* status, double* latency_ms);

/* Latency percentiles over fetched requests and prediction throughput
 * since creation or the last reset. */
int32_t lagp_server_stats(lagp_server* server, double* p50_ms, double* p99_ms, double* pred_per_s,
                          int32_t reset);

/* Drain outstanding work and release the server (NULL is ignored). */
void lagp_server_destroy(lagp_server* server);

#ifdef __cplusplus
}
#endif

#endif /* LAGP_H */
