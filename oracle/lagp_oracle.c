/*
 * Plain FP64 CPU oracle for local approximate GP prediction with greedy
 * local designs (Gramacy & Haaland, "Speeding up neighborhood search in
 * local Gaussian process prediction").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker for the HIP library:
 * only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code, header or constant with the
 * GPU path.  Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC.
 *
 * What it computes, per predictive location x (all FP64):
 *   O1 kernel      K(a,b) = exp(-sum_k (a_k-b_k)^2 / d_k)           (Sec. 2.1),
 *                  evaluated with the reciprocals 1/d_k
 *                  design covariance K_J = [K(x_i,x_l)] + g I         (Sec. 2.1,
 *                  nugget; Eq. alc uses K_eta on the diagonal)
 *   O2 candidates  the N' design rows nearest to x, ordered by
 *                  (squared distance, row index)                      (Sec. 2.2)
 *   O3 start       J = the n0 nearest; K_J^{-1} via Cholesky          (Sec. 2.2)
 *   O4 greedy step for j = n0..n-1 add the candidate that maximises the
 *                  integrand of Eq. alc (reduction in variance at x), found
 *                  by exhaustive scoring of C \ J or by ray search     (Sec. 3.1,
 *                  Sec. 4)
 *   O5 update      partitioned inverse: K_{j+1}^{-1} from K_j^{-1} with
 *                  G_j = g_j g_j^T, g_j = -K_j^{-1} k_j(x_{j+1}) / v_j  (Sec. 3.1,
 *                  the quantities under Eq. alc, sign of g_j corrected)
 *   O6 predict     Student-t mean and scale with n degrees of freedom (Eqs.
 *                  predgp and preds2 with N -> n)                     (Sec. 2.1)
 *   O7 Cholesky    the same exhaustive search and prediction through the
 *      form        Cholesky factor of K_J grown one row per step (local_one_chol
 *                  below): the criterion and prediction of O4-O6 in another
 *                  rounding order, and the checker of the library's Cholesky
 *                  scoring form
 *   O8 local MLE   the isotropic lengthscale maximising the local marginal
 *                  likelihood (Eq. gpk with the n local points) by a
 *                  safeguarded Newton iteration on its analytic derivatives,
 *                  and the two-stage re-design: search under d0, estimate,
 *                  search again under the estimate, estimate again, predict
 *                  (Sec. 5)
 *
 * Rounding is defined, not left to the compiler, so that another
 * implementation can reproduce every value here bit for bit: squared
 * distances and every inner product accumulate their terms in index order
 * from 0.0 with one fused multiply-add per term; exp is the routine oexp
 * below (Cody-Waite reduction, Taylor series of degree 13); division and
 * square root are IEEE; nothing else is fused (-ffp-contract=off).
 *
 * Readings where the paper is silent or garbled (each listed in the design
 * notes of the repository): ties in distance, ALC,
 * ray value and snap distance go to the smaller candidate rank (or row index
 * for the nearest-neighbour order); g_j carries a minus sign so that the
 * integrand of Eq. alc equals (K(x_c,x) - k_c^T K^{-1} k_x)^2 / v_c, the
 * squared posterior covariance over the posterior variance; the prior
 * variance at a candidate, at a point on a ray and at x is 1 + g; v_c <= 0
 * scores 0 and raises a status flag; Brent's tolerance defaults to
 * 2^-13 = eps^(1/4) and its iteration budget to 100.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_NDIAG 8
#define ORC_STATUS_VNONPOS 1   /* some v_c <= 0 was scored as 0 */
#define ORC_STATUS_NONFINITE 2 /* non-finite prediction */
#define ORC_STATUS_NOTPD 4     /* starting K_J not positive definite */
#define ORC_STATUS_BADRAY 8    /* too few remaining candidates for the rays */
#define ORC_STATUS_MLE_BOUND 16 /* the lengthscale estimate sits at a bound of its range */
#define ORC_STATUS_MLE_NOTPD 32 /* K was not positive definite at some Newton iterate */
#define ORC_STATUS_MLE_MAXIT 64 /* the Newton iteration ran out of iterations */

/* ---------------------------------------------------------------- O1 ---- */

/* Squared Euclidean distance, dimensions accumulated in order with one fused
 * multiply-add each: s <- fma(t_k, t_k, s), t_k = a_k - b_k. */
static double sqdist(const double *a, const double *b, int p)
{
    double s = 0.0;
    for (int k = 0; k < p; k++) {
        double t = a[k] - b[k];
        s = fma(t, t, s);
    }
    return s;
}

/* exp(x): write x = k ln2 + r with k = nearest integer to x/ln2 and
 * |r| <= ln2/2 (Cody & Waite's reduction, ln2 split into the nearest double
 * and its remainder, each step one fused multiply-add), sum the Taylor series
 * of exp(r) to degree 13 by Horner's rule with fused multiply-adds (the
 * truncation error r^14/14! is below 1e-17), then scale by 2^k.  Results
 * that would be subnormal (x < -708) are flushed to 0; every argument used
 * here is <= 0. */
static double oexp(double x)
{
    if (x != x) return x;
    if (x < -708.0) return 0.0;
    if (x > 709.0) return INFINITY;
    const double ln2_hi = 0.6931471805599453;      /* 0x1.62e42fefa39efp-1 */
    const double ln2_lo = 2.3190468138462996e-17;  /* ln2 - ln2_hi */
    const double inv_ln2 = 1.4426950408889634;     /* 0x1.71547652b82fep+0 */
    double k = nearbyint(x * inv_ln2);
    double r = fma(-k, ln2_hi, x);
    r = fma(-k, ln2_lo, r);
    double q = 1.0 / 6227020800.0;                 /* 1/13! */
    q = fma(q, r, 1.0 / 479001600.0);              /* 1/12! */
    q = fma(q, r, 1.0 / 39916800.0);
    q = fma(q, r, 1.0 / 3628800.0);
    q = fma(q, r, 1.0 / 362880.0);
    q = fma(q, r, 1.0 / 40320.0);
    q = fma(q, r, 1.0 / 5040.0);
    q = fma(q, r, 1.0 / 720.0);
    q = fma(q, r, 1.0 / 120.0);
    q = fma(q, r, 1.0 / 24.0);
    q = fma(q, r, 1.0 / 6.0);
    q = fma(q, r, 0.5);
    q = fma(q, r, 1.0);
    q = fma(q, r, 1.0);
    return ldexp(q, (int)k);
}

/* Gaussian correlation, Sec. 2.1: isotropic exp(-r^2/d) when d_len == 1,
 * separable exp(-sum_k (a_k-b_k)^2/d_k) otherwise.  No nugget here.  The
 * lengthscales enter through their reciprocals w_k = 1/d_k (each rounded
 * once): isotropic exp(-(r^2 w)), separable s <- fma(t_k t_k, w_k, s). */
static double kern(const double *a, const double *b, int p, const double *w, int d_len)
{
    if (d_len == 1)
        return oexp(-(sqdist(a, b, p) * w[0]));
    double s = 0.0;
    for (int k = 0; k < p; k++) {
        double t = a[k] - b[k];
        s = fma(t * t, w[k], s);
    }
    return oexp(-s);
}

/* ---------------------------------------------------------------- O2 ---- */

typedef struct {
    double d2;
    int64_t idx;
} nbr;

/* strict total order: (d2, idx) */
static int nbr_less(nbr a, nbr b)
{
    return a.d2 < b.d2 || (a.d2 == b.d2 && a.idx < b.idx);
}

static void heap_sift_down(nbr *h, int n, int i)
{
    for (;;) {
        int l = 2 * i + 1, r = l + 1, top = i;
        if (l < n && nbr_less(h[top], h[l])) top = l;
        if (r < n && nbr_less(h[top], h[r])) top = r;
        if (top == i) return;
        nbr t = h[i]; h[i] = h[top]; h[top] = t;
        i = top;
    }
}

static int nbr_cmp(const void *a, const void *b)
{
    nbr x = *(const nbr *)a, y = *(const nbr *)b;
    return nbr_less(x, y) ? -1 : (nbr_less(y, x) ? 1 : 0);
}

/* The ncand design rows nearest to x, ascending in (d2, row).  A max-heap of
 * size ncand keeps the best seen so far; the survivors are then sorted. */
static void knn_one(const double *X, int64_t N, int p, const double *x, int ncand,
                    int64_t *idx_out, double *d2_out, nbr *heap)
{
    int size = 0;
    for (int64_t i = 0; i < N; i++) {
        nbr c = {sqdist(X + i * p, x, p), i};
        if (size < ncand) {
            heap[size] = c;
            for (int k = size++; k > 0;) {
                int par = (k - 1) / 2;
                if (!nbr_less(heap[par], heap[k])) break;
                nbr t = heap[par]; heap[par] = heap[k]; heap[k] = t;
                k = par;
            }
        } else if (nbr_less(c, heap[0])) {
            heap[0] = c;
            heap_sift_down(heap, size, 0);
        }
    }
    qsort(heap, size, sizeof(nbr), nbr_cmp);
    for (int r = 0; r < size; r++) {
        idx_out[r] = heap[r].idx;
        if (d2_out) d2_out[r] = heap[r].d2;
    }
}

/* ------------------------------------------------------------- linalg --- */

/* Inverse of a small symmetric positive definite matrix A (n x n, row-major)
 * through its Cholesky factor: A = L L^T, A^{-1} = L^{-T} L^{-1}.
 * Returns 0 on success, -1 if a pivot is not positive. */
static int spd_inverse(const double *A, int n, double *Ainv, double *work)
{
    double *L = work;             /* n*n */
    double *Li = work + n * n;    /* n*n, inverse of L (lower) */
    memset(L, 0, sizeof(double) * n * n);
    for (int i = 0; i < n; i++) {
        for (int k = 0; k <= i; k++) {
            double s = A[i * n + k];
            for (int m = 0; m < k; m++) s = fma(-L[i * n + m], L[k * n + m], s);
            if (i == k) {
                if (!(s > 0.0)) return -1;
                L[i * n + i] = sqrt(s);
            } else {
                L[i * n + k] = s / L[k * n + k];
            }
        }
    }
    memset(Li, 0, sizeof(double) * n * n);
    for (int c = 0; c < n; c++) {            /* solve L Li[:,c] = e_c */
        for (int i = c; i < n; i++) {
            double s = (i == c) ? 1.0 : 0.0;
            for (int m = c; m < i; m++) s = fma(-L[i * n + m], Li[m * n + c], s);
            Li[i * n + c] = s / L[i * n + i];
        }
    }
    for (int i = 0; i < n; i++)              /* Ainv = Li^T Li */
        for (int k = 0; k < n; k++) {
            double s = 0.0;
            for (int m = (i > k ? i : k); m < n; m++) s = fma(Li[m * n + i], Li[m * n + k], s);
            Ainv[i * n + k] = s;
        }
    return 0;
}

/* y = A x, A is j x j with leading dimension ld */
static void matvec(const double *A, int ld, int j, const double *x, double *y)
{
    for (int i = 0; i < j; i++) {
        double s = 0.0;
        for (int k = 0; k < j; k++) s = fma(A[i * ld + k], x[k], s);
        y[i] = s;
    }
}

static double dot(const double *a, const double *b, int j)
{
    double s = 0.0;
    for (int i = 0; i < j; i++) s = fma(a[i], b[i], s);
    return s;
}

/* ------------------------------------------------------ per location ---- */

typedef struct {
    const double *X, *y;
    int64_t N;
    int p;
    int n0, n, ncand, search, numrays;
    const double *d; /* reciprocal lengthscales 1/d_k */
    int d_len;
    double g;
    int brent_maxit;
    double brent_tol;
    const double *lo, *hi; /* bounding box of the whole design */
    int scoring;           /* exhaustive search: 0 partitioned inverse (O5), 1 Cholesky form (O7) */
} ctx_t;

typedef struct {
    /* per location scratch */
    nbr *heap;
    int64_t *cand;       /* ncand row ids, nearest first */
    double *cand_d2;
    double *Kc;          /* n x ncand: K(x_{J_i}, x_c) for every candidate c */
    double *kxc;         /* ncand: K(x_c, x) */
    double *Ki;          /* n x n, leading dimension n */
    double *kx, *h, *w, *gv, *kz, *tmp;
    double *cv, *cr;     /* ncand: Cholesky form, v_c and y_c - z^T u_c */
    int *J;              /* ranks of the selected candidates */
    char *inJ;           /* ncand flags */
    char *forbid;        /* ncand flags (ray starts) */
} scratch_t;

/* Continuous-point ALC for ray search (Eq. alc integrand at z, Sec. 4):
 * (K(z,x) - k_J(z)^T K^{-1} k_J(x))^2 / ((1+g) - k_J(z)^T K^{-1} k_J(z)). */
typedef struct {
    const ctx_t *c;
    scratch_t *s;
    const double *x;
    int j;
    const double *a, *dir; /* segment p(s) = a + s * dir */
    double *z;
    int vflag;
} rayfn_t;

static double alc_at(const ctx_t *c, scratch_t *s, const double *x, int j, const double *z, int *vflag)
{
    for (int i = 0; i < j; i++)
        s->kz[i] = kern(c->X + s->cand[s->J[i]] * c->p, z, c->p, c->d, c->d_len);
    matvec(s->Ki, c->n, j, s->kz, s->w);
    double v = (1.0 + c->g) - dot(s->kz, s->w, j);
    double cov = kern(z, x, c->p, c->d, c->d_len) - dot(s->w, s->kx, j);
    if (!(v > 0.0)) {
        *vflag = 1;
        return 0.0;
    }
    return cov * cov / v;
}

static double ray_negalc(double t, void *vp)
{
    rayfn_t *r = (rayfn_t *)vp;
    for (int k = 0; k < r->c->p; k++) r->z[k] = fma(t, r->dir[k], r->a[k]);
    return -alc_at(r->c, r->s, r->x, r->j, r->z, &r->vflag);
}

/* relative gap of a comparison: |a-b| / max(|a|,|b|).  Two exact zeros are
 * not a near-tie (they come out of underflowed kernels on any machine). */
static double relgap(double a, double b)
{
    double m = fmax(fabs(a), fabs(b));
    if (m == 0.0) return INFINITY;
    return fabs(a - b) / m;
}

/*
 * Brent's (1973) derivative-free minimiser of a function on [lo, hi]: golden
 * section search, replaced by a parabolic step through the three best points
 * whenever that step falls inside the bracket and is shorter than half the
 * step before last; no evaluation closer than tol1 = sqrt(eps)|x| + tol/3
 * to the current best point; stop once the bracket half-width about the
 * best point is within 2 tol1 (Sec. 4 names this routine, Brent_fmin).
 * Direction conventions of that routine: a parabolic step that would land
 * within 2 tol1 of an end becomes a step of tol1 towards the midpoint, taken
 * downwards when the best point is at or above the midpoint; a step shorter
 * than tol1 is lengthened to tol1 in its own direction, downwards when it is
 * zero.
 * *mingap (if given) receives the smallest relative gap among the decisions
 * the iteration took, so callers can tell near-tie steps apart.
 */
double orc_brent_min(double (*f)(double, void *), void *arg, double lo, double hi, double tol,
                     int maxit, int *nevals, double *mingap, double *fbest)
{
    const double gold = 0.5 * (3.0 - sqrt(5.0));
    const double sqeps = sqrt(DBL_EPSILON);
    double a = lo, b = hi;
    double x = a + gold * (b - a);
    double w = x, v = x;
    double fx = f(x, arg);
    double fw = fx, fv = fx;
    double step = 0.0, prev = 0.0; /* last step and the one before it */
    double gap = INFINITY;
    int evals = 1;

    for (int it = 0; it < maxit; it++) {
        double mid = 0.5 * (a + b);
        double tol1 = sqeps * fabs(x) + tol / 3.0;
        double tol2 = 2.0 * tol1;
        double lhs = fabs(x - mid), rhs = tol2 - 0.5 * (b - a);
        gap = fmin(gap, relgap(lhs, rhs));
        if (lhs <= rhs) break;

        int parabolic = 0;
        if (fabs(prev) > tol1) {
            /* parabola through (x,fx), (w,fw), (v,fv): step = num/den */
            double r = (x - w) * (fx - fv);
            double q = (x - v) * (fx - fw);
            double num = (x - v) * q - (x - w) * r;
            double den = 2.0 * (q - r);
            if (den > 0.0) num = -num;
            den = fabs(den);
            double older = prev;
            prev = step;
            double half = fabs(0.5 * den * older);
            gap = fmin(gap, relgap(fabs(num), half));
            gap = fmin(gap, relgap(num, den * (a - x)));
            gap = fmin(gap, relgap(num, den * (b - x)));
            if (fabs(num) < half && num > den * (a - x) && num < den * (b - x)) {
                step = num / den;
                double u = x + step;
                if (u - a < tol2 || b - u < tol2) step = (x >= mid) ? -tol1 : tol1;
                parabolic = 1;
            }
        }
        if (!parabolic) {
            prev = (x >= mid) ? a - x : b - x;
            step = gold * prev;
        }
        double u = (fabs(step) >= tol1) ? x + step : ((step > 0.0) ? x + tol1 : x - tol1);
        double fu = f(u, arg);
        evals++;
        gap = fmin(gap, relgap(fu, fx));
        if (fu <= fx) {
            if (u >= x) a = x; else b = x;
            v = w; fv = fw;
            w = x; fw = fx;
            x = u; fx = fu;
        } else {
            if (u < x) a = u; else b = u;
            gap = fmin(gap, relgap(fu, fw));
            if (fu <= fw || w == x) {
                v = w; fv = fw;
                w = u; fw = fu;
            } else {
                gap = fmin(gap, relgap(fu, fv));
                if (fu <= fv || v == x || v == w) {
                    v = u; fv = fu;
                }
            }
        }
    }
    if (nevals) *nevals = evals;
    if (mingap) *mingap = gap;
    if (fbest) *fbest = fx;
    return x;
}

/* Round-robin start of the ray sequence, Sec. 4: k = t mod floor(sqrt(t)),
 * t = j - n0 + 1 (0-based rank among the remaining candidates). */
int orc_ray_k0(int t)
{
    int r = 0;
    while ((r + 1) * (r + 1) <= t) r++;
    return r > 0 ? t % r : 0;
}

/* Segment of a ray, Sec. 4: from start a, directed away from x, of length
 * ten times |a - x|, cut at the bounding box [lo, hi] of the design.
 * dir receives e - a for the clipped end e; returns the cut fraction tau. */
double orc_ray_segment(const double *a, const double *x, const double *lo, const double *hi, int p,
                       double *dir)
{
    double tau = 1.0;
    for (int k = 0; k < p; k++) {
        double dk = 10.0 * (a[k] - x[k]);
        dir[k] = dk;
        if (dk > 0.0) tau = fmin(tau, (hi[k] - a[k]) / dk);
        else if (dk < 0.0) tau = fmin(tau, (lo[k] - a[k]) / dk);
    }
    if (tau < 0.0) tau = 0.0;
    for (int k = 0; k < p; k++) dir[k] = tau * dir[k];
    return tau;
}

/*
 * O7: exhaustive search through the Cholesky factor.  With K_J + g I = L L^T
 * for the design J so far, free candidate q carries the column
 * u_q = L^{-1} k_J(x_q) (entries U[k*ncand + q], k < |J|) and
 *   v_q   = (1 + g) - u_q^T u_q        (v_j of Eq. alc at x_q)
 *   cov_q = K(x_q, x) - w^T u_q        w = L^{-1} k_J(x)
 *   r_q   = y_q - z^T u_q              z = L^{-1} y_J
 * so that k_J(x_q)^T K_J^{-1} k_J(x) = u_q^T w and the integrand of Eq. alc
 * at x is cov_q^2 / v_q.  Taking candidate t appends (u_t^T, l) to L with
 * l = sqrt(v_t); with li = 1/l (one IEEE division), w_j = cov_t li,
 * z_j = r_t li, and every free q gets
 *   u_q[j] = (K(x_t, x_q) - u_t^T u_q) li
 * after which v_q, cov_q and r_q drop u_q[j]^2, w_j u_q[j] and z_j u_q[j].
 * The n0 nearest enter first, in rank order (that is the Cholesky
 * factorisation of the starting K_J, Sec. 2.2).  Prediction: mean w^T z,
 * psi = z^T z, k_x^T K^{-1} k_x = w^T w (Eqs. predgp, preds2, N -> n).
 * Sums run in index order with one fused multiply-add per term; ties go to
 * the smaller rank; v_q <= 0 scores 0 and raises the status flag, as in O4.
 * trace_Ki (nullable) is filled with NaN: this form never forms K^{-1}.
 */
static int local_one_chol(const ctx_t *c, scratch_t *s, const double *x, const int32_t *forced,
                          double *mean, double *s2, double *df, int32_t *sel, double *diag, double *trace_alc,
                          double *trace_Ki)
{
    const int p = c->p, n = c->n, nc = c->ncand, n0 = c->n0;
    const double *X = c->X;
    double *U = s->Kc, *v = s->cv, *cov = s->kxc, *r = s->cr;
    int status = 0;

    knn_one(X, c->N, p, x, nc, s->cand, s->cand_d2, s->heap);
    memset(s->inJ, 0, nc);
    for (int q = 0; q < nc; q++) {
        v[q] = 1.0 + c->g;
        cov[q] = kern(X + s->cand[q] * p, x, p, c->d, c->d_len);
        r[q] = c->y[s->cand[q]];
    }
    if (trace_Ki)
        for (int i = 0; i < n * n; i++) trace_Ki[i] = NAN;
    double mu = 0.0, psi = 0.0, qq = 0.0;
    int done = 0;
    for (int j = 0; j < n; j++) {
        int take = j, best = -1;
        double alc1 = -INFINITY, alc2 = -INFINITY, gap = INFINITY;
        if (j >= n0) {
            for (int q = 0; q < nc; q++) {
                if (trace_alc) trace_alc[(size_t)(j - n0) * nc + q] = NAN;
                if (s->inJ[q]) continue;
                double a;
                if (v[q] > 0.0) a = cov[q] * cov[q] / v[q];
                else { a = 0.0; status |= ORC_STATUS_VNONPOS; }
                if (trace_alc) trace_alc[(size_t)(j - n0) * nc + q] = a;
                if (a > alc1) { alc2 = alc1; alc1 = a; best = q; }
                else if (a > alc2) alc2 = a;
            }
            gap = (alc1 > 0.0) ? (alc1 - alc2) / alc1 : 0.0;
            take = best;
            if (forced) {
                take = -1;
                for (int q = 0; q < nc; q++)
                    if (s->cand[q] == (int64_t)forced[j]) { take = q; break; }
                if (take < 0 || s->inJ[take]) return -2;
            }
            if (take < 0) break; /* no finite criterion anywhere: no prediction */
        }
        if (j < n0 && !(v[take] > 0.0)) {
            /* the starting covariance is not positive definite */
            *mean = NAN;
            *s2 = NAN;
            *df = (double)n;
            if (sel)
                for (int i = 0; i < n; i++) sel[i] = (i < n0) ? (int32_t)s->cand[i] : -1;
            return ORC_STATUS_NOTPD | ORC_STATUS_NONFINITE;
        }
        if (!(v[take] > 0.0)) status |= ORC_STATUS_VNONPOS;
        const double l = sqrt(v[take]), li = 1.0 / l;
        const double wj = cov[take] * li, zj = r[take] * li;
        const double bj = (1.0 + c->g) - qq; /* (1+g) - k_x^T K_j^{-1} k_x before the step */
        mu = fma(wj, zj, mu);
        psi = fma(zj, zj, psi);
        qq = fma(wj, wj, qq);
        if (diag && j >= n0) {
            double *dg = diag + (size_t)(j - n0) * ORC_NDIAG;
            dg[0] = (best >= 0) ? (double)s->cand[best] : -1.0;
            dg[1] = alc1;
            dg[2] = alc2;
            dg[3] = (v[take] > 0.0) ? cov[take] * cov[take] / v[take] : 0.0;
            dg[4] = gap;
            dg[5] = 0.0;
            dg[6] = bj;
            dg[7] = 0.0;
        }
        s->J[j] = take;
        s->inJ[take] = 1;
        done = j + 1;
        if (j + 1 == n) break;
        const double *xt = X + s->cand[take] * p;
        for (int q = 0; q < nc; q++) {
            if (s->inJ[q]) continue;
            double d = 0.0;
            for (int k = 0; k < j; k++) d = fma(U[(size_t)k * nc + take], U[(size_t)k * nc + q], d);
            const double e = (kern(xt, X + s->cand[q] * p, p, c->d, c->d_len) - d) * li;
            U[(size_t)j * nc + q] = e;
            v[q] = fma(-e, e, v[q]);
            cov[q] = fma(-wj, e, cov[q]);
            r[q] = fma(-zj, e, r[q]);
        }
    }
    if (done == n) {
        *mean = mu;
        *s2 = psi * ((1.0 + c->g) - qq) / (double)n;
    } else {
        *mean = NAN;
        *s2 = NAN;
    }
    *df = (double)n;
    if (!isfinite(*mean) || !isfinite(*s2)) status |= ORC_STATUS_NONFINITE;
    if (sel)
        for (int i = 0; i < n; i++) sel[i] = (i < done) ? (int32_t)s->cand[s->J[i]] : -1;
    return status;
}

/* One location: local design, then prediction.  forced (nullable) gives a
 * selection sequence (design row ids, n entries) to follow instead of the
 * oracle's own choices; the oracle's own choice is still recorded per step.
 * diag (nullable): per greedy step ORC_NDIAG values
 *   [0] oracle's choice (row id)      [1] best score (ALC_1)
 *   [2] runner-up score (ALC_2)       [3] ALC of the candidate actually added
 *   [4] smallest relative decision gap [5] Brent evaluations (ray)
 *   [6] b_j = (1+g) - k_x^T K_j^{-1} k_x before the step
 *   [7] ray search: s* of the winning ray (0 when its start was taken)
 * trace_alc (nullable): (n-n0) x ncand ALC of every candidate (NaN if in J)
 * trace_Ki (nullable): final n x n inverse.
 */
static int local_one(const ctx_t *c, scratch_t *s, const double *x, const int32_t *forced,
                     double *mean, double *s2, double *df, int32_t *sel, double *diag,
                     double *trace_alc, double *trace_Ki)
{
    if (c->scoring == 1) return local_one_chol(c, s, x, forced, mean, s2, df, sel, diag, trace_alc, trace_Ki);
    const int p = c->p, n = c->n, nc = c->ncand;
    const double *X = c->X;
    int status = 0;
    int n0 = (c->search == 2) ? n : c->n0; /* nearest-neighbour mode: J = n nearest */

    knn_one(X, c->N, p, x, nc, s->cand, s->cand_d2, s->heap);
    memset(s->inJ, 0, nc);
    for (int q = 0; q < nc; q++) s->kxc[q] = kern(X + s->cand[q] * p, x, p, c->d, c->d_len);

    /* O3: J = the n0 nearest */
    for (int i = 0; i < n0; i++) {
        s->J[i] = i;
        s->inJ[i] = 1;
        const double *xi = X + s->cand[i] * p;
        for (int q = 0; q < nc; q++) s->Kc[(size_t)i * nc + q] = kern(xi, X + s->cand[q] * p, p, c->d, c->d_len);
    }
    {
        double *A = s->tmp;                       /* n0 x n0 */
        double *work = s->tmp + (size_t)n * n;    /* 2 n0 n0 */
        double *Ai = s->tmp + (size_t)3 * n * n;
        for (int i = 0; i < n0; i++)
            for (int k = 0; k < n0; k++) A[i * n0 + k] = s->Kc[(size_t)i * nc + k] + (i == k ? c->g : 0.0);
        if (spd_inverse(A, n0, Ai, work) != 0) {
            /* the paper is silent here; reading: no prediction for this x */
            *mean = NAN;
            *s2 = NAN;
            *df = (double)n;
            if (sel)
                for (int i = 0; i < n; i++) sel[i] = (i < n0) ? (int32_t)s->cand[i] : -1;
            return ORC_STATUS_NOTPD | ORC_STATUS_NONFINITE;
        }
        for (int i = 0; i < n0; i++)
            for (int k = 0; k < n0; k++) s->Ki[i * n + k] = Ai[i * n0 + k];
    }
    for (int i = 0; i < n0; i++) s->kx[i] = s->kxc[i];

    /* O4 / O5: greedy growth */
    for (int j = n0; j < n; j++) {
        double *dg = diag ? diag + (size_t)(j - n0) * ORC_NDIAG : NULL;
        matvec(s->Ki, n, j, s->kx, s->h);                 /* h = K^{-1} k_x */
        double bj = (1.0 + c->g) - dot(s->kx, s->h, j);
        int best = -1;
        double alc1 = -INFINITY, alc2 = -INFINITY, gap = INFINITY, swin = 0.0;
        int evals = 0;

        if (c->search == 0 || trace_alc) {
            /* exhaustive scoring of every remaining candidate, rank order */
            for (int q = 0; q < nc; q++) {
                if (trace_alc) trace_alc[(size_t)(j - n0) * nc + q] = NAN;
                if (s->inJ[q]) continue;
                for (int i = 0; i < j; i++) s->kz[i] = s->Kc[(size_t)i * nc + q];
                matvec(s->Ki, n, j, s->kz, s->w);                      /* w = K^{-1} k_c */
                double v = (1.0 + c->g) - dot(s->kz, s->w, j);
                double cov = s->kxc[q] - dot(s->w, s->kx, j);
                double a;
                if (v > 0.0) a = cov * cov / v;
                else { a = 0.0; status |= ORC_STATUS_VNONPOS; }
                if (trace_alc) trace_alc[(size_t)(j - n0) * nc + q] = a;
                if (c->search != 0) continue;
                if (a > alc1) { alc2 = alc1; alc1 = a; best = q; }
                else if (a > alc2) alc2 = a;
            }
            if (c->search == 0) gap = (alc1 > 0.0) ? (alc1 - alc2) / alc1 : 0.0;
        }
        if (c->search == 1) {
            /* ray search, Sec. 4 */
            int R = c->numrays > 0 ? c->numrays : p;
            int t = j - n0 + 1, k0 = orc_ray_k0(t);
            int starts[64];
            int got = 0, seen = 0;
            memset(s->forbid, 0, nc);
            for (int q = 0; q < nc && got < R; q++) {
                if (s->inJ[q]) continue;
                if (seen++ >= k0) { starts[got++] = q; s->forbid[q] = 1; }
            }
            if (got < R) { status |= ORC_STATUS_BADRAY; R = got; }
            double bestval = -INFINITY, secondval = -INFINITY, bests = 0.0;
            int bestr = -1;
            double dirs[64 * 16], zs[16], bestz[16];
            for (int r = 0; r < R; r++) {
                const double *a = X + s->cand[starts[r]] * p;
                double *dir = dirs + r * p;
                double tau = orc_ray_segment(a, x, c->lo, c->hi, p, dir);
                rayfn_t fn = {c, s, x, j, a, dir, zs, 0};
                double sstar = 0.0, val;
                int vflag = 0;
                double a0 = alc_at(c, s, x, j, a, &vflag);
                if (tau > 0.0) {
                    int ne = 0;
                    double bg = INFINITY, fb = 0.0;
                    sstar = orc_brent_min(ray_negalc, &fn, 0.0, 1.0, c->brent_tol, c->brent_maxit, &ne, &bg, &fb);
                    evals += ne;
                    gap = fmin(gap, bg);
                    val = -fb;
                    gap = fmin(gap, relgap(a0, val));
                    if (a0 >= val) { sstar = 0.0; val = a0; } /* s = 0 post-check */
                } else {
                    val = a0;
                }
                if (fn.vflag || vflag) status |= ORC_STATUS_VNONPOS;
                if (val > bestval) {
                    secondval = bestval; bestval = val; bestr = r; bests = sstar;
                } else if (val > secondval) secondval = val;
            }
            if (R > 1) gap = fmin(gap, relgap(bestval, secondval));
            alc1 = bestval;
            alc2 = secondval;
            swin = bests;
            if (bests == 0.0) {
                best = starts[bestr];
            } else {
                /* snap the continuous optimum to the nearest allowed candidate */
                const double *a = X + s->cand[starts[bestr]] * p;
                const double *dir = dirs + bestr * p;
                for (int k = 0; k < p; k++) bestz[k] = fma(bests, dir[k], a[k]);
                double dbest = INFINITY, dsec = INFINITY;
                for (int q = 0; q < nc; q++) {
                    if (s->inJ[q] || s->forbid[q]) continue;
                    double dq = sqdist(X + s->cand[q] * p, bestz, p);
                    if (dq < dbest) { dsec = dbest; dbest = dq; best = q; }
                    else if (dq < dsec) dsec = dq;
                }
                gap = fmin(gap, relgap(dbest, dsec));
            }
        }
        if (c->search == 2) best = -1; /* unreachable: n0 == n */

        /* the candidate actually added */
        int take = best;
        if (forced) {
            take = -1;
            for (int q = 0; q < nc; q++)
                if (s->cand[q] == (int64_t)forced[j]) { take = q; break; }
            if (take < 0 || s->inJ[take]) return -2; /* forced choice not a free candidate */
        }
        if (take < 0) return -3;

        /* O5: partitioned-inverse update with the chosen candidate */
        for (int i = 0; i < j; i++) s->kz[i] = s->Kc[(size_t)i * nc + take];
        matvec(s->Ki, n, j, s->kz, s->w);
        double v = (1.0 + c->g) - dot(s->kz, s->w, j);
        double cov = s->kxc[take] - dot(s->w, s->kx, j);
        double alc_take = (v > 0.0) ? cov * cov / v : 0.0;
        if (!(v > 0.0)) status |= ORC_STATUS_VNONPOS;
        for (int i = 0; i < j; i++) s->gv[i] = -s->w[i] / v;       /* g_j */
        for (int i = 0; i < j; i++)
            for (int k = 0; k < j; k++) s->Ki[i * n + k] = fma(s->gv[i] * s->gv[k], v, s->Ki[i * n + k]); /* + G_j v_j */
        for (int i = 0; i < j; i++) {
            s->Ki[i * n + j] = s->gv[i];
            s->Ki[j * n + i] = s->gv[i];
        }
        s->Ki[j * n + j] = 1.0 / v;

        if (dg) {
            dg[0] = (best >= 0) ? (double)s->cand[best] : -1.0;
            dg[1] = alc1;
            dg[2] = alc2;
            dg[3] = alc_take;
            dg[4] = gap;
            dg[5] = (double)evals;
            dg[6] = bj;
            dg[7] = swin;
        }
        s->J[j] = take;
        s->inJ[take] = 1;
        s->kx[j] = s->kxc[take];
        const double *xt = X + s->cand[take] * p;
        for (int q = 0; q < nc; q++) s->Kc[(size_t)j * nc + q] = kern(xt, X + s->cand[q] * p, p, c->d, c->d_len);
    }

    /* O6: prediction with the local design of size n */
    {
        double *yJ = s->tmp;
        for (int i = 0; i < n; i++) yJ[i] = c->y[s->cand[s->J[i]]];
        matvec(s->Ki, n, n, s->kx, s->h);
        double mu = dot(s->h, yJ, n);
        matvec(s->Ki, n, n, yJ, s->w);
        double psi = dot(yJ, s->w, n);
        double sc = psi * ((1.0 + c->g) - dot(s->kx, s->h, n)) / (double)n;
        *mean = mu;
        *s2 = sc;
        *df = (double)n;
        if (!isfinite(mu) || !isfinite(sc)) status |= ORC_STATUS_NONFINITE;
    }
    if (sel)
        for (int i = 0; i < n; i++) sel[i] = (int32_t)s->cand[s->J[i]];
    if (trace_Ki) memcpy(trace_Ki, s->Ki, sizeof(double) * n * n);
    return status;
}

static int scratch_alloc(scratch_t *s, int n, int ncand)
{
    memset(s, 0, sizeof(*s));
    s->heap = malloc(sizeof(nbr) * ncand);
    s->cand = malloc(sizeof(int64_t) * ncand);
    s->cand_d2 = malloc(sizeof(double) * ncand);
    s->Kc = malloc(sizeof(double) * (size_t)n * ncand);
    s->kxc = malloc(sizeof(double) * ncand);
    s->Ki = calloc((size_t)n * n, sizeof(double));
    s->kx = malloc(sizeof(double) * n);
    s->h = malloc(sizeof(double) * n);
    s->w = malloc(sizeof(double) * n);
    s->gv = malloc(sizeof(double) * n);
    s->kz = malloc(sizeof(double) * n);
    s->tmp = malloc(sizeof(double) * (size_t)4 * n * n + 16);
    s->cv = malloc(sizeof(double) * ncand);
    s->cr = malloc(sizeof(double) * ncand);
    s->J = malloc(sizeof(int) * n);
    s->inJ = malloc(ncand);
    s->forbid = malloc(ncand);
    return (s->heap && s->cand && s->cand_d2 && s->Kc && s->kxc && s->Ki && s->kx && s->h && s->w &&
            s->gv && s->kz && s->tmp && s->cv && s->cr && s->J && s->inJ && s->forbid) ? 0 : -1;
}

static void scratch_free(scratch_t *s)
{
    free(s->heap); free(s->cand); free(s->cand_d2); free(s->Kc); free(s->kxc); free(s->Ki);
    free(s->kx); free(s->h); free(s->w); free(s->gv); free(s->kz); free(s->tmp); free(s->cv); free(s->cr); free(s->J);
    free(s->inJ); free(s->forbid);
}

static int check_args(int64_t N, int p, int n0, int n, int ncand, int search, int numrays, const double *d,
                      int d_len, double g, int scoring)
{
    if (scoring < 0 || scoring > 1 || (scoring == 1 && search != 0)) return -1;
    if (N < 1 || p < 1 || p > 16) return -1;
    if (n0 < 1 || n < n0 || ncand < n || (int64_t)ncand > N) return -1;
    if (search < 0 || search > 2) return -1;
    if (search == 1 && (numrays > 64)) return -1;
    if (!(d_len == 1 || d_len == p)) return -1;
    for (int k = 0; k < d_len; k++)
        if (!(d[k] > 0.0)) return -1;
    if (!(g >= 0.0)) return -1;
    return 0;
}

/* bounding box of the whole design */
static void bbox(const double *X, int64_t N, int p, double *lo, double *hi)
{
    for (int k = 0; k < p; k++) { lo[k] = INFINITY; hi[k] = -INFINITY; }
    for (int64_t i = 0; i < N; i++)
        for (int k = 0; k < p; k++) {
            double v = X[i * p + k];
            if (v < lo[k]) lo[k] = v;
            if (v > hi[k]) hi[k] = v;
        }
}

/* ---------------------------------------------------------------- O8 ---- */

/*
 * Local marginal likelihood of an isotropic lengthscale theta on a fixed
 * local design (Eq. gpk with N -> n and the nugget g fixed):
 *   l(theta) = -1/2 log|K| - n/2 log psi,  psi = y^T K^{-1} y,
 *   K = E + g I,  E_ik = exp(-a_ik),  a_ik = D_ik w,  w = 1/theta,
 * D_ik the squared distances of the design points (O1 rounding).  With
 * Kd = dK/dtheta = E a w and Kdd = d2K/dtheta2 = E (a^2 - 2a) w^2,
 * alpha = K^{-1} y, beta = Kd alpha:
 *   l'  = -1/2 tr(K^{-1} Kd) + n/2 (alpha^T beta) / psi
 *   l'' = -1/2 [tr(K^{-1} Kdd) - tr(K^{-1} Kd K^{-1} Kd)]
 *         + n/2 [(alpha^T Kdd alpha - 2 beta^T K^{-1} beta) / psi + ((alpha^T beta) / psi)^2]
 * (differentiating log|K| and psi).  Every sum runs in index order with one
 * fused multiply-add per term; a trace is the in-order sum of its row sums.
 * ws: 8 n^2 + 4 n doubles.  Returns 0, or -1 if K is not positive definite.
 */
static int mle_eval_tail(int n, const double *y, double *ws, double *l, double *d1, double *d2);

static int mle_eval(int n, const double *D, const double *y, double g, double theta, double *ws, double *l,
                    double *d1, double *d2)
{
    const double w = 1.0 / theta;
    double *E = ws, *K = E + n * n, *Kd = K + n * n, *Kdd = Kd + n * n;
    for (int i = 0; i < n; i++)
        for (int k = 0; k < n; k++) {
            const double a = D[i * n + k] * w;
            const double e = oexp(-a);
            E[i * n + k] = e;
            K[i * n + k] = e + (i == k ? g : 0.0);
            Kd[i * n + k] = (e * a) * w;
            Kdd[i * n + k] = (e * (a * a - 2.0 * a)) * (w * w);
        }
    return mle_eval_tail(n, y, ws, l, d1, d2);
}

/* The rest of an evaluation, from K, Kd and Kdd in ws (laid out as in
 * mle_eval): K^{-1}, the vectors, P = K^{-1} Kd, the traces, l, l', l''. */
static int mle_eval_tail(int n, const double *y, double *ws, double *l, double *d1, double *d2)
{
    double *E = ws, *K = E + n * n, *Kd = K + n * n, *Kdd = Kd + n * n, *Ki = Kdd + n * n, *P = Ki + n * n;
    double *work = P + n * n; /* 2 n^2: L, then L^{-1} */
    double *al = work + 2 * n * n, *be = al + n, *ga = be + n, *de = ga + n;
    if (spd_inverse(K, n, Ki, work) != 0) return -1;
    double logdet = 0.0; /* log|K| / 2 = sum_i log L_ii */
    for (int i = 0; i < n; i++) logdet += log(work[i * n + i]);
    matvec(Ki, n, n, y, al);
    const double psi = dot(y, al, n);
    matvec(Kd, n, n, al, be);
    const double ab = dot(al, be, n);
    matvec(Ki, n, n, be, ga);
    const double bgb = dot(be, ga, n);
    matvec(Kdd, n, n, al, de);
    const double add = dot(al, de, n);
    for (int i = 0; i < n; i++) /* P = K^{-1} Kd */
        for (int k = 0; k < n; k++) {
            double t = 0.0;
            for (int m = 0; m < n; m++) t = fma(Ki[i * n + m], Kd[m * n + k], t);
            P[i * n + k] = t;
        }
    double t1 = 0.0, t2 = 0.0, t3 = 0.0;
    for (int i = 0; i < n; i++) {
        double r1 = 0.0, r2 = 0.0, r3 = 0.0;
        for (int k = 0; k < n; k++) {
            r1 = fma(Ki[i * n + k], Kd[k * n + i], r1);
            r2 = fma(Ki[i * n + k], Kdd[k * n + i], r2);
            r3 = fma(P[i * n + k], P[k * n + i], r3);
        }
        t1 = t1 + r1;
        t2 = t2 + r2;
        t3 = t3 + r3;
    }
    const double hn = 0.5 * (double)n;
    const double q = ab / psi;
    *l = -logdet - hn * log(psi);
    *d1 = -0.5 * t1 + hn * q;
    *d2 = -0.5 * (t2 - t3) + hn * ((add - 2.0 * bgb) / psi + q * q);
    return 0;
}

/*
 * The maximiser of l on [dmin, dmax] by Newton's method on l' = 0, kept
 * inside a bracket: lo and hi start at the bounds; every iterate theta moves
 * lo up (l'(theta) > 0: the maximum lies above) or hi down; the Newton step
 * theta - l'/l'' is taken when l'' < 0 and it lands strictly inside the
 * bracket, else the geometric midpoint sqrt(lo hi); a K that is not positive
 * definite counts as l' < 0.  Stops when a step moves theta by at most
 * tol theta (or l' = 0), or after maxit evaluations.  The paper names the
 * method only as Newton-like maximisation of the local posterior; reading:
 * a flat prior on theta (the likelihood itself).
 */
typedef int (*eval1_fn)(void *ctx, double theta, double *l, double *d1, double *d2);

static double newton_1d(eval1_fn f, void *ctx, double theta0, double dmin, double dmax, double tol, int maxit,
                        int *iters, int *flags)
{
    double lo = dmin, hi = dmax;
    double theta = theta0 < lo ? lo : (theta0 > hi ? hi : theta0);
    int it = 0, conv = 0;
    *flags = 0;
    while (it < maxit) {
        double l, d1, d2;
        const int bad = f(ctx, theta, &l, &d1, &d2) != 0;
        it++;
        if (bad) {
            *flags |= ORC_STATUS_MLE_NOTPD;
            d1 = -1.0;
            d2 = 0.0;
        }
        if (d1 == 0.0) {
            conv = 1;
            break;
        }
        if (d1 > 0.0) lo = theta;
        else hi = theta;
        double tn = (d2 < 0.0) ? theta - d1 / d2 : lo;
        if (!(tn > lo && tn < hi)) tn = sqrt(lo * hi);
        const int done = fabs(tn - theta) <= tol * theta;
        theta = tn;
        if (done) {
            conv = 1;
            break;
        }
    }
    if (!conv) *flags |= ORC_STATUS_MLE_MAXIT;
    if (theta <= dmin * (1.0 + tol) || theta >= dmax * (1.0 - tol)) *flags |= ORC_STATUS_MLE_BOUND;
    *iters = it;
    return theta;
}

typedef struct {
    int n;
    const double *D, *y;
    double g;
    double *ws;
} iso_ctx;

static int iso_eval1(void *vp, double theta, double *l, double *d1, double *d2)
{
    const iso_ctx *c = (const iso_ctx *)vp;
    return mle_eval(c->n, c->D, c->y, c->g, theta, c->ws, l, d1, d2);
}

static double mle_fit(int n, const double *D, const double *y, double g, double theta0, double dmin, double dmax,
                      double tol, int maxit, double *ws, int *iters, int *flags)
{
    iso_ctx c = {n, D, y, g, ws};
    return newton_1d(iso_eval1, &c, theta0, dmin, dmax, tol, maxit, iters, flags);
}

/* Squared distances of the n design points (coordinates XJ, n x p). */
static void design_sqdist(int n, int p, const double *XJ, double *D)
{
    for (int i = 0; i < n; i++)
        for (int k = 0; k < n; k++) D[i * n + k] = sqdist(XJ + i * p, XJ + k * p, p);
}

/* The prediction of O6 at lengthscale theta on a given design, through the
 * Cholesky factor K = L L^T (O7's form, accurate where K is ill
 * conditioned): w = L^{-1} k_x, z = L^{-1} y by forward substitution
 * (x_i = (b_i - sum_{m<i} L_im x_m) / L_ii, the sum in m order with fused
 * multiply-adds), mean = w^T z, psi = z^T z, k_x^T K^{-1} k_x = w^T w. */
static int predict_theta(int n, int p, const double *XJ, const double *yJ, const double *x, double g, double theta,
                         double *mean, double *s2, double *ws)
{
    const double w = 1.0 / theta;
    double *K = ws, *L = K + n * n, *kx = L + n * n, *wv = kx + n, *z = wv + n;
    for (int i = 0; i < n; i++)
        for (int k = 0; k < n; k++)
            K[i * n + k] = kern(XJ + i * p, XJ + k * p, p, &w, 1) + (i == k ? g : 0.0);
    memset(L, 0, sizeof(double) * n * n);
    for (int i = 0; i < n; i++)
        for (int k = 0; k <= i; k++) {
            double t = K[i * n + k];
            for (int m = 0; m < k; m++) t = fma(-L[i * n + m], L[k * n + m], t);
            if (i == k) {
                if (!(t > 0.0)) {
                    *mean = NAN;
                    *s2 = NAN;
                    return -1;
                }
                L[i * n + i] = sqrt(t);
            } else {
                L[i * n + k] = t / L[k * n + k];
            }
        }
    for (int i = 0; i < n; i++) kx[i] = kern(XJ + i * p, x, p, &w, 1);
    for (int i = 0; i < n; i++) {
        double a = kx[i], b = yJ[i];
        for (int m = 0; m < i; m++) {
            a = fma(-L[i * n + m], wv[m], a);
            b = fma(-L[i * n + m], z[m], b);
        }
        wv[i] = a / L[i * n + i];
        z[i] = b / L[i * n + i];
    }
    *mean = dot(wv, z, n);
    const double psi = dot(z, z, n);
    *s2 = psi * ((1.0 + g) - dot(wv, wv, n)) / (double)n;
    return 0;
}

/* One location, local MLE (mode 1: estimate on the design searched under
 * d0 and predict there; mode 2: then search again under the estimate,
 * estimate again from it, and predict on the second design). */
static int local_mle(const ctx_t *c, scratch_t *s, const double *x, int mode, double dmin, double dmax, double tol,
                     int maxit, double *mean, double *s2, double *df, int32_t *sel, double *dhat, int32_t *iters)
{
    const int n = c->n, p = c->p;
    int32_t *J = malloc(sizeof(int32_t) * n);
    double *XJ = malloc(sizeof(double) * n * p), *yJ = malloc(sizeof(double) * n);
    double *D = malloc(sizeof(double) * n * n), *ws = malloc(sizeof(double) * (8 * n * n + 8 * n));
    int status = -2;
    if (!J || !XJ || !yJ || !D || !ws) goto out;
    status = 0; /* the flags of every stage, or'ed */
    const double d0 = 1.0 / c->d[0];
    double theta = d0;
    int total = 0;
    ctx_t cs = *c;
    double wstage;
    for (int stage = 1; stage <= mode; stage++) {
        if (stage == 2) {
            wstage = 1.0 / theta;
            cs.d = &wstage;
        }
        double m0, s0, f0;
        const int st = local_one(&cs, s, x, NULL, &m0, &s0, &f0, J, NULL, NULL, NULL);
        if (st < 0) {
            status = st;
            goto out;
        }
        status |= st;
        if (st & (ORC_STATUS_NOTPD | ORC_STATUS_NONFINITE)) {
            *mean = NAN;
            *s2 = NAN;
            *df = (double)n;
            *dhat = theta;
            *iters = total;
            if (sel) memcpy(sel, J, sizeof(int32_t) * n);
            goto out;
        }
        for (int i = 0; i < n; i++) {
            memcpy(XJ + i * p, c->X + (int64_t)J[i] * p, sizeof(double) * p);
            yJ[i] = c->y[J[i]];
        }
        design_sqdist(n, p, XJ, D);
        int it, flags;
        theta = mle_fit(n, D, yJ, c->g, theta, dmin, dmax, tol, maxit, ws, &it, &flags);
        total += it;
        status |= flags;
    }
    if (predict_theta(n, p, XJ, yJ, x, c->g, theta, mean, s2, ws) != 0) status |= ORC_STATUS_NOTPD;
    if (!isfinite(*mean) || !isfinite(*s2)) status |= ORC_STATUS_NONFINITE;
    *df = (double)n;
    *dhat = theta;
    *iters = total;
    if (sel) memcpy(sel, J, sizeof(int32_t) * n);
out:
    free(J);
    free(XJ);
    free(yJ);
    free(D);
    free(ws);
    return status;
}

/* ---------------------------------------------------------------- O9 ---- */

/*
 * Global separable lengthscales from a data subset, for pre-scaling the
 * inputs (Sec. 5.3: inputs divided by the square roots of global
 * lengthscales estimated on subsets of the data).  The likelihood is O8's
 * with the separable kernel of O1, K_ij = exp(-sum_k (x_ik - x_jk)^2 w_k)
 * + g [i = j], w_k = 1/theta_k, the exponent summed in k order with one
 * fused multiply-add per term.  Its derivatives in theta_k are O8's with
 * a_ij = (x_ik - x_jk)^2 w_k: dK/dtheta_k = E a w_k, d2K/dtheta_k^2 =
 * E (a^2 - 2a) w_k^2.  Reading (the paper names no optimiser for the
 * global fit): coordinate-wise maximisation, each coordinate by O8's
 * bracketed Newton iteration with the others fixed, in sweeps over
 * k = 0..p-1 that repeat until a sweep moves no theta_k by more than
 * tol theta_k, or maxsweep sweeps.  With p = 1 the exponent and derivatives
 * are O8's exactly.
 */
static int sep_eval(int n, int p, const double *XS, const double *y, double g, const double *theta, int k,
                    double *ws, double *l, double *d1, double *d2)
{
    double w[16];
    for (int q = 0; q < p; q++) w[q] = 1.0 / theta[q];
    const double wk = w[k];
    double *E = ws, *K = E + n * n, *Kd = K + n * n, *Kdd = Kd + n * n;
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) {
            double s = 0.0;
            for (int q = 0; q < p; q++) {
                const double t = XS[i * p + q] - XS[j * p + q];
                s = fma(t * t, w[q], s);
            }
            const double e = oexp(-s);
            const double tk = XS[i * p + k] - XS[j * p + k];
            const double a = (tk * tk) * wk;
            E[i * n + j] = e;
            K[i * n + j] = e + (i == j ? g : 0.0);
            Kd[i * n + j] = (e * a) * wk;
            Kdd[i * n + j] = (e * (a * a - 2.0 * a)) * (wk * wk);
        }
    return mle_eval_tail(n, y, ws, l, d1, d2);
}

typedef struct {
    int n, p, k;
    const double *XS, *y;
    double g;
    double *theta, *ws;
} sep_ctx;

static int sep_eval1(void *vp, double t, double *l, double *d1, double *d2)
{
    sep_ctx *c = (sep_ctx *)vp;
    const double keep = c->theta[c->k];
    c->theta[c->k] = t;
    const int r = sep_eval(c->n, c->p, c->XS, c->y, c->g, c->theta, c->k, c->ws, l, d1, d2);
    c->theta[c->k] = keep;
    return r;
}

/* theta: p starting values in, estimates out.  Returns the status flags
 * (ORC_STATUS_MLE_*), or -2 if out of memory. */
static int sep_fit(int n, int p, const double *XS, const double *y, double g, double *theta, double dmin,
                   double dmax, double tol, int maxit, int maxsweep, int *iters)
{
    double *ws = malloc(sizeof(double) * (8 * (size_t)n * n + 4 * (size_t)n));
    if (!ws) return -2;
    int flags = 0, total = 0, conv = 0;
    sep_ctx c = {n, p, 0, XS, y, g, theta, ws};
    for (int sweep = 0; sweep < maxsweep && !conv; sweep++) {
        int moved = 0;
        for (int k = 0; k < p; k++) {
            const double before = theta[k];
            int it, fl;
            c.k = k;
            const double t = newton_1d(sep_eval1, &c, before, dmin, dmax, tol, maxit, &it, &fl);
            theta[k] = t;
            total += it;
            flags |= fl & (ORC_STATUS_MLE_NOTPD | ORC_STATUS_MLE_MAXIT);
            if (fabs(t - before) > tol * before) moved = 1;
        }
        if (!moved) conv = 1;
    }
    if (!conv) flags |= ORC_STATUS_MLE_MAXIT;
    for (int k = 0; k < p; k++)
        if (theta[k] <= dmin * (1.0 + tol) || theta[k] >= dmax * (1.0 - tol)) flags |= ORC_STATUS_MLE_BOUND;
    *iters = total;
    free(ws);
    return flags;
}

/* ------------------------------------------------------------ exports --- */

/* Nearest candidates for M locations: idx (M x ncand row ids), d2 (M x ncand). */
int orc_knn(const double *X, int64_t N, int p, const double *XX, int64_t M, int ncand, int64_t *idx,
            double *d2, int nthreads)
{
    if (N < 1 || p < 1 || ncand < 1 || (int64_t)ncand > N || M < 0) return -1;
    int err = 0;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
    {
        nbr *heap = malloc(sizeof(nbr) * ncand);
        if (!heap) {
#pragma omp atomic write
            err = -2;
        }
#pragma omp for schedule(dynamic)
        for (int64_t m = 0; m < M; m++)
            if (heap) knn_one(X, N, p, XX + m * p, ncand, idx + m * ncand, d2 ? d2 + m * ncand : NULL, heap);
        free(heap);
    }
    return err;
}

/* Local GP prediction for M locations (OpenMP over locations, Sec. 5).
 * forced (nullable, M x n): follow these selections (replay).
 * Outputs mean/s2/df (M), sel (nullable, M x n), diag (nullable,
 * M x (n-n0) x ORC_NDIAG), status (M).  Returns 0, or -1 on bad arguments,
 * -2 on allocation failure. */
int orc_predict(const double *X, const double *y, int64_t N, int p, const double *XX, int64_t M, int n0,
                int n, int ncand, int search, int numrays, const double *d, int d_len, double g,
                int brent_maxit, double brent_tol, int scoring, const int32_t *forced, int nthreads,
                double *mean, double *s2, double *df, int32_t *sel, double *diag, int32_t *status)
{
    if (check_args(N, p, n0, n, ncand, search, numrays, d, d_len, g, scoring) != 0 || M < 0) return -1;
    double lo[16], hi[16], w[16];
    bbox(X, N, p, lo, hi);
    for (int k = 0; k < d_len; k++) w[k] = 1.0 / d[k];
    ctx_t c = {X, y, N, p, n0, n, ncand, search, numrays, w, d_len, g,
               brent_maxit > 0 ? brent_maxit : 100, brent_tol > 0.0 ? brent_tol : ldexp(1.0, -13), lo, hi,
               scoring};
    int nd = (search == 2) ? 0 : n - n0;
    int err = 0;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
    {
        scratch_t s;
        int ok = scratch_alloc(&s, n, ncand) == 0;
        if (!ok) {
#pragma omp atomic write
            err = -2;
        }
#pragma omp for schedule(dynamic)
        for (int64_t m = 0; m < M; m++) {
            if (!ok) continue;
            int st = local_one(&c, &s, XX + m * p, forced ? forced + m * n : NULL, mean + m, s2 + m, df + m,
                               sel ? sel + m * n : NULL, diag ? diag + (size_t)m * nd * ORC_NDIAG : NULL,
                               NULL, NULL);
            if (st < 0) {
#pragma omp atomic write
                err = st;
                st = 0x100;
            }
            if (status) status[m] = st;
        }
        scratch_free(&s);
    }
    return err;
}

/* One location with full traces for the brute-force checks: ALC of every
 * candidate at every step (exhaustive scoring is run in every search mode),
 * the final inverse, the candidate list and the per-step diagnostics. */
int orc_trace(const double *X, const double *y, int64_t N, int p, const double *x, int n0, int n, int ncand,
              int search, int numrays, const double *d, int d_len, double g, int brent_maxit,
              double brent_tol, int scoring, const int32_t *forced, double *mean, double *s2, double *df,
              int32_t *sel, double *diag, double *trace_alc, double *trace_Ki, int64_t *cand)
{
    if (check_args(N, p, n0, n, ncand, search, numrays, d, d_len, g, scoring) != 0) return -1;
    double lo[16], hi[16], w[16];
    bbox(X, N, p, lo, hi);
    for (int k = 0; k < d_len; k++) w[k] = 1.0 / d[k];
    ctx_t c = {X, y, N, p, n0, n, ncand, search, numrays, w, d_len, g,
               brent_maxit > 0 ? brent_maxit : 100, brent_tol > 0.0 ? brent_tol : ldexp(1.0, -13), lo, hi,
               scoring};
    scratch_t s;
    if (scratch_alloc(&s, n, ncand) != 0) return -2;
    int st = local_one(&c, &s, x, forced, mean, s2, df, sel, diag, trace_alc, trace_Ki);
    if (cand) memcpy(cand, s.cand, sizeof(int64_t) * ncand);
    scratch_free(&s);
    return st;
}

/* Local MLE prediction for M locations (mode 1: one stage, 2: two stages;
 * exhaustive search, isotropic d0 = d[0]; dmin, dmax, tol, maxit as mle_fit,
 * <= 0 for the defaults d0/1000, 100 d0, 1e-8, 100).  Outputs mean, s2, df,
 * dhat (the estimate used), iters (Newton evaluations), sel (M x n), status. */
int orc_predict_mle(const double *X, const double *y, int64_t N, int p, const double *XX, int64_t M, int n0, int n,
                    int ncand, int search, int numrays, double d0, double g, int brent_maxit, double brent_tol,
                    int scoring, int mode, double dmin, double dmax, double tol, int maxit, int nthreads,
                    double *mean, double *s2, double *df, int32_t *sel, double *dhat, int32_t *iters,
                    int32_t *status)
{
    if (check_args(N, p, n0, n, ncand, search, numrays, &d0, 1, g, scoring) != 0 || M < 0) return -1;
    if (mode < 1 || mode > 2) return -1;
    if (!(dmin > 0.0)) dmin = d0 / 1000.0;
    if (!(dmax > 0.0)) dmax = 100.0 * d0;
    if (!(tol > 0.0)) tol = 1e-8;
    if (maxit <= 0) maxit = 100;
    if (!(dmin < dmax)) return -1;
    double lo[16], hi[16], w0 = 1.0 / d0;
    bbox(X, N, p, lo, hi);
    ctx_t c = {X, y, N, p, n0, n, ncand, search, numrays, &w0, 1, g,
               brent_maxit > 0 ? brent_maxit : 100, brent_tol > 0.0 ? brent_tol : ldexp(1.0, -13), lo, hi,
               scoring};
    int err = 0;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
    {
        scratch_t s;
        int ok = scratch_alloc(&s, n, ncand) == 0;
        if (!ok) {
#pragma omp atomic write
            err = -2;
        }
#pragma omp for schedule(dynamic)
        for (int64_t m = 0; m < M; m++) {
            if (!ok) continue;
            int st = local_mle(&c, &s, XX + m * p, mode, dmin, dmax, tol, maxit, mean + m, s2 + m, df + m,
                               sel ? sel + m * n : NULL, dhat + m, iters + m);
            if (st < 0) {
#pragma omp atomic write
                err = st;
                st = 0x100;
            }
            status[m] = st;
        }
        scratch_free(&s);
    }
    return err;
}

/* The local log-likelihood and its first two derivatives at theta on the
 * design XJ (n x p), yJ (for direct checks).  Returns 0, or -1 if K is not
 * positive definite. */
int orc_mle_eval(int n, int p, const double *XJ, const double *yJ, double g, double theta, double *out3)
{
    double *D = malloc(sizeof(double) * n * n), *ws = malloc(sizeof(double) * (8 * n * n + 8 * n));
    int rc = -2;
    if (D && ws) {
        design_sqdist(n, p, XJ, D);
        rc = mle_eval(n, D, yJ, g, theta, ws, out3, out3 + 1, out3 + 2);
    }
    free(D);
    free(ws);
    return rc;
}

/* mle_fit on the design XJ, yJ. */
double orc_mle_fit(int n, int p, const double *XJ, const double *yJ, double g, double theta0, double dmin,
                   double dmax, double tol, int maxit, int *iters, int *flags)
{
    double *D = malloc(sizeof(double) * n * n), *ws = malloc(sizeof(double) * (8 * n * n + 8 * n));
    double t = NAN;
    if (D && ws) {
        design_sqdist(n, p, XJ, D);
        t = mle_fit(n, D, yJ, g, theta0, dmin, dmax, tol, maxit, ws, iters, flags);
    }
    free(D);
    free(ws);
    return t;
}

/* Exported for direct checks of the pieces. */
/* O9 exports: one evaluation (l, l', l'' in theta_k) and the global fit. */
int orc_sep_eval(int n, int p, const double *XS, const double *y, double g, const double *theta, int k,
                 double *out3)
{
    if (n < 1 || p < 1 || p > 16 || k < 0 || k >= p) return -2;
    double *ws = malloc(sizeof(double) * (8 * (size_t)n * n + 4 * (size_t)n));
    if (!ws) return -2;
    const int r = sep_eval(n, p, XS, y, g, theta, k, ws, out3, out3 + 1, out3 + 2);
    free(ws);
    return r;
}

int orc_sep_fit(int n, int p, const double *XS, const double *y, double g, double *theta, double dmin,
                double dmax, double tol, int maxit, int maxsweep, int *iters)
{
    if (n < 1 || p < 1 || p > 16 || !(dmin > 0.0) || !(dmin < dmax) || maxit < 1 || maxsweep < 1) return -1;
    return sep_fit(n, p, XS, y, g, theta, dmin, dmax, tol, maxit, maxsweep, iters);
}

double orc_exp(double x)
{
    return oexp(x);
}

double orc_kern(const double *a, const double *b, int p, const double *d, int d_len)
{
    double w[16];
    for (int k = 0; k < d_len && k < 16; k++) w[k] = 1.0 / d[k];
    return kern(a, b, p, w, d_len);
}

double orc_sqdist(const double *a, const double *b, int p)
{
    return sqdist(a, b, p);
}

int orc_spd_inverse(const double *A, int n, double *Ainv)
{
    double *work = malloc(sizeof(double) * 2 * n * n);
    if (!work) return -2;
    int r = spd_inverse(A, n, Ainv, work);
    free(work);
    return r;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
