/*
 * cde_oracle.c -- plain FP64 CPU oracle for the exact leave-one-out (LOO)
 * cross-validated log-likelihood of the double-kernel (Nadaraya-Watson)
 * conditional density estimator, its bandwidth gradient, and density queries.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the HIP library and is never a product path.
 *
 * Source: Holmes, Gray & Isbell, "Fast Nonparametric Conditional Density
 * Estimation".
 *   - Section 2: the scaled kernel K_h(t) = h^{-d} K(t/h); K here is the
 *     Gaussian, applied as a product over dimensions with one bandwidth per
 *     dimension (a scalar bandwidth is the same value in every dimension).
 *   - Section 2, eq. (1): f(y|x) = sum_i K_hy(y-y_i) K_hx(x-x_i) /
 *     sum_i K_hx(x-x_i).  (The paper's h1 is the y-bandwidth and h2 the
 *     x-bandwidth; this file writes hx and hy.)
 *   - Section 3, eq. (3) and its expansion in Section 3.2: for each point i,
 *     num_i = sum_{j!=i} K_hx(x_i-x_j) K_hy(y_i-y_j)  (the paper's A_i) and
 *     den_i = sum_{j!=i} K_hx(x_i-x_j).
 *       CONDITIONAL: l_i = log(num_i / den_i)  = log f^{-i}(y_i|x_i)
 *       JOINT      : l_i = log(num_i / (n-1)) = log f^{-i}(y_i|x_i) f^{-i}(x_i)
 *     and L = (1/n) sum_i l_i for JOINT is eq. (3).
 *
 * Evaluation (plain definition, no blocking, no factorisation): for each i,
 * in index order, form the Gaussian exponents a_j = -1/2 sum_k (dx_k/hx_k)^2
 * and b_j = -1/2 sum_l (dy_l/hy_l)^2 for every j != i, take the maxima
 * Mx = max_j a_j and Mxy = max_j (a_j + b_j), and sum the shifted
 * exponentials D = sum_j exp(a_j - Mx), U = sum_j exp(a_j + b_j - Mxy) in j
 * order (log-sum-exp: the common factor cancels in each ratio, so the value
 * is the plain definition without overflow or underflow).  Then
 *   CONDITIONAL: l_i = log c_y + (Mxy + log U) - (Mx + log D)
 *   JOINT      : l_i = log c_x + log c_y + Mxy + log U - log(n-1)
 * with log c_x = -sum_k (log hx_k + log(2 pi)/2) and likewise log c_y.
 *
 * Gradient with respect to the per-dimension bandwidths (differentiating
 * the Gaussian kernels of Section 2 under the ratio of eq. (1)):
 *   d l_i / d hx_k = (Mv_k/U - Mw_k/D) / hx_k^3           (CONDITIONAL)
 *                  = (Mv_k/U) / hx_k^3 - 1/hx_k           (JOINT)
 *   d l_i / d hy_l = (Mvy_l/U) / hy_l^3 - 1/hy_l          (both)
 * where Mw_k = sum_j exp(a_j-Mx) dx_k^2, Mv_k = sum_j exp(a_j+b_j-Mxy) dx_k^2
 * and Mvy_l = sum_j exp(a_j+b_j-Mxy) dy_l^2.
 *
 * Epanechnikov kernel (the kernel of the paper's experiments, Section 4),
 * radial over the bandwidth-scaled coordinates as in Section 2's K_h of a
 * norm: K_h(t) = c_d / prod_k h_k * max(0, 1 - sum_k (t_k/h_k)^2) with the
 * multivariate normalisation c_d = (d+2) / (2 V_d), V_d = pi^{d/2} /
 * Gamma(d/2 + 1) the volume of the unit d-ball (Silverman's multivariate
 * Epanechnikov kernel; c_1 = 3/4, c_2 = 2/pi).  With wx_j = max(0, 1 -
 * sum_k (dx_k/hx_k)^2) and wy_j likewise, D = sum_{j!=i} wx_j and U =
 * sum_{j!=i} wx_j wy_j in j order, and
 *   CONDITIONAL: l_i = log c_y + log U - log D
 *   JOINT      : l_i = log c_x + log c_y + log U - log(n-1)
 * with log c_x = log c_dx - sum_k log hx_k.  U = 0 (no j inside both
 * windows; the divergence of L at tiny bandwidths noted in Section 4.1) gives
 * l_i = -inf.
 *
 * Query-side products (Section 1 lists the expectation, modes and prediction
 * intervals as what a conditional density yields; Section 4.2 predicts y by
 * the expectation of f(y|x) and builds prediction intervals by searching for
 * the narrowest set of quantiles with the desired coverage):
 *   - conditional mean E[y|x] = sum_i K_hx(x-x_i) y_i / sum_i K_hx(x-x_i),
 *     the mean of eq. (1)'s density (Gaussian kernel; the y-kernel is
 *     symmetric, so each component's mean is y_i);
 *   - summary of a density f on an increasing y grid (dy = 1): mass = the
 *     trapezoid integral; mode = the first grid point of maximal f; the
 *     narrowest interval [lo, hi] holding 1 - alpha of the grid's CDF G
 *     (trapezoid partial sums over mass, linear between grid points), over
 *     the candidates with lo on a grid point (hi = G^-1(G(lo) + 1 - alpha))
 *     and then those with hi on a grid point (lo = G^-1(G(hi) - (1 - alpha))),
 *     the first of least width in that order (a later candidate replaces it
 *     only when narrower by more than 1e-12 of the grid's span, so ties do
 *     not depend on rounding).
 *
 * Cross-validated integrated squared error (Section 3, eq. (2) and the
 * cross-validated estimate that follows it, taken from Fan & Yim), Gaussian
 * product kernels: per point i
 *   T1_i = integral over y of f^{-i}(y|x_i)^2
 *        = sum_{j!=i} sum_{l!=i} w_j w_l G(y_j - y_l) / (sum_{j!=i} w_j)^2,
 *   T2_i = f^{-i}(y_i|x_i),
 * with w_j the x-kernel weights of eq. (1) and G the integral of the product
 * of two y-kernels centred at y_j and y_l, i.e. the Gaussian of standard
 * deviation sqrt(2) hy_l in each dimension:
 *   G(t) = prod_l exp(-(t_l / hy_l)^2 / 4) / (2 sqrt(pi) hy_l).
 * The estimate is ISE = (1/n) sum_i T1_i - (2/n) sum_i T2_i.  The double sum
 * over (j, l) makes the cost O(n^2) per point, O(n^3) in all.
 *
 * Threads: points i are split into contiguous ranges, one per thread; each
 * l_i is computed by exactly the same code whatever the split, so results are
 * bitwise independent of the thread count.  Totals are formed by the caller
 * with oracle_sum (index order, Neumaier-compensated).
 */
#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_COND 0
#define ORACLE_JOINT 1
#define ORACLE_GAUSSIAN 0
#define ORACLE_EPANECHNIKOV 1

static const double HALF_LOG_2PI = 0.91893853320467274178032973640562;
static const double PI = 3.14159265358979323846264338327950288;

typedef struct {
    const double* x;     /* [n][dx] */
    const double* y;     /* [n][dy] */
    long n;
    int dx, dy;
    const double* h;     /* [dx+dy]: hx..., hy... */
    int criterion;
    int kernel;          /* ORACLE_GAUSSIAN or ORACLE_EPANECHNIKOV */
    const long* idx;     /* points to evaluate, or NULL for 0..m-1 */
    long m;
    double* ell;         /* [m] */
    double* dell;        /* [m][dx+dy] or NULL */
    long lo, hi;         /* this worker's range of [0, m) */
    int status;
} loo_job;

static double log_norm(const double* h, int d)
{
    double s = 0.0;
    for (int k = 0; k < d; ++k) s -= log(h[k]) + HALF_LOG_2PI;
    return s;
}

/* One point i: fills *ell and, if grad != NULL, grad[0..dx+dy). */
static int loo_point(const loo_job* J, long i, double* a, double* ab,
                     double* ell, double* grad)
{
    const long n = J->n;
    const int dx = J->dx, dy = J->dy;
    const double* hx = J->h;
    const double* hy = J->h + dx;
    const double* xi = J->x + (size_t)i * dx;
    const double* yi = J->y + (size_t)i * dy;
    double Mx = -INFINITY, Mxy = -INFINITY;

    for (long j = 0; j < n; ++j) {
        if (j == i) continue;           /* leave point i out (eq. 3) */
        const double* xj = J->x + (size_t)j * dx;
        const double* yj = J->y + (size_t)j * dy;
        double sx = 0.0, sy = 0.0;
        for (int k = 0; k < dx; ++k) {
            double t = (xi[k] - xj[k]) / hx[k];
            sx += t * t;
        }
        for (int l = 0; l < dy; ++l) {
            double t = (yi[l] - yj[l]) / hy[l];
            sy += t * t;
        }
        a[j] = -0.5 * sx;
        ab[j] = -0.5 * sx - 0.5 * sy;
        if (a[j] > Mx) Mx = a[j];
        if (ab[j] > Mxy) Mxy = ab[j];
    }

    /* a[j] and ab[j] now become the shifted weights exp(a_j - Mx) and
     * exp(a_j + b_j - Mxy); D and U are their sums in j order. */
    double D = 0.0, U = 0.0;
    for (long j = 0; j < n; ++j) {
        if (j == i) continue;
        a[j] = exp(a[j] - Mx);
        ab[j] = exp(ab[j] - Mxy);
        D += a[j];
        U += ab[j];
    }

    const double lcx = log_norm(hx, dx);
    const double lcy = log_norm(hy, dy);
    if (J->criterion == ORACLE_JOINT)
        *ell = lcx + lcy + Mxy + log(U) - log((double)(n - 1));
    else
        *ell = lcy + (Mxy + log(U)) - (Mx + log(D));

    if (grad) {
        for (int k = 0; k < dx; ++k) {
            double mw = 0.0, mv = 0.0;
            for (long j = 0; j < n; ++j) {
                if (j == i) continue;
                double d = xi[k] - J->x[(size_t)j * dx + k];
                mw += a[j] * d * d;
                mv += ab[j] * d * d;
            }
            double h3 = hx[k] * hx[k] * hx[k];
            if (J->criterion == ORACLE_JOINT)
                grad[k] = (mv / U) / h3 - 1.0 / hx[k];
            else
                grad[k] = (mv / U - mw / D) / h3;
        }
        for (int l = 0; l < dy; ++l) {
            double mvy = 0.0;
            for (long j = 0; j < n; ++j) {
                if (j == i) continue;
                double d = yi[l] - J->y[(size_t)j * dy + l];
                mvy += ab[j] * d * d;
            }
            double h3 = hy[l] * hy[l] * hy[l];
            grad[dx + l] = (mvy / U) / h3 - 1.0 / hy[l];
        }
    }
    return 0;
}

/* log of the multivariate Epanechnikov kernel's normalisation for
 * bandwidths h[0..d): log((d+2) / (2 V_d)) - sum_k log h_k. */
static double log_norm_epan(const double* h, int d)
{
    const double log_vd = 0.5 * d * log(PI) - lgamma(0.5 * d + 1.0);
    double s = log((d + 2.0) / 2.0) - log_vd;
    for (int k = 0; k < d; ++k) s -= log(h[k]);
    return s;
}

/* One point i with the Epanechnikov kernel: fills *ell. */
static int loo_point_epan(const loo_job* J, long i, double* ell)
{
    const long n = J->n;
    const int dx = J->dx, dy = J->dy;
    const double* hx = J->h;
    const double* hy = J->h + dx;
    const double* xi = J->x + (size_t)i * dx;
    const double* yi = J->y + (size_t)i * dy;
    double D = 0.0, U = 0.0;
    for (long j = 0; j < n; ++j) {
        if (j == i) continue;           /* leave point i out (eq. 3) */
        const double* xj = J->x + (size_t)j * dx;
        const double* yj = J->y + (size_t)j * dy;
        double sx = 0.0, sy = 0.0;
        for (int k = 0; k < dx; ++k) {
            double t = (xi[k] - xj[k]) / hx[k];
            sx += t * t;
        }
        for (int l = 0; l < dy; ++l) {
            double t = (yi[l] - yj[l]) / hy[l];
            sy += t * t;
        }
        const double wx = sx < 1.0 ? 1.0 - sx : 0.0;
        const double wy = sy < 1.0 ? 1.0 - sy : 0.0;
        D += wx;
        U += wx * wy;
    }
    const double lcy = log_norm_epan(hy, dy);
    if (!(U > 0.0))
        *ell = -INFINITY;
    else if (J->criterion == ORACLE_JOINT)
        *ell = log_norm_epan(hx, dx) + lcy + log(U) - log((double)(n - 1));
    else
        *ell = lcy + log(U) - log(D);
    return 0;
}

static void* loo_worker(void* arg)
{
    loo_job* J = (loo_job*)arg;
    double* a = (double*)malloc(sizeof(double) * (size_t)J->n);
    double* ab = (double*)malloc(sizeof(double) * (size_t)J->n);
    if (!a || !ab) {
        free(a);
        free(ab);
        J->status = 2;
        return NULL;
    }
    const int p = J->dx + J->dy;
    for (long t = J->lo; t < J->hi; ++t) {
        long i = J->idx ? J->idx[t] : t;
        if (J->kernel == ORACLE_EPANECHNIKOV)
            loo_point_epan(J, i, &J->ell[t]);
        else
            loo_point(J, i, a, ab, &J->ell[t], J->dell ? J->dell + (size_t)t * p : NULL);
    }
    free(a);
    free(ab);
    J->status = 0;
    return NULL;
}

static int check_args(const double* x, const double* y, long n, int dx, int dy,
                      const double* h)
{
    if (!x || !y || !h || n < 2 || dx < 1 || dy < 1) return 1;
    for (int k = 0; k < dx + dy; ++k)
        if (!(h[k] > 0.0) || !isfinite(h[k])) return 1;
    return 0;
}

static int run_jobs_with(loo_job* base, long m, int nthreads, void* (*worker)(void*))
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > m) nthreads = (int)(m > 0 ? m : 1);
    loo_job* jobs = (loo_job*)calloc((size_t)nthreads, sizeof(loo_job));
    pthread_t* th = (pthread_t*)calloc((size_t)nthreads, sizeof(pthread_t));
    if (!jobs || !th) {
        free(jobs);
        free(th);
        return 2;
    }
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = *base;
        jobs[t].lo = m * t / nthreads;
        jobs[t].hi = m * (t + 1) / nthreads;
        jobs[t].status = 0;
    }
    int status = 0;
    if (nthreads == 1) {
        worker(&jobs[0]);
        status = jobs[0].status;
    } else {
        for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, worker, &jobs[t]);
        for (int t = 0; t < nthreads; ++t) {
            pthread_join(th[t], NULL);
            if (jobs[t].status) status = jobs[t].status;
        }
    }
    free(jobs);
    free(th);
    return status;
}

static int run_jobs(loo_job* base, long m, int nthreads)
{
    return run_jobs_with(base, m, nthreads, loo_worker);
}

/* One point i of the cross-validated ISE: *t1 = T1_i, *t2 = T2_i (see the
 * file header).  w[] is scratch of n doubles. */
static void ise_point(const loo_job* J, long i, double* w, double* t1, double* t2)
{
    const long n = J->n;
    const int dx = J->dx, dy = J->dy;
    const double* hx = J->h;
    const double* hy = J->h + dx;
    const double* xi = J->x + (size_t)i * dx;
    const double* yi = J->y + (size_t)i * dy;
    /* x-kernel exponents, shifted by their maximum (cancels in both ratios) */
    double Mx = -INFINITY;
    for (long j = 0; j < n; ++j) {
        if (j == i) continue;
        const double* xj = J->x + (size_t)j * dx;
        double sx = 0.0;
        for (int k = 0; k < dx; ++k) {
            double t = (xi[k] - xj[k]) / hx[k];
            sx += t * t;
        }
        w[j] = -0.5 * sx;
        if (w[j] > Mx) Mx = w[j];
    }
    double W = 0.0;
    for (long j = 0; j < n; ++j) {
        if (j == i) continue;
        w[j] = exp(w[j] - Mx);
        W += w[j];
    }
    /* T2: the LOO conditional density at the point itself */
    const double cy = exp(log_norm(hy, dy));
    double num = 0.0;
    for (long j = 0; j < n; ++j) {
        if (j == i) continue;
        const double* yj = J->y + (size_t)j * dy;
        double sy = 0.0;
        for (int l = 0; l < dy; ++l) {
            double t = (yi[l] - yj[l]) / hy[l];
            sy += t * t;
        }
        num += w[j] * exp(-0.5 * sy);
    }
    *t2 = cy * num / W;
    /* T1: the double sum over j != i and l != i */
    double cg = 1.0;
    for (int l = 0; l < dy; ++l) cg /= 2.0 * sqrt(PI) * hy[l];
    double Q = 0.0;
    for (long j = 0; j < n; ++j) {
        if (j == i) continue;
        const double* yj = J->y + (size_t)j * dy;
        double inner = 0.0;
        for (long l = 0; l < n; ++l) {
            if (l == i) continue;
            const double* yl = J->y + (size_t)l * dy;
            double s = 0.0;
            for (int d = 0; d < dy; ++d) {
                double t = (yj[d] - yl[d]) / hy[d];
                s += t * t;
            }
            inner += w[l] * exp(-0.25 * s);
        }
        Q += w[j] * inner;
    }
    *t1 = cg * Q / (W * W);
}

static void* ise_worker(void* arg)
{
    loo_job* J = (loo_job*)arg;
    double* w = (double*)malloc(sizeof(double) * (size_t)J->n);
    if (!w) {
        J->status = 2;
        return NULL;
    }
    for (long t = J->lo; t < J->hi; ++t) {
        long i = J->idx ? J->idx[t] : t;
        ise_point(J, i, w, &J->ell[t], &J->dell[t]);
    }
    free(w);
    J->status = 0;
    return NULL;
}

/* Per-point terms of the cross-validated ISE for one diagonal setting
 * h[dx+dy] (Gaussian kernels): t1[t] = T1_i, t2[t] = T2_i for i = idx[t]
 * (idx == NULL: i = 0..m-1, m == n).  Returns 0 on success, 1 on invalid
 * arguments, 2 on allocation failure. */
int oracle_cv_ise(const double* x, const double* y, long n, int dx, int dy,
                  const double* h, const long* idx, long m, double* t1, double* t2,
                  int nthreads)
{
    if (check_args(x, y, n, dx, dy, h) || !t1 || !t2 || m < 0) return 1;
    if (!idx && m != n) return 1;
    if (idx)
        for (long t = 0; t < m; ++t)
            if (idx[t] < 0 || idx[t] >= n) return 1;
    loo_job J;
    memset(&J, 0, sizeof J);
    J.x = x; J.y = y; J.n = n; J.dx = dx; J.dy = dy; J.h = h;
    J.idx = idx; J.m = m; J.ell = t1; J.dell = t2;
    return run_jobs_with(&J, m, nthreads, ise_worker);
}

/* Per-point LOO log-likelihood (and optionally its bandwidth gradient) for
 * one diagonal bandwidth setting h[dx+dy].  idx selects the points i that are
 * evaluated (each against all j != i); idx == NULL means i = 0..m-1 (m == n).
 * Returns 0 on success, 1 on invalid arguments, 2 on allocation failure. */
int oracle_loo(const double* x, const double* y, long n, int dx, int dy,
               const double* h, int criterion, const long* idx, long m,
               double* ell, double* dell, int nthreads)
{
    if (check_args(x, y, n, dx, dy, h) || !ell || m < 0) return 1;
    if (!idx && m != n) return 1;
    if (idx)
        for (long t = 0; t < m; ++t)
            if (idx[t] < 0 || idx[t] >= n) return 1;
    loo_job J;
    memset(&J, 0, sizeof J);
    J.x = x; J.y = y; J.n = n; J.dx = dx; J.dy = dy; J.h = h;
    J.criterion = criterion; J.idx = idx; J.m = m; J.ell = ell; J.dell = dell;
    return run_jobs(&J, m, nthreads);
}

/* Per-point LOO log-likelihood with the Epanechnikov kernel for one diagonal
 * bandwidth setting h[dx+dy] (values only); arguments as oracle_loo. */
int oracle_loo_epan(const double* x, const double* y, long n, int dx, int dy,
                    const double* h, int criterion, const long* idx, long m,
                    double* ell, int nthreads)
{
    if (check_args(x, y, n, dx, dy, h) || !ell || m < 0) return 1;
    if (!idx && m != n) return 1;
    if (idx)
        for (long t = 0; t < m; ++t)
            if (idx[t] < 0 || idx[t] >= n) return 1;
    loo_job J;
    memset(&J, 0, sizeof J);
    J.x = x; J.y = y; J.n = n; J.dx = dx; J.dy = dy; J.h = h;
    J.criterion = criterion; J.kernel = ORACLE_EPANECHNIKOV;
    J.idx = idx; J.m = m; J.ell = ell; J.dell = NULL;
    return run_jobs(&J, m, nthreads);
}

/* Scalar bandwidth grid, evaluated directly setting by setting: for every
 * (a, b) the exponent of each pair is formed from hx[a] and hy[b] and
 * exponentiated as a whole (no factorisation of the two kernels).  Output is
 * hx-major: ell[(a*nhy + b)*m + t]. */
int oracle_loo_grid(const double* x, const double* y, long n, int dx, int dy,
                    const double* hx, int nhx, const double* hy, int nhy,
                    int criterion, const long* idx, long m, double* ell,
                    int nthreads)
{
    if (!hx || !hy || nhx < 1 || nhy < 1 || dx + dy > 256) return 1;
    double h[256];
    for (int a = 0; a < nhx; ++a) {
        for (int b = 0; b < nhy; ++b) {
            for (int k = 0; k < dx; ++k) h[k] = hx[a];
            for (int l = 0; l < dy; ++l) h[dx + l] = hy[b];
            int s = oracle_loo(x, y, n, dx, dy, h, criterion, idx, m,
                               ell + ((size_t)a * nhy + b) * (size_t)m, NULL, nthreads);
            if (s) return s;
        }
    }
    return 0;
}

/* Sum in index order with Neumaier's compensation.  A non-finite entry
 * makes the plain sum the answer (-inf for a diverged point, NaN for NaN). */
double oracle_sum(const double* v, long m)
{
    double p = 0.0;
    for (long t = 0; t < m; ++t) p += v[t];
    if (!isfinite(p)) return p;
    double s = 0.0, c = 0.0;
    for (long t = 0; t < m; ++t) {
        double u = s + v[t];
        if (fabs(s) >= fabs(v[t]))
            c += (s - u) + v[t];
        else
            c += (v[t] - u) + s;
        s = u;
    }
    return s + c;
}

typedef struct {
    const double *x, *y, *h, *xq, *yg;
    long n, q, k;
    int dx, dy;
    double* f;
    long lo, hi;
    int status;
} dens_job;

static void* dens_worker(void* arg)
{
    dens_job* J = (dens_job*)arg;
    const long n = J->n;
    const int dx = J->dx, dy = J->dy;
    const double* hx = J->h;
    const double* hy = J->h + dx;
    double* a = (double*)malloc(sizeof(double) * (size_t)n);
    double* ab = (double*)malloc(sizeof(double) * (size_t)n);
    if (!a || !ab) {
        free(a);
        free(ab);
        J->status = 2;
        return NULL;
    }
    const double lcy = log_norm(hy, dy);
    for (long qq = J->lo; qq < J->hi; ++qq) {
        const double* xq = J->xq + (size_t)qq * dx;
        double Mx = -INFINITY;
        for (long i = 0; i < n; ++i) {
            double sx = 0.0;
            for (int k = 0; k < dx; ++k) {
                double t = (xq[k] - J->x[(size_t)i * dx + k]) / hx[k];
                sx += t * t;
            }
            a[i] = -0.5 * sx;
            if (a[i] > Mx) Mx = a[i];
        }
        double D = 0.0;
        for (long i = 0; i < n; ++i) D += exp(a[i] - Mx);
        for (long g = 0; g < J->k; ++g) {
            const double* yg = J->yg + (size_t)g * dy;
            double Mxy = -INFINITY;
            for (long i = 0; i < n; ++i) {
                double sy = 0.0;
                for (int l = 0; l < dy; ++l) {
                    double t = (yg[l] - J->y[(size_t)i * dy + l]) / hy[l];
                    sy += t * t;
                }
                ab[i] = a[i] - 0.5 * sy;
                if (ab[i] > Mxy) Mxy = ab[i];
            }
            double U = 0.0;
            for (long i = 0; i < n; ++i) U += exp(ab[i] - Mxy);
            J->f[(size_t)qq * J->k + g] = exp(lcy + (Mxy + log(U)) - (Mx + log(D)));
        }
    }
    free(a);
    free(ab);
    J->status = 0;
    return NULL;
}

/* Density queries, eq. (1) over all n training points (no point left out):
 * f[qq][g] = f(yg[g] | xq[qq]) for q query x's and k y values. */
int oracle_density(const double* x, const double* y, long n, int dx, int dy,
                   const double* h, const double* xq, long q, const double* yg,
                   long k, double* f, int nthreads)
{
    if (check_args(x, y, n, dx, dy, h) || !xq || !yg || !f || q < 0 || k < 0) return 1;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > q) nthreads = (int)(q > 0 ? q : 1);
    dens_job* jobs = (dens_job*)calloc((size_t)nthreads, sizeof(dens_job));
    pthread_t* th = (pthread_t*)calloc((size_t)nthreads, sizeof(pthread_t));
    if (!jobs || !th) {
        free(jobs);
        free(th);
        return 2;
    }
    for (int t = 0; t < nthreads; ++t) {
        dens_job J = {x, y, h, xq, yg, n, q, k, dx, dy, f, q * t / nthreads,
                      q * (t + 1) / nthreads, 0};
        jobs[t] = J;
    }
    for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, dens_worker, &jobs[t]);
    int status = 0;
    for (int t = 0; t < nthreads; ++t) {
        pthread_join(th[t], NULL);
        if (jobs[t].status) status = jobs[t].status;
    }
    free(jobs);
    free(th);
    return status;
}

/* Density queries with the Epanechnikov kernel, eq. (1) over all n training
 * points: f[qq][g] = c_y sum_i wx wy / sum_i wx (0 where no training x lies
 * inside the x window, i.e. where eq. (1) is 0/0). */
int oracle_density_epan(const double* x, const double* y, long n, int dx, int dy,
                        const double* h, const double* xq, long q, const double* yg,
                        long k, double* f)
{
    if (check_args(x, y, n, dx, dy, h) || !xq || !yg || !f || q < 0 || k < 0) return 1;
    const double* hx = h;
    const double* hy = h + dx;
    const double cy = exp(log_norm_epan(hy, dy));
    for (long qq = 0; qq < q; ++qq) {
        for (long g = 0; g < k; ++g) {
            double D = 0.0, U = 0.0;
            for (long i = 0; i < n; ++i) {
                double sx = 0.0, sy = 0.0;
                for (int kk = 0; kk < dx; ++kk) {
                    double t = (xq[(size_t)qq * dx + kk] - x[(size_t)i * dx + kk]) / hx[kk];
                    sx += t * t;
                }
                for (int l = 0; l < dy; ++l) {
                    double t = (yg[(size_t)g * dy + l] - y[(size_t)i * dy + l]) / hy[l];
                    sy += t * t;
                }
                const double wx = sx < 1.0 ? 1.0 - sx : 0.0;
                const double wy = sy < 1.0 ? 1.0 - sy : 0.0;
                D += wx;
                U += wx * wy;
            }
            f[(size_t)qq * k + g] = D > 0.0 ? cy * U / D : 0.0;
        }
    }
    return 0;
}

/* Conditional mean (Gaussian kernel): mean[qq][l] = sum_i w_i y_il / sum_i w_i
 * with w_i = exp(-1/2 sum_k ((xq_k - x_ik)/hx_k)^2), shifted by the largest
 * exponent (the common factor cancels in the ratio).  h holds hx in its first
 * dx entries (the y bandwidth does not enter the mean). */
int oracle_cond_mean(const double* x, const double* y, long n, int dx, int dy,
                     const double* h, const double* xq, long q, double* mean)
{
    if (check_args(x, y, n, dx, dy, h) || !xq || !mean || q < 0) return 1;
    double* a = (double*)malloc(sizeof(double) * (size_t)n);
    if (!a) return 2;
    for (long qq = 0; qq < q; ++qq) {
        double M = -INFINITY;
        for (long i = 0; i < n; ++i) {
            double s = 0.0;
            for (int k = 0; k < dx; ++k) {
                double t = (xq[(size_t)qq * dx + k] - x[(size_t)i * dx + k]) / h[k];
                s += t * t;
            }
            a[i] = -0.5 * s;
            if (a[i] > M) M = a[i];
        }
        for (int l = 0; l < dy; ++l) {
            double D = 0.0, S = 0.0;
            for (long i = 0; i < n; ++i) {
                const double w = exp(a[i] - M);
                D += w;
                S += w * y[(size_t)i * dy + l];
            }
            mean[(size_t)qq * dy + l] = S / D;
        }
    }
    free(a);
    return 0;
}

/* Smallest y on the grid's piecewise-linear CDF with G(y) >= p (0 <= p <= 1),
 * G[0..k) non-decreasing with G[0] = 0. */
static double grid_inverse(const double* G, const double* yg, long k, double p)
{
    long g = 0;
    while (g < k - 1 && G[g] < p) ++g;
    if (g == 0 || G[g] <= G[g - 1]) return yg[g];
    return yg[g - 1] + (p - G[g - 1]) / (G[g] - G[g - 1]) * (yg[g] - yg[g - 1]);
}

/* Summary of each row of f[q][k] on the increasing grid yg[k] (k >= 2):
 * out[qq][0..4) = mass, mode, lo, hi as described in the header.  A row of
 * zero mass gives mass 0, mode yg[0] and lo = hi = NaN. */
int oracle_density_summary(const double* f, const double* yg, long q, long k, double alpha,
                           double* out)
{
    if (!f || !yg || !out || q < 0 || k < 2 || !(alpha > 0.0) || !(alpha < 1.0)) return 1;
    double* G = (double*)malloc(sizeof(double) * (size_t)k);
    if (!G) return 2;
    for (long qq = 0; qq < q; ++qq) {
        const double* r = f + (size_t)qq * k;
        double* o = out + (size_t)qq * 4;
        double c = 0.0;
        G[0] = 0.0;
        for (long g = 0; g + 1 < k; ++g) {
            c += (r[g] + r[g + 1]) * 0.5 * (yg[g + 1] - yg[g]);
            G[g + 1] = c;
        }
        const double mass = c;
        long imax = 0;
        for (long g = 1; g < k; ++g)
            if (r[g] > r[imax]) imax = g;
        o[0] = mass;
        o[1] = yg[imax];
        if (!(mass > 0.0)) {
            o[2] = o[3] = NAN;
            continue;
        }
        for (long g = 0; g < k; ++g) G[g] = G[g] / mass;
        const double cover = 1.0 - alpha;
        const double tie = 1e-12 * (yg[k - 1] - yg[0]);
        double best = INFINITY, blo = NAN, bhi = NAN;
        for (long g = 0; g < k; ++g) {          /* lo on a grid point */
            const double p = G[g] + cover;
            if (p > 1.0) break;
            const double hi = grid_inverse(G, yg, k, p);
            if (hi - yg[g] < best - tie) { best = hi - yg[g]; blo = yg[g]; bhi = hi; }
        }
        for (long g = 0; g < k; ++g) {          /* hi on a grid point */
            const double p = G[g] - cover;
            if (p < 0.0) continue;
            const double lo = grid_inverse(G, yg, k, p);
            if (yg[g] - lo < best - tie) { best = yg[g] - lo; blo = lo; bhi = yg[g]; }
        }
        o[2] = blo;
        o[3] = bhi;
    }
    free(G);
    return 0;
}
