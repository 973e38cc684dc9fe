/*
 * cde.h -- C ABI of the MI355X (gfx950) library for the exact leave-one-out
 * (LOO) cross-validated log-likelihood of the double-kernel (Nadaraya-Watson)
 * conditional density estimator, its bandwidth gradient, and density queries.
 *
 * Method: Holmes, Gray & Isbell, "Fast Nonparametric Conditional Density
 * Estimation".
 *   - Kernel (Section 2): K_h(t) = h^{-d} K(t/h).  K is the Gaussian, used
 *     as a product over dimensions with one bandwidth per dimension, or the
 *     Epanechnikov kernel of the paper's experiments (Section 4), radial over
 *     the bandwidth-scaled coordinates: c_d (1 - |t/h|^2)_+ / prod h with
 *     c_d = (d+2) / (2 V_d), V_d the volume of the unit d-ball.
 *   - Estimator (Section 2, eq. 1): f(y|x) = sum_i K_hy(y-y_i) K_hx(x-x_i) /
 *     sum_i K_hx(x-x_i).  The paper calls the y-bandwidth h1 and the
 *     x-bandwidth h2; this header writes hx and hy.
 *   - Criterion (Section 3, eq. 3 and the A_i expansion of Section 3.2):
 *     num_i = sum_{j!=i} K_hx(x_i-x_j) K_hy(y_i-y_j), den_i = sum_{j!=i}
 *     K_hx(x_i-x_j);
 *       CDE_COND : S = sum_i log(num_i / den_i)      (log f^{-i}(y_i|x_i))
 *       CDE_JOINT: S = sum_i log(num_i / (n - 1))    (n * L of eq. 3)
 *     The exact O(n^2) sum is evaluated (the paper's "naive" evaluation in
 *     Section 3); no pruning or sampling approximation is applied.
 *
 * Conventions for every call:
 *   - Device pointers are HIP device memory (e.g. torch tensors' data_ptr).
 *     Host pointers (bandwidth arrays) are read during the call only.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls only enqueue work on `stream`; outputs are valid once the stream
 *     has passed the call.  Calls on one model share that model's device
 *     scratch, so they must not overlap in time: issue them on one stream (or
 *     order them across streams with events).  Different models may run
 *     concurrently on different streams.  A call that needs more scratch
 *     than the model holds frees and reallocates it, which synchronises the
 *     device.
 *   - Outputs are caller-owned device buffers.
 *   - Errors are reported by status code only; no exception crosses the ABI.
 *     After a non-OK status, cde_last_error() returns a message (per thread).
 *   - Results are deterministic: fixed reduction orders, no float atomics on
 *     result paths, so repeated calls give identical bits.
 *   - Bandwidths: every h must be finite and > 0 (else CDE_EINVAL) and inside
 *     the range the kernels' arithmetic represents for the model's data
 *     (else CDE_EUNSUPPORTED, with a message).  With range_k = max_i x_ik -
 *     min_i x_ik the extent of dimension k, c_k = log2(e) / (2 h_k^2), and
 *     X, Y = sum_k range_k^2 c_k over the x and over the y dimensions (the
 *     largest exponent a pair can have):
 *       every call:   each c_k <= 2^59, X <= 2^100 and Y <= 2^100 (FP32
 *                     models; 2^900 for all three on FP64 models);
 *       calls on the diagonal pass (cde_loo_grad, cde_loo_grad_noalloc,
 *       cde_loo_loglik_list with the Gaussian kernel, cde_cv_ise, and the
 *       Gaussian cde_loo_loglik and cde_density_query of FP64 models), whose
 *       exponents are formed in the model's precision relative to a
 *       per-point reference: also (X + Y)(dx + dy + 2) <= 2^29 (FP32 models;
 *       2^61 on FP64 models).
 *     These bounds rule out overflow (inf, NaN), not rounding: far below
 *     them, the diagonal pass's FP32 exponents still carry an absolute error
 *     of about (dx + dy + 2) u times the nearest neighbour's exponent
 *     d_nn^2 c.  cde_check_bandwidths applies the same test on the host.
 *     Training data must be finite: a model whose data hold a NaN or an
 *     infinity rejects every call with CDE_EINVAL.  The extent is computed
 *     by cde_create on its stream; the model's first call that checks
 *     bandwidths waits for that work to finish.
 */
#ifndef CDE_H
#define CDE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CDE_ABI_VERSION 4

typedef struct cde_model cde_model; /* opaque handle */

typedef enum {
    CDE_GAUSSIAN = 0,     /* product Gaussian, one bandwidth per dimension */
    CDE_EPANECHNIKOV = 1  /* radial Epanechnikov over scaled coordinates (Section 4's
                             kernel); exactly zero outside its window, so a point
                             with no j inside both windows has l_i = -inf, the
                             divergence at tiny bandwidths Section 4.1 notes */
} cde_kernel;

typedef enum {
    CDE_OK = 0,
    CDE_EINVAL = 1,       /* bad argument: null pointer, n < 2, h <= 0 or non-finite, ... */
    CDE_ENOMEM = 2,       /* device allocation failed */
    CDE_EDEVICE = 3,      /* a HIP runtime call or kernel launch failed */
    CDE_EUNSUPPORTED = 4  /* valid but outside what the library supports: dx > 64, dy > 4, ... */
} cde_status;

typedef enum {
    CDE_F32 = 0, /* FP32 data and kernel values, compensated tile sums, FP64 log and reduce */
    CDE_F64 = 1  /* FP64 throughout */
} cde_precision;

typedef enum {
    CDE_COND = 0, /* sum_i log(num_i / den_i): the conditional LOO log-likelihood */
    CDE_JOINT = 1 /* sum_i log(num_i / (n-1)): eq. (3) times n */
} cde_criterion;

/* How the grid pass (cde_loo_loglik on FP32 models) forms the squared
 * x-distances ||x_i - x_j||^2 of Section 2's kernel argument. */
typedef enum {
    CDE_XTERM_AUTO = 0,       /* library choice: CDE_XTERM_VALU */
    CDE_XTERM_VALU = 1,       /* FP64 differences of the FP32 coordinates on the VALU (exact
                                 differences, FP64 squares and sums); the parity path */
    CDE_XTERM_MFMA_BF16X3 = 2,/* dx = 16: |u_i|^2 + |u_j|^2 - 2 u_i.u_j on mean-centred
                                 coordinates u, the cross term from a split-bf16 x3 MFMA
                                 product (hi.hi + hi.lo + lo.hi, FP32 accumulate), in the
                                 FP32 pass and in the FP64 rerun of flagged points; an
                                 approximation whose error the tests bound at its measured
                                 size, above the parity tolerance */
    CDE_XTERM_VALU_F32 = 3    /* dx = 16: the differences, squares, sums and neighbour shift in
                                 FP32 on the VALU, in the FP32 pass (flagged points are rerun
                                 with FP64 differences); an approximation, bounded like the
                                 above */
} cde_xterm;

/* ABI version of the loaded library (CDE_ABI_VERSION at build time). */
int cde_abi_version(void);

/* Message for the last non-OK status returned on the calling thread. */
const char* cde_last_error(void);

/* Create a model from a training set {(x_i, y_i)}, i < n (Section 2 data).
 *   x_dev: [n][dx] row-major, y_dev: [n][dy] row-major, device memory, of
 *          float (CDE_F32) or double (CDE_F64).  The values handed in ARE the
 *          dataset: nothing is re-rounded or re-centred.
 *   The model copies the data into its own device memory (structure-of-arrays,
 *   padded to a whole number of 256-point tiles) on `stream`; the caller may
 *   free x_dev / y_dev once the stream has passed this call.
 *   Limits: n >= 2, 1 <= dx <= 64, 1 <= dy <= 4, n < 2^31.
 *   The model owns its device memory until cde_destroy.  */
cde_status cde_create(cde_model** out, const void* x_dev, const void* y_dev, int64_t n,
                      int32_t dx, int32_t dy, cde_precision precision, void* stream);

/* Release a model made by cde_create (the training set of Section 2 held on
 * the device) and all of its device and pinned host memory.  Frees
 * synchronise the device, so no call on the model may still be running on
 * any stream.  NULL is accepted (CDE_OK).  Returns CDE_EDEVICE if a HIP
 * release call fails; the handle is invalid afterwards either way. */
cde_status cde_destroy(cde_model* m);

/* Device bytes the model holds now: the packed training set of Section 2
 * (with its extent record), per-point shifts, the spatial index and the
 * per-call scratch of the criterion of Section 3, which grows to the largest
 * call so far and is kept.  Host-only; 0 for NULL.  A serving admission
 * controller budgets HBM with it. */
size_t cde_model_device_bytes(const cde_model* m);

/* Host-only form of the bandwidth range test of the model calls (see
 * "Bandwidths" above) for one diagonal setting of the Gaussian kernel of
 * Section 2: range [dx+dy] are the data's per-dimension extents (max - min,
 * finite, >= 0), h [dx+dy] the bandwidths (hx_1..hx_dx, hy_1..hy_dy);
 * diagonal_pass != 0 adds the diagonal pass's rule.
 * Returns CDE_OK, CDE_EINVAL (NULL pointer, dx or dy < 1, dx + dy > 18,
 * non-finite or negative range, h not finite and > 0) or CDE_EUNSUPPORTED
 * (outside the representable range of `precision`).  No device is used. */
cde_status cde_check_bandwidths(const double* range, int32_t dx, int32_t dy, const double* h,
                                cde_precision precision, int32_t diagonal_pass);

/* Device bytes a model of this shape holds after cde_create and one
 * cde_loo_loglik call over an n_hx x n_hy grid (Gaussian kernel, default cross term)
 * (n_hx = n_hy = 0: after cde_create alone), i.e. what cde_model_device_bytes
 * then reports: the budget a caller (such as an admission controller) needs
 * for such a bandwidth-selection job (Section 3 criterion over a grid).
 * Host-only arithmetic; it reads the current device's compute-unit count.
 * Returns 0 for shapes or grid sizes cde_create or cde_loo_loglik reject.  */
size_t cde_workspace_bytes(int64_t n, int32_t dx, int32_t dy, cde_precision precision,
                           int32_t n_hx, int32_t n_hy);

/* Exact LOO log-likelihood over a grid of scalar bandwidths (one hx for all
 * x-dimensions, one hy for all y-dimensions), Section 3 eq. (3).
 *   hx[n_hx], hy[n_hy]: host arrays, every value finite and > 0.
 *   totals_dev: [n_hx*n_hy] doubles, hx-major (index a*n_hy + b): S(hx[a], hy[b]).
 *   per_point_dev: optional [n_hx*n_hy][n] doubles (l_i per setting) or NULL.
 *   n_nonfinite_dev: optional [1] int64: number of non-finite l_i (0 for
 *   finite data; a non-finite l_i makes its total non-finite), or NULL.
 *   kernel: CDE_GAUSSIAN or CDE_EPANECHNIKOV (the latter runs every setting
 *   as a diagonal setting over the model's spatial order, built on first use;
 *   per-point outputs stay in the caller's point order).
 *   xterm: CDE_XTERM_MFMA_BF16X3 and CDE_XTERM_VALU_F32 are accepted for
 *   dx = 16, FP32 data and the Gaussian kernel only (CDE_EUNSUPPORTED
 *   otherwise); they change only how x-distances are formed (see
 *   cde_xterm).
 *   Limits: n_hx, n_hy in [1, 64]. */
cde_status cde_loo_loglik(cde_model* m, const double* hx, int32_t n_hx, const double* hy,
                          int32_t n_hy, cde_criterion criterion, cde_kernel kernel,
                          cde_xterm xterm,
                          double* totals_dev, double* per_point_dev,
                          int64_t* n_nonfinite_dev, void* stream);

/* One work item of a grouped launch (cde_launch_batch): the points
 * [i0, i1) of one model, each against all of that model's points. */
typedef struct cde_work_item {
    cde_model* model;          /* an FP32 model (cde_create with CDE_F32) */
    int64_t i0, i1;            /* 0 <= i0 < i1 <= n; i0 a multiple of 256; i1 a multiple of 256 or n */
    double* totals_dev;        /* [n_hx * n_hy] doubles, hx-major; written by the range with i1 = n
                                  (required there, ignored otherwise) */
    int64_t* n_nonfinite_dev;  /* [1] int64 or NULL; written with the totals */
} cde_work_item;

/* Grouped launch of the exact LOO log-likelihood over a grid of scalar
 * bandwidths (Section 3, eq. 3, the A_i expansion of Section 3.2; Gaussian
 * kernel, default cross term) for a work list of point ranges of several
 * models: every stage of the grid pass runs as one launch over all items
 * (per 8 items), so many small bandwidth-selection jobs, and the slices of
 * large ones, share the device in one kernel instead of one launch each.
 * A range runs the FP32 pass over its points and lists the ones that need
 * FP64 recomputation; the recomputation, the finalisation and the sums run
 * once per model, in the call whose range ends at n, over the whole model
 * (so a model's last range costs more than its others).
 *   items [n_items], 1 <= n_items <= 512: all models FP32, with the same dx
 *     and dy and on the same device, each model at most once per call.
 *   hx [n_hx], hy [n_hy]: one grid for all items, 1 <= n_hx, n_hy <= 16.
 * A model's ranges run over successive calls in order: its first range
 * starts at 0 and each next one at the previous i1, with the same grid and
 * criterion, until a range ends at n, which writes the totals (bit-identical
 * to cde_loo_loglik's for the same grid) and completes the evaluation.
 * Between its first and last range the model's scratch holds the
 * evaluation, so every other call on that model returns CDE_EINVAL until
 * the last range has been issued; calls of one evaluation must be ordered on
 * the device (one stream, or events).  The first range of a model may
 * allocate its scratch (as cde_loo_loglik does).  Errors leave every
 * model's evaluation state unchanged. */
cde_status cde_launch_batch(const cde_work_item* items, int32_t n_items, const double* hx, int32_t n_hx,
                            const double* hy, int32_t n_hy, cde_criterion criterion, void* stream);

/* Scheduling hint for cde_launch_batch: the number of points whose ranges
 * fill one full round of the grouped grid pass on the current device
 * (compute units x resident blocks per unit x points per block) for models
 * of this shape.  Ranges that are whole multiples of it keep the pass's last
 * round of blocks full; a range of 2.4 rounds costs as much as 3.  Returns 0
 * for unsupported shapes or when no device is visible.  No work is launched. */
int64_t cde_batch_round_points(int32_t dx, int32_t dy);

/* Exact LOO log-likelihood for a list of g diagonal bandwidth settings.
 *   h: host [g][dx+dy] (hx_1..hx_dx, hy_1..hy_dy per setting).
 *   kernel: CDE_GAUSSIAN, or CDE_EPANECHNIKOV (FP64 pair arithmetic over
 *   the model's spatial order, built on first use: the Morton order of x,
 *   with (point block, j tile) pairs whose x boxes lie a window apart
 *   skipped, since every term there is exactly zero).
 *   totals_dev: [g] doubles; per_point_dev: optional [g][n] doubles (in the
 *   caller's point order) or NULL.
 *   Limits: 1 <= g <= 4096. */
cde_status cde_loo_loglik_list(cde_model* m, const double* h, int32_t g,
                               cde_criterion criterion, cde_kernel kernel,
                               double* totals_dev, double* per_point_dev, void* stream);

/* Value and bandwidth gradient for one diagonal setting (adjoint of eq. 3).
 *   h: host [dx+dy].  total_dev: [1] double S(h).  grad_dev: [dx+dy] doubles,
 *   dS/dh_k (with respect to the bandwidths themselves, not their logs).
 *   Gaussian kernel.
 *   per_point_dev: optional [n] doubles (l_i) or NULL. */
cde_status cde_loo_grad(cde_model* m, const double* h, cde_criterion criterion,
                        double* total_dev, double* grad_dev, double* per_point_dev,
                        void* stream);

/* Allocation-free variant of cde_loo_grad, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, and
 * harnesses that forbid hipMalloc.  Same arguments, kernels and results as
 * cde_loo_grad (bit for bit whenever cde_loo_grad's j-chunk count fits the
 * scratch below; otherwise fewer chunks, which changes only the rounding).
 * The call allocates nothing and frees nothing: its scratch is a
 * library-owned static device array of 64 MiB on each GPU, created when the
 * library's code is loaded on that GPU and held until the process ends.
 * Every call on one GPU shares that array, so calls that overlap in time on
 * one GPU (on different streams, or from different threads) race; order
 * them.  Nothing in the array needs clearing between calls.
 * Limit: the per-block rows plus one j-chunk of partials,
 * 8 ((n_pad / 256)(dx + dy + 2) + 1 + n_pad (4 + 2 dx + dy)) + 256 bytes
 * with n_pad = n rounded up to 256, must fit the 64 MiB (n <= 557,824 at
 * dx = 5, dy = 1; n <= 220,160 at dx = 16, dy = 2); beyond it
 * CDE_EUNSUPPORTED with a message.
 * The model's first call that checks bandwidths still waits for cde_create's
 * extent copy (no allocation). */
cde_status cde_loo_grad_noalloc(cde_model* m, const double* h, cde_criterion criterion,
                                double* total_dev, double* grad_dev, double* per_point_dev,
                                void* stream);

/* Conditional density queries, eq. (1) over all n training points (no point
 * left out): f_dev[qq][g] = f(ygrid[g] | xq[qq]).
 *   xq_dev: [q][dx], ygrid_dev: [k][dy], device memory of the model's
 *   precision type.  h: host [dx+dy].  kernel: CDE_GAUSSIAN, or
 *   CDE_EPANECHNIKOV (the kernel of Section 4, radial over the scaled
 *   coordinates; FP32 models only; f = 0 where no training x lies inside the
 *   query's x window, where eq. (1) is 0/0).  f_dev: [q][k] doubles.
 *   Limits: q >= 0, 0 <= k <= 4096. */
cde_status cde_density_query(cde_model* m, const void* xq_dev, int64_t q, const void* ygrid_dev,
                             int64_t k, const double* h, cde_kernel kernel, double* f_dev,
                             void* stream);

/* Conditional mean E[y | x_q] = sum_i K_hx(x_q - x_i) y_i / sum_i K_hx(x_q - x_i),
 * the mean of eq. (1)'s density (each y-kernel component has mean y_i): the
 * prediction of y by the expectation of f(y|x) in Section 4.2.  Gaussian
 * kernel, FP64 arithmetic.
 *   xq_dev: [q][dx] device memory of the model's precision type.  h: host
 *   [dx+dy] (the y bandwidths do not enter the mean).  mean_dev: [q][dy]
 *   doubles.  */
cde_status cde_conditional_mean(cde_model* m, const void* xq_dev, int64_t q, const double* h,
                                double* mean_dev, void* stream);

/* Summaries of conditional densities on a y grid (dy = 1): the mode and the
 * narrowest prediction interval of Section 4 (there: the narrowest set of
 * quantiles with coverage 1 - alpha, found from a sample; here, deterministic
 * on the grid).  For each row of f_dev [q][k] (e.g. from cde_density_query on
 * the increasing grid ygrid_dev [k], doubles), out_dev[row] = {mass, mode, lo,
 * hi}: mass = trapezoid integral of the row; mode = the first grid point of
 * maximal f; [lo, hi] = the narrowest interval holding 1 - alpha of the
 * grid's CDF G (trapezoid partial sums over mass, linear between grid
 * points), over the intervals with one end on a grid point (lower ends
 * first, then upper ends), the first of least width (a later one replaces it
 * only when narrower by more than 1e-12 of the grid's span).  A row of zero
 * mass gives lo = hi = NaN.  No model is needed.
 *   Limits: q >= 0, 2 <= k <= 4096, 0 < alpha < 1.  */
cde_status cde_density_summary(const double* f_dev, const double* ygrid_dev, int64_t q, int64_t k,
                               double alpha, double* out_dev, void* stream);

/* Cross-validated integrated squared error of Section 3 (eq. (2) and the
 * cross-validated estimate that follows it), Gaussian product kernels, one
 * diagonal setting h (host [dx+dy]):
 *   ISE = (1/n) sum_i T1_i - (2/n) sum_i T2_i,
 *   T1_i = integral over y of f^{-i}(y|x_i)^2   (a double sum over j, l != i:
 *          O(n^2) per point, O(n^3) in all, on the matrix cores),
 *   T2_i = f^{-i}(y_i|x_i)                      (exp of cde_loo_loglik's l_i).
 *   out_dev: [3] doubles {ISE, (1/n) sum T1, (1/n) sum T2}.
 *   terms_dev: optional [n][2] doubles {T1_i, T2_i}, or NULL.
 * FP32 models only (CDE_EUNSUPPORTED otherwise); n <= 262144.  */
cde_status cde_cv_ise(cde_model* m, const double* h, double* out_dev, double* terms_dev, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* CDE_H */
