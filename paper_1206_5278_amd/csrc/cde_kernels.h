// cde_kernels.h -- launch functions of the gfx950 kernels (library-internal).
#pragma once

#include "cde_common.h"

namespace cde {

// Pack row-major x [n][dx] and y [n][dy] into the model's [npad][stride] rows.
template <typename T>
hipError_t launch_pack(cde_model* m, const T* x, const T* y, hipStream_t stream);
// Per-dimension minimum and maximum of the packed rows and a non-finite flag
// into ext [2 * MAXP + 1] (order-preserving 64-bit encodings of the doubles).
template <typename T>
hipError_t launch_extent(const cde_model* m, unsigned long long* ext, hipStream_t stream);

// Diagonal-bandwidth LOO pass (value, optionally gradient) for `nsets`
// settings.  The j range is split into `chunks` chunks (diag_chunks); the
// pair kernel writes per-(setting, chunk, point) partial sums to `partial`
// (diag_partial_doubles), and a combine kernel merges the chunks in fixed
// order, finalises each point in FP64 and writes one row per (setting,
// 256-point block) to `part`.
template <typename T>
hipError_t launch_diag(const cde_model* m, const DiagSets<T>& sets, int nsets, int crit, bool grad,
                       int chunks, double* partial, double* per_point, double* part,
                       hipStream_t stream);
// Number of j chunks that best fills the device for `nsets` settings per
// launch (a makespan model over the kernel's occupancy), within `max_doubles`
// of partial storage.
template <typename T>
int diag_chunks(const cde_model* m, int nsets, bool grad, size_t max_doubles);
size_t diag_partial_doubles(const cde_model* m, int nsets, bool grad, int chunks);
// Shared makespan model behind diag_chunks and epan_chunks: `kern` is the
// pair kernel (for its occupancy), np the partial planes per chunk.
int choose_chunks(const void* kern, const cde_model* m, int nsets, int np, size_t max_doubles);

// Stable LSD radix sort (k_sort.hip) of n (key, value) pairs by key bits
// [bit0, bit1), 6 bits per pass, ping-ponging between (k0, v0) and
// (k1, v1); on return *result_in_alt says whether the sorted pairs are in
// (k1, v1).  `work` holds radix_sort_work_bytes(n) bytes.  n < 2^31.
size_t radix_sort_work_bytes(int64_t n);
hipError_t radix_sort_pairs(unsigned long long* k0, int* v0, unsigned long long* k1, int* v1, int64_t n,
                            int bit0, int bit1, void* work, bool* result_in_alt, hipStream_t stream);

// Spatial order of the model's points (Morton order of x, sorted FP64 rows,
// permutation, per-tile x boxes) into m->spts / m->perm / m->tbox; `work`
// holds index_work_bytes(m) bytes of temporaries.
size_t index_work_bytes(const cde_model* m);
hipError_t launch_build_index(cde_model* m, void* work, size_t work_bytes, hipStream_t stream);

// Epanechnikov LOO pass over the spatially ordered points for `nsets`
// settings (up to 8): pair kernel with exact tile skipping into `partial`
// ([nsets][chunks][2][npad] doubles), then the fixed-order combine into
// per_point (original order) and block rows (l, non-finite) in `part`.
hipError_t launch_epan(const cde_model* m, const EpanSets& sets, int nsets, int crit, int chunks,
                       double* partial, double* per_point, double* part, hipStream_t stream);
int epan_chunks(const cde_model* m, int nsets, size_t max_doubles);

// Conditional mean E[y | xq] (Gaussian kernel) for q queries of the model's
// precision: mean [q][dy] doubles; `work` holds cond_mean_work_doubles().
hipError_t launch_cond_mean(const cde_model* m, const void* xq, int64_t q, const double* h, double* mean,
                            double* work, hipStream_t stream);
size_t cond_mean_work_doubles(const cde_model* m, int64_t q);
// Mass, mode and narrowest 1 - alpha interval of each row of f [q][k] on the
// increasing grid yg [k]: out [q][4] doubles.
hipError_t launch_density_summary(const double* f, const double* yg, int64_t q, int64_t k, double alpha,
                                  double* out, hipStream_t stream);

// Density queries f(yg[g] | xq[q]) over all training points -> f [q][k].
template <typename T>
hipError_t launch_query(const cde_model* m, const T* xq, int64_t q, const T* yg, int64_t k,
                        const DiagSets<T>& sets, double* f, hipStream_t stream);

// Density queries on FP32 models, on the matrix cores: f [q][k]; `work`
// holds query_work_doubles(m, q, k) doubles (shifts and chunk partials).
hipError_t launch_query_mfma(const cde_model* m, const float* xq, int q, const float* yg, int k,
                             const double* h, double* f, double* work, hipStream_t stream);
// Query decomposition shared by the Gaussian and Epanechnikov query kernels
// (functions of n and k only): training-point chunk size, grid tiles of 16
// per block, queries per slice.
int64_t query_chunk_points(int64_t n);
int query_grid_tiles(int64_t k);
int64_t query_slice(int64_t nch, int64_t q, int64_t k);
// Epanechnikov queries (k_query_epan.hip): FP32 models with the spatial
// index built; work = query_epan_work_bytes of device scratch.
size_t query_epan_work_bytes(const cde_model* m, int64_t q, int64_t k);
hipError_t launch_query_epan(const cde_model* m, const float* xq, int q, const float* yg, int k,
                             const double* h, double* f, char* work, hipStream_t stream);
// log of the radial Epanechnikov normalisation c_d / prod h_k (cde_api.hip)
double log_epan_norm(const double* h, int d);
size_t query_work_doubles(const cde_model* m, int64_t q, int64_t k);

// Cross-validated ISE (k_ise.hip): FP32 models; ell = the conditional LOO
// log-likelihood per point; out[3] = {ISE, mean T1, mean T2}; terms [n][2].
size_t ise_work_doubles(const cde_model* m);
hipError_t launch_cv_ise(const cde_model* m, const double* h, const double* ell, double* out,
                         double* terms, double* work, hipStream_t stream);

// Scalar-bandwidth grid on FP32 models: per-point neighbour shifts (first
// call only), the MFMA grid pass, FP64 finalisation, exact fixup of extreme
// entries and the fixed-order row sums.  `work` must hold grid_work_bytes();
// `counts` receives the per-setting non-finite counts [n_hx * n_hy].
// xm: how the FP32 pass forms x-distances: 0 FP64 differences (the
// library's path), 1 FP32 differences, 2 split-bf16 x3 cross term on the
// matrix cores (1 and 2: dx = 16 only).
hipError_t launch_grid(cde_model* m, const double* hx, int n_hx, const double* hy, int n_hy, int crit,
                       int xm, double* totals, double* per_point, void* work, size_t work_bytes,
                       double* counts, hipStream_t stream);
size_t grid_work_bytes(const cde_model* m, int n_hx, int n_hy);

// One work item of the grouped grid launch: points [i0, i1) of model m (FP32,
// grid work area `work` of work_bytes >= grid_work_bytes, non-finite counts
// in `counts`), against all of its points; the range ending at i1 = n also
// writes totals [G] and, if non-NULL, *nonfinite.  do_nn: compute the
// range's neighbour shifts first (the model has none yet).
struct GridRange {
    cde_model* m;
    int64_t i0, i1;
    double* totals;
    int64_t* nonfinite;
    void* work;
    size_t work_bytes;
    double* counts;
    bool do_nn;
};
// Points per full round of the grouped launch's FP32 grid pass on the
// current device: compute units x resident blocks per CU x points per
// block (0 for an unsupported shape).
int64_t grid_round_points(int dx, int dy, int ncu);
// The grid pipeline over a work list of ranges of models sharing dx and dy,
// for a grid of at most 16 x 16 cells: one launch per stage per 8 items.
hipError_t launch_grid_batch(const GridRange* r, int count, const double* hx, int n_hx, const double* hy,
                             int n_hy, int crit, hipStream_t stream);

// Fixed-order FP64 sum of the per-block partial rows of `nsets` settings:
// part [nsets][nblocks][nv] -> totals [nsets] (column 0), grad [nsets][nv-2]
// (columns 1..nv-2, if grad != NULL); if nonfinite != NULL, the per-setting
// non-finite counts (last column) go to counts [nsets] (scratch) and their
// sum is written to *nonfinite.
hipError_t launch_reduce_parts(const double* part, int nsets, int nblocks, int nv, double* totals,
                               double* grad, double* counts, int64_t* nonfinite, hipStream_t stream);

// *out = sum of counts[0..nsets) in order (one thread).
hipError_t launch_sum_counts(const double* counts, int nsets, int64_t* out, hipStream_t stream);

}  // namespace cde
