// k_query.hip -- conditional density queries on the matrix cores (FP32 models).
//
// Eq. (1) of Holmes, Gray & Isbell over all n training points:
//     f(y_g | x_q) = sum_i K_hx(x_q - x_i) K_hy(y_g - y_i) / sum_i K_hx(x_q - x_i).
// For a batch of queries q and a shared grid of y values g, the numerator is
//     F[q][g] = sum_i w(q, i) k(i, g),
// a dense contraction over the training points of a [Q x n] matrix of
// x-kernels with an [n x k] matrix of y-kernels.  It runs on
// v_mfma_f32_16x16x4f32: per training point, one x-kernel value per query and
// one y-kernel value per grid point are formed on the VALU (not one product
// kernel per (q, g)).
//
// Shifts: w' = 2^-(d2x(q,i) - m_q), k' = 2^-(d2y(g,i) - mu_g), with m_q the
// smallest scaled x-distance of query q to the data and mu_g the smallest
// scaled y-distance of grid point g (FP64 prepasses; exact minima, so the
// nearest point has w' = 1 and den' >= 1).  Distances and the shifted
// exponents are formed in FP64 and rounded to FP32 after the subtraction.
// Kernel values and products are FP32; sums over a 256-point tile are folded
// into Kahan-compensated FP32 totals.  A value of f more than ~2^-100 below
// its query's peak is not carried to full relative precision (FP32 range);
// such tail values are far below the accuracy floor of a density estimate.
//
// Work decomposition: a 256-lane block owns 64 queries (16 per wave), a chunk
// of up to 128 grid points (blockIdx.y) and a chunk of training points
// (blockIdx.z); chunk partial sums (FP64) are combined in a fixed order by
// k_query_reduce.  The training-point chunks depend on n alone and every
// query row is accumulated on its own, so a query's result does not depend
// on which other queries share its launch; large batches run in slices of
// queries that bound the partial storage.
#include <type_traits>

#include "cde_device.h"
#include "cde_kernels.h"

namespace cde {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr float QEXCLUDED = 1e20f;

struct QueryArgs {
    double cx[16];   // log2(e) / (2 hx_k^2)
    double cy[4];    // log2(e) / (2 hy_l^2)
    double log_cy;
};

// Non-negative doubles order like their bit patterns: an exact, order-free
// minimum through a 64-bit integer atomic.
__device__ __forceinline__ void atomic_min_nonneg(double* p, double v)
{
    atomicMin((unsigned long long*)p, (unsigned long long)__double_as_longlong(v));
}

__global__ void k_fill_inf(double* p, int cnt)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cnt) p[i] = __builtin_inf();
}

}  // namespace

// m_q = min_i sum_k c_k (x_qk - x_ik)^2 (FP64): lane = query, blockIdx.y =
// range of training points.
template <int DX, int DY>
__global__ __launch_bounds__(TILE) void k_qshift_x(const float* __restrict__ pts, int n, int chunk,
                                                   const float* __restrict__ xq, int q,
                                                   QueryArgs qa, double* __restrict__ mq)
{
    constexpr int S = row_stride(DX, DY);
    __shared__ float tile[TILE * S];
    const int tid = threadIdx.x;
    const int e = blockIdx.x * TILE + tid;
    const int ec = e < q ? e : q - 1;
    double xo[DX];
#pragma unroll
    for (int k = 0; k < DX; ++k) xo[k] = (double)xq[(size_t)ec * DX + k];
    double best = inf_<double>();
    const int j0 = blockIdx.y * chunk, j1 = min(n, j0 + chunk);
    for (int t0 = j0; t0 < j1; t0 += TILE) {
        __syncthreads();
        float pre[S];
        load_row<S>(pre, pts + ((size_t)t0 + tid) * S);
        store_row<S>(tile + tid * S, pre);
        __syncthreads();
        const int cnt = min(TILE, j1 - t0);
        for (int j = 0; j < cnt; ++j) {
            float pj[S];
            load_row<S>(pj, tile + j * S);
            double d2 = 0.0;
#pragma unroll
            for (int k = 0; k < DX; ++k) {
                const double d = xo[k] - (double)pj[k];
                d2 = fma_(d * d, qa.cx[k], d2);
            }
            best = min_(best, d2);
        }
    }
    if (e < q) atomic_min_nonneg(mq + e, best);
}

// mu_g = min_i sum_l c'_l (y_gl - y_il)^2 (FP64), same decomposition.
template <int DX, int DY>
__global__ __launch_bounds__(TILE) void k_qshift_y(const float* __restrict__ pts, int n, int chunk,
                                                   const float* __restrict__ yg, int k,
                                                   QueryArgs qa, double* __restrict__ mu)
{
    constexpr int S = row_stride(DX, DY);
    __shared__ float tile[TILE * S];
    const int tid = threadIdx.x;
    const int e = blockIdx.x * TILE + tid;
    const int ec = e < k ? e : k - 1;
    double yo[DY];
#pragma unroll
    for (int l = 0; l < DY; ++l) yo[l] = (double)yg[(size_t)ec * DY + l];
    double best = inf_<double>();
    const int j0 = blockIdx.y * chunk, j1 = min(n, j0 + chunk);
    for (int t0 = j0; t0 < j1; t0 += TILE) {
        __syncthreads();
        float pre[S];
        load_row<S>(pre, pts + ((size_t)t0 + tid) * S);
        store_row<S>(tile + tid * S, pre);
        __syncthreads();
        const int cnt = min(TILE, j1 - t0);
        for (int j = 0; j < cnt; ++j) {
            float pj[S];
            load_row<S>(pj, tile + j * S);
            double d2 = 0.0;
#pragma unroll
            for (int l = 0; l < DY; ++l) {
                const double d = yo[l] - (double)pj[DX + l];
                d2 = fma_(d * d, qa.cy[l], d2);
            }
            best = min_(best, d2);
        }
    }
    if (e < k) atomic_min_nonneg(mu + e, best);
}

template <int DX, int DY>
__global__ __launch_bounds__(TILE) void k_query_mfma(const float* __restrict__ pts, int n, int chunk,
                                                     const float* __restrict__ xq, int q,
                                                     const float* __restrict__ yg, int k,
                                                     QueryArgs qa, const double* __restrict__ mq,
                                                     const double* __restrict__ mu,
                                                     double* __restrict__ fpart,
                                                     double* __restrict__ dpart)
{
    constexpr int S = row_stride(DX, DY);
    constexpr int GT = 8;  // grid tiles of 16 per block (128 grid points)
    __shared__ float tile[TILE * S];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int q0 = blockIdx.x * 64 + wave * 16;
    const int g0 = blockIdx.y * 16 * GT;
    const int c = blockIdx.z;
    const int kr = lane >> 4;  // k-row of the MFMA operands: training point i0 + kr

    // A role: query q0 + lane%16
    const int qa_idx = min(q0 + (lane & 15), q - 1);
    double xo[DX];
#pragma unroll
    for (int kk = 0; kk < DX; ++kk) xo[kk] = (double)xq[(size_t)qa_idx * DX + kk];
    const double m_q = mq[qa_idx];
    // B role: grid points g0 + 16 t + lane%16, t < GT
    double yo[GT][DY];
    double mu_g[GT];
#pragma unroll
    for (int t = 0; t < GT; ++t) {
        const int g = min(g0 + 16 * t + (lane & 15), k - 1);
#pragma unroll
        for (int l = 0; l < DY; ++l) yo[t][l] = (double)yg[(size_t)g * DY + l];
        mu_g[t] = mu[g];
    }
    const int ntg = min(GT, (k - g0 + 15) / 16);  // grid tiles present in this chunk

    v4f acc[GT];
    Kahan<float> tot[GT][4];
#pragma unroll
    for (int t = 0; t < GT; ++t) {
        acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int r = 0; r < 4; ++r) tot[t][r].zero();
    }
    float dp = 0.f;
    Kahan<float> dtot;
    dtot.zero();

    const int j0 = c * chunk, j1 = min(n, j0 + chunk);
    float pre[S];
    load_row<S>(pre, pts + ((size_t)j0 + tid) * S);
    for (int t0 = j0; t0 < j1; t0 += TILE) {
        __syncthreads();
        store_row<S>(tile + tid * S, pre);
        __syncthreads();
        if (t0 + TILE < j1) load_row<S>(pre, pts + ((size_t)t0 + TILE + tid) * S);
        const int cnt = min(TILE, j1 - t0);
        for (int i4 = 0; i4 < cnt; i4 += 4) {
            const int ii = i4 + kr;
            float pj[S];
            load_row<S>(pj, tile + ii * S);  // rows >= cnt are packed rows (in bounds)
            const bool live = ii < cnt;
            double d2 = 0.0;
#pragma unroll
            for (int kk = 0; kk < DX; ++kk) {
                const double d = xo[kk] - (double)pj[kk];
                d2 = fma_(d * d, qa.cx[kk], d2);
            }
            const float xa = live ? (float)(d2 - m_q) : QEXCLUDED;
            const float w = exp2_<float>(-xa);
            dp += w;
#pragma unroll
            for (int t = 0; t < GT; ++t) {
                if (t < ntg) {
                    double e = 0.0;
#pragma unroll
                    for (int l = 0; l < DY; ++l) {
                        const double d = yo[t][l] - (double)pj[DX + l];
                        e = fma_(d * d, qa.cy[l], e);
                    }
                    const float ya = live ? (float)(e - mu_g[t]) : QEXCLUDED;
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(w, exp2_<float>(-ya), acc[t], 0, 0, 0);
                }
            }
        }
#pragma unroll
        for (int t = 0; t < GT; ++t) {
#pragma unroll
            for (int r = 0; r < 4; ++r) tot[t][r].add(acc[t][r]);
            acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
        }
        dtot.add(dp);
        dp = 0.f;
    }
    // den' partial of query q0 + lane%16: the four k-rows in a fixed order
    double dsum = dtot.value();
    dsum += __shfl_xor(dsum, 16, 64);
    dsum += __shfl_xor(dsum, 32, 64);
    if (blockIdx.y == 0 && lane < 16 && q0 + lane < q) dpart[(size_t)c * q + q0 + lane] = dsum;
    // f32 16x16x4 result layout: register r holds query 4*(lane/16) + r,
    // grid column lane%16
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int qq = q0 + 4 * (lane >> 4) + r;
#pragma unroll
        for (int t = 0; t < GT; ++t) {
            const int g = g0 + 16 * t + (lane & 15);
            if (t < ntg && qq < q && g < k) fpart[((size_t)c * q + qq) * k + g] = tot[t][r].value();
        }
    }
}

// f = c_y 2^-mu_g F'/D' with F' and D' summed over the point chunks in order.
__global__ void k_query_reduce(const double* __restrict__ fpart, const double* __restrict__ dpart,
                               const double* __restrict__ mu, int q, int k, int nchunks,
                               double log_cy, double* __restrict__ f)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)q * k) return;
    const int qq = (int)(e / k), g = (int)(e - (int64_t)qq * k);
    double num = 0.0, den = 0.0;
    for (int c = 0; c < nchunks; ++c) {
        num += fpart[((size_t)c * q + qq) * k + g];
        den += dpart[(size_t)c * q + qq];
    }
    f[e] = num > 0.0 ? exp(log_cy - mu[g] * LN2 + log(num / den)) : 0.0;
}

// Training-point chunks: whole tiles, at most 256 chunks, a function of n
// only (never of the batch).
static int64_t query_chunk_points(int64_t n)
{
    const int64_t ntiles = (n + TILE - 1) / TILE;
    return (ntiles + 255) / 256 * TILE;
}

// Queries per slice: chunk partials of one slice within 2^26 doubles.
static int64_t query_slice(int64_t nch, int64_t q, int64_t k)
{
    int64_t s = ((int64_t(1) << 26) / (nch * (k + 1))) / 64 * 64;
    return std::min(q, std::max<int64_t>(64, s));
}

size_t query_work_doubles(const cde_model* m, int64_t q, int64_t k)
{
    const int64_t chunk = query_chunk_points(m->n);
    const int64_t nch = (m->n + chunk - 1) / chunk;
    const int64_t qs = query_slice(nch, q, k);
    return (size_t)(q + k + nch * qs * (k + 1) + 64);
}

template <int DX, int DY>
static hipError_t query_t(const cde_model* m, const float* xq, int q, const float* yg, int k,
                          const double* h, double* f, double* work, hipStream_t stream)
{
    QueryArgs qa;
    for (int kk = 0; kk < 16; ++kk) qa.cx[kk] = kk < DX ? LOG2E / (2.0 * h[kk] * h[kk]) : 0.0;
    double lcy = 0.0;
    for (int l = 0; l < 4; ++l) {
        qa.cy[l] = l < DY ? LOG2E / (2.0 * h[DX + l] * h[DX + l]) : 0.0;
        if (l < DY) lcy -= log(h[DX + l]) + HALF_LOG_2PI;
    }
    qa.log_cy = lcy;
    const int n = (int)m->n;
    const float* pts = (const float*)m->pts;
    const int gb = (k + 127) / 128;
    const int chunk = (int)query_chunk_points(n);
    const int nch = (n + chunk - 1) / chunk;
    const int qs = (int)query_slice(nch, q, k);
    double* mq = work;
    double* mu = work + q;
    double* dpart = mu + k;
    double* fpart = dpart + (size_t)nch * qs;
    // shifts: exact minima over point chunks
    const int sch = 16 * TILE;
    const int nsch = (n + sch - 1) / sch;
    hipLaunchKernelGGL(k_fill_inf, dim3((q + k + 255) / 256), dim3(256), 0, stream, mq, q + k);
    hipLaunchKernelGGL((k_qshift_x<DX, DY>), dim3((q + TILE - 1) / TILE, nsch), dim3(TILE), 0, stream,
                       pts, n, sch, xq, q, qa, mq);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_qshift_y<DX, DY>), dim3((k + TILE - 1) / TILE, nsch), dim3(TILE), 0, stream,
                       pts, n, sch, yg, k, qa, mu);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    for (int q0 = 0; q0 < q; q0 += qs) {
        const int qn = std::min(qs, q - q0);
        const int qb = (qn + 63) / 64;
        hipLaunchKernelGGL((k_query_mfma<DX, DY>), dim3(qb, gb, nch), dim3(TILE), 0, stream, pts, n,
                           chunk, xq + (size_t)q0 * DX, qn, yg, k, qa, (const double*)(mq + q0),
                           (const double*)mu, fpart, dpart);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        const int64_t total = (int64_t)qn * k;
        hipLaunchKernelGGL(k_query_reduce, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream,
                           (const double*)fpart, (const double*)dpart, (const double*)mu, qn, k, nch,
                           lcy, f + (size_t)q0 * k);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

#define CDE_QM_CASE(DX_, DY_) \
    case (DX_) * 8 + (DY_): return query_t<DX_, DY_>(m, xq, q, yg, k, h, f, work, stream);

hipError_t launch_query_mfma(const cde_model* m, const float* xq, int q, const float* yg, int k,
                             const double* h, double* f, double* work, hipStream_t stream)
{
    switch (m->dx * 8 + m->dy) {
        CDE_QM_CASE(1, 1) CDE_QM_CASE(1, 2) CDE_QM_CASE(2, 1) CDE_QM_CASE(2, 2)
        CDE_QM_CASE(3, 1) CDE_QM_CASE(3, 2) CDE_QM_CASE(4, 1) CDE_QM_CASE(4, 2)
        CDE_QM_CASE(5, 1) CDE_QM_CASE(5, 2) CDE_QM_CASE(6, 1) CDE_QM_CASE(6, 2)
        CDE_QM_CASE(7, 1) CDE_QM_CASE(7, 2) CDE_QM_CASE(8, 1) CDE_QM_CASE(8, 2)
        CDE_QM_CASE(16, 1) CDE_QM_CASE(16, 2)
        default: return hipErrorInvalidValue;
    }
}

}  // namespace cde
