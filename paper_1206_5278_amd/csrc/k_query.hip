// k_query.hip -- conditional density queries on the matrix cores (FP32 models).
//
// Eq. (1) of Holmes, Gray & Isbell over all n training points:
//     f(y_g | x_q) = sum_i K_hx(x_q - x_i) K_hy(y_g - y_i) / sum_i K_hx(x_q - x_i).
// For a batch of queries q and a shared grid of y values g, the numerator is
//     F[q][g] = sum_i w(q, i) k(i, g),
// a dense contraction over the training points of a [Q x n] matrix of
// x-kernels with an [n x k] matrix of y-kernels.  It runs on
// v_mfma_f64_16x16x4f64: per training point, one x-kernel value per query and
// one y-kernel value per grid point are formed on the VALU (not one product
// kernel per (q, g)).
//
// Shifts: w' = 2^-(d2x(q,i) - m_q), k' = 2^-(d2y(g,i) - mu_g), with m_q the
// smallest scaled x-distance of query q to the data and mu_g the smallest
// scaled y-distance of grid point g (FP64 prepasses), so w' <= 1 (= 1 at the
// query's neighbour: den' >= 1) and k' <= 1; kernel values are v_exp_f32 of
// the fractional exponent scaled exactly by a power of two in FP64, as in the
// grid kernel.  f = c_y 2^-mu_g F'/D' is formed in FP64 in the epilogue.
//
// Work decomposition: a 256-lane block owns 64 queries (16 per wave) and a
// chunk of up to 128 grid points (blockIdx.y); training points stream through
// LDS in 256-point tiles.
#include <type_traits>

#include "cde_device.h"
#include "cde_kernels.h"

namespace cde {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double exp2_neg_wide_q(float t)
{
#pragma clang fp contract(off)
    const float fl = floorf(t);
    const float fr = t - fl;
    return ldexp((double)__builtin_amdgcn_exp2f(-fr), (int)(-fl));
}

constexpr float QEXCLUDED = 1e20f;

struct QueryArgs {
    double cx[16];   // log2(e) / (2 hx_k^2)
    double cy[4];    // log2(e) / (2 hy_l^2)
    double log_cy;
};

}  // namespace

// m_q = min_i sum_k c_k (x_qk - x_ik)^2 (FP64), one lane per query.
template <int DX, int DY>
__global__ __launch_bounds__(TILE) void k_qshift_x(const float* __restrict__ pts, int n,
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
    const int ntiles = (n + TILE - 1) / TILE;
    for (int t = 0; t < ntiles; ++t) {
        __syncthreads();
        float pre[S];
        load_row<S>(pre, pts + ((size_t)t * TILE + tid) * S);
        store_row<S>(tile + tid * S, pre);
        __syncthreads();
        const int cnt = min(TILE, n - t * TILE);
        for (int j = 0; j < cnt; ++j) {
            double d2 = 0.0;
#pragma unroll
            for (int k = 0; k < DX; ++k) {
                const double d = xo[k] - (double)tile[j * S + k];
                d2 = fma_(d * d, qa.cx[k], d2);
            }
            best = min_(best, d2);
        }
    }
    if (e < q) mq[e] = best;
}

// mu_g = min_i sum_l c'_l (y_gl - y_il)^2 (FP64), one lane per grid point.
template <int DX, int DY>
__global__ __launch_bounds__(TILE) void k_qshift_y(const float* __restrict__ pts, int n,
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
    const int ntiles = (n + TILE - 1) / TILE;
    for (int t = 0; t < ntiles; ++t) {
        __syncthreads();
        float pre[S];
        load_row<S>(pre, pts + ((size_t)t * TILE + tid) * S);
        store_row<S>(tile + tid * S, pre);
        __syncthreads();
        const int cnt = min(TILE, n - t * TILE);
        for (int j = 0; j < cnt; ++j) {
            double d2 = 0.0;
#pragma unroll
            for (int l = 0; l < DY; ++l) {
                const double d = yo[l] - (double)tile[j * S + DX + l];
                d2 = fma_(d * d, qa.cy[l], d2);
            }
            best = min_(best, d2);
        }
    }
    if (e < k) mu[e] = best;
}

template <int DX, int DY>
__global__ __launch_bounds__(TILE) void k_query_mfma(const float* __restrict__ pts, int n,
                                                     const float* __restrict__ xq, int q,
                                                     const float* __restrict__ yg, int k,
                                                     QueryArgs qa, const double* __restrict__ mq,
                                                     const double* __restrict__ mu,
                                                     double* __restrict__ f)
{
    constexpr int S = row_stride(DX, DY);
    constexpr int GT = 8;  // grid tiles of 16 per block (128 grid points)
    __shared__ float tile[TILE * S];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int q0 = blockIdx.x * 64 + wave * 16;
    const int g0 = blockIdx.y * 16 * GT;
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

    v4d acc[GT];
#pragma unroll
    for (int t = 0; t < GT; ++t) acc[t] = v4d{0.0, 0.0, 0.0, 0.0};
    double dsum = 0.0;

    const int ntiles = (n + TILE - 1) / TILE;
    float pre[S];
    load_row<S>(pre, pts + (size_t)tid * S);
    for (int tt = 0; tt < ntiles; ++tt) {
        __syncthreads();
        store_row<S>(tile + tid * S, pre);
        __syncthreads();
        if (tt + 1 < ntiles) load_row<S>(pre, pts + ((size_t)(tt + 1) * TILE + tid) * S);
        const int cnt = min(TILE, n - tt * TILE);
        for (int i4 = 0; i4 < cnt; i4 += 4) {
            const int ii = i4 + kr;
            float pj[S];
            load_row<S>(pj, tile + ii * S);  // rows >= cnt are packed padding (in bounds)
            const bool live = ii < cnt;
            double d2 = 0.0;
#pragma unroll
            for (int kk = 0; kk < DX; ++kk) {
                const double d = xo[kk] - (double)pj[kk];
                d2 = fma_(d * d, qa.cx[kk], d2);
            }
            const float xa = live ? (float)(d2 - m_q) : QEXCLUDED;
            const double w = exp2_neg_wide_q(xa);
            dsum += w;
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
                    acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(w, exp2_neg_wide_q(ya), acc[t], 0,
                                                                  0, 0);
                }
            }
        }
    }
    // den' of query q0 + lane%16: sum over the four k-rows in a fixed order
    dsum += __shfl_xor(dsum, 16, 64);
    dsum += __shfl_xor(dsum, 32, 64);
    // result layout (f64 16x16x4): register r holds query (lane/16) + 4 r,
    // grid column lane%16
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int qi = (lane >> 4) + 4 * r;
        const double den = __shfl(dsum, qi, 64);
        const int qq = q0 + qi;
#pragma unroll
        for (int t = 0; t < GT; ++t) {
            const int g = g0 + 16 * t + (lane & 15);
            if (t < ntg && qq < q && g < k) {
                const double num = acc[t][r];
                f[(size_t)qq * k + g] =
                    num > 0.0 ? exp(qa.log_cy - mu_g[t] * LN2 + log(num / den)) : 0.0;
            }
        }
    }
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
    const float* pts = (const float*)m->pts;
    double* mq = work;
    double* mu = work + q;
    hipLaunchKernelGGL((k_qshift_x<DX, DY>), dim3((q + TILE - 1) / TILE), dim3(TILE), 0, stream,
                       pts, (int)m->n, xq, q, qa, mq);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_qshift_y<DX, DY>), dim3((k + TILE - 1) / TILE), dim3(TILE), 0, stream,
                       pts, (int)m->n, yg, k, qa, mu);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL((k_query_mfma<DX, DY>), dim3((q + 63) / 64, (k + 127) / 128), dim3(TILE), 0,
                       stream, pts, (int)m->n, xq, q, yg, k, qa, (const double*)mq,
                       (const double*)mu, f);
    return hipGetLastError();
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
