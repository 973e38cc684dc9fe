// k_products.hip -- query-side products of the conditional density estimate.
//
// Holmes, Gray & Isbell list the expectation, modes and prediction intervals
// among what a conditional density yields (Section 1); Section 4.2 predicts y
// by the expectation of f(y|x) and builds prediction intervals by searching
// for the narrowest set of quantiles with the desired coverage.
//
//   - Conditional mean (Gaussian kernel): E[y|x] = sum_i w_i y_i / sum_i w_i,
//     w_i = K_hx(x - x_i), the mean of eq. (1)'s density (each y-kernel
//     component has mean y_i).  FP64 throughout: the exact smallest scaled x
//     distance m_q per query (an integer atomic minimum on the bit patterns
//     of non-negative doubles, exact and order-free), then w_i =
//     exp(-(d_i - m_q)) <= 1 summed per chunk of training points, chunks
//     reduced in a fixed order.
//   - Summary of a density on an increasing y grid (dy = 1): mass (trapezoid
//     rule), mode (first grid point of maximal f) and the narrowest interval
//     holding 1 - alpha of the grid's piecewise-linear CDF G, over candidates
//     with one end on a grid node (lower ends first, then upper ends), the
//     first of least width (a later one replaces it only when narrower by
//     more than 1e-12 of the span).  One thread per row runs the scan
//     sequentially, so the result does not depend on any reduction order; the
//     inverse of G is found with a pointer that only moves forward, since the
//     targets increase along each scan.
#include <algorithm>
#include <type_traits>

#include "cde_device.h"
#include "cde_kernels.h"

namespace cde {

namespace {

struct MeanArgs {
    double cx[16];  // 1 / (2 hx_k^2): natural-log exponent coefficients
};

__device__ __forceinline__ void atomic_min_nonneg_d(double* p, double v)
{
    atomicMin((unsigned long long*)p, (unsigned long long)__double_as_longlong(v));
}

__global__ void k_fill_inf_d(double* p, int cnt)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cnt) p[i] = __builtin_inf();
}

// Scaled squared x distance of query x to a tile row (FP64).
template <typename T, int DX>
__device__ __forceinline__ double xdist(const double (&xo)[DX], const T* pj, const MeanArgs& a)
{
    double d2 = 0.0;
#pragma unroll
    for (int k = 0; k < DX; ++k) {
        const double d = xo[k] - (double)pj[k];
        d2 = fma(d * d, a.cx[k], d2);
    }
    return d2;
}

// m_q = min_i d(q, i) over one chunk of training points (lane = query,
// blockIdx.y = chunk), merged by an exact atomic minimum.
template <typename T, int DX, int DY>
__global__ __launch_bounds__(TILE) void k_cmean_shift(const T* __restrict__ pts, int n, int chunk,
                                                      const T* __restrict__ xq, int q, MeanArgs a,
                                                      double* __restrict__ mq)
{
    constexpr int S = row_stride(DX, DY);
    __shared__ T tile[TILE * S];
    const int tid = threadIdx.x;
    const int e = blockIdx.x * TILE + tid;
    const int ec = e < q ? e : q - 1;
    double xo[DX];
    float xo32[DX], c32[DX];
#pragma unroll
    for (int k = 0; k < DX; ++k) {
        xo[k] = (double)xq[(size_t)ec * DX + k];
        xo32[k] = (float)xq[(size_t)ec * DX + k];
        c32[k] = (float)a.cx[k];
    }
    ScreenedMin screen;
    double best = __builtin_inf();
    const int j0 = blockIdx.y * chunk, j1 = min(n, j0 + chunk);
    for (int t0 = j0; t0 < j1; t0 += TILE) {
        __syncthreads();
        T pre[S];
        load_row<S>(pre, pts + ((size_t)t0 + tid) * S);
        store_row<S>(tile + tid * S, pre);
        __syncthreads();
        const int cnt = min(TILE, j1 - t0);
        if constexpr (std::is_same<T, float>::value) {
            // FP32 screening against the running FP32 minimum; the FP64
            // distance is taken for every candidate, so best is exactly the
            // FP64 minimum (ScreenedMin, cde_device.h)
            for (int j = 0; j < cnt; ++j) {
                const float* pj = tile + j * S;
                float e32 = 0.f;
#pragma unroll
                for (int k = 0; k < DX; ++k) {
                    const float d = xo32[k] - pj[k];
                    e32 = fmaf(d * d, c32[k], e32);
                }
                if (screen.candidate(e32)) best = fmin(best, xdist<T, DX>(xo, pj, a));
            }
        } else {
            for (int j = 0; j < cnt; ++j) best = fmin(best, xdist<T, DX>(xo, tile + j * S, a));
        }
    }
    if (e < q) atomic_min_nonneg_d(mq + e, best);
}

// Per chunk of training points: D = sum exp(-(d - m_q)), S_l = sum of the
// same weights times y_il, written to part[(chunk * q + query) * (1 + DY)].
template <typename T, int DX, int DY>
__global__ __launch_bounds__(TILE) void k_cmean_sums(const T* __restrict__ pts, int n, int chunk,
                                                     const T* __restrict__ xq, int q, MeanArgs a,
                                                     const double* __restrict__ mq,
                                                     double* __restrict__ part)
{
    constexpr int S = row_stride(DX, DY);
    __shared__ T tile[TILE * S];
    const int tid = threadIdx.x;
    const int e = blockIdx.x * TILE + tid;
    const int ec = e < q ? e : q - 1;
    double xo[DX];
#pragma unroll
    for (int k = 0; k < DX; ++k) xo[k] = (double)xq[(size_t)ec * DX + k];
    const double m = mq[ec];
    double D = 0.0, Sy[DY];
#pragma unroll
    for (int l = 0; l < DY; ++l) Sy[l] = 0.0;
    const int j0 = blockIdx.y * chunk, j1 = min(n, j0 + chunk);
    for (int t0 = j0; t0 < j1; t0 += TILE) {
        __syncthreads();
        T pre[S];
        load_row<S>(pre, pts + ((size_t)t0 + tid) * S);
        store_row<S>(tile + tid * S, pre);
        __syncthreads();
        const int cnt = min(TILE, j1 - t0);
        for (int j = 0; j < cnt; ++j) {
            const T* pj = tile + j * S;
            const double w = exp(m - xdist<T, DX>(xo, pj, a));
            D += w;
#pragma unroll
            for (int l = 0; l < DY; ++l) Sy[l] = fma(w, (double)pj[DX + l], Sy[l]);
        }
    }
    if (e < q) {
        double* o = part + ((size_t)blockIdx.y * q + e) * (1 + DY);
        o[0] = D;
#pragma unroll
        for (int l = 0; l < DY; ++l) o[1 + l] = Sy[l];
    }
}

// mean[q][l] = (sum over chunks, in order, of S_l) / (sum of D).
__global__ void k_cmean_reduce(const double* __restrict__ part, int q, int dy, int nch,
                               double* __restrict__ mean)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= q) return;
    double D = 0.0, Sy[4] = {0.0, 0.0, 0.0, 0.0};
    for (int c = 0; c < nch; ++c) {
        const double* r = part + ((size_t)c * q + e) * (1 + dy);
        D += r[0];
        for (int l = 0; l < dy; ++l) Sy[l] += r[1 + l];
    }
    for (int l = 0; l < dy; ++l) mean[(size_t)e * dy + l] = Sy[l] / D;
}

// Density summary, one thread per row (see the file header).
__global__ void k_density_summary(const double* __restrict__ f, const double* __restrict__ yg, int q,
                                  int k, double alpha, double* __restrict__ out)
{
#pragma clang fp contract(off)  // the same roundings as the plain scalar definition
    const int row = blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= q) return;
    const double* r = f + (size_t)row * k;
    double* o = out + (size_t)row * 4;
    // mass and mode
    double c = 0.0;
    int imax = 0;
    double fmax_ = r[0];
    for (int g = 0; g + 1 < k; ++g) {
        c += (r[g] + r[g + 1]) * 0.5 * (yg[g + 1] - yg[g]);
        if (r[g + 1] > fmax_) {
            fmax_ = r[g + 1];
            imax = g + 1;
        }
    }
    const double mass = c;
    o[0] = mass;
    o[1] = yg[imax];
    if (!(mass > 0.0)) {
        o[2] = o[3] = __builtin_nan("");
        return;
    }
    const double cover = 1.0 - alpha;
    const double tie = 1e-12 * (yg[k - 1] - yg[0]);
    double best = __builtin_inf(), blo = __builtin_nan(""), bhi = __builtin_nan("");
    // running cumulative sums (the same sequence of additions as the mass)
    // at the scan position a and at the inverse pointer p (and p - 1)
    for (int pass = 0; pass < 2; ++pass) {
        double ca = 0.0, cp = 0.0, cpm = 0.0;
        int ptr = 0;
        for (int a = 0; a < k; ++a) {
            if (a > 0) ca += (r[a - 1] + r[a]) * 0.5 * (yg[a] - yg[a - 1]);
            const double Ga = ca / mass;
            const double target = pass == 0 ? Ga + cover : Ga - cover;
            if (pass == 0 && target > 1.0) break;
            if (pass == 1 && target < 0.0) continue;
            // first index g with G_g >= target (g < k - 1 bound, as a scan from 0)
            while (ptr < k - 1 && cp / mass < target) {
                cpm = cp;
                cp += (r[ptr] + r[ptr + 1]) * 0.5 * (yg[ptr + 1] - yg[ptr]);
                ++ptr;
            }
            const double Gp = cp / mass, Gpm = cpm / mass;
            double y;
            if (ptr == 0 || Gp <= Gpm)
                y = yg[ptr];
            else
                y = yg[ptr - 1] + (target - Gpm) / (Gp - Gpm) * (yg[ptr] - yg[ptr - 1]);
            const double lo = pass == 0 ? yg[a] : y, hi = pass == 0 ? y : yg[a];
            if (hi - lo < best - tie) {
                best = hi - lo;
                blo = lo;
                bhi = hi;
            }
        }
    }
    o[2] = blo;
    o[3] = bhi;
}

MeanArgs mean_args(const double* h, int dx)
{
    MeanArgs a;
    for (int k = 0; k < 16; ++k) a.cx[k] = k < dx ? 1.0 / (2.0 * h[k] * h[k]) : 0.0;
    return a;
}

int mean_chunk_points(int64_t n)
{
    const int64_t ntiles = (n + TILE - 1) / TILE;
    return (int)((ntiles + 63) / 64 * TILE);
}

int64_t mean_slice(int64_t q) { return std::min<int64_t>(q, 16384); }

template <typename T, int DX, int DY>
static hipError_t cmean_t(const cde_model* m, const T* xq, int64_t q, const double* h, double* mean,
                          double* work, hipStream_t stream)
{
    const MeanArgs a = mean_args(h, DX);
    const int n = (int)m->n;
    const T* pts = (const T*)m->pts;
    const int chunk = mean_chunk_points(n);
    const int nch = (n + chunk - 1) / chunk;
    const int64_t qs = mean_slice(q);
    double* mq = work;
    double* part = work + qs;
    for (int64_t q0 = 0; q0 < q; q0 += qs) {
        const int qn = (int)std::min(qs, q - q0);
        const T* xs = xq + (size_t)q0 * DX;
        hipLaunchKernelGGL(k_fill_inf_d, dim3((qn + 255) / 256), dim3(256), 0, stream, mq, qn);
        hipLaunchKernelGGL((k_cmean_shift<T, DX, DY>), dim3((qn + TILE - 1) / TILE, nch), dim3(TILE), 0,
                           stream, pts, n, chunk, xs, qn, a, mq);
        hipLaunchKernelGGL((k_cmean_sums<T, DX, DY>), dim3((qn + TILE - 1) / TILE, nch), dim3(TILE), 0,
                           stream, pts, n, chunk, xs, qn, a, (const double*)mq, part);
        hipLaunchKernelGGL(k_cmean_reduce, dim3((qn + 255) / 256), dim3(256), 0, stream,
                           (const double*)part, qn, DY, nch, mean + (size_t)q0 * DY);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

size_t cond_mean_work_doubles(const cde_model* m, int64_t q)
{
    const int chunk = mean_chunk_points(m->n);
    const int64_t nch = (m->n + chunk - 1) / chunk;
    const int64_t qs = mean_slice(q);
    return (size_t)(qs + nch * qs * (1 + m->dy) + 64);
}

#define CDE_MEAN_CASE(DX_, DY_)                                                                    \
    case (DX_) * 8 + (DY_):                                                                        \
        return m->prec == CDE_F64                                                                  \
                   ? cmean_t<double, DX_, DY_>(m, (const double*)xq, q, h, mean, work, stream)     \
                   : cmean_t<float, DX_, DY_>(m, (const float*)xq, q, h, mean, work, stream);

hipError_t launch_cond_mean(const cde_model* m, const void* xq, int64_t q, const double* h, double* mean,
                            double* work, hipStream_t stream)
{
    switch (m->dx * 8 + m->dy) {
        CDE_MEAN_CASE(1, 1) CDE_MEAN_CASE(1, 2) CDE_MEAN_CASE(2, 1) CDE_MEAN_CASE(2, 2)
        CDE_MEAN_CASE(3, 1) CDE_MEAN_CASE(3, 2) CDE_MEAN_CASE(4, 1) CDE_MEAN_CASE(4, 2)
        CDE_MEAN_CASE(5, 1) CDE_MEAN_CASE(5, 2) CDE_MEAN_CASE(6, 1) CDE_MEAN_CASE(6, 2)
        CDE_MEAN_CASE(7, 1) CDE_MEAN_CASE(7, 2) CDE_MEAN_CASE(8, 1) CDE_MEAN_CASE(8, 2)
        CDE_MEAN_CASE(16, 1) CDE_MEAN_CASE(16, 2)
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_density_summary(const double* f, const double* yg, int64_t q, int64_t k, double alpha,
                                  double* out, hipStream_t stream)
{
    hipLaunchKernelGGL(k_density_summary, dim3((unsigned)((q + 63) / 64)), dim3(64), 0, stream, f, yg, (int)q,
                       (int)k, alpha, out);
    return hipGetLastError();
}

}  // namespace cde
