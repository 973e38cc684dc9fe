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
//     more than 1e-12 of the span).  One wave per row: the running sums and
//     the tie rule's scan over the candidates stay sequential (lane 0, in the
//     scalar order), the candidates are evaluated by all lanes, and the
//     inverse of the (non-decreasing) grid CDF is a binary search that finds
//     the node the scalar definition's forward-moving pointer finds.
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
        c32[k] = vreg((float)a.cx[k]);  // vector operands: the FMAs dual-issue
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
            auto d32 = [&](const float* pj) {
                float e32 = (xo32[0] - pj[0]) * (xo32[0] - pj[0]) * c32[0];
#pragma unroll
                for (int k = 1; k < DX; ++k) {
                    const float d = xo32[k] - pj[k];
                    e32 = fmaf(d * d, c32[k], e32);
                }
                return e32;
            };
            // four rows per branch, screened in order inside (as one at a time)
            int j = 0;
            for (; j + 4 <= cnt; j += 4) {
                float e4[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) e4[u] = d32(tile + (j + u) * S);
                if (screen.passes(fminf(fminf(e4[0], e4[1]), fminf(e4[2], e4[3])))) {
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        if (screen.candidate(e4[u])) best = fmin(best, xdist<T, DX>(xo, tile + (j + u) * S, a));
                }
            }
            for (; j < cnt; ++j) {
                if (screen.candidate(d32(tile + j * S))) best = fmin(best, xdist<T, DX>(xo, tile + j * S, a));
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
    __shared__ double tile[TILE * S];  // staged as doubles: one exact conversion per row
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
        double pd[S];
#pragma unroll
        for (int c = 0; c < S; ++c) pd[c] = (double)pre[c];
        store_row<S>(tile + tid * S, pd);
        __syncthreads();
        const int cnt = min(TILE, j1 - t0);
        for (int j = 0; j < cnt; ++j) {
            const double* pj = tile + j * S;
            const double w = exp(m - xdist<double, DX>(xo, pj, a));
            D += w;
#pragma unroll
            for (int l = 0; l < DY; ++l) Sy[l] = fma(w, pj[DX + l], Sy[l]);
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

// Density summary, one wave per row (see the file header).  Rows are
// densities (f >= 0), so the grid CDF C[g] / mass is non-decreasing: the
// inverse the scalar definition finds with a pointer that only moves
// forward is the first node g with C[g] / mass >= target (at most k - 1),
// found here by a binary search over the same values.  What decides bits
// stays sequential: lane 0 forms the running sums C[g] in the scalar order
// (the same additions as the mass), and lane 0 scans the candidate widths
// in candidate order for the tie rule.  The mode is a first-index argmax
// over the wave (exact).  Candidate evaluation runs on all 64 lanes.
// LDS per block: yg [k], then per row C [k] and the candidate widths [2k].
__device__ __forceinline__ int first_at_least(const double* G, int k, double target)
{
    // smallest g in [0, k-1) with G[g] >= target, else k - 1
    int lo = 0, hi = k - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (G[mid] < target)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// Interval of candidate c (c < k: lower end on node c; else upper end on
// node c - k) on the grid CDF G[g] = C[g] / mass (the quotients the scalar
// definition forms); returns false when the candidate is not admitted.
__device__ __forceinline__ bool summary_candidate(const double* G, const double* yg, int k, double cover,
                                                  int c, double& lo, double& hi)
{
#pragma clang fp contract(off)
    const int pass = c >= k, a = pass ? c - k : c;
    const double Ga = G[a];
    const double target = pass == 0 ? Ga + cover : Ga - cover;
    if (pass == 0 && target > 1.0) return false;
    if (pass == 1 && target < 0.0) return false;
    const int ptr = first_at_least(G, k, target);
    const double Gp = G[ptr], Gpm = ptr > 0 ? G[ptr - 1] : 0.0;
    double y;
    if (ptr == 0 || Gp <= Gpm)
        y = yg[ptr];
    else
        y = yg[ptr - 1] + (target - Gpm) / (Gp - Gpm) * (yg[ptr] - yg[ptr - 1]);
    lo = pass == 0 ? yg[a] : y;
    hi = pass == 0 ? y : yg[a];
    return true;
}

// LDS of the summary kernel (doubles, sized per launch): the y grid [k]
// when YLDS (k <= 2048; larger grids are read from global memory), then per
// row the running sums C [k] and one chunk of candidate widths [SUMMARY_WCH].
constexpr int SUMMARY_WCH = 256;

// Within one wave: LDS writes of some lanes are visible to the reads that
// follow them in program order.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <bool YLDS>
__global__ __launch_bounds__(256) void k_density_summary(const double* __restrict__ f,
                                                         const double* __restrict__ yg, int q, int k,
                                                         int rows_per_block, double alpha,
                                                         double* __restrict__ out)
{
#pragma clang fp contract(off)  // the same roundings as the plain scalar definition
    extern __shared__ double sm[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const double* ysh = yg;
    if (YLDS) {
        for (int g = tid; g < k; g += blockDim.x) sm[g] = yg[g];
        ysh = sm;
    }
    __syncthreads();  // the only block-wide barrier: everything below is per wave
    const int row = blockIdx.x * rows_per_block + wave;
    if (row >= q) return;
    double* C = sm + (YLDS ? k : 0) + (size_t)wave * (k + SUMMARY_WCH);
    double* wid = C + k;
    const double* r = f + (size_t)row * k;
    double* o = out + (size_t)row * 4;
    // stage the row (coalesced)
    for (int g = lane; g < k; g += 64) C[g] = r[g];
    wave_sync();
    // mode: first index of the maximum, as the scalar scan from r[0] finds it
    double bv = -__builtin_inf();
    int bi = 0;
    for (int g = lane; g < k; g += 64) {
        const double v = C[g];
        if (v > bv) {
            bv = v;
            bi = g;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(bv, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        if (ov > bv || (ov == bv && oi < bi)) {
            bv = ov;
            bi = oi;
        }
    }
    const double r0 = C[0];
    // the scalar scan starts at r[0] and moves only on a strictly larger value
    const int imax = (r0 != r0 || !(bv > r0)) ? 0 : bi;
    wave_sync();
    // running sums in the scalar order, in place (lane 0)
    if (lane == 0) {
        double c = 0.0, prev = C[0];
        C[0] = 0.0;
#pragma unroll 8
        for (int g = 0; g + 1 < k; ++g) {
            const double cur = C[g + 1];
            c += (prev + cur) * 0.5 * (ysh[g + 1] - ysh[g]);
            C[g + 1] = c;
            prev = cur;
        }
    }
    wave_sync();
    const double mass = C[k - 1];
    if (lane == 0) {
        o[0] = mass;
        o[1] = ysh[imax];
    }
    if (!(mass > 0.0)) {
        if (lane == 0) o[2] = o[3] = __builtin_nan("");
        return;
    }
    wave_sync();  // every lane holds mass before C becomes G
    for (int g = lane; g < k; g += 64) C[g] = C[g] / mass;
    wave_sync();
    const double cover = 1.0 - alpha;
    const double tie = 1e-12 * (ysh[k - 1] - ysh[0]);
    double best = __builtin_inf();
    int win = -1;
    for (int c0 = 0; c0 < 2 * k; c0 += SUMMARY_WCH) {
        const int cn = min(SUMMARY_WCH, 2 * k - c0);
        for (int e = lane; e < cn; e += 64) {
            double lo, hi;
            wid[e] = summary_candidate(C, ysh, k, cover, c0 + e, lo, hi) ? hi - lo : __builtin_nan("");
        }
        wave_sync();
        if (lane == 0) {
            // candidate order: the first of least width; a later one only
            // when narrower by more than tie
#pragma unroll 8
            for (int e = 0; e < cn; ++e) {
                const double w = wid[e];
                if (w == w && w < best - tie) {
                    best = w;
                    win = c0 + e;
                }
            }
        }
        wave_sync();
    }
    if (lane == 0) {
        double lo = __builtin_nan(""), hi = __builtin_nan("");
        if (win >= 0) summary_candidate(C, ysh, k, cover, win, lo, hi);
        o[2] = lo;
        o[3] = hi;
    }
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
    if (q == 0) return hipSuccess;
    // rows per block (one wave each): 4, 2 or 1, within 64 KiB of LDS
    const bool ylds = k <= 2048;
    const int64_t base = ylds ? k : 0, per_row = k + SUMMARY_WCH;
    int rpb = 4;
    while (rpb > 1 && (base + rpb * per_row) * (int64_t)sizeof(double) > 65536) rpb /= 2;
    const size_t lds = (size_t)(base + rpb * per_row) * sizeof(double);
    const dim3 grid((unsigned)((q + rpb - 1) / rpb)), block(64 * rpb);
    if (ylds)
        hipLaunchKernelGGL(k_density_summary<true>, grid, block, lds, stream, f, yg, (int)q, (int)k, rpb, alpha,
                           out);
    else
        hipLaunchKernelGGL(k_density_summary<false>, grid, block, lds, stream, f, yg, (int)q, (int)k, rpb,
                           alpha, out);
    return hipGetLastError();
}

}  // namespace cde
