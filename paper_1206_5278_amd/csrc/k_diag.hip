// k_diag.hip -- exact LOO log-likelihood, and optionally its bandwidth
// gradient, for diagonal (per-dimension) Gaussian bandwidths.
//
// Definitions (Holmes, Gray & Isbell): the scaled kernel of Section 2, the
// estimator of eq. (1), and the criterion of eq. (3) expanded as in
// Section 3.2 into, for each point i, num_i = sum_{j!=i} K_hx(x_i-x_j)
// K_hy(y_i-y_j) and den_i = sum_{j!=i} K_hx(x_i-x_j).  The gradient is the
// derivative of each log(num_i/den_i) with respect to the bandwidths; it needs
// the moments sum_j w dx_k^2, sum_j v dx_k^2 and sum_j v dy_l^2 (w the x-kernel,
// v the product kernel), which are accumulated beside num and den, so the
// adjoint costs one O(n^2) pass, not two.
//
// Work decomposition: one lane owns one point i (its coordinates, shifts and
// accumulators live in registers); a 256-lane block owns 256 consecutive
// points and streams all j through LDS in 256-point tiles, loaded with
// coalesced 16-byte rows and read back as wave-wide broadcasts.  blockIdx.y
// selects one of up to MAX_SETS_PER_LAUNCH bandwidth settings.
//
// Numerics (FP32 instance): each pair's exponent is formed from coordinate
// differences (no |x|^2 cancellation), kernel values are v_exp_f32 of that
// exponent relative to a per-point reference (a running minimum, so the
// largest term is about 1 and nothing overflows or underflows: den' >= 1 and
// num' >= 1 by construction), values are summed in FP32 over 32-point
// subtiles and the subtile partials are folded into Kahan-compensated totals.
// The reference is moved lazily, only when a subtile holds a term more than
// 2^32 above it; the subtile is then recomputed against the new reference and
// the totals rescaled, which is exact in real arithmetic (the common factor
// cancels in num/den).  The log of the ratio, the gradient combination and
// the sum over i run in FP64.

#include "cde_device.h"
#include "cde_kernels.h"

namespace cde {

namespace {

template <typename T, int DX, int DY, bool GRAD>
struct DiagLane {
    static constexpr int S = row_stride(DX, DY);
    static constexpr int GX = GRAD ? DX : 1;
    static constexpr int GY = GRAD ? DY : 1;
    static constexpr int SUB = 32;

    T xi[DX], yi[DY], cx[DX], cy[DY];
    T m, m2;  // references of the x-kernel sums and of the product-kernel sums
    Kahan<T> den, num, mw[GX], mv[GX], mvy[GY];

    __device__ __forceinline__ void init_accumulators()
    {
        den.zero();
        num.zero();
#pragma unroll
        for (int k = 0; k < GX; ++k) { mw[k].zero(); mv[k].zero(); }
#pragma unroll
        for (int l = 0; l < GY; ++l) mvy[l].zero();
    }

    // Base-2 exponents of the x-kernel and of the product kernel for one j.
    __device__ __forceinline__ void exponents(const T* pj, T& ex, T& exy) const
    {
        T e = T(0);
#pragma unroll
        for (int k = 0; k < DX; ++k) {
            T d = xi[k] - pj[k];
            e = fma_(d * d, cx[k], e);
        }
        T f = e;
#pragma unroll
        for (int l = 0; l < DY; ++l) {
            T d = yi[l] - pj[DX + l];
            f = fma_(d * d, cy[l], f);
        }
        ex = e;
        exy = f;
    }

    // Initial references: minima over the first points of the first tile.
    __device__ __forceinline__ void prologue(const T* tile, int len, int self)
    {
        T a = inf_<T>(), b = inf_<T>();
        for (int q = 0; q < len; ++q) {
            if (q == self) continue;
            T pj[S];
            load_row<S>(pj, tile + q * S);
            T ex, exy;
            exponents(pj, ex, exy);
            a = min_(a, ex);
            b = min_(b, exy);
        }
        m = a;
        m2 = b;
    }

    // One subtile of `len` points starting at tile row j0.  `self` is the
    // tile row of point i itself (diagonal tile) or -1.
    template <bool FULL, bool DIAG>
    __device__ __forceinline__ void subtile(const T* tile, int j0, int len, int self)
    {
        const T slack = sizeof(T) == 4 ? T(32) : T(512);
        for (;;) {
            T pden = T(0), pnum = T(0), pmw[GX], pmv[GX], pmvy[GY];
#pragma unroll
            for (int k = 0; k < GX; ++k) { pmw[k] = T(0); pmv[k] = T(0); }
#pragma unroll
            for (int l = 0; l < GY; ++l) pmvy[l] = T(0);
            T mn1 = inf_<T>(), mn2 = inf_<T>();
            const T dm = m - m2;
            const int L = FULL ? SUB : len;
#pragma unroll 8
            for (int q = 0; q < L; ++q) {
                const int jj = j0 + q;
                T pj[S];
                load_row<S>(pj, tile + jj * S);
                T sq[DX], sqy[DY];
                T e1 = -m;
#pragma unroll
                for (int k = 0; k < DX; ++k) {
                    T d = xi[k] - pj[k];
                    sq[k] = d * d;
                    e1 = fma_(sq[k], cx[k], e1);
                }
                T e2 = e1 + dm;
#pragma unroll
                for (int l = 0; l < DY; ++l) {
                    T d = yi[l] - pj[DX + l];
                    sqy[l] = d * d;
                    e2 = fma_(sqy[l], cy[l], e2);
                }
                if (DIAG) {
                    const bool me = (jj == self);
                    e1 = me ? inf_<T>() : e1;
                    e2 = me ? inf_<T>() : e2;
                }
                mn1 = min_(mn1, e1);
                mn2 = min_(mn2, e2);
                const T w = exp2_<T>(-e1);
                const T v = exp2_<T>(-e2);
                pden += w;
                pnum += v;
                if (GRAD) {
#pragma unroll
                    for (int k = 0; k < DX; ++k) {
                        pmw[k] = fma_(w, sq[k], pmw[k]);
                        pmv[k] = fma_(v, sq[k], pmv[k]);
                    }
#pragma unroll
                    for (int l = 0; l < DY; ++l) pmvy[l] = fma_(v, sqy[l], pmvy[l]);
                }
            }
            const bool need = (mn1 < -slack) || (mn2 < -slack);
            if (!__any(need)) {
                den.add(pden);
                num.add(pnum);
                if (GRAD) {
#pragma unroll
                    for (int k = 0; k < DX; ++k) { mw[k].add(pmw[k]); mv[k].add(pmv[k]); }
#pragma unroll
                    for (int l = 0; l < DY; ++l) mvy[l].add(pmvy[l]);
                }
                return;
            }
            // A much heavier term appeared: move the reference to it, rescale
            // the totals, and recompute this subtile against the new reference.
            if (mn1 < -slack) {
                const T f = exp2_<T>(mn1);
                den.scale(f);
#pragma unroll
                for (int k = 0; k < GX; ++k) mw[k].scale(f);
                m += mn1;
            }
            if (mn2 < -slack) {
                const T f = exp2_<T>(mn2);
                num.scale(f);
#pragma unroll
                for (int k = 0; k < GX; ++k) mv[k].scale(f);
#pragma unroll
                for (int l = 0; l < GY; ++l) mvy[l].scale(f);
                m2 += mn2;
            }
        }
    }
};

}  // namespace

template <typename T, int DX, int DY, bool GRAD>
__global__ __launch_bounds__(TILE) void k_loo_diag(const T* __restrict__ pts, int n,
                                                   DiagSets<T> sets, int crit,
                                                   double* __restrict__ per_point,
                                                   double* __restrict__ part)
{
    using L = DiagLane<T, DX, DY, GRAD>;
    constexpr int S = L::S;
    constexpr int P = DX + DY;
    constexpr int NV = GRAD ? P + 2 : 2;  // l_i, [gradient], non-finite count
    __shared__ T tile[TILE * S];
    __shared__ double red[4 * NV];

    const DiagSet<T>& st = sets.s[blockIdx.y];
    const int tid = threadIdx.x;
    const int i = blockIdx.x * TILE + tid;  // < npad: rows beyond n hold zeros

    L lane;
    {
        T own[S];
        load_row<S>(own, pts + (size_t)i * S);
#pragma unroll
        for (int k = 0; k < DX; ++k) { lane.xi[k] = own[k]; lane.cx[k] = st.c[k]; }
#pragma unroll
        for (int l = 0; l < DY; ++l) { lane.yi[l] = own[DX + l]; lane.cy[l] = st.c[DX + l]; }
    }
    lane.init_accumulators();

    const int ntiles = (n + TILE - 1) / TILE;
    T pre[S];
    load_row<S>(pre, pts + (size_t)tid * S);
    for (int t = 0; t < ntiles; ++t) {
        __syncthreads();
        store_row<S>(tile + tid * S, pre);
        __syncthreads();
        if (t + 1 < ntiles) load_row<S>(pre, pts + ((size_t)(t + 1) * TILE + tid) * S);
        const int cnt = min(TILE, n - t * TILE);
        const bool diag = (t == (int)blockIdx.x);
        const int self = diag ? tid : -1;
        if (t == 0) lane.prologue(tile, min(L::SUB, cnt), self);
        for (int j0 = 0; j0 < cnt; j0 += L::SUB) {
            const int len = min(L::SUB, cnt - j0);
            if (len == L::SUB) {
                if (diag) lane.template subtile<true, true>(tile, j0, len, self);
                else lane.template subtile<true, false>(tile, j0, len, self);
            } else {
                if (diag) lane.template subtile<false, true>(tile, j0, len, self);
                else lane.template subtile<false, false>(tile, j0, len, self);
            }
        }
    }

    // Per-point finalisation in FP64.
    const bool valid = i < n;
    const double D = lane.den.value(), U = lane.num.value();
    double v[NV];
    double ell;
    if (crit == CDE_COND)
        ell = log(U / D) + ((double)lane.m - (double)lane.m2) * LN2 + st.log_cy;
    else
        ell = log(U) - (double)lane.m2 * LN2 + st.log_cx + st.log_cy - log((double)(n - 1));
    v[0] = valid ? ell : 0.0;
    if (GRAD) {
#pragma unroll
        for (int k = 0; k < DX; ++k) {
            const double gv = lane.mv[k].value() / U;
            const double gw = lane.mw[k].value() / D;
            const double g = crit == CDE_COND ? (gv - gw) * st.inv_h3[k]
                                              : gv * st.inv_h3[k] - st.inv_h[k];
            v[1 + k] = valid ? g : 0.0;
        }
#pragma unroll
        for (int l = 0; l < DY; ++l) {
            const double g = (lane.mvy[l].value() / U) * st.inv_h3[DX + l] - st.inv_h[DX + l];
            v[1 + DX + l] = valid ? g : 0.0;
        }
    }
    v[NV - 1] = (valid && !isfinite(ell)) ? 1.0 : 0.0;
    if (per_point && valid) per_point[(size_t)blockIdx.y * n + i] = ell;

    block_sum<NV>(v, red);
    if (tid == 0) {
        double* o = part + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * NV;
#pragma unroll
        for (int q = 0; q < NV; ++q) o[q] = v[q];
    }
}

// Conditional density queries on FP64 models, eq. (1) over all n training
// points (no point left out): lane e of the flattened [q][k] output evaluates
// f(yg | xq) with the same shifted sums as the LOO pass, so den' >= 1 and
// num' >= 1 hold.  (FP32 models use the matrix-core kernel of k_query.hip.)
template <typename T, int DX, int DY>
__global__ __launch_bounds__(TILE) void k_query(const T* __restrict__ pts, int n,
                                                const T* __restrict__ xq,
                                                const T* __restrict__ yg, int64_t q, int64_t k,
                                                DiagSets<T> sets, double* __restrict__ f)
{
    using L = DiagLane<T, DX, DY, false>;
    constexpr int S = L::S;
    __shared__ T tile[TILE * S];
    const DiagSet<T>& st = sets.s[0];
    const int tid = threadIdx.x;
    const int64_t e = (int64_t)blockIdx.x * TILE + tid;
    const int64_t total = q * k;
    const int64_t ec = e < total ? e : total - 1;  // lanes past the end mirror the last pair
    const int64_t qq = ec / k, gg = ec - qq * k;

    L lane;
#pragma unroll
    for (int kk = 0; kk < DX; ++kk) { lane.xi[kk] = xq[qq * DX + kk]; lane.cx[kk] = st.c[kk]; }
#pragma unroll
    for (int l = 0; l < DY; ++l) { lane.yi[l] = yg[gg * DY + l]; lane.cy[l] = st.c[DX + l]; }
    lane.init_accumulators();

    const int ntiles = (n + TILE - 1) / TILE;
    T pre[S];
    load_row<S>(pre, pts + (size_t)tid * S);
    for (int t = 0; t < ntiles; ++t) {
        __syncthreads();
        store_row<S>(tile + tid * S, pre);
        __syncthreads();
        if (t + 1 < ntiles) load_row<S>(pre, pts + ((size_t)(t + 1) * TILE + tid) * S);
        const int cnt = min(TILE, n - t * TILE);
        if (t == 0) lane.prologue(tile, min(L::SUB, cnt), -1);
        for (int j0 = 0; j0 < cnt; j0 += L::SUB) {
            const int len = min(L::SUB, cnt - j0);
            if (len == L::SUB) lane.template subtile<true, false>(tile, j0, len, -1);
            else lane.template subtile<false, false>(tile, j0, len, -1);
        }
    }
    if (e < total) {
        const double D = lane.den.value(), U = lane.num.value();
        f[e] = exp(log(U / D) + ((double)lane.m - (double)lane.m2) * LN2 + st.log_cy);
    }
}

template <typename T, int DX, int DY>
static hipError_t launch_query_t(const cde_model* m, const T* xq, int64_t q, const T* yg, int64_t k,
                                 const DiagSets<T>& sets, double* f, hipStream_t stream)
{
    const int64_t total = q * k;
    const unsigned blocks = (unsigned)((total + TILE - 1) / TILE);
    hipLaunchKernelGGL((k_query<T, DX, DY>), dim3(blocks), dim3(TILE), 0, stream,
                       (const T*)m->pts, (int)m->n, xq, yg, q, k, sets, f);
    return hipGetLastError();
}

#define CDE_QUERY_CASE(DX_, DY_) \
    case (DX_) * 8 + (DY_): return launch_query_t<T, DX_, DY_>(m, xq, q, yg, k, sets, f, stream);

template <typename T>
hipError_t launch_query(const cde_model* m, const T* xq, int64_t q, const T* yg, int64_t k,
                        const DiagSets<T>& sets, double* f, hipStream_t stream)
{
    switch (m->dx * 8 + m->dy) {
        CDE_QUERY_CASE(1, 1) CDE_QUERY_CASE(1, 2) CDE_QUERY_CASE(2, 1) CDE_QUERY_CASE(2, 2)
        CDE_QUERY_CASE(3, 1) CDE_QUERY_CASE(3, 2) CDE_QUERY_CASE(4, 1) CDE_QUERY_CASE(4, 2)
        CDE_QUERY_CASE(5, 1) CDE_QUERY_CASE(5, 2) CDE_QUERY_CASE(6, 1) CDE_QUERY_CASE(6, 2)
        CDE_QUERY_CASE(7, 1) CDE_QUERY_CASE(7, 2) CDE_QUERY_CASE(8, 1) CDE_QUERY_CASE(8, 2)
        CDE_QUERY_CASE(16, 1) CDE_QUERY_CASE(16, 2)
        default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_query<float>(const cde_model*, const float*, int64_t, const float*, int64_t,
                                        const DiagSets<float>&, double*, hipStream_t);
template hipError_t launch_query<double>(const cde_model*, const double*, int64_t, const double*,
                                         int64_t, const DiagSets<double>&, double*, hipStream_t);

template <typename T, int DX, int DY, bool GRAD>
static hipError_t launch_diag_t(const cde_model* m, const DiagSets<T>& sets, int nsets, int crit,
                                double* per_point, double* part, hipStream_t stream)
{
    dim3 grid((unsigned)(m->npad / TILE), (unsigned)nsets);
    hipLaunchKernelGGL((k_loo_diag<T, DX, DY, GRAD>), grid, dim3(TILE), 0, stream,
                       (const T*)m->pts, (int)m->n, sets, crit, per_point, part);
    return hipGetLastError();
}

#define CDE_DIAG_CASE(DX_, DY_)                                                            \
    case (DX_) * 8 + (DY_):                                                                \
        return grad ? launch_diag_t<T, DX_, DY_, true>(m, sets, nsets, crit, per_point, part, \
                                                       stream)                             \
                    : launch_diag_t<T, DX_, DY_, false>(m, sets, nsets, crit, per_point,   \
                                                        part, stream);

template <typename T>
hipError_t launch_diag(const cde_model* m, const DiagSets<T>& sets, int nsets, int crit, bool grad,
                       double* per_point, double* part, hipStream_t stream)
{
    switch (m->dx * 8 + m->dy) {
        CDE_DIAG_CASE(1, 1) CDE_DIAG_CASE(1, 2) CDE_DIAG_CASE(2, 1) CDE_DIAG_CASE(2, 2)
        CDE_DIAG_CASE(3, 1) CDE_DIAG_CASE(3, 2) CDE_DIAG_CASE(4, 1) CDE_DIAG_CASE(4, 2)
        CDE_DIAG_CASE(5, 1) CDE_DIAG_CASE(5, 2) CDE_DIAG_CASE(6, 1) CDE_DIAG_CASE(6, 2)
        CDE_DIAG_CASE(7, 1) CDE_DIAG_CASE(7, 2) CDE_DIAG_CASE(8, 1) CDE_DIAG_CASE(8, 2)
        CDE_DIAG_CASE(16, 1) CDE_DIAG_CASE(16, 2)
        default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_diag<float>(const cde_model*, const DiagSets<float>&, int, int, bool,
                                       double*, double*, hipStream_t);
template hipError_t launch_diag<double>(const cde_model*, const DiagSets<double>&, int, int, bool,
                                        double*, double*, hipStream_t);

}  // namespace cde
