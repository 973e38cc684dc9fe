// k_ise.hip -- exact cross-validated integrated squared error on the matrix
// cores (FP32 models, Gaussian product kernels, one diagonal setting).
//
// Holmes, Gray & Isbell, Section 3: the ISE of eq. (2) has the
// cross-validated estimate (1/n) sum_i T1_i - (2/n) sum_i T2_i with
//     T1_i = integral over y of f^{-i}(y|x_i)^2,   T2_i = f^{-i}(y_i|x_i).
// With w_ij the x-kernel weights of eq. (1) (j != i), the square of the
// mixture integrates in closed form: the product of two Gaussian y-kernels
// centred at y_j and y_l integrates to the Gaussian of standard deviation
// sqrt(2) hy at y_j - y_l, so
//     T1_i = c_G sum_{j != i} sum_{l != i} w_ij w_il G(y_j - y_l) / W_i^2,
//     G(t) = 2^-(sum_d t_d^2 log2(e) / (4 hy_d^2)),  c_G = prod_d 1 / (2 sqrt(pi) hy_d),
// W_i = sum_{j != i} w_ij.  The double sum is O(n^2) per point, O(n^3) in all
// (the cost the paper cites for leaving this criterion aside), and it is a
// dense contraction:  Q_i = sum_l w_il M_il  with  M = W G  (W the x-kernel
// matrix with a zero diagonal, G the symmetric y-convolution matrix).
//
// k_ise_mfma: a 512-lane block owns 128 rows i and 256 columns l, and runs
// over all training points j.  For each panel of 32 j the block writes to LDS
// the x-kernel values w'(i, j) of its 128 rows (zero for j = i) and G'(j, l)
// of its 256 columns, each formed once per block; wave w then takes rows
// 32 (w % 4) .. and the columns of half w / 4, and runs 2-point
// v_mfma_f32_32x32x2f32 steps (A = w', lane % 32 = row, lane / 32 = j;
// B = G', lane / 32 = j, lane % 32 = column).  Every 8 tiles of j (64
// panels, FP32 sums) the block folds sum_l w'(i, l) M_il into FP64 row sums
// (w'(i, i) = 0 leaves l = i out).  Row sums of the column halves and of the
// column blocks are combined in a fixed order.
//
// Shifts: w'(i, j) = 2^-(d2x(i, j) - m_i) with m_i the exact FP64 minimum
// over j != i (prepass k_ise_shift), so the nearest point has w' = 1 up to
// one rounding, W'_i >= 1 and Q'_i >= 1 (its own j = l term); the common
// factor cancels in Q_i / W_i^2.  G' needs no shift (G <= 1 = G(0)).
// Exponents are formed in FP64 and rounded once to FP32.
#include <algorithm>

#include "cde_device.h"
#include "cde_kernels.h"

namespace cde {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));

constexpr float IEXCL = 1e20f;     // exponent of an excluded pair (2^-1e20 = 0)
constexpr int IWAVES = 8;          // waves per block
constexpr int INT = 64 * IWAVES;   // threads per block
constexpr int IPB = 128;           // rows i per block
constexpr int IGW = 256;           // columns l per block
constexpr int ISEG = 8;            // tiles of j per FP64 fold

struct IseArgs {
    double cx[16];  // log2(e) / (2 hx_k^2)
    double cg[4];   // log2(e) / (4 hy_l^2)
    double sx[16];  // sqrt(cx_k): coordinate scales of the main kernel
    double sg[4];   // sqrt(cg_l)
};

__device__ __forceinline__ void atomic_min_nonneg(double* p, double v)
{
    // non-negative doubles order like their bit patterns
    atomicMin((unsigned long long*)p, (unsigned long long)__double_as_longlong(v));
}

__global__ void k_ise_fill_inf(double* p, int cnt)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cnt) p[i] = __builtin_inf();
}

template <int DX>
__device__ __forceinline__ double xdist2(const double* xo, const double* pj, const IseArgs& a)
{
    double d2 = 0.0;
#pragma unroll
    for (int k = 0; k < DX; ++k) {
        const double d = xo[k] - pj[k];
        d2 = fma_(d * d, a.cx[k], d2);
    }
    return d2;
}

// Squared distance of pre-scaled coordinates (each multiplied by the square
// root of its c in FP64), started from -shift: a difference and an FMA per
// dimension.  The scaling rounds each coordinate once (relative 2^-53); the
// exponent is rounded to FP32 afterwards, far above that.  The shift is the
// exact minimum of the unscaled form, so the nearest pair's exponent can fall
// a few ulps below 0, which is harmless.
template <int N>
__device__ __forceinline__ double sdist2_shifted(const double* o, const double* pj, double shift)
{
    double e = -shift;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const double d = o[k] - pj[k];
        e = fma_(d, d, e);
    }
    return e;
}

// A training row staged in LDS as doubles scaled by sqrt(c): x by sx, y by sg.
template <int DX, int DY>
__device__ __forceinline__ void stage_tile_scaled(double* tile, const float* pre, int tid, const IseArgs& a)
{
#pragma unroll
    for (int d = 0; d < DX; ++d) tile[tid * (DX + DY) + d] = (double)pre[d] * a.sx[d];
#pragma unroll
    for (int l = 0; l < DY; ++l) tile[tid * (DX + DY) + DX + l] = (double)pre[DX + l] * a.sg[l];
}

template <int DX, int DY>
__device__ __forceinline__ void stage_tile(double* tile, const float* pre, int tid)
{
#pragma unroll
    for (int d = 0; d < DX + DY; ++d) tile[tid * (DX + DY) + d] = (double)pre[d];
}

// m_i = min_{j != i} d2x(i, j) (FP64): lane = point i, blockIdx.y = range of j.
template <int DX, int DY>
__global__ __launch_bounds__(TILE) void k_ise_shift(const float* __restrict__ pts, int n, int chunk,
                                                    IseArgs a, double* __restrict__ mi)
{
    constexpr int S = row_stride(DX, DY), SD = DX + DY;
    __shared__ double tile[TILE * SD];
    const int tid = threadIdx.x;
    const int i = blockIdx.x * TILE + tid;
    const int ic = i < n ? i : n - 1;
    double xo[DX];
#pragma unroll
    for (int k = 0; k < DX; ++k) xo[k] = (double)pts[(size_t)ic * S + k];
    double best = __builtin_inf();
    const int j0 = blockIdx.y * chunk, j1 = min(n, j0 + chunk);
    for (int t0 = j0; t0 < j1; t0 += TILE) {
        __syncthreads();
        float pre[S];
        load_row<S>(pre, pts + ((size_t)t0 + tid) * S);
        stage_tile<DX, DY>(tile, pre, tid);
        __syncthreads();
        const int cnt = min(TILE, j1 - t0);
        for (int j = 0; j < cnt; ++j) {
            const double d = xdist2<DX>(xo, tile + j * SD, a);
            best = t0 + j == i ? best : min_(best, d);
        }
    }
    if (i < n) atomic_min_nonneg(mi + i, best);
}

// Row sums Q'_i over the block's 256 columns (qpart[blockIdx.y][i]) and, in
// column block 0, W'_i (den[i]); see the file header.
template <int DX, int DY>
__global__ __launch_bounds__(INT) void k_ise_mfma(const float* __restrict__ pts, int n, IseArgs a,
                                                  const double* __restrict__ mi,
                                                  double* __restrict__ qpart, double* __restrict__ den)
{
    constexpr int S = row_stride(DX, DY), SD = DX + DY;
    constexpr int GWW = IGW / 2;                          // columns per wave
    constexpr int GT = GWW / 32;                          // column tiles of 32 per wave
    constexpr int SUB = 32;                               // j per panel
    // LDS rows padded by 32 floats: the two 32-lane halves of a wave, which
    // read consecutive rows, start 128 bytes apart in the banks.
    constexpr int YS = IGW + 32, XS = IPB + 32;
    constexpr int YSTEP = INT / IGW, YPT = SUB / YSTEP;  // G panel rows: per pass, per thread
    constexpr int XSTEP = INT / IPB, XPT = SUB / XSTEP;  // w panel rows: per pass, per thread
    static_assert(GT == 4 && SUB % YSTEP == 0 && SUB % XSTEP == 0, "panel shape");
    static_assert(SUB * XS >= 2 * INT, "the w panel holds the denominator reduction");
    __shared__ double tile[TILE * SD];
    __shared__ __align__(16) float ykv[SUB * YS];  // [j][position]; position = half, then 4 n + t
    __shared__ __align__(16) float xkv[SUB * XS];  // [j][row]
    __shared__ double xrow[IPB * DX];
    __shared__ double mrow[IPB];
    __shared__ double xcol[IGW * DX];
    __shared__ double qrow[2 * IPB];  // [column half][row]: folded row sums
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int i0 = blockIdx.x * IPB, l0 = blockIdx.y * IGW;

    for (int v = tid; v < IPB; v += INT) {
        const int i = min(i0 + v, n - 1);
#pragma unroll
        for (int k = 0; k < DX; ++k) xrow[v * DX + k] = (double)pts[(size_t)i * S + k] * a.sx[k];
        mrow[v] = mi[i];
        qrow[v] = 0.0;
        qrow[IPB + v] = 0.0;
    }
    for (int v = tid; v < IGW; v += INT) {
        const int l = min(l0 + v, n - 1);
#pragma unroll
        for (int k = 0; k < DX; ++k) xcol[v * DX + k] = (double)pts[(size_t)l * S + k] * a.sx[k];
    }

    // w panel role: row i0 + tid % IPB, panel rows tid / IPB + XSTEP r
    const int wcol = tid % IPB, wrow = tid / IPB;
    const int wi = i0 + wcol;
    const int wc = min(wi, n - 1);
    double xo[DX];
#pragma unroll
    for (int k = 0; k < DX; ++k) xo[k] = (double)pts[(size_t)wc * S + k] * a.sx[k];
    const double m_q = mi[wc];
    // G panel role: LDS position tid % IGW, panel rows tid / IGW + YSTEP r.
    // Position h GWW + 4 n + t holds column h GWW + 32 t + n, so a lane of
    // half h reads its four column tiles' values as one vector.
    const int ypos = tid % IGW, yrow = tid / IGW;
    const int yh = ypos / GWW, yr = ypos % GWW;
    const int gl = min(l0 + yh * GWW + 32 * (yr % GT) + yr / GT, n - 1);
    double yo[DY];
#pragma unroll
    for (int l = 0; l < DY; ++l) yo[l] = (double)pts[(size_t)gl * S + DX + l] * a.sg[l];
    // MFMA role: rows 32 (wave % 4) .., columns of half wave / 4
    const int qg = wave & 3, half = wave >> 2;
    const int kr = lane >> 5, m32 = lane & 31;
    const float* arow = xkv + kr * XS + 32 * qg + m32;
    const float* brow = ykv + kr * YS + half * GWW + GT * m32;

    float tot[GT][16];
#pragma unroll
    for (int t = 0; t < GT; ++t)
#pragma unroll
        for (int r = 0; r < 16; ++r) tot[t][r] = 0.f;
    double dtot = 0.0;

    const bool stager = tid < TILE;
    float pre[S];
    if (stager) load_row<S>(pre, pts + (size_t)tid * S);
    const int ntiles = (n + TILE - 1) / TILE;
    for (int tt = 0; tt < ntiles; ++tt) {
        const int t0 = tt * TILE;
        __syncthreads();
        if (stager) {
            stage_tile_scaled<DX, DY>(tile, pre, tid, a);
            if (tt + 1 < ntiles) load_row<S>(pre, pts + ((size_t)t0 + TILE + tid) * S);
        }
        const int cnt = min(TILE, n - t0);
        float dp = 0.f;
        for (int s0 = 0; s0 < cnt; s0 += SUB) {
            __syncthreads();  // tile staged / previous panel read by every wave
#pragma unroll
            for (int r = 0; r < YPT; ++r) {
                const int p = yrow + YSTEP * r;
                const float e = (float)sdist2_shifted<DY>(yo, tile + (s0 + p) * SD + DX, 0.0);
                ykv[p * YS + ypos] = exp2_<float>(-e);
            }
            // w'(i, j), zero for j = i and for rows past cnt
#pragma unroll
            for (int r = 0; r < XPT; ++r) {
                const int p = wrow + XSTEP * r;
                const double d2 = sdist2_shifted<DX>(xo, tile + (s0 + p) * SD, m_q);
                const float w = exp2_<float>(-((s0 + p < cnt && t0 + s0 + p != wi) ? (float)d2 : IEXCL));
                dp += w;
                xkv[p * XS + wcol] = w;
            }
            __syncthreads();
            v16f acc[GT];
#pragma unroll
            for (int s = 0; s < SUB; s += 2) {
                const float av = arow[s * XS];
                const v4f b = *(const v4f*)(brow + s * YS);
#pragma unroll
                for (int t = 0; t < GT; ++t)
                    acc[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, b[t], s == 0 ? v16f{} : acc[t], 0, 0, 0);
            }
#pragma unroll
            for (int t = 0; t < GT; ++t)
#pragma unroll
                for (int r = 0; r < 16; ++r) tot[t][r] += acc[t][r];
        }
        dtot += (double)dp;
        if (tt % ISEG == ISEG - 1 || tt + 1 == ntiles) {
            // fold: qrow[half][i] += sum over the wave's columns l of
            // M(i, l) w'(i, l).  f32 32x32x2 result layout: register r of lane
            // l holds row 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32.
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int ir = 32 * qg + 8 * (r >> 2) + 4 * kr + (r & 3);
                const int gi = i0 + ir;
                double s = 0.0;
#pragma unroll
                for (int t = 0; t < GT; ++t) {
                    const int lc = half * GWW + 32 * t + m32;
                    const int l = l0 + lc;
                    const double e = sdist2_shifted<DX>(xrow + ir * DX, xcol + lc * DX, mrow[ir]);
                    const float wil = (l < n && l != gi) ? exp2_<float>(-(float)e) : 0.f;
                    s = fma_((double)tot[t][r], (double)wil, s);
                    tot[t][r] = 0.f;
                }
                // the row's 32 lanes of this half, in a fixed butterfly
                s += __shfl_xor(s, 1, 64);
                s += __shfl_xor(s, 2, 64);
                s += __shfl_xor(s, 4, 64);
                s += __shfl_xor(s, 8, 64);
                s += __shfl_xor(s, 16, 64);
                if (m32 == 0) qrow[half * IPB + ir] += s;  // one writer per entry
                // keep the weight evaluations of different rows from being
                // hoisted together (register pressure)
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
    // W'_i of row wi: the XSTEP row groups in a fixed order; Q'_i: the two
    // column halves in order
    double* red = (double*)xkv;
    __syncthreads();
    red[wrow * IPB + wcol] = dtot;
    __syncthreads();
    if (tid < IPB && i0 + tid < n) {
        qpart[(size_t)blockIdx.y * n + i0 + tid] = qrow[tid] + qrow[IPB + tid];
        if (blockIdx.y == 0) {
            double dsum = red[tid];
#pragma unroll
            for (int r = 1; r < XSTEP; ++r) dsum += red[r * IPB + tid];
            den[i0 + tid] = dsum;
        }
    }
}

// T1_i = c_G Q'_i / W'_i^2 (column blocks summed in order), T2_i = exp(l_i)
// from the conditional LOO log-likelihood; terms[i] = {T1_i, T2_i}.
__global__ void k_ise_terms(const double* __restrict__ qpart, int nlb, const double* __restrict__ den,
                            const double* __restrict__ ell, int n, double cgn,
                            double* __restrict__ terms)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double q = 0.0;
    for (int b = 0; b < nlb; ++b) q += qpart[(size_t)b * n + i];
    const double w = den[i];
    terms[2 * (size_t)i] = cgn * q / (w * w);
    terms[2 * (size_t)i + 1] = exp(ell[i]);
}

// out = {mean T1 - 2 mean T2, mean T1, mean T2}: one block; thread t sums
// points t, t + 256, ... in order, then a fixed tree.
__global__ __launch_bounds__(256) void k_ise_total(const double* __restrict__ terms, int n,
                                                   double* __restrict__ out)
{
    __shared__ double s1[256], s2[256];
    const int t = threadIdx.x;
    double a = 0.0, b = 0.0;
    for (int i = t; i < n; i += 256) {
        a += terms[2 * (size_t)i];
        b += terms[2 * (size_t)i + 1];
    }
    s1[t] = a;
    s2[t] = b;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
            s1[t] += s1[t + w];
            s2[t] += s2[t + w];
        }
        __syncthreads();
    }
    if (t == 0) {
        const double m1 = s1[0] / n, m2 = s2[0] / n;
        out[0] = m1 - 2.0 * m2;
        out[1] = m1;
        out[2] = m2;
    }
}

template <int DX, int DY>
hipError_t ise_t(const cde_model* m, const double* h, const double* ell, double* out, double* terms,
                 double* work, hipStream_t stream)
{
    IseArgs a;
    for (int k = 0; k < 16; ++k) {
        a.cx[k] = k < DX ? LOG2E / (2.0 * h[k] * h[k]) : 0.0;
        a.sx[k] = sqrt(a.cx[k]);
    }
    double cgn = 1.0;
    for (int l = 0; l < 4; ++l) {
        a.cg[l] = l < DY ? LOG2E / (4.0 * h[DX + l] * h[DX + l]) : 0.0;
        a.sg[l] = sqrt(a.cg[l]);
        if (l < DY) cgn /= 2.0 * 1.7724538509055160273 * h[DX + l];  // 2 sqrt(pi) hy
    }
    const int n = (int)m->n;
    const float* pts = (const float*)m->pts;
    const int nlb = (n + IGW - 1) / IGW;
    double* mi = work;
    double* den = mi + n;
    double* qpart = den + n;
    const int sch = 16 * TILE;
    hipLaunchKernelGGL(k_ise_fill_inf, dim3((n + 255) / 256), dim3(256), 0, stream, mi, n);
    hipLaunchKernelGGL((k_ise_shift<DX, DY>), dim3((n + TILE - 1) / TILE, (n + sch - 1) / sch), dim3(TILE),
                       0, stream, pts, n, sch, a, mi);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_ise_mfma<DX, DY>), dim3((n + IPB - 1) / IPB, nlb), dim3(INT), 0, stream, pts, n,
                       a, (const double*)mi, qpart, den);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_ise_terms, dim3((n + 255) / 256), dim3(256), 0, stream, (const double*)qpart, nlb,
                       (const double*)den, ell, n, cgn, terms);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_ise_total, dim3(1), dim3(256), 0, stream, (const double*)terms, n, out);
    return hipGetLastError();
}

}  // namespace

size_t ise_work_doubles(const cde_model* m)
{
    const int64_t nlb = (m->n + IGW - 1) / IGW;
    return (size_t)(2 * m->n + nlb * m->n + 64);
}

#define CDE_ISE_CASE(DX_, DY_) \
    case (DX_) * 8 + (DY_): return ise_t<DX_, DY_>(m, h, ell, out, terms, work, stream);

hipError_t launch_cv_ise(const cde_model* m, const double* h, const double* ell, double* out,
                         double* terms, double* work, hipStream_t stream)
{
    switch (m->dx * 8 + m->dy) {
        CDE_ISE_CASE(1, 1) CDE_ISE_CASE(1, 2) CDE_ISE_CASE(2, 1) CDE_ISE_CASE(2, 2)
        CDE_ISE_CASE(3, 1) CDE_ISE_CASE(3, 2) CDE_ISE_CASE(4, 1) CDE_ISE_CASE(4, 2)
        CDE_ISE_CASE(5, 1) CDE_ISE_CASE(5, 2) CDE_ISE_CASE(6, 1) CDE_ISE_CASE(6, 2)
        CDE_ISE_CASE(7, 1) CDE_ISE_CASE(7, 2) CDE_ISE_CASE(8, 1) CDE_ISE_CASE(8, 2)
        CDE_ISE_CASE(16, 1) CDE_ISE_CASE(16, 2)
        default: return hipErrorInvalidValue;
    }
}

}  // namespace cde
