// k_query.hip -- conditional density queries on the matrix cores (FP32 models).
//
// Eq. (1) of Holmes, Gray & Isbell over all n training points:
//     f(y_g | x_q) = sum_i K_hx(x_q - x_i) K_hy(y_g - y_i) / sum_i K_hx(x_q - x_i).
// For a batch of queries q and a shared grid of y values g, the numerator is
//     F[q][g] = sum_i w(q, i) k(i, g),
// a dense contraction over the training points of a [Q x n] matrix of
// x-kernels with an [n x k] matrix of y-kernels.  It runs on
// v_mfma_f32_32x32x2f32: per training point, one x-kernel value per query and
// one y-kernel value per grid point are formed on the VALU (not one product
// kernel per (q, g)).
//
// Shifts: w' = 2^-(d2x(q,i) - m_q), k' = 2^-(d2y(g,i) - mu_g), with m_q the
// smallest scaled x-distance of query q to the data and mu_g the smallest
// scaled y-distance of grid point g (FP64 prepasses; exact minima, so the
// nearest point has w' = 1 up to one rounding and den' >= 1).  The shifted
// exponents are formed in FP64 (each sum starts from the negated shift) and
// rounded once to FP32.  Kernel values and products are FP32 (see
// k_query_mfma for the sums).  A value of f more than ~2^-100 below its
// query's peak is not carried to full relative precision (FP32 range); such
// tail values are far below the accuracy floor of a density estimate.
//
// Work decomposition: a 512-lane block owns 128 queries, a chunk of 64, 128
// or 256 grid points (blockIdx.y) and a chunk of training points
// (blockIdx.z).  For each panel of 32 training points, the x-kernel values of
// the block's queries and the y-kernel values of its grid points are formed
// once per block in LDS and read by the eight waves as MFMA operands (wave w:
// 32 queries by half of the grid points).  Chunk partial sums (FP32
// numerators, FP64 denominators) are combined in FP64 in a fixed order by
// k_query_reduce.  The training-point chunks depend on n alone and every
// query row is accumulated on its own, so a query's result does not depend on
// which other queries share its launch; large batches run in slices of
// queries that bound the partial storage.
#include <type_traits>

#include "cde_device.h"
#include "cde_kernels.h"

namespace cde {

namespace {

typedef float v16f __attribute__((ext_vector_type(16)));

constexpr float QEXCLUDED = 1e20f;

struct QueryArgs {
    double cx[16];   // log2(e) / (2 hx_k^2)
    double cy[4];    // log2(e) / (2 hy_l^2)
    double sx[16];   // sqrt(cx_k): coordinate scales of the main kernel
    double sy[4];    // sqrt(cy_l)
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

// Scaled squared distances in FP64 of a query's x (or a grid point's y) to
// a training row staged as doubles (the shift prepasses).
template <int DX>
__device__ __forceinline__ double xdist2(const double (&xo)[DX], const double* pj, const QueryArgs& qa)
{
    double d2 = 0.0;
#pragma unroll
    for (int kk = 0; kk < DX; ++kk) {
        const double d = xo[kk] - pj[kk];
        d2 = fma_(d * d, qa.cx[kk], d2);
    }
    return d2;
}

template <int DX, int DY>
__device__ __forceinline__ double ydist2(const double (&yo)[DY], const double* pj, const QueryArgs& qa)
{
    double e = 0.0;
#pragma unroll
    for (int l = 0; l < DY; ++l) {
        const double d = yo[l] - pj[DX + l];
        e = fma_(d * d, qa.cy[l], e);
    }
    return e;
}

// Shifted squared distance of pre-scaled coordinates (each multiplied by the
// square root of its c in FP64), started from -shift: a difference and an
// FMA per dimension.  The scaling rounds each coordinate once (relative
// 2^-53); the exponent is rounded to FP32 afterwards, far above that.  The
// shift is the exact minimum of the unscaled form, so the nearest pair's
// exponent can fall a few ulps below 0, which the main kernel tolerates.
template <int N>
__device__ __forceinline__ double sdist2_shifted(const double (&o)[N], const double* pj, double shift)
{
    double e = -shift;
#pragma unroll
    for (int kk = 0; kk < N; ++kk) {
        const double d = o[kk] - pj[kk];
        e = fma_(d, d, e);
    }
    return e;
}

// One tile of packed FP32 rows staged in LDS as doubles scaled by sqrt(c),
// [TILE][DX + DY].
template <int DX, int DY>
__device__ __forceinline__ void stage_tile_scaled(double* tile, const float* pre, int tid, const QueryArgs& qa)
{
#pragma unroll
    for (int d = 0; d < DX; ++d) tile[tid * (DX + DY) + d] = (double)pre[d] * qa.sx[d];
#pragma unroll
    for (int l = 0; l < DY; ++l) tile[tid * (DX + DY) + DX + l] = (double)pre[DX + l] * qa.sy[l];
}

// One tile of packed FP32 rows staged in LDS as doubles, [TILE][DX + DY]
// (exact conversions).
template <int DX, int DY>
__device__ __forceinline__ void stage_tile_d(double* tile, const float* pre, int tid)
{
#pragma unroll
    for (int d = 0; d < DX + DY; ++d) tile[tid * (DX + DY) + d] = (double)pre[d];
}

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
    float xo32[DX], c32[DX];
#pragma unroll
    for (int k = 0; k < DX; ++k) {
        xo32[k] = xq[(size_t)ec * DX + k];
        xo[k] = (double)xo32[k];
        c32[k] = vreg((float)qa.cx[k]);  // vector operands: the FMAs dual-issue
    }
    ScreenedMin screen;  // FP32 screen, exact FP64 minimum (cde_device.h)
    double best = inf_<double>();
    const int j0 = blockIdx.y * chunk, j1 = min(n, j0 + chunk);
    for (int t0 = j0; t0 < j1; t0 += TILE) {
        __syncthreads();
        float pre[S];
        load_row<S>(pre, pts + ((size_t)t0 + tid) * S);
        store_row<S>(tile + tid * S, pre);
        __syncthreads();
        const int cnt = min(TILE, j1 - t0);
        auto d32 = [&](const float* pj) {
            float e32 = (xo32[0] - pj[0]) * (xo32[0] - pj[0]) * c32[0];
#pragma unroll
            for (int k = 1; k < DX; ++k) {
                const float d = xo32[k] - pj[k];
                e32 = fmaf(d * d, c32[k], e32);
            }
            return e32;
        };
        auto exact = [&](const float* pj) {
            double d2 = 0.0;
#pragma unroll
            for (int k = 0; k < DX; ++k) {
                const double d = xo[k] - (double)pj[k];
                d2 = fma_(d * d, qa.cx[k], d2);
            }
            best = min_(best, d2);
        };
        // four rows per branch: the group is entered when its smallest FP32
        // distance passes the screen, and its rows are then screened in order
        int j = 0;
        for (; j + 4 <= cnt; j += 4) {
            float e4[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) e4[u] = d32(tile + (j + u) * S);
            if (screen.passes(fminf(fminf(e4[0], e4[1]), fminf(e4[2], e4[3])))) {
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (screen.candidate(e4[u])) exact(tile + (j + u) * S);
            }
        }
        for (; j < cnt; ++j) {
            if (screen.candidate(d32(tile + j * S))) exact(tile + j * S);
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
    constexpr int S = row_stride(DX, DY), SD = DX + DY;
    __shared__ double tile[TILE * SD];
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
        stage_tile_d<DX, DY>(tile, pre, tid);
        __syncthreads();
        const int cnt = min(TILE, j1 - t0);
        for (int j = 0; j < cnt; ++j) best = min_(best, ydist2<DX, DY>(yo, tile + j * SD, qa));
    }
    if (e < k) atomic_min_nonneg(mu + e, best);
}

// Numerator and denominator partials of one chunk of training points for
// 128 queries and GW = 64 GT grid points.  The training tile is staged in LDS
// as doubles.  For each panel of 32 of its points the block writes to LDS the
// x-kernel values w'(q, i) of its 128 queries and the y-kernel values k'(i, g)
// of its GW grid points, each formed once per block.  Wave w then owns the 32
// queries 32 (w % 4) .. and the GT column tiles of half w / 4 of the grid
// points, and runs 2-point v_mfma_f32_32x32x2f32 steps: A = w' (lane % 32 =
// query, lane / 32 = point), B = k' (lane / 32 = point, lane % 32 = column).
// Each panel's MFMA sums (16 steps) are added into FP32 chunk sums (at most 64
// panels), so a chunk partial carries a relative error of at most about
// 96 x 2^-24 of its all-positive terms; chunks are combined in FP64.
constexpr int QWAVES = 8;         // waves per query block
constexpr int QNT = 64 * QWAVES;  // threads per query block
constexpr int QPB = 128;          // queries per query block

template <int GT>
struct QPanelB;  // a lane's GT consecutive y-kernel values (one per column tile)
template <>
struct QPanelB<1> {
    float v[1];
    __device__ __forceinline__ void load(const float* p) { v[0] = p[0]; }
};
template <>
struct QPanelB<2> {
    float v[2];
    __device__ __forceinline__ void load(const float* p)
    {
        const float2 t = *(const float2*)p;
        v[0] = t.x;
        v[1] = t.y;
    }
};
template <>
struct QPanelB<4> {
    float v[4];
    __device__ __forceinline__ void load(const float* p)
    {
        const float4 t = *(const float4*)p;
        v[0] = t.x;
        v[1] = t.y;
        v[2] = t.z;
        v[3] = t.w;
    }
};

template <int DX, int DY, int GT>
__global__ __launch_bounds__(QNT) void k_query_mfma(const float* __restrict__ pts, int n, int chunk,
                                                     const float* __restrict__ xq, int q,
                                                     const float* __restrict__ yg, int k,
                                                     QueryArgs qa, const double* __restrict__ mq,
                                                     const double* __restrict__ mu,
                                                     float* __restrict__ fpart,
                                                     double* __restrict__ dpart)
{
    constexpr int S = row_stride(DX, DY), SD = DX + DY;
    constexpr int GWW = 32 * GT;  // grid columns per wave
    constexpr int GW = 2 * GWW;   // grid columns per block
    constexpr int SUB = 32;       // training points per panel
    // LDS rows padded by 32 floats: the two 32-lane halves of a wave, which
    // read consecutive rows, start 128 bytes apart in the banks.
    constexpr int YS = GW + 32, XS = QPB + 32;
    constexpr int YSTEP = QNT / GW, YPT = SUB / YSTEP;   // y panel rows: per pass, per thread
    constexpr int XSTEP = QNT / QPB, XPT = SUB / XSTEP;  // x panel rows: per pass, per thread
    static_assert(QNT % GW == 0 && SUB % YSTEP == 0 && SUB % XSTEP == 0, "panel shape");
    static_assert(YS % 4 == 0 && GWW % 4 == 0, "B vector reads stay aligned");
    static_assert(TILE * SD >= QNT, "the tile area holds the denominator reduction");
    __shared__ double tile[TILE * SD];
    __shared__ __align__(16) float ykv[SUB * YS];  // [point][position]; position = half, then GT n + t
    __shared__ float xkv[SUB * XS];  // [point][query]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int q0 = blockIdx.x * QPB;
    const int g0 = blockIdx.y * GW;
    const int c = blockIdx.z;

    // x-kernel role: query q0 + tid % QPB, panel rows tid / QPB + XSTEP r
    const int xcol = tid % QPB, xrow = tid / QPB;
    const int qi = min(q0 + xcol, q - 1);
    double xo[DX];
#pragma unroll
    for (int kk = 0; kk < DX; ++kk) xo[kk] = (double)xq[(size_t)qi * DX + kk] * qa.sx[kk];
    const double m_q = mq[qi];
    // y-kernel role: LDS position tid % GW, panel rows tid / GW + YSTEP r.
    // Position h GWW + GT n + t holds grid column h GWW + 32 t + n, so a lane
    // of half h reads its GT column tiles' values as one vector.
    const int ypos = tid % GW, yrow = tid / GW;
    const int yh = ypos / GWW, yr = ypos % GWW;
    const int gy = min(g0 + yh * GWW + 32 * (yr % GT) + yr / GT, k - 1);
    double yo[DY];
#pragma unroll
    for (int l = 0; l < DY; ++l) yo[l] = (double)yg[(size_t)gy * DY + l] * qa.sy[l];
    const double mu_g = mu[gy];
    // MFMA role
    const int qg = wave & 3, half = wave >> 2;
    const int kr = lane >> 5, m32 = lane & 31;
    const float* arow = xkv + kr * XS + 32 * qg + m32;
    const float* brow = ykv + kr * YS + half * GWW + GT * m32;

    // Panel sums (MFMA, 32 points) are added into FP32 chunk sums; a chunk
    // holds at most 8 tiles (64 panels).
    float tot[GT][16];
#pragma unroll
    for (int t = 0; t < GT; ++t)
#pragma unroll
        for (int r = 0; r < 16; ++r) tot[t][r] = 0.f;
    double dtot = 0.0;

    const int j0 = c * chunk, j1 = min(n, j0 + chunk);
    const bool stager = tid < TILE;  // the first TILE threads stage the rows
    float pre[S];
    if (stager) load_row<S>(pre, pts + ((size_t)j0 + tid) * S);
    for (int t0 = j0; t0 < j1; t0 += TILE) {
        __syncthreads();
        if (stager) {
            stage_tile_scaled<DX, DY>(tile, pre, tid, qa);
            if (t0 + TILE < j1) load_row<S>(pre, pts + ((size_t)t0 + TILE + tid) * S);
        }
        const int cnt = min(TILE, j1 - t0);
        float dp = 0.f;
        for (int s0 = 0; s0 < cnt; s0 += SUB) {
            __syncthreads();  // tile staged / previous panel read by every wave
            // Rows past cnt (padding or the next chunk's points) get finite
            // values <= 1 from the clamp; their x-kernel values are 0.
#pragma unroll
            for (int r = 0; r < YPT; ++r) {
                const int p = yrow + YSTEP * r;
                const float a = (float)sdist2_shifted<DY>(yo, tile + (s0 + p) * SD + DX, mu_g);
                ykv[p * YS + ypos] = exp2_<float>(-fmaxf(a, 0.f));
            }
#pragma unroll
            for (int r = 0; r < XPT; ++r) {
                const int p = xrow + XSTEP * r;
                const double d2 = sdist2_shifted<DX>(xo, tile + (s0 + p) * SD, m_q);
                const float w = exp2_<float>(-(s0 + p < cnt ? (float)d2 : QEXCLUDED));
                dp += w;
                xkv[p * XS + xcol] = w;
            }
            __syncthreads();
            v16f acc[GT];
#pragma unroll
            for (int s = 0; s < SUB; s += 2) {
                const float a = arow[s * XS];
                QPanelB<GT> b;
                b.load(brow + s * YS);
#pragma unroll
                for (int t = 0; t < GT; ++t)
                    acc[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b.v[t], s == 0 ? v16f{} : acc[t], 0, 0, 0);
            }
#pragma unroll
            for (int t = 0; t < GT; ++t)
#pragma unroll
                for (int r = 0; r < 16; ++r) tot[t][r] += acc[t][r];
        }
        dtot += (double)dp;
    }
    // den' partial of query q0 + xcol: the XSTEP row groups in a fixed order
    __syncthreads();
    tile[xrow * QPB + xcol] = dtot;
    __syncthreads();
    if (tid < QPB && blockIdx.y == 0 && q0 + tid < q) {
        double dsum = tile[tid];
#pragma unroll
        for (int r = 1; r < XSTEP; ++r) dsum += tile[r * QPB + tid];
        dpart[(size_t)c * q + q0 + tid] = dsum;
    }
    // f32 32x32x2 result layout: register r of lane l holds row (query)
    // 8 (r / 4) + 4 (l / 32) + r % 4 and column (grid point) l % 32
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int qq = q0 + 32 * qg + 8 * (r >> 2) + 4 * kr + (r & 3);
#pragma unroll
        for (int t = 0; t < GT; ++t) {
            const int g = g0 + half * GWW + 32 * t + m32;
            if (qq < q && g < k) fpart[((size_t)c * q + qq) * k + g] = tot[t][r];
        }
    }
}

// f = c_y 2^-mu_g F'/D' with F' and D' summed over the point chunks in order.
__global__ void k_query_reduce(const float* __restrict__ fpart, const double* __restrict__ dpart,
                               const double* __restrict__ mu, int q, int k, int nchunks,
                               double log_cy, double* __restrict__ f)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)q * k) return;
    const int qq = (int)(e / k), g = (int)(e - (int64_t)qq * k);
    double num = 0.0, den = 0.0;
    for (int c = 0; c < nchunks; ++c) {
        num += (double)fpart[((size_t)c * q + qq) * k + g];
        den += dpart[(size_t)c * q + qq];
    }
    f[e] = num > 0.0 ? exp(log_cy - mu[g] * LN2 + log(num / den)) : 0.0;
}

// Training-point chunks: whole tiles, at most 256 chunks while that keeps a
// chunk within 8 tiles (the FP32 chunk sums above), a function of n only
// (never of the batch).
int64_t query_chunk_points(int64_t n)
{
    const int64_t ntiles = (n + TILE - 1) / TILE;
    return std::min<int64_t>(8, (ntiles + 255) / 256) * TILE;
}

// Grid tiles of 16 points per block of the Epanechnikov query: 4, 8 or 16
// (a function of k only).
int query_grid_tiles(int64_t k)
{
    const int64_t nt = (k + 15) / 16;
    return nt <= 4 ? 4 : nt <= 8 ? 8 : 16;
}

// Column tiles of 32 grid points per wave of k_query_mfma: 1, 2 or 4, so a
// block covers 64, 128 or 256 grid points (a function of k only).
static int query_col_tiles(int64_t k)
{
    return k <= 64 ? 1 : k <= 128 ? 2 : 4;
}

// Queries per slice: chunk partials of one slice (k FP32 numerators and one
// FP64 denominator per query and chunk) within 512 MiB.
int64_t query_slice(int64_t nch, int64_t q, int64_t k)
{
    int64_t s = ((int64_t(1) << 29) / (nch * (4 * k + 8))) / QPB * QPB;
    return std::min(q, std::max<int64_t>(QPB, s));
}

size_t query_work_doubles(const cde_model* m, int64_t q, int64_t k)
{
    const int64_t chunk = query_chunk_points(m->n);
    const int64_t nch = (m->n + chunk - 1) / chunk;
    const int64_t qs = query_slice(nch, q, k);
    return (size_t)(q + k + nch * qs + (nch * qs * k + 1) / 2 + 64);
}

template <int DX, int DY>
static hipError_t query_t(const cde_model* m, const float* xq, int q, const float* yg, int k,
                          const double* h, double* f, double* work, hipStream_t stream)
{
    QueryArgs qa;
    for (int kk = 0; kk < 16; ++kk) {
        qa.cx[kk] = kk < DX ? LOG2E / (2.0 * h[kk] * h[kk]) : 0.0;
        qa.sx[kk] = sqrt(qa.cx[kk]);
    }
    double lcy = 0.0;
    for (int l = 0; l < 4; ++l) {
        qa.cy[l] = l < DY ? LOG2E / (2.0 * h[DX + l] * h[DX + l]) : 0.0;
        qa.sy[l] = sqrt(qa.cy[l]);
        if (l < DY) lcy -= log(h[DX + l]) + HALF_LOG_2PI;
    }
    qa.log_cy = lcy;
    const int n = (int)m->n;
    const float* pts = (const float*)m->pts;
    const int gt = query_col_tiles(k);
    const int gb = (k + 64 * gt - 1) / (64 * gt);
    const int chunk = (int)query_chunk_points(n);
    const int nch = (n + chunk - 1) / chunk;
    const int qs = (int)query_slice(nch, q, k);
    double* mq = work;
    double* mu = work + q;
    double* dpart = mu + k;
    float* fpart = (float*)(dpart + (size_t)nch * qs);
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
        const int qb = (qn + QPB - 1) / QPB;
        const dim3 grid(qb, gb, nch);
        const float* xs = xq + (size_t)q0 * DX;
        const double* mqs = mq + q0;
        if (gt == 1)
            hipLaunchKernelGGL((k_query_mfma<DX, DY, 1>), grid, dim3(QNT), 0, stream, pts, n, chunk, xs,
                               qn, yg, k, qa, mqs, (const double*)mu, fpart, dpart);
        else if (gt == 2)
            hipLaunchKernelGGL((k_query_mfma<DX, DY, 2>), grid, dim3(QNT), 0, stream, pts, n, chunk, xs,
                               qn, yg, k, qa, mqs, (const double*)mu, fpart, dpart);
        else
            hipLaunchKernelGGL((k_query_mfma<DX, DY, 4>), grid, dim3(QNT), 0, stream, pts, n, chunk, xs,
                               qn, yg, k, qa, mqs, (const double*)mu, fpart, dpart);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        const int64_t total = (int64_t)qn * k;
        hipLaunchKernelGGL(k_query_reduce, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream,
                           (const float*)fpart, (const double*)dpart, (const double*)mu, qn, k, nch,
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
