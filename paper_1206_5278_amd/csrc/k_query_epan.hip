// k_query_epan.hip -- conditional density queries with the Epanechnikov
// kernel (the kernel of the paper's experiments, Section 4, radial over the
// bandwidth-scaled coordinates) on the matrix cores, with exact skipping.
//
//     f(y_g | x_q) = c_y sum_i wx(q, i) wy(i, g) / sum_i wx(q, i),
//     wx = (1 - |(x_q - x_i) / hx|^2)_+,   wy = (1 - |(y_g - y_i) / hy|^2)_+,
//
// and f = 0 where no training x lies inside the query's window (eq. (1) is
// 0/0 there).  Window values are formed in FP64 (the edge 1 - |u|^2 cancels)
// on rows, queries and grid points scaled by 1/h when staged (one rounding
// each, relative 2^-53), and rounded once to FP32; products run on
// v_mfma_f32_16x16x4f32 with 8 waves x 16 queries per block, each wave
// forming its own queries' window values, and y-kernel panels of 32 training
// points shared through LDS (16 queries per wave keep the per-wave skip test
// below fine-grained).
//
// Exact skipping: the training points are read in the model's spatial
// (kd-leaf) order with their 256-row tile and 32-row panel boxes, and the
// queries are processed in Morton order of their window-sized cells, so a
// block's 128 queries have a compact bounding box.  A tile or panel whose x
// box lies more than one window (with a 2^-40 margin) from the block's query
// box holds only exact zeros for every query of the block and is skipped;
// within a loaded panel, each wave also skips its MFMA steps when the panel
// lies outside the windows of its own 16 queries.
// Skipping removes exact-zero terms only and the point chunks and panel
// order are fixed, so a query's bits do not depend on the other queries of
// its launch.
#include <algorithm>

#include "cde_device.h"
#include "cde_kernels.h"

namespace cde {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int EWAVES = 8;
constexpr int ENT = 64 * EWAVES;   // threads per block
constexpr int EQPB = 16 * EWAVES;  // queries per block
constexpr double EQ_SKIP_MARGIN = 1.0 + 0x1p-40;

struct EpanQArgs {
    double inv[16];  // 1 / hx_k (box gaps, Morton cells, scaled rows)
    double iny[4];   // 1 / hy_l (scaled rows)
};

// Squared scaled box distance between [alo, ahi] and [blo, bhi].
template <int DX>
__device__ __forceinline__ double box_gap2(const double* alo, const double* ahi, const double* blo,
                                           const double* bhi, const EpanQArgs& a)
{
    double d2 = 0.0;
#pragma unroll
    for (int k = 0; k < DX; ++k) {
        const double gap = fmax(0.0, fmax(blo[k] - ahi[k], alo[k] - bhi[k])) * a.inv[k];
        d2 = fma(gap, gap, d2);
    }
    return d2;
}

// Morton key of the query's window-sized cell: floor(x_k / hx_k), clamped
// to B = min(31, 64 / DX) signed bits per dimension, bits interleaved.
template <int DX>
__global__ void k_qe_keys(const float* __restrict__ xq, int q, EpanQArgs a,
                          unsigned long long* __restrict__ keys, int* __restrict__ idx)
{
    constexpr int B = 64 / DX < 31 ? 64 / DX : 31;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= q) return;
    unsigned long long u[DX];
#pragma unroll
    for (int k = 0; k < DX; ++k) {
        const double c = floor((double)xq[(size_t)e * DX + k] * a.inv[k]) + (double)(1ll << (B - 1));
        const double lim = (double)((1ll << B) - 1);
        u[k] = (unsigned long long)fmin(fmax(c, 0.0), lim);
    }
    unsigned long long key = 0;
    for (int b = B - 1; b >= 0; --b)
#pragma unroll
        for (int k = 0; k < DX; ++k) key = (key << 1) | ((u[k] >> b) & 1ull);
    keys[e] = key;
    idx[e] = e;
}

template <int DX, int DY, int GT>
__global__ __launch_bounds__(ENT) void k_query_epan(const double* __restrict__ spts,
                                                    const double* __restrict__ tbox,
                                                    const double* __restrict__ sbox, int n, int chunk,
                                                    const float* __restrict__ xq,
                                                    const int* __restrict__ order, int q,
                                                    const float* __restrict__ yg, int k, EpanQArgs a,
                                                    float* __restrict__ fpart,
                                                    double* __restrict__ dpart)
{
    constexpr int S = row_stride(DX, DY), SD = DX + DY;
    constexpr int GW = 16 * GT;
    constexpr int YS = (GW % 32 == 16) ? GW : GW + 16;
    constexpr int SUB = 32;
    constexpr int NSUB = TILE / SUB;
    constexpr int PSTEP = ENT / GW;
    constexpr int YPT = SUB / PSTEP;
    static_assert(ENT % GW == 0 && SUB % PSTEP == 0 && SUB == SUBROWS, "block shape");
    __shared__ double tile[TILE * SD];
    __shared__ float ykv[SUB * YS];
    __shared__ double qxs[EQPB * DX];
    __shared__ double qbox[2 * DX];
    __shared__ double wbox[EWAVES * 2 * DX];  // per wave: the box of its 16 queries
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int s0 = blockIdx.x * EQPB;  // first query of the block, in Morton order
    const int g0 = blockIdx.y * GW;
    const int c = blockIdx.z;
    const int kr = lane >> 4;

    // query box of the block
    if (tid < EQPB) {
        const int o = order[min(s0 + tid, q - 1)];
#pragma unroll
        for (int kk = 0; kk < DX; ++kk) qxs[tid * DX + kk] = (double)xq[(size_t)o * DX + kk];
    }
    __syncthreads();
    if (tid < EWAVES * DX) {
        const int w = tid / DX, kk = tid % DX;
        double lo = qxs[w * 16 * DX + kk], hi = lo;
        for (int r = 1; r < 16; ++r) {
            lo = fmin(lo, qxs[(w * 16 + r) * DX + kk]);
            hi = fmax(hi, qxs[(w * 16 + r) * DX + kk]);
        }
        wbox[w * 2 * DX + kk] = lo;
        wbox[w * 2 * DX + DX + kk] = hi;
    }
    __syncthreads();
    if (tid < DX) {
        double lo = wbox[tid], hi = wbox[DX + tid];
        for (int w = 1; w < EWAVES; ++w) {
            lo = fmin(lo, wbox[w * 2 * DX + tid]);
            hi = fmax(hi, wbox[w * 2 * DX + DX + tid]);
        }
        qbox[tid] = lo;
        qbox[DX + tid] = hi;
    }

    // A role: query s0 + 16 wave + lane % 16 (Morton order)
    const int sq = s0 + wave * 16 + (lane & 15);
    const int oq = order[min(sq, q - 1)];
    double xo[DX];
#pragma unroll
    for (int kk = 0; kk < DX; ++kk) xo[kk] = (double)xq[(size_t)oq * DX + kk] * a.inv[kk];
    // panel role: grid column tid % GW
    const int gcol = tid % GW;
    const int gy = min(g0 + gcol, k - 1);
    double yo[DY];
#pragma unroll
    for (int l = 0; l < DY; ++l) yo[l] = (double)yg[(size_t)gy * DY + l] * a.iny[l];
    const int prow = tid / GW;

    float tot[GT][4];
#pragma unroll
    for (int t = 0; t < GT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) tot[t][r] = 0.f;
    double dtot = 0.0;
    __syncthreads();  // query box ready

    const int j0 = c * chunk, j1 = min(n, j0 + chunk);
    for (int t0 = j0; t0 < j1; t0 += TILE) {
        const int tt = t0 / TILE;
        const double* tb = tbox + (size_t)tt * 2 * DX;
        if (box_gap2<DX>(qbox, qbox + DX, tb, tb + DX, a) > EQ_SKIP_MARGIN) continue;  // block-uniform
        __syncthreads();  // previous tile fully read
        if (tid < TILE) {
            double pre[S];
            load_row<S>(pre, spts + ((size_t)t0 + tid) * S);
#pragma unroll
            for (int d = 0; d < SD; ++d) tile[tid * SD + d] = pre[d] * (d < DX ? a.inv[d] : a.iny[d - DX]);
        }
        const int cnt = min(TILE, j1 - t0);
        float dp = 0.f;
        for (int p = 0; p * SUB < cnt; ++p) {
            const double* sb = sbox + ((size_t)tt * NSUB + p) * 2 * DX;
            if (box_gap2<DX>(qbox, qbox + DX, sb, sb + DX, a) > EQ_SKIP_MARGIN) continue;  // uniform
            const int s0p = p * SUB;
            __syncthreads();  // tile staged / previous panel read
#pragma unroll
            for (int r = 0; r < YPT; ++r) {
                const int pr = prow + PSTEP * r;
                double e = -1.0;
#pragma unroll
                for (int l = 0; l < DY; ++l) {
                    const double d = yo[l] - tile[(s0p + pr) * SD + DX + l];
                    e = fma(d, d, e);
                }
                ykv[pr * YS + gcol] = (float)fmax(-e, 0.0);  // (1 - |v|^2)_+, in [0, 1] for any row
            }
            __syncthreads();
            // this wave's 16 queries: skip the panel's steps when it lies
            // outside all their windows (exact zeros; wave-uniform)
            const double* wb = wbox + wave * 2 * DX;
            if (box_gap2<DX>(wb, wb + DX, sb, sb + DX, a) > EQ_SKIP_MARGIN) continue;
            auto weight = [&](int ii) {
                double s2 = -1.0;
#pragma unroll
                for (int kk = 0; kk < DX; ++kk) {
                    const double d = xo[kk] - tile[ii * SD + kk];
                    s2 = fma(d, d, s2);
                }
                return ii < cnt ? (float)fmax(-s2, 0.0) : 0.f;
            };
            v4f acc[GT];
            float w = weight(s0p + kr);
#pragma unroll
            for (int s = 0; s < SUB; s += 4) {
                const float wn = s + 4 < SUB ? weight(s0p + s + 4 + kr) : 0.f;
                dp += w;
                const float* brow = ykv + (s + kr) * YS + (lane & 15);
#pragma unroll
                for (int t = 0; t < GT; ++t)
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                        w, brow[16 * t], s == 0 ? v4f{0.f, 0.f, 0.f, 0.f} : acc[t], 0, 0, 0);
                w = wn;
            }
#pragma unroll
            for (int t = 0; t < GT; ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r) tot[t][r] += acc[t][r];
        }
        dtot += (double)dp;
    }
    double dsum = dtot;
    dsum += __shfl_xor(dsum, 16, 64);
    dsum += __shfl_xor(dsum, 32, 64);
    if (blockIdx.y == 0 && lane < 16 && s0 + wave * 16 + lane < q)
        dpart[(size_t)c * q + s0 + wave * 16 + lane] = dsum;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int qq = s0 + wave * 16 + 4 * (lane >> 4) + r;
#pragma unroll
        for (int t = 0; t < GT; ++t) {
            const int g = g0 + 16 * t + (lane & 15);
            if (qq < q && g < k) fpart[((size_t)c * q + qq) * k + g] = tot[t][r];
        }
    }
}

// f[order[s]][g] = c_y F/D for slice rows s (Morton order), 0 where D = 0.
__global__ void k_query_epan_reduce(const float* __restrict__ fpart, const double* __restrict__ dpart,
                                    const int* __restrict__ order, int q, int k, int nchunks,
                                    double cy, double* __restrict__ f)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)q * k) return;
    const int qq = (int)(e / k), g = (int)(e - (int64_t)qq * k);
    double num = 0.0, den = 0.0;
    for (int ch = 0; ch < nchunks; ++ch) {
        num += (double)fpart[((size_t)ch * q + qq) * k + g];
        den += dpart[(size_t)ch * q + qq];
    }
    f[(size_t)order[qq] * k + g] = den > 0.0 ? cy * num / den : 0.0;
}

size_t sort_temp_bytes(int q)
{
    return (radix_sort_work_bytes(q) + 255) / 256 * 256;
}

template <int DX, int DY>
hipError_t query_epan_t(const cde_model* m, const float* xq, int q, const float* yg, int k,
                        const double* h, double* f, char* work, hipStream_t stream)
{
    EpanQArgs a;
    for (int kk = 0; kk < 16; ++kk) {
        a.inv[kk] = kk < DX ? 1.0 / h[kk] : 0.0;
    }
    for (int l = 0; l < 4; ++l) {
        a.iny[l] = l < DY ? 1.0 / h[DX + l] : 0.0;
    }
    const double cy = exp(log_epan_norm(h + DX, DY));
    const int n = (int)m->n;
    const int gt = query_grid_tiles(k);
    const int gb = (k + 16 * gt - 1) / (16 * gt);
    const int chunk = (int)query_chunk_points(n);
    const int nch = (n + chunk - 1) / chunk;
    const int qs = (int)query_slice(nch, q, k);
    // work: keys [2][q], order [2][q], sort temp, then the slice partials
    unsigned long long* k0 = (unsigned long long*)work;
    unsigned long long* k1 = k0 + q;
    int* o0 = (int*)(k1 + q);
    int* o1 = o0 + q;
    char* tmp = (char*)(((uintptr_t)(o1 + q) + 255) & ~(uintptr_t)255);
    size_t tmp_bytes = sort_temp_bytes(q);
    double* dpart = (double*)(tmp + tmp_bytes);
    float* fpart = (float*)(dpart + (size_t)nch * qs);
    hipLaunchKernelGGL(k_qe_keys<DX>, dim3((q + 255) / 256), dim3(256), 0, stream, xq, q, a, k0, o0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    bool alt = false;
    e = radix_sort_pairs(k0, o0, k1, o1, q, 0, 64, tmp, &alt, stream);
    if (e != hipSuccess) return e;
    const int* order = alt ? o1 : o0;
    for (int q0 = 0; q0 < q; q0 += qs) {
        const int qn = std::min(qs, q - q0);
        const dim3 grid((qn + EQPB - 1) / EQPB, gb, nch);
        const int* ord = order + q0;
        if (gt == 4)
            hipLaunchKernelGGL((k_query_epan<DX, DY, 4>), grid, dim3(ENT), 0, stream, (const double*)m->spts,
                               (const double*)m->tbox, (const double*)m->sbox, n, chunk, xq, ord, qn, yg,
                               k, a, fpart, dpart);
        else if (gt == 8)
            hipLaunchKernelGGL((k_query_epan<DX, DY, 8>), grid, dim3(ENT), 0, stream, (const double*)m->spts,
                               (const double*)m->tbox, (const double*)m->sbox, n, chunk, xq, ord, qn, yg,
                               k, a, fpart, dpart);
        else
            hipLaunchKernelGGL((k_query_epan<DX, DY, 16>), grid, dim3(ENT), 0, stream, (const double*)m->spts,
                               (const double*)m->tbox, (const double*)m->sbox, n, chunk, xq, ord, qn, yg,
                               k, a, fpart, dpart);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        const int64_t total = (int64_t)qn * k;
        hipLaunchKernelGGL(k_query_epan_reduce, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream,
                           (const float*)fpart, (const double*)dpart, ord, qn, k, nch, cy, f);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

size_t query_epan_work_bytes(const cde_model* m, int64_t q, int64_t k)
{
    const int64_t chunk = query_chunk_points(m->n);
    const int64_t nch = (m->n + chunk - 1) / chunk;
    const int64_t qs = query_slice(nch, q, k);
    return (size_t)(2 * q * 8 + 2 * q * 4 + 256) + sort_temp_bytes((int)q) +
           (size_t)(nch * qs * 8 + nch * qs * k * 4 + 256);
}

#define CDE_QE_CASE(DX_, DY_) \
    case (DX_) * 8 + (DY_): return query_epan_t<DX_, DY_>(m, xq, q, yg, k, h, f, work, stream);

hipError_t launch_query_epan(const cde_model* m, const float* xq, int q, const float* yg, int k,
                             const double* h, double* f, char* work, hipStream_t stream)
{
    switch (m->dx * 8 + m->dy) {
        CDE_QE_CASE(1, 1) CDE_QE_CASE(1, 2) CDE_QE_CASE(2, 1) CDE_QE_CASE(2, 2)
        CDE_QE_CASE(3, 1) CDE_QE_CASE(3, 2) CDE_QE_CASE(4, 1) CDE_QE_CASE(4, 2)
        CDE_QE_CASE(5, 1) CDE_QE_CASE(5, 2) CDE_QE_CASE(6, 1) CDE_QE_CASE(6, 2)
        CDE_QE_CASE(7, 1) CDE_QE_CASE(7, 2) CDE_QE_CASE(8, 1) CDE_QE_CASE(8, 2)
        CDE_QE_CASE(16, 1) CDE_QE_CASE(16, 2)
        default: return hipErrorInvalidValue;
    }
}

}  // namespace cde
