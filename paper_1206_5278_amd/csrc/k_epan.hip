// k_epan.hip -- exact LOO log-likelihood with the Epanechnikov kernel.
//
// Kernel (the paper's experiments, Section 4; scaled-kernel form of
// Section 2, radial over bandwidth-scaled coordinates):
//     K_h(t) = c_d / prod_k h_k * max(0, 1 - sum_k (t_k / h_k)^2),
// c_d = (d + 2) / (2 V_d), V_d the volume of the unit d-ball.  Per point i,
// over j != i: D = sum wx_j, U = sum wx_j wy_j with wx = max(0, 1 - ux),
// wy = max(0, 1 - uy) and ux, uy the scaled squared distances; then
//     CONDITIONAL: l_i = log c_y + log U - log D
//     JOINT      : l_i = log c_x + log c_y + log U - log(n - 1)
// and l_i = -inf when U = 0 (no j inside both windows: the divergence at
// tiny bandwidths that Section 4.1 notes).
//
// The kernel is exactly zero outside its window, so a (point block, j tile)
// pair whose x boxes (in the model's spatial order) are at scaled distance
// above 1 contributes exactly nothing and is skipped without loading it; the
// candidate tiles of a block are tested in parallel and compacted in order.
// Inside a loaded tile each wave skips the 32-row subtiles whose boxes lie a
// window from its own 64 points.  The margin 2^-40 keeps these decisions
// clear of the rounding of the distances.
// Everything else follows the Gaussian diagonal pass: one lane per point i,
// j tiles through LDS, blockIdx.y a setting, blockIdx.z a chunk of j tiles,
// partial sums per chunk combined in a fixed order.  The pair arithmetic is
// FP64 (the window edge 1 - u cancels, and FP32 would lose the relative
// accuracy of the small terms near it); coordinates are pre-scaled by
// 1/h_k as tiles are staged, so a pair costs a difference and an FMA per
// dimension.
#include <cmath>

#include "cde_device.h"
#include "cde_kernels.h"

namespace cde {

namespace {

constexpr double SKIP_MARGIN = 1.0 + 0x1p-40;

// Scaled squared gap between two x boxes (lo[0..DX), hi[0..DX) each).
template <int DX>
__device__ __forceinline__ double box_gap2(const double* alo, const double* ahi, const double* blo,
                                           const double* bhi, const double (&inv)[DX])
{
    double d2 = 0.0;
#pragma unroll
    for (int k = 0; k < DX; ++k) {
        const double gap = fmax(0.0, fmax(blo[k] - ahi[k], alo[k] - bhi[k])) * inv[k];
        d2 = fma(gap, gap, d2);
    }
    return d2;
}

// One 32-row subtile of the staged (pre-scaled) tile against this lane's
// point: adds the x weights to D and the product weights to U.  MASK drops
// row `self` (point i itself) and rows at or beyond `cnt`.
template <int DX, int DY, bool MASK>
__device__ __forceinline__ void epan_subtile(const double* tile, int q0, int cnt, int self,
                                             const double (&xs)[DX + DY], double& D, double& U)
{
    constexpr int S = row_stride(DX, DY);
    constexpr int P = DX + DY;
#pragma unroll 4
    for (int r = 0; r < SUBROWS; ++r) {
        const int q = q0 + r;
        double pj[S];
        load_cols<P, S>(pj, tile + q * S);
        double ux = 0.0, uy = 0.0;
#pragma unroll
        for (int k = 0; k < DX; ++k) {
            const double d = xs[k] - pj[k];
            ux = fma(d, d, ux);
        }
#pragma unroll
        for (int l = 0; l < DY; ++l) {
            const double d = xs[DX + l] - pj[DX + l];
            uy = fma(d, d, uy);
        }
        double wx = fmax(1.0 - ux, 0.0);
        const double wy = fmax(1.0 - uy, 0.0);
        if (MASK && (q == self || q >= cnt)) wx = 0.0;
        D += wx;
        U = fma(wx, wy, U);
    }
}

template <int DX, int DY>
__global__ __launch_bounds__(TILE) void k_loo_epan(const double* __restrict__ spts,
                                                   const double* __restrict__ tbox,
                                                   const double* __restrict__ sbox, int n, int npad,
                                                   EpanSets sets, int tiles_per_chunk,
                                                   double* __restrict__ partial)
{
    constexpr int S = row_stride(DX, DY);
    constexpr int P = DX + DY;
    constexpr int NSUB = TILE / SUBROWS;
    __shared__ double tile[TILE * S];
    __shared__ int list[TILE];
    __shared__ int wcount[4];
    const EpanSet& st = sets.s[blockIdx.y];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int b = blockIdx.x;
    const int i = b * TILE + tid;

    double inv[P], invx[DX];
#pragma unroll
    for (int k = 0; k < P; ++k) inv[k] = st.inv_h[k];
#pragma unroll
    for (int k = 0; k < DX; ++k) invx[k] = inv[k];
    double own[S], xs[P];
    load_row<S>(own, spts + (size_t)i * S);
#pragma unroll
    for (int k = 0; k < P; ++k) xs[k] = own[k] * inv[k];

    // this wave's x box (its 64 points; padding rows excluded)
    double wlo[DX], whi[DX];
#pragma unroll
    for (int k = 0; k < DX; ++k) {
        double a = i < n ? own[k] : __builtin_inf();
        double c = i < n ? own[k] : -__builtin_inf();
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            a = fmin(a, __shfl_xor(a, off, 64));
            c = fmax(c, __shfl_xor(c, off, 64));
        }
        wlo[k] = a;
        whi[k] = c;
    }
    double blo[DX], bhi[DX];
#pragma unroll
    for (int k = 0; k < DX; ++k) {
        blo[k] = tbox[(size_t)b * 2 * DX + k];
        bhi[k] = tbox[(size_t)b * 2 * DX + DX + k];
    }

    const int ntiles = (n + TILE - 1) / TILE;
    const int t0 = blockIdx.z * tiles_per_chunk;
    const int t1 = min(ntiles, t0 + tiles_per_chunk);
    double D = 0.0, U = 0.0;
    for (int base = t0; base < t1; base += TILE) {
        // Candidate tiles base..base+255 in parallel, compacted in order.
        const int cand = base + tid;
        bool act = false;
        if (cand < t1) {
            const double* cb = tbox + (size_t)cand * 2 * DX;
            act = box_gap2<DX>(blo, bhi, cb, cb + DX, invx) <= SKIP_MARGIN;
        }
        const unsigned long long mask = __ballot(act);
        __syncthreads();  // the previous round has finished with list[] and tile[]
        if (lane == 0) wcount[wave] = __popcll(mask);
        __syncthreads();
        int ofs = 0;
        for (int w = 0; w < wave; ++w) ofs += wcount[w];
        const int nact = wcount[0] + wcount[1] + wcount[2] + wcount[3];
        if (act) list[ofs + __popcll(mask & ((1ull << lane) - 1ull))] = cand;
        __syncthreads();

        double pre[S];
        if (nact > 0) load_row<S>(pre, spts + ((size_t)list[0] * TILE + tid) * S);
        for (int a = 0; a < nact; ++a) {
            const int t = list[a];
            __syncthreads();
#pragma unroll
            for (int k = 0; k < S; ++k) tile[tid * S + k] = k < P ? pre[k] * inv[k] : 0.0;
            __syncthreads();
            if (a + 1 < nact) load_row<S>(pre, spts + ((size_t)list[a + 1] * TILE + tid) * S);
            const int cnt = min(TILE, n - t * TILE);
            const int self = (t == b) ? tid : -1;
            const bool mask_rows = self >= 0 || cnt < TILE;
            for (int sb = 0; sb < NSUB; ++sb) {
                if (sb * SUBROWS >= cnt) break;
                // this wave's box against the subtile's: skip when a window apart
                const double* xb = sbox + ((size_t)t * NSUB + sb) * 2 * DX;
                if (box_gap2<DX>(wlo, whi, xb, xb + DX, invx) > SKIP_MARGIN) continue;
                if (mask_rows)
                    epan_subtile<DX, DY, true>(tile, sb * SUBROWS, cnt, self, xs, D, U);
                else
                    epan_subtile<DX, DY, false>(tile, sb * SUBROWS, cnt, self, xs, D, U);
            }
        }
    }
    double* o = partial + ((size_t)(blockIdx.y * gridDim.z + blockIdx.z) * 2) * npad + i;
    o[0] = D;
    o[npad] = U;
}

// Sums the chunk partials of each point in chunk order, finalises l_i in
// FP64, writes it at the point's original index (perm maps sorted position
// to original index) and one fixed-order block row (l, non-finite count) per
// (setting, 256-point block of the sorted order).
__global__ __launch_bounds__(TILE) void k_epan_combine(const double* __restrict__ partial, int chunks,
                                                       int n, int npad, EpanSets sets, int crit,
                                                       const int* __restrict__ perm,
                                                       double* __restrict__ per_point,
                                                       double* __restrict__ part)
{
    __shared__ double red[4 * 2];
    const EpanSet& st = sets.s[blockIdx.y];
    const int tid = threadIdx.x;
    const int i = blockIdx.x * TILE + tid;
    const double* base = partial + (size_t)blockIdx.y * chunks * 2 * npad + i;
    double D = 0.0, U = 0.0;
    for (int c = 0; c < chunks; ++c) {
        D += base[(size_t)c * 2 * npad];
        U += base[((size_t)c * 2 + 1) * npad];
    }
    const bool valid = i < n;
    double ell;
    if (U == 0.0)
        ell = -__builtin_inf();
    else if (crit == CDE_COND)
        ell = st.log_cy + log(U / D);
    else
        ell = st.log_cx + st.log_cy + log(U) - log((double)(n - 1));
    double v[2];
    v[0] = valid ? ell : 0.0;
    v[1] = (valid && !isfinite(ell)) ? 1.0 : 0.0;
    if (per_point && valid) per_point[(size_t)blockIdx.y * n + perm[i]] = ell;
    block_sum<2>(v, red);
    if (tid == 0) {
        double* o = part + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * 2;
        o[0] = v[0];
        o[1] = v[1];
    }
}

template <int DX, int DY>
static hipError_t launch_epan_t(const cde_model* m, const EpanSets& sets, int nsets, int crit,
                                int chunks, double* partial, double* per_point, double* part,
                                hipStream_t stream)
{
    const int nblocks = (int)(m->npad / TILE);
    const int tpc = (nblocks + chunks - 1) / chunks;
    const int used = (nblocks + tpc - 1) / tpc;
    hipLaunchKernelGGL((k_loo_epan<DX, DY>), dim3(nblocks, nsets, used), dim3(TILE), 0, stream,
                       (const double*)m->spts, (const double*)m->tbox, (const double*)m->sbox,
                       (int)m->n, (int)m->npad, sets, tpc, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_epan_combine, dim3(nblocks, nsets), dim3(TILE), 0, stream,
                       (const double*)partial, used, (int)m->n, (int)m->npad, sets, crit,
                       (const int*)m->perm, per_point, part);
    return hipGetLastError();
}

template <int DX, int DY>
static int epan_chunks_t(const cde_model* m, int nsets, size_t max_doubles)
{
    return choose_chunks((const void*)k_loo_epan<DX, DY>, m, nsets, 2, max_doubles);
}

}  // namespace

#define CDE_EPAN_CASE(DX_, DY_) \
    case (DX_) * 8 + (DY_):     \
        return launch_epan_t<DX_, DY_>(m, sets, nsets, crit, chunks, partial, per_point, part, stream);

hipError_t launch_epan(const cde_model* m, const EpanSets& sets, int nsets, int crit, int chunks,
                       double* partial, double* per_point, double* part, hipStream_t stream)
{
    switch (m->dx * 8 + m->dy) {
        CDE_EPAN_CASE(1, 1) CDE_EPAN_CASE(1, 2) CDE_EPAN_CASE(2, 1) CDE_EPAN_CASE(2, 2)
        CDE_EPAN_CASE(3, 1) CDE_EPAN_CASE(3, 2) CDE_EPAN_CASE(4, 1) CDE_EPAN_CASE(4, 2)
        CDE_EPAN_CASE(5, 1) CDE_EPAN_CASE(5, 2) CDE_EPAN_CASE(6, 1) CDE_EPAN_CASE(6, 2)
        CDE_EPAN_CASE(7, 1) CDE_EPAN_CASE(7, 2) CDE_EPAN_CASE(8, 1) CDE_EPAN_CASE(8, 2)
        CDE_EPAN_CASE(16, 1) CDE_EPAN_CASE(16, 2)
        default: return hipErrorInvalidValue;
    }
}

#define CDE_EPAN_CHUNK_CASE(DX_, DY_) \
    case (DX_) * 8 + (DY_): return epan_chunks_t<DX_, DY_>(m, nsets, max_doubles);

int epan_chunks(const cde_model* m, int nsets, size_t max_doubles)
{
    switch (m->dx * 8 + m->dy) {
        CDE_EPAN_CHUNK_CASE(1, 1) CDE_EPAN_CHUNK_CASE(1, 2) CDE_EPAN_CHUNK_CASE(2, 1)
        CDE_EPAN_CHUNK_CASE(2, 2) CDE_EPAN_CHUNK_CASE(3, 1) CDE_EPAN_CHUNK_CASE(3, 2)
        CDE_EPAN_CHUNK_CASE(4, 1) CDE_EPAN_CHUNK_CASE(4, 2) CDE_EPAN_CHUNK_CASE(5, 1)
        CDE_EPAN_CHUNK_CASE(5, 2) CDE_EPAN_CHUNK_CASE(6, 1) CDE_EPAN_CHUNK_CASE(6, 2)
        CDE_EPAN_CHUNK_CASE(7, 1) CDE_EPAN_CHUNK_CASE(7, 2) CDE_EPAN_CHUNK_CASE(8, 1)
        CDE_EPAN_CHUNK_CASE(8, 2) CDE_EPAN_CHUNK_CASE(16, 1) CDE_EPAN_CHUNK_CASE(16, 2)
        default: return 1;
    }
}

}  // namespace cde
