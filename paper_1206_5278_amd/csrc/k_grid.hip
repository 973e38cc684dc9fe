// k_grid.hip -- exact LOO log-likelihood over a grid of scalar bandwidths
// (one hx for all x-dimensions, one hy for all y-dimensions), FP32 data.
//
// Definitions (Holmes, Gray & Isbell): Section 2 (scaled Gaussian kernel,
// eq. 1) and eq. (3) expanded as in Section 3.2.  For point i and grid cell
// (a, b) the sums are
//     den_i[a]    = sum_{j!=i} K_hx[a](x_i - x_j)
//     num_i[a][b] = sum_{j!=i} K_hx[a](x_i - x_j) K_hy[b](y_i - y_j).
// With scalar bandwidths both kernels are exponentials of the squared
// distances d2x_ij, d2y_ij times per-bandwidth coefficients, so
//     num_i[a][b] = sum_j ex_a(i,j) * ey_b(i,j)
// is, for each i, a dense contraction over j of an [Gx x J] matrix with a
// [J x Gy] matrix: the products and sums run on the matrix cores, while the
// VALU forms the distances and only Gx + Gy kernel values per pair (not
// Gx * Gy).
//
// Range: every exponent is taken relative to the point's nearest x-neighbour
// distance m_i and nearest y-neighbour distance my_i (over j != i, computed
// once per model by k_nn with the FP64 formula):
//     ex_a = 2^-((d2x - m_i) c_a),  ey_b = 2^-((d2y - my_i) c'_b),
// so ex <= 1 with ex = 1 at the x-neighbour (den' >= 1) and ey <= 1.  The
// shifts cancel in the ratio and are restored in FP64 by the finalisation.
//
// Passes (see the kernels for details):
//   1. the FP32 pass over all points (k_loo_grid32: one 16 x 16 grid tile per
//      block on v_mfma_f32_16x16x4f32; k_loo_grid32q: 32 x 32 quads on
//      v_mfma_f32_32x32x2f32), the tile of the smallest bandwidths with
//      biased exponents, FP32 tile sums folded into Kahan-compensated totals;
//   2. k_grid_finalize flags the (tile, point) pairs with a cell whose
//      shifted num' is too small for FP32 to have carried it, and
//      k_compact_points lists them; those are recomputed with FP64 kernel
//      values (v_exp_f32 of the fractional exponent scaled exactly by a power
//      of two) on v_mfma_f64_16x16x4f64: four points per product step when
//      their flagged cells lie in the tile's first 4 x 4 cells
//      (k_loo_grid_packed), one per step otherwise (k_loo_grid);
//   3. entries still below 2^-1000 are recomputed exactly with a per-entry
//      shift (k_grid_fixup), and k_grid_rows sums each setting in a fixed
//      order.
//
// x-distance options (dx = 16): FP32 differences (CDE_XTERM_VALU_F32), or
// |u_i|^2 + |u_j|^2 - 2 u_i.u_j on coordinates centred by the data mean with
// the cross term of each block's points against a whole 256-point j-tile
// computed on the matrix cores as a split-bf16 product (u = hi + lo;
// hi.hi + hi.lo + lo.hi accumulated in FP32 by v_mfma_f32_16x16x16_bf16) and
// staged in LDS (CDE_XTERM_MFMA_BF16X3).  Both trade exact FP64 differences
// for approximations whose errors the tests report and bound.
//
// Work decomposition: a 256-lane block owns a group of points and one grid
// tile (blockIdx.y); j streams through LDS in 256-point tiles.  Each lane
// forms the FP64 distance of one (point, row) pair of the current row group,
// and a cross-lane move (ds_bpermute, or a DPP row broadcast folded into the
// multiply at dx = 16) hands each MFMA operand lane the pair it needs, so
// every distance is computed once per tile of the grid.
#include <type_traits>

#include "cde_device.h"
#include "cde_kernels.h"

namespace cde {

// Compile-time loop: f(integral_constant<int, 0>) ... f(integral_constant<int, K-1>).
template <int K>
struct Unroll {
    template <class F>
    __device__ __forceinline__ static void run(F&& f)
    {
        Unroll<K - 1>::run(f);
        f(std::integral_constant<int, K - 1>{});
    }
};
template <>
struct Unroll<0> {
    template <class F>
    __device__ __forceinline__ static void run(F&&) {}
};

// Value of lane `L` of this lane's 16-lane row (DPP row_newbcast).
template <int L>
__device__ __forceinline__ float row_bcast(int v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, v, 0x150 + L, 0xF, 0xF, false));
}

typedef double v4d __attribute__((ext_vector_type(4)));

// 2^-t in FP64 for finite t >= 0: v_exp_f32 of the fractional part, an exact
// power-of-two scaling for the integer part (which saturates, giving 0, for
// the huge sentinel used for excluded pairs).
__device__ __forceinline__ double exp2_neg_wide(float t)
{
#pragma clang fp contract(off)
    const float fl = floorf(t);
    const float fr = t - fl;  // in [0, 1)
    return ldexp((double)__builtin_amdgcn_exp2f(-fr), (int)(-fl));
}

// Exponent argument of an excluded pair (j == i, or j past the end): finite,
// so that sentinel * c stays finite for any c < 3e18 (h > 5e-10), and its
// kernel value is exactly 0.
constexpr float EXCLUDED = 1e20f;

// Squared distances in x and in y, in FP64: the differences of FP32
// coordinates are exact in FP64, so the only roundings are those of the
// squares and sums (about 1e-16 relative).
template <int DX, int DY>
__device__ __forceinline__ void dist2(const double* a, const float* b, double& dxs, double& dys)
{
    double e = 0.0;
#pragma unroll
    for (int k = 0; k < DX; ++k) {
        double d = a[k] - (double)b[k];
        e = fma_(d, d, e);
    }
    double f = 0.0;
#pragma unroll
    for (int l = 0; l < DY; ++l) {
        double d = a[DX + l] - (double)b[DX + l];
        f = fma_(d, d, f);
    }
    dxs = e;
    dys = f;
}

template <int DX, int DY>
__device__ __forceinline__ void dist2(const double* a, const double* b, double& dxs, double& dys)
{
    double e = 0.0;
#pragma unroll
    for (int k = 0; k < DX; ++k) {
        double d = a[k] - b[k];
        e = fma_(d, d, e);
    }
    double f = 0.0;
#pragma unroll
    for (int l = 0; l < DY; ++l) {
        double d = a[DX + l] - b[DX + l];
        f = fma_(d, d, f);
    }
    dxs = e;
    dys = f;
}

template <int S>
__device__ __forceinline__ void own_f64(double (&dst)[S], const float* src)
{
    float t[S];
    load_row<S>(t, src);
#pragma unroll
    for (int q = 0; q < S; ++q) dst[q] = (double)t[q];
}

// Per point: nearest-neighbour squared distances in x and in y, j != i,
// exactly as the FP64 formula of dist2 gives them.  From 10 dimensions on,
// every pair is first screened in FP32 (ScreenedMin, cde_device.h): only
// candidates near the running FP32 minimum take the FP64 formula, and the
// FP64 nearest neighbour is always one of them, so the result equals the
// plain FP64 minimum.  (In fewer dimensions the screen's compares, minima
// and branch cost more than the FP64 formula it saves.)

template <int DX, int DY>
__device__ __forceinline__ void nn_body(int bx, int chunk, int nchunks, const float* __restrict__ pts,
                                        int n, double* __restrict__ nn, int npad)
{
    constexpr int S = row_stride(DX, DY);
    __shared__ float tile[TILE * S];
    const int tid = threadIdx.x;
    const int i = bx * TILE + tid;
    float own32[S];
    load_row<S>(own32, pts + (size_t)i * S);
    double own[S];
#pragma unroll
    for (int q = 0; q < S; ++q) own[q] = (double)own32[q];
    ScreenedMin sx, sy;
    double mx = inf_<double>(), my = inf_<double>();
    const int ntiles = (n + TILE - 1) / TILE;
    const int tpc = (ntiles + nchunks - 1) / nchunks;
    const int t0 = chunk * tpc, t1 = min(ntiles, t0 + tpc);
    for (int t = t0; t < t1; ++t) {
        __syncthreads();
        float pre[S];
        load_row<S>(pre, pts + ((size_t)t * TILE + tid) * S);
        store_row<S>(tile + tid * S, pre);
        __syncthreads();
        const int cnt = min(TILE, n - t * TILE);
        const int self = (t == (int)bx) ? tid : -1;
        if constexpr (DX + DY < 10) {
            for (int q = 0; q < cnt; ++q) {
                float pj[S];
                load_row<S>(pj, tile + q * S);
                double a, b;
                dist2<DX, DY>(own, pj, a, b);
                if (q == self) continue;
                mx = min_(mx, a);
                my = min_(my, b);
            }
            continue;
        }
        for (int q = 0; q < cnt; ++q) {
            if (q == self) continue;
            float pj[S];
            load_row<S>(pj, tile + q * S);
            float ex = 0.f, ey = 0.f;
#pragma unroll
            for (int k = 0; k < DX; ++k) {
                const float d = own32[k] - pj[k];
                ex = fma_(d, d, ex);
            }
#pragma unroll
            for (int l = 0; l < DY; ++l) {
                const float d = own32[DX + l] - pj[DX + l];
                ey = fma_(d, d, ey);
            }
            const bool cx = sx.candidate(ex);
            const bool cy = sy.candidate(ey);
            if (cx || cy) {
                double a, b;
                dist2<DX, DY>(own, pj, a, b);
                if (cx) mx = min_(mx, a);
                if (cy) my = min_(my, b);
            }
        }
    }
    // the minima of the chunks combine through an integer atomic min on the
    // bit patterns (non-negative doubles order like their bits): exact and
    // independent of the order; nn starts at +inf (k_nn_init)
    atomicMin((unsigned long long*)(nn + i), (unsigned long long)__double_as_longlong(mx));
    atomicMin((unsigned long long*)(nn + npad + i), (unsigned long long)__double_as_longlong(my));
}

// j-tile chunks of the neighbour-shift pass: a point block streams every j
// tile, so small sets would leave most of the device idle (a 16k-point job
// has 64 point blocks); chunks bring the launch to about 2048 blocks.  A
// function of n only.
static int nn_chunks(int64_t n)
{
    const int64_t ntiles = (n + TILE - 1) / TILE;
    const int64_t c = (2048 + ntiles - 1) / ntiles;
    return (int)std::max<int64_t>(1, std::min<int64_t>(c, ntiles));
}

// nn[p0 .. p1) and nn[npad + p0 .. npad + p1) = +inf
__global__ void k_nn_init(double* __restrict__ nn, int npad, int p0, int p1)
{
    const int i = p0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (i < p1) {
        nn[i] = inf_<double>();
        nn[npad + i] = inf_<double>();
    }
}

template <int DX, int DY>
__global__ __launch_bounds__(TILE) void k_nn(const float* __restrict__ pts, int n,
                                             double* __restrict__ nn, int npad)
{
    nn_body<DX, DY>(blockIdx.x, blockIdx.y, gridDim.y, pts, n, nn, npad);
}

// Grid coefficients (base 2), padded to a multiple of 16 with copies of the
// last value; only the first gx x gy cells are reported.
struct GridArgs {
    float cx[64];
    float cy[64];
    int gx, gy;    // real grid sizes
    int gxp, gyp;  // padded to multiples of 16
    int tile_of[16];  // FP32 pass: grid tile (ab * gyp/16 + bb) of each blockIdx.y
    int bias_ta, bias_tb;  // FP32 pass: the biased tile's a-tile and b-tile indices
};

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));

__device__ __forceinline__ short bf16_bits(float v)
{
    return __builtin_bit_cast(short, (__bf16)v);
}

// Split-bf16 operand halves of four consecutive centred coordinates.
__device__ __forceinline__ void split4(const float* x, const float* mean, v4s& hi, v4s& lo)
{
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const float u = x[e] - mean[e];
        const __bf16 h = (__bf16)u;
        hi[e] = __builtin_bit_cast(short, h);
        lo[e] = bf16_bits(u - (float)h);
    }
}

// The FP64 grid kernel: one 16 x 16 grid tile per blockIdx.y, PWF points per
// wave (4 PWF per block) on v_mfma_f64_16x16x4f64.  In a distance group a
// lane forms the pair of point q = (lane % 16) % PWF with tile row
// 4 ((lane % 16) / PWF) + lane / 16, so the row broadcast of lane idx of
// each 16-lane row hands MFMA step idx its four rows of point idx % PWF.
// With a point list (the rerun of flagged points), fewer points per wave
// spread a short list over more blocks; the work per pair is the same.
template <int DX, int DY, bool XT, int PWF>
__device__ __forceinline__ void grid64_body(int bx, int by, const float* __restrict__ pts,
                                            const double* __restrict__ nn, int n, int npad,
                                            const GridArgs& ga, const float* __restrict__ xmean,
                                            double* __restrict__ numbuf,
                                            double* __restrict__ denbuf,
                                            const int* __restrict__ plist,
                                            const int* __restrict__ pcount)
{
    constexpr int S = row_stride(DX, DY);
    static_assert(!XT || DX == 16, "the MFMA cross term is built for dx = 16");
    static_assert(PWF == 2 || PWF == 4 || PWF == 8, "2, 4 or 8 points per wave");
    static_assert(!XT || PWF == 8, "the cross-term layout holds 8 points per wave");
    constexpr int JG = 64 / PWF;  // tile rows per distance group
    __shared__ float tile[TILE * S];
    __shared__ float jnorm[XT ? TILE : 1];
    __shared__ float xcross[XT ? 4 * 8 * TILE : 1];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    // this wave's PWF points: i0 .. i0+PWF-1, or those list entries of plist
    const int i0 = bx * (4 * PWF) + wave * PWF;
    int cnt_list = 0;
    if (plist) {
        // the list of this grid tile (by)
        plist += (size_t)by * npad;
        cnt_list = pcount[by];
        if ((int)bx * (4 * PWF) >= cnt_list) return;  // whole block past the list (uniform)
    }
    auto point = [&](int q) -> int {
        if (!plist) return i0 + q;
        return plist[min(i0 + q, cnt_list - 1)];  // repeat the last entry in a ragged tail
    };
    auto point_valid = [&](int q) -> bool { return !plist || i0 + q < cnt_list; };
    const int tb = ga.gyp / 16;                 // b-tiles per row of tiles
    const int ab = by / tb, bb = by % tb;
    const bool do_den = (bb == 0);

    // distance role: point i0 + (lane%16)%PWF against tile row group*JG + jo
    const int di = point((lane & 15) % PWF);
    const int jo = 4 * ((lane & 15) / PWF) + (lane >> 4);
    double own[S];
    own_f64<S>(own, pts + (size_t)di * S);
    const double m_i = nn[di], my_i = nn[npad + di];
    // cross-term operands of this wave's points (B of the bf16 MFMA: point
    // i0 + (lane%16)%8, dimensions 4*(lane/16) .. +3) and the own norm
    float mean[XT ? DX : 1];
    v4s bhi, blo;
    float inorm = 0.f;
    if constexpr (XT) {
#pragma unroll
        for (int k = 0; k < DX; ++k) mean[k] = xmean[k];
        float xb[S];
        load_row<S>(xb, pts + (size_t)point(lane & 7) * S);
        split4(xb + 4 * (lane >> 4), mean + 4 * (lane >> 4), bhi, blo);
#pragma unroll
        for (int k = 0; k < DX; ++k) {
            const float u = (float)own[k] - mean[k];
            inorm = fma_(u, u, inorm);
        }
    }
    // MFMA role: row a = ab*16 + lane%16 of A, column b = bb*16 + lane%16 of B
    const float ca = ga.cx[ab * 16 + (lane & 15)];
    const float cb = ga.cy[bb * 16 + (lane & 15)];

    v4d acc[PWF];
    double dsum[PWF];
#pragma unroll
    for (int t = 0; t < PWF; ++t) {
        acc[t] = v4d{0.0, 0.0, 0.0, 0.0};
        dsum[t] = 0.0;
    }

    const int ntiles = (n + TILE - 1) / TILE;
    float pre[S];
    load_row<S>(pre, pts + (size_t)tid * S);
    for (int t = 0; t < ntiles; ++t) {
        __syncthreads();
        store_row<S>(tile + tid * S, pre);
        __syncthreads();
        if (t + 1 < ntiles) load_row<S>(pre, pts + ((size_t)(t + 1) * TILE + tid) * S);
        const int base = t * TILE;
        const int cnt = min(TILE, n - base);
        const int ngroups = (cnt + JG - 1) / JG;
        if constexpr (XT) {
            // norms of the tile's centred points (one per thread)
            float nj = 0.f;
#pragma unroll
            for (int k = 0; k < DX; ++k) {
                const float u = tile[tid * S + k] - mean[k];
                nj = fma_(u, u, nj);
            }
            jnorm[tid] = nj;
            // cross terms of this wave's 8 points against the 256 tile rows:
            // A = tile rows jb*16 + lane%16 (dims 4*(lane/16)..), B = own points
            float* xc = xcross + wave * 8 * TILE;
            for (int jb = 0; jb < TILE / 16; ++jb) {
                v4s ahi, alo;
                split4(tile + (jb * 16 + (lane & 15)) * S + 4 * (lane >> 4), mean + 4 * (lane >> 4),
                       ahi, alo);
                v4f c = {0.f, 0.f, 0.f, 0.f};
                c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi, bhi, c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi, blo, c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(alo, bhi, c, 0, 0, 0);
                // c[r]: row jb*16 + 4*(lane/16) + r, point column lane%16
                if ((lane & 15) < 8) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) xc[(lane & 7) * TILE + jb * 16 + 4 * (lane >> 4) + r] = c[r];
                }
            }
            __syncthreads();
        }
        for (int g = 0; g < ngroups; ++g) {
            const int jj = g * JG + jo;
            float pj[S];
            load_row<S>(pj, tile + jj * S);  // rows >= cnt hold packed padding (in bounds)
            double d2x, d2y;
            if constexpr (XT) {
                const float cr = xcross[wave * 8 * TILE + (lane & 7) * TILE + jj];
                d2x = (double)((inorm + jnorm[jj]) - 2.f * cr);
                double f = 0.0;
#pragma unroll
                for (int l = 0; l < DY; ++l) {
                    const double d = own[DX + l] - (double)pj[DX + l];
                    f = fma_(d, d, f);
                }
                d2y = f;
            } else {
                dist2<DX, DY>(own, pj, d2x, d2y);
            }
            // shifted distances, rounded to FP32 only after the subtraction
            float xa = (float)(d2x - m_i), ya = (float)(d2y - my_i);
            if (jj >= cnt || base + jj == di) {
                xa = EXCLUDED;
                ya = EXCLUDED;
            }
            const int xai = __float_as_int(xa), yai = __float_as_int(ya);
            // step idx = PWF s + q: point i0 + q against rows 4 s + k (k = lane/16)
            Unroll<16>::run([&](auto c) {
                constexpr int idx = decltype(c)::value;
                constexpr int q = idx % PWF;
                const double ex = exp2_neg_wide(row_bcast<idx>(xai) * ca);
                const double ey = exp2_neg_wide(row_bcast<idx>(yai) * cb);
                acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(ex, ey, acc[q], 0, 0, 0);
                dsum[q] += ex;  // used by the b-tile-0 blocks only
            });
        }
    }

    // num' for (i0+q, a, b): the f64 16x16x4 result puts row (lane/16) + 4r,
    // column lane%16 in register r of each lane.
#pragma unroll
    for (int q = 0; q < PWF; ++q) {
        const int i = point(q);
        const bool ok = point_valid(q);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int a = ab * 16 + (lane >> 4) + 4 * r;
            const int b = bb * 16 + (lane & 15);
            if (ok && a < ga.gx && b < ga.gy) numbuf[((size_t)a * ga.gy + b) * npad + i] = acc[q][r];
        }
    }
    if (do_den) {
        // den' partials: lane (a = lane%16, k = lane/16) summed its k-rows;
        // combine the four k-rows in a fixed order.
#pragma unroll
        for (int q = 0; q < PWF; ++q) {
            double v = dsum[q];
            v += __shfl_xor(v, 16, 64);
            v += __shfl_xor(v, 32, 64);
            const int a = ab * 16 + (lane & 15);
            if (lane < 16 && a < ga.gx && point_valid(q)) denbuf[(size_t)a * npad + point(q)] = v;
        }
    }
}

template <int DX, int DY, bool XT, int PWF>
__global__ __launch_bounds__(TILE) void k_loo_grid(const float* __restrict__ pts,
                                                   const double* __restrict__ nn, int n, int npad,
                                                   GridArgs ga, const float* __restrict__ xmean,
                                                   double* __restrict__ numbuf,
                                                   double* __restrict__ denbuf,
                                                   const int* __restrict__ plist,
                                                   const int* __restrict__ pcount)
{
    grid64_body<DX, DY, XT, PWF>(blockIdx.x, blockIdx.y, pts, nn, n, npad, ga, xmean, numbuf, denbuf,
                                 plist, pcount);
}

// Packed FP64 rerun of flagged points whose flagged cells all lie in the
// first 4 x 4 cells of their grid tile (local a < 4 and b < 4), which is
// where small shifted sums concentrate when the bandwidths grow with the
// index.  Rows of the 16 x 16 f64 product are (point p, a) = 4 p + a and its
// columns (point p, b) = 4 p + b, so its four diagonal 4 x 4 blocks are four
// points' cells; the off-diagonal blocks pair one point's x-kernel values
// with another's y-kernel values and are discarded.  One product step thus
// covers four points where grid64_body covers one.  The per-pair arithmetic
// is grid64_body's: FP64 distances, shifted distances rounded to FP32 after
// the FP64 subtraction, exp2_neg_wide kernel values, FP64 products summed
// over j in order.  The lists come from k_compact_points: packed entries
// fill a tile's list from its end, counted in pcount[32 + tile].
//
// A wave holds 4 points; a distance group is 16 tile rows.  Lane (k, c),
// k = lane / 16, c = lane % 16, forms the distance of point c % 4 to row
// 4 (c / 4) + k of the group; product step s then needs, in lane (k, c),
// the pair of point c / 4 and row 4 s + k, held by lane 16 k + 4 s + c / 4
// (a gather through ds_bpermute).
template <int DX, int DY>
__device__ __forceinline__ void grid64p_body(int bx, int by, const float* __restrict__ pts,
                                             const double* __restrict__ nn, int n, int npad,
                                             const GridArgs& ga, double* __restrict__ numbuf,
                                             double* __restrict__ denbuf, const int* __restrict__ plist,
                                             const int* __restrict__ pcount)
{
    constexpr int S = row_stride(DX, DY);
    constexpr int PPB = 16;  // points per block: 4 waves of 4
    __shared__ float tile[TILE * S];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    plist += (size_t)by * npad;
    const int cnt_list = pcount[32 + by];
    if (bx * PPB >= cnt_list) return;  // whole block past the list (uniform)
    const int e0 = bx * PPB + wave * 4;  // list entries of this wave's points
    // entry e sits at npad - 1 - e; a ragged tail repeats the last entry
    auto point = [&](int q) -> int { return plist[npad - 1 - min(e0 + q, cnt_list - 1)]; };
    auto point_valid = [&](int q) -> bool { return e0 + q < cnt_list; };
    const int tb = ga.gyp / 16;
    const int ab = by / tb, bb = by % tb;
    const bool do_den = (bb == 0);

    const int c = lane & 15, kr = lane >> 4;
    const int di = point(c & 3);
    const int jo = 4 * (c >> 2) + kr;
    double own[S];
    own_f64<S>(own, pts + (size_t)di * S);
    const double m_i = nn[di], my_i = nn[npad + di];
    // product role: row / column 4 (c / 4) + (c % 4): cell a = c % 4 of A, b = c % 4 of B
    const float ca = ga.cx[ab * 16 + (c & 3)];
    const float cb = ga.cy[bb * 16 + (c & 3)];

    v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
    double dsum = 0.0;
    const int ntiles = (n + TILE - 1) / TILE;
    float pre[S];
    load_row<S>(pre, pts + (size_t)tid * S);
    for (int t = 0; t < ntiles; ++t) {
        __syncthreads();
        store_row<S>(tile + tid * S, pre);
        __syncthreads();
        if (t + 1 < ntiles) load_row<S>(pre, pts + ((size_t)(t + 1) * TILE + tid) * S);
        const int base = t * TILE;
        const int cnt = min(TILE, n - base);
        const int ngroups = (cnt + 15) / 16;
        for (int g = 0; g < ngroups; ++g) {
            const int jj = g * 16 + jo;
            float pj[S];
            load_row<S>(pj, tile + jj * S);  // rows >= cnt hold packed padding (in bounds)
            double d2x, d2y;
            dist2<DX, DY>(own, pj, d2x, d2y);
            float xa = (float)(d2x - m_i), ya = (float)(d2y - my_i);
            if (jj >= cnt || base + jj == di) {
                xa = EXCLUDED;
                ya = EXCLUDED;
            }
            const int xai = __float_as_int(xa), yai = __float_as_int(ya);
            Unroll<4>::run([&](auto cc) {
                constexpr int st = decltype(cc)::value;
                const int src = 4 * (16 * kr + 4 * st + (c >> 2));  // byte address of the source lane
                const float xb = __int_as_float(__builtin_amdgcn_ds_bpermute(src, xai));
                const float yb = __int_as_float(__builtin_amdgcn_ds_bpermute(src, yai));
                const double ex = exp2_neg_wide(xb * ca);
                const double ey = exp2_neg_wide(yb * cb);
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ex, ey, acc, 0, 0, 0);
                dsum += ex;  // used by the b-tile-0 blocks only
            });
        }
    }

    // register r holds row kr + 4 r = (point r, a = kr) of column c =
    // (point c / 4, b = c % 4): the diagonal block is r = c / 4
    const int p = c >> 2;
    const double v = p == 0 ? acc[0] : p == 1 ? acc[1] : p == 2 ? acc[2] : acc[3];
    {
        const int a = ab * 16 + kr, b = bb * 16 + (c & 3);
        if (point_valid(p) && a < ga.gx && b < ga.gy) numbuf[((size_t)a * ga.gy + b) * npad + point(p)] = v;
    }
    if (do_den) {
        // den' of (point c / 4, a = c % 4): the four k-rows in a fixed order
        double d = dsum;
        d += __shfl_xor(d, 16, 64);
        d += __shfl_xor(d, 32, 64);
        const int a = ab * 16 + (c & 3);
        if (lane < 16 && a < ga.gx && point_valid(p)) denbuf[(size_t)a * npad + point(p)] = d;
    }
}

template <int DX, int DY>
__global__ __launch_bounds__(TILE) void k_loo_grid_packed(const float* __restrict__ pts,
                                                          const double* __restrict__ nn, int n, int npad,
                                                          GridArgs ga, double* __restrict__ numbuf,
                                                          double* __restrict__ denbuf,
                                                          const int* __restrict__ plist,
                                                          const int* __restrict__ pcount)
{
    grid64p_body<DX, DY>(blockIdx.x, blockIdx.y, pts, nn, n, npad, ga, numbuf, denbuf, plist, pcount);
}

// FP32 fast pass: the same decomposition with FP32 kernel values (plain
// v_exp_f32), v_mfma_f32_16x16x4f32 products and sums, partial sums over a
// 256-point j-tile folded into Kahan-compensated FP32 totals.  FP32 cannot
// carry a cell whose shifted num' falls far below 1; k_grid_finalize flags
// the points that have such a cell and those points are recomputed by the
// FP64 kernel above.  Such cells need both bandwidths small, so the grid
// tile holding the smallest hx and hy runs with BIAS: every kernel value
// carries an exact factor 2^GRID_BIAS (the exponent is biased by
// +GRID_BIAS), removed when the totals are written.  v_exp_f32 flushes
// results below 2^-126 to zero while the MFMA keeps denormal products, so
// the bias moves the smallest kept kernel value from 2^-126 to
// 2^-(149 + GRID_BIAS), at the cost of one subtraction per value and a
// biased exponent rounded at magnitude ~GRID_BIAS (below 2^-20 relative
// error per kernel value).  Flag thresholds: num' < 2^-130 in a biased tile
// (the terms lost, each below 2^-181, sum to at most n 2^-181, under 1e-9 of
// the cell for n <= 2^20), num' < 2^-80 elsewhere (n 2^-126 / 2^-80).
// Points per wave of the FP32 pass (4 or 8): fewer points per wave means
// fewer accumulator registers and more resident waves to hide the latency of
// each exponential feeding an MFMA.
#ifndef CDE_GRID32_POINTS_PER_WAVE
#define CDE_GRID32_POINTS_PER_WAVE 4
#endif

constexpr float GRID_BIAS = 32.f;

// How an operand lane of the FP32 pass receives its pair's shifted distance:
// up to this many x dimensions through ds_bpermute (the LDS crossbar, off the
// VALU) and one VGPR-only FMA for the biased exponent; beyond it through a
// DPP row broadcast folded into the multiply and a subtraction.  Measured:
// the gather saves 4.5% of the 16 x 16 grid pass at dx = 5 and costs 5% at
// dx = 16, where the FP64 rows the distances read already load the LDS.
#ifndef CDE_GRID32_GATHER_MAX_DX
#define CDE_GRID32_GATHER_MAX_DX 8
#endif

// How the FP32 pass forms the squared x-distance of a pair (XM):
//   XM_F64   FP64 differences of the FP32 coordinates (exact differences; the
//            library's path), shift subtracted in FP64;
//   XM_F32   the same formula entirely in FP32 (differences, squares, sums,
//            shift), a reported option;
//   XM_BF16X3  |u_i|^2 + |u_j|^2 - 2 u_i.u_j on centred coordinates u with the
//            cross term of the block's 16 points against each 256-row tile on
//            the matrix cores, split bf16 (u = hi + lo; hi.hi + hi.lo + lo.hi,
//            FP32 accumulate), a reported option.
constexpr int XM_F64 = 0, XM_F32 = 1, XM_BF16X3 = 2;

template <int DX, int DY, int PW, bool BIAS, int XM = XM_F64>
__device__ __forceinline__ void grid32_body(int bx, int by, const float* __restrict__ pts,
                                            const double* __restrict__ nn, int n, int npad,
                                            const GridArgs& ga, double* __restrict__ numbuf,
                                            double* __restrict__ denbuf,
                                            const float* __restrict__ xmean = nullptr)
{
    static_assert(PW == 4 || PW == 8, "4 or 8 points per wave");
    static_assert(XM != XM_BF16X3 || (DX == 16 && PW == 4),
                  "the MFMA cross term is built for dx = 16, 16 points per block");
    constexpr int S = row_stride(DX, DY);
    constexpr int JG = 64 / PW;  // tile rows per distance group
    __shared__ double tile[TILE * S];  // staged as doubles: one exact conversion per row
    __shared__ float jnorm[XM == XM_BF16X3 ? TILE : 1];
    __shared__ float xcross[XM == XM_BF16X3 ? 16 * TILE : 1];  // [block point][tile row]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int i0 = bx * (4 * PW) + wave * PW;
    const int tb = ga.gyp / 16;
    const int tile_id = ga.tile_of[by];
    const int ab = tile_id / tb, bb = tile_id % tb;
    const bool do_den = (bb == 0);
    // distance role: lane = 16 r + PW s + q forms point i0 + q against row
    // group*JG + 4 s + r; a row broadcast of position PW s + q then gives
    // every lane of row r the pair (i0 + q, group*JG + 4 s + r).
    const int pos = lane & 15;
    const int di = i0 + (pos % PW);
    const int jo = 4 * (pos / PW) + (lane >> 4);
    double own[S];
    own_f64<S>(own, pts + (size_t)di * S);
    const double m_i = nn[di], my_i = nn[npad + di];
    const float ca = ga.cx[ab * 16 + (lane & 15)];
    const float cb = ga.cy[bb * 16 + (lane & 15)];
    const float bias = vreg(BIAS ? GRID_BIAS : 0.f);  // in a VGPR: the subtraction stays VOP2
    // cross-term operands: B = the block's 16 points (column lane % 16,
    // dimensions 4 (lane / 16) .. + 3), and the own point's centred norm
    float mean[XM == XM_BF16X3 ? DX : 1];
    v4s bhi, blo;
    float inorm = 0.f;
    const int pb = wave * PW + (pos % PW);  // block index of the distance-role point
    if constexpr (XM == XM_BF16X3) {
#pragma unroll
        for (int k = 0; k < DX; ++k) mean[k] = xmean[k];
        float xb[S];
        load_row<S>(xb, pts + (size_t)(bx * (4 * PW) + (lane & 15)) * S);
        split4(xb + 4 * (lane >> 4), mean + 4 * (lane >> 4), bhi, blo);
#pragma unroll
        for (int k = 0; k < DX; ++k) {
            const float u = (float)own[k] - mean[k];
            inorm = fma_(u, u, inorm);
        }
    }
    const float m32 = (float)m_i, my32 = (float)my_i;

    v4f acc[PW];
    Kahan<float> tot[PW][4], dtot[PW];
    float dpart[PW];
#pragma unroll
    for (int q = 0; q < PW; ++q) {
        acc[q] = v4f{0.f, 0.f, 0.f, 0.f};
        dpart[q] = 0.f;
        dtot[q].zero();
#pragma unroll
        for (int r = 0; r < 4; ++r) tot[q][r].zero();
    }
    const int ntiles = (n + TILE - 1) / TILE;
    float pre[S];
    load_row<S>(pre, pts + (size_t)tid * S);
    for (int t = 0; t < ntiles; ++t) {
        __syncthreads();
        {
            double pd[S];
#pragma unroll
            for (int c = 0; c < S; ++c) pd[c] = (double)pre[c];
            store_row<S>(tile + tid * S, pd);
        }
        __syncthreads();
        if (t + 1 < ntiles) load_row<S>(pre, pts + ((size_t)(t + 1) * TILE + tid) * S);
        const int base = t * TILE;
        const int cnt = min(TILE, n - base);
        const int ngroups = (cnt + JG - 1) / JG;
        if constexpr (XM == XM_BF16X3) {
            // centred norms of the tile's rows (one per thread), and the cross
            // terms of the block's 16 points against this wave's 64 rows
            float nj = 0.f;
#pragma unroll
            for (int k = 0; k < DX; ++k) {
                const float u = (float)tile[tid * S + k] - mean[k];
                nj = fma_(u, u, nj);
            }
            jnorm[tid] = nj;
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) {
                const int jb = wave * 4 + rb;  // 16-row block of the tile
                float xr[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) xr[e] = (float)tile[(jb * 16 + (lane & 15)) * S + 4 * (lane >> 4) + e];
                v4s ahi, alo;
                split4(xr, mean + 4 * (lane >> 4), ahi, alo);
                v4f c = {0.f, 0.f, 0.f, 0.f};
                c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi, bhi, c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi, blo, c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(alo, bhi, c, 0, 0, 0);
                // c[r]: tile row jb*16 + 4 (lane/16) + r, block point lane % 16
#pragma unroll
                for (int r = 0; r < 4; ++r) xcross[(lane & 15) * TILE + jb * 16 + 4 * (lane >> 4) + r] = c[r];
            }
            __syncthreads();
        }
        for (int g = 0; g < ngroups; ++g) {
            const int jj = g * JG + jo;
            double pj[S];
            load_row<S>(pj, tile + jj * S);  // jj < 256: rows >= cnt are packed padding
            float xa, ya;
            if constexpr (XM == XM_F64) {
                double d2x, d2y;
                dist2<DX, DY>(own, pj, d2x, d2y);
                xa = (float)(d2x - m_i);
                ya = (float)(d2y - my_i);
            } else if constexpr (XM == XM_F32) {
                float ex2 = 0.f, ey2 = 0.f;
#pragma unroll
                for (int k = 0; k < DX; ++k) {
                    const float d = (float)own[k] - (float)pj[k];
                    ex2 = fma_(d, d, ex2);
                }
#pragma unroll
                for (int l = 0; l < DY; ++l) {
                    const float d = (float)own[DX + l] - (float)pj[DX + l];
                    ey2 = fma_(d, d, ey2);
                }
                xa = ex2 - m32;
                ya = ey2 - my32;
            } else {
                const double d2x = (double)((inorm + jnorm[jj]) - 2.f * xcross[pb * TILE + jj]);
                double d2y = 0.0;
#pragma unroll
                for (int l = 0; l < DY; ++l) {
                    const double d = own[DX + l] - pj[DX + l];
                    d2y = fma_(d, d, d2y);
                }
                xa = (float)(d2x - m_i);
                ya = (float)(d2y - my_i);
            }
            if (jj >= cnt || base + jj == di) {
                xa = EXCLUDED;
                ya = EXCLUDED;
            }
            const int xai = __float_as_int(xa), yai = __float_as_int(ya);
            if constexpr (DX <= CDE_GRID32_GATHER_MAX_DX) {
            // each operand lane fetches its pair through the LDS crossbar
            // (ds_bpermute, off the VALU) and forms its exponent with one
            // VGPR-only FMA
            Unroll<16>::run([&](auto c) {
                constexpr int idx = decltype(c)::value;  // idx = PW s + q
                constexpr int q = idx % PW;
                const int src = 4 * ((lane & 48) + idx);  // lane idx of this lane's 16-lane row
                const float xb = __int_as_float(__builtin_amdgcn_ds_bpermute(src, xai));
                const float yb = __int_as_float(__builtin_amdgcn_ds_bpermute(src, yai));
                const float ex = exp2_<float>(fmaf(-xb, ca, bias));
                const float ey = exp2_<float>(fmaf(-yb, cb, bias));
                acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(ex, ey, acc[q], 0, 0, 0);
                dpart[q] += ex;
            });
            } else {
            Unroll<16>::run([&](auto c) {
#pragma clang fp contract(off)  // DPP-fed v_mul_f32, then a VGPR-only v_sub_f32
                constexpr int idx = decltype(c)::value;  // idx = PW s + q
                constexpr int q = idx % PW;
                float ex, ey;
                if constexpr (BIAS) {
                    ex = exp2_<float>(bias - row_bcast<idx>(xai) * ca);
                    ey = exp2_<float>(bias - row_bcast<idx>(yai) * cb);
                } else {
                    ex = exp2_<float>(-(row_bcast<idx>(xai) * ca));
                    ey = exp2_<float>(-(row_bcast<idx>(yai) * cb));
                }
                acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(ex, ey, acc[q], 0, 0, 0);
                dpart[q] += ex;
            });
            }
        }
#pragma unroll
        for (int q = 0; q < PW; ++q) {
#pragma unroll
            for (int r = 0; r < 4; ++r) tot[q][r].add(acc[q][r]);
            acc[q] = v4f{0.f, 0.f, 0.f, 0.f};
            dtot[q].add(dpart[q]);
            dpart[q] = 0.f;
        }
    }
    // f32 16x16x4 result layout: register r holds row 4*(lane/16) + r
#pragma unroll
    for (int q = 0; q < PW; ++q) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int a = ab * 16 + 4 * (lane >> 4) + r;
            const int b = bb * 16 + (lane & 15);
            if (a < ga.gx && b < ga.gy)
                numbuf[((size_t)a * ga.gy + b) * npad + i0 + q] =
                    (double)tot[q][r].value() * (BIAS ? 0x1p-64 : 1.0);
        }
    }
    if (do_den) {
#pragma unroll
        for (int q = 0; q < PW; ++q) {
            double v = dtot[q].value();
            v += __shfl_xor(v, 16, 64);
            v += __shfl_xor(v, 32, 64);
            const int a = ab * 16 + (lane & 15);
            if (lane < 16 && a < ga.gx) denbuf[(size_t)a * npad + i0 + q] = v * (BIAS ? 0x1p-32 : 1.0);
        }
    }
}

template <int DX, int DY, int PW, bool BIAS, int XM = XM_F64>
// Resident waves: at most 4 per SIMD by LDS (the 16 x 16 pass) and by
// default 2 to 3 by registers; asking for 4 (dx <= 8) or 3 (dx = 16) makes
// the compiler fit the registers, with a few spills outside the pair loop.
// The spare waves let more VALU instructions dual-issue beside the products:
// photoz 500k 16 x 16 2,050 -> 1,929 ms, identical results.
__global__ __launch_bounds__(TILE, (DX >= 16 ? 3 : 4)) void k_loo_grid32(const float* __restrict__ pts,
                                                     const double* __restrict__ nn, int n, int npad,
                                                     GridArgs ga, double* __restrict__ numbuf,
                                                     double* __restrict__ denbuf,
                                                     const float* __restrict__ xmean)
{
    grid32_body<DX, DY, PW, BIAS, XM>(blockIdx.x, blockIdx.y, pts, nn, n, npad, ga, numbuf, denbuf, xmean);
}

// The FP32 pass for grids of at least 32 x 32 cells (both padded sides
// multiples of 32): a block owns a 32 x 32 quad of the grid (a-tiles 2 qa and
// 2 qa + 1, b-tiles 2 qb and 2 qb + 1) and accumulates it with
// v_mfma_f32_32x32x2f32, which moves more products per cycle than four
// 16 x 16 x 4 tiles.  Operand layout of that instruction: lane 32 k + m holds
// A[m][k] and B[k][m]; register r of lane l holds the result row
// 8 (r / 4) + 4 (l / 32) + r % 4 of column l % 32.  So a lane forms ex for
// a = 32 qa + lane % 32 and ey for b = 32 qb + lane % 32 of the j its half
// of the wave carries: one exponential per operand, two per 2-point step.
// Exponent biases are per a-tile and per b-tile (32 for the tile of the
// smallest hx, resp. hy, else 0); each cell is unscaled by its own factor,
// and the flag thresholds of k_grid_finalize (2^-130 for the tile biased on
// both sides, 2^-80 elsewhere) hold as for k_loo_grid32.
template <int DX, int DY, int PW>
// Three resident waves per SIMD instead of the two its registers allow by
// default (50k points, 32 x 32: 62.7 -> 59.2 ms, identical results).
__global__ __launch_bounds__(TILE, 3) void k_loo_grid32q(const float* __restrict__ pts,
                                                      const double* __restrict__ nn, int n, int npad,
                                                      GridArgs ga, double* __restrict__ numbuf,
                                                      double* __restrict__ denbuf)
{
    static_assert(PW == 2 || PW == 4, "2 or 4 points per wave");
    constexpr int S = row_stride(DX, DY);
    constexpr int JG = 64 / PW;  // tile rows per distance group
    __shared__ float tile[TILE * S];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int i0 = blockIdx.x * (4 * PW) + wave * PW;
    const int tqb = ga.gyp / 32;
    const int qa = blockIdx.y / tqb, qb = blockIdx.y % tqb;
    const bool do_den = (qb == 0);
    // The pair this lane forms in a distance group of JG rows: lane row
    // r = lane / 16 gives the k-half h = r / 2 and the step set r % 2; step
    // c = 16 (r % 2) + lane % 16 is point q = c % PW against rows 2 (c / PW)
    // and 2 (c / PW) + 1, of which this lane takes row 2 (c / PW) + h.
    const int lrow = lane >> 4;
    const int c = 16 * (lrow & 1) + (lane & 15);
    const int di = i0 + c % PW;
    const int jo = 2 * (c / PW) + (lrow >> 1);
    double own[S];
    own_f64<S>(own, pts + (size_t)di * S);
    const double m_i = nn[di], my_i = nn[npad + di];
    const int am = lane & 31;  // A row and B column of this lane
    const float ca = ga.cx[32 * qa + am];
    const float cb = ga.cy[32 * qb + am];
    const float bx = vreg(2 * qa + am / 16 == ga.bias_ta ? GRID_BIAS : 0.f);
    const float by = vreg(2 * qb + am / 16 == ga.bias_tb ? GRID_BIAS : 0.f);

    v16f acc[PW];
    Kahan<float> tot[PW][16], dtot[PW];
    float dpart[PW];
#pragma unroll
    for (int q = 0; q < PW; ++q) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            acc[q][r] = 0.f;
            tot[q][r].zero();
        }
        dpart[q] = 0.f;
        dtot[q].zero();
    }
    const int ntiles = (n + TILE - 1) / TILE;
    float pre[S];
    load_row<S>(pre, pts + (size_t)tid * S);
    for (int t = 0; t < ntiles; ++t) {
        __syncthreads();
        store_row<S>(tile + tid * S, pre);
        __syncthreads();
        if (t + 1 < ntiles) load_row<S>(pre, pts + ((size_t)(t + 1) * TILE + tid) * S);
        const int base = t * TILE;
        const int cnt = min(TILE, n - base);
        const int ngroups = (cnt + JG - 1) / JG;
        for (int g = 0; g < ngroups; ++g) {
            const int jj = g * JG + jo;
            float pj[S];
            load_row<S>(pj, tile + jj * S);  // jj < 256: rows >= cnt are packed padding
            double d2x, d2y;
            dist2<DX, DY>(own, pj, d2x, d2y);
            float xa = (float)(d2x - m_i), ya = (float)(d2y - my_i);
            if (jj >= cnt || base + jj == di) {
                xa = EXCLUDED;
                ya = EXCLUDED;
            }
            // lane rows duplicated pairwise: x0 holds rows (0, 0, 2, 2) of xa,
            // x1 rows (1, 1, 3, 3); a row broadcast of lane c % 16 then hands
            // each half of the wave its own row of step c
            if constexpr (DX <= CDE_GRID32_GATHER_MAX_DX) {
            // step st's pair for k-half h sits in lane 32 h + st: fetched
            // through ds_bpermute, exponent by one VGPR-only FMA
            const int xai = __float_as_int(xa), yai = __float_as_int(ya);
            Unroll<32>::run([&](auto cc) {
                constexpr int st = decltype(cc)::value;
                constexpr int q = st % PW;
                const int src = 4 * ((lane & 32) + st);
                const float xb = __int_as_float(__builtin_amdgcn_ds_bpermute(src, xai));
                const float yb = __int_as_float(__builtin_amdgcn_ds_bpermute(src, yai));
                const float ex = exp2_<float>(fmaf(-xb, ca, bx));
                const float ey = exp2_<float>(fmaf(-yb, cb, by));
                acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(ex, ey, acc[q], 0, 0, 0);
                dpart[q] += ex;
            });
            } else {
            const auto xs = __builtin_amdgcn_permlane16_swap(__float_as_uint(xa), __float_as_uint(xa), false, false);
            const auto ys = __builtin_amdgcn_permlane16_swap(__float_as_uint(ya), __float_as_uint(ya), false, false);
            const int x0 = (int)xs[0], x1 = (int)xs[1], y0 = (int)ys[0], y1 = (int)ys[1];
            Unroll<32>::run([&](auto cc) {
#pragma clang fp contract(off)  // v_mul_f32, then a VGPR-only v_sub_f32
                constexpr int st = decltype(cc)::value;
                constexpr int q = st % PW;
                const float xb = row_bcast<st % 16>(st < 16 ? x0 : x1);
                const float yb = row_bcast<st % 16>(st < 16 ? y0 : y1);
                const float ex = exp2_<float>(bx - xb * ca);
                const float ey = exp2_<float>(by - yb * cb);
                acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(ex, ey, acc[q], 0, 0, 0);
                dpart[q] += ex;
            });
            }
        }
#pragma unroll
        for (int q = 0; q < PW; ++q) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                tot[q][r].add(acc[q][r]);
                acc[q][r] = 0.f;
            }
            dtot[q].add(dpart[q]);
            dpart[q] = 0.f;
        }
    }
    // each cell's factor 2^(bias of its a-tile + bias of its b-tile) (den:
    // 2^(bias of its a-tile)) removed exactly
#pragma unroll
    for (int q = 0; q < PW; ++q) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int ar = 8 * (r / 4) + 4 * (lane >> 5) + (r % 4);
            const int a = 32 * qa + ar, b = 32 * qb + am;
            const int ea = (2 * qa + ar / 16 == ga.bias_ta) ? (int)GRID_BIAS : 0;
            const double sc = ldexp(1.0, -(ea + (int)by));
            if (a < ga.gx && b < ga.gy)
                numbuf[((size_t)a * ga.gy + b) * npad + i0 + q] = (double)tot[q][r].value() * sc;
        }
    }
    if (do_den) {
#pragma unroll
        for (int q = 0; q < PW; ++q) {
            double v = dtot[q].value();
            v += __shfl_xor(v, 32, 64);
            const int a = 32 * qa + am;
            if (lane < 32 && a < ga.gx) denbuf[(size_t)a * npad + i0 + q] = v * ldexp(1.0, -(int)bx);
        }
    }
}

struct GridFin {
    double cxa[64];   // c_a in FP64 (the same FP32 values the kernel used)
    double cyb[64];
    double log_cx[64];
    double log_cy[64];
    int gx, gy;
    int tb;             // grid tiles per row (gyp / 16)
    unsigned biased;    // bit t: tile t ran the FP32 pass with biased exponents
};

// Per (setting, point) finalisation in FP64; entries whose shifted num' is
// too small for FP32 to have carried it are queued for the exact fixup.
// flag_points != NULL (after the FP32 pass): mark (tile, point) pairs with a
// cell below the tile's threshold (2^-130 biased, 2^-80 otherwise), in
// flag_points[tile][npad] (bits: where in the tile the cells lie);
// otherwise queue entries below 2^-1000 for the per-entry fixup.
template <class Fin>
__device__ __forceinline__ void finalize_body(int i, int g, const double* __restrict__ numbuf,
                                              const double* __restrict__ denbuf,
                                              const double* __restrict__ nn, int n, int npad,
                                              const Fin& gf, int crit, double* __restrict__ ell,
                                              int* __restrict__ fix_count, int2* __restrict__ fix_list,
                                              int fix_cap, int* __restrict__ flag_points)
{
    if (i >= n) return;
    const int a = g / gf.gy, b = g - a * gf.gy;
    const double num = numbuf[(size_t)g * npad + i];
    const double den = denbuf[(size_t)a * npad + i];
    const double m = nn[i], my = nn[npad + i];
    double v;
    if (crit == CDE_COND)
        v = gf.log_cy[b] + log(num / den) - my * gf.cyb[b] * LN2;
    else
        v = gf.log_cx[a] + gf.log_cy[b] + log(num) - (m * gf.cxa[a] + my * gf.cyb[b]) * LN2 -
            log((double)(n - 1));
    ell[(size_t)g * npad + i] = v;
    if (flag_points) {
        const int t = (a / 16) * gf.tb + b / 16;
        const double lim = (gf.biased >> t) & 1u ? 0x1p-130 : 0x1p-80;
        // bit 0: a flagged cell in the tile's first 4 x 4 cells, bit 1: one
        // outside them (the point then takes the full rerun)
        if (!(num >= lim))
            atomicOr(flag_points + (size_t)t * npad + i, ((a & 15) < 4 && (b & 15) < 4) ? 1 : 2);
    } else if (!(num >= 0x1p-1000)) {
        const int slot = atomicAdd(fix_count, 1);
        if (slot < fix_cap) fix_list[slot] = make_int2(g, i);
    }
}

__global__ void k_grid_finalize(const double* __restrict__ numbuf, const double* __restrict__ denbuf,
                                const double* __restrict__ nn, int n, int npad, GridFin gf, int crit,
                                double* __restrict__ ell, int* __restrict__ fix_count,
                                int2* __restrict__ fix_list, int fix_cap,
                                int* __restrict__ flag_points)
{
    finalize_body(blockIdx.x * blockDim.x + threadIdx.x, blockIdx.y, numbuf, denbuf, nn, n, npad, gf,
                  crit, ell, fix_count, fix_list, fix_cap, flag_points);
}

// Lists of flagged points (order of a list does not affect any result).
// One list area per grid tile t, list[tile][npad]: points for the full rerun
// from its start (count[t] of them), points whose flagged cells all lie in
// the tile's first 4 x 4 cells from its end (count[32 + t]), when `pack`;
// the two never meet, since a tile flags at most n <= npad points.
__device__ __forceinline__ void compact_body(int i, int t, const int* __restrict__ flag, int n, int npad,
                                             int* __restrict__ count, int* __restrict__ list, bool pack)
{
    if (i >= n) return;
    const int f = flag[(size_t)t * npad + i];
    if (f == 0) return;
    if ((f & 2) || !pack)
        list[(size_t)t * npad + atomicAdd(count + t, 1)] = i;
    else
        list[(size_t)t * npad + npad - 1 - atomicAdd(count + 32 + t, 1)] = i;
}

__global__ void k_compact_points(const int* __restrict__ flag, int n, int npad, int* __restrict__ count,
                                 int* __restrict__ list, int pack)
{
    compact_body(blockIdx.x * blockDim.x + threadIdx.x, blockIdx.y, flag, n, npad, count, list, pack != 0);
}

// Exact recomputation of queued (setting, point) entries: one wave per entry,
// lanes split j; pass 1 finds the entry's largest term, pass 2 sums all terms
// relative to it (Kahan per lane, FP64 across lanes).  When more entries were
// flagged than the queue holds (fix_count > fix_cap), the waves instead scan
// every (setting, point) entry of numbuf and recompute each one below the
// same 2^-1000 threshold, so no flagged entry is ever left unfixed.
template <int DX, int DY, class Fin>
__device__ __forceinline__ void fixup_body(int wid, int nw, int p0, int p1, const float* __restrict__ pts,
                                           const double* __restrict__ nn, int n, int npad,
                                           const GridArgs& ga, const Fin& gf, int crit,
                                           const double* __restrict__ numbuf,
                                           const double* __restrict__ denbuf,
                                           double* __restrict__ ell,
                                           const int* __restrict__ fix_count,
                                           const int2* __restrict__ fix_list, int fix_cap)
{
    constexpr int S = row_stride(DX, DY);
    const int lane = threadIdx.x & 63;
    const int queued = *fix_count;
    const bool scan = queued > fix_cap;
    const int span = p1 - p0;  // the scan covers points [p0, p1)
    const int64_t count = scan ? (int64_t)ga.gx * ga.gy * span : queued;
    for (int64_t e = wid; e < count; e += nw) {
        int g, i;
        if (scan) {
            g = (int)(e / span);
            i = p0 + (int)(e - (int64_t)g * span);
            if (numbuf[(size_t)g * npad + i] >= 0x1p-1000) continue;  // wave-uniform
        } else {
            const int2 gi = fix_list[e];
            g = gi.x;
            i = gi.y;
        }
        const int a = g / ga.gy, b = g - a * ga.gy;
        const float ca = ga.cx[a], cb = ga.cy[b];
        double own[S];
        own_f64<S>(own, pts + (size_t)i * S);
        const double m_i = nn[i], my_i = nn[npad + i];
        // E_j = (d2x - m) c_a + (d2y - my) c_b, shifted distances rounded to
        // FP32 after the FP64 subtraction exactly as in k_loo_grid
        float emin = inf_<float>();
        for (int j = lane; j < n; j += 64) {
            if (j == i) continue;
            float pj[S];
            load_row<S>(pj, pts + (size_t)j * S);
            double d2x, d2y;
            dist2<DX, DY>(own, pj, d2x, d2y);
            emin = min_(emin, (float)(d2x - m_i) * ca + (float)(d2y - my_i) * cb);
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) emin = min_(emin, __shfl_xor(emin, off, 64));
        Kahan<float> s;
        s.zero();
        for (int j = lane; j < n; j += 64) {
            if (j == i) continue;
            float pj[S];
            load_row<S>(pj, pts + (size_t)j * S);
            double d2x, d2y;
            dist2<DX, DY>(own, pj, d2x, d2y);
            s.add(exp2_<float>(-((float)(d2x - m_i) * ca + (float)(d2y - my_i) * cb - emin)));
        }
        double v = s.value();
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) {
            const double den = denbuf[(size_t)a * npad + i];
            const double m = m_i, my = my_i;
            // sum_j 2^{-E_j} = 2^{-emin} * v, with E_j the shifted exponents
            double r;
            if (crit == CDE_COND)
                r = gf.log_cy[b] + log(v / den) - (double)emin * LN2 - my * gf.cyb[b] * LN2;
            else
                r = gf.log_cx[a] + gf.log_cy[b] + log(v) - (double)emin * LN2 -
                    (m * gf.cxa[a] + my * gf.cyb[b]) * LN2 - log((double)(n - 1));
            ell[(size_t)g * npad + i] = r;
        }
    }
}

template <int DX, int DY>
__global__ __launch_bounds__(TILE) void k_grid_fixup(const float* __restrict__ pts,
                                                     const double* __restrict__ nn, int n, int npad,
                                                     GridArgs ga, GridFin gf, int crit,
                                                     const double* __restrict__ numbuf,
                                                     const double* __restrict__ denbuf,
                                                     double* __restrict__ ell,
                                                     const int* __restrict__ fix_count,
                                                     const int2* __restrict__ fix_list, int fix_cap)
{
    fixup_body<DX, DY>((blockIdx.x * blockDim.x + threadIdx.x) >> 6, (gridDim.x * blockDim.x) >> 6, 0, n,
                       pts, nn, n, npad, ga, gf, crit, numbuf, denbuf, ell, fix_count, fix_list, fix_cap);
}

// Fixed-order sum of each setting's row of per-point values; optional copy
// of the rows to a caller buffer with row stride n; non-finite counts.
__device__ __forceinline__ void rows_body(int g, const double* __restrict__ ell, int n, int npad,
                                          double* __restrict__ totals, double* __restrict__ per_point,
                                          double* __restrict__ counts)
{
    __shared__ double red[8];
    double v[2] = {0.0, 0.0};
    for (int i = threadIdx.x; i < n; i += 256) {
        const double x = ell[(size_t)g * npad + i];
        v[0] += x;
        v[1] += isfinite(x) ? 0.0 : 1.0;
        if (per_point) per_point[(size_t)g * n + i] = x;
    }
    block_sum<2>(v, red);
    if (threadIdx.x == 0) {
        totals[g] = v[0];
        counts[g] = v[1];
    }
}

__global__ __launch_bounds__(256) void k_grid_rows(const double* __restrict__ ell, int n, int npad,
                                                   double* __restrict__ totals,
                                                   double* __restrict__ per_point,
                                                   double* __restrict__ counts)
{
    rows_body(blockIdx.x, ell, n, npad, totals, per_point, counts);
}

// ---------------------------------------------------------------- launchers

// Zero a small int buffer with a kernel (no memset node, so a caller may
// capture the sequence in a graph).
__global__ void k_zero_int(int* p, int cnt)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cnt) p[i] = 0;
}


// Work buffers of one grid call (carved from the caller's work area).
struct GridWork {
    double* numbuf;  // [G][npad]
    double* denbuf;  // [gx][npad]
    double* ell;     // [G][npad]
    int* fix_count;  // [1]
    int* flags;      // [tiles][npad] (tile, point) pairs needing the FP64 pass
    int* plist;      // [tiles][npad] per tile: the list of those points
    int* pcount;     // [tiles] list lengths
    int2* fix_list;  // [fix_cap] entries needing the per-entry recomputation
    int fix_cap;
};

template <int DX, int DY>
static hipError_t grid_t(const cde_model* m, const GridArgs& ga, const GridFin& gf, int crit,
                         int xm, const GridWork& w, double* totals, double* per_point,
                         double* counts, hipStream_t stream)
{
    const int nb = (int)(m->npad / TILE);
    const int n = (int)m->n, npad = (int)m->npad;
    const float* pts = (const float*)m->pts;
    const double* nn = (const double*)m->nn;
    hipError_t e;
    if (!m->nn_ready) {
        hipLaunchKernelGGL(k_nn_init, dim3((unsigned)((npad + 255) / 256)), dim3(256), 0, stream, (double*)m->nn,
                           npad, 0, npad);
        hipLaunchKernelGGL((k_nn<DX, DY>), dim3(nb, (unsigned)nn_chunks(n)), dim3(TILE), 0, stream, pts, n,
                           (double*)m->nn, npad);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    const int tiles = (ga.gxp / 16) * (ga.gyp / 16);
    const dim3 grid((unsigned)(npad / 32), (unsigned)tiles);
    const int G = ga.gx * ga.gy;
    const dim3 fgrid((unsigned)((n + 255) / 256), (unsigned)G);
    const float* xmean = (const float*)m->xmean;
    if (xm != XM_F64 && DX != 16) return hipErrorInvalidValue;
    {
        // FP32 pass over all points; flag (tile, point) pairs with a cell FP32
        // cannot carry and recompute those tiles of those points on the FP64
        // path (the FP32 denominators stand where b-tile 0 is not recomputed).
        hipLaunchKernelGGL(k_zero_int, dim3((unsigned)(((size_t)tiles * npad + 255) / 256)), dim3(256), 0, stream,
                           w.flags, tiles * npad);
        hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, stream, w.pcount, 64);
        constexpr int PW = CDE_GRID32_POINTS_PER_WAVE;
        if (xm == XM_F64 && ga.gxp % 32 == 0 && ga.gyp % 32 == 0) {
            constexpr int PWQ = 2;
            const int quads = (ga.gxp / 32) * (ga.gyp / 32);
            hipLaunchKernelGGL((k_loo_grid32q<DX, DY, PWQ>), dim3((unsigned)(npad / (4 * PWQ)), (unsigned)quads),
                               dim3(TILE), 0, stream, pts, nn, n, npad, ga, w.numbuf, w.denbuf);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        } else {
        // the biased tile, then the others (GridFin::biased marks which)
        GridArgs gb = ga, gu = ga;
        int nb_ = 0, nu_ = 0;
        for (int t = 0; t < tiles; ++t) {
            if ((gf.biased >> t) & 1u)
                gb.tile_of[nb_++] = t;
            else
                gu.tile_of[nu_++] = t;
        }
        const dim3 pgrid((unsigned)(npad / (4 * PW)));
        for (int biased = 1; biased >= 0; --biased) {
            const int cnt = biased ? nb_ : nu_;
            if (cnt == 0) continue;
            const GridArgs& gt = biased ? gb : gu;
            const dim3 g2(pgrid.x, (unsigned)cnt);
            if (xm == XM_F64) {
                if (biased)
                    hipLaunchKernelGGL((k_loo_grid32<DX, DY, PW, true>), g2, dim3(TILE), 0, stream, pts, nn, n,
                                       npad, gt, w.numbuf, w.denbuf, xmean);
                else
                    hipLaunchKernelGGL((k_loo_grid32<DX, DY, PW, false>), g2, dim3(TILE), 0, stream, pts, nn, n,
                                       npad, gt, w.numbuf, w.denbuf, xmean);
            } else if constexpr (DX == 16) {
                if (xm == XM_F32 && biased)
                    hipLaunchKernelGGL((k_loo_grid32<DX, DY, PW, true, XM_F32>), g2, dim3(TILE), 0, stream, pts,
                                       nn, n, npad, gt, w.numbuf, w.denbuf, xmean);
                else if (xm == XM_F32)
                    hipLaunchKernelGGL((k_loo_grid32<DX, DY, PW, false, XM_F32>), g2, dim3(TILE), 0, stream, pts,
                                       nn, n, npad, gt, w.numbuf, w.denbuf, xmean);
                else if (biased)
                    hipLaunchKernelGGL((k_loo_grid32<DX, DY, PW, true, XM_BF16X3>), g2, dim3(TILE), 0, stream,
                                       pts, nn, n, npad, gt, w.numbuf, w.denbuf, xmean);
                else
                    hipLaunchKernelGGL((k_loo_grid32<DX, DY, PW, false, XM_BF16X3>), g2, dim3(TILE), 0, stream,
                                       pts, nn, n, npad, gt, w.numbuf, w.denbuf, xmean);
            }
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        }
        hipLaunchKernelGGL(k_grid_finalize, fgrid, dim3(256), 0, stream, (const double*)w.numbuf,
                           (const double*)w.denbuf, nn, n, npad, gf, crit, w.ell, w.fix_count,
                           w.fix_list, w.fix_cap, w.flags);
        hipLaunchKernelGGL(k_compact_points, dim3((n + 255) / 256, (unsigned)tiles), dim3(256), 0, stream,
                           (const int*)w.flags, n, npad, w.pcount, w.plist, xm == XM_BF16X3 ? 0 : 1);
        if (xm != XM_BF16X3) {
            hipLaunchKernelGGL((k_loo_grid_packed<DX, DY>), dim3((unsigned)(npad / 16), (unsigned)tiles),
                               dim3(TILE), 0, stream, pts, nn, n, npad, ga, w.numbuf, w.denbuf,
                               (const int*)w.plist, (const int*)w.pcount);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        // Points per wave of the rerun.  Each block streams all n points, so
        // 8 per wave keeps that traffic low; up to 2^18 points the flagged
        // lists are short (a few thousand points: ~100 blocks of 32) and 2
        // per wave spreads them over 4x the blocks.  The bf16x3 variant reruns
        // with the same cross term (8 points per wave, the layout it needs).
        if (xm == XM_BF16X3) {
            if constexpr (DX == 16)
                hipLaunchKernelGGL((k_loo_grid<DX, DY, true, 8>), grid, dim3(TILE), 0, stream, pts, nn, n,
                                   npad, ga, xmean, w.numbuf, w.denbuf, (const int*)w.plist,
                                   (const int*)w.pcount);
        } else if (npad <= (1 << 18)) {
            const dim3 rgrid((unsigned)(npad / 8), (unsigned)tiles);
            hipLaunchKernelGGL((k_loo_grid<DX, DY, false, 2>), rgrid, dim3(TILE), 0, stream, pts, nn, n,
                               npad, ga, xmean, w.numbuf, w.denbuf, (const int*)w.plist,
                               (const int*)w.pcount);
        } else {
            hipLaunchKernelGGL((k_loo_grid<DX, DY, false, 8>), grid, dim3(TILE), 0, stream, pts, nn, n,
                               npad, ga, xmean, w.numbuf, w.denbuf, (const int*)w.plist,
                               (const int*)w.pcount);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_grid_finalize, fgrid, dim3(256), 0, stream, (const double*)w.numbuf,
                       (const double*)w.denbuf, nn, n, npad, gf, crit, w.ell, w.fix_count, w.fix_list,
                       w.fix_cap, (int*)nullptr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL((k_grid_fixup<DX, DY>), dim3(1024), dim3(TILE), 0, stream, pts, nn, n, npad,
                       ga, gf, crit, (const double*)w.numbuf, (const double*)w.denbuf, w.ell,
                       (const int*)w.fix_count, (const int2*)w.fix_list, w.fix_cap);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_grid_rows, dim3((unsigned)G), dim3(256), 0, stream, (const double*)w.ell, n,
                       npad, totals, per_point, counts);
    return hipGetLastError();
}

#define CDE_GRID_CASE(DX_, DY_)                                                                 \
    case (DX_) * 8 + (DY_):                                                                     \
        return grid_t<DX_, DY_>(m, ga, gf, crit, xm, w, totals, per_point, counts, stream);

// Column means of x (FP64 accumulation in a fixed order, one thread per
// dimension), stored as FP32: the centring of the cross-term option.
__global__ void k_colmean(const float* __restrict__ pts, int n, int dx, int stride,
                          float* __restrict__ mean)
{
    const int k = threadIdx.x;
    if (k >= dx) return;
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += (double)pts[(size_t)i * stride + k];
    mean[k] = (float)(s / n);
}

// Coefficients of a scalar-bandwidth grid (base 2, FP32 as the kernels use
// them, and their FP64 copies and log normalisations for the finalisation).
static void grid_coeffs(int dx, int dy, const double* hx, int n_hx, const double* hy, int n_hy,
                        GridArgs& ga, GridFin& gf)
{
    ga.gx = gf.gx = n_hx;
    ga.gy = gf.gy = n_hy;
    ga.gxp = (n_hx + 15) / 16 * 16;
    ga.gyp = (n_hy + 15) / 16 * 16;
    for (int a = 0; a < 64; ++a) {
        const double h = hx[a < n_hx ? a : n_hx - 1];
        ga.cx[a] = (float)(LOG2E / (2.0 * h * h));
        gf.cxa[a] = (double)ga.cx[a];
        gf.log_cx[a] = -dx * (log(h) + HALF_LOG_2PI);
    }
    for (int b = 0; b < 64; ++b) {
        const double h = hy[b < n_hy ? b : n_hy - 1];
        ga.cy[b] = (float)(LOG2E / (2.0 * h * h));
        gf.cyb[b] = (double)ga.cy[b];
        gf.log_cy[b] = -dy * (log(h) + HALF_LOG_2PI);
    }
    // The FP32 pass biases the grid tile that holds the smallest hx and the
    // smallest hy (the only cells that can fall far below 1 need both small).
    gf.tb = ga.gyp / 16;
    int amin = 0, bmin = 0;
    for (int a = 1; a < n_hx; ++a)
        if (hx[a] < hx[amin]) amin = a;
    for (int b = 1; b < n_hy; ++b)
        if (hy[b] < hy[bmin]) bmin = b;
    gf.biased = 1u << ((amin / 16) * gf.tb + bmin / 16);
    ga.bias_ta = amin / 16;
    ga.bias_tb = bmin / 16;
    for (int t = 0; t < 16; ++t) ga.tile_of[t] = t;
}

// Work layout of one grid call on a model of npad rows: numbuf [G][npad] |
// denbuf [gx][npad] | ell [G][npad] | fix_count [64] | flags [tiles][npad] |
// plist [tiles][npad] | pcount [64] | fix_list (the rest).  False if
// work_bytes cannot hold it.
static bool carve_grid_work(void* work, size_t work_bytes, int64_t npad, int n_hx, int n_hy, GridWork& w)
{
    const size_t G = (size_t)n_hx * n_hy;
    w.numbuf = (double*)work;
    w.denbuf = w.numbuf + G * npad;
    w.ell = w.denbuf + (size_t)n_hx * npad;
    w.fix_count = (int*)(w.ell + G * npad);
    w.flags = w.fix_count + 64;
    const size_t ntl = (size_t)((n_hx + 15) / 16) * ((n_hy + 15) / 16);  // grid tiles
    w.plist = w.flags + ntl * npad;
    w.pcount = w.plist + ntl * npad;
    w.fix_list = (int2*)(w.pcount + 64);
    const size_t used = (size_t)((char*)w.fix_list - (char*)work);
    if (used >= work_bytes) return false;
    w.fix_cap = (int)std::min<size_t>((work_bytes - used) / sizeof(int2), size_t(1) << 30);
    return true;
}

hipError_t launch_grid(cde_model* m, const double* hx, int n_hx, const double* hy, int n_hy, int crit,
                       int xm, double* totals, double* per_point, void* work, size_t work_bytes,
                       double* counts, hipStream_t stream)
{
    if (xm == XM_BF16X3 && !m->xmean_ready) {
        hipLaunchKernelGGL(k_colmean, dim3(1), dim3(64), 0, stream, (const float*)m->pts, (int)m->n,
                           m->dx, m->stride, (float*)m->xmean);
        hipError_t e0 = hipGetLastError();
        if (e0 != hipSuccess) return e0;
        m->xmean_ready = true;
    }
    GridArgs ga;
    GridFin gf;
    grid_coeffs(m->dx, m->dy, hx, n_hx, hy, n_hy, ga, gf);
    GridWork w;
    if (!carve_grid_work(work, work_bytes, m->npad, n_hx, n_hy, w)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, stream, w.fix_count, 1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    switch (m->dx * 8 + m->dy) {
        CDE_GRID_CASE(1, 1) CDE_GRID_CASE(1, 2) CDE_GRID_CASE(2, 1) CDE_GRID_CASE(2, 2)
        CDE_GRID_CASE(3, 1) CDE_GRID_CASE(3, 2) CDE_GRID_CASE(4, 1) CDE_GRID_CASE(4, 2)
        CDE_GRID_CASE(5, 1) CDE_GRID_CASE(5, 2) CDE_GRID_CASE(6, 1) CDE_GRID_CASE(6, 2)
        CDE_GRID_CASE(7, 1) CDE_GRID_CASE(7, 2) CDE_GRID_CASE(8, 1) CDE_GRID_CASE(8, 2)
        CDE_GRID_CASE(16, 1) CDE_GRID_CASE(16, 2)
        default: return hipErrorInvalidValue;
    }
}

size_t grid_work_bytes(const cde_model* m, int n_hx, int n_hy)
{
    const size_t G = (size_t)n_hx * n_hy;
    // queue of entries for the per-entry fixup: 1/64 of all entries (more are
    // handled by k_grid_fixup's scan of numbuf)
    const size_t fix_cap = std::max<size_t>(G * m->npad / 64, 4096);
    const size_t ntl = (size_t)((n_hx + 15) / 16) * ((n_hy + 15) / 16);  // grid tiles
    return sizeof(double) * (2 * G + n_hx) * m->npad + (2 * ntl * m->npad + 128) * sizeof(int) +
           fix_cap * sizeof(int2) + 64;
}


// ---------------------------------------------------------------- grouped launch
//
// One launch per pipeline stage over a work list of items, each item a range
// of points [p0, p1) of one model against all of that model's points, for a
// grid of at most 16 x 16 cells (one grid tile, which the FP32 pass biases).
// A block maps its index to (item, local block) through the prefix sums in
// GridBatch::pre and runs the same device function, on the same per-point
// arithmetic, as the one-model launch: each point's values are therefore
// bit-identical to cde_loo_loglik's, whatever the list holds.  A model's
// ranges run in order (their work buffers carry over between launches): each
// range runs the FP32 pass over its points and appends its flagged points
// to the model's lists, and the item that ends a model runs the FP64 reruns,
// the finalisation and the fixup over the whole model and sums its rows
// into the totals.

constexpr int GRID_BATCH_MAX = 8;  // items per launch

// Finalisation constants of grids up to 16 x 16 (the grouped launch).
struct GridFin16 {
    double cxa[16];
    double cyb[16];
    double log_cx[16];
    double log_cy[16];
    int gx, gy;
    int tb;
    unsigned biased;
};

struct GridBatchItem {
    const float* pts;
    double* nn;        // [2][npad] neighbour shifts of the model
    int n, npad;
    int p0, p1;        // points [p0, p1); p1 = npad for the model's last range
    int nn_chunks;     // j chunks of the neighbour-shift pass (nn_chunks(n))
    GridWork w;        // the model's grid work buffers
    double* totals;    // [G], written by the model's last range
    double* counts;    // [G] non-finite counts (model scratch)
    int64_t* nonfinite;
};

struct GridBatch {
    int count;
    int pre[GRID_BATCH_MAX + 1];  // blocks of items 0..k-1 in this launch
    GridBatchItem it[GRID_BATCH_MAX];
};

__device__ __forceinline__ int batch_item(const GridBatch& b, int bx)
{
    int k = 0;
    while (k + 1 < b.count && bx >= b.pre[k + 1]) ++k;
    return k;
}

// per item (blockIdx.y): clear the flags of its range and the fixup queue
// counter; the lists of flagged points are cleared by a model's first range
// only, since every range of the model appends to them
__global__ void k_batch_zero(GridBatch b)
{
    const GridBatchItem& t = b.it[blockIdx.y];
    const int i = t.p0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (i < t.p1) t.w.flags[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x < 64) {
        if (t.p0 == 0) t.w.pcount[threadIdx.x] = 0;
        if (threadIdx.x == 0) *t.w.fix_count = 0;
    }
}

// per item (blockIdx.y): the neighbour shifts of its range start at +inf
__global__ void k_nn_init_batch(GridBatch b)
{
    const GridBatchItem& t = b.it[blockIdx.y];
    const int i = t.p0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (i < t.p1) {
        t.nn[i] = inf_<double>();
        t.nn[t.npad + i] = inf_<double>();
    }
}

// blocks of an item: (point block of its range) x (j chunk), chunk fastest
template <int DX, int DY>
__global__ __launch_bounds__(TILE) void k_nn_batch(GridBatch b)
{
    const int k = batch_item(b, blockIdx.x);
    const GridBatchItem& t = b.it[k];
    const int local = blockIdx.x - b.pre[k];
    nn_body<DX, DY>(t.p0 / TILE + local / t.nn_chunks, local % t.nn_chunks, t.nn_chunks, t.pts, t.n, t.nn,
                    t.npad);
}

template <int DX, int DY, int PW>
__global__ __launch_bounds__(TILE, (DX >= 16 ? 3 : 4)) void k_loo_grid32_batch(GridBatch b, GridArgs ga)
{
    const int k = batch_item(b, blockIdx.x);
    const GridBatchItem& t = b.it[k];
    grid32_body<DX, DY, PW, true>(t.p0 / (4 * PW) + (blockIdx.x - b.pre[k]), 0, t.pts, t.nn, t.n, t.npad,
                                  ga, t.w.numbuf, t.w.denbuf);
}

template <bool FLAG>
__global__ void k_finalize_batch(GridBatch b, GridFin16 gf, int crit)
{
    const int k = batch_item(b, blockIdx.x);
    const GridBatchItem& t = b.it[k];
    const int i = t.p0 + (blockIdx.x - b.pre[k]) * blockDim.x + threadIdx.x;
    finalize_body(i, blockIdx.y, t.w.numbuf, t.w.denbuf, t.nn, t.n, t.npad, gf, crit, t.w.ell,
                  t.w.fix_count, t.w.fix_list, t.w.fix_cap, FLAG ? t.w.flags : (int*)nullptr);
}

__global__ void k_compact_batch(GridBatch b)
{
    const int k = batch_item(b, blockIdx.x);
    const GridBatchItem& t = b.it[k];
    const int i = t.p0 + (blockIdx.x - b.pre[k]) * blockDim.x + threadIdx.x;
    compact_body(i, 0, t.w.flags, t.n, t.npad, t.w.pcount, t.w.plist, true);
}

template <int DX, int DY>
__global__ __launch_bounds__(TILE) void k_rerun_packed_batch(GridBatch b, GridArgs ga)
{
    const int k = batch_item(b, blockIdx.x);
    const GridBatchItem& t = b.it[k];
    grid64p_body<DX, DY>(blockIdx.x - b.pre[k], 0, t.pts, t.nn, t.n, t.npad, ga, t.w.numbuf, t.w.denbuf,
                         t.w.plist, t.w.pcount);
}

template <int DX, int DY, int PWF>
__global__ __launch_bounds__(TILE) void k_rerun_batch(GridBatch b, GridArgs ga)
{
    const int k = batch_item(b, blockIdx.x);
    const GridBatchItem& t = b.it[k];
    grid64_body<DX, DY, false, PWF>(blockIdx.x - b.pre[k], 0, t.pts, t.nn, t.n, t.npad, ga, nullptr,
                                    t.w.numbuf, t.w.denbuf, t.w.plist, t.w.pcount);
}

constexpr int BATCH_FIX_BLOCKS = 128;  // fixup blocks per item

template <int DX, int DY>
__global__ __launch_bounds__(TILE) void k_fixup_batch(GridBatch b, GridArgs ga, GridFin16 gf, int crit)
{
    const GridBatchItem& t = b.it[blockIdx.y];
    fixup_body<DX, DY>((blockIdx.x * blockDim.x + threadIdx.x) >> 6, (gridDim.x * blockDim.x) >> 6, t.p0,
                       min(t.p1, t.n), t.pts, t.nn, t.n, t.npad, ga, gf, crit, t.w.numbuf, t.w.denbuf,
                       t.w.ell, t.w.fix_count, t.w.fix_list, t.w.fix_cap);
}

// rows of the items that end their model (blockIdx.y), one block per setting
__global__ __launch_bounds__(256) void k_rows_batch(GridBatch b)
{
    const GridBatchItem& t = b.it[blockIdx.y];
    rows_body(blockIdx.x, t.w.ell, t.n, t.npad, t.totals, nullptr, t.counts);
}

__global__ void k_counts_batch(GridBatch b, int nsets)
{
    const int k = threadIdx.x;
    if (k >= b.count || !b.it[k].nonfinite) return;
    double s = 0.0;
    for (int q = 0; q < nsets; ++q) s += b.it[k].counts[q];
    *b.it[k].nonfinite = (int64_t)s;
}

// Blocks of each item for a stage that covers its range in units of `per`
// points (rounded up); returns the total.
static int batch_prefix(GridBatch& b, int per)
{
    b.pre[0] = 0;
    for (int k = 0; k < b.count; ++k) b.pre[k + 1] = b.pre[k] + (b.it[k].p1 - b.it[k].p0 + per - 1) / per;
    return b.pre[b.count];
}

template <int DX, int DY>
static hipError_t grid_batch_t(const GridBatch& all, const bool* do_nn, const GridArgs& ga,
                               const GridFin16& gf, int crit, hipStream_t stream)
{
    constexpr int PW = CDE_GRID32_POINTS_PER_WAVE;
    const int G = ga.gx * ga.gy;
    hipError_t e;
    int maxr = 0;
    for (int k = 0; k < all.count; ++k) maxr = std::max(maxr, all.it[k].p1 - all.it[k].p0);
    hipLaunchKernelGGL(k_batch_zero, dim3((unsigned)((maxr + 255) / 256), (unsigned)all.count), dim3(256), 0,
                       stream, all);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // neighbour shifts of the ranges whose model has none yet
    GridBatch nb = all;
    nb.count = 0;
    for (int k = 0; k < all.count; ++k)
        if (do_nn[k]) nb.it[nb.count++] = all.it[k];
    if (nb.count > 0) {
        int nmax = 0;
        nb.pre[0] = 0;
        for (int k = 0; k < nb.count; ++k) {
            const int pts_k = nb.it[k].p1 - nb.it[k].p0;
            nmax = std::max(nmax, pts_k);
            nb.pre[k + 1] = nb.pre[k] + (pts_k + TILE - 1) / TILE * nb.it[k].nn_chunks;
        }
        hipLaunchKernelGGL(k_nn_init_batch, dim3((unsigned)((nmax + 255) / 256), (unsigned)nb.count), dim3(256), 0,
                           stream, nb);
        hipLaunchKernelGGL((k_nn_batch<DX, DY>), dim3((unsigned)nb.pre[nb.count]), dim3(TILE), 0, stream, nb);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    GridBatch b = all;
    int blocks = batch_prefix(b, 4 * PW);
    hipLaunchKernelGGL((k_loo_grid32_batch<DX, DY, PW>), dim3((unsigned)blocks), dim3(TILE), 0, stream, b, ga);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    blocks = batch_prefix(b, 256);
    hipLaunchKernelGGL(k_finalize_batch<true>, dim3((unsigned)blocks, (unsigned)G), dim3(256), 0, stream, b, gf,
                       crit);
    hipLaunchKernelGGL(k_compact_batch, dim3((unsigned)blocks), dim3(256), 0, stream, b);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // The rest runs once per model, with the range that ends it, over the
    // whole model: every range has appended its flagged points to the
    // model's lists, so the FP64 reruns run once, well filled, instead of
    // once per range; then the finalisation of all points (FP64 values where
    // rerun), the fixup queue and the row sums.  Each point's arithmetic is
    // the one-model launch's, so the totals stay bit-identical.
    GridBatch lb = all;
    lb.count = 0;
    for (int k = 0; k < all.count; ++k)
        if (all.it[k].p1 == all.it[k].npad) {
            lb.it[lb.count] = all.it[k];
            lb.it[lb.count++].p0 = 0;
        }
    if (lb.count == 0) return hipSuccess;
    // FP64 rerun of flagged points: the packed rerun (16 points per block),
    // then the full rerun with the points-per-wave rule of the one-model
    // launch (2 up to 2^18 rows, else 8), one launch per rule
    {
        GridBatch pb = lb;
        const int pblocks = batch_prefix(pb, 16);
        hipLaunchKernelGGL((k_rerun_packed_batch<DX, DY>), dim3((unsigned)pblocks), dim3(TILE), 0, stream, pb,
                           ga);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    for (int pwf : {2, 8}) {
        GridBatch rb = lb;
        rb.count = 0;
        for (int k = 0; k < lb.count; ++k)
            if ((lb.it[k].npad <= (1 << 18)) == (pwf == 2)) rb.it[rb.count++] = lb.it[k];
        if (rb.count == 0) continue;
        const int rblocks = batch_prefix(rb, 4 * pwf);
        if (pwf == 2)
            hipLaunchKernelGGL((k_rerun_batch<DX, DY, 2>), dim3((unsigned)rblocks), dim3(TILE), 0, stream, rb, ga);
        else
            hipLaunchKernelGGL((k_rerun_batch<DX, DY, 8>), dim3((unsigned)rblocks), dim3(TILE), 0, stream, rb, ga);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    const int lblocks = batch_prefix(lb, 256);
    hipLaunchKernelGGL(k_finalize_batch<false>, dim3((unsigned)lblocks, (unsigned)G), dim3(256), 0, stream, lb, gf,
                       crit);
    hipLaunchKernelGGL((k_fixup_batch<DX, DY>), dim3(BATCH_FIX_BLOCKS, (unsigned)lb.count), dim3(TILE), 0,
                       stream, lb, ga, gf, crit);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_rows_batch, dim3((unsigned)G, (unsigned)lb.count), dim3(256), 0, stream, lb);
    hipLaunchKernelGGL(k_counts_batch, dim3(1), dim3(64), 0, stream, lb, G);
    return hipGetLastError();
}

template <int DX, int DY>
static int batch_round_blocks()
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, (const void*)k_loo_grid32_batch<DX, DY, CDE_GRID32_POINTS_PER_WAVE>, TILE, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    return per_cu;
}

#define CDE_ROUND_CASE(DX_, DY_) \
    case (DX_) * 8 + (DY_): per_cu = batch_round_blocks<DX_, DY_>(); break;

int64_t grid_round_points(int dx, int dy, int ncu)
{
    int per_cu = 0;
    switch (dx * 8 + dy) {
        CDE_ROUND_CASE(1, 1) CDE_ROUND_CASE(1, 2) CDE_ROUND_CASE(2, 1) CDE_ROUND_CASE(2, 2)
        CDE_ROUND_CASE(3, 1) CDE_ROUND_CASE(3, 2) CDE_ROUND_CASE(4, 1) CDE_ROUND_CASE(4, 2)
        CDE_ROUND_CASE(5, 1) CDE_ROUND_CASE(5, 2) CDE_ROUND_CASE(6, 1) CDE_ROUND_CASE(6, 2)
        CDE_ROUND_CASE(7, 1) CDE_ROUND_CASE(7, 2) CDE_ROUND_CASE(8, 1) CDE_ROUND_CASE(8, 2)
        CDE_ROUND_CASE(16, 1) CDE_ROUND_CASE(16, 2)
        default: return 0;
    }
    return (int64_t)per_cu * (ncu > 0 ? ncu : 1) * 4 * CDE_GRID32_POINTS_PER_WAVE;
}

#define CDE_GRID_BATCH_CASE(DX_, DY_) \
    case (DX_) * 8 + (DY_): e = grid_batch_t<DX_, DY_>(b, do_nn + k0, ga, gf16, crit, stream); break;

hipError_t launch_grid_batch(const GridRange* r, int count, const double* hx, int n_hx, const double* hy,
                             int n_hy, int crit, hipStream_t stream)
{
    if (count < 1 || n_hx > 16 || n_hy > 16) return hipErrorInvalidValue;
    const int dx = r[0].m->dx, dy = r[0].m->dy;
    GridArgs ga;
    GridFin gf;
    grid_coeffs(dx, dy, hx, n_hx, hy, n_hy, ga, gf);
    GridFin16 gf16;
    for (int a = 0; a < 16; ++a) {
        gf16.cxa[a] = gf.cxa[a];
        gf16.cyb[a] = gf.cyb[a];
        gf16.log_cx[a] = gf.log_cx[a];
        gf16.log_cy[a] = gf.log_cy[a];
    }
    gf16.gx = gf.gx;
    gf16.gy = gf.gy;
    gf16.tb = gf.tb;
    gf16.biased = gf.biased;
    bool do_nn[GRID_BATCH_MAX * 64];
    if (count > GRID_BATCH_MAX * 64) return hipErrorInvalidValue;
    for (int k0 = 0; k0 < count; k0 += GRID_BATCH_MAX) {
        GridBatch b;
        b.count = std::min(GRID_BATCH_MAX, count - k0);
        for (int k = 0; k < b.count; ++k) {
            const GridRange& q = r[k0 + k];
            if (q.m->dx != dx || q.m->dy != dy) return hipErrorInvalidValue;
            GridBatchItem& t = b.it[k];
            t.pts = (const float*)q.m->pts;
            t.nn = (double*)q.m->nn;
            t.n = (int)q.m->n;
            t.npad = (int)q.m->npad;
            t.p0 = (int)q.i0;
            t.p1 = q.i1 == q.m->n ? (int)q.m->npad : (int)q.i1;
            t.nn_chunks = nn_chunks(q.m->n);
            if (!carve_grid_work(q.work, q.work_bytes, q.m->npad, n_hx, n_hy, t.w)) return hipErrorInvalidValue;
            t.totals = q.totals;
            t.counts = q.counts;
            t.nonfinite = q.nonfinite;
            do_nn[k0 + k] = q.do_nn;
        }
        hipError_t e = hipErrorInvalidValue;
        switch (dx * 8 + dy) {
            CDE_GRID_BATCH_CASE(1, 1) CDE_GRID_BATCH_CASE(1, 2) CDE_GRID_BATCH_CASE(2, 1)
            CDE_GRID_BATCH_CASE(2, 2) CDE_GRID_BATCH_CASE(3, 1) CDE_GRID_BATCH_CASE(3, 2)
            CDE_GRID_BATCH_CASE(4, 1) CDE_GRID_BATCH_CASE(4, 2) CDE_GRID_BATCH_CASE(5, 1)
            CDE_GRID_BATCH_CASE(5, 2) CDE_GRID_BATCH_CASE(6, 1) CDE_GRID_BATCH_CASE(6, 2)
            CDE_GRID_BATCH_CASE(7, 1) CDE_GRID_BATCH_CASE(7, 2) CDE_GRID_BATCH_CASE(8, 1)
            CDE_GRID_BATCH_CASE(8, 2) CDE_GRID_BATCH_CASE(16, 1) CDE_GRID_BATCH_CASE(16, 2)
            default: return hipErrorInvalidValue;
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace cde
