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
// num' >= 1 by construction).  Values are summed in FP32 over 32-point
// subtiles, the subtile sums are added into plain FP32 per-tile sums, and
// those are added once per 256-point tile into FP64 per-point totals held in
// LDS (FP64 accumulation in place of a compensated FP32 pair).  The
// reference is moved lazily, only when a subtile holds a term more than 2^32
// above it: the totals and the subtile's own sums are then rescaled, which is
// exact in real arithmetic (the common factor cancels in num/den); a subtile
// whose heaviest term may have overflowed is summed again against the moved
// reference.  The log of the ratio, the gradient combination and the sum
// over i run in FP64.

#include <cmath>

#include "cde_device.h"
#include "cde_kernels.h"

namespace cde {

namespace {

template <typename T, int DX, int DY, bool GRAD>
struct DiagLane {
    static constexpr int S = row_stride(DX, DY);
    static constexpr int SUB = 32;
    // Accumulated quantities: den, num, then (gradient) sum w dx_k^2,
    // sum v dx_k^2 and sum v dy_l^2.  The first group (den, w moments) is
    // relative to m, the second (num, v moments) to m2.
    static constexpr int NA = GRAD ? 2 + 2 * DX + DY : 2;
    static constexpr int NP = NA + 2;  // partial record: m, m2, then the NA totals
    static constexpr int MW = 2, MV = 2 + DX, MVY = 2 + 2 * DX;

    // Per-point totals: FP64 columns in LDS (column a of thread t at
    // lds[a * TILE + t]), touched once per tile, conflict-free, and kept off
    // the registers of the pair loop.
    static constexpr int LDS_DOUBLES = NA * TILE;

    T xi[DX], yi[DY], ncx[DX], ncy[DY];  // coordinates of i; negated kernel scales
    T m, m2;         // references of the x-kernel sums and of the product-kernel sums
    bool empty;      // no pair in this lane's j range
    double* lds;     // this thread's first total
    T mid[NA];       // plain sums of the subtiles of the current tile

    __device__ __forceinline__ void init_accumulators(double* lds_base)
    {
        lds = lds_base + threadIdx.x;
#pragma unroll
        for (int a = 0; a < NA; ++a) lds[a * TILE] = 0.0;
    }
    __device__ __forceinline__ void scale_total(int a, T f) { lds[a * TILE] *= (double)f; }
    __device__ __forceinline__ double total(int a) const { return lds[a * TILE]; }
    __device__ __forceinline__ void begin_tile()
    {
#pragma unroll
        for (int a = 0; a < NA; ++a) mid[a] = T(0);
    }
    __device__ __forceinline__ void end_tile()
    {
#pragma unroll
        for (int a = 0; a < NA; ++a) lds[a * TILE] += (double)mid[a];
    }
    static __host__ __device__ constexpr bool in_first(int a)
    {
        return a == 0 || (GRAD && a >= MW && a < MV);
    }

    // Negated base-2 exponents of the x-kernel and of the product kernel for
    // one j (ncx, ncy hold the negated scales).
    __device__ __forceinline__ void neg_exponents(const T* pj, T& g1, T& g2) const
    {
        T g = T(0);
#pragma unroll
        for (int k = 0; k < DX; ++k) {
            T d = xi[k] - pj[k];
            g = fma_(d * d, ncx[k], g);
        }
        T h = g;
#pragma unroll
        for (int l = 0; l < DY; ++l) {
            T d = yi[l] - pj[DX + l];
            h = fma_(d * d, ncy[l], h);
        }
        g1 = g;
        g2 = h;
    }

    // Initial references: minima of the exponents over the first points of
    // the first tile.
    __device__ __forceinline__ void prologue(const T* tile, int len, int self)
    {
        T a = -inf_<T>(), b = -inf_<T>();
        for (int q = 0; q < len; ++q) {
            if (q == self) continue;
            T pj[S];
            load_row<S>(pj, tile + q * S);
            T g1, g2;
            neg_exponents(pj, g1, g2);
            a = max_(a, g1);
            b = max_(b, g2);
        }
        // No candidate: the chunk's first tile holds point i alone, so the
        // chunk has no j != i; any finite reference serves (all terms are 0).
        empty = !(a > -inf_<T>());
        m = empty ? T(0) : -a;
        m2 = empty ? T(0) : -b;
    }

    // One pair (i, j): its kernel values relative to the current references
    // and the squared coordinate differences the moments need.
    struct Pair {
        T w, v, sq[DX], sqy[DY];
    };

    // Evaluates pair (i, row jj).  The exponent is formed negated (reference
    // minus exponent), so each kernel value is a plain 2^g.  TRACK also keeps
    // the largest g of the subtile (its heaviest term); FIRST starts it.
    template <bool MASK, bool TRACK, bool FIRST>
    __device__ __forceinline__ void eval(const T* tile, int jj, int lim, int self, T dmn, Pair& r,
                                         T& hi1, T& hi2) const
    {
        T pj[S];
        load_cols<DX + DY, S>(pj, tile + jj * S);
        T g1 = m;
#pragma unroll
        for (int k = 0; k < DX; ++k) {
            T d = xi[k] - pj[k];
            r.sq[k] = d * d;
            g1 = fma_(r.sq[k], ncx[k], g1);
        }
        T g2 = g1 + dmn;
#pragma unroll
        for (int l = 0; l < DY; ++l) {
            T d = yi[l] - pj[DX + l];
            r.sqy[l] = d * d;
            g2 = fma_(r.sqy[l], ncy[l], g2);
        }
        if (MASK) {
            const bool off = (jj == self) || (jj >= lim);
            g1 = off ? -inf_<T>() : g1;
            g2 = off ? -inf_<T>() : g2;
        }
        r.w = exp2_<T>(g1);
        r.v = exp2_<T>(g2);
        if (TRACK) {
            hi1 = FIRST ? g1 : max_(hi1, g1);
            hi2 = FIRST ? g2 : max_(hi2, g2);
        }
    }

    // Adds one evaluated pair to the subtile sums (FIRST starts them).
    template <bool FIRST>
    __device__ __forceinline__ void accum(T (&p)[NA], const Pair& r) const
    {
        if (FIRST) {
            p[0] = r.w;
            p[1] = r.v;
            if (GRAD) {
#pragma unroll
                for (int k = 0; k < DX; ++k) { p[MW + k] = r.w * r.sq[k]; p[MV + k] = r.v * r.sq[k]; }
#pragma unroll
                for (int l = 0; l < DY; ++l) p[MVY + l] = r.v * r.sqy[l];
            }
        } else {
            p[0] += r.w;
            p[1] += r.v;
            if (GRAD) {
#pragma unroll
                for (int k = 0; k < DX; ++k) {
                    p[MW + k] = fma_(r.w, r.sq[k], p[MW + k]);
                    p[MV + k] = fma_(r.v, r.sq[k], p[MV + k]);
                }
#pragma unroll
                for (int l = 0; l < DY; ++l) p[MVY + l] = fma_(r.v, r.sqy[l], p[MVY + l]);
            }
        }
    }

    // Sums of one subtile of SUB points starting at tile row j0, relative to
    // the current references (and, with TRACK, the subtile's largest negated
    // exponents).  MASK drops row `self` (point i itself) and rows at or
    // beyond `lim`.  Without the gradient the loop is software-pipelined by
    // one pair (pair q's exponentials are in flight while pair q-1 is added);
    // with it, the moments already fill the registers of four waves per SIMD
    // and the plain loop is kept.
    template <bool MASK, bool TRACK>
    __device__ __forceinline__ void sums(const T* tile, int j0, int lim, int self, T (&p)[NA],
                                         T& hi1, T& hi2) const
    {
        const T dmn = m2 - m;
        if constexpr (GRAD) {
            Pair r;
            eval<MASK, TRACK, true>(tile, j0, lim, self, dmn, r, hi1, hi2);
            accum<true>(p, r);
#pragma unroll
            for (int q = 1; q < 8; ++q) {
                eval<MASK, TRACK, false>(tile, j0 + q, lim, self, dmn, r, hi1, hi2);
                accum<false>(p, r);
            }
#pragma unroll 8
            for (int q = 8; q < SUB; ++q) {
                eval<MASK, TRACK, false>(tile, j0 + q, lim, self, dmn, r, hi1, hi2);
                accum<false>(p, r);
            }
        } else {
            Pair cur, nxt;
            eval<MASK, TRACK, true>(tile, j0, lim, self, dmn, cur, hi1, hi2);
            eval<MASK, TRACK, false>(tile, j0 + 1, lim, self, dmn, nxt, hi1, hi2);
            accum<true>(p, cur);
            cur = nxt;
#pragma unroll 6
            for (int q = 2; q < SUB; ++q) {
                eval<MASK, TRACK, false>(tile, j0 + q, lim, self, dmn, nxt, hi1, hi2);
                accum<false>(p, cur);
                cur = nxt;
            }
            accum<false>(p, cur);
        }
    }

    // Moves the reference of each lane whose subtile holds a term above it
    // to that heaviest term and rescales what the lane has summed so far
    // (exact in real arithmetic: the common factor cancels in num/den).  With
    // WITH_P the current subtile's sums are rescaled too.
    template <bool WITH_P>
    __device__ __forceinline__ void move_refs(T hi1, T hi2, T (&p)[NA])
    {
        if (hi1 > T(0)) {
            const T f = exp2_<T>(-hi1);
#pragma unroll
            for (int a = 0; a < NA; ++a)
                if (in_first(a)) {
                    scale_total(a, f);
                    mid[a] *= f;
                    if (WITH_P) p[a] *= f;
                }
            m -= hi1;
        }
        if (hi2 > T(0)) {
            const T f = exp2_<T>(-hi2);
#pragma unroll
            for (int a = 0; a < NA; ++a)
                if (!in_first(a)) {
                    scale_total(a, f);
                    mid[a] *= f;
                    if (WITH_P) p[a] *= f;
                }
            m2 -= hi2;
        }
    }

    // One subtile, added to the tile sums.  The pair loop keeps no minima: a
    // subtile sum above 2^slack (or an overflow) is what reveals a term far
    // above its reference.  Then the subtile is summed again with its largest
    // negated exponents tracked and the references move to the heaviest
    // terms.  A term up to 2^big above its reference is representable, so
    // below that the subtile's sums are rescaled with the totals (terms that
    // underflowed against the old reference are negligible against the new,
    // lower one); a heavier term, which may have overflowed, makes the
    // subtile be summed a third time against the moved references.
    template <bool MASK>
    __device__ __forceinline__ void subtile(const T* tile, int j0, int lim, int self)
    {
        const T sum_lim = sizeof(T) == 4 ? T(0x1p32) : T(0x1p512);
        const T big = sizeof(T) == 4 ? T(64) : T(640);
        T p[NA], hi1, hi2;
        sums<MASK, false>(tile, j0, lim, self, p, hi1, hi2);
        if (__any((p[0] > sum_lim) || (p[1] > sum_lim))) {
            sums<MASK, true>(tile, j0, lim, self, p, hi1, hi2);
            if (__any((hi1 > big) || (hi2 > big))) {
                move_refs<false>(hi1, hi2, p);
                sums<MASK, false>(tile, j0, lim, self, p, hi1, hi2);
            } else {
                move_refs<true>(hi1, hi2, p);
            }
        }
#pragma unroll
        for (int a = 0; a < NA; ++a) mid[a] += p[a];
    }

    // All rows of one LDS tile holding `cnt` points; `self` is the tile row
    // of point i (diagonal tile) or -1.  Full off-diagonal tiles take the
    // unmasked path.
    __device__ __forceinline__ void tile_pass(const T* tile, int cnt, int self)
    {
        begin_tile();
        if (self >= 0 || cnt < TILE) {
            for (int j0 = 0; j0 < cnt; j0 += SUB) subtile<true>(tile, j0, cnt, self);
        } else {
            for (int j0 = 0; j0 < TILE; j0 += SUB) subtile<false>(tile, j0, TILE, -1);
        }
        end_tile();
    }

    __device__ __forceinline__ double den() const { return total(0); }
    __device__ __forceinline__ double num() const { return total(1); }
};

}  // namespace

// Pair pass over one chunk of j tiles for 256 points and one setting
// (blockIdx.x: point block, blockIdx.y: setting, blockIdx.z: chunk of
// `tiles_per_chunk` tiles).  Each lane writes its partial record (the two
// references, then the NA totals relative to them) as NP planes of npad
// doubles at partial[((setting * chunks + chunk) * NP + field) * npad + i];
// an empty j range is marked by infinite references.
template <typename T, int DX, int DY, bool GRAD>
__global__ __launch_bounds__(TILE) void k_loo_diag(const T* __restrict__ pts, int n, int npad,
                                                   DiagSets<T> sets, int tiles_per_chunk,
                                                   double* __restrict__ partial)
{
    using L = DiagLane<T, DX, DY, GRAD>;
    constexpr int S = L::S;
    __shared__ T tile[TILE * S];
    __shared__ double totals[L::LDS_DOUBLES];

    const DiagSet<T>& st = sets.s[blockIdx.y];
    const int tid = threadIdx.x;
    const int i = blockIdx.x * TILE + tid;  // < npad: rows beyond n hold zeros

    L lane;
    {
        T own[S];
        load_row<S>(own, pts + (size_t)i * S);
#pragma unroll
        for (int k = 0; k < DX; ++k) { lane.xi[k] = own[k]; lane.ncx[k] = vreg(-st.c[k]); }
#pragma unroll
        for (int l = 0; l < DY; ++l) { lane.yi[l] = own[DX + l]; lane.ncy[l] = vreg(-st.c[DX + l]); }
    }
    lane.init_accumulators(totals);

    const int ntiles = (n + TILE - 1) / TILE;
    const int t0 = blockIdx.z * tiles_per_chunk;
    const int t1 = min(ntiles, t0 + tiles_per_chunk);
    T pre[S];
    load_row<S>(pre, pts + ((size_t)t0 * TILE + tid) * S);
    for (int t = t0; t < t1; ++t) {
        __syncthreads();
        store_row<S>(tile + tid * S, pre);
        __syncthreads();
        if (t + 1 < t1) load_row<S>(pre, pts + ((size_t)(t + 1) * TILE + tid) * S);
        const int cnt = min(TILE, n - t * TILE);
        const int self = (t == (int)blockIdx.x) ? tid : -1;
        if (t == t0) lane.prologue(tile, min(L::SUB, cnt), self);
        lane.tile_pass(tile, cnt, self);
    }

    double* o = partial + ((size_t)(blockIdx.y * gridDim.z + blockIdx.z) * L::NP) * npad + i;
    o[0] = lane.empty ? inf_<double>() : (double)lane.m;
    o[npad] = lane.empty ? inf_<double>() : (double)lane.m2;
#pragma unroll
    for (int a = 0; a < L::NA; ++a) o[(size_t)(2 + a) * npad] = lane.total(a);
}

// Merges the chunk partials of each point in chunk order and finalises it
// in FP64: totals relative to the smallest reference M are the sum over
// chunks of total_c * 2^(M - m_c) (each factor <= 1; an empty chunk, with
// m_c infinite, contributes nothing).  Then l_i (and its gradient terms),
// the per-point output and one fixed-order block row of part per (setting,
// 256-point block).
template <typename T, int DX, int DY, bool GRAD>
__global__ __launch_bounds__(TILE) void k_diag_combine(const double* __restrict__ partial,
                                                       int chunks, int n, int npad,
                                                       DiagSets<T> sets, int crit,
                                                       double* __restrict__ per_point,
                                                       double* __restrict__ part)
{
    using L = DiagLane<T, DX, DY, GRAD>;
    constexpr int NA = L::NA, NP = L::NP;
    constexpr int P = DX + DY;
    constexpr int NV = GRAD ? P + 2 : 2;  // l_i, [gradient], non-finite count
    __shared__ double red[4 * NV];

    const DiagSet<T>& st = sets.s[blockIdx.y];
    const int tid = threadIdx.x;
    const int i = blockIdx.x * TILE + tid;
    const double* base = partial + (size_t)blockIdx.y * chunks * NP * npad + i;

    double M = inf_<double>(), M2 = inf_<double>();
    for (int c = 0; c < chunks; ++c) {
        M = fmin(M, base[(size_t)c * NP * npad]);
        M2 = fmin(M2, base[((size_t)c * NP + 1) * npad]);
    }
    double tot[NA];
#pragma unroll
    for (int a = 0; a < NA; ++a) tot[a] = 0.0;
    for (int c = 0; c < chunks; ++c) {
        const double* r = base + (size_t)c * NP * npad;
        const double mc = r[0], m2c = r[npad];
        const double f1 = isinf(mc) ? 0.0 : exp2(M - mc);
        const double f2 = isinf(m2c) ? 0.0 : exp2(M2 - m2c);
#pragma unroll
        for (int a = 0; a < NA; ++a) tot[a] += r[(size_t)(2 + a) * npad] * (L::in_first(a) ? f1 : f2);
    }

    const bool valid = i < n;
    const double D = tot[0], U = tot[1];
    double v[NV];
    double ell;
    if (crit == CDE_COND)
        ell = log(U / D) + (M - M2) * LN2 + st.log_cy;
    else
        ell = log(U) - M2 * LN2 + st.log_cx + st.log_cy - log((double)(n - 1));
    v[0] = valid ? ell : 0.0;
    if (GRAD) {
#pragma unroll
        for (int k = 0; k < DX; ++k) {
            const double gv = tot[L::MV + k] / U;
            const double gw = tot[L::MW + k] / D;
            const double g = crit == CDE_COND ? (gv - gw) * st.inv_h3[k]
                                              : gv * st.inv_h3[k] - st.inv_h[k];
            v[1 + k] = valid ? g : 0.0;
        }
#pragma unroll
        for (int l = 0; l < DY; ++l) {
            const double g = (tot[L::MVY + l] / U) * st.inv_h3[DX + l] - st.inv_h[DX + l];
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
    __shared__ double totals[L::LDS_DOUBLES];
    const DiagSet<T>& st = sets.s[0];
    const int tid = threadIdx.x;
    const int64_t e = (int64_t)blockIdx.x * TILE + tid;
    const int64_t total = q * k;
    const int64_t ec = e < total ? e : total - 1;  // lanes past the end mirror the last pair
    const int64_t qq = ec / k, gg = ec - qq * k;

    L lane;
#pragma unroll
    for (int kk = 0; kk < DX; ++kk) { lane.xi[kk] = xq[qq * DX + kk]; lane.ncx[kk] = -st.c[kk]; }
#pragma unroll
    for (int l = 0; l < DY; ++l) { lane.yi[l] = yg[gg * DY + l]; lane.ncy[l] = -st.c[DX + l]; }
    lane.init_accumulators(totals);

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
        lane.tile_pass(tile, cnt, -1);
    }
    if (e < total) {
        const double D = lane.den(), U = lane.num();
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

// Tiles per chunk for a given chunk count (every chunk non-empty).
static int tiles_per_chunk(int ntiles, int chunks) { return (ntiles + chunks - 1) / chunks; }

// Chunk count by a makespan model: with B = blocks per chunk layer and R
// resident blocks per CU of `kern`, C chunks of ceil(ntiles / C) tiles run in
// ceil(B C / (R * CUs)) rounds, each as long as its tiles plus the chunk's
// start-up (about 1/8 of a tile).  The smallest C of least modelled time
// wins, within `max_doubles` of partial storage (np planes per chunk).
int choose_chunks(const void* kern, const cde_model* m, int nsets, int np, size_t max_doubles)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, TILE, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    const double slots = (double)per_cu * (m->ncu > 0 ? m->ncu : 1);
    const int ntiles = (int)(m->npad / TILE);
    const double layer = (double)ntiles * nsets;
    int best = 1;
    double best_t = 0.0;
    for (int c = 1; c <= 64 && c <= ntiles; ++c) {
        const int tpc = tiles_per_chunk(ntiles, c);
        const int used = (ntiles + tpc - 1) / tpc;
        if (used != c) continue;
        if ((size_t)nsets * used * np * (size_t)m->npad > max_doubles) break;
        const double t = std::ceil(layer * used / slots) * (tpc + 0.125);
        if (c == 1 || t < best_t * (1.0 - 1e-9)) {
            best = c;
            best_t = t;
        }
    }
    return best;
}

template <typename T, int DX, int DY, bool GRAD>
static hipError_t launch_diag_t(const cde_model* m, const DiagSets<T>& sets, int nsets, int crit,
                                int chunks, double* partial, double* per_point, double* part,
                                hipStream_t stream)
{
    const int nblocks = (int)(m->npad / TILE);
    const int tpc = tiles_per_chunk(nblocks, chunks);
    const int used = (nblocks + tpc - 1) / tpc;
    hipLaunchKernelGGL((k_loo_diag<T, DX, DY, GRAD>), dim3(nblocks, nsets, used), dim3(TILE), 0,
                       stream, (const T*)m->pts, (int)m->n, (int)m->npad, sets, tpc, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_diag_combine<T, DX, DY, GRAD>), dim3(nblocks, nsets), dim3(TILE), 0,
                       stream, (const double*)partial, used, (int)m->n, (int)m->npad, sets, crit,
                       per_point, part);
    return hipGetLastError();
}

template <typename T, int DX, int DY, bool GRAD>
static int diag_chunks_t(const cde_model* m, int nsets, size_t max_doubles)
{
    return choose_chunks((const void*)k_loo_diag<T, DX, DY, GRAD>, m, nsets,
                         DiagLane<T, DX, DY, GRAD>::NP, max_doubles);
}

#define CDE_DIAG_CASE(DX_, DY_)                                                                 \
    case (DX_) * 8 + (DY_):                                                                     \
        return grad ? launch_diag_t<T, DX_, DY_, true>(m, sets, nsets, crit, chunks, partial,    \
                                                       per_point, part, stream)                 \
                    : launch_diag_t<T, DX_, DY_, false>(m, sets, nsets, crit, chunks, partial,   \
                                                        per_point, part, stream);

template <typename T>
hipError_t launch_diag(const cde_model* m, const DiagSets<T>& sets, int nsets, int crit, bool grad,
                       int chunks, double* partial, double* per_point, double* part,
                       hipStream_t stream)
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

#define CDE_CHUNK_CASE(DX_, DY_)                                                 \
    case (DX_) * 8 + (DY_):                                                      \
        return grad ? diag_chunks_t<T, DX_, DY_, true>(m, nsets, max_doubles)    \
                    : diag_chunks_t<T, DX_, DY_, false>(m, nsets, max_doubles);

template <typename T>
int diag_chunks(const cde_model* m, int nsets, bool grad, size_t max_doubles)
{
    switch (m->dx * 8 + m->dy) {
        CDE_CHUNK_CASE(1, 1) CDE_CHUNK_CASE(1, 2) CDE_CHUNK_CASE(2, 1) CDE_CHUNK_CASE(2, 2)
        CDE_CHUNK_CASE(3, 1) CDE_CHUNK_CASE(3, 2) CDE_CHUNK_CASE(4, 1) CDE_CHUNK_CASE(4, 2)
        CDE_CHUNK_CASE(5, 1) CDE_CHUNK_CASE(5, 2) CDE_CHUNK_CASE(6, 1) CDE_CHUNK_CASE(6, 2)
        CDE_CHUNK_CASE(7, 1) CDE_CHUNK_CASE(7, 2) CDE_CHUNK_CASE(8, 1) CDE_CHUNK_CASE(8, 2)
        CDE_CHUNK_CASE(16, 1) CDE_CHUNK_CASE(16, 2)
        default: return 1;
    }
}

size_t diag_partial_doubles(const cde_model* m, int nsets, bool grad, int chunks)
{
    const int na = grad ? 2 + 2 * m->dx + m->dy : 2;
    return (size_t)nsets * chunks * (na + 2) * (size_t)m->npad;
}

template hipError_t launch_diag<float>(const cde_model*, const DiagSets<float>&, int, int, bool, int,
                                       double*, double*, double*, hipStream_t);
template hipError_t launch_diag<double>(const cde_model*, const DiagSets<double>&, int, int, bool,
                                        int, double*, double*, double*, hipStream_t);
template int diag_chunks<float>(const cde_model*, int, bool, size_t);
template int diag_chunks<double>(const cde_model*, int, bool, size_t);

}  // namespace cde
