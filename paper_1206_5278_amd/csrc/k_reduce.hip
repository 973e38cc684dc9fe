// k_reduce.hip -- data packing and the fixed-order FP64 reduction of
// per-block partials (the sum over i of eq. 3).
#include "cde_device.h"
#include "cde_kernels.h"

namespace cde {

template <typename T>
__global__ void k_pack(const T* __restrict__ x, const T* __restrict__ y, int64_t n, int dx, int dy,
                       int stride, int64_t npad, T* __restrict__ pts)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= npad * stride) return;
    const int64_t r = e / stride;
    const int c = (int)(e - r * stride);
    T v = T(0);
    if (r < n) {
        if (c < dx) v = x[r * dx + c];
        else if (c < dx + dy) v = y[r * dy + (c - dx)];
    }
    pts[e] = v;
}

template <typename T>
hipError_t launch_pack(cde_model* m, const T* x, const T* y, hipStream_t stream)
{
    const int64_t total = m->npad * m->stride;
    const unsigned blocks = (unsigned)((total + 255) / 256);
    hipLaunchKernelGGL((k_pack<T>), dim3(blocks), dim3(256), 0, stream, x, y, m->n, m->dx, m->dy,
                       m->stride, m->npad, (T*)m->pts);
    return hipGetLastError();
}

template hipError_t launch_pack<float>(cde_model*, const float*, const float*, hipStream_t);
template hipError_t launch_pack<double>(cde_model*, const double*, const double*, hipStream_t);

// Order-preserving map of a double onto unsigned 64-bit integers (negative
// values reversed below the positive ones), so that integer atomics take an
// exact, order-independent minimum and maximum.
__device__ __forceinline__ unsigned long long ordered_bits(double v)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

// Per-dimension minimum and maximum of the packed rows r < n, and a flag for
// non-finite values: ext[2 c] = min, ext[2 c + 1] = max (ordered bits) for
// column c < d, ext[2 MAXP] = non-finite flag.  ext must hold the identity
// values (k_extent_init) before the first block runs.
__global__ void k_extent_init(unsigned long long* ext)
{
    const int c = threadIdx.x;
    if (c < MAXP) {
        ext[2 * c] = ~0ull;
        ext[2 * c + 1] = 0ull;
    }
    if (c == 0) ext[2 * MAXP] = 0ull;
}

template <typename T>
__global__ __launch_bounds__(256) void k_extent(const T* __restrict__ pts, int64_t n, int d, int stride,
                                                unsigned long long* __restrict__ ext)
{
    __shared__ unsigned long long lo[4][MAXP], hi[4][MAXP];
    __shared__ int bad[4];
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int nonfinite = 0;
    for (int c = 0; c < d; ++c) {
        double v = r < n ? (double)pts[r * stride + c] : 0.0;
        nonfinite |= (r < n && !isfinite(v)) ? 1 : 0;
        if (!isfinite(v)) v = 0.0;
        double a = r < n ? v : __builtin_inf(), b = r < n ? v : -__builtin_inf();
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            a = fmin(a, __shfl_xor(a, off, 64));
            b = fmax(b, __shfl_xor(b, off, 64));
        }
        if (lane == 0) {
            lo[wave][c] = ordered_bits(a);
            hi[wave][c] = ordered_bits(b);
        }
    }
    nonfinite = __any(nonfinite) ? 1 : 0;
    if (lane == 0) bad[wave] = nonfinite;
    __syncthreads();
    if (threadIdx.x < d) {
        const int c = threadIdx.x;
        unsigned long long a = lo[0][c], b = hi[0][c];
        for (int w = 1; w < 4; ++w) {
            a = lo[w][c] < a ? lo[w][c] : a;
            b = hi[w][c] > b ? hi[w][c] : b;
        }
        atomicMin(ext + 2 * c, a);
        atomicMax(ext + 2 * c + 1, b);
    }
    if (threadIdx.x == 0 && (bad[0] | bad[1] | bad[2] | bad[3])) atomicOr(ext + 2 * MAXP, 1ull);
}

template <typename T>
hipError_t launch_extent(const cde_model* m, unsigned long long* ext, hipStream_t stream)
{
    hipLaunchKernelGGL(k_extent_init, dim3(1), dim3(64), 0, stream, ext);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const unsigned blocks = (unsigned)((m->n + 255) / 256);
    hipLaunchKernelGGL((k_extent<T>), dim3(blocks), dim3(256), 0, stream, (const T*)m->pts, m->n,
                       m->dx + m->dy, m->stride, ext);
    return hipGetLastError();
}

template hipError_t launch_extent<float>(const cde_model*, unsigned long long*, hipStream_t);
template hipError_t launch_extent<double>(const cde_model*, unsigned long long*, hipStream_t);

// One 256-thread block per setting; thread t sums blocks t, t+256, ... in
// order, then a fixed butterfly and wave order combine the 256 partial sums.
template <int NVMAX>
__global__ __launch_bounds__(256) void k_reduce_parts(const double* __restrict__ part, int nblocks,
                                                      int nv, double* __restrict__ totals,
                                                      double* __restrict__ grad,
                                                      double* __restrict__ counts)
{
    __shared__ double red[4 * NVMAX];
    const int s = blockIdx.x;
    double v[NVMAX];
#pragma unroll
    for (int q = 0; q < NVMAX; ++q) v[q] = 0.0;
    const double* base = part + (size_t)s * nblocks * nv;
    for (int b = threadIdx.x; b < nblocks; b += 256) {
#pragma unroll
        for (int q = 0; q < NVMAX; ++q)
            if (q < nv) v[q] += base[(size_t)b * nv + q];
    }
    block_sum<NVMAX>(v, red);
    if (threadIdx.x == 0) {
        totals[s] = v[0];
        if (grad)
            for (int q = 1; q < nv - 1; ++q) grad[(size_t)s * (nv - 2) + (q - 1)] = v[q];
        if (counts) counts[s] = v[nv - 1];
    }
}

// Sum of the per-setting non-finite counts, in setting order (one thread).
__global__ void k_sum_counts(const double* __restrict__ counts, int nsets, int64_t* __restrict__ out)
{
    double s = 0.0;
    for (int q = 0; q < nsets; ++q) s += counts[q];
    *out = (int64_t)s;
}

hipError_t launch_reduce_parts(const double* part, int nsets, int nblocks, int nv, double* totals,
                               double* grad, double* counts, int64_t* nonfinite, hipStream_t stream)
{
    double* c = nonfinite ? counts : nullptr;
    if (nv <= 2)
        hipLaunchKernelGGL((k_reduce_parts<2>), dim3(nsets), dim3(256), 0, stream, part, nblocks, nv,
                           totals, grad, c);
    else if (nv <= MAXP + 2)
        hipLaunchKernelGGL((k_reduce_parts<MAXP + 2>), dim3(nsets), dim3(256), 0, stream, part,
                           nblocks, nv, totals, grad, c);
    else
        return hipErrorInvalidValue;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !nonfinite) return e;
    hipLaunchKernelGGL(k_sum_counts, dim3(1), dim3(1), 0, stream, (const double*)counts, nsets, nonfinite);
    return hipGetLastError();
}

hipError_t launch_sum_counts(const double* counts, int nsets, int64_t* out, hipStream_t stream)
{
    hipLaunchKernelGGL(k_sum_counts, dim3(1), dim3(1), 0, stream, counts, nsets, out);
    return hipGetLastError();
}

}  // namespace cde
