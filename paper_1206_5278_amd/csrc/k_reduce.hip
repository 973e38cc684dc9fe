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
