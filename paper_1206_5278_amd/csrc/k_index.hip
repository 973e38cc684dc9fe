// k_index.hip -- a spatial order of a model's points, for compact-support
// kernels (the Epanechnikov kernel of the paper's experiments, Section 5).
//
// A kernel that is exactly zero outside its window lets a whole (point
// block, j tile) pair be skipped when the two tiles' bounding boxes lie a
// window apart: every pair term there is exactly zero.  That only pays when
// tiles are spatially compact, so points are put in Morton (bit-interleaved
// Z-curve) order of their quantised x coordinates.  Built once per model on
// first use: per-dimension x range, Morton codes, a radix sort of (code,
// index) pairs, the sorted rows in FP64, and per-tile x boxes.
#include <hipcub/hipcub.hpp>

#include "cde_device.h"
#include "cde_kernels.h"

namespace cde {

namespace {

// Per-dimension min and max of x over the n points (block k: dimension k).
template <typename T>
__global__ __launch_bounds__(TILE) void k_xrange(const T* __restrict__ pts, int n, int stride,
                                                 double* __restrict__ lo, double* __restrict__ hi)
{
    __shared__ double sa[TILE], sb[TILE];
    const int k = blockIdx.x, tid = threadIdx.x;
    double a = __builtin_inf(), b = -__builtin_inf();
    for (int i = tid; i < n; i += TILE) {
        const double v = (double)pts[(size_t)i * stride + k];
        a = fmin(a, v);
        b = fmax(b, v);
    }
    sa[tid] = a;
    sb[tid] = b;
    __syncthreads();
    for (int off = TILE / 2; off > 0; off >>= 1) {
        if (tid < off) {
            sa[tid] = fmin(sa[tid], sa[tid + off]);
            sb[tid] = fmax(sb[tid], sb[tid + off]);
        }
        __syncthreads();
    }
    if (tid == 0) {
        lo[k] = sa[0];
        hi[k] = sb[0];
    }
}

// Morton code of each point's x quantised to `bits` bits per dimension
// (bits * dx <= 63); padding rows get the largest code and sort last.
template <typename T>
__global__ void k_morton(const T* __restrict__ pts, int n, int npad, int dx, int stride, int bits,
                         const double* __restrict__ lo, const double* __restrict__ hi,
                         unsigned long long* __restrict__ code, int* __restrict__ idx)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npad) return;
    unsigned long long c = ~0ull;
    if (i < n) {
        const double top = (double)((1ull << bits) - 1);
        unsigned int q[16];
        for (int k = 0; k < dx; ++k) {
            const double span = hi[k] - lo[k];
            double t = span > 0.0 ? ((double)pts[(size_t)i * stride + k] - lo[k]) / span * top : 0.0;
            t = fmin(fmax(t, 0.0), top);
            q[k] = (unsigned int)t;
        }
        c = 0ull;
        for (int b = bits - 1; b >= 0; --b)
            for (int k = 0; k < dx; ++k) c = (c << 1) | ((q[k] >> b) & 1u);
    }
    code[i] = c;
    idx[i] = i;
}

// Sorted rows in FP64 (exact for FP32 data): spts[s] = pts[perm[s]].
template <typename T>
__global__ void k_gather_sorted(const T* __restrict__ pts, const int* __restrict__ perm, int npad,
                                int stride, double* __restrict__ spts)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= npad) return;
    const int src = perm[s];
    for (int c = 0; c < stride; ++c) spts[(size_t)s * stride + c] = (double)pts[(size_t)src * stride + c];
}

// x box of each 256-row tile of the sorted rows (rows < n only):
// box[(t * 2 + 0) * dx + k] = min, box[(t * 2 + 1) * dx + k] = max.
__global__ __launch_bounds__(TILE) void k_tile_boxes(const double* __restrict__ spts, int n, int dx,
                                                     int stride, double* __restrict__ box)
{
    __shared__ double sa[TILE], sb[TILE];
    const int t = blockIdx.x, tid = threadIdx.x;
    const int s = t * TILE + tid;
    for (int k = 0; k < dx; ++k) {
        const double v = s < n ? spts[(size_t)s * stride + k] : 0.0;
        sa[tid] = s < n ? v : __builtin_inf();
        sb[tid] = s < n ? v : -__builtin_inf();
        __syncthreads();
        for (int off = TILE / 2; off > 0; off >>= 1) {
            if (tid < off) {
                sa[tid] = fmin(sa[tid], sa[tid + off]);
                sb[tid] = fmax(sb[tid], sb[tid + off]);
            }
            __syncthreads();
        }
        if (tid == 0) {
            box[((size_t)t * 2 + 0) * dx + k] = sa[0];
            box[((size_t)t * 2 + 1) * dx + k] = sb[0];
        }
        __syncthreads();
    }
}

// x box of each 32-row subtile of the sorted rows (rows < n only), same
// layout as the tile boxes; one thread per subtile.
__global__ void k_sub_boxes(const double* __restrict__ spts, int n, int nsub, int dx, int stride,
                            double* __restrict__ box)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nsub) return;
    for (int k = 0; k < dx; ++k) {
        double a = __builtin_inf(), b = -__builtin_inf();
        for (int r = 0; r < SUBROWS; ++r) {
            const int s = g * SUBROWS + r;
            if (s < n) {
                const double v = spts[(size_t)s * stride + k];
                a = fmin(a, v);
                b = fmax(b, v);
            }
        }
        box[((size_t)g * 2 + 0) * dx + k] = a;
        box[((size_t)g * 2 + 1) * dx + k] = b;
    }
}

template <typename T>
static hipError_t build_index_t(cde_model* m, void* work, size_t work_bytes, hipStream_t stream)
{
    const int n = (int)m->n, npad = (int)m->npad, dx = m->dx, stride = m->stride;
    char* w = (char*)work;
    double* lo = (double*)w;
    double* hi = lo + 16;
    unsigned long long* k0 = (unsigned long long*)(w + 256);
    unsigned long long* k1 = k0 + npad;
    int* v0 = (int*)(k1 + npad);
    int* v1 = v0 + npad;
    const size_t used = ((size_t)((char*)(v1 + npad) - w) + 255) & ~size_t(255);  // 256-byte aligned
    void* tmp = (void*)(w + used);
    size_t tmp_bytes = 0;
    hipError_t e = hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, k0, k1, v0, v1, npad, 0, 64,
                                                      stream);
    if (e != hipSuccess) return e;
    if (used + tmp_bytes > work_bytes) return hipErrorInvalidValue;
    const T* pts = (const T*)m->pts;
    hipLaunchKernelGGL((k_xrange<T>), dim3(dx), dim3(TILE), 0, stream, pts, n, stride, lo, hi);
    const int bits = 63 / dx < 21 ? 63 / dx : 21;
    hipLaunchKernelGGL((k_morton<T>), dim3((npad + 255) / 256), dim3(256), 0, stream, pts, n, npad, dx,
                       stride, bits, (const double*)lo, (const double*)hi, k0, v0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    e = hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, k0, k1, v0, v1, npad, 0, 64, stream);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(m->perm, v1, sizeof(int) * (size_t)npad, hipMemcpyDeviceToDevice, stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_gather_sorted<T>), dim3((npad + 255) / 256), dim3(256), 0, stream, pts,
                       (const int*)m->perm, npad, stride, (double*)m->spts);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_tile_boxes, dim3(npad / TILE), dim3(TILE), 0, stream, (const double*)m->spts, n,
                       dx, stride, (double*)m->tbox);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int nsub = npad / SUBROWS;
    hipLaunchKernelGGL(k_sub_boxes, dim3((nsub + 255) / 256), dim3(256), 0, stream, (const double*)m->spts,
                       n, nsub, dx, stride, (double*)m->sbox);
    return hipGetLastError();
}

}  // namespace

size_t index_work_bytes(const cde_model* m)
{
    size_t tmp_bytes = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, (unsigned long long*)nullptr,
                                             (unsigned long long*)nullptr, (int*)nullptr, (int*)nullptr,
                                             (int)m->npad, 0, 64, (hipStream_t)0);
    return 256 + (size_t)m->npad * (2 * sizeof(unsigned long long) + 2 * sizeof(int)) + 256 +
           tmp_bytes + 256;
}

hipError_t launch_build_index(cde_model* m, void* work, size_t work_bytes, hipStream_t stream)
{
    return m->prec == CDE_F64 ? build_index_t<double>(m, work, work_bytes, stream)
                              : build_index_t<float>(m, work, work_bytes, stream);
}

}  // namespace cde
