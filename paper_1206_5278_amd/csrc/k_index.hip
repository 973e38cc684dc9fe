// k_index.hip -- a spatial order of a model's points, for compact-support
// kernels (the Epanechnikov kernel of the paper's experiments, Section 4).
//
// A kernel that is exactly zero outside its window lets a (point block, j
// tile) pair be skipped when the two tiles' bounding boxes lie a window
// apart: every pair term there is exactly zero.  That only pays when tiles
// are spatially compact, so the points are put in the leaf order of a
// kd-tree over x: each node splits at a 32-row-aligned median of its widest
// dimension, down to 32-point leaves (so 256-point tiles are whole subtrees
// of 8 leaves).  The tree is built level by level on the device: per node
// the widest dimension, then one stable radix sort of (node, coordinate
// along that dimension) keys over all points.  Then the sorted rows in FP64
// and the x boxes of every 256-row tile and 32-row subtile.
#include <algorithm>
#include <vector>

#include "cde_device.h"
#include "cde_kernels.h"

namespace cde {

namespace {

// Widest x dimension of each node (positions start..start+size of the
// current order) and its extent along it; one block per node.
template <typename T>
__global__ __launch_bounds__(TILE) void k_node_split(const T* __restrict__ pts, int stride, int dx,
                                                     const int* __restrict__ perm,
                                                     const int2* __restrict__ nodes, int* __restrict__ dim,
                                                     double* __restrict__ lo, double* __restrict__ hi)
{
    __shared__ double sa[TILE], sb[TILE];
    const int node = blockIdx.x, tid = threadIdx.x;
    const int2 r = nodes[node];
    int best = 0;
    double bw = -1.0, blo = 0.0, bhi = 0.0;
    for (int k = 0; k < dx; ++k) {
        double a = __builtin_inf(), c = -__builtin_inf();
        for (int s = r.x + tid; s < r.x + r.y; s += TILE) {
            const double v = (double)pts[(size_t)perm[s] * stride + k];
            a = fmin(a, v);
            c = fmax(c, v);
        }
        sa[tid] = a;
        sb[tid] = c;
        __syncthreads();
        for (int off = TILE / 2; off > 0; off >>= 1) {
            if (tid < off) {
                sa[tid] = fmin(sa[tid], sa[tid + off]);
                sb[tid] = fmax(sb[tid], sb[tid + off]);
            }
            __syncthreads();
        }
        const double w = sb[0] - sa[0];
        if (w > bw) {
            bw = w;
            best = k;
            blo = sa[0];
            bhi = sb[0];
        }
        __syncthreads();
    }
    if (tid == 0) {
        dim[node] = best;
        lo[node] = blo;
        hi[node] = bhi;
    }
}

// Sort keys of one level: node id in the high 32 bits, the position along
// the node's widest dimension (quantised to 32 bits) in the low bits; rows
// beyond n keep the largest key.  One block per node.
template <typename T>
__global__ __launch_bounds__(TILE) void k_node_keys(const T* __restrict__ pts, int stride,
                                                    const int* __restrict__ perm,
                                                    const int2* __restrict__ nodes,
                                                    const int* __restrict__ dim,
                                                    const double* __restrict__ lo,
                                                    const double* __restrict__ hi,
                                                    unsigned long long* __restrict__ key)
{
    const int node = blockIdx.x;
    const int2 r = nodes[node];
    const int k = dim[node];
    const double l = lo[node], span = hi[node] - lo[node];
    const double top = 4294967295.0;
    for (int s = r.x + threadIdx.x; s < r.x + r.y; s += TILE) {
        const double v = (double)pts[(size_t)perm[s] * stride + k];
        double t = span > 0.0 ? (v - l) / span * top : 0.0;
        t = fmin(fmax(t, 0.0), top);
        key[s] = ((unsigned long long)node << 32) | (unsigned long long)(unsigned int)t;
    }
}

__global__ void k_init_order(int npad, int n, int* __restrict__ perm, unsigned long long* __restrict__ key)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= npad) return;
    perm[s] = s;
    key[s] = s < n ? 0ull : ~0ull;
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

// Node ranges of every level of the kd-tree over n points (leaves of at most
// LEAF points, splits at LEAF-aligned medians): levels[l] lists (start,
// size) of all nodes of level l in position order.
static std::vector<std::vector<int2>> kd_levels(int n)
{
    constexpr int LEAF = SUBROWS;
    std::vector<std::vector<int2>> levels;
    std::vector<int2> cur{make_int2(0, n)};
    for (;;) {
        bool split = false;
        std::vector<int2> next;
        for (const int2& r : cur) {
            if (r.y > LEAF) {
                const int m = (r.y / 2 + LEAF - 1) / LEAF * LEAF;
                next.push_back(make_int2(r.x, m));
                next.push_back(make_int2(r.x + m, r.y - m));
                split = true;
            } else {
                next.push_back(r);
            }
        }
        if (!split) break;
        levels.push_back(cur);
        cur.swap(next);
    }
    return levels;
}

template <typename T>
static hipError_t build_index_t(cde_model* m, void* work, size_t work_bytes, hipStream_t stream)
{
    const int n = (int)m->n, npad = (int)m->npad, dx = m->dx, stride = m->stride;
    // all levels' node tables, concatenated, uploaded once
    const std::vector<std::vector<int2>> levels = kd_levels(n);
    std::vector<int2> table;
    std::vector<size_t> first;
    size_t max_nodes = 1;
    for (const auto& l : levels) {
        first.push_back(table.size());
        table.insert(table.end(), l.begin(), l.end());
        max_nodes = std::max(max_nodes, l.size());
    }
    char* w = (char*)work;
    unsigned long long* k0 = (unsigned long long*)w;
    unsigned long long* k1 = k0 + npad;
    int* v0 = (int*)(k1 + npad);
    int* v1 = v0 + npad;
    double* lo = (double*)(((size_t)(v1 + npad) + 7) & ~size_t(7));
    double* hi = lo + max_nodes;
    int* dim = (int*)(hi + max_nodes);
    int2* nodes = (int2*)(((size_t)(dim + max_nodes) + 7) & ~size_t(7));
    const size_t used = ((size_t)((char*)(nodes + table.size()) - w) + 255) & ~size_t(255);
    void* tmp = (void*)(w + used);
    if (used + radix_sort_work_bytes(npad) > work_bytes) return hipErrorInvalidValue;
    hipError_t e;
    const T* pts = (const T*)m->pts;
    if (!table.empty()) {
        e = hipMemcpyAsync(nodes, table.data(), sizeof(int2) * table.size(), hipMemcpyHostToDevice, stream);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_init_order, dim3((npad + 255) / 256), dim3(256), 0, stream, npad, n, v0, k0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    for (size_t l = 0; l < levels.size(); ++l) {
        const int nn = (int)levels[l].size();
        const int2* lv = nodes + first[l];
        hipLaunchKernelGGL((k_node_split<T>), dim3(nn), dim3(TILE), 0, stream, pts, stride, dx,
                           (const int*)v0, lv, dim, lo, hi);
        hipLaunchKernelGGL((k_node_keys<T>), dim3(nn), dim3(TILE), 0, stream, pts, stride, (const int*)v0,
                           lv, (const int*)dim, (const double*)lo, (const double*)hi, k0);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        // keys: node id (below 2^nb) above 32 position bits; rows past n
        // hold all-ones keys and stay last
        int nb = 1;
        while ((int64_t(1) << nb) < nn) ++nb;
        bool alt = false;
        e = radix_sort_pairs(k0, v0, k1, v1, npad, 0, std::min(64, 32 + nb), tmp, &alt, stream);
        if (e != hipSuccess) return e;
        if (alt) {
            std::swap(k0, k1);
            std::swap(v0, v1);
        }
    }
    e = hipMemcpyAsync(m->perm, v0, sizeof(int) * (size_t)npad, hipMemcpyDeviceToDevice, stream);
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
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // the node table is read from host memory by the stream: wait before it goes
    return hipStreamSynchronize(stream);
}

}  // namespace

size_t index_work_bytes(const cde_model* m)
{
    const size_t tmp_bytes = radix_sort_work_bytes(m->npad);
    // node tables: at most npad/SUBROWS leaves, so at most 2 npad/SUBROWS
    // nodes over all levels and npad/SUBROWS on one level
    const size_t leaves = (size_t)m->npad / SUBROWS + 1;
    return (size_t)m->npad * (2 * sizeof(unsigned long long) + 2 * sizeof(int)) + 16 +
           leaves * (2 * sizeof(double) + sizeof(int)) + 16 + 2 * leaves * sizeof(int2) + 256 +
           tmp_bytes + 256;
}

hipError_t launch_build_index(cde_model* m, void* work, size_t work_bytes, hipStream_t stream)
{
    return m->prec == CDE_F64 ? build_index_t<double>(m, work, work_bytes, stream)
                              : build_index_t<float>(m, work, work_bytes, stream);
}

}  // namespace cde
