// k_sort.hip -- stable least-significant-digit radix sort of (64-bit key,
// 32-bit value) pairs, for the spatial orders that let compact-support
// kernels (the Epanechnikov kernel of the paper's experiments, Section 4)
// skip exactly-zero tile pairs: the kd-tree levels of a model's points and
// the Morton order of a query batch.
//
// One pass per 6-bit digit, three kernels per pass:
//   k_sort_hist    each block takes a tile of 2048 items, 8 consecutive items
//                  per thread, and counts each digit per thread in LDS; it
//                  writes the block's count of every digit to hist[digit][block];
//   k_sort_scan    one block: exclusive prefix over hist in digit-major order,
//                  so hist[d][b] becomes the output position of the first
//                  item of digit d in block b;
//   k_sort_scatter each block counts again, takes one exclusive prefix over
//                  its (digit, thread) counts in digit-major order (the rank
//                  of each thread's first item of each digit within the
//                  tile), and writes every item to hist[d][b] + its rank.
// Items keep their order within a digit (block, then thread, then item), so
// each pass is stable and the passes together sort by the chosen key bits.
#include "cde_device.h"
#include "cde_kernels.h"

namespace cde {

namespace {

constexpr int SORT_BITS = 6;
constexpr int SORT_BINS = 1 << SORT_BITS;  // 64 digits
constexpr int SORT_THREADS = 256;
constexpr int SORT_ITEMS = 8;                         // consecutive items per thread
constexpr int SORT_TILE = SORT_THREADS * SORT_ITEMS;  // 2048 items per block

__device__ __forceinline__ int digit_of(unsigned long long key, int shift)
{
    return (int)((key >> shift) & (SORT_BINS - 1));
}

// Per-thread digit counts of this block's tile into cnt[digit * 256 + tid]
// (digit-major); a tile holds at most 2048 items, so 16 bits suffice.
__device__ __forceinline__ void count_tile(const unsigned long long* __restrict__ keys, int64_t n,
                                           int shift, unsigned short* cnt)
{
    const int tid = threadIdx.x;
    for (int d = 0; d < SORT_BINS; ++d) cnt[d * SORT_THREADS + tid] = 0;
    __syncthreads();
    const int64_t first = (int64_t)blockIdx.x * SORT_TILE + (int64_t)tid * SORT_ITEMS;
#pragma unroll
    for (int j = 0; j < SORT_ITEMS; ++j) {
        const int64_t s = first + j;
        if (s < n) cnt[digit_of(keys[s], shift) * SORT_THREADS + tid] += 1;  // own column only
    }
    __syncthreads();
}

__global__ __launch_bounds__(SORT_THREADS) void k_sort_hist(const unsigned long long* __restrict__ keys,
                                                            int64_t n, int shift,
                                                            unsigned* __restrict__ hist)
{
    __shared__ unsigned short cnt[SORT_BINS * SORT_THREADS];
    count_tile(keys, n, shift, cnt);
    const int tid = threadIdx.x;
    if (tid < SORT_BINS) {
        unsigned s = 0;
        for (int t = 0; t < SORT_THREADS; ++t) s += cnt[tid * SORT_THREADS + t];
        hist[(size_t)tid * gridDim.x + blockIdx.x] = s;
    }
}

// Exclusive prefix sum of v[0..m) in place, one block of 1024 threads:
// each thread sums a contiguous segment, the segment sums are scanned in
// LDS, and each thread rewrites its segment.
__global__ __launch_bounds__(1024) void k_sort_scan(unsigned* __restrict__ v, int64_t m)
{
    __shared__ unsigned part[1024];
    const int tid = threadIdx.x;
    const int64_t seg = (m + 1023) / 1024;
    const int64_t b = (int64_t)tid * seg, e = b + seg < m ? b + seg : m;
    unsigned s = 0;
    for (int64_t k = b; k < e; ++k) s += v[k];
    part[tid] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {  // inclusive Hillis-Steele scan
        const unsigned add = tid >= off ? part[tid - off] : 0u;
        __syncthreads();
        part[tid] += add;
        __syncthreads();
    }
    unsigned run = tid > 0 ? part[tid - 1] : 0u;
    for (int64_t k = b; k < e; ++k) {
        const unsigned x = v[k];
        v[k] = run;
        run += x;
    }
}

__global__ __launch_bounds__(SORT_THREADS) void k_sort_scatter(const unsigned long long* __restrict__ kin,
                                                               const int* __restrict__ vin, int64_t n,
                                                               int shift, const unsigned* __restrict__ offs,
                                                               unsigned long long* __restrict__ kout,
                                                               int* __restrict__ vout)
{
    __shared__ unsigned short cnt[SORT_BINS * SORT_THREADS];
    __shared__ unsigned short start[SORT_BINS];
    __shared__ unsigned short tsum[SORT_THREADS];
    count_tile(kin, n, shift, cnt);
    const int tid = threadIdx.x;
    // exclusive prefix over all (digit, thread) counts, digit-major: thread
    // tid owns entries [64 tid, 64 tid + 64)
    constexpr int PER = SORT_BINS * SORT_THREADS / SORT_THREADS;
    unsigned short* mine = cnt + tid * PER;
    unsigned short s = 0;
    for (int k = 0; k < PER; ++k) s += mine[k];
    tsum[tid] = s;
    __syncthreads();
    if (tid == 0) {
        unsigned short run = 0;
        for (int t = 0; t < SORT_THREADS; ++t) {
            const unsigned short x = tsum[t];
            tsum[t] = run;
            run += x;
        }
    }
    __syncthreads();
    unsigned short run = tsum[tid];
    for (int k = 0; k < PER; ++k) {
        const unsigned short x = mine[k];
        mine[k] = run;
        run += x;
    }
    __syncthreads();
    if (tid < SORT_BINS) start[tid] = cnt[tid * SORT_THREADS];  // rank of the tile's first item of digit tid
    __syncthreads();
    const int64_t first = (int64_t)blockIdx.x * SORT_TILE + (int64_t)tid * SORT_ITEMS;
#pragma unroll
    for (int j = 0; j < SORT_ITEMS; ++j) {
        const int64_t src = first + j;
        if (src >= n) break;
        const unsigned long long key = kin[src];
        const int d = digit_of(key, shift);
        unsigned short& rank = cnt[d * SORT_THREADS + tid];  // own column only
        const int64_t dst = (int64_t)offs[(size_t)d * gridDim.x + blockIdx.x] + (rank - start[d]);
        rank += 1;
        kout[dst] = key;
        vout[dst] = vin[src];
    }
}

}  // namespace

size_t radix_sort_work_bytes(int64_t n)
{
    const int64_t blocks = (n + SORT_TILE - 1) / SORT_TILE;
    return sizeof(unsigned) * (size_t)SORT_BINS * (size_t)(blocks > 0 ? blocks : 1) + 256;
}

hipError_t radix_sort_pairs(unsigned long long* k0, int* v0, unsigned long long* k1, int* v1, int64_t n,
                            int bit0, int bit1, void* work, bool* result_in_alt, hipStream_t stream)
{
    *result_in_alt = false;
    if (n <= 1 || bit1 <= bit0) return hipSuccess;
    if (bit0 < 0 || bit1 > 64 || n >= (int64_t(1) << 31)) return hipErrorInvalidValue;
    const int64_t blocks = (n + SORT_TILE - 1) / SORT_TILE;
    if (blocks >= (int64_t(1) << 31) / SORT_BINS) return hipErrorInvalidValue;
    unsigned* hist = (unsigned*)work;
    for (int shift = bit0; shift < bit1; shift += SORT_BITS) {
        hipLaunchKernelGGL(k_sort_hist, dim3((unsigned)blocks), dim3(SORT_THREADS), 0, stream,
                           (const unsigned long long*)k0, n, shift, hist);
        hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(1024), 0, stream, hist, (int64_t)SORT_BINS * blocks);
        hipLaunchKernelGGL(k_sort_scatter, dim3((unsigned)blocks), dim3(SORT_THREADS), 0, stream,
                           (const unsigned long long*)k0, (const int*)v0, n, shift, (const unsigned*)hist, k1,
                           v1);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        unsigned long long* tk = k0;
        k0 = k1;
        k1 = tk;
        int* tv = v0;
        v0 = v1;
        v1 = tv;
        *result_in_alt = !*result_in_alt;
    }
    return hipSuccess;
}

}  // namespace cde
