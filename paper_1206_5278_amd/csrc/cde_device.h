// cde_device.h -- small device helpers shared by the gfx950 kernels.
#pragma once

#include "cde_common.h"

namespace cde {

template <typename T>
__device__ __forceinline__ T exp2_(T x);

// v_exp_f32: base-2 exponential on the transcendental unit (about 1 ulp).
template <>
__device__ __forceinline__ float exp2_<float>(float x) { return __builtin_amdgcn_exp2f(x); }

template <>
__device__ __forceinline__ double exp2_<double>(double x) { return exp2(x); }

__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float min_(float a, float b) { return __builtin_fminf(a, b); }
__device__ __forceinline__ double min_(double a, double b) { return __builtin_fmin(a, b); }
__device__ __forceinline__ float max_(float a, float b) { return __builtin_fmaxf(a, b); }
__device__ __forceinline__ double max_(double a, double b) { return __builtin_fmax(a, b); }

template <typename T>
__device__ __forceinline__ T inf_();
template <>
__device__ __forceinline__ float inf_<float>() { return __builtin_inff(); }
template <>
__device__ __forceinline__ double inf_<double>() { return __builtin_inf(); }

// Compensated (Kahan) accumulator: `s - c` carries the running sum with the
// rounding error of each addition fed back into the next one.
template <typename T>
struct Kahan {
    T s, c;
    __device__ __forceinline__ void zero() { s = T(0); c = T(0); }
    __device__ __forceinline__ void add(T x)
    {
        T y = x - c;
        T t = s + y;
        c = (t - s) - y;
        s = t;
    }
    __device__ __forceinline__ void scale(T f) { s *= f; c *= f; }
    __device__ __forceinline__ double value() const { return (double)s - (double)c; }
};

// Load one point row of S values (S a multiple of 4) with 16-byte loads.
template <int S>
__device__ __forceinline__ void load_row(float (&dst)[S], const float* src)
{
    static_assert(S % 4 == 0, "row stride must be a multiple of 4");
#pragma unroll
    for (int q = 0; q < S; q += 4) {
        float4 v = *reinterpret_cast<const float4*>(src + q);
        dst[q] = v.x; dst[q + 1] = v.y; dst[q + 2] = v.z; dst[q + 3] = v.w;
    }
}

template <int S>
__device__ __forceinline__ void load_row(double (&dst)[S], const double* src)
{
    static_assert(S % 2 == 0, "row stride must be even");
#pragma unroll
    for (int q = 0; q < S; q += 2) {
        double2 v = *reinterpret_cast<const double2*>(src + q);
        dst[q] = v.x; dst[q + 1] = v.y;
    }
}

// Load the first P values of a point row (P <= S; the rest of the row is
// padding) with the widest aligned loads.
template <int P, int S>
__device__ __forceinline__ void load_cols(float (&dst)[S], const float* src)
{
    static_assert(P <= S && S % 4 == 0, "bad row shape");
    constexpr int Q4 = P / 4 * 4;
#pragma unroll
    for (int q = 0; q < Q4; q += 4) {
        float4 v = *reinterpret_cast<const float4*>(src + q);
        dst[q] = v.x; dst[q + 1] = v.y; dst[q + 2] = v.z; dst[q + 3] = v.w;
    }
    if constexpr (P - Q4 >= 2) {
        float2 v = *reinterpret_cast<const float2*>(src + Q4);
        dst[Q4] = v.x; dst[Q4 + 1] = v.y;
    }
    if constexpr ((P - Q4) % 2 == 1) dst[P - 1] = src[P - 1];
}

template <int P, int S>
__device__ __forceinline__ void load_cols(double (&dst)[S], const double* src)
{
    static_assert(P <= S && S % 2 == 0, "bad row shape");
    constexpr int Q2 = P / 2 * 2;
#pragma unroll
    for (int q = 0; q < Q2; q += 2) {
        double2 v = *reinterpret_cast<const double2*>(src + q);
        dst[q] = v.x; dst[q + 1] = v.y;
    }
    if constexpr (P % 2 == 1) dst[P - 1] = src[P - 1];
}

// A wave-uniform value kept in a vector register, so that the FP32 ops using
// it have vector operands only (those issue at the higher rate on gfx950).
__device__ __forceinline__ float vreg(float x)
{
    float r;
    asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}
__device__ __forceinline__ double vreg(double x) { return x; }

template <int S, typename T>
__device__ __forceinline__ void store_row(T* dst, const T (&src)[S])
{
#pragma unroll
    for (int q = 0; q < S; ++q) dst[q] = src[q];
}

// Deterministic block sum of NV doubles per thread over a 256-thread block:
// fixed butterfly inside each 64-lane wave, then waves 0..3 in order.
// The result is valid in thread 0 only.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* red /* [4][NV] LDS */)
{
#pragma unroll
    for (int q = 0; q < NV; ++q) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v[q] += __shfl_xor(v[q], off, 64);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) red[wave * NV + q] = v[q];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) v[q] = ((red[q] + red[NV + q]) + red[2 * NV + q]) + red[3 * NV + q];
    }
}

// Exact FP64 minimum of a squared distance over a stream of points, with an
// FP32 screen: a point is a candidate (its FP64 distance is taken) when its
// FP32 distance is within a factor 1 + 2^-10 of the running FP32 minimum, or
// at most 2^-100.  An FP32 distance formed from the same FP32 inputs
// (differences, squares and weights rounded to FP32) lies within a relative
// 2^-18 of the FP64 value for up to 18 dimensions, so the FP64 minimiser j*
// satisfies d32(j*) <= (1 + 2^-18) / (1 - 2^-18) min_j d32(j), below the
// factor times any running minimum: it is always a candidate, and the
// minimum over the candidates equals the plain FP64 minimum.  A point that
// is not a candidate lies above the running minimum and would not lower it,
// so the minimum and the threshold change only on candidates and the common
// case costs one compare.
struct ScreenedMin {
    float s = __builtin_inff();  // FP32 minimum so far
    float t = __builtin_inff();  // max(s (1 + 2^-10), 2^-100)
    // the screen alone, without updating the minimum: the smallest of a
    // group of distances passes exactly when one of them is a candidate
    __device__ __forceinline__ bool passes(float d32) const { return d32 <= t; }
    __device__ __forceinline__ bool candidate(float d32)
    {
        if (!(d32 <= t)) return false;
        s = __builtin_fminf(s, d32);
        t = __builtin_fmaxf(s * (1.0f + 0x1p-10f), 0x1p-100f);
        return true;
    }
};

}  // namespace cde
