// Device helpers shared by the kernel files of libbem_hip.so: wave primitives, the FP32
// complex type, FP32/BF16 conversions and the leaf range of a B-spline.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "bem_core.h"

namespace bem {

constexpr int kWave = 64;

__device__ inline int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Workgroups are dispatched to the 8 XCDs round-robin (block b to XCD b % 8), and each XCD
// has its own L2.  Renumbering so that XCD x runs a contiguous range of logical blocks
// lets neighbouring blocks (which read overlapping data) share an L2.  A bijection of
// [0, n).
constexpr int kXcds = 8;
__device__ inline int64_t xcd_block(int64_t b, int64_t n) {
    const int64_t x = b % kXcds, i = b / kXcds, q = n / kXcds, r = n % kXcds;
    return x * q + (x < r ? x : r) + i;
}

// orders the wave's LDS accesses before and after this point
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// leaves (per direction) whose interval meets the support of B-spline j: [lo, hi]
__host__ __device__ inline void leaf_range(int j, int stride, int nloc, int nleaf1, int& lo, int& hi) {
    hi = j / stride;
    if (hi > nleaf1 - 1) hi = nleaf1 - 1;
    const int l = j - nloc + 1;
    lo = l <= 0 ? 0 : (l + stride - 1) / stride;
}

// ------------------------------------------------------------------ FP32 arithmetic
struct cflt {
    float re, im;
};
__device__ inline cflt operator+(cflt a, cflt b) { return {a.re + b.re, a.im + b.im}; }
__device__ inline cflt operator*(cflt a, cflt b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline cflt& operator+=(cflt& a, cflt b) {
    a.re += b.re;
    a.im += b.im;
    return a;
}
template <class F>
__device__ inline F zero_f();
template <>
__device__ inline float zero_f<float>() { return 0.0f; }
template <>
__device__ inline cflt zero_f<cflt>() { return {0.0f, 0.0f}; }
template <>
__device__ inline double zero_f<double>() { return 0.0; }
template <>
__device__ inline cdbl zero_f<cdbl>() { return {0.0, 0.0}; }
__device__ inline float to_f(double v) { return (float)v; }
__device__ inline cflt to_f(cdbl v) { return {(float)v.re, (float)v.im}; }
__device__ inline double to_d(float v) { return (double)v; }
__device__ inline cdbl to_d(cflt v) { return {(double)v.re, (double)v.im}; }
__device__ inline double to_d(double v) { return v; }
__device__ inline cdbl to_d(cdbl v) { return v; }

// BF16 by round-to-nearest-even of the FP32 value (finite inputs)
__device__ inline uint16_t f2bf(float f) {
    const uint32_t u = __float_as_uint(f);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ inline float bf2f(uint32_t b) { return __uint_as_float(b << 16); }

}  // namespace bem
