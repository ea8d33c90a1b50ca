// Device helpers shared by the kernel translation units of the library.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/ovl.h"
#include "ovl_common.h"

namespace ovl {

// ============================================================================
// reductions (fixed order: butterfly within a wave, serial over waves)
// ============================================================================
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) t += sh[i];
    __syncthreads();
    return t;
}

// Four block sums at once, each in the order of block_sum (so each result
// is bitwise that of block_sum), with one pair of barriers instead of four:
// the four butterflies are independent and overlap.  sh holds 4 NT/64 values.
template <int NT>
__device__ __forceinline__ void block_sum4(double (&v)[4], double* sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] += __shfl_xor(v[i], o, 64);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0)
#pragma unroll
        for (int i = 0; i < 4; ++i) sh[i * (NT / 64) + w] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < NT / 64; ++q) t += sh[i * (NT / 64) + q];
        v[i] = t;
    }
    __syncthreads();
}

// A block sum and a block maximum at once (each in the order of block_sum /
// block_max), with one pair of barriers.  sh holds 2 NT/64 values.
template <int NT>
__device__ __forceinline__ void block_sum_max(double& s, double& m, double* sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        s += __shfl_xor(s, o, 64);
        m = fmax(m, __shfl_xor(m, o, 64));
    }
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) {
        sh[w] = s;
        sh[NT / 64 + w] = m;
    }
    __syncthreads();
    double ts = 0.0, tm = 0.0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) {
        ts += sh[i];
        tm = fmax(tm, sh[NT / 64 + i]);
    }
    __syncthreads();
    s = ts;
    m = tm;
}

template <int NT>
__device__ __forceinline__ double block_max(double v, double* sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) t = fmax(t, sh[i]);
    __syncthreads();
    return t;
}

// ============================================================================
// complex helpers (FP64 scalars)
// ============================================================================
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
    // Smith's algorithm keeps the quotient finite for |b| far from 1
    if (fabs(b.x) >= fabs(b.y)) {
        const double r = b.y / b.x, d = b.x + b.y * r;
        return make_double2((a.x + a.y * r) / d, (a.y - a.x * r) / d);
    } else {
        const double r = b.x / b.y, d = b.x * r + b.y;
        return make_double2((a.x * r + a.y) / d, (a.y * r - a.x) / d);
    }
}
__device__ __forceinline__ double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }
__device__ __forceinline__ bool finite2(double2 a) { return isfinite(a.x) && isfinite(a.y); }

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2.
// Remap the linear block id so that XCD k works on one contiguous range of
// (rhs, site tile): the z and t neighbours of a tile then sit in the same L2.
__device__ __forceinline__ unsigned xcd_remap(unsigned b, unsigned nb) {
    const unsigned per = nb / 8u;
    return (b < per * 8u) ? (b % 8u) * per + b / 8u : b;
}

// A source is live at iteration k while it has no error, k is below the
// iteration limit and some shift is still active (per-slice counts written by
// the previous iteration).
__device__ __forceinline__ bool src_live(const SrcState& S, const ShiftDev& sh, int n, int k) {
    if (S.status != 0 || k >= sh.maxk) return false;
    const int* c = sh.cnt + ((size_t)(k & 1) * sh.nsrc + n) * kMaxSlices;
    int t = 0;
    for (int i = 0; i < sh.nslices; ++i) t += c[i];
    return t > 0;
}

}  // namespace ovl
