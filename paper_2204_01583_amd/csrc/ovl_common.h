// Internal definitions shared by the HIP kernels and the host library.
// Not part of the public ABI (include/ovl.h is).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ovl {

// Complex numbers in device memory are the HIP vector types double2 / float2
// (x = real, y = imaginary), so one element is one 16- or 8-byte load.
template <typename R> struct cvec;
template <> struct cvec<double> { using type = double2; };
template <> struct cvec<float>  { using type = float2; };
template <typename R> using C2 = typename cvec<R>::type;

template <typename R> struct cx {
    R re, im;
};

template <typename R> __device__ __forceinline__ cx<R> mk(R a, R b) { return cx<R>{a, b}; }
template <typename R> __device__ __forceinline__ cx<R> ld(const C2<R>* p, int64_t i) {
    C2<R> v = p[i];
    return cx<R>{v.x, v.y};
}
template <typename R> __device__ __forceinline__ void stc(C2<R>* p, int64_t i, cx<R> v) {
    C2<R> w; w.x = v.re; w.y = v.im;
    p[i] = w;
}
template <typename R> __device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R> __device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R> __device__ __forceinline__ cx<R> operator-(cx<R> a) { return {-a.re, -a.im}; }
template <typename R> __device__ __forceinline__ cx<R> operator*(cx<R> a, cx<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R> __device__ __forceinline__ cx<R> operator*(R s, cx<R> a) { return {s * a.re, s * a.im}; }
// conj(a) * b
template <typename R> __device__ __forceinline__ cx<R> cmul_conj(cx<R> a, cx<R> b) {
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// i * a, -i * a
template <typename R> __device__ __forceinline__ cx<R> ti(cx<R> a) { return {-a.im, a.re}; }
template <typename R> __device__ __forceinline__ cx<R> tmi(cx<R> a) { return {a.im, -a.re}; }
// a += b * c
template <typename R> __device__ __forceinline__ void fma_(cx<R>& a, cx<R> b, cx<R> c) {
    a.re += b.re * c.re - b.im * c.im;
    a.im += b.re * c.im + b.im * c.re;
}
// a += conj(b) * c
template <typename R> __device__ __forceinline__ void fmac_(cx<R>& a, cx<R> b, cx<R> c) {
    a.re += b.re * c.re + b.im * c.im;
    a.im += b.re * c.im - b.im * c.re;
}

// Lattice geometry of one context.  Sites are numbered
// s = x + Lx*(y + Ly*(z + Lz*t)); internal fields are structure-of-arrays:
// spinor [rhs][12][V] (component 3*spin + colour), links [mu][9][V]
// (element 3*row + col), so consecutive lanes read consecutive sites.
struct Geom {
    int L[4];        // Lx, Ly, Lz, Lt
    int64_t stride[4];
    int64_t V;
};

constexpr int kBlock = 256;           // threads per block of the site kernels
constexpr int kMaxShifts = 1024;      // shifted systems per apply

// Per-source solver state in device memory (one struct per right-hand side).
struct SrcState {
    double rr;          // ||r_k||^2 of the seed residual
    double bb;          // ||b||^2
    double2 alpha;      // alpha_k
    double2 alpha_prev; // alpha_{k-1}
    double2 beta_prev;  // beta_{k-1}
    double maxres;      // max over active shifts of ||r_j|| / ||b|| (estimate)
    int iter;           // iterations done
    int nact;           // shifts still active
    int done;           // 1 when no shift is active or on error
    int status;         // OVL_OK / error code
    int nlist;          // entries in this iteration's sweep list
    int pad;
};

}  // namespace ovl
