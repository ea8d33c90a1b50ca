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

// Element accesses to device buffers.  Every vector, link and state buffer
// the kernels read through ld / stc is global memory, and the accesses go
// through address-space-1 pointers: the compiler then emits global (not
// flat) loads and stores, also where the base pointer was read from memory
// (a job table) and not passed as a kernel argument.  A flat load may be
// served by LDS, so the compiler can only wait for all of them at once
// (vmcnt and lgkmcnt both zero); global loads complete in order and are
// waited for one by one, which keeps a hop's loads in flight together.
// LDS tiles are read directly, never through these helpers.
#define OVL_GLOBAL __attribute__((address_space(1)))
template <typename R> struct nvec;   // native two-element vector, no constructors
template <> struct nvec<double> { typedef double __attribute__((ext_vector_type(2))) type; };
template <> struct nvec<float>  { typedef float  __attribute__((ext_vector_type(2))) type; };
template <typename R> __device__ __forceinline__ cx<R> ld(const C2<R>* p, int64_t i) {
    typedef const OVL_GLOBAL typename nvec<R>::type G;
    const typename nvec<R>::type v = ((G*)p)[i];
    return cx<R>{v.x, v.y};
}
// 32-bit element index from a wave-uniform base: the byte offset is formed
// in 32 bits, so the load can use a scalar base plus one VGPR offset.
template <typename R> __device__ __forceinline__ cx<R> ld(const C2<R>* p, uint32_t i) {
    typedef const OVL_GLOBAL typename nvec<R>::type G;
    const OVL_GLOBAL char* b = (const OVL_GLOBAL char*)p;
    const typename nvec<R>::type v = *(G*)(b + i * (uint32_t)sizeof(C2<R>));
    return cx<R>{v.x, v.y};
}
template <typename R> __device__ __forceinline__ void stc(C2<R>* p, uint32_t i, cx<R> v) {
    typedef OVL_GLOBAL typename nvec<R>::type G;
    OVL_GLOBAL char* b = (OVL_GLOBAL char*)p;
    typename nvec<R>::type w;
    w.x = v.re;
    w.y = v.im;
    *(G*)(b + i * (uint32_t)sizeof(C2<R>)) = w;
}
__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
template <typename R> __device__ __forceinline__ void stc(C2<R>* p, int64_t i, cx<R> v) {
    typedef OVL_GLOBAL typename nvec<R>::type G;
    typename nvec<R>::type w;
    w.x = v.re;
    w.y = v.im;
    ((G*)p)[i] = w;
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
// s = x + Lx*(y + Ly*(z + Lz*t)).  Internal fields are tiled over 64-site
// tiles (see tix): a spinor is [rhs][Vt/64][12][64] (component 3*spin +
// colour), the links of one direction [Vt/64][NE][64] (element 3*row + col),
// so the 64 lanes of a wave read one contiguous 512 B (FP32) or 1 KiB (FP64)
// segment per component, and the 12 components of a tile lie in one
// contiguous block.  Vt = V rounded up to whole tiles; the sites from V to
// Vt of the last tile are zeros, kept at zero by every kernel.
struct Geom {
    int L[4];        // Lx, Ly, Lz, Lt
    int64_t stride[4];
    int64_t V;       // sites
    int64_t Vt;      // V rounded up to a multiple of kTile
    int bc[4];       // boundary sign per direction (+1 periodic, -1 antiperiodic)
};

constexpr int kTile = 64;  // sites per tile of the internal layouts

// Offset of component c of site s in one tiled array of nc components per site.
__host__ __device__ __forceinline__ uint32_t tix(uint32_t c, uint32_t s, uint32_t nc) {
    return ((s / (uint32_t)kTile) * nc + c) * (uint32_t)kTile + s % (uint32_t)kTile;
}
__host__ __device__ __forceinline__ int64_t tix64(int64_t c, int64_t s, int64_t nc) {
    return ((s / kTile) * nc + c) * kTile + s % kTile;
}

constexpr int kBlock = 256;           // threads per block of the site kernels
constexpr int kMaxShifts = 2048;      // shifted systems per apply
constexpr int kMaxSweepShifts = 1024; // ... for the sweep forms (LDS list of the active shifts)

constexpr int kMaxSlices = kMaxShifts / 256;  // 256-shift slices

// Per-source scalar state of the seed recurrence, in device memory.  Values
// produced in iteration k are stored at parity k&1 (see kernels.hip).
struct SrcState {
    double bb;          // ||b||^2
    double rr[2];       // ||r_k||^2 at [k&1]
    double2 alpha[2];   // alpha_k at [k&1]
    double2 beta[2];    // beta_k at [k&1]
    int iter;           // iterations done
    int status;         // OVL_OK / error code
    int pad[2];
};

// Device arrays of the shifted systems (all [..][nsrc][J] unless noted).
struct ShiftDev {
    double2* pi;        // [3][nsrc][J]: pi_k^j at [k%3]
    int* active;        // [2][nsrc][J]: shift active at the start of iteration k, at [k&1]
    double2* aj;        // alpha^j of the current iteration
    double* res;        // latest residual estimate ||r_j|| / ||b||
    int* cnt;           // [2][nsrc][kMaxSlices]: active shifts per slice at [k&1]
    double* mres;       // [nsrc][kMaxSlices]: max residual estimate per slice
    const double2* dz;  // [J] z_j - z_seed
    const double2* c;   // [J] quadrature weights
    int J, nsrc, nslices;
    double tol;
    // basis forms, may be null: [nsrc][maxk+1][J]
    double2 *h_a, *h_b, *h_pi;
    // seed scalars per iteration, may be null: [nsrc][maxk+1][3] =
    // (alpha_k, beta_k, (||r_k||^2, ||r_{k+1}||^2)), the Lanczos data of the
    // seed system
    double2* seed;
    int maxk;
};

// One job of a (possibly batched) shifted solve: one lattice with its links,
// nsrc right-hand sides and its own solver buffers.  The iteration kernels
// take a device array of these and find their job from the block index, so
// one launch advances every job of a batch by one stage.
constexpr int kMaxJobs = 64;
constexpr int kSlotChunk = 32;  // basis form: residual slots per allocation
// Grid blocks a job owns in a job-table stencil launch: its block count
// padded to a multiple of 8 (one per XCD), so every job starts on XCD 0.
inline __host__ __device__ int job_grid_blocks(int nb) { return (nb + 7) & ~7; }

struct JobDesc {
    Geom g;
    double kappa;
    double2 zs;                 // seed shift
    const void* U[2];           // links, [0] FP64 [1] FP32 (internal layout)
    int nsrc;
    int nsb;                    // site blocks of the stencil
    int sten_b0[2], sten_nb[2]; // this job's blocks in the FP64 / FP32 stencil grid: it owns
                                // [sten_b0, sten_b0 + job_grid_blocks(sten_nb)), sten_b0 a
                                // multiple of 8
    int vec_b0, nbe;            // this job's first block in the vector grid; blocks per source
    SrcState* st;
    ShiftDev sh;
    double4* part_w;            // [nsrc][nsb]: <r_k, q> (re, im), ||q||^2, ||r_k||^2 per block;
                                // fused iteration: two such arrays, kernel k writes [k&1]
    size_t part_stride;         // fused iteration: elements between the two partial arrays
    size_t qpp;                 // fused iteration: elements between q[k&1 = 0] and q[1]
    // working vectors [nsrc][12 Vt], index [0] FP64, [1] FP32
    void* q[2];
    void* r[2];                 // fused/reference: r in place; two-pass: r_k at r[..] + (k&1) * rpp
    size_t rpp;                 // two-pass: element offset of the second r buffer
    double2* b64;               // packed source
    double2* s64;               // quadrature sum
    void* pj[2];                // sweep forms: [nsrc][J][12 Vt]
    double2* xj;                // reference form
    char* const* slots;         // basis form: device table of slot-chunk bases
    size_t slot_bytes;          // bytes of one slot (nsrc * 12 Vt FP64 complex)
    const double2* h;           // two-pass, second pass: h[src][i] weights of r_i
    int ksw;                    // first FP32 iteration (slots from it hold FP32), or large
    int form;                   // OVL_FORM_* of this solve
    int phase;                  // precision of this job's iterations now: 0 FP64, 1 FP32 (the
                                // kernels of the other precision skip its blocks)
    // state export at the end of each chunk: the state block (SrcState array,
    // active counts, residual maxima; state_bytes, a multiple of 8) goes to
    // pinned host slot (k / chunk) & 1, state_stride bytes apart; none if
    // state_host is null
    const char* state_dev;
    char* state_host;           // device address of the pinned slots
    int state_bytes, state_stride;
};

// r_k and r_{k+1} of a job (element pointers of source 0; sources are 12 Vt apart)
template <typename T>
__device__ __forceinline__ T* job_rk(const JobDesc& J, int k, int fp32) {
    if (J.form == 2) {  // basis: slot k (FP32 slots packed at the slot base)
        return reinterpret_cast<T*>(J.slots[k / kSlotChunk] + (size_t)(k % kSlotChunk) * J.slot_bytes);
    }
    T* r = static_cast<T*>(J.r[fp32]);
    return J.form == 3 ? r + (size_t)(k & 1) * J.rpp : r;
}

}  // namespace ovl
