// HIP kernels for gfx950: layout conversion, the seed iteration's vector
// kernels with their deterministic reductions and shifted-system scalars, the
// shift sweeps and the basis-form sum.  Everything here is bandwidth bound (no
// dense contraction), so the kernels stream the vectors (tiled, 12 Vt complex
// elements per source) with one lane per element or pair of elements.  The
// stencil is in stencil.hip.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "device_util.h"
#include "kernels.h"
#include "seed_iter.h"

namespace ovl {

// ============================================================================
// layout conversion
// ============================================================================
template <typename R>
__global__ __launch_bounds__(kBlock) void k_pack_spinor(const double2* __restrict__ ext,
                                                        C2<R>* __restrict__ in, int64_t V,
                                                        int64_t Vt) {
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int n = blockIdx.y;
    if (s >= V) return;
    const double2* src = ext + ((int64_t)n * V + s) * 12;
    C2<R>* dst = in + (int64_t)n * 12 * Vt;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        double2 v = src[c];
        C2<R> w;
        w.x = (R)v.x;
        w.y = (R)v.y;
        dst[tix64(c, s, 12)] = w;
    }
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_unpack_spinor(const C2<R>* __restrict__ in,
                                                          double2* __restrict__ ext, int64_t V,
                                                          int64_t Vt) {
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int n = blockIdx.y;
    if (s >= V) return;
    const C2<R>* src = in + (int64_t)n * 12 * Vt;
    double2* dst = ext + ((int64_t)n * V + s) * 12;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        const C2<R> v = src[tix64(c, s, 12)];
        dst[c] = make_double2((double)v.x, (double)v.y);
    }
}

__global__ __launch_bounds__(kBlock) void k_unpack_dov(const double2* __restrict__ sin,
                                                       const double2* __restrict__ bext,
                                                       double2* __restrict__ ext, double a,
                                                       double bm, int64_t V, int64_t Vt) {
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int n = blockIdx.y;
    if (s >= V) return;
    const double2* src = sin + (int64_t)n * 12 * Vt;
    const double2* b = bext + ((int64_t)n * V + s) * 12;
    double2* dst = ext + ((int64_t)n * V + s) * 12;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        const double g5 = (c < 6) ? bm : -bm;  // gamma5 = diag(1,1,-1,-1) on spin
        double2 sv = src[tix64(c, s, 12)], bv = b[c], o;
        o.x = a * bv.x + g5 * sv.x;
        o.y = a * bv.y + g5 * sv.y;
        dst[c] = o;
    }
}

// ext [4][V][9] -> per direction the tiled [Vt/64][9][64] FP64 and FP32, and
// rows 0 and 1 alone as [Vt/64][6][64]; the boundary sign multiplies the links of the last slice of each
// direction.  defect[mu][blk] = max over the block's input links of
// max(|U U^dag - 1|, |det U - 1|), or NaN if any input element of the block is
// NaN or infinite (NaN propagates through the max).
__global__ __launch_bounds__(kBlock) void k_pack_gauge(const double2* __restrict__ ext,
                                                       double2* __restrict__ U64,
                                                       float2* __restrict__ U32,
                                                       double2* __restrict__ U64c,
                                                       float2* __restrict__ U32c, Geom g,
                                                       double* __restrict__ defect) {
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int mu = blockIdx.y;
    double dev = 0.0;
    if (s < g.V) {
        const int coord = (int)((s / g.stride[mu]) % g.L[mu]);
        const double sign = (coord == g.L[mu] - 1) ? (double)g.bc[mu] : 1.0;
        const double2* src = ext + ((int64_t)mu * g.V + s) * 9;
        double2 u[9];
        bool fin = true;
#pragma unroll
        for (int e = 0; e < 9; ++e) {
            u[e] = src[e];
            fin = fin && isfinite(u[e].x) && isfinite(u[e].y);
        }
#pragma unroll
        for (int e = 0; e < 9; ++e) {
            const double2 v = make_double2(u[e].x * sign, u[e].y * sign);
            U64[(int64_t)mu * 9 * g.Vt + tix64(e, s, 9)] = v;
            U32[(int64_t)mu * 9 * g.Vt + tix64(e, s, 9)] = make_float2((float)v.x, (float)v.y);
            if (e < 6) {
                U64c[(int64_t)mu * 6 * g.Vt + tix64(e, s, 6)] = v;
                U32c[(int64_t)mu * 6 * g.Vt + tix64(e, s, 6)] = make_float2((float)v.x, (float)v.y);
            }
        }
        // unitarity: (U U^dag)_ab = sum_c u_ac conj(u_bc)
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                double re = a == b ? -1.0 : 0.0, im = 0.0;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const double2 x = u[3 * a + c], y = u[3 * b + c];
                    re += x.x * y.x + x.y * y.y;
                    im += x.y * y.x - x.x * y.y;
                }
                dev = fmax(dev, sqrt(re * re + im * im));
            }
        const double2 m0 = csub(cmul(u[4], u[8]), cmul(u[5], u[7]));
        const double2 m1 = csub(cmul(u[3], u[8]), cmul(u[5], u[6]));
        const double2 m2 = csub(cmul(u[3], u[7]), cmul(u[4], u[6]));
        const double2 det = cadd(csub(cmul(u[0], m0), cmul(u[1], m1)), cmul(u[2], m2));
        const double dd = sqrt((det.x - 1.0) * (det.x - 1.0) + det.y * det.y);
        dev = (dev != dev || dd != dd) ? dd + dev : fmax(dev, dd);
        // a non-finite entry marks the block whatever the products gave
        // (Inf - Inf is NaN, but Inf alone would only read as "not SU(3)")
        if (!fin) dev = __builtin_nan("");
    }
    __shared__ double sh[kBlock / 64];
    // max over the block; a NaN anywhere makes the result NaN
    double v = dev;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double w = __shfl_xor(v, o, 64);
        v = (v != v || w != w) ? v + w : fmax(v, w);
    }
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = sh[0];
#pragma unroll
        for (int i = 1; i < kBlock / 64; ++i) t = (t != t || sh[i] != sh[i]) ? t + sh[i] : fmax(t, sh[i]);
        defect[(size_t)mu * gridDim.x + blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(kBlock) void k_convert(const double2* __restrict__ a,
                                                    float2* __restrict__ b, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    double2 v = a[i];
    b[i] = make_float2((float)v.x, (float)v.y);
}

void launch_pack_spinor64(const double2* ext, double2* in, int64_t V, int64_t Vt, int n,
                          hipStream_t s) {
    dim3 grid((unsigned)((V + kBlock - 1) / kBlock), n);
    hipLaunchKernelGGL(k_pack_spinor<double>, grid, dim3(kBlock), 0, s, ext, in, V, Vt);
}
void launch_pack_spinor32(const double2* ext, float2* in, int64_t V, int64_t Vt, int n,
                          hipStream_t s) {
    dim3 grid((unsigned)((V + kBlock - 1) / kBlock), n);
    hipLaunchKernelGGL(k_pack_spinor<float>, grid, dim3(kBlock), 0, s, ext, in, V, Vt);
}
void launch_unpack_spinor64(const double2* in, double2* ext, int64_t V, int64_t Vt, int n,
                            hipStream_t s) {
    dim3 grid((unsigned)((V + kBlock - 1) / kBlock), n);
    hipLaunchKernelGGL(k_unpack_spinor<double>, grid, dim3(kBlock), 0, s, in, ext, V, Vt);
}
void launch_unpack_spinor32(const float2* in, double2* ext, int64_t V, int64_t Vt, int n,
                            hipStream_t s) {
    dim3 grid((unsigned)((V + kBlock - 1) / kBlock), n);
    hipLaunchKernelGGL(k_unpack_spinor<float>, grid, dim3(kBlock), 0, s, in, ext, V, Vt);
}
void launch_unpack_dov(const double2* s_int, const double2* b_ext, double2* out_ext, double a,
                       double bm, int64_t V, int64_t Vt, int n, hipStream_t s) {
    dim3 grid((unsigned)((V + kBlock - 1) / kBlock), n);
    hipLaunchKernelGGL(k_unpack_dov, grid, dim3(kBlock), 0, s, s_int, b_ext, out_ext, a, bm, V, Vt);
}
int gauge_blocks(const Geom& g) { return (int)((g.V + kBlock - 1) / kBlock); }
void launch_pack_gauge(const double2* ext, double2* U64, float2* U32, double2* U64c, float2* U32c,
                       const Geom& g, double* defect, hipStream_t s) {
    dim3 grid((unsigned)gauge_blocks(g), 4);
    hipLaunchKernelGGL(k_pack_gauge, grid, dim3(kBlock), 0, s, ext, U64, U32, U64c, U32c, g,
                       defect);
}
// y += a x
__global__ __launch_bounds__(kBlock) void k_axpy(double2* __restrict__ y,
                                                 const double2* __restrict__ x, double a,
                                                 int64_t n) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e < n) {
        double2 v = y[e];
        const double2 w = x[e];
        v.x += a * w.x;
        v.y += a * w.y;
        y[e] = v;
    }
}
void launch_axpy(double2* y, const double2* x, double a, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_axpy, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, y,
                       x, a, n);
}

// One block per job: copy the job's state block into pinned host slot
// (k / chunk) & 1, k the iteration counter after the chunk.
__global__ __launch_bounds__(kBlock) void k_export_state(const JobDesc* __restrict__ jobs,
                                                         const int* __restrict__ kdev, int chunk) {
    const JobDesc& J = jobs[blockIdx.x];
    if (J.state_host == nullptr) return;
    const int slot = (*kdev / chunk) & 1;
    const uint2* src = reinterpret_cast<const uint2*>(J.state_dev);
    uint2* dst = reinterpret_cast<uint2*>(J.state_host + (size_t)slot * J.state_stride);
    for (int e = threadIdx.x; e < J.state_bytes / 8; e += kBlock) dst[e] = src[e];
}
void launch_export_state(const JobDesc* jobs, int njobs, const int* kdev, int chunk,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_export_state, dim3(njobs), dim3(kBlock), 0, s, jobs, kdev, chunk);
}

// One job's iteration precision, written in stream order (the job kernels
// queued after it read the new value).
__global__ void k_set_phase(JobDesc* __restrict__ job, int phase) {
    if (threadIdx.x == 0) job->phase = phase;
}
void launch_set_phase(JobDesc* job, int phase, hipStream_t s) {
    hipLaunchKernelGGL(k_set_phase, dim3(1), dim3(64), 0, s, job, phase);
}

void launch_convert_64_to_32(const double2* a, float2* b, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_convert, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       s, a, b, n);
}

// ============================================================================
// The seed iteration k is two kernels:
//   K1  q_k = z_s r_k - H r_k + beta_{k-1} q_{k-1} with per-block <r_k, q_k>,
//       ||q_k||^2, ||r_k||^2 (k_wilson_jobs, mode 1)
//   K2  alpha_k, beta_k (every block, from K1's partials), shifted pi_{k+1},
//       alpha^j, beta^j, residual estimates and deactivation (blocks
//       0..nslices-1 own one 256-shift slice each, one lane per shift), then
//       r_{k+1} = r_k - alpha_k q_k, alone or with the shift sweep.
// Quantities written in iteration k live in parity (k&1) or mod-3 buffers, so
// no block reads what another block of the same kernel writes:
//   SrcState.rr[k&1] = ||r_k||^2, alpha[k&1], beta[k&1];
//   pi[k%3] = pi_k^j; active[k&1][j] = shift j active at the start of k;
//   cnt[k&1][slice] = active shifts per 256-shift slice (a source is live at
//   iteration k while status == 0 and some count is nonzero).
// ============================================================================

// sum of partial[0..nb) in a fixed order (strided per lane, then block_sum)
template <typename T>
__device__ __forceinline__ double sum_partials_re(const T* p, int nb, double* sh);
template <>
__device__ __forceinline__ double sum_partials_re<double>(const double* p, int nb, double* sh) {
    double v = 0.0;
    for (int b = threadIdx.x; b < nb; b += kBlock) v += p[b];
    return block_sum<kBlock>(v, sh);
}
int vec_blocks(int64_t n12, int nslices, bool slice_blocks) {
    int nb = (int)((n12 + 4 * kBlock - 1) / (4 * kBlock));
    // slice_blocks (update kernel of the basis forms): at most 256 vector
    // blocks per source, each block reducing the stencil partials once for
    // more of the vector (at 16^4 x 4 the update took 3.33 / 5.75 ms per
    // step in FP64 / FP32 with 256, 3.46 / 5.95 with 512, 3.36 / 6.28 with
    // 1024, and more with 128 or 192), plus one block per 256-shift slice,
    // which advances the slice while the others share the vector pass.
    // Otherwise up to 512 blocks, every one also taking vector work.
    if (slice_blocks) return (nb > 256 ? 256 : nb) + nslices;
    if (nb > 512) nb = 512;
    return nb < nslices ? nslices : nb;
}

// Decode a vector-grid block: job, source n and block bx of nbe for it.
struct VecBlock {
    int j, n, bx;
};
__device__ __forceinline__ VecBlock vec_block(const JobDesc* jobs, int njobs) {
    const int gb = (int)blockIdx.x;
    int j = 0;
    while (j + 1 < njobs && gb >= jobs[j + 1].vec_b0) ++j;
    const int local = gb - jobs[j].vec_b0;
    return VecBlock{j, local / jobs[j].nbe, local % jobs[j].nbe};
}

// seed scalars of iteration k from the stencil's partials of source n
__device__ __forceinline__ SeedScalars seed_scalars(const JobDesc& J, int n, double* shm) {
    return seed_scalars_from(J.part_w + (size_t)n * J.nsb, J.nsb, shm);
}

// The seed iteration's second kernel (after the stencil), for every form:
// scalars, shift bookkeeping (the 256-shift slice of block bx), then one pass
// over the components: r_{k+1} = r_k - alpha q (basis forms; two-pass second
// pass also s += h_{k+1} r_{k+1}), or that with the shift sweep (fused:
// s += c_j alpha^j p_j; reference: x_j += alpha^j p_j; then
// p_j = r_{k+1}/pi_{k+1} + beta^j p_j).  In the first iteration p_j = b for
// every j, read from b instead.  The seed direction p is never formed: the
// stencil builds q_{k+1} = A r_{k+1} + beta_k q_k from r_{k+1} directly.
template <typename R, int KIND>  // KIND 0 basis / two-pass, 1 fused sweep, 2 reference sweep
__device__ __forceinline__ void update_block(const JobDesc& J, int n, int bx, int k) {
    constexpr bool SWEEP = KIND != 0;
    const int f = sizeof(R) == 4 ? 1 : 0;
    const ShiftDev& sh = J.sh;
    SrcState& S = J.st[n];
    __shared__ double shm[4 * kBlock / 64];
    int* cnt_next = sh.cnt + ((size_t)((k + 1) & 1) * sh.nsrc + n) * kMaxSlices;
    if (!src_live(S, sh, n, k)) {
        // a finished source stays finished; at the iteration limit the counts
        // of the last iteration are kept, so the host sees what is still active
        if (k < sh.maxk && bx < sh.nslices && threadIdx.x == 0) cnt_next[bx] = 0;
        return;
    }
    const SeedScalars sc = seed_scalars(J, n, shm);
    if (sc.status) {
        if (bx == 0 && threadIdx.x == 0) S.status = sc.status;
        if (bx < sh.nslices && threadIdx.x == 0) cnt_next[bx] = 0;
        return;
    }
    if (bx == 0 && threadIdx.x == 0) {
        S.alpha[k & 1] = sc.alpha;
        S.beta[k & 1] = sc.beta;
        S.rr[k & 1] = sc.rr;
        S.iter = k + 1;
        if (sh.seed != nullptr) {
            double2* sd = sh.seed + ((size_t)n * (sh.maxk + 1) + k) * 3;
            sd[0] = sc.alpha;
            sd[1] = sc.beta;
            sd[2] = make_double2(sc.rr, sc.rrn);
        }
    }
    const double2 c1 = cdiv(cmul(sc.alpha, S.beta[(k + 1) & 1]), S.alpha[(k + 1) & 1]);
    const size_t stride3 = (size_t)sh.nsrc * sh.J;
    // LDS list of the active shifts (sweep forms)
    extern __shared__ unsigned char lds_raw[];
    double2* l_coef = reinterpret_cast<double2*>(lds_raw);
    double2* l_ipi = l_coef + sh.J;
    double2* l_b = l_ipi + sh.J;
    int* l_j = reinterpret_cast<int*>(l_b + sh.J);
    __shared__ int wcount[kBlock / 64];
    __shared__ int base;
    if (SWEEP) {
        if (threadIdx.x == 0) base = 0;
        __syncthreads();
    }
    for (int j0 = 0; j0 < sh.J; j0 += kBlock) {
        const bool mine = (j0 / kBlock) == bx;  // this block keeps the state of slice j0
        if (!SWEEP && !mine) continue;
        const int j = j0 + threadIdx.x;
        const size_t o = (size_t)n * sh.J + j;
        const bool act = j < sh.J && sh.active[(size_t)(k & 1) * stride3 + o] != 0;
        ShiftScalars t{};
        if (act) t = shift_scalars(sh, o, j, k, sc, c1, S.bb);
        if (mine) {
            int stay = 0;
            if (j < sh.J) {
                if (act) {
                    sh.pi[(size_t)((k + 1) % 3) * stride3 + o] = t.pn;
                    sh.aj[o] = t.aj;
                    sh.res[o] = t.res;
                    stay = (t.res > sh.tol && isfinite(t.res)) ? 1 : 0;
                }
                sh.active[(size_t)((k + 1) & 1) * stride3 + o] = stay;
                if (sh.h_a != nullptr) {
                    const size_t ho = ((size_t)n * (sh.maxk + 1) + k) * sh.J + j;
                    sh.h_a[ho] = act ? t.aj : make_double2(0, 0);
                    sh.h_b[ho] = act ? t.bj : make_double2(0, 0);
                    sh.h_pi[ho + sh.J] = act ? t.pn : make_double2(1, 0);
                }
            }
            double tot = (double)stay, mx = act ? t.res : 0.0;  // (shm: 2 kBlock/64 values)
            block_sum_max<kBlock>(tot, mx, shm);
            if (threadIdx.x == 0) {
                cnt_next[bx] = (int)(tot + 0.5);
                sh.mres[(size_t)n * kMaxSlices + bx] = mx;
            }
        }
        if (SWEEP) {
            const double2 coef = act ? (KIND == 2 ? t.aj : cmul(sh.c[j], t.aj)) : make_double2(0, 0);
            const unsigned long long m = __ballot(act);
            const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
            const int before = __popcll(m & ((1ull << lane) - 1ull));
            if (lane == 0) wcount[w] = __popcll(m);
            __syncthreads();
            int off = base;
            for (int i = 0; i < w; ++i) off += wcount[i];
            if (act) {
                l_j[off + before] = j;
                l_coef[off + before] = coef;
                l_ipi[off + before] = t.ipi;
                l_b[off + before] = t.bj;
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                int tot = 0;
                for (int i = 0; i < kBlock / 64; ++i) tot += wcount[i];
                base += tot;
            }
            __syncthreads();
        }
    }
    const int64_t n12 = 12 * J.g.Vt;
    const R ar = (R)sc.alpha.x, ai = (R)sc.alpha.y;
    // basis forms: the blocks that advance a shift slice (bx < nslices) take
    // no part in the vector pass, which the other nbe - nslices blocks share,
    // so the slice bookkeeping runs beside it instead of before a share of it
    const int64_t vbx = SWEEP ? bx : bx - sh.nslices;
    const int64_t vnb = SWEEP ? J.nbe : J.nbe - sh.nslices;
    if (vbx < 0) return;
    const C2<R>* ri = job_rk<const C2<R>>(J, k, f) + (size_t)n * n12;
    C2<R>* ro = job_rk<C2<R>>(J, k + 1, f) + (size_t)n * n12;
    const C2<R>* qq = static_cast<const C2<R>*>(J.q[f]) + (size_t)n * n12;
    if constexpr (!SWEEP && sizeof(R) == 4) {
        // FP32: two components per lane in one 16-byte access of each array
        // (every vector starts 16-byte aligned and 12 Vt is even)
        const bool acc2 = J.h != nullptr;
        const double2 hk = acc2 ? J.h[(size_t)n * (sh.maxk + 1) + k + 1] : make_double2(0, 0);
        double2* sacc = J.s64 + (size_t)n * n12;
        // (global address-space pointers: global, not flat, loads and stores)
        typedef float __attribute__((ext_vector_type(4))) F4;
        const OVL_GLOBAL F4* ri4 = (const OVL_GLOBAL F4*)ri;
        const OVL_GLOBAL F4* qq4 = (const OVL_GLOBAL F4*)qq;
        OVL_GLOBAL F4* ro4 = (OVL_GLOBAL F4*)ro;
        const int64_t n2 = n12 / 2;
        for (int64_t e = vbx * kBlock + threadIdx.x; e < n2; e += vnb * kBlock) {
            const F4 r = ri4[e], qv = qq4[e];
            F4 rn;
            rn.x = r.x - ((float)ar * qv.x - (float)ai * qv.y);
            rn.y = r.y - ((float)ar * qv.y + (float)ai * qv.x);
            rn.z = r.z - ((float)ar * qv.z - (float)ai * qv.w);
            rn.w = r.w - ((float)ar * qv.w + (float)ai * qv.z);
            ro4[e] = rn;
            if (acc2) {
                double2 s0 = sacc[2 * e], s1 = sacc[2 * e + 1];
                s0.x += hk.x * (double)rn.x - hk.y * (double)rn.y;
                s0.y += hk.x * (double)rn.y + hk.y * (double)rn.x;
                s1.x += hk.x * (double)rn.z - hk.y * (double)rn.w;
                s1.y += hk.x * (double)rn.w + hk.y * (double)rn.z;
                sacc[2 * e] = s0;
                sacc[2 * e + 1] = s1;
            }
        }
    } else if constexpr (!SWEEP) {
        const bool acc2 = J.h != nullptr;
        const double2 hk = acc2 ? J.h[(size_t)n * (sh.maxk + 1) + k + 1] : make_double2(0, 0);
        double2* sacc = J.s64 + (size_t)n * n12;
        for (int64_t e = vbx * kBlock + threadIdx.x; e < n12; e += vnb * kBlock) {
            const cx<R> r = ld<R>(ri, e), qv = ld<R>(qq, e);
            const cx<R> rn = mk<R>(r.re - (ar * qv.re - ai * qv.im), r.im - (ar * qv.im + ai * qv.re));
            stc<R>(ro, e, rn);
            if (acc2) {
                double2 sv = sacc[e];
                sv.x += hk.x * (double)rn.re - hk.y * (double)rn.im;
                sv.y += hk.x * (double)rn.im + hk.y * (double)rn.re;
                sacc[e] = sv;
            }
        }
    } else {
        const int nl = base;
        C2<R>* pj = static_cast<C2<R>*>(J.pj[f]);
        double2* acc_out = KIND == 2 ? J.xj : J.s64;
        const double2* b0 = J.b64;
        for (int64_t e = (int64_t)bx * kBlock + threadIdx.x; e < n12; e += (int64_t)J.nbe * kBlock) {
            const cx<R> r = ld<R>(ri, e), qv = ld<R>(qq, e);
            const cx<R> rv = mk<R>(r.re - (ar * qv.re - ai * qv.im), r.im - (ar * qv.im + ai * qv.re));
            stc<R>(ro, e, rv);
            const cx<R> bfirst = (k == 0) ? mk<R>((R)b0[(size_t)n * n12 + e].x, (R)b0[(size_t)n * n12 + e].y)
                                          : mk<R>(0, 0);
            double sre = 0.0, sim = 0.0;
            for (int l = 0; l < nl; ++l) {
                const int j = l_j[l];
                const double2 ca = l_coef[l], ip = l_ipi[l], bj = l_b[l];
                C2<R>* pjp = pj + ((size_t)n * sh.J + j) * n12;
                const cx<R> pv = (k == 0) ? bfirst : ld<R>(pjp, e);
                if constexpr (KIND == 2) {
                    double2* xp = acc_out + ((size_t)n * sh.J + j) * n12;
                    double2 x = xp[e];
                    x.x += ca.x * (double)pv.re - ca.y * (double)pv.im;
                    x.y += ca.x * (double)pv.im + ca.y * (double)pv.re;
                    xp[e] = x;
                } else {
                    sre += ca.x * (double)pv.re - ca.y * (double)pv.im;
                    sim += ca.x * (double)pv.im + ca.y * (double)pv.re;
                }
                const R ipr = (R)ip.x, ipi_ = (R)ip.y, bjr = (R)bj.x, bji = (R)bj.y;
                stc<R>(pjp, e, mk<R>(rv.re * ipr - rv.im * ipi_ + bjr * pv.re - bji * pv.im,
                                     rv.re * ipi_ + rv.im * ipr + bjr * pv.im + bji * pv.re));
            }
            if constexpr (KIND == 1) {
                double2 sv = acc_out[(size_t)n * n12 + e];
                sv.x += sre;
                sv.y += sim;
                acc_out[(size_t)n * n12 + e] = sv;
            }
        }
    }
}

// The iteration counter lives in two device slots: iteration k reads slot
// kread and the update kernel's first lane publishes k + 1 in the other slot,
// kwrite, which no block of the same launch reads.
template <typename R, int KIND>
__global__ __launch_bounds__(kBlock) void k_update_jobs(const JobDesc* __restrict__ jobs, int njobs,
                                                        const int* __restrict__ kread,
                                                        int* __restrict__ kwrite) {
    const int k = (int)uniform((uint32_t)*kread);
    // (when both precisions run in one iteration, both launches write the
    // same k + 1: the counter stays consistent)
    if (blockIdx.x == 0 && threadIdx.x == 0) *kwrite = k + 1;
    const VecBlock v = vec_block(jobs, njobs);
    if (jobs[v.j].phase != (sizeof(R) == 4 ? 1 : 0)) return;  // the other precision's job
    update_block<R, KIND>(jobs[v.j], v.n, v.bx, k);
}

template <typename R>
void launch_iteration_update(const JobDesc* jobs, int njobs, const int* kread, int* kwrite,
                             int vec_blocks_total, int form, int maxJ, hipStream_t s,
                             hipEvent_t ev0, hipEvent_t ev1) {
    const dim3 grid(vec_blocks_total), blk(kBlock);
    const size_t lds = (size_t)maxJ * (3 * sizeof(double2) + sizeof(int));
    auto go = [&](auto kern, size_t shmem) {
        if (ev0)
            hipExtLaunchKernelGGL(kern, grid, blk, (uint32_t)shmem, s, ev0, ev1, 0, jobs, njobs,
                                  kread, kwrite);
        else
            hipLaunchKernelGGL(kern, grid, blk, shmem, s, jobs, njobs, kread, kwrite);
    };
    if (form == OVL_FORM_BASIS || form == OVL_FORM_TWOPASS)
        go(k_update_jobs<R, 0>, 0);
    else if (form == OVL_FORM_FUSED)
        go(k_update_jobs<R, 1>, lds);
    else
        go(k_update_jobs<R, 2>, lds);
}
template void launch_iteration_update<double>(const JobDesc*, int, const int*, int*, int, int, int,
                                              hipStream_t, hipEvent_t, hipEvent_t);
template void launch_iteration_update<float>(const JobDesc*, int, const int*, int*, int, int, int,
                                             hipStream_t, hipEvent_t, hipEvent_t);

// two-pass form, second pass: s = h_0 b (r_0 = b)
__global__ __launch_bounds__(kBlock) void k_s_init(const double2* __restrict__ b,
                                                   const double2* __restrict__ h, int maxk,
                                                   double2* __restrict__ sv, int64_t n12) {
    const int n = blockIdx.y;
    const double2 h0 = h[(size_t)n * (maxk + 1)];
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < n12;
         e += (int64_t)gridDim.x * kBlock) {
        const double2 v = b[(size_t)n * n12 + e];
        sv[(size_t)n * n12 + e] = make_double2(h0.x * v.x - h0.y * v.y, h0.x * v.y + h0.y * v.x);
    }
}
void launch_s_init(const double2* b, const double2* h, int maxk, double2* s, int64_t n12, int nsrc,
                   hipStream_t st) {
    hipLaunchKernelGGL(k_s_init, dim3(vec_blocks(n12, 1, false), nsrc), dim3(kBlock), 0, st, b, h, maxk,
                       s, n12);
}

// s = sum_j c_j x_j (reference form, once at the end; fixed order in j)
__global__ __launch_bounds__(kBlock) void k_sum_ref(const double2* __restrict__ xj,
                                                    const double2* __restrict__ c,
                                                    double2* __restrict__ sacc, int J,
                                                    int64_t n12) {
    const int n = blockIdx.y;
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= n12) return;
    double re = 0.0, im = 0.0;
    for (int j = 0; j < J; ++j) {
        const double2 x = xj[((int64_t)n * J + j) * n12 + e];
        const double2 cj = c[j];
        re += cj.x * x.x - cj.y * x.y;
        im += cj.x * x.y + cj.y * x.x;
    }
    sacc[n * n12 + e] = make_double2(re, im);
}
void launch_sum_ref(const double2* xj, const double2* c, double2* sacc, int J, int64_t n12,
                    int nsrc, hipStream_t s) {
    dim3 grid((unsigned)((n12 + kBlock - 1) / kBlock), nsrc);
    hipLaunchKernelGGL(k_sum_ref, grid, dim3(kBlock), 0, s, xj, c, sacc, J, n12);
}

// ============================================================================
// basis forms
// ============================================================================
// x_j = sum_i u_i^j r_i with u_i^j = P_i^j / pi_i^j,
// P_i^j = alpha_i^j + beta_i^j P_{i+1}^j, P_K^j = 0 (alpha^j recorded as 0
// once shift j stopped, which freezes x_j exactly as the sweep does).  The
// backward recursion is split over kSeg segments of i per shift, so that
// kSeg lanes share it: each lane composes its segment's affine maps
// (P_lo = A + B P_hi), one lane per shift chains the segment ends from
// P_K = 0, and each lane then runs the recursion over its segment from its
// P_hi, storing P_i^j in W[src][i][j]; the row kernel below divides by
// pi_i^j in place, in parallel over (i, j).  Block: kCoefShifts shifts x
// kSeg segments of one source.
constexpr int kSeg = 16, kCoefShifts = kBlock / kSeg;
__global__ __launch_bounds__(kBlock) void k_coef(const double2* __restrict__ h_a,
                                                 const double2* __restrict__ h_b,
                                                 const SrcState* __restrict__ st,
                                                 double2* __restrict__ W, int J, int maxk) {
    __shared__ double2 lA[kSeg][kCoefShifts], lB[kSeg][kCoefShifts], lP[kSeg][kCoefShifts];
    const int n = blockIdx.y;
    const int jl = (int)(threadIdx.x % kCoefShifts), seg = (int)(threadIdx.x / kCoefShifts);
    const int j = blockIdx.x * kCoefShifts + jl;
    const bool on = j < J;
    const int K = st[n].iter;
    const int len = (K + kSeg - 1) / kSeg;
    const int lo = seg * len < K ? seg * len : K, hi = lo + len < K ? lo + len : K;
    const int64_t hb = (int64_t)n * (maxk + 1) * J;
    // loads of U steps are issued before the steps that use them
    constexpr int U = 16;
    // 1. this segment's map: P_lo = A + B P_hi
    double2 A = make_double2(0, 0), B = make_double2(1, 0);
    for (int i0 = hi - 1; on && i0 >= lo; i0 -= U) {
        double2 a[U], b[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (i0 - u >= lo) {
                a[u] = h_a[hb + (int64_t)(i0 - u) * J + j];
                b[u] = h_b[hb + (int64_t)(i0 - u) * J + j];
            }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (i0 - u >= lo) {
                A = cadd(a[u], cmul(b[u], A));
                B = cmul(b[u], B);
            }
    }
    lA[seg][jl] = A;
    lB[seg][jl] = B;
    __syncthreads();
    // 2. segment ends, from the last segment (P_K = 0) down
    if (seg == 0) {
        double2 P = make_double2(0, 0);
        for (int q = kSeg - 1; q >= 0; --q) {
            lP[q][jl] = P;  // P at the segment's upper end
            P = cadd(lA[q][jl], cmul(lB[q][jl], P));
        }
    }
    __syncthreads();
    // 3. the recursion over this segment from its upper end
    double2 P = lP[seg][jl];
    for (int i0 = hi - 1; on && i0 >= lo; i0 -= U) {
        double2 a[U], b[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (i0 - u >= lo) {
                a[u] = h_a[hb + (int64_t)(i0 - u) * J + j];
                b[u] = h_b[hb + (int64_t)(i0 - u) * J + j];
            }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (i0 - u >= lo) {
                P = cadd(a[u], cmul(b[u], P));
                W[hb + (int64_t)(i0 - u) * J + j] = P;
            }
    }
}
// Row i of source n, one wave per row: u_i^j = P_i^j / pi_i^j (pi_0 = 1)
// over P in W, and h[src][i] = sum_j c_j u_i^j with lane l adding the shifts
// j = l, l + 64, ... in that order, then a butterfly over the lanes (a fixed
// order; the row is read in coalesced 1 KiB pieces).  Rows from the source's
// iteration count on get h = 0.
__global__ __launch_bounds__(kBlock) void k_hsum(double2* __restrict__ W,
                                                 const double2* __restrict__ h_pi,
                                                 const double2* __restrict__ c,
                                                 const SrcState* __restrict__ st,
                                                 double2* __restrict__ h, int J, int maxk) {
    const int n = blockIdx.y;
    const int i = blockIdx.x * (kBlock / 64) + (int)(threadIdx.x >> 6);
    const int l = (int)(threadIdx.x & 63);
    if (i > maxk) return;  // wave-uniform
    const int K = st[n].iter;
    double2 t = make_double2(0, 0);
    if (i < K) {
        const int64_t o = ((int64_t)n * (maxk + 1) + i) * J;
        for (int j = l; j < J; j += 64) {
            const double2 u = i == 0 ? W[o + j] : cdiv(W[o + j], h_pi[o + j]);
            W[o + j] = u;
            t = cadd(t, cmul(c[j], u));
        }
    }
    t.x = wave_sum(t.x);
    t.y = wave_sum(t.y);
    if (l == 0) h[(int64_t)n * (maxk + 1) + i] = t;
}
void launch_basis_coef(const double2* h_a, const double2* h_b, const double2* h_pi,
                       const double2* c, const SrcState* st, double2* W, double2* h, int J,
                       int maxk, int nsrc, hipStream_t s) {
    hipLaunchKernelGGL(k_coef, dim3((J + kCoefShifts - 1) / kCoefShifts, nsrc), dim3(kBlock), 0, s,
                       h_a, h_b, st, W, J, maxk);
    hipLaunchKernelGGL(k_hsum, dim3((maxk + 1 + kBlock / 64 - 1) / (kBlock / 64), nsrc),
                       dim3(kBlock), 0, s, W, h_pi, c, st, h, J, maxk);
}

// The in-band residual check: for every source pick one shift (below), and
// copy its basis coefficients u_i^j = W[src][i][j] into hx[src][i] (zero
// beyond the source's iteration count) and its node into zc[src].  One block
// per source.
__global__ __launch_bounds__(kBlock) void k_pick_check(const double* __restrict__ res,
                                                       const double2* __restrict__ W,
                                                       const double2* __restrict__ z,
                                                       const SrcState* __restrict__ st, int J,
                                                       int maxk, double2* __restrict__ hx,
                                                       double2* __restrict__ zc) {
    // The checked shift is the one that stayed active longest (its last
    // nonzero coefficient u_i^j comes latest), ties to the largest final
    // estimate, then the lower index.  Every converged shift ends with an
    // estimate just below the tolerance, so the estimate alone does not tell
    // which shift ran through the most FP32 iterations of a mixed solve; the
    // one active longest carries the most of their rounding.
    const int n = blockIdx.x;
    const int K = st[n].iter;
    const double2* Wn = W + (size_t)n * (maxk + 1) * J;
    int bl = -1;
    double best = -1.0;
    int bj = 0;
    for (int j = threadIdx.x; j < J; j += kBlock) {
        // u_i^j is nonzero while the shift is active and zero from its
        // deactivation on (its history then holds zeros): bisect for the
        // last nonzero coefficient, about log2 K loads
        int lo = -1, hi = K;  // Wn[lo] nonzero (or lo = -1), Wn[hi] zero (or hi = K)
        while (hi - lo > 1) {
            const int mid = (lo + hi) / 2;
            const double2 u = Wn[(size_t)mid * J + j];
            if (u.x != 0.0 || u.y != 0.0) lo = mid;
            else hi = mid;
        }
        const int last = lo;
        const double v = res[(size_t)n * J + j];
        if (last > bl || (last == bl && v > best)) {  // j increases: ties keep the lower j
            bl = last;
            best = v;
            bj = j;
        }
    }
    // block argmax of (last, estimate), ties to the lower index
    __shared__ int sl[kBlock];
    __shared__ double sv[kBlock];
    __shared__ int sj[kBlock];
    sl[threadIdx.x] = bl;
    sv[threadIdx.x] = best;
    sj[threadIdx.x] = bj;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            const int la = sl[threadIdx.x], lb = sl[threadIdx.x + o];
            const double a = sv[threadIdx.x], b = sv[threadIdx.x + o];
            const int ja = sj[threadIdx.x], jb = sj[threadIdx.x + o];
            if (lb > la || (lb == la && (b > a || (b == a && jb < ja)))) {
                sl[threadIdx.x] = lb;
                sv[threadIdx.x] = b;
                sj[threadIdx.x] = jb;
            }
        }
        __syncthreads();
    }
    const int j = sj[0];
    for (int i = threadIdx.x; i <= maxk; i += kBlock)
        hx[(size_t)n * (maxk + 1) + i] =
            i < K ? W[((size_t)n * (maxk + 1) + i) * J + j] : make_double2(0, 0);
    if (threadIdx.x == 0) zc[n] = z[j];
}
void launch_pick_check(const double* res, const double2* W, const double2* z, const SrcState* st,
                       int J, int maxk, int nsrc, double2* hx, double2* zc, hipStream_t s) {
    hipLaunchKernelGGL(k_pick_check, dim3(nsrc), dim3(kBlock), 0, s, res, W, z, st, J, maxk, hx, zc);
}

// ============================================================================
// solver initialisation
// ============================================================================
// partial[src][blk] = ||b||^2 over the block
__global__ __launch_bounds__(kBlock) void k_norm2(const double2* __restrict__ b,
                                                  double* __restrict__ partial, int64_t n12) {
    const int n = blockIdx.y;
    double acc = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < n12;
         e += (int64_t)gridDim.x * kBlock) {
        const double2 v = b[n * n12 + e];
        acc += v.x * v.x + v.y * v.y;
    }
    __shared__ double sh[kBlock / 64];
    const double t = block_sum<kBlock>(acc, sh);
    if (threadIdx.x == 0) partial[(int64_t)n * gridDim.x + blockIdx.x] = t;
}
// Iteration 0 state: r = p = b, pi_0 = pi_{-1} = 1, every shift active,
// alpha_{-1} = 1, beta_{-1} = 0.  One block per (slice, source).
__global__ __launch_bounds__(kBlock) void k_init_state(SrcState* __restrict__ st,
                                                       const double* __restrict__ partial,
                                                       int nblk, ShiftDev sh) {
    const int n = blockIdx.y;
    __shared__ double shm[kBlock / 64];
    const double bb = sum_partials_re<double>(partial + (size_t)n * nblk, nblk, shm);
    const bool ok = bb > 0.0 && isfinite(bb);
    const size_t stride3 = (size_t)sh.nsrc * sh.J;
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j < sh.J) {
        const size_t o = (size_t)n * sh.J + j;
        sh.pi[o] = make_double2(1, 0);
        sh.pi[2 * stride3 + o] = make_double2(1, 0);
        sh.active[o] = ok ? 1 : 0;
        sh.res[o] = ok ? 1.0 : 0.0;
        if (sh.h_pi != nullptr) sh.h_pi[(size_t)n * (sh.maxk + 1) * sh.J + j] = make_double2(1, 0);
    }
    if (threadIdx.x == 0) {
        int c = sh.J - blockIdx.x * kBlock;
        c = c > kBlock ? kBlock : c;
        // both parities: the two-kernel iteration k reads counts [k&1], the
        // fused kernel k reads [(k-1)&1]
        sh.cnt[(size_t)n * kMaxSlices + blockIdx.x] = ok ? c : 0;
        sh.cnt[((size_t)sh.nsrc + n) * kMaxSlices + blockIdx.x] = ok ? c : 0;
        sh.mres[(size_t)n * kMaxSlices + blockIdx.x] = ok ? 1.0 : 0.0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        SrcState S;
        S.bb = bb;
        S.rr[0] = bb;
        S.rr[1] = 0.0;
        S.alpha[0] = make_double2(0, 0);
        S.alpha[1] = make_double2(1, 0);
        S.beta[0] = make_double2(0, 0);
        S.beta[1] = make_double2(0, 0);
        S.iter = 0;
        S.status = isfinite(bb) ? 0 : OVL_E_NONFINITE;
        S.pad[0] = S.pad[1] = 0;
        st[n] = S;
    }
}
size_t init_partials(int64_t n12, int nslices, int nsrc) {
    return (size_t)nsrc * vec_blocks(n12, nslices, false);
}
void launch_init_state(SrcState* st, const double2* b, double* partial, int64_t n12,
                       const ShiftDev& sh, hipStream_t s) {
    const int nb = vec_blocks(n12, sh.nslices, false);  // partial holds init_partials(...)
    hipLaunchKernelGGL(k_norm2, dim3(nb, sh.nsrc), dim3(kBlock), 0, s, b, partial, n12);
    hipLaunchKernelGGL(k_init_state, dim3(sh.nslices, sh.nsrc), dim3(kBlock), 0, s, st, partial,
                       nb, sh);
}

// ============================================================================
// force (derivative of S = |D_ov phi|^2 with respect to the links)
// ============================================================================
// d = a b + bm gamma5 s ;  psi = bm gamma5 d ;  partial[blk] = |d|^2  (one source)
__global__ __launch_bounds__(kBlock) void k_dov_psi(const double2* __restrict__ b,
                                                    const double2* __restrict__ sv,
                                                    double2* __restrict__ psi, double a, double bm,
                                                    int64_t Vt, double* __restrict__ partial) {
    const int64_t n12 = 12 * Vt;
    double acc = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < n12;
         e += (int64_t)gridDim.x * kBlock) {
        // tiled layout: component = (e / 64) % 12, spin = component / 3
        const double g5 = ((e / kTile) % 12) < 6 ? 1.0 : -1.0;
        const double2 bv = b[e], s = sv[e];
        const double2 d = make_double2(a * bv.x + bm * g5 * s.x, a * bv.y + bm * g5 * s.y);
        acc += d.x * d.x + d.y * d.y;
        psi[e] = make_double2(bm * g5 * d.x, bm * g5 * d.y);
    }
    __shared__ double sh[kBlock / 64];
    const double t = block_sum<kBlock>(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}
void launch_dov_psi(const double2* b, const double2* s, double2* psi, double a, double bm,
                    int64_t Vt, double* partial, int nblk, hipStream_t st) {
    hipLaunchKernelGGL(k_dov_psi, dim3(nblk), dim3(kBlock), 0, st, b, s, psi, a, bm, Vt, partial);
}

// Y[j][e] = sum_{i < K} u_i^{j} r_i[e] for shifts j0 .. j0+jn-1 (jn <= JG) of
// one source: every stored slot in turn (FP64 below ksw, FP32 from it, at
// the slot base), through the device table of slot chunks, each output
// written once.  The basis is read once per group of JG shifts.
template <int JG>
__global__ __launch_bounds__(kBlock) void k_materialize(char* const* __restrict__ chunks,
                                                        size_t slot_bytes, int K, int ksw,
                                                        const double2* __restrict__ W, int J,
                                                        int j0, int jn, double2* __restrict__ Y,
                                                        int64_t n12, int64_t eoff) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= n12) return;
    double re[JG], im[JG];
#pragma unroll
    for (int q = 0; q < JG; ++q) re[q] = im[q] = 0.0;
    // the slot bases come from a table in memory: the loads go through
    // global address-space pointers (global, not flat, loads)
    typedef double __attribute__((ext_vector_type(2))) D2;
    typedef float __attribute__((ext_vector_type(2))) F2;
    for (int i = 0; i < K; ++i) {
        const OVL_GLOBAL char* slot =
            (const OVL_GLOBAL char*)chunks[i / kSlotChunk] + (size_t)(i % kSlotChunk) * slot_bytes;
        double vr, vi;
        if (i < ksw) {
            const D2 v = ((const OVL_GLOBAL D2*)slot)[eoff + e];
            vr = v.x;
            vi = v.y;
        } else {
            const F2 v = ((const OVL_GLOBAL F2*)slot)[eoff + e];
            vr = v.x;
            vi = v.y;
        }
        const double2* wr = W + (size_t)i * J + j0;
#pragma unroll
        for (int q = 0; q < JG; ++q) {
            if (q < jn) {
                const double2 u = wr[q];
                re[q] += u.x * vr - u.y * vi;
                im[q] += u.x * vi + u.y * vr;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < JG; ++q)
        if (q < jn) Y[(size_t)q * n12 + e] = make_double2(re[q], im[q]);
}
constexpr int kMatGroup = 16;
void launch_materialize(char* const* chunks, size_t slot_bytes, int K, int ksw, const double2* W,
                        int J, int j0, int jn, double2* Y, int64_t n12, int64_t eoff,
                        hipStream_t s) {
    dim3 grid((unsigned)((n12 + kBlock - 1) / kBlock));
    for (int q0 = 0; q0 < jn; q0 += kMatGroup) {
        const int m = jn - q0 < kMatGroup ? jn - q0 : kMatGroup;
        hipLaunchKernelGGL(k_materialize<kMatGroup>, grid, dim3(kBlock), 0, s, chunks, slot_bytes,
                           K, ksw, W, J, j0 + q0, m, Y + (size_t)q0 * n12, n12, eoff);
    }
}

// Basis form, the whole sum in one pass over the stored slots: for source n
// (grid.y) s_n = sum_{i < K_n} h[n][i] r_i, K_n = min(kend, iter_n + 1), and
// with hx also x_n = sum_i hx[n][i] r_i (the in-band check's solution).
// Slots below ksw hold FP64, from ksw on FP32 packed at the slot base; slot i
// is chunks[i / kSlotChunk] + (i % kSlotChunk) slot_bytes, source n at
// element n n12.  Each output is written once, and the terms are added in
// slot order.
__global__ __launch_bounds__(kBlock) void k_basis_sum(char* const* __restrict__ chunks,
                                                      size_t slot_bytes, int kend, int ksw,
                                                      const double2* __restrict__ h,
                                                      const double2* __restrict__ hx, int maxk,
                                                      const SrcState* __restrict__ st,
                                                      double2* __restrict__ sacc,
                                                      double2* __restrict__ xc, int64_t n12) {
    typedef double __attribute__((ext_vector_type(2))) D2;
    typedef float __attribute__((ext_vector_type(2))) F2;
    const int n = blockIdx.y;
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= n12) return;
    const int kn = st[n].iter + 1;
    const int K = kend < kn ? kend : kn;
    const int k64 = ksw < K ? ksw : K;
    const int64_t off = (int64_t)n * n12 + e;
    const double2* hh = h + (int64_t)n * (maxk + 1);
    const double2* hc = hx ? hx + (int64_t)n * (maxk + 1) : nullptr;
    double re = 0.0, im = 0.0, xr = 0.0, xi = 0.0;
    auto term = [&](int i, double vr, double vi) {
        const double2 c = hh[i];
        re += c.x * vr - c.y * vi;
        im += c.x * vi + c.y * vr;
        if (hc) {
            const double2 u = hc[i];
            xr += u.x * vr - u.y * vi;
            xi += u.x * vi + u.y * vr;
        }
    };
#pragma unroll 4
    for (int i = 0; i < k64; ++i) {
        const OVL_GLOBAL char* slot =
            (const OVL_GLOBAL char*)chunks[i / kSlotChunk] + (size_t)(i % kSlotChunk) * slot_bytes;
        const D2 v = ((const OVL_GLOBAL D2*)slot)[off];
        term(i, v.x, v.y);
    }
#pragma unroll 4
    for (int i = k64; i < K; ++i) {
        const OVL_GLOBAL char* slot =
            (const OVL_GLOBAL char*)chunks[i / kSlotChunk] + (size_t)(i % kSlotChunk) * slot_bytes;
        const F2 v = ((const OVL_GLOBAL F2*)slot)[off];
        term(i, (double)v.x, (double)v.y);
    }
    sacc[off] = make_double2(re, im);
    if (hc) xc[off] = make_double2(xr, xi);
}
void launch_basis_sum(char* const* chunks, size_t slot_bytes, int kend, int ksw, const double2* h,
                      const double2* hx, int maxk, const SrcState* st, double2* sacc, double2* xc,
                      int64_t n12, int nsrc, hipStream_t s) {
    const dim3 grid((unsigned)((n12 + kBlock - 1) / kBlock), (unsigned)nsrc);
    hipLaunchKernelGGL(k_basis_sum, grid, dim3(kBlock), 0, s, chunks, slot_bytes, kend, ksw, h, hx,
                       maxk, st, sacc, xc, n12);
}

// t = b - (z x - H x) over one source; partial[blk] = (|t|^2, |b|^2) of the block
__global__ __launch_bounds__(kBlock) void k_true_res(const double2* __restrict__ b,
                                                     const double2* __restrict__ x,
                                                     const double2* __restrict__ hx, double2 z,
                                                     double2* __restrict__ partial, int64_t n12) {
    double tt = 0.0, bb = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < n12;
         e += (int64_t)gridDim.x * kBlock) {
        const double2 bv = b[e], xv = x[e], hv = hx[e];
        const double tr = bv.x - (z.x * xv.x - z.y * xv.y - hv.x);
        const double ti = bv.y - (z.x * xv.y + z.y * xv.x - hv.y);
        tt += tr * tr + ti * ti;
        bb += bv.x * bv.x + bv.y * bv.y;
    }
    __shared__ double sh[kBlock / 64];
    tt = block_sum<kBlock>(tt, sh);
    bb = block_sum<kBlock>(bb, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = make_double2(tt, bb);
}
void launch_true_res(const double2* b, const double2* x, const double2* hx, double2 z,
                     double2* partial, int nblk, int64_t n12, hipStream_t s) {
    hipLaunchKernelGGL(k_true_res, dim3(nblk), dim3(kBlock), 0, s, b, x, hx, z, partial, n12);
}
// The same for nsrc sources at once, source n with its own node zc[n]:
// partial[n][blk] = (|b_n - (zc_n x_n - H x_n)|^2, |b_n|^2) of the block
__global__ __launch_bounds__(kBlock) void k_true_res_multi(const double2* __restrict__ b,
                                                           const double2* __restrict__ x,
                                                           const double2* __restrict__ hx,
                                                           const double2* __restrict__ zc,
                                                           double2* __restrict__ partial,
                                                           int64_t n12) {
    const int n = blockIdx.y;
    const double2 z = zc[n];
    const size_t o = (size_t)n * n12;
    double tt = 0.0, bb = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < n12;
         e += (int64_t)gridDim.x * kBlock) {
        const double2 bv = b[o + e], xv = x[o + e], hv = hx[o + e];
        const double tr = bv.x - (z.x * xv.x - z.y * xv.y - hv.x);
        const double ti = bv.y - (z.x * xv.y + z.y * xv.x - hv.y);
        tt += tr * tr + ti * ti;
        bb += bv.x * bv.x + bv.y * bv.y;
    }
    __shared__ double sh[kBlock / 64];
    tt = block_sum<kBlock>(tt, sh);
    bb = block_sum<kBlock>(bb, sh);
    if (threadIdx.x == 0) partial[(size_t)n * gridDim.x + blockIdx.x] = make_double2(tt, bb);
}
void launch_true_res_multi(const double2* b, const double2* x, const double2* hx,
                           const double2* zc, double2* partial, int nblk, int64_t n12, int nsrc,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_true_res_multi, dim3(nblk, nsrc), dim3(kBlock), 0, s, b, x, hx, zc,
                       partial, n12);
}

// (M v) for M = gamma5 (1 -+ gamma_mu) (sg = -1: 1 - gamma, +1: 1 + gamma):
// (1 -+ gamma) v = [h ; -+ A^dag h], h = v_up -+ A v_dn; gamma5 flips the lower half.
__device__ __forceinline__ void proj_g5(int mu, double sg, const double2 (&v)[4][3],
                                        double2 (&o)[4][3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double2 p0 = v[0][c], p1 = v[1][c], p2 = v[2][c], p3 = v[3][c];
        double2 a0, a1;  // A (p2, p3)
        switch (mu) {
            case 0: a0 = make_double2(p3.y, -p3.x); a1 = make_double2(p2.y, -p2.x); break;
            case 1: a0 = make_double2(-p3.x, -p3.y); a1 = p2; break;
            case 2: a0 = make_double2(p2.y, -p2.x); a1 = make_double2(-p3.y, p3.x); break;
            default: a0 = p2; a1 = p3; break;
        }
        const double2 h0 = make_double2(p0.x + sg * a0.x, p0.y + sg * a0.y);
        const double2 h1 = make_double2(p1.x + sg * a1.x, p1.y + sg * a1.y);
        double2 b0, b1;  // A^dag (h0, h1)
        switch (mu) {
            case 0: b0 = make_double2(-h1.y, h1.x); b1 = make_double2(-h0.y, h0.x); break;
            case 1: b0 = h1; b1 = make_double2(-h0.x, -h0.y); break;
            case 2: b0 = make_double2(-h0.y, h0.x); b1 = make_double2(h1.y, -h1.x); break;
            default: b0 = h0; b1 = h1; break;
        }
        // lower half of (1 -+ gamma) v is sg * A^dag h; gamma5 negates it
        o[0][c] = h0;
        o[1][c] = h1;
        o[2][c] = make_double2(-sg * b0.x, -sg * b0.y);
        o[3][c] = make_double2(-sg * b1.x, -sg * b1.y);
    }
}

// One lane per link (x, mu).  For shifts j of the current chunk:
//   A_ab += c_j sum_s conj(X_j(x)_{s a}) (M Y_j(x+mu))_{s b},        M  = gamma5 (1 - gamma_mu)
//   B_cd += c_j sum_s conj(X_j(x+mu)_{s c}) (M' Y_j(x))_{s d},       M' = gamma5 (1 + gamma_mu)
// acc holds [A | B] (18 complex) per link across chunks.  With last != 0 the
// result -2 kappa ph (conj(A) + B^T) is written as the complex gradient G, or
// converted to the traceless hermitian force F = TH[(Z + Z^dag)/2], Z = i U G^dag.
__global__ __launch_bounds__(kBlock) void k_force(const double2* __restrict__ X,
                                                  const double2* __restrict__ Y,
                                                  const double2* __restrict__ c, int jn,
                                                  Geom g, const double2* __restrict__ Uint,
                                                  int bc0, int bc1, int bc2, int bc3,
                                                  double kappa, double2* __restrict__ acc,
                                                  int first, int last, int kind,
                                                  double2* __restrict__ out) {
    const int64_t V = g.V, Vt = g.Vt;
    const int64_t lk = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (lk >= 4 * V) return;
    const int mu = (int)(lk / V);
    const int64_t x = lk - (int64_t)mu * V;
    const int cm = (int)((x / g.stride[mu]) % g.L[mu]);
    const int64_t xp = (cm == g.L[mu] - 1) ? x - (int64_t)(g.L[mu] - 1) * g.stride[mu] : x + g.stride[mu];
    const int64_t n12 = 12 * Vt;
    double2 A[3][3], B[3][3];
    double2* ac = acc + (size_t)lk * 18;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            A[a][b] = first ? make_double2(0, 0) : ac[3 * a + b];
            B[a][b] = first ? make_double2(0, 0) : ac[9 + 3 * a + b];
        }
#pragma unroll 1
    for (int j = 0; j < jn; ++j) {
        const double2* Xj = X + (size_t)j * n12;
        const double2* Yj = Y + (size_t)j * n12;
        const double2 cj = c[j];
        double2 v[4][3], m[4][3], xs[4][3];
        // term 1: X(x), M Y(x+mu)
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                v[sp][cc] = Yj[tix64(3 * sp + cc, xp, 12)];
                xs[sp][cc] = Xj[tix64(3 * sp + cc, x, 12)];
            }
        proj_g5(mu, -1.0, v, m);
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                double2 t = make_double2(0, 0);
#pragma unroll
                for (int sp = 0; sp < 4; ++sp) {  // conj(X) * (M Y)
                    const double2 xa = xs[sp][a], mb = m[sp][b];
                    t.x += xa.x * mb.x + xa.y * mb.y;
                    t.y += xa.x * mb.y - xa.y * mb.x;
                }
                A[a][b] = cadd(A[a][b], cmul(cj, t));
            }
        // term 2: X(x+mu), M' Y(x)
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                v[sp][cc] = Yj[tix64(3 * sp + cc, x, 12)];
                xs[sp][cc] = Xj[tix64(3 * sp + cc, xp, 12)];
            }
        proj_g5(mu, 1.0, v, m);
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                double2 t = make_double2(0, 0);
#pragma unroll
                for (int sp = 0; sp < 4; ++sp) {
                    const double2 xa = xs[sp][a], mb = m[sp][b];
                    t.x += xa.x * mb.x + xa.y * mb.y;
                    t.y += xa.x * mb.y - xa.y * mb.x;
                }
                B[a][b] = cadd(B[a][b], cmul(cj, t));
            }
    }
    if (!last) {
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                ac[3 * a + b] = A[a][b];
                ac[9 + 3 * a + b] = B[a][b];
            }
        return;
    }
    const int bcm = mu == 0 ? bc0 : mu == 1 ? bc1 : mu == 2 ? bc2 : bc3;
    const double f = -2.0 * kappa * ((cm == g.L[mu] - 1) ? (double)bcm : 1.0);
    double2 G[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)  // G = f (conj(A) + B^T)
            G[a][b] = make_double2(f * (A[a][b].x + B[b][a].x), f * (-A[a][b].y + B[b][a].y));
    double2* o = out + ((size_t)mu * V + x) * 9;
    if (kind == 1) {
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) o[3 * a + b] = G[a][b];
        return;
    }
    // Z = i U G^dag ; F = (Z + Z^dag)/2 - tr/3.  The internal links carry the
    // boundary phase (+-1); multiplying by it again restores the caller's U.
    const double ph = (cm == g.L[mu] - 1) ? (double)bcm : 1.0;
    double2 Z[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            double2 t = make_double2(0, 0);
#pragma unroll
            for (int q = 0; q < 3; ++q) {  // U[a][q] conj(G[b][q])
                double2 u = Uint[(size_t)mu * 9 * Vt + tix64(3 * a + q, x, 9)];
                u.x *= ph;
                u.y *= ph;
                const double2 gg = G[b][q];
                t.x += u.x * gg.x + u.y * gg.y;
                t.y += u.y * gg.x - u.x * gg.y;
            }
            Z[a][b] = make_double2(-t.y, t.x);  // i t
        }
    double2 F[3][3];
    double tr = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            F[a][b] = make_double2(0.5 * (Z[a][b].x + Z[b][a].x), 0.5 * (Z[a][b].y - Z[b][a].y));
            if (a == b) tr += F[a][b].x;
        }
#pragma unroll
    for (int a = 0; a < 3; ++a) F[a][a].x -= tr / 3.0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) o[3 * a + b] = F[a][b];
}
void launch_force(const double2* X, const double2* Y, const double2* c, int jn, const Geom& g,
                  const double2* Uint, const int bc[4], double kappa, double2* acc, bool first,
                  bool last, int kind, double2* out, hipStream_t s) {
    dim3 grid((unsigned)((4 * g.V + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(k_force, grid, dim3(kBlock), 0, s, X, Y, c, jn, g, Uint, bc[0], bc[1],
                       bc[2], bc[3], kappa, acc, (int)first, (int)last, kind, out);
}

}  // namespace ovl
