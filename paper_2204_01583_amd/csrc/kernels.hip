// HIP kernels for gfx950: layout conversion, the hermitian Wilson stencil,
// deterministic Krylov reductions, shifted-system scalars and the shift
// sweeps.  Everything here is bandwidth bound (no dense contraction), so the
// kernels are written for coalesced structure-of-arrays access: one lane per
// site (stencil) or per complex component (vector kernels).
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "../../include/ovl.h"

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
// layout conversion
// ============================================================================
template <typename R>
__global__ __launch_bounds__(kBlock) void k_pack_spinor(const double2* __restrict__ ext,
                                                        C2<R>* __restrict__ in, int64_t V) {
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int n = blockIdx.y;
    if (s >= V) return;
    const double2* src = ext + ((int64_t)n * V + s) * 12;
    C2<R>* dst = in + (int64_t)n * 12 * V + s;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        double2 v = src[c];
        C2<R> w;
        w.x = (R)v.x;
        w.y = (R)v.y;
        dst[(int64_t)c * V] = w;
    }
}

__global__ __launch_bounds__(kBlock) void k_unpack_spinor(const double2* __restrict__ in,
                                                          double2* __restrict__ ext, int64_t V) {
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int n = blockIdx.y;
    if (s >= V) return;
    const double2* src = in + (int64_t)n * 12 * V + s;
    double2* dst = ext + ((int64_t)n * V + s) * 12;
#pragma unroll
    for (int c = 0; c < 12; ++c) dst[c] = src[(int64_t)c * V];
}

__global__ __launch_bounds__(kBlock) void k_unpack_dov(const double2* __restrict__ sin,
                                                       const double2* __restrict__ bext,
                                                       double2* __restrict__ ext, double a,
                                                       double bm, int64_t V) {
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int n = blockIdx.y;
    if (s >= V) return;
    const double2* src = sin + (int64_t)n * 12 * V + s;
    const double2* b = bext + ((int64_t)n * V + s) * 12;
    double2* dst = ext + ((int64_t)n * V + s) * 12;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        const double g5 = (c < 6) ? bm : -bm;  // gamma5 = diag(1,1,-1,-1) on spin
        double2 sv = src[(int64_t)c * V], bv = b[c], o;
        o.x = a * bv.x + g5 * sv.x;
        o.y = a * bv.y + g5 * sv.y;
        dst[c] = o;
    }
}

__global__ __launch_bounds__(kBlock) void k_pack_gauge(const double2* __restrict__ ext,
                                                       double2* __restrict__ U64,
                                                       float2* __restrict__ U32, Geom g,
                                                       int bc0, int bc1, int bc2, int bc3) {
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int mu = blockIdx.y;
    if (s >= g.V) return;
    const int coord = (int)((s / g.stride[mu]) % g.L[mu]);
    const int bcm = mu == 0 ? bc0 : mu == 1 ? bc1 : mu == 2 ? bc2 : bc3;
    const double sign = (coord == g.L[mu] - 1) ? (double)bcm : 1.0;
    const double2* src = ext + ((int64_t)mu * g.V + s) * 9;
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        double2 v = src[e];
        v.x *= sign;
        v.y *= sign;
        U64[((int64_t)mu * 9 + e) * g.V + s] = v;
        float2 f;
        f.x = (float)v.x;
        f.y = (float)v.y;
        U32[((int64_t)mu * 9 + e) * g.V + s] = f;
    }
}

__global__ __launch_bounds__(kBlock) void k_convert(const double2* __restrict__ a,
                                                    float2* __restrict__ b, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    double2 v = a[i];
    b[i] = make_float2((float)v.x, (float)v.y);
}

void launch_pack_spinor64(const double2* ext, double2* in, int64_t V, int n, hipStream_t s) {
    dim3 grid((unsigned)((V + kBlock - 1) / kBlock), n);
    hipLaunchKernelGGL(k_pack_spinor<double>, grid, dim3(kBlock), 0, s, ext, in, V);
}
void launch_pack_spinor32(const double2* ext, float2* in, int64_t V, int n, hipStream_t s) {
    dim3 grid((unsigned)((V + kBlock - 1) / kBlock), n);
    hipLaunchKernelGGL(k_pack_spinor<float>, grid, dim3(kBlock), 0, s, ext, in, V);
}
void launch_unpack_spinor64(const double2* in, double2* ext, int64_t V, int n, hipStream_t s) {
    dim3 grid((unsigned)((V + kBlock - 1) / kBlock), n);
    hipLaunchKernelGGL(k_unpack_spinor, grid, dim3(kBlock), 0, s, in, ext, V);
}
void launch_unpack_dov(const double2* s_int, const double2* b_ext, double2* out_ext, double a,
                       double bm, int64_t V, int n, hipStream_t s) {
    dim3 grid((unsigned)((V + kBlock - 1) / kBlock), n);
    hipLaunchKernelGGL(k_unpack_dov, grid, dim3(kBlock), 0, s, s_int, b_ext, out_ext, a, bm, V);
}
void launch_pack_gauge(const double2* ext, double2* U64, float2* U32, const Geom& g,
                       const int bc[4], hipStream_t s) {
    dim3 grid((unsigned)((g.V + kBlock - 1) / kBlock), 4);
    hipLaunchKernelGGL(k_pack_gauge, grid, dim3(kBlock), 0, s, ext, U64, U32, g, bc[0], bc[1],
                       bc[2], bc[3]);
}
void launch_convert_64_to_32(const double2* a, float2* b, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_convert, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       s, a, b, n);
}

// ============================================================================
// Wilson stencil
// ============================================================================
// Chiral basis: gamma_mu = [[0, A_mu], [A_mu^dag, 0]] with A_k = -i sigma_k,
// A_4 = 1.  For the lower half-spinor d = (psi_2, psi_3):
//   (1 -+ gamma_mu) psi = [ h ; -+ A^dag h ],  h = psi_up -+ A_mu d,
// so each hop moves a 2-spin x 3-colour half-spinor through the link.

// h = psi_up - A d (FWD) or psi_up + A d (backward), colour c
template <typename R, int MU, bool FWD>
__device__ __forceinline__ void project(cx<R> p0, cx<R> p1, cx<R> p2, cx<R> p3, cx<R>& h0,
                                        cx<R>& h1) {
    cx<R> a0, a1;  // A_mu (p2, p3)
    if constexpr (MU == 0) { a0 = tmi(p3); a1 = tmi(p2); }
    else if constexpr (MU == 1) { a0 = -p3; a1 = p2; }
    else if constexpr (MU == 2) { a0 = tmi(p2); a1 = ti(p3); }
    else { a0 = p2; a1 = p3; }
    if constexpr (FWD) { h0 = p0 - a0; h1 = p1 - a1; }
    else { h0 = p0 + a0; h1 = p1 + a1; }
}

// acc_up += u ; acc_dn -+= A_mu^dag u
template <typename R, int MU, bool FWD>
__device__ __forceinline__ void reconstruct(cx<R> (&acc)[4][3], const cx<R> (&u)[2][3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const cx<R> u0 = u[0][c], u1 = u[1][c];
        cx<R> b0, b1;  // A^dag (u0, u1)
        if constexpr (MU == 0) { b0 = ti(u1); b1 = ti(u0); }
        else if constexpr (MU == 1) { b0 = u1; b1 = -u0; }
        else if constexpr (MU == 2) { b0 = ti(u0); b1 = tmi(u1); }
        else { b0 = u0; b1 = u1; }
        acc[0][c] = acc[0][c] + u0;
        acc[1][c] = acc[1][c] + u1;
        if constexpr (FWD) { acc[2][c] = acc[2][c] - b0; acc[3][c] = acc[3][c] - b1; }
        else { acc[2][c] = acc[2][c] + b0; acc[3][c] = acc[3][c] + b1; }
    }
}

template <typename R, int MU, bool FWD>
__device__ __forceinline__ void hop(cx<R> (&acc)[4][3], const C2<R>* __restrict__ psi,
                                    const C2<R>* __restrict__ U, int64_t V, int64_t nb,
                                    int64_t lsite) {
    cx<R> h[2][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const cx<R> p0 = ld<R>(psi, (0 + c) * V + nb), p1 = ld<R>(psi, (3 + c) * V + nb);
        const cx<R> p2 = ld<R>(psi, (6 + c) * V + nb), p3 = ld<R>(psi, (9 + c) * V + nb);
        project<R, MU, FWD>(p0, p1, p2, p3, h[0][c], h[1][c]);
    }
    const C2<R>* Um = U + (int64_t)MU * 9 * V + lsite;
    cx<R> u[2][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        u[0][a] = mk<R>(0, 0);
        u[1][a] = mk<R>(0, 0);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            if constexpr (FWD) {  // U_mu(x) h
                const cx<R> l = ld<R>(Um, (int64_t)(3 * a + b) * V);
                fma_(u[0][a], l, h[0][b]);
                fma_(u[1][a], l, h[1][b]);
            } else {  // U_mu(x-mu)^dag h : element (a,b) = conj(U[b][a])
                const cx<R> l = ld<R>(Um, (int64_t)(3 * b + a) * V);
                fmac_(u[0][a], l, h[0][b]);
                fmac_(u[1][a], l, h[1][b]);
            }
        }
    }
    reconstruct<R, MU, FWD>(acc, u);
}

template <typename R, int MU>
__device__ __forceinline__ void hop_pair(cx<R> (&acc)[4][3], const C2<R>* __restrict__ psi,
                                         const C2<R>* __restrict__ U, const Geom& g,
                                         int64_t s, int coord) {
    const int64_t sd = g.stride[MU];
    const int L = g.L[MU];
    const int64_t fw = (coord == L - 1) ? s - (int64_t)(L - 1) * sd : s + sd;
    const int64_t bw = (coord == 0) ? s + (int64_t)(L - 1) * sd : s - sd;
    hop<R, MU, true>(acc, psi, U, g.V, fw, s);
    hop<R, MU, false>(acc, psi, U, g.V, bw, bw);
}

template <typename R, int MODE>
__global__ __launch_bounds__(kBlock) void k_wilson(const C2<R>* __restrict__ in,
                                                   C2<R>* __restrict__ out,
                                                   const C2<R>* __restrict__ U, Geom g, R kappa,
                                                   double zsr, double zsi,
                                                   const C2<R>* __restrict__ rdot,
                                                   double2* __restrict__ partial,
                                                   const SrcState* __restrict__ stt) {
    const int n = blockIdx.y;
    if constexpr (MODE == 1) {
        if (stt != nullptr && stt[n].done) return;
    }
    const int64_t V = g.V;
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool valid = s < V;
    double dre = 0.0, dim = 0.0;
    if (valid) {
        const C2<R>* psi = in + (int64_t)n * 12 * V;
        int64_t rem = s;
        const int x = (int)(rem % g.L[0]); rem /= g.L[0];
        const int y = (int)(rem % g.L[1]); rem /= g.L[1];
        const int z = (int)(rem % g.L[2]);
        const int t = (int)(rem / g.L[2]);
        cx<R> acc[4][3];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[a][c] = mk<R>(0, 0);
        hop_pair<R, 0>(acc, psi, U, g, s, x);
        hop_pair<R, 1>(acc, psi, U, g, s, y);
        hop_pair<R, 2>(acc, psi, U, g, s, z);
        hop_pair<R, 3>(acc, psi, U, g, s, t);
        C2<R>* o = out + (int64_t)n * 12 * V + s;
        const C2<R>* rd = (MODE == 1) ? rdot + (int64_t)n * 12 * V + s : nullptr;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int comp = 3 * a + c;
                const cx<R> p = ld<R>(psi + s, (int64_t)comp * V);
                // D psi = psi - kappa acc ; H = gamma5 D
                cx<R> hv = p - kappa * acc[a][c];
                if (a >= 2) hv = -hv;
                if constexpr (MODE == 0) {
                    stc<R>(o, (int64_t)comp * V, hv);
                } else {
                    // q = zs p - H p
                    const R zr = (R)zsr, zi = (R)zsi;
                    cx<R> q = mk<R>(zr * p.re - zi * p.im - hv.re, zr * p.im + zi * p.re - hv.im);
                    stc<R>(o, (int64_t)comp * V, q);
                    const cx<R> r = ld<R>(rd, (int64_t)comp * V);
                    // <r, q> = sum conj(r) q, accumulated in FP64
                    dre += (double)r.re * (double)q.re + (double)r.im * (double)q.im;
                    dim += (double)r.re * (double)q.im - (double)r.im * (double)q.re;
                }
            }
        }
    }
    if constexpr (MODE == 1) {
        __shared__ double sh[kBlock / 64];
        const double tr = block_sum<kBlock>(dre, sh);
        const double ti_ = block_sum<kBlock>(dim, sh);
        if (threadIdx.x == 0) partial[(int64_t)n * gridDim.x + blockIdx.x] = make_double2(tr, ti_);
    }
}

int wilson_blocks(const Geom& g) { return (int)((g.V + kBlock - 1) / kBlock); }

template <typename R>
void launch_wilson(int mode, const C2<R>* in, C2<R>* out, const C2<R>* U, const Geom& g,
                   double kappa, double2 zs, const C2<R>* r, double2* partial,
                   const SrcState* stt, int nrhs, hipStream_t s) {
    dim3 grid(wilson_blocks(g), nrhs);
    if (mode == 0)
        hipLaunchKernelGGL((k_wilson<R, 0>), grid, dim3(kBlock), 0, s, in, out, U, g, (R)kappa,
                           zs.x, zs.y, r, partial, stt);
    else
        hipLaunchKernelGGL((k_wilson<R, 1>), grid, dim3(kBlock), 0, s, in, out, U, g, (R)kappa,
                           zs.x, zs.y, r, partial, stt);
}
template void launch_wilson<double>(int, const double2*, double2*, const double2*, const Geom&,
                                    double, double2, const double2*, double2*, const SrcState*,
                                    int, hipStream_t);
template void launch_wilson<float>(int, const float2*, float2*, const float2*, const Geom&,
                                   double, double2, const float2*, double2*, const SrcState*,
                                   int, hipStream_t);

// ============================================================================
// Krylov scalars
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

// One block per source.  alpha_k = ||r_k||^2 / <r_k, A_s p_k>; for every active
// shift j (Delta_j = z_j - z_s):
//   pi_{k+1} = (1 + alpha_k Delta_j) pi_k + (alpha_k beta_{k-1}/alpha_{k-1}) (pi_k - pi_{k-1})
//   alpha^j  = alpha_k pi_k / pi_{k+1}
__global__ __launch_bounds__(kBlock) void k_alpha(SrcState* __restrict__ st,
                                                  const double2* __restrict__ partial, int nblk,
                                                  const double2* __restrict__ dz,
                                                  const double2* __restrict__ pi,
                                                  const double2* __restrict__ pi_prev,
                                                  double2* __restrict__ pi_next,
                                                  double2* __restrict__ aj,
                                                  const int* __restrict__ active, int J) {
    const int n = blockIdx.x;
    SrcState& S = st[n];
    if (S.done) {
        if (threadIdx.x == 0) S.nlist = 0;
        return;
    }
    __shared__ double sh[kBlock / 64];
    double re = 0.0, im = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kBlock) {
        const double2 v = partial[(int64_t)n * nblk + b];
        re += v.x;
        im += v.y;
    }
    re = block_sum<kBlock>(re, sh);
    im = block_sum<kBlock>(im, sh);
    const double2 rq = make_double2(re, im);
    const bool bad = !finite2(rq);
    const bool brk = cabs2(rq) <= 1e-300 * (S.rr > 0 ? S.rr : 1.0);
    const double2 alpha = (bad || brk) ? make_double2(0, 0) : cdiv(make_double2(S.rr, 0.0), rq);
    if (!bad && !brk) {
        const double2 c1 = cdiv(cmul(alpha, S.beta_prev), S.alpha_prev);
        for (int j = threadIdx.x; j < J; j += kBlock) {
            const int64_t o = (int64_t)n * J + j;
            if (!active[o]) continue;
            const double2 p = pi[o], pp = pi_prev[o];
            const double2 one_ad = make_double2(1.0 + (alpha.x * dz[j].x - alpha.y * dz[j].y),
                                                alpha.x * dz[j].y + alpha.y * dz[j].x);
            const double2 pn = cadd(cmul(one_ad, p), cmul(c1, csub(p, pp)));
            pi_next[o] = pn;
            aj[o] = cdiv(cmul(alpha, p), pn);
        }
    }
    if (threadIdx.x == 0) {
        S.alpha = alpha;
        if (bad || brk) {
            S.status = bad ? OVL_E_NONFINITE : OVL_E_BREAKDOWN;
            S.done = 1;
            S.nlist = 0;
        }
    }
}

void launch_alpha(SrcState* st, const double2* partial, int nblk, const double2* dz,
                  const double2* pi, const double2* pi_prev, double2* pi_next, double2* aj,
                  const int* active, int J, int nsrc, hipStream_t s) {
    hipLaunchKernelGGL(k_alpha, dim3(nsrc), dim3(kBlock), 0, s, st, partial, nblk, dz, pi,
                       pi_prev, pi_next, aj, active, J);
}

// One block per source.  beta_k = (alpha_k / conj(alpha_k)) ||r_{k+1}||^2 / ||r_k||^2,
// beta^j = (pi_k / pi_{k+1})^2 beta_k; shift j's residual estimate is
// ||r_{k+1}|| / |pi_{k+1}^j|.  Shifts active at the start of this iteration
// enter the sweep list; those now below tol*||b|| are deactivated afterwards.
__global__ __launch_bounds__(kBlock) void k_beta(BetaArgs a) {
    const int n = blockIdx.x;
    SrcState& S = a.st[n];
    if (S.done) return;
    __shared__ double sh[kBlock / 64];
    __shared__ int wcount[kBlock / 64];
    __shared__ int base;
    double v = 0.0;
    for (int b = threadIdx.x; b < a.nblk; b += kBlock) v += a.partial[(int64_t)n * a.nblk + b];
    const double rrn = block_sum<kBlock>(v, sh);
    const double2 al = S.alpha;
    // alpha / conj(alpha) has unit modulus
    const double2 ph = cdiv(al, make_double2(al.x, -al.y));
    const double ratio = rrn / S.rr;
    const double2 beta = make_double2(ph.x * ratio, ph.y * ratio);
    const double rn = sqrt(rrn), bn = sqrt(S.bb);
    const int k = S.iter;
    if (threadIdx.x == 0) base = 0;
    __syncthreads();
    double mres = 0.0;
    int nstay = 0;
    for (int j0 = 0; j0 < a.J; j0 += kBlock) {
        const int j = j0 + threadIdx.x;
        const int64_t o = (int64_t)n * a.J + j;
        const bool act = (j < a.J) && a.active[o];
        double2 bj = make_double2(0, 0), ipi = make_double2(0, 0), coef = make_double2(0, 0);
        if (act) {
            const double2 pn = a.pi_next[o], p = a.pi[o];
            const double2 rt = cdiv(p, pn);
            bj = cmul(cmul(rt, rt), beta);
            ipi = cdiv(make_double2(1.0, 0.0), pn);
            const double2 aj = a.aj[o];
            coef = (a.c != nullptr) ? cmul(a.c[j], aj) : aj;
            const double res = rn / sqrt(cabs2(pn)) / bn;
            mres = fmax(mres, res);
            a.pi_prev[o] = p;
            a.pi[o] = pn;
            if (res <= a.tol) a.active[o] = 0; else ++nstay;
        }
        if (a.h_a != nullptr && j < a.J) {
            const int64_t ho = ((int64_t)n * (a.maxk + 1) + k) * a.J + j;
            a.h_a[ho] = act ? a.aj[o] : make_double2(0, 0);
            a.h_b[ho] = bj;
            a.h_pi[ho + a.J] = act ? a.pi_next[o] : a.pi[o];
        }
        // compact the active shifts into the sweep list (order of j kept)
        const unsigned long long m = __ballot(act);
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        const int before = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) wcount[w] = __popcll(m);
        __syncthreads();
        int off = base;
        for (int i = 0; i < w; ++i) off += wcount[i];
        if (act) {
            const int64_t lo = (int64_t)n * a.J + off + before;
            a.lst_j[lo] = j;
            a.lst_a[lo] = coef;
            a.lst_ipi[lo] = ipi;
            a.lst_b[lo] = bj;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int tot = 0;
            for (int i = 0; i < kBlock / 64; ++i) tot += wcount[i];
            base += tot;
        }
        __syncthreads();
    }
    const double mall = block_max<kBlock>(mres, sh);
    const double nall = block_sum<kBlock>((double)nstay, sh);
    if (threadIdx.x == 0) {
        const int tot = (int)(nall + 0.5);
        S.nlist = base;
        S.nact = tot;
        S.maxres = mall;
        S.rr = rrn;
        S.alpha_prev = al;
        S.beta_prev = beta;
        S.iter = k + 1;
        if (tot == 0) S.done = 1;
        if (!isfinite(rrn)) {
            S.status = OVL_E_NONFINITE;
            S.done = 1;
        }
    }
}

void launch_beta(const BetaArgs& a, int nsrc, hipStream_t s) {
    hipLaunchKernelGGL(k_beta, dim3(nsrc), dim3(kBlock), 0, s, a);
}


// ============================================================================
// vector kernels: one lane per complex component, grid.y = source
// ============================================================================
int elem_blocks(int64_t n12) { return (int)((n12 + kBlock - 1) / kBlock); }

template <typename R>
__global__ __launch_bounds__(kBlock) void k_update_r(const C2<R>* __restrict__ rin,
                                                     C2<R>* __restrict__ rout,
                                                     const C2<R>* __restrict__ q,
                                                     const SrcState* __restrict__ st,
                                                     double* __restrict__ partial, int64_t n12,
                                                     int64_t sin_, int64_t sout) {
    const int n = blockIdx.y;
    if (st[n].done) return;
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double acc = 0.0;
    if (e < n12) {
        const double2 al = st[n].alpha;
        const cx<R> r = ld<R>(rin + n * sin_, e), qq = ld<R>(q + n * n12, e);
        const R ar = (R)al.x, ai = (R)al.y;
        cx<R> rn = mk<R>(r.re - (ar * qq.re - ai * qq.im), r.im - (ar * qq.im + ai * qq.re));
        stc<R>(rout + n * sout, e, rn);
        acc = (double)rn.re * (double)rn.re + (double)rn.im * (double)rn.im;
    }
    __shared__ double sh[kBlock / 64];
    const double t = block_sum<kBlock>(acc, sh);
    if (threadIdx.x == 0) partial[(int64_t)n * gridDim.x + blockIdx.x] = t;
}

template <typename R>
void launch_update_r(const C2<R>* rin, C2<R>* rout, const C2<R>* q, const SrcState* st,
                     double* partial, int64_t n12, int64_t src_stride_in,
                     int64_t src_stride_out, int nsrc, hipStream_t s) {
    dim3 grid(elem_blocks(n12), nsrc);
    hipLaunchKernelGGL(k_update_r<R>, grid, dim3(kBlock), 0, s, rin, rout, q, st, partial, n12,
                       src_stride_in, src_stride_out);
}
template void launch_update_r<double>(const double2*, double2*, const double2*, const SrcState*,
                                      double*, int64_t, int64_t, int64_t, int, hipStream_t);
template void launch_update_r<float>(const float2*, float2*, const float2*, const SrcState*,
                                     double*, int64_t, int64_t, int64_t, int, hipStream_t);

// The fused sweep: for every shift in this iteration's list (uniform per
// source, read through the scalar cache)
//   s += (c_j alpha^j) p_j ;  p_j <- r / pi_{k+1}^j + beta^j p_j
// and the seed direction p <- r + beta p, in one pass over the components.
// In the first iteration p_j = b for every j, read from b0 instead.
template <typename R, bool REF>
__global__ __launch_bounds__(kBlock) void k_sweep(const C2<R>* __restrict__ r,
                                                  C2<R>* __restrict__ p, C2<R>* __restrict__ pj,
                                                  double2* __restrict__ acc_out,
                                                  const double2* __restrict__ b0,
                                                  const SrcState* __restrict__ st,
                                                  const int* __restrict__ lst_j,
                                                  const double2* __restrict__ lst_a,
                                                  const double2* __restrict__ lst_ipi,
                                                  const double2* __restrict__ lst_b, int J,
                                                  int64_t n12, int first) {
    const int n = blockIdx.y;
    const int nl = st[n].nlist;
    if (nl == 0) return;
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= n12) return;
    const cx<R> rv = ld<R>(r + n * n12, e);
    const double2 beta = st[n].beta_prev;
    const int64_t lb = (int64_t)n * J;
    const cx<R> bfirst = first ? mk<R>((R)b0[n * n12 + e].x, (R)b0[n * n12 + e].y) : mk<R>(0, 0);
    double sre = 0.0, sim = 0.0;
    for (int l = 0; l < nl; ++l) {
        const int j = lst_j[lb + l];
        const double2 ca = lst_a[lb + l], ip = lst_ipi[lb + l], bj = lst_b[lb + l];
        C2<R>* pp = pj + ((int64_t)n * J + j) * n12;
        const cx<R> pv = first ? bfirst : ld<R>(pp, e);
        if constexpr (REF) {
            // x_j += alpha^j p_j  (x_j kept in FP64)
            double2* xp = acc_out + ((int64_t)n * J + j) * n12;
            double2 x = xp[e];
            x.x += ca.x * (double)pv.re - ca.y * (double)pv.im;
            x.y += ca.x * (double)pv.im + ca.y * (double)pv.re;
            xp[e] = x;
        } else {
            sre += ca.x * (double)pv.re - ca.y * (double)pv.im;
            sim += ca.x * (double)pv.im + ca.y * (double)pv.re;
        }
        const R ipr = (R)ip.x, ipi = (R)ip.y, br = (R)bj.x, bi = (R)bj.y;
        cx<R> np = mk<R>(rv.re * ipr - rv.im * ipi + br * pv.re - bi * pv.im,
                         rv.re * ipi + rv.im * ipr + br * pv.im + bi * pv.re);
        stc<R>(pp, e, np);
    }
    if constexpr (!REF) {
        double2 sv = acc_out[n * n12 + e];
        sv.x += sre;
        sv.y += sim;
        acc_out[n * n12 + e] = sv;
    }
    const cx<R> po = ld<R>(p + n * n12, e);
    const R br = (R)beta.x, bi = (R)beta.y;
    stc<R>(p + n * n12, e, mk<R>(rv.re + br * po.re - bi * po.im, rv.im + br * po.im + bi * po.re));
}

template <typename R>
void launch_sweep_fused(const C2<R>* r, C2<R>* p, C2<R>* pj, double2* sacc, const double2* b0,
                        const SrcState* st, const int* lst_j, const double2* lst_a,
                        const double2* lst_ipi, const double2* lst_b, int J, int64_t n12,
                        int nsrc, bool first, hipStream_t s) {
    dim3 grid(elem_blocks(n12), nsrc);
    hipLaunchKernelGGL((k_sweep<R, false>), grid, dim3(kBlock), 0, s, r, p, pj, sacc, b0, st,
                       lst_j, lst_a, lst_ipi, lst_b, J, n12, (int)first);
}
template <typename R>
void launch_sweep_ref(const C2<R>* r, C2<R>* p, C2<R>* pj, double2* xj, const double2* b0,
                      const SrcState* st, const int* lst_j, const double2* lst_a,
                      const double2* lst_ipi, const double2* lst_b, int J, int64_t n12,
                      int nsrc, bool first, hipStream_t s) {
    dim3 grid(elem_blocks(n12), nsrc);
    hipLaunchKernelGGL((k_sweep<R, true>), grid, dim3(kBlock), 0, s, r, p, pj, xj, b0, st,
                       lst_j, lst_a, lst_ipi, lst_b, J, n12, (int)first);
}
#define OVL_INST_SWEEP(R)                                                                      \
    template void launch_sweep_fused<R>(const C2<R>*, C2<R>*, C2<R>*, double2*, const double2*, \
                                        const SrcState*, const int*, const double2*,            \
                                        const double2*, const double2*, int, int64_t, int,      \
                                        bool, hipStream_t);                                     \
    template void launch_sweep_ref<R>(const C2<R>*, C2<R>*, C2<R>*, double2*, const double2*,   \
                                      const SrcState*, const int*, const double2*,              \
                                      const double2*, const double2*, int, int64_t, int, bool,  \
                                      hipStream_t);
OVL_INST_SWEEP(double)
OVL_INST_SWEEP(float)

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
    dim3 grid(elem_blocks(n12), nsrc);
    hipLaunchKernelGGL(k_sum_ref, grid, dim3(kBlock), 0, s, xj, c, sacc, J, n12);
}

// p = r + beta p (basis forms; the sweep kernel does this in the sweep forms)
template <typename R>
__global__ __launch_bounds__(kBlock) void k_update_p(const C2<R>* __restrict__ r,
                                                     C2<R>* __restrict__ p,
                                                     const SrcState* __restrict__ st,
                                                     int64_t n12, int64_t sr) {
    const int n = blockIdx.y;
    if (st[n].nlist == 0) return;
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= n12) return;
    const double2 beta = st[n].beta_prev;
    const cx<R> rv = ld<R>(r + n * sr, e), po = ld<R>(p + n * n12, e);
    const R br = (R)beta.x, bi = (R)beta.y;
    stc<R>(p + n * n12, e, mk<R>(rv.re + br * po.re - bi * po.im, rv.im + br * po.im + bi * po.re));
}
template <typename R>
void launch_update_p(const C2<R>* r, C2<R>* p, const SrcState* st, int64_t n12,
                     int64_t src_stride_r, int nsrc, hipStream_t s) {
    dim3 grid(elem_blocks(n12), nsrc);
    hipLaunchKernelGGL(k_update_p<R>, grid, dim3(kBlock), 0, s, r, p, st, n12, src_stride_r);
}
template void launch_update_p<double>(const double2*, double2*, const SrcState*, int64_t, int64_t,
                                      int, hipStream_t);
template void launch_update_p<float>(const float2*, float2*, const SrcState*, int64_t, int64_t,
                                     int, hipStream_t);

// ============================================================================
// basis forms
// ============================================================================
// x_j = sum_i u_i^j r_i with u_i^j = P_i^j / pi_i^j,
// P_i^j = alpha_i^j + beta_i^j P_{i+1}^j (alpha^j recorded as 0 once shift j
// stopped, which freezes x_j exactly as the sweep does).  One thread per
// shift runs the backward recursion; W[src][i][j] = c_j u_i^j.
__global__ __launch_bounds__(kBlock) void k_coef(const double2* __restrict__ h_a,
                                                 const double2* __restrict__ h_b,
                                                 const double2* __restrict__ h_pi,
                                                 const double2* __restrict__ c,
                                                 const SrcState* __restrict__ st,
                                                 double2* __restrict__ W, int J, int maxk) {
    const int n = blockIdx.y;
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= J) return;
    const int K = st[n].iter;
    const int64_t hb = (int64_t)n * (maxk + 1) * J;
    double2 P = make_double2(0, 0);
    for (int i = K - 1; i >= 0; --i) {
        const double2 a = h_a[hb + (int64_t)i * J + j], b = h_b[hb + (int64_t)i * J + j];
        P = cadd(a, cmul(b, P));
        const double2 pi = (i == 0) ? make_double2(1, 0) : h_pi[hb + (int64_t)i * J + j];
        W[hb + (int64_t)i * J + j] = cmul(c[j], cdiv(P, pi));
    }
}
// h[src][i] = sum_j W[src][i][j] (fixed order)
__global__ __launch_bounds__(kBlock) void k_hsum(const double2* __restrict__ W,
                                                 const SrcState* __restrict__ st,
                                                 double2* __restrict__ h, int J, int maxk) {
    const int n = blockIdx.y;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i > maxk) return;
    const int K = st[n].iter;
    double2 t = make_double2(0, 0);
    if (i < K) {
        const double2* w = W + ((int64_t)n * (maxk + 1) + i) * J;
        for (int j = 0; j < J; ++j) t = cadd(t, w[j]);
    }
    h[(int64_t)n * (maxk + 1) + i] = t;
}
void launch_basis_coef(const double2* h_a, const double2* h_b, const double2* h_pi,
                       const double2* c, const SrcState* st, double2* W, double2* h, int J,
                       int maxk, int nsrc, hipStream_t s) {
    hipLaunchKernelGGL(k_coef, dim3((J + kBlock - 1) / kBlock, nsrc), dim3(kBlock), 0, s, h_a,
                       h_b, h_pi, c, st, W, J, maxk);
    hipLaunchKernelGGL(k_hsum, dim3((maxk + 1 + kBlock - 1) / kBlock, nsrc), dim3(kBlock), 0, s,
                       W, st, h, J, maxk);
}

// s[src] = (s[src] +) sum_l h[src][g0 + l] * slot_l[src] over local slots
// l0 <= l < l1 of one contiguous chunk whose slot 0 is global slot g0;
// slots at or beyond K_src + 1 are skipped (they were never written).
template <typename R>
__global__ __launch_bounds__(kBlock) void k_gemv(const C2<R>* __restrict__ slots,
                                                 int64_t slot_stride, int64_t src_stride,
                                                 const double2* __restrict__ h, int maxk,
                                                 const SrcState* __restrict__ st, int g0, int l0,
                                                 int l1, double2* __restrict__ sacc,
                                                 int accumulate, int64_t n12) {
    const int n = blockIdx.y;
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= n12) return;
    const int K = st[n].iter + 1;  // r_0 .. r_K exist; h is zero beyond K-1
    const int lend = (K - g0) < l1 ? (K - g0) : l1;
    double re = 0.0, im = 0.0;
    const double2* hh = h + (int64_t)n * (maxk + 1) + g0;
    const C2<R>* base = slots + n * src_stride + e;
    for (int l = l0; l < lend; ++l) {
        const double2 c = hh[l];
        const C2<R> v = base[(int64_t)l * slot_stride];
        re += c.x * (double)v.x - c.y * (double)v.y;
        im += c.x * (double)v.y + c.y * (double)v.x;
    }
    double2 o = make_double2(re, im);
    if (accumulate) {
        const double2 prev = sacc[n * n12 + e];
        o.x += prev.x;
        o.y += prev.y;
    }
    sacc[n * n12 + e] = o;
}
template <typename R>
void launch_basis_gemv(const void* slots, int64_t slot_stride, int64_t src_stride,
                       const double2* h, int maxk, const SrcState* st, int g0, int l0, int l1,
                       double2* sacc, bool accumulate, int64_t n12, int nsrc, hipStream_t s) {
    dim3 grid(elem_blocks(n12), nsrc);
    hipLaunchKernelGGL(k_gemv<R>, grid, dim3(kBlock), 0, s, (const C2<R>*)slots, slot_stride,
                       src_stride, h, maxk, st, g0, l0, l1, sacc, (int)accumulate, n12);
}
template void launch_basis_gemv<double>(const void*, int64_t, int64_t, const double2*, int,
                                        const SrcState*, int, int, int, double2*, bool, int64_t,
                                        int, hipStream_t);
template void launch_basis_gemv<float>(const void*, int64_t, int64_t, const double2*, int,
                                       const SrcState*, int, int, int, double2*, bool, int64_t,
                                       int, hipStream_t);

// ============================================================================
// solver initialisation
// ============================================================================
// partial[src][blk] = ||b||^2 over the block
__global__ __launch_bounds__(kBlock) void k_norm2(const double2* __restrict__ b,
                                                  double* __restrict__ partial, int64_t n12) {
    const int n = blockIdx.y;
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double acc = 0.0;
    if (e < n12) {
        const double2 v = b[n * n12 + e];
        acc = v.x * v.x + v.y * v.y;
    }
    __shared__ double sh[kBlock / 64];
    const double t = block_sum<kBlock>(acc, sh);
    if (threadIdx.x == 0) partial[(int64_t)n * gridDim.x + blockIdx.x] = t;
}
// r = p = b, pi = pi_prev = 1, every shift active, alpha_{-1} = 1, beta_{-1} = 0
__global__ __launch_bounds__(kBlock) void k_init_state(SrcState* __restrict__ st,
                                                       const double* __restrict__ partial,
                                                       int nblk, double2* __restrict__ pi,
                                                       double2* __restrict__ pi_prev,
                                                       int* __restrict__ active, int J,
                                                       double2* __restrict__ h_pi, int maxk) {
    const int n = blockIdx.x;
    __shared__ double sh[kBlock / 64];
    double v = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kBlock) v += partial[(int64_t)n * nblk + b];
    const double bb = block_sum<kBlock>(v, sh);
    const bool zero = !(bb > 0.0);
    for (int j = threadIdx.x; j < J; j += kBlock) {
        const int64_t o = (int64_t)n * J + j;
        pi[o] = make_double2(1, 0);
        pi_prev[o] = make_double2(1, 0);
        active[o] = zero ? 0 : 1;
        if (h_pi != nullptr) h_pi[(int64_t)n * (maxk + 1) * J + j] = make_double2(1, 0);
    }
    if (threadIdx.x == 0) {
        SrcState S;
        S.rr = bb;
        S.bb = bb;
        S.alpha = make_double2(0, 0);
        S.alpha_prev = make_double2(1, 0);
        S.beta_prev = make_double2(0, 0);
        S.maxres = zero ? 0.0 : 1.0;
        S.iter = 0;
        S.nact = zero ? 0 : J;
        S.done = (zero || !isfinite(bb)) ? 1 : 0;
        S.status = isfinite(bb) ? 0 : OVL_E_NONFINITE;
        S.nlist = 0;
        S.pad = 0;
        st[n] = S;
    }
}
void launch_init_state(SrcState* st, const double2* b, double* partial, int64_t n12, double2* pi,
                       double2* pi_prev, int* active, int J, double2* h_pi, int maxk, int nsrc,
                       hipStream_t s) {
    const int nb = elem_blocks(n12);
    hipLaunchKernelGGL(k_norm2, dim3(nb, nsrc), dim3(kBlock), 0, s, b, partial, n12);
    hipLaunchKernelGGL(k_init_state, dim3(nsrc), dim3(kBlock), 0, s, st, partial, nb, pi, pi_prev,
                       active, J, h_pi, maxk);
}

}  // namespace ovl
