// Scalar parts of the seed iteration shared by the two-kernel iteration
// (kernels.hip) and the fused one-kernel iteration (stencil.hip).
#pragma once
#include "device_util.h"

namespace ovl {

// Seed scalars of iteration k from the stencil's per-block partials:
//   alpha_k = ||r_k||^2 / <r_k, q_k>,   q_k = A_s p_k,
//   ||r_{k+1}||^2 = ||r_k - alpha q||^2 = |alpha|^2 ||q||^2 - ||r_k||^2
//     (alpha <r,q> = ||r||^2 is real), clamped at 0,
//   beta_k = (alpha / conj(alpha)) ||r_{k+1}||^2 / ||r_k||^2.
// The next stencil pass measures ||r_{k+1}||^2 from the vector itself, so
// alpha_{k+1} is always taken from the true residual.
struct SeedScalars {
    double2 alpha, beta;
    double rr, rrn;
    int status;
};
__device__ __forceinline__ SeedScalars seed_scalars_from(const double4* pw, int nsb, double* shm) {
    double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    for (int b = threadIdx.x; b < nsb; b += kBlock) {
        const double4 v = pw[b];
        a0 += v.x;
        a1 += v.y;
        a2 += v.z;
        a3 += v.w;
    }
    double a[4] = {a0, a1, a2, a3};
    block_sum4<kBlock>(a, shm);  // shm: 4 kBlock/64 values
    a0 = a[0];
    a1 = a[1];
    a2 = a[2];
    a3 = a[3];
    SeedScalars r;
    const double2 rq = make_double2(a0, a1);
    r.rr = a3;
    r.status = 0;
    if (!finite2(rq) || !isfinite(a2) || !isfinite(a3)) r.status = OVL_E_NONFINITE;
    else if (cabs2(rq) <= 1e-300 * a3) r.status = OVL_E_BREAKDOWN;
    if (r.status) {
        r.alpha = r.beta = make_double2(0, 0);
        r.rrn = 0;
        return r;
    }
    r.alpha = cdiv(make_double2(a3, 0.0), rq);
    r.rrn = fmax(cabs2(r.alpha) * a2 - a3, 0.0);
    const double2 ph = cdiv(r.alpha, make_double2(r.alpha.x, -r.alpha.y));
    const double ratio = r.rrn / a3;
    r.beta = make_double2(ph.x * ratio, ph.y * ratio);
    return r;
}

// Per-shift scalars of iteration k for shift j (active at the start of k):
//   pi_{k+1} = (1 + alpha Dz_j) pi_k + (alpha beta_{k-1}/alpha_{k-1}) (pi_k - pi_{k-1})
//   alpha^j = alpha pi_k / pi_{k+1},  beta^j = (pi_k / pi_{k+1})^2 beta,
//   shifted residual estimate ||r_{k+1}|| / |pi_{k+1}| / ||b||.
struct ShiftScalars {
    double2 pn, aj, bj, ipi;
    double res;
};
__device__ __forceinline__ ShiftScalars shift_scalars(const ShiftDev& sh, size_t o, int j, int k,
                                                      const SeedScalars& sc, double2 c1, double bb) {
    const size_t stride3 = (size_t)sh.nsrc * sh.J;
    const double2 p = sh.pi[(size_t)(k % 3) * stride3 + o];
    const double2 pp = sh.pi[(size_t)((k + 2) % 3) * stride3 + o];
    const double2 dz = sh.dz[j];
    const double2 al = sc.alpha;
    const double2 one_ad = make_double2(1.0 + (al.x * dz.x - al.y * dz.y), al.x * dz.y + al.y * dz.x);
    ShiftScalars t;
    t.pn = cadd(cmul(one_ad, p), cmul(c1, csub(p, pp)));
    const double2 rt = cdiv(p, t.pn);
    t.aj = cmul(al, rt);
    t.bj = cmul(cmul(rt, rt), sc.beta);
    t.ipi = cdiv(make_double2(1.0, 0.0), t.pn);
    t.res = sqrt(sc.rrn / cabs2(t.pn) / bb);
    return t;
}

// The shift update of iteration i for the 256-shift slice `slice` of source
// n (one lane per shift), given the seed scalars sc of iteration i and the
// previous ones in S: pi_{i+1}^j, alpha^j, beta^j, the residual estimate and
// deactivation, the slice's active count into cnt[(i+1)&1] and its largest
// estimate, and the basis-form history of row i.  The same arithmetic as the
// scalar part of the two-kernel update.
__device__ __forceinline__ void advance_shift_slice(const ShiftDev& sh, const SrcState& S, int n,
                                                    int slice, int i, const SeedScalars& sc,
                                                    double* shm) {
    const double2 c1 = cdiv(cmul(sc.alpha, S.beta[(i + 1) & 1]), S.alpha[(i + 1) & 1]);
    const size_t stride3 = (size_t)sh.nsrc * sh.J;
    int* cnt_next = sh.cnt + ((size_t)((i + 1) & 1) * sh.nsrc + n) * kMaxSlices;
    const int j = slice * kBlock + threadIdx.x;
    const size_t o = (size_t)n * sh.J + j;
    const bool act = j < sh.J && sh.active[(size_t)(i & 1) * stride3 + o] != 0;
    ShiftScalars t{};
    if (act) t = shift_scalars(sh, o, j, i, sc, c1, S.bb);
    int stay = 0;
    if (j < sh.J) {
        if (act) {
            sh.pi[(size_t)((i + 1) % 3) * stride3 + o] = t.pn;
            sh.aj[o] = t.aj;
            sh.res[o] = t.res;
            stay = (t.res > sh.tol && isfinite(t.res)) ? 1 : 0;
        }
        sh.active[(size_t)((i + 1) & 1) * stride3 + o] = stay;
        if (sh.h_a != nullptr) {
            const size_t ho = ((size_t)n * (sh.maxk + 1) + i) * sh.J + j;
            sh.h_a[ho] = act ? t.aj : make_double2(0, 0);
            sh.h_b[ho] = act ? t.bj : make_double2(0, 0);
            sh.h_pi[ho + sh.J] = act ? t.pn : make_double2(1, 0);
        }
    }
    double tot = (double)stay, mx = act ? t.res : 0.0;  // (shm: 2 kBlock/64 values)
    block_sum_max<kBlock>(tot, mx, shm);
    if (threadIdx.x == 0) {
        cnt_next[slice] = (int)(tot + 0.5);
        sh.mres[(size_t)n * kMaxSlices + slice] = mx;
    }
}

// Liveness in the fused iteration: kernel k (which forms r_k and q_k and
// advances the shifts by iteration k-1) runs source n while it has no error,
// k <= maxk and some shift was active at the start of iteration k-1 (counts
// written by kernel k-1; the initial counts sit in both parities).
__device__ __forceinline__ bool src_live_fused(const SrcState& S, const ShiftDev& sh, int n, int k) {
    if (S.status != 0 || k > sh.maxk) return false;
    const int* c = sh.cnt + ((size_t)((k - 1) & 1) * sh.nsrc + n) * kMaxSlices;
    int t = 0;
    for (int q = 0; q < sh.nslices; ++q) t += c[q];
    return t > 0;
}

}  // namespace ovl
