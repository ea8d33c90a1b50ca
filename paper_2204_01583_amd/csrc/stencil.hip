// The hermitian Wilson stencil H_W = gamma5 D_W(-m0) for gfx950 (HIP).
// Bandwidth bound (at most ~3.6 flop per algorithmic byte in FP64), so no
// matrix cores: one or two lanes per site (and rhs), tiled spinors and links
// (64-site tiles, components contiguous within a tile), 32-bit offsets from
// uniform bases, an XCD-aware block order, optional LDS tiles of the block's
// sites or links, and 28 register/latency/locality trade-off variants chosen
// by the autotuner.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "device_util.h"
#include "kernels.h"
#include "seed_iter.h"

namespace ovl {

// ============================================================================
// Wilson stencil
// ============================================================================
// Chiral basis: gamma_mu = [[0, A_mu], [A_mu^dag, 0]] with A_k = -i sigma_k,
// A_4 = 1.  For the lower half-spinor d = (psi_2, psi_3):
//   (1 -+ gamma_mu) psi = [ h ; -+ A^dag h ],  h = psi_up -+ A_mu d,
// so each hop moves a 2-spin x 3-colour half-spinor through the link.

// h = psi_up - A d (forward, sg = -1) or psi_up + A d (backward, sg = +1)
template <typename R>
__device__ __forceinline__ void project(int mu, R sg, cx<R> p0, cx<R> p1, cx<R> p2, cx<R> p3,
                                        cx<R>& h0, cx<R>& h1) {
    cx<R> a0, a1;  // A_mu (p2, p3)
    switch (mu) {
        case 0: a0 = tmi(p3); a1 = tmi(p2); break;
        case 1: a0 = -p3; a1 = p2; break;
        case 2: a0 = tmi(p2); a1 = ti(p3); break;
        default: a0 = p2; a1 = p3; break;
    }
    h0 = p0 + sg * a0;
    h1 = p1 + sg * a1;
}

// acc_up += u ; acc_dn += sg * A_mu^dag u
template <typename R>
__device__ __forceinline__ void reconstruct(int mu, R sg, cx<R> (&acc)[4][3],
                                            const cx<R> (&u)[2][3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const cx<R> u0 = u[0][c], u1 = u[1][c];
        cx<R> b0, b1;  // A^dag (u0, u1)
        switch (mu) {
            case 0: b0 = ti(u1); b1 = ti(u0); break;
            case 1: b0 = u1; b1 = -u0; break;
            case 2: b0 = ti(u0); b1 = tmi(u1); break;
            default: b0 = u0; b1 = u1; break;
        }
        acc[0][c] = acc[0][c] + u0;
        acc[1][c] = acc[1][c] + u1;
        acc[2][c] = acc[2][c] + sg * b0;
        acc[3][c] = acc[3][c] + sg * b1;
    }
}

// One hop for RPT right-hand sides sharing the link: project each neighbour
// spinor to a half-spinor, move it through the link (U_mu(x) forward,
// U_mu(x-mu)^dag backward), reconstruct into acc.  Per-lane offsets are 32-bit
// element indices from uniform base pointers.  With an LDS tile (TIL = 1:
// the block's 256 sites [s0, s0 + 256) of every rhs, component-major), a
// neighbour inside the tile is read from LDS instead of memory.  With LNK = 1
// the links are stored as their first two rows (6 elements per link) and the
// third is rebuilt as lsgn * conj(row0 x row1), exact for SU(3); lsgn is the
// boundary sign folded into the stored rows of that link.
// Input of the fused seed iteration (FU = 1): the stencil acts on
// r_k = r_{k-1} - a q_{k-1}, formed at each neighbour from psi = r_{k-1} and
// q = q_{k-1} as it is loaded (a neighbour inside the LDS tile is read there,
// where the block has already formed it).
template <typename R, int RPT>
struct FusedIn {
    const C2<R>* q[RPT];
    cx<R> a[RPT];
};

// The operands of one hop: the neighbour spinor of every rhs and the stored
// elements of the link, loaded before any of them is used (hop_load), then
// consumed by hop_apply.  Keeping the two apart lets a caller issue the
// loads of two hops before the first hop's projection, which branches on mu
// (loads placed after such a branch wait for the earlier ones to return).
template <typename R, int RPT>
struct HopIn {
    cx<R> pv[RPT][4][3];
    cx<R> m[3][3];
};

template <typename R, int RPT, int TIL, int LNK, int LT = 0, int FU = 0>
__device__ __forceinline__ void hop_load(HopIn<R, RPT>& d, const C2<R>* const (&psi)[RPT],
                                         const C2<R>* __restrict__ Um, uint32_t nb,
                                         uint32_t lsite, const C2<R>* tile, uint32_t s0,
                                         const C2<R>* lut = nullptr,
                                         const FusedIn<R, RPT>* fi = nullptr) {
    constexpr uint32_t NE = LNK ? 6 : 9;  // stored elements per link
    // link element e of this hop's link: from the LDS link tile (LT = 1: the
    // forward links of the block's sites, [NE][256] for this mu) when the
    // link's site lies in the tile, else from memory
    const uint32_t llo = lsite - s0;
    const bool lin = LT && llo < (uint32_t)kBlock;
    auto lload = [&](uint32_t e) -> cx<R> {
        if (LT && lin) {
            const C2<R> v = lut[e * (uint32_t)kBlock + llo];
            return mk<R>(v.x, v.y);
        }
        return ld<R>(Um, tix(e, lsite, NE));
    };
    const uint32_t lo = nb - s0;
    if (TIL && lo < (uint32_t)kBlock) {
#pragma unroll
        for (int r = 0; r < RPT; ++r)
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const C2<R> v = tile[(uint32_t)((r * 12 + 3 * a + c) * kBlock) + lo];
                    d.pv[r][a][c] = mk<R>(v.x, v.y);
                }
    } else if constexpr (FU == 1) {
#pragma unroll
        for (int r = 0; r < RPT; ++r)
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const uint32_t o = tix((uint32_t)(3 * a + c), nb, 12);
                    const cx<R> rv = ld<R>(psi[r], o), qv = ld<R>(fi->q[r], o);
                    const cx<R> al = fi->a[r];
                    d.pv[r][a][c] = mk<R>(rv.re - (al.re * qv.re - al.im * qv.im),
                                          rv.im - (al.re * qv.im + al.im * qv.re));
                }
    } else {
#pragma unroll
        for (int r = 0; r < RPT; ++r)
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    d.pv[r][a][c] = ld<R>(psi[r], tix((uint32_t)(3 * a + c), nb, 12));
    }
#pragma unroll
    for (int a = 0; a < (LNK ? 2 : 3); ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) d.m[a][b] = lload((uint32_t)(3 * a + b));
}

template <typename R, int RPT, int LNK>
__device__ __forceinline__ void hop_apply(int mu, bool fwd, cx<R> (&acc)[RPT][4][3],
                                          HopIn<R, RPT>& d, R lsgn) {
    const R sg = fwd ? R(-1) : R(1);
    cx<R> h[RPT][2][3];
#pragma unroll
    for (int r = 0; r < RPT; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            project<R>(mu, sg, d.pv[r][0][c], d.pv[r][1][c], d.pv[r][2][c], d.pv[r][3][c],
                       h[r][0][c], h[r][1][c]);
    if constexpr (LNK == 1) {
        // row 2 = lsgn * conj(row0 x row1)
        const cx<R> c0 = d.m[0][1] * d.m[1][2] - d.m[0][2] * d.m[1][1];
        const cx<R> c1 = d.m[0][2] * d.m[1][0] - d.m[0][0] * d.m[1][2];
        const cx<R> c2 = d.m[0][0] * d.m[1][1] - d.m[0][1] * d.m[1][0];
        d.m[2][0] = mk<R>(lsgn * c0.re, -lsgn * c0.im);
        d.m[2][1] = mk<R>(lsgn * c1.re, -lsgn * c1.im);
        d.m[2][2] = mk<R>(lsgn * c2.re, -lsgn * c2.im);
    }
    // element (a,b) of the hop matrix: U[a][b] forward, conj(U[b][a]) backward
    const R ci = fwd ? R(1) : R(-1);
    cx<R> u[RPT][2][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            u[r][0][a] = mk<R>(0, 0);
            u[r][1][a] = mk<R>(0, 0);
        }
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            cx<R> l = fwd ? d.m[a][b] : d.m[b][a];
            l.im *= ci;
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                fma_(u[r][0][a], l, h[r][0][b]);
                fma_(u[r][1][a], l, h[r][1][b]);
            }
        }
    }
#pragma unroll
    for (int r = 0; r < RPT; ++r) reconstruct<R>(mu, sg, acc[r], u[r]);
}

template <typename R, int RPT, int TIL, int LNK, int LT = 0, int FU = 0>
__device__ __forceinline__ void hop(int mu, bool fwd, cx<R> (&acc)[RPT][4][3],
                                    const C2<R>* const (&psi)[RPT],
                                    const C2<R>* __restrict__ Um, uint32_t nb,
                                    uint32_t lsite, const C2<R>* tile, uint32_t s0, R lsgn,
                                    const C2<R>* lut = nullptr,
                                    const FusedIn<R, RPT>* fi = nullptr) {
    HopIn<R, RPT> d;
    hop_load<R, RPT, TIL, LNK, LT, FU>(d, psi, Um, nb, lsite, tile, s0, lut, fi);
    hop_apply<R, RPT, LNK>(mu, fwd, acc, d, lsgn);
}

__device__ __forceinline__ uint32_t nbr(const Geom& g, uint32_t s, const int (&coord)[4], int mu,
                                        bool fwd) {
    const uint32_t sd = (uint32_t)g.stride[mu];
    const int L = g.L[mu];
    const int cm = coord[mu];
    if (fwd) return (cm == L - 1) ? s - (uint32_t)(L - 1) * sd : s + sd;
    return (cm == 0) ? s + (uint32_t)(L - 1) * sd : s - sd;
}

// acc = sum over the hops of this lane.  The hop loop stays rolled so that
// only HPI hops' loads are live at a time (fully unrolled, the scheduler
// hoists every neighbour's loads and the kernel spills).  SPL = 1: one lane
// takes all 8 hops; HPI = 2 takes both hops of one direction per iteration
// (twice the loads in flight for more registers).  SPL = 2: two neighbouring
// lanes share a site, lane h = 0 the four forward hops and h = 1 the four
// backward ones, so mu stays wave-uniform; HPI = 2 takes two directions per
// iteration.
template <typename R, int HPI, int RPT, int SPL, int TIL, int LNK, int LT = 0, int FU = 0>
__device__ __forceinline__ void dslash_site(cx<R> (&acc)[RPT][4][3],
                                            const C2<R>* const (&psi)[RPT],
                                            const C2<R>* __restrict__ U, const Geom& g,
                                            uint32_t s, const int (&coord)[4], int h,
                                            const C2<R>* tile, uint32_t s0,
                                            const C2<R>* lu = nullptr,
                                            const FusedIn<R, RPT>* fi = nullptr) {
    const uint32_t Vt = (uint32_t)g.Vt;
    constexpr uint32_t NE = LNK ? 6 : 9;  // stored elements per link
    // boundary sign of the link a hop uses: U_mu(x) forward (last slice when
    // x_mu = L-1), U_mu(x - mu) backward (last slice when x_mu = 0)
    auto lsg = [&](int mu, bool fwd) -> R {
        const int edge = fwd ? g.L[mu] - 1 : 0;
        return (coord[mu] == edge && g.bc[mu] < 0) ? R(-1) : R(1);
    };
    // Direction of step i of the one-lane-per-site loops (2-bit field i of
    // kOrd): FP64 z, x, y, t and FP32 x, z, y, t.  The order decides how long
    // after the block's LDS tile fill (and its neighbours' fills) each
    // neighbour is read, and so how many of those reads L2 still serves: at
    // 16^4 x 4 sources in the solver, z before the LDS-served x and y hops
    // took the FP64 stencil from 55.4 to 52 us per launch against the order
    // x, y, z, t; t or z first slowed the FP32 one by 2-5%.
    constexpr unsigned kOrd = sizeof(R) == 8 ? 0xD2u : 0xD8u;
    if constexpr (SPL == 2) {
        const bool fwd = h == 0;
        if constexpr (HPI == 1) {
#pragma unroll 1
            for (int mu = 0; mu < 4; ++mu) {
                const uint32_t nb = nbr(g, s, coord, mu, fwd);
                hop<R, RPT, TIL, LNK, LT, FU>(mu, fwd, acc, psi, U + (size_t)mu * NE * Vt, nb, fwd ? s : nb, tile, s0, lsg(mu, fwd), lu + (size_t)(mu) * NE * kBlock, fi);
            }
        } else {
#pragma unroll 1
            for (int mu = 0; mu < 4; mu += 2) {
                const uint32_t n0 = nbr(g, s, coord, mu, fwd), n1 = nbr(g, s, coord, mu + 1, fwd);
                // both hops' loads are issued before either is used
                HopIn<R, RPT> d0, d1;
                hop_load<R, RPT, TIL, LNK, LT, FU>(d0, psi, U + (size_t)mu * NE * Vt, n0,
                                                   fwd ? s : n0, tile, s0,
                                                   lu + (size_t)(mu) * NE * kBlock, fi);
                hop_load<R, RPT, TIL, LNK, LT, FU>(d1, psi, U + (size_t)(mu + 1) * NE * Vt, n1,
                                                   fwd ? s : n1, tile, s0,
                                                   lu + (size_t)(mu + 1) * NE * kBlock, fi);
                hop_apply<R, RPT, LNK>(mu, fwd, acc, d0, lsg(mu, fwd));
                hop_apply<R, RPT, LNK>(mu + 1, fwd, acc, d1, lsg(mu + 1, fwd));
            }
        }
    } else if constexpr (HPI == 1) {
#pragma unroll 1
        for (int d = 0; d < 8; ++d) {
            const int mu = (int)((kOrd >> (2 * (d >> 1))) & 3u);
            const bool fwd = (d & 1) == 0;
            const uint32_t nb = nbr(g, s, coord, mu, fwd);
            hop<R, RPT, TIL, LNK, LT, FU>(mu, fwd, acc, psi, U + (size_t)mu * NE * Vt, nb, fwd ? s : nb, tile, s0, lsg(mu, fwd), lu + (size_t)(mu) * NE * kBlock, fi);
        }
    } else {
#pragma unroll 1
        for (int i = 0; i < 4; ++i) {
            const int mu = (int)((kOrd >> (2 * i)) & 3u);
            const uint32_t fw = nbr(g, s, coord, mu, true), bw = nbr(g, s, coord, mu, false);
            // both hops' loads are issued before either is used
            HopIn<R, RPT> d0, d1;
            hop_load<R, RPT, TIL, LNK, LT, FU>(d0, psi, U + (size_t)mu * NE * Vt, fw, s, tile, s0,
                                               lu + (size_t)(mu) * NE * kBlock, fi);
            hop_load<R, RPT, TIL, LNK, LT, FU>(d1, psi, U + (size_t)mu * NE * Vt, bw, bw, tile, s0,
                                               lu + (size_t)(mu) * NE * kBlock, fi);
            hop_apply<R, RPT, LNK>(mu, true, acc, d0, lsg(mu, true));
            hop_apply<R, RPT, LNK>(mu, false, acc, d1, lsg(mu, false));
        }
    }
}


// With rhs groups fastest, the XCD-aware remap hands each XCD a run of nsb/8
// consecutive site blocks.  Where a site block is one whole (z, t) plane
// (Lx Ly = kBlock sites, no padding) and Lz is even and Lt a multiple of 4,
// that run is Lt/8 whole t-slices; this maps it to a Lz/2 x Lt/4 patch of
// (z, t) planes instead, whose z and t faces (the neighbours the XCD reads
// from the others') are 3/4 the size.  A bijection of the site blocks, so
// the per-block partials keep their indices and summation order.
__device__ __forceinline__ int plane_patch(int sb, const Geom& g, int nsb) {
    const int Lz = g.L[2], Lt = g.L[3];
    if (g.L[0] * g.L[1] != kBlock || nsb != Lz * Lt || (Lz & 1) || (Lt & 3)) return sb;
    const int per = nsb / 8, x = sb / per, q = sb % per, zl = Lz / 2;
    return (x & 1) * zl + q % zl + Lz * ((x >> 1) * (Lt / 4) + q / zl);
}

// Body of the stencil for one block, `tile` being the block's position in
// the (site tile, rhs group) space after the XCD-aware remap.
template <typename R, int MODE, int HPI, int RPT, int ORD, int SPL, int TIL, int LNK>
__device__ __forceinline__ void wilson_block(const C2<R>* __restrict__ in, C2<R>* __restrict__ out,
                                             const C2<R>* __restrict__ U, const Geom& g, R kappa,
                                             double zsr, double zsi,
                                             const C2<R>* __restrict__ rdot,
                                             double4* __restrict__ partial,
                                             const SrcState* __restrict__ stt,
                                             const ShiftDev& sh, int k, int nsb, int nrhs,
                                             unsigned tile) {
    // ORD 0: rhs groups fastest, so the blocks of one site tile (all rhs) run
    // back to back on one XCD and share its links through L2 (few rhs).
    // ORD 1: site tiles fastest within an rhs group, so a tile's z and t
    // neighbours were fetched moments earlier by the same XCD (many rhs).
    const int ngrp = (nrhs + RPT - 1) / RPT;
    const int n0 = (int)uniform(ORD == 0 ? tile % (unsigned)ngrp : tile / (unsigned)nsb) * RPT;
    const int sb = (int)uniform(ORD == 0 ? plane_patch((int)(tile / (unsigned)ngrp), g, nsb)
                                         : (int)(tile % (unsigned)nsb));
    bool on[RPT];
    bool any = false;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        on[r] = n0 + r < nrhs;
        if constexpr (MODE == 1) on[r] = on[r] && src_live(stt[n0 + r], sh, n0 + r, k);
        any = any || on[r];
    }
    if (!any) return;
    constexpr int NT = kBlock * SPL;
    const uint32_t V = (uint32_t)g.V, Vt = (uint32_t)g.Vt;
    const int h = SPL == 2 ? (int)(threadIdx.x & 1u) : 0;
    const uint32_t s = (uint32_t)sb * kBlock + (SPL == 2 ? threadIdx.x >> 1 : threadIdx.x);
    const bool valid = s < V;
    // per rhs: <r, q> (re, im), ||q||^2 and ||r||^2 of this block's sites
    double dre[RPT], dim[RPT], dqq[RPT], drr[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) dre[r] = dim[r] = dqq[r] = drr[r] = 0.0;
    const C2<R>* psi[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) psi[r] = in + (size_t)(n0 + (on[r] ? r : 0)) * 12 * Vt;
    cx<R> acc[RPT][4][3];
#pragma unroll
    for (int r = 0; r < RPT; ++r)
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[r][a][c] = mk<R>(0, 0);
    // TIL: the block's sites of every rhs staged in LDS once, read there by
    // the site itself and by every neighbour that falls inside the block
    static_assert(TIL == 0 || SPL == 1, "the LDS tile assumes one lane per site");
    __shared__ C2<R> lt[TIL ? RPT * 12 * kBlock : 1];
    const uint32_t s0 = (uint32_t)sb * kBlock;
    if constexpr (TIL == 1) {
        if (valid) {
#pragma unroll
            for (int r = 0; r < RPT; ++r)
#pragma unroll
                for (int comp = 0; comp < 12; ++comp) {
                    const cx<R> v = ld<R>(psi[r], tix((uint32_t)comp, s, 12));
                    C2<R> w;
                    w.x = v.re;
                    w.y = v.im;
                    lt[(r * 12 + comp) * kBlock + threadIdx.x] = w;
                }
        }
        __syncthreads();
    }
    if (valid) {
        uint32_t rem = s;
        int coord[4];
        coord[0] = (int)(rem % (uint32_t)g.L[0]); rem /= (uint32_t)g.L[0];
        coord[1] = (int)(rem % (uint32_t)g.L[1]); rem /= (uint32_t)g.L[1];
        coord[2] = (int)(rem % (uint32_t)g.L[2]);
        coord[3] = (int)(rem / (uint32_t)g.L[2]);
        dslash_site<R, HPI, RPT, SPL, TIL, LNK>(acc, psi, U, g, s, coord, h, lt, s0);
    }
    if constexpr (SPL == 2) {
        // lane h keeps spins 2h, 2h+1 (in acc[.][0..1]) and adds the partner's
        // partial sums of them; both lanes of a pair share the site's validity
#pragma unroll
        for (int r = 0; r < RPT; ++r)
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const cx<R> lo = acc[r][i][c], hi = acc[r][2 + i][c];
                    const cx<R> snd = h ? lo : hi;
                    const cx<R> got = mk<R>(__shfl_xor(snd.re, 1), __shfl_xor(snd.im, 1));
                    acc[r][i][c] = (h ? hi : lo) + got;
                }
    }
    if (valid) {
        constexpr int NA = 4 / SPL;  // spins written by this lane: 2h + ai
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            if (!on[r]) continue;
            C2<R>* o = out + (size_t)(n0 + r) * 12 * Vt;
            // solver form: beta_{k-1} of this rhs (written by the previous update)
            R br = 0, bi = 0;
            if constexpr (MODE == 1) {
                if (k > 0) {
                    const double2 b = stt[n0 + r].beta[(k - 1) & 1];
                    br = (R)b.x;
                    bi = (R)b.y;
                }
            }
            // every load of the site's own r_k and q_{k-1} is issued before the
            // first store: o may alias psi as far as the compiler knows, so a
            // load placed after a store would wait for it
            cx<R> pv[NA][3], qv[NA][3];
#pragma unroll
            for (int ai = 0; ai < NA; ++ai) {
                const int a = SPL == 2 ? 2 * h + ai : ai;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const uint32_t comp = (uint32_t)(3 * a + c);
                    if constexpr (TIL == 1) {
                        const C2<R> w = lt[(r * 12 + (int)comp) * kBlock + threadIdx.x];
                        pv[ai][c] = mk<R>(w.x, w.y);
                    } else {
                        pv[ai][c] = ld<R>(psi[r], tix(comp, s, 12));
                    }
                    qv[ai][c] = mk<R>(0, 0);
                    if constexpr (MODE == 1)
                        if (k > 0) qv[ai][c] = ld<R>(o, tix(comp, s, 12));
                }
            }
#pragma unroll
            for (int ai = 0; ai < NA; ++ai) {
                const int a = SPL == 2 ? 2 * h + ai : ai;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const uint32_t comp = (uint32_t)(3 * a + c);
                    const cx<R> p = pv[ai][c];
                    // D psi = psi - kappa acc ; H = gamma5 D
                    cx<R> hv = p - kappa * acc[r][ai][c];
                    if (a >= 2) hv = -hv;
                    if constexpr (MODE == 0) {
                        stc<R>(o, tix(comp, s, 12), hv);
                    } else {
                        // q_k = z_s r_k - H r_k + beta_{k-1} q_{k-1}, in place (this lane
                        // read its own q_{k-1} above, before any write of q_k)
                        const R zr = (R)zsr, zi = (R)zsi;
                        cx<R> q = mk<R>(zr * p.re - zi * p.im - hv.re, zr * p.im + zi * p.re - hv.im);
                        const cx<R> qo = qv[ai][c];
                        q.re += br * qo.re - bi * qo.im;
                        q.im += br * qo.im + bi * qo.re;
                        stc<R>(o, tix(comp, s, 12), q);
                        // <r_k, q_k> = sum conj(r) q with r_k = p, accumulated in FP64
                        dre[r] += (double)p.re * (double)q.re + (double)p.im * (double)q.im;
                        dim[r] += (double)p.re * (double)q.im - (double)p.im * (double)q.re;
                        dqq[r] += (double)q.re * (double)q.re + (double)q.im * (double)q.im;
                        drr[r] += (double)p.re * (double)p.re + (double)p.im * (double)p.im;
                    }
                }
            }
        }
    }
    if constexpr (MODE == 1) {
        __shared__ double shd[4 * NT / 64];
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            double t[4] = {dre[r], dim[r], dqq[r], drr[r]};
            block_sum4<NT>(t, shd);
            if (on[r] && threadIdx.x == 0)
                partial[(int64_t)(n0 + r) * nsb + sb] = make_double4(t[0], t[1], t[2], t[3]);
        }
    }
}

// Link-tile body: RB right-hand sides of one 256-site tile per block (RB
// groups of four waves, one lane per site and rhs).  The block stages the
// forward links of its sites in LDS once and every rhs reads them there, as
// does a backward hop whose link site lies in the tile; blocks are ordered
// rhs-group fastest, so the blocks of one tile run back to back on one XCD.
template <typename R, int MODE, int HPI, int RB, int LNK>
__device__ __forceinline__ void wilson_block_lt(const C2<R>* __restrict__ in, C2<R>* __restrict__ out,
                                                const C2<R>* __restrict__ U, const Geom& g, R kappa,
                                                double zsr, double zsi,
                                                const C2<R>* __restrict__ rdot,
                                                double4* __restrict__ partial,
                                                const SrcState* __restrict__ stt,
                                                const ShiftDev& sh, int k, int nsb, int nrhs,
                                                unsigned tile) {
    constexpr int NT = kBlock * RB;
    constexpr uint32_t NE = LNK ? 6 : 9;
    const int ngrp = (nrhs + RB - 1) / RB;
    const int grp = (int)uniform(tile % (unsigned)ngrp);
    const int sb = (int)uniform(tile / (unsigned)ngrp);
    bool onr[RB];
    bool any = false;
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        const int n = grp * RB + r;
        onr[r] = n < nrhs;
        if constexpr (MODE == 1) onr[r] = onr[r] && src_live(stt[n], sh, n, k);
        any = any || onr[r];
    }
    if (!any) return;
    const int w = (int)(threadIdx.x / kBlock);  // rhs of this lane within the block (wave-uniform)
    const uint32_t t = threadIdx.x % kBlock;
    bool on = false;
#pragma unroll
    for (int r = 0; r < RB; ++r)
        if (r == w) on = onr[r];
    const int n = grp * RB + w;
    const uint32_t V = (uint32_t)g.V, Vt = (uint32_t)g.Vt;
    const uint32_t s0 = (uint32_t)sb * kBlock;
    const uint32_t s = s0 + t;
    const bool valid = s < V;
    __shared__ C2<R> lu[4 * NE * kBlock];
    for (uint32_t q = threadIdx.x; q < 4 * NE * (uint32_t)kBlock; q += NT) {
        const uint32_t me = q / (uint32_t)kBlock, tt = q % (uint32_t)kBlock;
        if (s0 + tt < V) lu[q] = U[(size_t)(me / NE) * NE * Vt + tix(me % NE, s0 + tt, NE)];
    }
    __syncthreads();
    double dre = 0.0, dim = 0.0, dqq = 0.0, drr = 0.0;
    if (valid && on) {
        const C2<R>* psi[1] = {in + (size_t)n * 12 * Vt};
        cx<R> acc[1][4][3];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[0][a][c] = mk<R>(0, 0);
        uint32_t rem = s;
        int coord[4];
        coord[0] = (int)(rem % (uint32_t)g.L[0]); rem /= (uint32_t)g.L[0];
        coord[1] = (int)(rem % (uint32_t)g.L[1]); rem /= (uint32_t)g.L[1];
        coord[2] = (int)(rem % (uint32_t)g.L[2]);
        coord[3] = (int)(rem / (uint32_t)g.L[2]);
        dslash_site<R, HPI, 1, 1, 0, LNK, 1>(acc, psi, U, g, s, coord, 0, nullptr, s0, lu);
        C2<R>* o = out + (size_t)n * 12 * Vt;
        R br = 0, bi = 0;
        if constexpr (MODE == 1) {
            if (k > 0) {
                const double2 b = stt[n].beta[(k - 1) & 1];
                br = (R)b.x;
                bi = (R)b.y;
            }
        }
        // the site's own r_k and q_{k-1} are loaded before the first store
        cx<R> pv[4][3], qv[4][3];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const uint32_t comp = (uint32_t)(3 * a + c);
                pv[a][c] = ld<R>(psi[0], tix(comp, s, 12));
                qv[a][c] = mk<R>(0, 0);
                if constexpr (MODE == 1)
                    if (k > 0) qv[a][c] = ld<R>(o, tix(comp, s, 12));
            }
#pragma unroll
        for (int a = 0; a < 4; ++a) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const uint32_t comp = (uint32_t)(3 * a + c);
                const cx<R> p = pv[a][c];
                cx<R> hv = p - kappa * acc[0][a][c];
                if (a >= 2) hv = -hv;
                if constexpr (MODE == 0) {
                    stc<R>(o, tix(comp, s, 12), hv);
                } else {
                    const R zr = (R)zsr, zi = (R)zsi;
                    cx<R> q = mk<R>(zr * p.re - zi * p.im - hv.re, zr * p.im + zi * p.re - hv.im);
                    const cx<R> qo = qv[a][c];
                    q.re += br * qo.re - bi * qo.im;
                    q.im += br * qo.im + bi * qo.re;
                    stc<R>(o, tix(comp, s, 12), q);
                    dre += (double)p.re * (double)q.re + (double)p.im * (double)q.im;
                    dim += (double)p.re * (double)q.im - (double)p.im * (double)q.re;
                    dqq += (double)q.re * (double)q.re + (double)q.im * (double)q.im;
                    drr += (double)p.re * (double)p.re + (double)p.im * (double)p.im;
                }
            }
        }
    }
    if constexpr (MODE == 1) {
        __shared__ double shd[4 * NT / 64];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const bool mine = w == r;
            double t[4] = {mine ? dre : 0.0, mine ? dim : 0.0, mine ? dqq : 0.0, mine ? drr : 0.0};
            block_sum4<NT>(t, shd);
            if (onr[r] && threadIdx.x == 0)
                partial[(int64_t)(grp * RB + r) * nsb + sb] = make_double4(t[0], t[1], t[2], t[3]);
        }
    }
}

template <typename R, int MODE, int HPI, int RB, int LNK>
__global__ __launch_bounds__(kBlock * RB) void k_wilson_lt(const C2<R>* __restrict__ in,
                                                           C2<R>* __restrict__ out,
                                                           const C2<R>* __restrict__ U, Geom g,
                                                           R kappa, double zsr, double zsi,
                                                           const C2<R>* __restrict__ rdot,
                                                           double4* __restrict__ partial,
                                                           const SrcState* __restrict__ stt,
                                                           ShiftDev sh, int k, int nsb, int nrhs) {
    const unsigned tile = uniform(xcd_remap(blockIdx.x, gridDim.x));
    wilson_block_lt<R, MODE, HPI, RB, LNK>(in, out, U, g, kappa, zsr, zsi, rdot, partial, stt, sh,
                                           k, nsb, nrhs, tile);
}

// Block -> (job, tile) of a job-table stencil launch.  Job j owns blocks
// [sten_b0, sten_b0 + pad8(sten_nb)) of the grid, sten_b0 a multiple of 8,
// so its blocks go round-robin over all eight XCDs like those of a launch of
// its own (dispatch assigns block b to XCD b mod 8), and within the job the
// XCD-aware remap groups neighbouring tiles on one XCD.  A job that has
// finished, or iterates in the other precision, thus leaves every XCD, not
// a contiguous few, to the jobs still running.  Returns false for the
// job's padding blocks and for jobs in the other precision phase.
__device__ __forceinline__ bool job_tile(const JobDesc* __restrict__ jobs, int njobs, int f,
                                         int& j, unsigned& tile) {
    const unsigned b = blockIdx.x;
    j = 0;
    while (j + 1 < njobs && b >= (unsigned)jobs[j + 1].sten_b0[f]) ++j;
    const JobDesc& J = jobs[j];
    if (J.phase != f) return false;  // this job iterates in the other precision
    const unsigned nb = (unsigned)J.sten_nb[f];
    tile = uniform(xcd_remap(b - (unsigned)J.sten_b0[f], (nb + 7u) & ~7u));
    return tile < nb;
}

template <typename R, int HPI, int RB, int LNK>
__global__ __launch_bounds__(kBlock * RB) void k_wilson_jobs_lt(const JobDesc* __restrict__ jobs,
                                                                int njobs,
                                                                const int* __restrict__ kdev) {
    const int k = (int)uniform((uint32_t)*kdev);
    const int f = sizeof(R) == 4 ? 1 : 0;
    int j;
    unsigned tile;
    if (!job_tile(jobs, njobs, f, j, tile)) return;
    const JobDesc& J = jobs[j];
    wilson_block_lt<R, 1, HPI, RB, LNK>(job_rk<const C2<R>>(J, k, f), static_cast<C2<R>*>(J.q[f]),
                                        static_cast<const C2<R>*>(J.U[f]), J.g, (R)J.kappa, J.zs.x,
                                        J.zs.y, nullptr, J.part_w, J.st, J.sh, k, J.nsb, J.nsrc,
                                        tile);
}

template <typename R, int MODE, int HPI, int RPT, int ORD, int SPL, int TIL, int LNK>
__global__ __launch_bounds__(kBlock * SPL) void k_wilson(const C2<R>* __restrict__ in,
                                                   C2<R>* __restrict__ out,
                                                   const C2<R>* __restrict__ U, Geom g, R kappa,
                                                   double zsr, double zsi,
                                                   const C2<R>* __restrict__ rdot,
                                                   double4* __restrict__ partial,
                                                   const SrcState* __restrict__ stt,
                                                   ShiftDev sh, int k, int nsb, int nrhs) {
    const unsigned tile = uniform(xcd_remap(blockIdx.x, gridDim.x));
    wilson_block<R, MODE, HPI, RPT, ORD, SPL, TIL, LNK>(in, out, U, g, kappa, zsr, zsi, rdot, partial, stt, sh,
                                         k, nsb, nrhs, tile);
}

// K1 over a job table: q_k = z_s r_k - H r_k + beta_{k-1} q_{k-1} (in place)
// and the partials <r_k, q_k>, ||q_k||^2, ||r_k||^2 for every job of a batch
// in one launch; the iteration index k is read from device memory so a
// captured graph can be replayed for any k.
template <typename R, int HPI, int RPT, int ORD, int SPL, int TIL, int LNK>
__global__ __launch_bounds__(kBlock * SPL) void k_wilson_jobs(const JobDesc* __restrict__ jobs, int njobs,
                                                        const int* __restrict__ kdev) {
    const int k = (int)uniform((uint32_t)*kdev);
    const int f = sizeof(R) == 4 ? 1 : 0;
    int j;
    unsigned tile;
    if (!job_tile(jobs, njobs, f, j, tile)) return;
    const JobDesc& J = jobs[j];
    wilson_block<R, 1, HPI, RPT, ORD, SPL, TIL, LNK>(job_rk<const C2<R>>(J, k, f),
                                      static_cast<C2<R>*>(J.q[f]),
                                      static_cast<const C2<R>*>(J.U[f]), J.g, (R)J.kappa, J.zs.x,
                                      J.zs.y, nullptr, J.part_w, J.st, J.sh, k, J.nsb, J.nsrc,
                                      tile);
}

// ============================================================================
// The fused seed iteration: one kernel per iteration of the shifted solver
// in the basis forms, without the seed direction p.  With A = z_s - H,
// p_k = r_k + beta_{k-1} p_{k-1} and q_k = A p_k, the direction enters only
// through q, and q_k = A r_k + beta_{k-1} q_{k-1}.  Kernel k
//   * reduces kernel k-1's partials to alpha_{k-1}, beta_{k-1} and the
//     estimate of ||r_k||^2 (every block, in the same fixed order);
//   * forms r_k = r_{k-1} - alpha_{k-1} q_{k-1} wherever it needs it: at its
//     own sites (stored as basis slot k, or the two-pass buffer k&1) and at
//     every neighbour of the stencil, from the loads of r_{k-1} and q_{k-1}
//     (with the LDS tile, the block's own r_k is formed once and the
//     neighbours inside the block read it there);
//   * q_k = z_s r_k - H r_k + beta_{k-1} q_{k-1} into q[k&1], and the
//     partials <r_k, q_k>, ||q_k||^2, ||r_k||^2 into part[k&1];
//   * block (site block sb, source n) advances the shift slices sb,
//     sb + nsb, ... by iteration k-1, and block (0, n) records the seed
//     scalars.
// r_{k-1}, q_{k-1} are read at neighbours while r_k, q_k are written, so
// each lives in a buffer of its own (q and the partials alternate with
// k&1).  Per iteration and rhs this moves 4 vectors (r_{k-1}, q_{k-1} read,
// r_k, q_k written) instead of the two-kernel iteration's 8.
// ============================================================================
template <typename R, int HPI, int ORD, int TIL, int LNK>
__device__ __forceinline__ void iter_block(const JobDesc& J, int k, unsigned tile) {
    const int f = sizeof(R) == 4 ? 1 : 0;
    const int nsb = J.nsb, nsrc = J.nsrc;
    const int n = (int)uniform(ORD == 0 ? tile % (unsigned)nsrc : tile / (unsigned)nsb);
    const int sb = (int)uniform(ORD == 0 ? tile / (unsigned)nsrc : tile % (unsigned)nsb);
    const ShiftDev& sh = J.sh;
    SrcState& S = J.st[n];
    __shared__ double shm[4 * kBlock / 64];
    // shift slices q = sb, sb + nsb, ... belong to site block sb (a small
    // lattice may have fewer site blocks than 256-shift slices)
    if (!src_live_fused(S, sh, n, k)) {
        // a finished source stays finished (its counts go to zero); past the
        // iteration limit the counts are kept for the host
        if (k <= sh.maxk && threadIdx.x == 0)
            for (int q = sb; q < sh.nslices; q += nsb)
                sh.cnt[((size_t)(k & 1) * sh.nsrc + n) * kMaxSlices + q] = 0;
        return;
    }
    SeedScalars sc{};
    sc.alpha = make_double2(0, 0);
    sc.beta = make_double2(0, 0);
    if (k > 0) {
        sc = seed_scalars_from(J.part_w + (size_t)((k - 1) & 1) * J.part_stride + (size_t)n * nsb,
                               nsb, shm);
        if (sc.status) {
            if (sb == 0 && threadIdx.x == 0) S.status = sc.status;
            if (threadIdx.x == 0)
                for (int q = sb; q < sh.nslices; q += nsb)
                    sh.cnt[((size_t)(k & 1) * sh.nsrc + n) * kMaxSlices + q] = 0;
            return;
        }
    }
    const uint32_t V = (uint32_t)J.g.V, Vt = (uint32_t)J.g.Vt;
    const uint32_t s = (uint32_t)sb * kBlock + threadIdx.x;
    const bool valid = s < V;
    const size_t n12 = (size_t)12 * Vt;
    const C2<R>* rin = job_rk<const C2<R>>(J, k > 0 ? k - 1 : 0, f) + (size_t)n * n12;
    C2<R>* rout = job_rk<C2<R>>(J, k, f) + (size_t)n * n12;
    const C2<R>* qin = static_cast<const C2<R>*>(J.q[f]) + (size_t)((k - 1) & 1) * J.qpp + (size_t)n * n12;
    C2<R>* qout = static_cast<C2<R>*>(J.q[f]) + (size_t)(k & 1) * J.qpp + (size_t)n * n12;
    // kernel 0 applies A to r_0 = b itself: no combination and no q term
    FusedIn<R, 1> fi;
    fi.q[0] = k > 0 ? qin : rin;
    fi.a[0] = mk<R>((R)sc.alpha.x, (R)sc.alpha.y);
    const C2<R>* psi[1] = {rin};
    const uint32_t s0 = (uint32_t)sb * kBlock;
    __shared__ C2<R> lt[TIL ? 12 * kBlock : 1];
    // the block's own r_k: formed once, stored as the new basis vector, and
    // (TIL) kept in LDS for the neighbours inside the block
    auto own_rk = [&](uint32_t comp) -> cx<R> {
        const uint32_t o = tix(comp, s, 12);
        const cx<R> rv = ld<R>(rin, o);
        if (k == 0) return rv;
        const cx<R> qv = ld<R>(qin, o);
        const cx<R> al = fi.a[0];
        return mk<R>(rv.re - (al.re * qv.re - al.im * qv.im), rv.im - (al.re * qv.im + al.im * qv.re));
    };
    if constexpr (TIL == 1) {
        if (valid) {
#pragma unroll
            for (uint32_t comp = 0; comp < 12; ++comp) {
                const cx<R> v = own_rk(comp);
                C2<R> w;
                w.x = v.re;
                w.y = v.im;
                lt[comp * kBlock + threadIdx.x] = w;
                if (k > 0) stc<R>(rout, tix(comp, s, 12), v);
            }
        }
        __syncthreads();
    }
    cx<R> acc[1][4][3];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[0][a][c] = mk<R>(0, 0);
    if (valid) {
        uint32_t rem = s;
        int coord[4];
        coord[0] = (int)(rem % (uint32_t)J.g.L[0]); rem /= (uint32_t)J.g.L[0];
        coord[1] = (int)(rem % (uint32_t)J.g.L[1]); rem /= (uint32_t)J.g.L[1];
        coord[2] = (int)(rem % (uint32_t)J.g.L[2]);
        coord[3] = (int)(rem / (uint32_t)J.g.L[2]);
        dslash_site<R, HPI, 1, 1, TIL, LNK, 0, 1>(acc, psi, static_cast<const C2<R>*>(J.U[f]), J.g,
                                                  s, coord, 0, lt, s0, nullptr, &fi);
    }
    double dre = 0.0, dim = 0.0, dqq = 0.0, drr = 0.0;
    const R kap = (R)J.kappa, zr = (R)J.zs.x, zi = (R)J.zs.y;
    const R br = (R)sc.beta.x, bi = (R)sc.beta.y;
    const bool acc2 = J.h != nullptr && k > 0;
    const double2 hk = acc2 ? J.h[(size_t)n * (sh.maxk + 1) + k] : make_double2(0, 0);
    double2* sacc = J.s64 + (size_t)n * n12;
    if (valid) {
        // every load of the site's own vectors is issued before the first
        // store (the outputs may alias the inputs as far as the compiler knows)
        cx<R> qv[12], rv[12];
#pragma unroll
        for (int comp = 0; comp < 12; ++comp) {
            const uint32_t o = tix((uint32_t)comp, s, 12);
            qv[comp] = k > 0 ? ld<R>(qin, o) : mk<R>(0, 0);
            if constexpr (TIL == 1) {
                const C2<R> w = lt[comp * kBlock + threadIdx.x];
                rv[comp] = mk<R>(w.x, w.y);
            } else {
                rv[comp] = ld<R>(rin, o);
            }
        }
#pragma unroll
        for (int a = 0; a < 4; ++a) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const uint32_t comp = (uint32_t)(3 * a + c);
                const uint32_t o = tix(comp, s, 12);
                const cx<R> qo = qv[comp];
                cx<R> r = rv[comp];
                if constexpr (TIL == 0) {
                    if (k > 0) {
                        const cx<R> al = fi.a[0];
                        r = mk<R>(r.re - (al.re * qo.re - al.im * qo.im),
                                  r.im - (al.re * qo.im + al.im * qo.re));
                        stc<R>(rout, o, r);
                    }
                }
                // H r = gamma5 (r - kappa acc); q_k = z_s r - H r + beta q_{k-1}
                cx<R> hv = r - kap * acc[0][a][c];
                if (a >= 2) hv = -hv;
                cx<R> q = mk<R>(zr * r.re - zi * r.im - hv.re, zr * r.im + zi * r.re - hv.im);
                if (k > 0) {
                    q.re += br * qo.re - bi * qo.im;
                    q.im += br * qo.im + bi * qo.re;
                }
                stc<R>(qout, o, q);
                dre += (double)r.re * (double)q.re + (double)r.im * (double)q.im;
                dim += (double)r.re * (double)q.im - (double)r.im * (double)q.re;
                dqq += (double)q.re * (double)q.re + (double)q.im * (double)q.im;
                drr += (double)r.re * (double)r.re + (double)r.im * (double)r.im;
                if (acc2) {
                    double2 sv = sacc[o];
                    sv.x += hk.x * (double)r.re - hk.y * (double)r.im;
                    sv.y += hk.x * (double)r.im + hk.y * (double)r.re;
                    sacc[o] = sv;
                }
            }
        }
    } else if (s < Vt) {
        // padding sites of the last layout tile stay zero in every output
#pragma unroll
        for (uint32_t comp = 0; comp < 12; ++comp) {
            const uint32_t o = tix(comp, s, 12);
            stc<R>(qout, o, mk<R>(0, 0));
            if (k > 0) stc<R>(rout, o, mk<R>(0, 0));
        }
    }
    {
        double t[4] = {dre, dim, dqq, drr};
        block_sum4<kBlock>(t, shm);
        if (threadIdx.x == 0)
            J.part_w[(size_t)(k & 1) * J.part_stride + (size_t)n * nsb + sb] =
                make_double4(t[0], t[1], t[2], t[3]);
    }
    if (k == 0) return;
    // iteration k-1 of the scalars: the seed's (block (0, n)) and the shifts'
    if (sb == 0 && threadIdx.x == 0) {
        S.alpha[(k - 1) & 1] = sc.alpha;
        S.beta[(k - 1) & 1] = sc.beta;
        S.rr[(k - 1) & 1] = sc.rr;
        S.iter = k;
        if (sh.seed != nullptr) {
            double2* sd = sh.seed + ((size_t)n * (sh.maxk + 1) + (k - 1)) * 3;
            sd[0] = sc.alpha;
            sd[1] = sc.beta;
            sd[2] = make_double2(sc.rr, sc.rrn);
        }
    }
    for (int q = sb; q < sh.nslices; q += nsb) advance_shift_slice(sh, S, n, q, k - 1, sc, shm);
}

template <typename R, int HPI, int ORD, int TIL, int LNK>
__global__ __launch_bounds__(kBlock) void k_iter_jobs(const JobDesc* __restrict__ jobs, int njobs,
                                                      const int* __restrict__ kread,
                                                      int* __restrict__ kwrite) {
    const int k = (int)uniform((uint32_t)*kread);
    if (blockIdx.x == 0 && threadIdx.x == 0) *kwrite = k + 1;
    const int f = sizeof(R) == 4 ? 1 : 0;
    int j;
    unsigned tile;
    if (!job_tile(jobs, njobs, f, j, tile)) return;
    iter_block<R, HPI, ORD, TIL, LNK>(jobs[j], k, tile);
}

int iter_grid_blocks(const Geom& g, int nrhs) { return wilson_blocks(g) * nrhs; }

// Variant v < kIterVariants of the fused iteration: hops per loop step
// (bit 0: 1 or 2), block order (bit 1: rhs fastest or sites fastest), LDS
// tile of the block's r_k (bit 2).
template <typename R>
void launch_iter_jobs(const JobDesc* jobs, int njobs, const int* kread, int* kwrite,
                      int total_blocks, int variant, int lnk, hipStream_t s, hipEvent_t ev0,
                      hipEvent_t ev1) {
    auto go = [&](auto kern) {
        if (ev0)
            hipExtLaunchKernelGGL(kern, dim3(total_blocks), dim3(kBlock), 0, s, ev0, ev1, 0, jobs,
                                  njobs, kread, kwrite);
        else
            hipLaunchKernelGGL(kern, dim3(total_blocks), dim3(kBlock), 0, s, jobs, njobs, kread,
                               kwrite);
    };
    using std::integral_constant;
    auto pick = [&](auto H, auto O, auto T) {
        if (lnk) go(k_iter_jobs<R, H.value, O.value, T.value, 1>);
        else go(k_iter_jobs<R, H.value, O.value, T.value, 0>);
    };
    switch (variant) {
#define OVL_IV(n)                                                                             \
    case n:                                                                                   \
        pick(integral_constant<int, ((n)&1) + 1>{}, integral_constant<int, ((n) >> 1) & 1>{}, \
             integral_constant<int, ((n) >> 2) & 1>{});                                       \
        break;
        OVL_IV(1) OVL_IV(2) OVL_IV(3) OVL_IV(4) OVL_IV(5) OVL_IV(6) OVL_IV(7)
#undef OVL_IV
        default:
            pick(integral_constant<int, 1>{}, integral_constant<int, 0>{}, integral_constant<int, 0>{});
    }
}
template void launch_iter_jobs<double>(const JobDesc*, int, const int*, int*, int, int, int,
                                       hipStream_t, hipEvent_t, hipEvent_t);
template void launch_iter_jobs<float>(const JobDesc*, int, const int*, int*, int, int, int,
                                      hipStream_t, hipEvent_t, hipEvent_t);

int wilson_blocks(const Geom& g) { return (int)((g.V + kBlock - 1) / kBlock); }
// right-hand sides per block of a variant: the rhs per lane (variants < 24)
// or the link tile's rhs groups (24 .. 27)
static int rhs_per_block(int variant) {
    if (variant >= kShapeVariants) return ((variant - kShapeVariants) & 2) ? 4 : 2;
    return (variant & 2) ? 2 : 1;
}
int wilson_grid_blocks(const Geom& g, int nrhs, int variant) {
    const int rb = rhs_per_block(variant);
    return wilson_blocks(g) * ((nrhs + rb - 1) / rb);
}

// Link-tile variants 24 .. 27: hops per step (bit 0) and rhs per block 2 or 4
// (bit 1); calls f(HPI, RB) as integral constants.
template <typename F>
void with_lt_variant(int v, F&& f) {
    using std::integral_constant;
    switch (v - kShapeVariants) {
        case 1: f(integral_constant<int, 2>{}, integral_constant<int, 2>{}); break;
        case 2: f(integral_constant<int, 1>{}, integral_constant<int, 4>{}); break;
        case 3: f(integral_constant<int, 2>{}, integral_constant<int, 4>{}); break;
        default: f(integral_constant<int, 1>{}, integral_constant<int, 2>{}); break;
    }
}

// Calls f(HPI, RPT, ORD, SPL, TIL) as integral constants for variant v =
// 16 TIL + 8 (SPL - 1) + 4 ORD + 2 (RPT - 1) + (HPI - 1), v < 24 (the LDS
// tile takes one lane per site); other values take variant 0.
template <typename F>
void with_variant(int v, F&& f) {
    using std::integral_constant;
    switch (v) {
#define OVL_V(n)                                                                     \
    case n:                                                                          \
        f(integral_constant<int, ((n)&1) + 1>{}, integral_constant<int, (((n) >> 1) & 1) + 1>{}, \
          integral_constant<int, ((n) >> 2) & 1>{}, integral_constant<int, (((n) >> 3) & 1) + 1>{}, \
          integral_constant<int, ((n) >> 4) & 1>{});                                 \
        break;
        OVL_V(1) OVL_V(2) OVL_V(3) OVL_V(4) OVL_V(5) OVL_V(6) OVL_V(7)
        OVL_V(8) OVL_V(9) OVL_V(10) OVL_V(11) OVL_V(12) OVL_V(13) OVL_V(14) OVL_V(15)
        OVL_V(16) OVL_V(17) OVL_V(18) OVL_V(19) OVL_V(20) OVL_V(21) OVL_V(22) OVL_V(23)
#undef OVL_V
        default:
            f(integral_constant<int, 1>{}, integral_constant<int, 1>{}, integral_constant<int, 0>{},
              integral_constant<int, 1>{}, integral_constant<int, 0>{});
    }
}

template <typename R>
void launch_wilson_jobs(const JobDesc* jobs, int njobs, const int* kdev, int total_blocks,
                        int variant, int lnk, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    auto go = [&](auto kern, int threads) {
        if (ev0)
            hipExtLaunchKernelGGL(kern, dim3(total_blocks), dim3(threads), 0, s, ev0, ev1, 0, jobs,
                                  njobs, kdev);
        else
            hipLaunchKernelGGL(kern, dim3(total_blocks), dim3(threads), 0, s, jobs, njobs, kdev);
    };
    if (variant >= kShapeVariants) {
        with_lt_variant(variant, [&](auto H, auto B) {
            if (lnk)
                go(k_wilson_jobs_lt<R, H.value, B.value, 1>, kBlock * B.value);
            else
                go(k_wilson_jobs_lt<R, H.value, B.value, 0>, kBlock * B.value);
        });
        return;
    }
    with_variant(variant, [&](auto H, auto P, auto O, auto S, auto C) {
        if (lnk)
            go(k_wilson_jobs<R, H.value, P.value, O.value, S.value, C.value, 1>, kBlock * S.value);
        else
            go(k_wilson_jobs<R, H.value, P.value, O.value, S.value, C.value, 0>, kBlock * S.value);
    });
}
template void launch_wilson_jobs<double>(const JobDesc*, int, const int*, int, int, int, hipStream_t,
                                         hipEvent_t, hipEvent_t);
template void launch_wilson_jobs<float>(const JobDesc*, int, const int*, int, int, int, hipStream_t,
                                        hipEvent_t, hipEvent_t);

template <typename R, int HPI, int RPT, int ORD, int SPL, int TIL, int LNK>
void launch_wilson_v(int mode, const C2<R>* in, C2<R>* out, const C2<R>* U, const Geom& g,
                     double kappa, double2 zs, const C2<R>* r, double4* partial,
                     const SrcState* stt, const ShiftDev& sh, int k, int nrhs, hipStream_t s) {
    const int nsb = wilson_blocks(g);
    const int ngrp = (nrhs + RPT - 1) / RPT;
    dim3 grid((unsigned)nsb * (unsigned)ngrp);
    if (mode == 0)
        hipLaunchKernelGGL((k_wilson<R, 0, HPI, RPT, ORD, SPL, TIL, LNK>), grid, dim3(kBlock * SPL),
                           0, s, in, out, U, g, (R)kappa, zs.x, zs.y, r, partial, stt, sh, k, nsb,
                           nrhs);
    else
        hipLaunchKernelGGL((k_wilson<R, 1, HPI, RPT, ORD, SPL, TIL, LNK>), grid, dim3(kBlock * SPL),
                           0, s, in, out, U, g, (R)kappa, zs.x, zs.y, r, partial, stt, sh, k, nsb,
                           nrhs);
}

template <typename R>
void launch_wilson(int mode, const C2<R>* in, C2<R>* out, const C2<R>* U, const Geom& g,
                   double kappa, double2 zs, const C2<R>* r, double4* partial,
                   const SrcState* stt, const ShiftDev* sh, int k, int nrhs, hipStream_t s,
                   int variant, int lnk) {
    ShiftDev none{};
    const ShiftDev& shv = sh ? *sh : none;
    if (variant >= kShapeVariants) {
        const int nsb = wilson_blocks(g);
        with_lt_variant(variant, [&](auto H, auto B) {
            const dim3 grid((unsigned)nsb * (unsigned)((nrhs + B.value - 1) / B.value));
            const dim3 blk(kBlock * B.value);
            if (lnk) {
                if (mode == 0)
                    hipLaunchKernelGGL((k_wilson_lt<R, 0, H.value, B.value, 1>), grid, blk, 0, s, in, out,
                                       U, g, (R)kappa, zs.x, zs.y, r, partial, stt, shv, k, nsb, nrhs);
                else
                    hipLaunchKernelGGL((k_wilson_lt<R, 1, H.value, B.value, 1>), grid, blk, 0, s, in, out,
                                       U, g, (R)kappa, zs.x, zs.y, r, partial, stt, shv, k, nsb, nrhs);
            } else {
                if (mode == 0)
                    hipLaunchKernelGGL((k_wilson_lt<R, 0, H.value, B.value, 0>), grid, blk, 0, s, in, out,
                                       U, g, (R)kappa, zs.x, zs.y, r, partial, stt, shv, k, nsb, nrhs);
                else
                    hipLaunchKernelGGL((k_wilson_lt<R, 1, H.value, B.value, 0>), grid, blk, 0, s, in, out,
                                       U, g, (R)kappa, zs.x, zs.y, r, partial, stt, shv, k, nsb, nrhs);
            }
        });
        return;
    }
    with_variant(variant, [&](auto H, auto P, auto O, auto S, auto C) {
        if (lnk)
            launch_wilson_v<R, H.value, P.value, O.value, S.value, C.value, 1>(
                mode, in, out, U, g, kappa, zs, r, partial, stt, shv, k, nrhs, s);
        else
            launch_wilson_v<R, H.value, P.value, O.value, S.value, C.value, 0>(
                mode, in, out, U, g, kappa, zs, r, partial, stt, shv, k, nrhs, s);
    });
}
template void launch_wilson<double>(int, const double2*, double2*, const double2*, const Geom&,
                                    double, double2, const double2*, double4*, const SrcState*,
                                    const ShiftDev*, int, int, hipStream_t, int, int);
template void launch_wilson<float>(int, const float2*, float2*, const float2*, const Geom&,
                                   double, double2, const float2*, double4*, const SrcState*,
                                   const ShiftDev*, int, int, hipStream_t, int, int);

}  // namespace ovl
