// Launch wrappers of the HIP kernels (internal to the library).
#pragma once
#include "ovl_common.h"

namespace ovl {

// ---- layout conversion -----------------------------------------------------
// ext [n][V][12] complex128  <->  internal [n][12][V] (double2 or float2)
void launch_pack_spinor64(const double2* ext, double2* in, int64_t V, int n, hipStream_t s);
void launch_pack_spinor32(const double2* ext, float2* in, int64_t V, int n, hipStream_t s);
void launch_unpack_spinor64(const double2* in, double2* ext, int64_t V, int n, hipStream_t s);
// out_ext = a*b_ext + bm*gamma5*s_int  (D_ov assembly, eq. (1))
void launch_unpack_dov(const double2* s_int, const double2* b_ext, double2* out_ext, double a,
                       double bm, int64_t V, int n, hipStream_t s);
// ext [4][V][9] complex128 -> [4][9][V] FP64 and FP32, boundary signs folded into
// the links on the last slice of each direction.
void launch_pack_gauge(const double2* ext, double2* U64, float2* U32, const Geom& g,
                       const int bc[4], hipStream_t s);
void launch_convert_64_to_32(const double2* a, float2* b, int64_t n, hipStream_t s);

// ---- Wilson stencil --------------------------------------------------------
// out = H_W in                                      (mode 0)
// out = zs*in - H_W in, partial[src][blk] = <r,out> (mode 1, per-block dot)
// `done` (mode 1, may be null) skips converged sources.
template <typename R>
void launch_wilson(int mode, const C2<R>* in, C2<R>* out, const C2<R>* U, const Geom& g,
                   double kappa, double2 zs, const C2<R>* r, double2* partial,
                   const SrcState* stt, int nrhs, hipStream_t s);
int wilson_blocks(const Geom& g);

// ---- Krylov scalars and vector updates --------------------------------------
int elem_blocks(int64_t n12);
// alpha_k and shifted pi_{k+1}, alpha^j (one block per source)
void launch_alpha(SrcState* st, const double2* partial, int nblk, const double2* dz,
                  const double2* pi, const double2* pi_prev, double2* pi_next, double2* aj,
                  const int* active, int J, int nsrc, hipStream_t s);
// r_out = r_in - alpha q ; partial[src][blk] = ||r_out||^2
template <typename R>
void launch_update_r(const C2<R>* rin, C2<R>* rout, const C2<R>* q, const SrcState* st,
                     double* partial, int64_t n12, int64_t src_stride_in,
                     int64_t src_stride_out, int nsrc, hipStream_t s);
// beta, beta^j, residual estimates, deactivation, sweep list (one block per source).
// form: 0 reference (list coefficient alpha^j), 1 fused (c_j alpha^j),
// 2 basis (records history, list coefficient c_j alpha^j).
struct BetaArgs {
    SrcState* st; const double* partial; int nblk;
    const double2* c; double2* pi; double2* pi_prev; const double2* pi_next; const double2* aj;
    int* active; int J;
    int* lst_j; double2* lst_a; double2* lst_ipi; double2* lst_b;
    double tol;
    // history (basis forms), may be null: [src][maxk+1][J]
    double2* h_a; double2* h_b; double2* h_pi; int maxk;
};
void launch_beta(const BetaArgs& a, int nsrc, hipStream_t s);
// fused sweep: s += sum_l lst_a[l] p_{j_l};  p_{j_l} = r*lst_ipi + lst_b p_{j_l};  p = r + beta p
template <typename R>
void launch_sweep_fused(const C2<R>* r, C2<R>* p, C2<R>* pj, double2* sacc, const double2* b0,
                        const SrcState* st, const int* lst_j, const double2* lst_a,
                        const double2* lst_ipi, const double2* lst_b, int J, int64_t n12,
                        int nsrc, bool first, hipStream_t s);
// reference sweep: x_j += alpha^j p_j (x_j FP64); p_j update; seed p update
template <typename R>
void launch_sweep_ref(const C2<R>* r, C2<R>* p, C2<R>* pj, double2* xj, const double2* b0,
                      const SrcState* st, const int* lst_j, const double2* lst_a,
                      const double2* lst_ipi, const double2* lst_b, int J, int64_t n12,
                      int nsrc, bool first, hipStream_t s);
void launch_sum_ref(const double2* xj, const double2* c, double2* sacc, int J, int64_t n12,
                    int nsrc, hipStream_t s);
// p = r + beta p
template <typename R>
void launch_update_p(const C2<R>* r, C2<R>* p, const SrcState* st, int64_t n12,
                     int64_t src_stride_r, int nsrc, hipStream_t s);

// ||b||^2 and the initial solver state (r = p = b, pi = 1, all shifts active)
void launch_init_state(SrcState* st, const double2* b, double* partial, int64_t n12, double2* pi,
                       double2* pi_prev, int* active, int J, double2* h_pi, int maxk, int nsrc,
                       hipStream_t s);

// ---- basis forms ------------------------------------------------------------
// h[src][i] = sum_j c_j P_i^j / pi_i^j with P_i = alpha_i^j + beta_i^j P_{i+1}
void launch_basis_coef(const double2* h_a, const double2* h_b, const double2* h_pi,
                       const double2* c, const SrcState* st, double2* W, double2* h, int J,
                       int maxk, int nsrc, hipStream_t s);
// s[src] (+)= sum_{l in [l0,l1)} h[src][g0+l] * slot_l[src] over one chunk of slots of type R
template <typename R>
void launch_basis_gemv(const void* slots, int64_t slot_stride, int64_t src_stride,
                       const double2* h, int maxk, const SrcState* st, int g0, int l0, int l1,
                       double2* sacc, bool accumulate, int64_t n12, int nsrc, hipStream_t s);

}  // namespace ovl
