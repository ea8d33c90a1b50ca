// Launch wrappers of the HIP kernels (internal to the library).
#pragma once
#include "ovl_common.h"

namespace ovl {

// ---- layout conversion -----------------------------------------------------
// ext [n][V][12] complex128  <->  internal tiled [n][Vt/64][12][64] (double2 or
// float2); the sites from V to Vt are not touched
void launch_pack_spinor64(const double2* ext, double2* in, int64_t V, int64_t Vt, int n,
                          hipStream_t s);
void launch_pack_spinor32(const double2* ext, float2* in, int64_t V, int64_t Vt, int n,
                          hipStream_t s);
void launch_unpack_spinor64(const double2* in, double2* ext, int64_t V, int64_t Vt, int n,
                            hipStream_t s);
void launch_unpack_spinor32(const float2* in, double2* ext, int64_t V, int64_t Vt, int n,
                            hipStream_t s);
// out_ext = a*b_ext + bm*gamma5*s_int  (D_ov assembly, eq. (1))
void launch_unpack_dov(const double2* s_int, const double2* b_ext, double2* out_ext, double a,
                       double bm, int64_t V, int64_t Vt, int n, hipStream_t s);
// ext [4][V][9] complex128 -> tiled [4][Vt/64][9][64] FP64 and FP32 and the
// two-row form [4][Vt/64][6][64], boundary signs (g.bc) folded into the links on the last slice of
// each direction; defect[4][gauge_blocks] = per-block max of
// max(|U U^dag - 1|, |det U - 1|) over the input links (NaN propagates).
int gauge_blocks(const Geom& g);
void launch_pack_gauge(const double2* ext, double2* U64, float2* U32, double2* U64c, float2* U32c,
                       const Geom& g, double* defect, hipStream_t s);
void launch_convert_64_to_32(const double2* a, float2* b, int64_t n, hipStream_t s);
// y += a x (complex vectors, real a)
void launch_axpy(double2* y, const double2* x, double a, int64_t n, hipStream_t s);

// ---- Wilson stencil --------------------------------------------------------
// out = H_W in                                               (mode 0)
// out = zs*in - H_W in, partial[src][blk] = (<r,out>, ||out||^2, ||r||^2) (mode 1); sources that are
// not live at iteration k (see kernels.hip) are skipped.
// variant v = 16*tile + 8*(lanes per site - 1) + 4*order +
// 2*(rhs per lane - 1) + (hops per loop step - 1): hops per step 1 or 2, 1 or
// 2 rhs per lane sharing each link load, block order 0 (rhs fastest) or 1
// (sites fastest), 1 lane per site (all 8 hops) or 2 (forward and backward
// hops on neighbouring lanes, 512-thread blocks), and (v >= 16, one lane per
// site) the block's 256 sites staged in LDS for the neighbours inside it.
// Variants 24 .. 27 keep one lane per site and rhs and stage the forward
// links of a 256-site tile in LDS, shared by the 2 or 4 rhs of the block
// (bit 1) with 1 or 2 hops per loop step (bit 0).
constexpr int kShapeVariants = 24;
constexpr int kStencilVariants = 28;
// lnk = 1: U holds the first two rows of every link ([mu][Vt/64][6][64]) and
// the stencil rebuilds the third (SU(3) fields); lnk = 0: full [mu][Vt/64][9][64]
template <typename R>
void launch_wilson(int mode, const C2<R>* in, C2<R>* out, const C2<R>* U, const Geom& g,
                   double kappa, double2 zs, const C2<R>* r, double4* partial,
                   const SrcState* stt, const ShiftDev* sh, int k, int nrhs, hipStream_t s,
                   int variant, int lnk);
int wilson_blocks(const Geom& g);

// ---- seed iteration over a job table (device-side iteration counter kdev) --
// Blocks per source of the vector kernels (see kernels.hip).
int vec_blocks(int64_t n12, int nslices, bool slice_blocks);
// Doubles launch_init_state writes into its partial buffer (nsrc sources).
size_t init_partials(int64_t n12, int nslices, int nsrc);
int wilson_grid_blocks(const Geom& g, int nrhs, int variant);
// K1 for every job: q = z_s p - H p, <r_k, q> partials.  For this launch and
// the next: non-null ev0/ev1 take the kernel's own start and end timestamps
// (hipExtLaunchKernel), for per-kernel timing without marker packets.
template <typename R>
void launch_wilson_jobs(const JobDesc* jobs, int njobs, const int* kdev, int total_blocks,
                        int variant, int lnk, hipStream_t s, hipEvent_t ev0 = nullptr,
                        hipEvent_t ev1 = nullptr);
// K2: seed and shift scalars, shift bookkeeping, r update and p update or
// sweep; reads the iteration index from kread and writes its successor to kwrite
template <typename R>
void launch_iteration_update(const JobDesc* jobs, int njobs, const int* kread, int* kwrite,
                             int vec_blocks_total, int form, int maxJ, hipStream_t s,
                             hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// The fused one-kernel seed iteration of the basis forms (stencil.hip): kernel
// k forms r_k and q_k = A r_k + beta q_{k-1} without the direction p, and
// advances the shifts by iteration k-1; reads k from kread, writes k + 1 to
// kwrite.  Variants 0 .. kIterVariants-1: hops per loop step (bit 0), block
// order (bit 1), LDS tile of the block's r_k (bit 2).
constexpr int kIterVariants = 8;
int iter_grid_blocks(const Geom& g, int nrhs);
template <typename R>
void launch_iter_jobs(const JobDesc* jobs, int njobs, const int* kread, int* kwrite,
                      int total_blocks, int variant, int lnk, hipStream_t s,
                      hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// job->phase = phase (0 FP64, 1 FP32) in stream order
void launch_set_phase(JobDesc* job, int phase, hipStream_t s);
// state block of every job into its pinned host slot (k / chunk) & 1, with k
// read from kdev (the iteration counter after a chunk)
void launch_export_state(const JobDesc* jobs, int njobs, const int* kdev, int chunk,
                         hipStream_t s);
// two-pass form, second pass: s = h_0 b
void launch_s_init(const double2* b, const double2* h, int maxk, double2* s, int64_t n12, int nsrc,
                   hipStream_t st);
void launch_sum_ref(const double2* xj, const double2* c, double2* sacc, int J, int64_t n12,
                    int nsrc, hipStream_t s);
// ||b||^2 and the iteration-0 state
void launch_init_state(SrcState* st, const double2* b, double* partial, int64_t n12,
                       const ShiftDev& sh, hipStream_t s);

// ---- basis forms ------------------------------------------------------------
// h[src][i] = sum_j c_j P_i^j / pi_i^j with P_i = alpha_i^j + beta_i^j P_{i+1}
void launch_basis_coef(const double2* h_a, const double2* h_b, const double2* h_pi,
                       const double2* c, const SrcState* st, double2* W, double2* h, int J,
                       int maxk, int nsrc, hipStream_t s);
// s_n = sum_{i < min(kend, iter_n + 1)} h[n][i] r_i over every stored slot in
// one launch (and x_n with the coefficients hx when non-null); slots below
// ksw FP64, from ksw FP32; chunks is the device table of slot-chunk bases
void launch_basis_sum(char* const* chunks, size_t slot_bytes, int kend, int ksw, const double2* h,
                      const double2* hx, int maxk, const SrcState* st, double2* sacc, double2* xc,
                      int64_t n12, int nsrc, hipStream_t s);
// per source, the shift that stayed active longest (latest nonzero basis
// coefficient), ties to the largest final residual estimate: its basis
// coefficients W[src][i][j] into hx[src][i] and its node z[j] into zc[src]
void launch_pick_check(const double* res, const double2* W, const double2* z, const SrcState* st,
                       int J, int maxk, int nsrc, double2* hx, double2* zc, hipStream_t s);

// ---- force ------------------------------------------------------------------
// d = a b + bm gamma5 s, psi = bm gamma5 d, partial[blk] = |d|^2 (one source,
// tiled layout of Vt sites)
void launch_dov_psi(const double2* b, const double2* s, double2* psi, double a, double bm,
                    int64_t Vt, double* partial, int nblk, hipStream_t st);
// Y[j] = sum_{i < K} u_i^{j0+j} r_i, j < jn, for the source whose slot
// elements start at element eoff (W already offset to that source); chunks is
// the device table of slot-chunk bases (slot i in chunk i / kSlotChunk),
// slots below ksw hold FP64, from ksw on FP32
void launch_materialize(char* const* chunks, size_t slot_bytes, int K, int ksw, const double2* W,
                        int J, int j0, int jn, double2* Y, int64_t n12, int64_t eoff,
                        hipStream_t s);
// partial[blk] = (|b - (z x - H x)|^2, |b|^2) per block over one source
void launch_true_res(const double2* b, const double2* x, const double2* hx, double2 z,
                     double2* partial, int nblk, int64_t n12, hipStream_t s);
// the same for nsrc sources (source n against node zc[n]); partial[n][blk]
void launch_true_res_multi(const double2* b, const double2* x, const double2* hx,
                           const double2* zc, double2* partial, int nblk, int64_t n12, int nsrc,
                           hipStream_t s);
// per-link accumulation of sum_j c_j X_j^dag dH Y_j; on the last chunk writes
// the complex gradient (kind 1) or the traceless hermitian force (kind 0)
void launch_force(const double2* X, const double2* Y, const double2* c, int jn, const Geom& g,
                  const double2* Uint, const int bc[4], double kappa, double2* acc, bool first,
                  bool last, int kind, double2* out, hipStream_t s);

}  // namespace ovl
