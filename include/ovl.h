/*
 * ovl.h -- C ABI of the MI355X (gfx950) library that applies the matrix sign
 * function of the hermitian Wilson-Dirac operator, and the overlap-Dirac
 * operator built from it, through the contour-integral projectors of
 * Nagai & Tomiya, "Extensively parallelizable chiral fermion"
 * (arXiv:2204.01583).
 *
 * What is computed (paper: eqs. (1), (3)-(7)):
 *   sgn(H_W) b  ~=  s = sum_j c_j y_j,   (z_j I - H_W) y_j = b,
 *   D_ov(m_q) b  =  (1+m_q)/2 b + (1-m_q)/2 gamma5 s,
 * with nodes z_j and weights c_j of the N_q-point trapezoidal rule on the
 * two ellipses Gamma_+ (centre +gamma) and Gamma_- (centre -gamma) of eq. (7)
 * (weights of Gamma_- negated, eq. (3)).  All 2 N_q shifted systems are
 * solved from ONE Krylov space of a seed system (z_seed - H_W) x = b by a
 * shifted Galerkin BiCG recurrence (the "shift solver" of the paper's method
 * description; seed z_seed = 1 + 0.05i in the Supplemental Material).
 *
 * Operator conventions (the paper names only H_W = gamma5 D_W(-m0)):
 *   D_W = 1 - kappa sum_mu [ (1-gamma_mu) U_mu(x) psi(x+mu)
 *                           + (1+gamma_mu) U_mu(x-mu)^dag psi(x-mu) ],
 *   kappa = 1/(2(4-m0)); chiral gamma basis, gamma5 = diag(1,1,-1,-1);
 *   a hop that wraps around direction mu is multiplied by bc[mu].
 *
 * Layouts (all complex numbers are interleaved (re, im) IEEE doubles,
 * row-major, contiguous, in DEVICE memory of the context's GPU, owned by the
 * caller; mu = 0..3 is x, y, z, t):
 *   gauge  U    : complex128 [4][Lt][Lz][Ly][Lx][3][3]
 *   spinors     : complex128 [nrhs][Lt][Lz][Ly][Lx][4][3]  (spin, then colour)
 *   force / grad: complex128 [4][Lt][Lz][Ly][Lx][3][3]
 * Scalars passed by host pointer (z_reim, c_reim, dims, bc) are HOST memory.
 *
 * Streams: every call enqueues on the context's HIP stream (ovl_set_stream).
 * Calls that take an ovl_stats* synchronise that stream once at the end and
 * fill it; they return only after the result is complete in `out`.  The
 * solves run on an internal stream of the context (default priority) that
 * waits for the caller's stream on entry and is waited for on exit; the
 * host reads the solver state once per 16 iterations, with the next 16
 * already queued while the residuals are far from the precision switch and
 * the tolerance.
 *
 * Memory: work buffers (internal vectors, the stored basis, job tables) are
 * allocated on the context's device on first use, zero-filled, grown when a
 * later call needs more, and freed by ovl_destroy.
 *
 * Errors: every call returns an int status.  It never aborts or throws.
 * On an error the output buffers are unspecified and ovl_last_error(ctx)
 * holds a message.  A context is not thread-safe; distinct contexts are.
 */
#ifndef OVL_H
#define OVL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define OVL_OK                0
#define OVL_NOT_CONVERGED     1   /* maxiter reached; out holds the last iterate  */
#define OVL_E_ARG           (-1)  /* bad argument (size, pointer, parameter)      */
#define OVL_E_STATE         (-2)  /* a required setter was not called            */
#define OVL_E_HIP           (-3)  /* a HIP runtime call failed                    */
#define OVL_E_OOM           (-4)  /* device allocation failed                     */
#define OVL_E_NONFINITE     (-5)  /* NaN or Inf met in a reduction                */
#define OVL_E_BREAKDOWN     (-6)  /* Krylov pivot <r, A p> vanished               */

/* ---- solver selectors ---------------------------------------------------- */
#define OVL_PREC_FP64   0   /* every vector operation in FP64                                */
#define OVL_PREC_MIXED  1   /* FP64 until the largest shifted residual falls below
                               `switch_res` * ||b||, then FP32 stencil and vectors; the scalar
                               recurrences, weights and the sum stay FP64 (in a batch, each
                               context switches on its own residuals)                         */

#define OVL_FORM_REFERENCE 0 /* per-shift solutions x_j kept in HBM, s = sum c_j x_j at the end */
#define OVL_FORM_FUSED     1 /* per-shift directions p_j only; s accumulated in the same sweep  */
#define OVL_FORM_BASIS     2 /* seed residuals r_k stored; s = sum_k h_k r_k from the scalars    */
#define OVL_FORM_TWOPASS   3 /* as BASIS without storing the r_k: a second pass regenerates them
                                bit for bit (deterministic reductions) and accumulates s       */

typedef struct ovl_ctx ovl_ctx;

typedef struct {
    int32_t iterations;        /* seed iterations of the last apply (max over rhs)          */
    int32_t fp32_iterations;   /* of which in FP32 (OVL_PREC_MIXED)                          */
    int32_t n_shifts;          /* number of shifted systems 2*N_q (or ovl_set_nodes n)       */
    int32_t n_active_end;      /* shifts still above tolerance at the end (0 if converged)   */
    double  max_est_rel_res;   /* max_j ||r_j|| / ||b|| from the recurrence, at the end      */
    double  seconds;           /* wall time of the apply on the stream                       */
    int32_t stencil_variant64; /* stencil choice used in FP64 (autotuned; see ovl_bench_kernel);
                                  1000 + v + 8 f for the fused iteration's variant v and link
                                  format f (basis forms)                                    */
    int32_t stencil_variant32; /* ... in FP32, or -1                                        */
    double  max_true_rel_res;  /* max ||b - (z_j - H) x_j|| / ||b|| over the checked shifts, or
                                  -1 when not checked (see ovl_set_residual_check)           */
    int32_t fp64_repeat;       /* 1 if an OVL_PREC_MIXED apply failed its in-band check and was
                                  solved again in FP64 (the result is the FP64 one), else 0   */
    int32_t reserved;
    double  mixed_true_rel_res;/* with fp64_repeat: the mixed attempt's max_true_rel_res, else -1 */
} ovl_stats;

/* Create a context for a Lx*Ly*Lz*Lt lattice on HIP device `device`.
 * dims = {Lx, Ly, Lz, Lt}, each >= 2; bc = {+1|-1} per direction (paper: the
 * boundary is not stated; the usual choice is {1,1,1,-1}).  `hip_stream` is a
 * hipStream_t or NULL for the null stream.  *ctx receives the context. */
int ovl_create(ovl_ctx** ctx, const int32_t dims[4], const int32_t bc[4],
               int32_t device, void* hip_stream);
int ovl_destroy(ovl_ctx* ctx);
int ovl_set_stream(ovl_ctx* ctx, void* hip_stream);

/* Copy the gauge field U_mu(x) of the Wilson-Dirac operator (paper: the
 * links of D_W in eq. (1); the Numerical experiments section uses quenched
 * SU(3) configurations) from complex128 [4][Lt][Lz][Ly][Lx][3][3] device
 * memory into the context's internal layout; the caller may free U
 * afterwards.  The links are used as given, so H_W stays hermitian for any
 * complex 3x3 links.  When every link is SU(3) to rounding (|U U^dag - 1|
 * and |det U - 1| below 1e-12) the stencil may also store two rows per link
 * and rebuild the third; other fields keep the full matrices.
 * OVL_E_NONFINITE if any entry is NaN or infinite: the context then has no
 * gauge field (operators return OVL_E_STATE) until a valid one is set. */
int ovl_set_gauge(ovl_ctx* ctx, const void* U_dev);

/* m0 > 0 is the negative Wilson mass of H_W = gamma5 D_W(-m0) (paper: after
 * eq. (1); m0 = 1 in the numerical experiments); requires 0 < m0 < 4.
 * mq is the fermion mass of D_ov(m_q) in eq. (1). */
int ovl_set_masses(ovl_ctx* ctx, double m0, double mq);

/* Nodes and weights of eq. (7) on both ellipses: theta_j = 2 pi (j-1/2)/nq,
 * z_j = +-gamma + rho (cos theta_j + i alpha sin theta_j),
 * c_j = +-rho (alpha cos theta_j + i sin theta_j)/nq.  nq counts the points
 * of ONE contour and must be even (an odd nq puts a node on the real axis);
 * 2*nq <= 2048, and the fused and reference forms take at most 1024 shifts
 * (OVL_E_ARG at apply time).  The paper's contour: alpha = 0.1,
 * rho = 1.1999, gamma = 1.2. */
int ovl_set_contour(ovl_ctx* ctx, int32_t nq, double gamma, double rho, double alpha);

/* One contour only: sgn(H_W) = P_+ - P_- and P_+ + P_- = 1 when H_W has no
 * exact zero mode, so sgn(H_W) b ~ 2 P_{Gamma+} b - b from the nq nodes of
 * Gamma_+ (eq. (7), the same parametrisation as ovl_set_contour) with twice
 * their weights: half the shifted systems.  Opt-in: an exact zero mode of
 * H_W gets 2 F_+(0) - 1 (F_+ the Gamma_+ filter; towards -1 as nq grows, the
 * faster the further 0 lies outside Gamma_+) where the sign function and
 * the two-contour form give 0.  nq even, 2 <= nq <= 2048. */
int ovl_set_contour_single(ovl_ctx* ctx, int32_t nq, double gamma, double rho, double alpha);

/* General rational function s = sum_j c_j (z_j - H_W)^-1 b (the resolvent
 * sum of eqs. (5)-(6) with caller-chosen nodes and weights, e.g. a subset of
 * the eq. (7) nodes): n nodes given as interleaved host arrays z_reim[2n],
 * c_reim[2n], 1 <= n <= 2048.  Every Im z_j must be nonzero.  Replaces any
 * contour set before. */
int ovl_set_nodes(ovl_ctx* ctx, int32_t n, const double* z_reim, const double* c_reim);

/* precision: OVL_PREC_*; form: OVL_FORM_*; tol: shift j stops when its
 * residual estimate ||r_j|| <= tol*||b||; maxiter: seed iterations;
 * (zseed_re, zseed_im): seed shift of the shifted BiCG, zseed_im != 0 (the
 * Supplemental Material's numerical setup uses z_seed = 1 + 0.05i);
 * switch_res: the MIXED switch point (ignored for FP64; <= 0 picks 1e-4).
 * precision, form and switch_res go beyond the paper's statement of the
 * problem (which is FP64 with per-shift directions): they select the
 * library's extensions. */
int ovl_set_solver(ovl_ctx* ctx, int32_t precision, int32_t form, double tol, int32_t maxiter,
                   double zseed_re, double zseed_im, double switch_res);

/* True-residual checks of the recurrence's residual estimates (shift j stops
 * on the estimate ||r_k|| / |pi_k^j|, not on its true residual).
 * In-band check (OVL_FORM_BASIS, on by default): after every solve, the
 * shift of each rhs that stayed active longest (ties: the largest final
 * estimate; every converged shift ends just below tol, and the one active
 * longest ran through the most FP32 iterations of a mixed solve) has its solution
 * x_j = sum_i u_i^j r_i rebuilt in the same pass over the stored basis that
 * forms the sum s (one more output vector), and its true residual
 * ||b - (z_j - H_W) x_j|| / ||b|| is computed in FP64 with one more FP64
 * stencil; the maximum over the rhs goes to ovl_stats.max_true_rel_res.  In
 * OVL_PREC_MIXED, when every shift met tol by its estimate but this true
 * residual exceeds the bound of ovl_set_check_bound, the apply is solved
 * again in FP64 (ovl_stats.fp64_repeat = 1); if that misses 10 tol, the call
 * returns OVL_NOT_CONVERGED.  The other forms report -1 for the in-band check.
 * nsample >= 1 adds a synchronous diagnostic after each ovl_apply_sign /
 * ovl_apply_dov: for the nsample shifts of each rhs first in that order (the
 * reference form: largest final estimate), x_j is formed (stored by OVL_FORM_REFERENCE, rebuilt from the
 * stored basis by OVL_FORM_BASIS) and its true residual computed with one
 * more stencil; max_true_rel_res becomes the maximum of both checks.
 * nsample = 0 (default) keeps the in-band check only; nsample = -1 turns the
 * in-band check off as well.  nsample in [-1, 64], else OVL_E_ARG. */
int ovl_set_residual_check(ovl_ctx* ctx, int32_t nsample);

/* The bound on the in-band true residual above which an OVL_PREC_MIXED apply
 * is repeated in FP64 (see ovl_set_residual_check).  The FP32 phase, which
 * starts once every shifted residual is below switch_res, adds to the true
 * residual a drift of a few eps32 * switch_res (eps32 = 2^-24; measured 2 to
 * 3 eps32 switch_res at 16^4) that the recurrence's estimates do not see; bound = 0 (default) takes
 * max(10 tol, 10 eps32 switch_res), so only more drift than that triggers the
 * repeat.  A caller that needs every apply's true residual within 10 tol sets
 * bound = 10 tol (mixed applies whose drift exceeds it then cost an FP64
 * solve more).  OVL_E_ARG for a negative or non-finite bound. */
int ovl_set_check_bound(ovl_ctx* ctx, double bound);

/* out = H_W in for nrhs spinors (eq. (1): H_W = gamma5 D_W(-m0)).  out must
 * not alias in. */
int ovl_apply_hw(ovl_ctx* ctx, const void* in, void* out, int32_t nrhs);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * out = H_W in as ovl_apply_hw, with the same argument rules, that allocates
 * nothing.  Its work buffers (the packed input and output, 2 nrhs 12 Vt
 * complex128, Vt the volume rounded up to 64 sites) live in a static device
 * array of 64 MiB per GPU, held until the process ends; a larger request
 * returns OVL_E_ARG.  The stencil choice is the one ovl_apply_hw already
 * tuned for this nrhs on this context, else the untuned default: the tuner,
 * which allocates, is never run.  Every context on one GPU shares that GPU's
 * array, so calls that overlap on one GPU (other streams, other threads)
 * race.  The gauge field must be set (ovl_set_gauge allocates). */
int ovl_apply_hw_noalloc(ovl_ctx* ctx, const void* in, void* out, int32_t nrhs);

/* The same operator through the FP32 stencil that OVL_PREC_MIXED uses after
 * its switch: `in` is rounded to complex64, the links are the context's FP32
 * copy, the arithmetic is FP32, and the result is widened to complex128 in
 * `out` (same layouts and argument rules as ovl_apply_hw).  For checking the
 * FP32 kernels; expect relative errors of order 1e-7. */
int ovl_apply_hw_fp32(ovl_ctx* ctx, const void* in, void* out, int32_t nrhs);

/* out = sum_j c_j (z_j - H_W)^-1 in  (eqs. (5)-(7)) for nrhs spinors.
 * Returns OVL_NOT_CONVERGED (out = last iterate) if maxiter is reached.
 * st may be NULL. */
int ovl_apply_sign(ovl_ctx* ctx, const void* in, void* out, int32_t nrhs, ovl_stats* st);

/* out = D_ov(m_q) in = (1+m_q)/2 in + (1-m_q)/2 gamma5 sgn(H_W) in  (eq. (1)). */
int ovl_apply_dov(ovl_ctx* ctx, const void* in, void* out, int32_t nrhs, ovl_stats* st);

/* Derivative of S = phi^dag D_ov^dag D_ov phi (one phi) with respect to the
 * links (eq. (1) with the resolvent form of the sign under eq. (4); the
 * paper gives no force), through adjoint shifted solves:
 * dS = 2 Re sum_j c_j X_j^dag dH Y_j, Y_j = (z_j-H)^-1 phi,
 * X_j = (conj z_j - H)^-1 psi, psi = (1-m_q)/2 gamma5 D_ov phi.
 * kind 0: the traceless hermitian force F with dS/dh = sum tr(Omega F) for
 *         U -> exp(i h Omega) U;  kind 1: the complex gradient G with
 *         dS = Re sum conj(G) dU (PyTorch's convention);  kind 2: S only
 *         (one solve; grad is not touched and may be NULL).
 * *action (host, may be NULL) receives S.  Two basis-form solves (phi, then
 * psi at the conjugate nodes) keep their stored bases side by side; the
 * shifted solutions Y_j and X_j are never all held: they are rebuilt from the
 * bases shift_chunk shifts at a time (<= 0: all at once) and contracted per
 * link, so the work space is the two bases plus 2 shift_chunk vectors. */
int ovl_force(ovl_ctx* ctx, const void* phi, void* grad, int32_t kind, int32_t shift_chunk,
              double* action, ovl_stats* st);

/* ovl_apply_sign for several contexts (different lattices allowed) at once
 * (eqs. (5)-(7) for every context, the independent (field, source) problems
 * of the Numerical experiments gathered into one solve):
 * out[i] = sum_j c_j (z_j - H_W[ctx i])^-1 in[i] with nrhs[i] spinors; every
 * context must have its gauge field and masses set.  The node set and solver
 * settings of ctxs[0] are used for every context during the call (each
 * context's own settings are restored afterwards).  All contexts must be on
 * one device, 1 <= nctx <= 64.  Each seed-iteration stage is ONE kernel launch
 * per precision over a job table of all contexts; chunks of 16 iterations are
 * captured once as a HIP graph and replayed (OVL_GRAPHS=0 launches eagerly
 * instead).  In MIXED precision every context switches to FP32 on its own
 * residuals, at a 16-iteration boundary: while some iterate in FP64 and
 * others in FP32, each stage runs the FP64 and the FP32 launch.  The
 * work follows ctxs[0]'s stream.  st (may be NULL) receives the aggregate:
 * max iterations, summed active shifts, max residual estimate. */
int ovl_apply_sign_batched(ovl_ctx* const* ctxs, int32_t nctx, const void* const* in,
                           void* const* out, const int32_t* nrhs, ovl_stats* st);

/* Stats of the last apply on this context. */
int ovl_get_stats(const ovl_ctx* ctx, ovl_stats* st);

/* Time one internal kernel on the context's stream with HIP events: `reps`
 * back-to-back launches after one warm-up, average milliseconds in *avg_ms
 * and the algorithmic bytes of one launch in *bytes.  which:
 *   0: FP64 stencil (out = H_W in) on nrhs internal spinors, autotuned variant
 *   1: the same in FP32
 *   100+c, 200+c: FP64 / FP32 stencil choice c = v + 28 f: variant v and
 *      link format f (0: full 3x3 links; 1: the first two rows, the third
 *      rebuilt in the kernel, for SU(3) fields only).  Variants 0..23 are
 *      16 tile + 8 (lanes per site - 1) + 4 order + 2 (rhs per lane - 1)
 *      + (hops per loop step - 1): one or two hops per loop step; one or two
 *      rhs per lane sharing each link load; blocks ordered rhs-fastest or
 *      site-fastest; one lane per site or two (forward and backward hops);
 *      the block's sites of every rhs staged in LDS (one lane per site).
 *      Variants 24..27 stage the forward links of a 256-site tile in LDS,
 *      shared by the 2 or 4 rhs of a block: 24 + 2 (4 rhs) + (hops - 1).
 * The first use of a (lattice, nrhs, precision, form) picks the fastest
 * choice by timing every variant in every allowed link format;
 * OVL_STENCIL_VARIANT=v forces variant v (two-row links for SU(3) fields
 * unless OVL_LINKS=full), OVL_AUTOTUNE=0 keeps variant 0, and
 * OVL_AUTOTUNE_CACHE=path persists the choices as a JSON object, and
 * OVL_AUTOTUNE_VERBOSE=1 prints every candidate's time to stderr.  The basis
 * forms time their stencil inside the solve (a chunk of a real solve from
 * its initial state, discarded; the four fastest choices are timed twice
 * more and each keeps its fastest run).  OVL_FUSED=1, read when a context is created, makes
 * the basis forms run one fused kernel per seed
 * iteration instead of the stencil and update kernels (slower on MI355X;
 * kept as a parity-tested alternative), with OVL_ITER_VARIANT=v forcing its
 * variant v < 8.
 * Buffers are internal scratch (contents arbitrary but finite). */
int ovl_bench_kernel(ovl_ctx* ctx, int32_t which, int32_t nrhs, int32_t reps,
                     double* avg_ms, double* bytes);

/* Per-kernel timing of the solver's own launches, for benchmarks.  While
 * enabled, the solver launches eagerly (no graph replay) and times every
 * launch of the classes below with HIP events on the context's stream: the
 * kernels of classes 0-5 are launched with hipExtLaunchKernel, whose events
 * take the kernel's own start and end; the others are bracketed by event
 * records, which adds their dispatch latency.  ovl_get_profile returns the
 * summed duration, the number of launches and the summed algorithmic bytes
 * since the last ovl_set_profiling(ctx, 1).  kclass:
 *   0 stencil FP64 (q = z_s p - H p with <r,q>,   1 the same in FP32
 *     ||q||^2 and ||r||^2)
 *   2 r and p update FP64 (one kernel)             3 the same in FP32
 *   4 r update with the shift sweep FP64           5 the same in FP32
 *   6 basis sum s = sum h_k r_k                    7 scalar kernels
 *   8 fused iteration FP64 (basis forms: r_k and   9 the same in FP32
 *     q_k = A r_k + beta q_{k-1} in one kernel)
 * Algorithmic bytes count every array element the kernel must read or write
 * once (links once per launch, neighbour spinors once); for classes 0-3, 8
 * and 9 they count the sources still iterating in each launch (a launch in
 * which every source has finished returns at once: it adds its time, and no
 * bytes).  Class 8/9 moves per live source r_{k-1} and q_{k-1} (read) and r_k
 * and q_k (written), plus the links once per launch. */
int ovl_set_profiling(ovl_ctx* ctx, int32_t enable);
int ovl_get_profile(const ovl_ctx* ctx, int32_t kclass, double* total_ms, int64_t* launches,
                    double* bytes);

/* Spectral bounds of H_W from the last solve's seed recurrence, a Lanczos
 * process on H_W, for rhs `src` of the last apply: bounds[0] and bounds[1]
 * are the smallest and largest Ritz value (inside the spectrum's hull and
 * converging to its ends first), bounds[2] the square root of the smallest
 * Ritz value of H_W^2 on the same Krylov space, an upper bound on
 * min |lambda| (the gap the contour has to resolve) that converges to it.
 * OVL_E_STATE before any apply. */
int ovl_spectral_bounds(ovl_ctx* ctx, int32_t src, double* bounds);

/* A circle contour (alpha = 1) for ovl_set_contour from a spectral gap
 * (smallest |eigenvalue| of H_W, > 0) and the largest |eigenvalue|: centre
 * gamma and radius rho put Gamma_+ from 1e-4 gap to 1.05 lmax, and nq is the
 * smallest even count whose two-contour filter error at |lambda| = gap and
 * at |lambda| = lmax (the circle's closed form, 1 - F(|lambda|) + F(-|lambda|)
 * with F(lambda) = 1/(1 + ((lambda - gamma)/rho)^nq)) is below `target`.
 * OVL_E_ARG for a bad input or when 2 nq would exceed 2048. */
int ovl_suggest_contour(double gap, double lmax, double target, int32_t* nq, double* gamma,
                        double* rho);

const char* ovl_status_string(int status);
const char* ovl_last_error(const ovl_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* OVL_H */
