// Host side of the library: contexts, argument checks, contour tables and the
// shifted-solver driver that enqueues the kernels of kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/ovl.h"
#include "kernels.h"

using namespace ovl;

// Scratch of ovl_apply_hw_noalloc: the packed input and output spinors of one
// call.  One copy per GPU, held until the process ends.  In host code the
// name is a host-side stand-in, not a device address: kernels and copies
// use the per-device address from hipGetSymbolAddress (scratch_address).
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

namespace {

// Device address of `scratch` on each device, looked up once per device with
// that device current (ovl_create); null until then or if the lookup failed.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {nullptr};
bool g_scratch_done[kMaxDevices] = {false};

void* scratch_address(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_done[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e == hipSuccess) {
            g_scratch_ptr[device] = ptr;
            g_scratch_done[device] = true;
        } else {
            (void)hipGetLastError();
        }
    }
    return g_scratch_ptr[device];
}

// A device allocation that only grows.  New memory is zeroed before ensure
// returns, so the padding sites of the tiled layouts start at zero; every
// kernel keeps them there.
struct DBuf {
    void* p = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t nb) {
        if (nb <= bytes) return hipSuccess;
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        hipError_t e = hipMalloc(&p, nb);
        if (e == hipSuccess) e = hipMemsetAsync(p, 0, nb, nullptr);
        if (e == hipSuccess) e = hipStreamSynchronize(nullptr);  // the fill, not other streams' work
        if (e == hipSuccess) {
            bytes = nb;
        } else if (p) {
            (void)hipFree(p);
            p = nullptr;
        }
        return e;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <typename T> T* as() const { return static_cast<T*>(p); }
};

}  // namespace

struct ovl_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    Geom g{};
    int bc[4] = {1, 1, 1, -1};
    double m0 = 0.0, mq = 0.0;
    bool masses_set = false, gauge_set = false;
    // nodes and weights (host, FP64)
    std::vector<double2> z, c;
    double c0 = 0.0;  // constant term: s = c0 b + sum_j c_j (z_j - H)^-1 b
    // solver settings
    int precision = OVL_PREC_FP64;
    int form = OVL_FORM_FUSED;
    double tol = 1e-12;
    int maxiter = 4000;
    double2 zseed = make_double2(1.0, 0.05);
    double switch_res = 1e-4;
    int poll = 8;  // iterations between convergence polls
    // OVL_FUSED=1: the basis forms run the fused one-kernel iteration instead
    // of the two-kernel one (stencil, then update)
    bool fused_iter = false;
    void* scratch = nullptr;  // this device's address of the ovl_apply_hw_noalloc scratch
    // device buffers
    DBuf U64, U32;    // links, tiled [mu][Vt/64][9][64], boundary sign folded in
    DBuf U64c, U32c;  // rows 0 and 1 only, [mu][Vt/64][6][64] (SU(3) fields)
    bool links12 = false;  // the field is SU(3): the stencil rebuilds row 2
    DBuf hw_in, hw_out;
    // p64: the solution rebuilt for the in-band residual check
    DBuf b64, r64, p64, q64, r32, q32, s64, pj64, pj32, xj;
    std::vector<DBuf> slot_chunks;   // basis forms: kSlotChunk residual slots each
    size_t slot_chunk_bytes = 0;
    DBuf part_w, part_b, state, shifts, lists, nodes_dev, hist, W, h, seed;
    // iterations per rhs and maxk of the last solve, whose seed scalars stay in
    // `seed` until the next one (for ovl_spectral_bounds)
    std::vector<int> last_iters;
    int last_maxk = 0;
    SrcState* host_state = nullptr;  // pinned mirror
    int host_state_n = 0;
    DBuf bench_a, bench_b, bench_c, tune_state, tune_flush, chk;
    int check_n = 0;  // shifts per source whose true residual is checked after a solve
    // in-band check (basis form): the true residual of one shift per source
    // (the one active longest), fused into the final basis sum; off when false
    bool inband_check = true;
    double check_bound = 0.0;  // > 0: the mixed repeat bound set by the caller
    DBuf chkdev;                   // hx [nsrc][maxk+1] | zc [nsrc] | partials [nsrc][kChkBlocks]
    double2* chk_host = nullptr;   // pinned copy of the partials
    size_t chk_host_bytes = 0;
    DBuf fY, fX, fpsi, facc, fc, fpart;  // force work space
    // the force keeps the first solve's basis (slot chunks, their device
    // table) and coefficients here while the second solve runs
    std::vector<DBuf> fslot_chunks;
    DBuf fslot_table, fW;
    DBuf slot_table;                       // basis form: device table of slot-chunk bases
    // solve stream (graphs cannot be captured on the legacy null stream) and handoff events
    hipStream_t ws = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    DBuf jobs_dev;                         // batch lead: JobDesc table + iteration counter
    // chunk graphs by precision mode (1 FP64 jobs only, 2 FP32 only, 3 both)
    struct GraphCache { std::string key; hipGraphExec_t exec = nullptr; } graphs[3];
    // per-kernel-class event timing (ovl_set_profiling)
    static constexpr int kClasses = 10;
    bool prof_on = false;
    std::vector<hipEvent_t> ev_pool;
    struct ProfRec { int cls; int ev; double bytes; };
    std::vector<ProfRec> prof_pending;
    double prof_ms[kClasses] = {0};
    int64_t prof_n[kClasses] = {0};
    double prof_bytes[kClasses] = {0};
    // stencil variant chosen per (nrhs, precision + 2 mode) by the autotuner
    std::map<std::pair<int, int>, int> stencil_variant;
    ovl_stats last{};
    char err[512] = {0};
};

namespace {

int fail(ovl_ctx* ctx, int code, const char* fmt, ...) {
    if (ctx) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(ctx->err, sizeof(ctx->err), fmt, ap);
        va_end(ap);
    }
    return code;
}

#define HIPCHK(ctx, call)                                                                   \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail((ctx), e_ == hipErrorOutOfMemory ? OVL_E_OOM : OVL_E_HIP,           \
                        "%s failed: %s", #call, hipGetErrorString(e_));                      \
    } while (0)

int check_dev_ptr(ovl_ctx* ctx, const void* p, const char* name) {
    if (p == nullptr) return fail(ctx, OVL_E_ARG, "%s is NULL", name);
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, OVL_E_ARG, "%s is not a HIP device pointer", name);
    }
    if (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged)
        return fail(ctx, OVL_E_ARG, "%s is not device memory", name);
    if (at.device != ctx->device)
        return fail(ctx, OVL_E_ARG, "%s lives on device %d, context is on device %d", name,
                    at.device, ctx->device);
    return OVL_OK;
}

// [a, a+na) and [b, b+nb) intersect
bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
    const char* x = static_cast<const char*>(a);
    const char* y = static_cast<const char*>(b);
    return x < y + nb && y < x + na;
}

double kappa_of(double m0) { return 1.0 / (2.0 * (4.0 - m0)); }

// elements of one source: internal (tiled, Vt sites) and caller layout (V sites)
int64_t n12(const ovl_ctx* ctx) { return 12 * ctx->g.Vt; }
int64_t n12_ext(const ovl_ctx* ctx) { return 12 * ctx->g.V; }
// A stencil choice is code = variant + kStencilVariants * lnk: the variant
// (0 .. kStencilVariants-1) and the link format (lnk = 1: the two-row form,
// only for SU(3) fields).  The links the stencil reads for a format:
template <typename R> const C2<R>* stencil_links(const ovl_ctx* ctx, int lnk);
template <> const double2* stencil_links<double>(const ovl_ctx* ctx, int lnk) {
    return lnk ? ctx->U64c.as<double2>() : ctx->U64.as<double2>();
}
template <> const float2* stencil_links<float>(const ovl_ctx* ctx, int lnk) {
    return lnk ? ctx->U32c.as<float2>() : ctx->U32.as<float2>();
}

struct DeviceGuard {
    int prev = 0;
    explicit DeviceGuard(int d) {
        (void)hipGetDevice(&prev);
        if (prev != d) (void)hipSetDevice(d);
    }
    ~DeviceGuard() {
        int cur = 0;
        (void)hipGetDevice(&cur);
        if (cur != prev) (void)hipSetDevice(prev);
    }
};

// Times one launch of class `cls` (profiling only): by default two marker
// events bracket the launch; with kernel_events the caller hands start() and
// stop() to a hipExtLaunchKernel launch instead, which stamps them with the
// kernel's own start and end, free of the markers' dispatch overhead.
struct ProfScope {
    ovl_ctx* ctx;
    hipStream_t st;
    int idx = -1;
    bool ext;
    ProfScope(ovl_ctx* c, hipStream_t s, int cls, double bytes, bool kernel_events = false)
        : ctx(c), st(s), ext(kernel_events) {
        if (!ctx->prof_on) return;
        const size_t need = 2 * (ctx->prof_pending.size() + 1);
        while (ctx->ev_pool.size() < need) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return;
            ctx->ev_pool.push_back(e);
        }
        idx = (int)ctx->prof_pending.size();
        ctx->prof_pending.push_back({cls, 2 * idx, bytes});
        if (!ext) (void)hipEventRecord(ctx->ev_pool[2 * idx], st);
    }
    hipEvent_t start() const { return idx >= 0 && ext ? ctx->ev_pool[2 * idx] : nullptr; }
    hipEvent_t stop() const { return idx >= 0 && ext ? ctx->ev_pool[2 * idx + 1] : nullptr; }
    ~ProfScope() {
        if (idx >= 0 && !ext) (void)hipEventRecord(ctx->ev_pool[2 * idx + 1], st);
    }
};

// After a stream synchronisation: fold the pending event pairs into the totals.
void prof_collect(ovl_ctx* ctx) {
    for (const auto& r : ctx->prof_pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ctx->ev_pool[r.ev], ctx->ev_pool[r.ev + 1]) == hipSuccess) {
            ctx->prof_ms[r.cls] += ms;
            ctx->prof_n[r.cls] += 1;
            ctx->prof_bytes[r.cls] += r.bytes;
        }
    }
    ctx->prof_pending.clear();
}

}  // namespace

extern "C" int ovl_set_profiling(ovl_ctx* ctx, int32_t enable) {
    if (!ctx) return OVL_E_ARG;
    ctx->prof_on = enable != 0;
    ctx->prof_pending.clear();
    for (int i = 0; i < ovl_ctx::kClasses; ++i) {
        ctx->prof_ms[i] = 0;
        ctx->prof_n[i] = 0;
        ctx->prof_bytes[i] = 0;
    }
    return OVL_OK;
}

extern "C" int ovl_get_profile(const ovl_ctx* ctx, int32_t kclass, double* total_ms,
                               int64_t* launches, double* bytes) {
    if (!ctx || kclass < 0 || kclass >= ovl_ctx::kClasses || !total_ms || !launches || !bytes)
        return OVL_E_ARG;
    *total_ms = ctx->prof_ms[kclass];
    *launches = ctx->prof_n[kclass];
    *bytes = ctx->prof_bytes[kclass];
    return OVL_OK;
}

// ============================================================================
// context
// ============================================================================
extern "C" int ovl_create(ovl_ctx** out, const int32_t dims[4], const int32_t bc[4],
                          int32_t device, void* hip_stream) {
    if (out == nullptr || dims == nullptr) return OVL_E_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
        (void)hipGetLastError();
        return OVL_E_HIP;
    }
    if (device < 0 || device >= ndev) return OVL_E_ARG;
    int64_t V = 1;
    for (int i = 0; i < 4; ++i) {
        if (dims[i] < 2 || dims[i] > (1 << 15)) return OVL_E_ARG;
        V *= dims[i];
    }
    if (V > (int64_t)1 << 31) return OVL_E_ARG;
    if (bc != nullptr)
        for (int i = 0; i < 4; ++i)
            if (bc[i] != 1 && bc[i] != -1) return OVL_E_ARG;
    ovl_ctx* ctx = new (std::nothrow) ovl_ctx();
    if (!ctx) return OVL_E_OOM;
    ctx->device = device;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    int64_t stride = 1;
    for (int i = 0; i < 4; ++i) {
        ctx->g.L[i] = dims[i];
        ctx->g.stride[i] = stride;
        stride *= dims[i];
        if (bc) ctx->bc[i] = bc[i];
        ctx->g.bc[i] = ctx->bc[i];
    }
    ctx->g.V = V;
    ctx->g.Vt = (V + kTile - 1) / kTile * kTile;
    {
        // the no-allocation entry point's scratch on this device (set-up, with
        // the device current; a failed lookup only disables that entry point)
        DeviceGuard dg(device);
        ctx->scratch = scratch_address(device);
    }
    const char* fz = getenv("OVL_FUSED");
    ctx->fused_iter = fz && fz[0] == '1';
    *out = ctx;
    return OVL_OK;
}

extern "C" int ovl_destroy(ovl_ctx* ctx) {
    if (!ctx) return OVL_OK;
    DeviceGuard dg(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (DBuf& b : ctx->fslot_chunks) b.release();
    ctx->fslot_table.release();
    ctx->fW.release();
    DBuf* bufs[] = {&ctx->U64,  &ctx->U32, &ctx->U64c, &ctx->U32c,   &ctx->hw_in,  &ctx->hw_out, &ctx->b64,   &ctx->r64,
                    &ctx->p64,  &ctx->q64,   &ctx->r32,    &ctx->q32,   &ctx->s64,
                    &ctx->pj64, &ctx->pj32,  &ctx->xj,     &ctx->part_w, &ctx->part_b,
                    &ctx->state, &ctx->shifts, &ctx->lists, &ctx->nodes_dev, &ctx->hist, &ctx->W,
                    &ctx->h,    &ctx->seed,    &ctx->bench_a, &ctx->bench_b, &ctx->bench_c, &ctx->tune_state, &ctx->tune_flush, &ctx->chk, &ctx->fY, &ctx->fX, &ctx->fpsi,
                    &ctx->facc, &ctx->fc, &ctx->fpart, &ctx->slot_table, &ctx->jobs_dev};
    for (DBuf* b : bufs) b->release();
    for (DBuf& b : ctx->slot_chunks) b.release();
    for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    for (auto& gc : ctx->graphs)
        if (gc.exec) (void)hipGraphExecDestroy(gc.exec);
    if (ctx->ev_in) (void)hipEventDestroy(ctx->ev_in);
    if (ctx->ev_out) (void)hipEventDestroy(ctx->ev_out);
    if (ctx->ws) (void)hipStreamDestroy(ctx->ws);
    if (ctx->host_state) (void)hipHostFree(ctx->host_state);
    if (ctx->chk_host) (void)hipHostFree(ctx->chk_host);
    ctx->chkdev.release();
    delete ctx;
    return OVL_OK;
}

extern "C" int ovl_set_stream(ovl_ctx* ctx, void* hip_stream) {
    if (!ctx) return OVL_E_ARG;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    return OVL_OK;
}

extern "C" int ovl_set_gauge(ovl_ctx* ctx, const void* U) {
    if (!ctx) return OVL_E_ARG;
    DeviceGuard dg(ctx->device);
    int rc = check_dev_ptr(ctx, U, "U");
    if (rc) return rc;
    const size_t nl = (size_t)36 * ctx->g.Vt;
    HIPCHK(ctx, ctx->U64.ensure(nl * sizeof(double2)));
    HIPCHK(ctx, ctx->U32.ensure(nl * sizeof(float2)));
    HIPCHK(ctx, ctx->U64c.ensure(nl / 9 * 6 * sizeof(double2)));
    HIPCHK(ctx, ctx->U32c.ensure(nl / 9 * 6 * sizeof(float2)));
    const int nblk = gauge_blocks(ctx->g);
    HIPCHK(ctx, ctx->chk.ensure((size_t)4 * nblk * sizeof(double)));
    launch_pack_gauge(static_cast<const double2*>(U), ctx->U64.as<double2>(),
                      ctx->U32.as<float2>(), ctx->U64c.as<double2>(), ctx->U32c.as<float2>(),
                      ctx->g, ctx->chk.as<double>(), ctx->stream);
    HIPCHK(ctx, hipGetLastError());
    // SU(3) to rounding (unitary, det 1) -> the two-row form; anything else
    // (a perturbed field, say) keeps the full matrices
    std::vector<double> defect((size_t)4 * nblk);
    HIPCHK(ctx, hipMemcpyAsync(defect.data(), ctx->chk.p, defect.size() * sizeof(double),
                               hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    // the kernel marks a block holding a NaN or infinite entry with NaN; keep
    // any NaN (std::max would drop it: max(x, NaN) returns x)
    double dmax = 0.0;
    bool nonfinite = false;
    for (double d : defect) {
        if (std::isnan(d)) nonfinite = true;
        else if (d > dmax) dmax = d;
    }
    if (nonfinite) {
        // the internal links now hold the bad field: no operator may use them
        ctx->gauge_set = false;
        ctx->links12 = false;
        return fail(ctx, OVL_E_NONFINITE, "the gauge field has a NaN or infinite entry");
    }
    const char* lf = getenv("OVL_LINKS");
    ctx->links12 = dmax < 1e-12 && !(lf && std::strcmp(lf, "full") == 0);
    ctx->gauge_set = true;
    return OVL_OK;
}

extern "C" int ovl_set_masses(ovl_ctx* ctx, double m0, double mq) {
    if (!ctx) return OVL_E_ARG;
    if (!(m0 > 0.0 && m0 < 4.0) || !std::isfinite(mq))
        return fail(ctx, OVL_E_ARG, "need 0 < m0 < 4 and finite mq (m0=%g, mq=%g)", m0, mq);
    ctx->m0 = m0;
    ctx->mq = mq;
    ctx->masses_set = true;
    return OVL_OK;
}

extern "C" int ovl_set_contour(ovl_ctx* ctx, int32_t nq, double gamma, double rho, double alpha) {
    if (!ctx) return OVL_E_ARG;
    if (nq < 2 || (nq & 1) || 2 * nq > kMaxShifts)
        return fail(ctx, OVL_E_ARG, "nq must be even and 2 <= nq <= %d (got %d)", kMaxShifts / 2, nq);
    if (!(rho > 0.0) || !(alpha > 0.0) || !std::isfinite(gamma))
        return fail(ctx, OVL_E_ARG, "need rho > 0, alpha > 0, finite gamma");
    // eq. (7): theta_j = 2 pi (j - 1/2)/N_q, z_j = +-gamma + rho (cos + i alpha sin),
    // weight rho (alpha cos + i sin)/N_q, negated on Gamma_- (eq. (3))
    ctx->z.assign(2 * nq, make_double2(0, 0));
    ctx->c.assign(2 * nq, make_double2(0, 0));
    for (int j = 1; j <= nq; ++j) {
        const double th = 2.0 * M_PI * (j - 0.5) / nq;
        const double ct = std::cos(th), sn = std::sin(th);
        const double er = rho * ct, ei = rho * alpha * sn;
        const double wr = rho * alpha * ct / nq, wi = rho * sn / nq;
        ctx->z[j - 1] = make_double2(gamma + er, ei);
        ctx->c[j - 1] = make_double2(wr, wi);
        ctx->z[nq + j - 1] = make_double2(-gamma + er, ei);
        ctx->c[nq + j - 1] = make_double2(-wr, -wi);
    }
    ctx->c0 = 0.0;
    return OVL_OK;
}

extern "C" int ovl_set_contour_single(ovl_ctx* ctx, int32_t nq, double gamma, double rho,
                                      double alpha) {
    if (!ctx) return OVL_E_ARG;
    if (nq < 2 || (nq & 1) || nq > kMaxShifts)
        return fail(ctx, OVL_E_ARG, "nq must be even and 2 <= nq <= %d (got %d)", kMaxShifts, nq);
    if (!(rho > 0.0) || !(alpha > 0.0) || !std::isfinite(gamma))
        return fail(ctx, OVL_E_ARG, "need rho > 0, alpha > 0, finite gamma");
    // sgn = P_+ - P_- and P_+ + P_- = 1 without exact zero modes, so
    // sgn = 2 P_+ - 1 from the Gamma_+ quadrature alone (twice its weights)
    ctx->z.assign(nq, make_double2(0, 0));
    ctx->c.assign(nq, make_double2(0, 0));
    for (int j = 1; j <= nq; ++j) {
        const double th = 2.0 * M_PI * (j - 0.5) / nq;
        const double ct = std::cos(th), sn = std::sin(th);
        ctx->z[j - 1] = make_double2(gamma + rho * ct, rho * alpha * sn);
        ctx->c[j - 1] = make_double2(2.0 * rho * alpha * ct / nq, 2.0 * rho * sn / nq);
    }
    ctx->c0 = -1.0;
    return OVL_OK;
}

extern "C" int ovl_set_nodes(ovl_ctx* ctx, int32_t n, const double* zr, const double* cr) {
    if (!ctx) return OVL_E_ARG;
    if (n < 1 || n > kMaxShifts || !zr || !cr)
        return fail(ctx, OVL_E_ARG, "need 1 <= n <= %d nodes and non-NULL arrays", kMaxShifts);
    for (int j = 0; j < n; ++j) {
        if (!std::isfinite(zr[2 * j]) || !std::isfinite(zr[2 * j + 1]) ||
            !std::isfinite(cr[2 * j]) || !std::isfinite(cr[2 * j + 1]))
            return fail(ctx, OVL_E_ARG, "node %d is not finite", j);
        if (zr[2 * j + 1] == 0.0)
            return fail(ctx, OVL_E_ARG, "node %d lies on the real axis", j);
    }
    ctx->z.resize(n);
    ctx->c.resize(n);
    for (int j = 0; j < n; ++j) {
        ctx->z[j] = make_double2(zr[2 * j], zr[2 * j + 1]);
        ctx->c[j] = make_double2(cr[2 * j], cr[2 * j + 1]);
    }
    ctx->c0 = 0.0;
    return OVL_OK;
}

extern "C" int ovl_set_solver(ovl_ctx* ctx, int32_t precision, int32_t form, double tol,
                              int32_t maxiter, double zr, double zi, double switch_res) {
    if (!ctx) return OVL_E_ARG;
    if (precision != OVL_PREC_FP64 && precision != OVL_PREC_MIXED)
        return fail(ctx, OVL_E_ARG, "unknown precision %d", precision);
    if (form < OVL_FORM_REFERENCE || form > OVL_FORM_TWOPASS)
        return fail(ctx, OVL_E_ARG, "unknown or unsupported form %d", form);
    if (!(tol > 0.0 && tol < 1.0)) return fail(ctx, OVL_E_ARG, "need 0 < tol < 1");
    if (maxiter < 1 || maxiter > 1000000) return fail(ctx, OVL_E_ARG, "bad maxiter %d", maxiter);
    if (!std::isfinite(zr) || !std::isfinite(zi) || zi == 0.0)
        return fail(ctx, OVL_E_ARG, "seed shift must be finite with a nonzero imaginary part");
    ctx->precision = precision;
    ctx->form = form;
    ctx->tol = tol;
    ctx->maxiter = maxiter;
    ctx->zseed = make_double2(zr, zi);
    ctx->switch_res = switch_res > 0.0 ? switch_res : 1e-4;
    return OVL_OK;
}

extern "C" int ovl_get_stats(const ovl_ctx* ctx, ovl_stats* st) {
    if (!ctx || !st) return OVL_E_ARG;
    *st = ctx->last;
    return OVL_OK;
}

extern "C" const char* ovl_last_error(const ovl_ctx* ctx) { return ctx ? ctx->err : "null context"; }

extern "C" const char* ovl_status_string(int s) {
    switch (s) {
        case OVL_OK: return "OVL_OK";
        case OVL_NOT_CONVERGED: return "OVL_NOT_CONVERGED";
        case OVL_E_ARG: return "OVL_E_ARG";
        case OVL_E_STATE: return "OVL_E_STATE";
        case OVL_E_HIP: return "OVL_E_HIP";
        case OVL_E_OOM: return "OVL_E_OOM";
        case OVL_E_NONFINITE: return "OVL_E_NONFINITE";
        case OVL_E_BREAKDOWN: return "OVL_E_BREAKDOWN";
        default: return "unknown status";
    }
}

// ============================================================================
// stencil autotuner
// ============================================================================
// The four stencil variants trade registers for loads in flight; which one
// wins depends on the lattice volume, the number of right-hand sides and the
// precision (how many waves the launch can keep resident).  The first use of a
// (lattice, nrhs, precision) times each variant with HIP events on the
// context's stream and keeps the fastest.  OVL_STENCIL_VARIANT=v forces a
// variant; OVL_AUTOTUNE=0 keeps variant 0; OVL_AUTOTUNE_CACHE=path keeps the
// choices in a flat JSON object {"key": variant} shared by processes.
namespace {

std::mutex g_tune_mu;

std::string tune_key(const ovl_ctx* ctx, int nrhs, int prec, int mode, int lnk) {
    hipDeviceProp_t prop;
    const char* arch = "gpu";
    if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) arch = prop.gcnArchName;
    int rt = 0;
    (void)hipRuntimeGetVersion(&rt);
    char buf[256];
    snprintf(buf, sizeof(buf), "%s|hip%d|t%d|%dx%dx%dx%d|n%d|%s|m%d|%s", arch, rt, kTile, ctx->g.L[0],
             ctx->g.L[1], ctx->g.L[2], ctx->g.L[3], nrhs, prec ? "fp32" : "fp64", mode,
             lnk ? "su3" : "gen");
    std::string k(buf);
    for (char& c : k)
        if (c == '"' || c == '\\') c = '_';
    return k;
}

std::map<std::string, int> read_cache(const char* path) {
    std::map<std::string, int> m;
    FILE* f = fopen(path, "r");
    if (!f) return m;
    std::string txt;
    char buf[4096];
    size_t n;
    while ((n = fread(buf, 1, sizeof(buf), f)) > 0) txt.append(buf, n);
    fclose(f);
    size_t i = 0;
    while ((i = txt.find('"', i)) != std::string::npos) {
        const size_t j = txt.find('"', i + 1);
        if (j == std::string::npos) break;
        const size_t c = txt.find(':', j);
        if (c == std::string::npos) break;
        m[txt.substr(i + 1, j - i - 1)] = atoi(txt.c_str() + c + 1);
        i = txt.find_first_of(",}", c);
        if (i == std::string::npos) break;
    }
    return m;
}

void write_cache(const char* path, const std::map<std::string, int>& m) {
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = fopen(tmp.c_str(), "w");
    if (!f) return;
    fprintf(f, "{");
    bool first = true;
    for (const auto& kv : m) {
        fprintf(f, "%s\n  \"%s\": %d", first ? "" : ",", kv.first.c_str(), kv.second);
        first = false;
    }
    fprintf(f, "\n}\n");
    fclose(f);
    (void)rename(tmp.c_str(), path);
}

// Inputs of a mode-1 timing launch: every source live at iteration 0.
struct TuneInputs {
    const void* r = nullptr;
    double4* partial = nullptr;
    const SrcState* st = nullptr;
    ShiftDev sh{};
};

template <typename R>
double time_variant(ovl_ctx* ctx, int v, int nrhs, int mode, int lnk, C2<R>* a, C2<R>* b,
                    const C2<R>* U, const TuneInputs& ti) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return 1e30;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return 1e30;
    }
    auto run = [&]() {
        if (mode == 1)
            launch_wilson<R>(1, a, b, U, ctx->g, kappa_of(ctx->m0), ctx->zseed,
                             static_cast<const C2<R>*>(ti.r), ti.partial, ti.st, &ti.sh, 1, nrhs,
                             ctx->stream, v, lnk);
        else
            launch_wilson<R>(0, a, b, U, ctx->g, kappa_of(ctx->m0), make_double2(0, 0), nullptr,
                             nullptr, nullptr, nullptr, 0, nrhs, ctx->stream, v, lnk);
    };
    run();
    // In the solver the stencil's operands arrive after the update kernel has
    // streamed the basis slot and the vectors through the caches, so each
    // timed launch here follows 512 MB of writes (twice the last-level cache)
    // and is timed on its own; the median of 9 is kept.
    const bool flush = ctx->tune_flush.ensure((size_t)512 << 20) == hipSuccess;
    std::vector<float> t;
    for (int i = 0; i < 9; ++i) {
        if (flush) (void)hipMemsetAsync(ctx->tune_flush.p, i & 0xff, (size_t)512 << 20, ctx->stream);
        (void)hipEventRecord(e0, ctx->stream);
        run();
        (void)hipEventRecord(e1, ctx->stream);
        float ms = 1e30f;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            ms = 1e30f;
        t.push_back(ms);
    }
    std::nth_element(t.begin(), t.begin() + 4, t.end());
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return t[4];
}

}  // namespace

// A stencil choice known without timing anything: forced by
// OVL_STENCIL_VARIANT, already chosen on this context, the untuned default
// under OVL_AUTOTUNE=0, or stored in the OVL_AUTOTUNE_CACHE file; else -1.
static int stencil_lookup(ovl_ctx* ctx, int nrhs, int prec, int mode) {
    const int nfmt = ctx->links12 ? 2 : 1;
    const char* force = getenv("OVL_STENCIL_VARIANT");
    if (force && *force) {
        const int v = atoi(force);
        if (v >= 0 && v < kStencilVariants) return v + kStencilVariants * (nfmt - 1);
    }
    const auto key = std::make_pair(nrhs, prec + 2 * mode);
    auto it = ctx->stencil_variant.find(key);
    if (it != ctx->stencil_variant.end()) return it->second;
    const char* at = getenv("OVL_AUTOTUNE");
    if (at && at[0] == '0') return ctx->stencil_variant[key] = kStencilVariants * (nfmt - 1);
    const char* path = getenv("OVL_AUTOTUNE_CACHE");
    if (path && *path) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto m = read_cache(path);
        auto f = m.find(tune_key(ctx, nrhs, prec, mode, nfmt == 2));
        if (f != m.end() && f->second >= 0 && f->second < kStencilVariants * nfmt)
            return ctx->stencil_variant[key] = f->second;
    }
    return -1;
}

static void stencil_store(ovl_ctx* ctx, int nrhs, int prec, int mode, int code) {
    ctx->stencil_variant[std::make_pair(nrhs, prec + 2 * mode)] = code;
    const char* path = getenv("OVL_AUTOTUNE_CACHE");
    if (path && *path) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto m = read_cache(path);
        m[tune_key(ctx, nrhs, prec, mode, ctx->links12)] = code;
        write_cache(path, m);
    }
}

// Variant of the stencil for nrhs right-hand sides in precision prec (0 FP64,
// 1 FP32) and mode (0: H_W alone; 1: the solver's q_k = z_s r_k - H r_k +
// beta q_{k-1} with its dot products, timed with every source live).  The
// basis forms tune mode 1 inside the solve instead (tune_solver_stencil).
static int stencil_variant(ovl_ctx* ctx, int nrhs, int prec, int mode) {
    const int nfmt = ctx->links12 ? 2 : 1;  // link formats to try: full, and two-row if SU(3)
    const char* force = getenv("OVL_STENCIL_VARIANT");
    if (force && *force) {
        const int v = atoi(force);
        if (v >= 0 && v < kStencilVariants) return v + kStencilVariants * (nfmt - 1);
    }
    const auto key = std::make_pair(nrhs, prec + 2 * mode);
    auto it = ctx->stencil_variant.find(key);
    if (it != ctx->stencil_variant.end()) return it->second;
    const char* at = getenv("OVL_AUTOTUNE");
    if (at && at[0] == '0') return ctx->stencil_variant[key] = kStencilVariants * (nfmt - 1);
    const char* path = getenv("OVL_AUTOTUNE_CACHE");
    const std::string k = tune_key(ctx, nrhs, prec, mode, nfmt == 2);
    if (path && *path) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto m = read_cache(path);
        auto f = m.find(k);
        if (f != m.end() && f->second >= 0 && f->second < kStencilVariants * nfmt)
            return ctx->stencil_variant[key] = f->second;
    }
    const size_t es = prec ? sizeof(float2) : sizeof(double2);
    const size_t nb = (size_t)nrhs * n12(ctx) * es;
    int best = 0;
    bool ok = ctx->bench_a.ensure(nb) == hipSuccess && ctx->bench_b.ensure(nb) == hipSuccess &&
              hipMemsetAsync(ctx->bench_a.p, 0, nb, ctx->stream) == hipSuccess;
    TuneInputs ti;
    if (ok && mode == 1) {
        // r (a vector of its own, so its loads cost what they do in the
        // solver), per-block partials and a state block with every source
        // live at iteration 0: status 0 and one active shift in slice 0
        const size_t st_bytes = ((size_t)nrhs * sizeof(SrcState) + 255) & ~(size_t)255;
        const size_t cnt_bytes = ((size_t)2 * nrhs * kMaxSlices * sizeof(int) + 255) & ~(size_t)255;
        const size_t part_bytes = (size_t)nrhs * wilson_blocks(ctx->g) * sizeof(double4);
        ok = ctx->bench_c.ensure(nb) == hipSuccess &&
             hipMemsetAsync(ctx->bench_c.p, 0, nb, ctx->stream) == hipSuccess &&
             hipMemsetAsync(ctx->bench_b.p, 0, nb, ctx->stream) == hipSuccess &&
             ctx->tune_state.ensure(st_bytes + cnt_bytes + part_bytes) == hipSuccess &&
             hipMemsetAsync(ctx->tune_state.p, 0, st_bytes + cnt_bytes, ctx->stream) == hipSuccess;
        if (ok) {
            // counts in both parities: the timed launch is iteration 1 (with
            // the beta q_{k-1} term of the solver's stencil)
            std::vector<int> cnt((size_t)2 * nrhs * kMaxSlices, 0);
            for (int n = 0; n < 2 * nrhs; ++n) cnt[(size_t)n * kMaxSlices] = 1;
            char* base = ctx->tune_state.as<char>();
            ok = hipMemcpyAsync(base + st_bytes, cnt.data(), cnt.size() * sizeof(int),
                                hipMemcpyHostToDevice, ctx->stream) == hipSuccess &&
                 hipStreamSynchronize(ctx->stream) == hipSuccess;
            ti.r = ctx->bench_c.p;
            ti.st = reinterpret_cast<const SrcState*>(base);
            ti.partial = reinterpret_cast<double4*>(base + st_bytes + cnt_bytes);
            ti.sh.cnt = reinterpret_cast<int*>(base + st_bytes);
            ti.sh.nsrc = nrhs;
            ti.sh.nslices = 1;
            ti.sh.maxk = 2;
        }
    }
    const char* vb = getenv("OVL_AUTOTUNE_VERBOSE");
    const bool verbose = vb && vb[0] == '1';
    if (ok) {
        double tbest = 1e30;
        for (int code = 0; code < kStencilVariants * nfmt; ++code) {
            const int v = code % kStencilVariants, lnk = code / kStencilVariants;
            const float2* U32 = lnk ? ctx->U32c.as<float2>() : ctx->U32.as<float2>();
            const double2* U64 = lnk ? ctx->U64c.as<double2>() : ctx->U64.as<double2>();
            const double t =
                prec ? time_variant<float>(ctx, v, nrhs, mode, lnk, ctx->bench_a.as<float2>(),
                                           ctx->bench_b.as<float2>(), U32, ti)
                     : time_variant<double>(ctx, v, nrhs, mode, lnk, ctx->bench_a.as<double2>(),
                                            ctx->bench_b.as<double2>(), U64, ti);
            if (verbose)
                fprintf(stderr, "ovl autotune %s: choice %d (variant %d, %s links) %.2f us\n",
                        k.c_str(), code, v, lnk ? "two-row" : "full", t * 1e3);
            if (t < tbest) {
                tbest = t;
                best = code;
            }
        }
    }
    (void)hipStreamSynchronize(ctx->stream);
    ctx->tune_flush.release();  // only needed while tuning
    (void)hipGetLastError();
    ctx->stencil_variant[key] = best;
    if (path && *path) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto m = read_cache(path);
        m[k] = best;
        write_cache(path, m);
    }
    return best;
}

// Variant of the fused iteration kernel (code v + kIterVariants * links) for
// nrhs right-hand sides in precision prec, tuned like the stencil: every
// variant in every allowed link format is timed on a one-job table whose
// buffers are scratch (kernel 1 with every source live, no shifts), each
// launch after 512 MB of writes, median of 9.  OVL_ITER_VARIANT=v forces
// variant v (two-row links for SU(3) fields unless OVL_LINKS=full).
static int iter_variant(ovl_ctx* ctx, int nrhs, int prec) {
    const int nfmt = ctx->links12 ? 2 : 1;
    const char* force = getenv("OVL_ITER_VARIANT");
    if (force && *force) {
        const int v = atoi(force);
        if (v >= 0 && v < kIterVariants) return v + kIterVariants * (nfmt - 1);
    }
    const auto key = std::make_pair(nrhs, prec + 4);
    auto it = ctx->stencil_variant.find(key);
    if (it != ctx->stencil_variant.end()) return it->second;
    const char* at = getenv("OVL_AUTOTUNE");
    if (at && at[0] == '0') return ctx->stencil_variant[key] = kIterVariants * (nfmt - 1);
    const char* path = getenv("OVL_AUTOTUNE_CACHE");
    const std::string k = tune_key(ctx, nrhs, prec, 2, nfmt == 2);
    if (path && *path) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto m = read_cache(path);
        auto f = m.find(k);
        if (f != m.end() && f->second >= 0 && f->second < kIterVariants * nfmt)
            return ctx->stencil_variant[key] = f->second;
    }
    const size_t es = prec ? sizeof(float2) : sizeof(double2);
    const size_t vec = (size_t)nrhs * n12(ctx) * es;
    const int nsb = wilson_blocks(ctx->g);
    const size_t part = (size_t)nrhs * nsb;
    // layout of tune_state: JobDesc | kdev[2] | slot table | SrcState[nrhs] |
    // cnt [2][nrhs][kMaxSlices] | mres [nrhs][kMaxSlices] | partials [2][part]
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t o_k = al(sizeof(JobDesc)), o_tab = o_k + 256, o_st = o_tab + 256;
    const size_t o_cnt = o_st + al((size_t)nrhs * sizeof(SrcState));
    const size_t o_mres = o_cnt + al((size_t)2 * nrhs * kMaxSlices * sizeof(int));
    const size_t o_part = o_mres + al((size_t)nrhs * kMaxSlices * sizeof(double));
    const size_t total = o_part + 2 * part * sizeof(double4);
    int best = kIterVariants * (nfmt - 1);
    bool ok = ctx->bench_a.ensure(2 * vec) == hipSuccess && ctx->bench_b.ensure(2 * vec) == hipSuccess &&
              ctx->tune_state.ensure(total) == hipSuccess &&
              hipMemsetAsync(ctx->bench_a.p, 0, 2 * vec, ctx->stream) == hipSuccess &&
              hipMemsetAsync(ctx->bench_b.p, 0, 2 * vec, ctx->stream) == hipSuccess &&
              hipMemsetAsync(ctx->tune_state.p, 0, total, ctx->stream) == hipSuccess;
    char* base = ctx->tune_state.as<char>();
    JobDesc* jd = reinterpret_cast<JobDesc*>(base);
    int* kdev = reinterpret_cast<int*>(base + o_k);
    const char* vb = getenv("OVL_AUTOTUNE_VERBOSE");
    const bool verbose = vb && vb[0] == '1';
    if (ok) {
        // host images: every source live at kernel 1 (counts [0][n][0] = 1),
        // kernel 0's partials (1, 0, 1, 1) per block give alpha = 1, beta = 0
        std::vector<int> cnt((size_t)2 * nrhs * kMaxSlices, 0);
        for (int n = 0; n < nrhs; ++n) cnt[(size_t)n * kMaxSlices] = 1;
        std::vector<double4> p0(part, make_double4(1.0, 0.0, 1.0, 1.0));
        char* tab[1] = {ctx->bench_a.as<char>()};
        const int kk[2] = {1, 2};
        ok = hipMemcpyAsync(base + o_cnt, cnt.data(), cnt.size() * sizeof(int),
                            hipMemcpyHostToDevice, ctx->stream) == hipSuccess &&
             hipMemcpyAsync(base + o_part, p0.data(), part * sizeof(double4), hipMemcpyHostToDevice,
                            ctx->stream) == hipSuccess &&
             hipMemcpyAsync(base + o_tab, tab, sizeof(tab), hipMemcpyHostToDevice, ctx->stream) ==
                 hipSuccess &&
             hipMemcpyAsync(kdev, kk, sizeof(kk), hipMemcpyHostToDevice, ctx->stream) == hipSuccess &&
             hipStreamSynchronize(ctx->stream) == hipSuccess;
    }
    const bool flush = ok && ctx->tune_flush.ensure((size_t)512 << 20) == hipSuccess;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ok = ok && hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
    double tbest = 1e30;
    for (int code = 0; ok && code < kIterVariants * nfmt; ++code) {
        const int v = code % kIterVariants, lnk = code / kIterVariants;
        JobDesc d{};
        d.g = ctx->g;
        d.kappa = kappa_of(ctx->m0);
        d.zs = ctx->zseed;
        d.U[0] = lnk ? ctx->U64c.p : ctx->U64.p;
        d.U[1] = lnk ? ctx->U32c.p : ctx->U32.p;
        d.nsrc = nrhs;
        d.nsb = nsb;
        d.sten_nb[0] = d.sten_nb[1] = iter_grid_blocks(ctx->g, nrhs);
        d.st = reinterpret_cast<SrcState*>(base + o_st);
        d.sh.cnt = reinterpret_cast<int*>(base + o_cnt);
        d.sh.mres = reinterpret_cast<double*>(base + o_mres);
        d.sh.nsrc = nrhs;
        d.sh.nslices = 1;
        d.sh.maxk = 4;
        d.part_w = reinterpret_cast<double4*>(base + o_part);
        d.part_stride = part;
        d.q[0] = d.q[1] = ctx->bench_b.p;
        d.qpp = (size_t)nrhs * n12(ctx);
        d.slots = reinterpret_cast<char* const*>(base + o_tab);
        d.slot_bytes = vec;
        d.ksw = 1 << 30;
        d.form = OVL_FORM_BASIS;
        d.phase = prec;
        if (hipMemcpyAsync(jd, &d, sizeof(d), hipMemcpyHostToDevice, ctx->stream) != hipSuccess) break;
        auto run = [&]() {
            // kread = kwrite: every timed launch is kernel 1
            if (prec)
                launch_iter_jobs<float>(jd, 1, kdev, kdev + 1, job_grid_blocks(d.sten_nb[1]), v,
                                        lnk, ctx->stream);
            else
                launch_iter_jobs<double>(jd, 1, kdev, kdev + 1, job_grid_blocks(d.sten_nb[0]), v,
                                         lnk, ctx->stream);
        };
        run();
        std::vector<float> t;
        for (int i = 0; i < 9; ++i) {
            if (flush) (void)hipMemsetAsync(ctx->tune_flush.p, i & 0xff, (size_t)512 << 20, ctx->stream);
            (void)hipEventRecord(e0, ctx->stream);
            run();
            (void)hipEventRecord(e1, ctx->stream);
            float ms = 1e30f;
            if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                ms = 1e30f;
            t.push_back(ms);
        }
        std::nth_element(t.begin(), t.begin() + 4, t.end());
        if (verbose)
            fprintf(stderr, "ovl autotune %s: fused choice %d (variant %d, %s links) %.2f us\n",
                    k.c_str(), code, v, lnk ? "two-row" : "full", t[4] * 1e3);
        if (t[4] < tbest) {
            tbest = t[4];
            best = code;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(ctx->stream);
    ctx->tune_flush.release();
    (void)hipGetLastError();
    ctx->stencil_variant[key] = best;
    if (path && *path) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto m = read_cache(path);
        m[k] = best;
        write_cache(path, m);
    }
    return best;
}

// ============================================================================
// H_W
// ============================================================================
static int check_apply_args(ovl_ctx* ctx, const void* in, const void* out, int nrhs,
                            bool need_nodes) {
    if (nrhs < 1 || nrhs > 65535) return fail(ctx, OVL_E_ARG, "bad nrhs %d", nrhs);
    if (!ctx->gauge_set) return fail(ctx, OVL_E_STATE, "ovl_set_gauge was not called");
    if (!ctx->masses_set) return fail(ctx, OVL_E_STATE, "ovl_set_masses was not called");
    if (need_nodes && ctx->z.empty())
        return fail(ctx, OVL_E_STATE, "ovl_set_contour / ovl_set_nodes was not called");
    int rc = check_dev_ptr(ctx, in, "in");
    if (rc) return rc;
    rc = check_dev_ptr(ctx, out, "out");
    if (rc) return rc;
    const size_t bytes = (size_t)nrhs * n12_ext(ctx) * sizeof(double2);
    if (overlaps(in, bytes, out, bytes)) return fail(ctx, OVL_E_ARG, "out aliases in");
    return OVL_OK;
}

extern "C" int ovl_apply_hw(ovl_ctx* ctx, const void* in, void* out, int32_t nrhs) {
    if (!ctx) return OVL_E_ARG;
    DeviceGuard dg(ctx->device);
    int rc = check_apply_args(ctx, in, out, nrhs, false);
    if (rc) return rc;
    const size_t nb = (size_t)nrhs * n12(ctx) * sizeof(double2);
    HIPCHK(ctx, ctx->hw_in.ensure(nb));
    HIPCHK(ctx, ctx->hw_out.ensure(nb));
    launch_pack_spinor64(static_cast<const double2*>(in), ctx->hw_in.as<double2>(), ctx->g.V, ctx->g.Vt,
                         nrhs, ctx->stream);
    const int code = stencil_variant(ctx, nrhs, 0, 0);
    const int var = code % kStencilVariants, lnk = code / kStencilVariants;
    launch_wilson<double>(0, ctx->hw_in.as<double2>(), ctx->hw_out.as<double2>(),
                          stencil_links<double>(ctx, lnk), ctx->g, kappa_of(ctx->m0),
                          make_double2(0, 0), nullptr, nullptr, nullptr, nullptr, 0, nrhs,
                          ctx->stream, var, lnk);
    launch_unpack_spinor64(ctx->hw_out.as<double2>(), static_cast<double2*>(out), ctx->g.V, ctx->g.Vt, nrhs,
                           ctx->stream);
    HIPCHK(ctx, hipGetLastError());
    return OVL_OK;
}

extern "C" int ovl_apply_hw_noalloc(ovl_ctx* ctx, const void* in, void* out, int32_t nrhs) {
    if (!ctx) return OVL_E_ARG;
    DeviceGuard dg(ctx->device);
    int rc = check_apply_args(ctx, in, out, nrhs, false);
    if (rc) return rc;
    if (!ctx->scratch) return fail(ctx, OVL_E_HIP, "the static scratch of this device is unavailable");
    const size_t nb = (size_t)nrhs * n12(ctx) * sizeof(double2);
    if (2 * nb > kNoAllocScratchBytes)
        return fail(ctx, OVL_E_ARG,
                    "nrhs %d needs %zu bytes of scratch; ovl_apply_hw_noalloc holds %zu "
                    "(2 nrhs * 12 * Vt complex128)", nrhs, 2 * nb, kNoAllocScratchBytes);
    // the stencil choice already tuned for this nrhs (by ovl_apply_hw), else
    // variant 0; never the tuner, which allocates
    int code = kStencilVariants * (ctx->links12 ? 1 : 0);
    auto it = ctx->stencil_variant.find(std::make_pair((int)nrhs, 0));
    if (it != ctx->stencil_variant.end()) code = it->second;
    const int var = code % kStencilVariants, lnk = code / kStencilVariants;
    double2* sin = static_cast<double2*>(ctx->scratch);
    double2* sout = reinterpret_cast<double2*>(static_cast<char*>(ctx->scratch) + nb);
    launch_pack_spinor64(static_cast<const double2*>(in), sin, ctx->g.V, ctx->g.Vt, nrhs, ctx->stream);
    launch_wilson<double>(0, sin, sout, stencil_links<double>(ctx, lnk), ctx->g, kappa_of(ctx->m0),
                          make_double2(0, 0), nullptr, nullptr, nullptr, nullptr, 0, nrhs,
                          ctx->stream, var, lnk);
    launch_unpack_spinor64(sout, static_cast<double2*>(out), ctx->g.V, ctx->g.Vt, nrhs, ctx->stream);
    HIPCHK(ctx, hipGetLastError());
    return OVL_OK;
}

extern "C" int ovl_apply_hw_fp32(ovl_ctx* ctx, const void* in, void* out, int32_t nrhs) {
    if (!ctx) return OVL_E_ARG;
    DeviceGuard dg(ctx->device);
    int rc = check_apply_args(ctx, in, out, nrhs, false);
    if (rc) return rc;
    const size_t nb = (size_t)nrhs * n12(ctx) * sizeof(float2);
    HIPCHK(ctx, ctx->hw_in.ensure(nb));
    HIPCHK(ctx, ctx->hw_out.ensure(nb));
    launch_pack_spinor32(static_cast<const double2*>(in), ctx->hw_in.as<float2>(), ctx->g.V, ctx->g.Vt,
                         nrhs, ctx->stream);
    const int code = stencil_variant(ctx, nrhs, 1, 0);
    const int var = code % kStencilVariants, lnk = code / kStencilVariants;
    launch_wilson<float>(0, ctx->hw_in.as<float2>(), ctx->hw_out.as<float2>(),
                         stencil_links<float>(ctx, lnk), ctx->g, kappa_of(ctx->m0),
                         make_double2(0, 0), nullptr, nullptr, nullptr, nullptr, 0, nrhs,
                         ctx->stream, var, lnk);
    launch_unpack_spinor32(ctx->hw_out.as<float2>(), static_cast<double2*>(out), ctx->g.V, ctx->g.Vt, nrhs,
                           ctx->stream);
    HIPCHK(ctx, hipGetLastError());
    return OVL_OK;
}

// ============================================================================
// shifted solver
// ============================================================================
namespace {


struct Work {
    int nsrc, J, maxk;
    int64_t N;  // 12 V
    double2 *b64, *r64, *p64, *q64, *s64, *pj64, *xj;
    float2 *r32, *q32, *pj32;
    std::vector<char*> chunks;  // basis: slot i at chunks[i / kSlotChunk] + (i % kSlotChunk) * slot_bytes
    size_t slot_bytes;          // nsrc * N * sizeof(double2)
    double4* part_w;       // K1 partials per source and stencil block
    double* part_b;        // ||b||^2 partials at initialisation
    int nbw, nbe;          // stencil blocks and vector-kernel blocks per source
    SrcState* st;          // device state block: st | cnt | mres (one copy to the host)
    size_t state_bytes;
    ShiftDev sh;
    int var64, var32;      // stencil variants (autotuned)
    bool fused;            // one-kernel iteration (basis forms): q and the partials double-buffered
    size_t qpp;            // fused: elements between q[0] and q[1]
    int k_switch;          // first basis slot (or iteration) held in FP32 (mixed), or -1
    int k_conv;            // iteration before which the job was converted to FP32, or -1
    int K;                 // seed iterations of the last solve (max over sources)
    size_t rpp;            // two-pass: elements between the two r buffers
    char** slot_tab;       // basis: device table of slot-chunk bases
    int n_tab;             // chunks published in slot_tab
    double2 *dz, *cj, *zj;
    double2 *h_a, *h_b, *h_pi, *W, *h;
    // in-band residual check (basis form), or null: coefficients of the
    // checked shift per source, its node, per-block partials, pinned copy
    double2 *hx, *zc, *cpart, *chost;
};

constexpr int kChkBlocks = 256;  // blocks per source of the in-band residual reduction

// layout of the state block shared by the device and its pinned host mirror
size_t state_cnt_off(int nsrc) { return ((size_t)nsrc * sizeof(SrcState) + 255) & ~(size_t)255; }
size_t state_mres_off(int nsrc) {
    return (state_cnt_off(nsrc) + (size_t)2 * nsrc * kMaxSlices * sizeof(int) + 255) & ~(size_t)255;
}
size_t state_bytes_for(int nsrc) { return state_mres_off(nsrc) + (size_t)nsrc * kMaxSlices * sizeof(double); }
// stride of the two pinned host copies of a job's state
size_t state_slot_bytes(const Work& w) { return (w.state_bytes + 255) & ~(size_t)255; }
const char* host_slot(const ovl_ctx* c, const Work& w, int slot) {
    return reinterpret_cast<const char*>(c->host_state) + (size_t)slot * state_slot_bytes(w);
}

int prepare(ovl_ctx* ctx, int nsrc, Work& w) {
    const int J = (int)ctx->z.size();
    const int64_t N = n12(ctx);
    const bool mixed = ctx->precision == OVL_PREC_MIXED;
    const int form = ctx->form;
    if ((form == OVL_FORM_FUSED || form == OVL_FORM_REFERENCE) && J > kMaxSweepShifts)
        return fail(ctx, OVL_E_ARG, "the fused and reference forms take at most %d shifts (have %d)",
                    kMaxSweepShifts, J);
    w.nsrc = nsrc;
    w.J = J;
    w.N = N;
    w.maxk = ctx->maxiter;
    const size_t vec64 = (size_t)nsrc * N * sizeof(double2);
    const size_t vec32 = (size_t)nsrc * N * sizeof(float2);
    const bool twopass = form == OVL_FORM_TWOPASS;
    w.fused = ctx->fused_iter && (form == OVL_FORM_BASIS || twopass);
    const size_t nq = w.fused ? 2 : 1;  // q buffers
    w.qpp = (size_t)nsrc * N;
    HIPCHK(ctx, ctx->b64.ensure(vec64));
    HIPCHK(ctx, ctx->r64.ensure(twopass ? 2 * vec64 : vec64));
    HIPCHK(ctx, ctx->p64.ensure(vec64));
    HIPCHK(ctx, ctx->q64.ensure(nq * vec64));
    HIPCHK(ctx, ctx->s64.ensure(vec64));
    w.b64 = ctx->b64.as<double2>();
    w.r64 = ctx->r64.as<double2>();
    w.p64 = ctx->p64.as<double2>();
    w.q64 = ctx->q64.as<double2>();
    w.s64 = ctx->s64.as<double2>();
    w.r32 = w.q32 = w.pj32 = nullptr;
    w.pj64 = w.xj = nullptr;
    w.chunks.clear();
    w.slot_bytes = vec64;
    w.rpp = (size_t)nsrc * N;
    w.slot_tab = nullptr;
    w.n_tab = 0;
    if (mixed) {
        HIPCHK(ctx, ctx->r32.ensure(twopass ? 2 * vec32 : vec32));
        HIPCHK(ctx, ctx->q32.ensure(nq * vec32));
        w.r32 = ctx->r32.as<float2>();
        w.q32 = ctx->q32.as<float2>();
    }
    if (form == OVL_FORM_FUSED || form == OVL_FORM_REFERENCE) {
        HIPCHK(ctx, ctx->pj64.ensure(vec64 * J));
        w.pj64 = ctx->pj64.as<double2>();
        if (mixed) {
            HIPCHK(ctx, ctx->pj32.ensure(vec32 * J));
            w.pj32 = ctx->pj32.as<float2>();
        }
        if (form == OVL_FORM_REFERENCE) {
            HIPCHK(ctx, ctx->xj.ensure(vec64 * J));
            w.xj = ctx->xj.as<double2>();
        }
    }
    const bool basis = form == OVL_FORM_BASIS;
    const bool hist = basis || twopass;
    if (basis) {
        HIPCHK(ctx, ctx->slot_table.ensure(((size_t)w.maxk / kSlotChunk + 2) * sizeof(char*)));
        w.slot_tab = ctx->slot_table.as<char*>();
    }
    if (basis && ctx->slot_chunk_bytes != vec64 * kSlotChunk) {
        // slot geometry changed: drop the old chunks
        for (DBuf& b : ctx->slot_chunks) b.release();
        ctx->slot_chunks.clear();
        ctx->slot_chunk_bytes = vec64 * kSlotChunk;
    }
    const int nslices = (J + 255) / 256;
    w.nbw = wilson_blocks(ctx->g);
    w.nbe = vec_blocks(N, nslices, basis || twopass);
    HIPCHK(ctx, ctx->part_w.ensure(nq * (size_t)nsrc * w.nbw * sizeof(double4)));
    // ||b||^2 partials of the initialisation: one per block of its own grid
    // (launch_init_state), which is not the update kernel's
    HIPCHK(ctx, ctx->part_b.ensure(init_partials(N, nslices, nsrc) * sizeof(double)));
    w.state_bytes = state_bytes_for(nsrc);
    HIPCHK(ctx, ctx->state.ensure(w.state_bytes));
    w.part_w = ctx->part_w.as<double4>();
    w.part_b = ctx->part_b.as<double>();
    w.st = ctx->state.as<SrcState>();
    const size_t sj = (size_t)nsrc * J;
    HIPCHK(ctx, ctx->shifts.ensure(sj * (4 * sizeof(double2) + sizeof(double) + 2 * sizeof(int))));
    ShiftDev& sh = w.sh;
    sh.pi = ctx->shifts.as<double2>();          // [3][nsrc][J]
    sh.aj = sh.pi + 3 * sj;
    sh.res = reinterpret_cast<double*>(sh.aj + sj);
    sh.active = reinterpret_cast<int*>(sh.res + sj);  // [2][nsrc][J]
    sh.cnt = reinterpret_cast<int*>(ctx->state.as<char>() + state_cnt_off(nsrc));
    sh.mres = reinterpret_cast<double*>(ctx->state.as<char>() + state_mres_off(nsrc));
    sh.J = J;
    sh.nsrc = nsrc;
    sh.nslices = nslices;
    sh.tol = ctx->tol;
    sh.maxk = w.maxk;
    HIPCHK(ctx, ctx->nodes_dev.ensure((size_t)3 * J * sizeof(double2)));
    w.dz = ctx->nodes_dev.as<double2>();
    w.cj = w.dz + J;
    w.zj = w.dz + 2 * J;
    sh.dz = w.dz;
    sh.c = w.cj;
    std::vector<double2> tab(3 * J);
    for (int j = 0; j < J; ++j) {
        tab[j] = make_double2(ctx->z[j].x - ctx->zseed.x, ctx->z[j].y - ctx->zseed.y);
        tab[J + j] = ctx->c[j];
        tab[2 * J + j] = ctx->z[j];
    }
    HIPCHK(ctx, hipMemcpyAsync(w.dz, tab.data(), tab.size() * sizeof(double2),
                               hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));  // tab is pageable and goes out of scope
    w.h_a = w.h_b = w.h_pi = w.W = w.h = nullptr;
    if (hist) {
        const size_t hs = (size_t)nsrc * (w.maxk + 1) * J;
        HIPCHK(ctx, ctx->hist.ensure(3 * hs * sizeof(double2)));
        HIPCHK(ctx, ctx->W.ensure(hs * sizeof(double2)));
        HIPCHK(ctx, ctx->h.ensure((size_t)nsrc * (w.maxk + 1) * sizeof(double2)));
        w.h_a = ctx->hist.as<double2>();
        w.h_b = w.h_a + hs;
        w.h_pi = w.h_b + hs;
        w.W = ctx->W.as<double2>();
        w.h = ctx->h.as<double2>();
    }
    sh.h_a = w.h_a;
    sh.h_b = w.h_b;
    sh.h_pi = w.h_pi;
    w.hx = w.zc = w.cpart = w.chost = nullptr;
    if (basis && ctx->inband_check) {
        const size_t nhx = (size_t)nsrc * (w.maxk + 1), npart = (size_t)nsrc * kChkBlocks;
        HIPCHK(ctx, ctx->chkdev.ensure((nhx + nsrc + npart) * sizeof(double2)));
        w.hx = ctx->chkdev.as<double2>();
        w.zc = w.hx + nhx;
        w.cpart = w.zc + nsrc;
        if (ctx->chk_host_bytes < npart * sizeof(double2)) {
            if (ctx->chk_host) (void)hipHostFree(ctx->chk_host);
            ctx->chk_host = nullptr;
            ctx->chk_host_bytes = 0;
            HIPCHK(ctx, hipHostMalloc((void**)&ctx->chk_host, npart * sizeof(double2),
                                      hipHostMallocDefault));
            ctx->chk_host_bytes = npart * sizeof(double2);
        }
        w.chost = ctx->chk_host;
    }
    HIPCHK(ctx, ctx->seed.ensure((size_t)nsrc * (w.maxk + 1) * 3 * sizeof(double2)));
    sh.seed = ctx->seed.as<double2>();
    // two pinned copies of the state: the poll reads one while the copy of
    // the next chunk's state may be in flight into the other
    if ((size_t)ctx->host_state_n < 2 * state_slot_bytes(w)) {
        if (ctx->host_state) (void)hipHostFree(ctx->host_state);
        ctx->host_state = nullptr;
        ctx->host_state_n = 0;
        HIPCHK(ctx, hipHostMalloc((void**)&ctx->host_state, 2 * state_slot_bytes(w),
                                  hipHostMallocDefault));
        ctx->host_state_n = (int)(2 * state_slot_bytes(w));
    }
    return OVL_OK;
}

template <typename R> R* slot_ptr(const Work& w, int i) {
    return reinterpret_cast<R*>(w.chunks[i / kSlotChunk] + (size_t)(i % kSlotChunk) * w.slot_bytes);
}

// make sure residual slots 0 .. upto exist and are published in the device table
int ensure_slots(ovl_ctx* ctx, Work& w, int upto, hipStream_t s) {
    const int need = std::min(upto, w.maxk) / kSlotChunk + 1;
    while ((int)ctx->slot_chunks.size() < need) {
        ctx->slot_chunks.emplace_back();
        HIPCHK(ctx, ctx->slot_chunks.back().ensure(ctx->slot_chunk_bytes));
    }
    w.chunks.clear();
    for (DBuf& b : ctx->slot_chunks) w.chunks.push_back(b.as<char>());
    if ((int)w.chunks.size() > w.n_tab) {
        // pageable source: the copy is staged at the call, before the next replay reads it
        HIPCHK(ctx, hipMemcpyAsync(w.slot_tab, w.chunks.data(), w.chunks.size() * sizeof(char*),
                                   hipMemcpyHostToDevice, s));
        w.n_tab = (int)w.chunks.size();
    }
    return OVL_OK;
}

// The basis slots that iterations [0, k_end) write (up to slot min(k_end, maxk))
// lie in slot chunks published in the device table: a host-side check before
// queueing kernels that write them.
bool slots_cover(const Work& w, int k_end) {
    return w.n_tab * kSlotChunk > std::min(k_end, w.maxk);
}

// Work stream of a context (created on first use; default priority).
int solve_stream(ovl_ctx* ctx, hipStream_t* out) {
    if (!ctx->ws) {
        HIPCHK(ctx, hipStreamCreateWithFlags(&ctx->ws, hipStreamNonBlocking));
        HIPCHK(ctx, hipEventCreateWithFlags(&ctx->ev_in, hipEventDisableTiming));
        HIPCHK(ctx, hipEventCreateWithFlags(&ctx->ev_out, hipEventDisableTiming));
    }
    *out = ctx->ws;
    return OVL_OK;
}

bool graphs_enabled(const ovl_ctx* ctx) {
    if (ctx->prof_on) return false;  // per-launch events need eager launches
    const char* e = getenv("OVL_GRAPHS");
    return !(e && e[0] == '0');
}

constexpr int kChunk = 16;  // seed iterations per captured graph / per convergence poll
// iteration i of a chunk reads the counter slot i & 1, so a chunk starts at slot 0
static_assert(kChunk % 2 == 0, "chunks must hold an even number of iterations");

struct Batch {
    std::vector<ovl_ctx*> ctx;
    std::vector<Work*> w;
    std::vector<JobDesc> desc;
    int sten_total[2] = {0, 0};  // stencil grid of the FP64 and of the FP32 variant
    int vec_total = 0, variant64 = 0, variant32 = 0, form = 0, maxJ = 0;
    int lnk[2] = {0, 0};  // link format of the FP64 and of the FP32 stencil
    bool fused = false;   // one-kernel iteration: variant64/32 are fused-kernel variants
    int check_variant = 0, check_lnk = 0;  // H_W stencil of the in-band check
    JobDesc* desc_dev = nullptr;
    int* kdev = nullptr;
    std::vector<char> retired;  // jobs taken out of the grids (every source finished)
};

void fill_desc(ovl_ctx* c, Work& w, JobDesc& d, const int (&variant)[2], const int (&lnk)[2],
               int (&sten_b0)[2], int& vec_b0) {
    d.g = c->g;
    d.kappa = kappa_of(c->m0);
    d.zs = c->zseed;
    d.U[0] = lnk[0] ? c->U64c.p : c->U64.p;
    d.U[1] = lnk[1] ? c->U32c.p : c->U32.p;
    d.nsrc = w.nsrc;
    d.nsb = wilson_blocks(c->g);
    for (int f = 0; f < 2; ++f) {
        d.sten_b0[f] = sten_b0[f];
        d.sten_nb[f] = w.fused ? iter_grid_blocks(c->g, w.nsrc)
                               : wilson_grid_blocks(c->g, w.nsrc, variant[f]);
        sten_b0[f] += job_grid_blocks(d.sten_nb[f]);
    }
    d.vec_b0 = vec_b0;
    d.nbe = w.nbe;
    vec_b0 += w.nbe * w.nsrc;
    d.st = w.st;
    d.sh = w.sh;
    d.part_w = w.part_w;
    d.part_stride = w.fused ? (size_t)w.nsrc * d.nsb : 0;
    d.qpp = w.fused ? w.qpp : 0;
    d.q[0] = w.q64; d.q[1] = w.q32;
    d.r[0] = w.r64; d.r[1] = w.r32;
    d.rpp = w.rpp;
    d.b64 = w.b64;
    d.s64 = w.s64;
    d.pj[0] = w.pj64; d.pj[1] = w.pj32;
    d.xj = w.xj;
    d.slots = w.slot_tab;
    d.slot_bytes = w.slot_bytes;
    d.h = nullptr;
    d.ksw = 1 << 30;
    d.form = c->form;
    d.phase = 0;
}

// Precision mode of a chunk: bit f set when some job iterates in precision f
// (0 FP64, 1 FP32).  Each job runs in its own phase; the kernels of one
// precision skip the blocks of jobs in the other.
int chunk_mode(const Batch& B) {
    int m = 0;
    for (size_t i = 0; i < B.desc.size(); ++i)
        if (B.retired.empty() || !B.retired[i]) m |= 1 << B.desc[i].phase;
    return m ? m : 1;
}

// Enqueue `count` seed iterations of every job, each in its own precision:
// per iteration the stencils of the precisions in `mode`, then their updates
// (both updates of an iteration write the same next counter).
void enqueue_chunk(const Batch& B, int mode, int count, hipStream_t s, bool prof,
                   int nact_total) {
    ovl_ctx* lead = B.ctx[0];
    const bool sweep = B.form == OVL_FORM_FUSED || B.form == OVL_FORM_REFERENCE;
    double vec_b[2] = {0, 0}, sweep_b[2] = {0, 0};
    if (prof) {
        for (size_t i = 0; i < B.w.size(); ++i) {
            const int f = B.desc[i].phase;
            const double es = f ? sizeof(float2) : sizeof(double2);
            const double V = (double)B.ctx[i]->g.V, n = B.w[i]->nsrc, N = 12 * V;
            vec_b[f] += 3.0 * es * N * n;  // r and q read, r written
            const bool ref = B.form == OVL_FORM_REFERENCE;
            sweep_b[f] += N * n * (ref ? 0.0 : 32.0);  // s read and written (fused sweep)
        }
        const int f0 = B.desc[0].phase;
        const double es0 = f0 ? sizeof(float2) : sizeof(double2);
        const double N0 = 12.0 * B.ctx[0]->g.V;
        sweep_b[f0] += N0 * nact_total * (2.0 * es0 + (B.form == OVL_FORM_REFERENCE ? 32.0 : 0.0));
    }
    const int vars[2] = {B.variant64, B.variant32};
    const int nj = (int)B.desc.size();
    for (int i = 0; i < count; ++i) {
        int* kr = B.kdev + (i & 1);
        int* kw = B.kdev + ((i + 1) & 1);
        if (B.fused) {
            for (int f = 0; f < 2; ++f) {
                if (!(mode & (1 << f))) continue;
                // bytes credited after the solve from the sources' live iterations
                ProfScope ps(lead, s, prof ? 8 + f : -1, 0.0, true);
                if (f) launch_iter_jobs<float>(B.desc_dev, nj, kr, kw, B.sten_total[1], vars[1],
                                               B.lnk[1], s, ps.start(), ps.stop());
                else launch_iter_jobs<double>(B.desc_dev, nj, kr, kw, B.sten_total[0], vars[0],
                                              B.lnk[0], s, ps.start(), ps.stop());
            }
            continue;
        }
        for (int f = 0; f < 2; ++f) {
            if (!(mode & (1 << f))) continue;
            // bytes credited after the solve from the sources' live iterations
            ProfScope ps(lead, s, prof ? 0 + f : -1, 0.0, true);
            if (f) launch_wilson_jobs<float>(B.desc_dev, nj, kr, B.sten_total[1], vars[1], B.lnk[1],
                                             s, ps.start(), ps.stop());
            else launch_wilson_jobs<double>(B.desc_dev, nj, kr, B.sten_total[0], vars[0], B.lnk[0],
                                            s, ps.start(), ps.stop());
        }
        for (int f = 0; f < 2; ++f) {
            if (!(mode & (1 << f))) continue;
            // K2: r update (r, q read, r written), with the sweep in the sweep forms
            ProfScope ps(lead, s, prof ? (sweep ? 4 + f : 2 + f) : -1,
                         sweep ? vec_b[f] + sweep_b[f] : 0.0, true);
            if (f) launch_iteration_update<float>(B.desc_dev, nj, kr, kw, B.vec_total, B.form,
                                                  B.maxJ, s, ps.start(), ps.stop());
            else launch_iteration_update<double>(B.desc_dev, nj, kr, kw, B.vec_total, B.form,
                                                 B.maxJ, s, ps.start(), ps.stop());
        }
    }
    // the chunk's final state to the pinned host slots (the counter after an
    // even number of iterations is in slot 0)
    launch_export_state(B.desc_dev, nj, B.kdev + (count & 1), kChunk, s);
}

// Capture (once per key) and replay a graph of kChunk iterations in precision
// mode `mode`.  The graph reads the job table from device memory at every
// replay, so the jobs' phases may change between replays.
int replay_chunk(Batch& B, int mode, hipStream_t s) {
    ovl_ctx* lead = B.ctx[0];
    char kb[256];
    snprintf(kb, sizeof(kb), "%p|%p|%zu|%d|%d|%d|%d|%d|%d|%d|%d|%d|%d", (void*)B.desc_dev,
             (void*)B.kdev, B.desc.size(), B.sten_total[0], B.sten_total[1], B.vec_total,
             B.variant64, B.variant32, B.form, B.maxJ, B.lnk[0], B.lnk[1], (int)B.fused);
    auto& gc = lead->graphs[mode - 1];
    if (!gc.exec || gc.key != kb) {
        if (gc.exec) (void)hipGraphExecDestroy(gc.exec);
        gc.exec = nullptr;
        hipGraph_t graph;
        HIPCHK(lead, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        enqueue_chunk(B, mode, kChunk, s, false, 0);
        HIPCHK(lead, hipStreamEndCapture(s, &graph));
        const hipError_t e = hipGraphInstantiate(&gc.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HIPCHK(lead, e);
        gc.key = kb;
    }
    HIPCHK(lead, hipGraphLaunch(gc.exec, s));
    return OVL_OK;
}

int run_chunk(Batch& B, bool graphs, hipStream_t s, int nact_total) {
    if (B.vec_total <= 0 || B.sten_total[0] <= 0 || B.sten_total[1] <= 0)
        return fail(B.ctx[0], OVL_E_STATE, "a chunk with no job left in the grids");
    const int mode = chunk_mode(B);
    if (graphs) return replay_chunk(B, mode, s);
    enqueue_chunk(B, mode, kChunk, s, B.ctx[0]->prof_on, nact_total);
    HIPCHK(B.ctx[0], hipGetLastError());
    return OVL_OK;
}

// Initial vectors and state of one job (r = p = b; s = 0; x_j = 0; slot 0 = b).
int init_job(ovl_ctx* c, Work& w, hipStream_t s) {
    const size_t vec64 = (size_t)w.nsrc * w.N * sizeof(double2);
    const int form = c->form;
    if (form == OVL_FORM_BASIS) {
        int rc = ensure_slots(c, w, kChunk + 1, s);
        if (rc) return rc;
        HIPCHK(c, hipMemcpyAsync(slot_ptr<double2>(w, 0), w.b64, vec64, hipMemcpyDeviceToDevice, s));
    } else {
        HIPCHK(c, hipMemcpyAsync(w.r64, w.b64, vec64, hipMemcpyDeviceToDevice, s));
    }
    if (form == OVL_FORM_FUSED) HIPCHK(c, hipMemsetAsync(w.s64, 0, vec64, s));
    if (form == OVL_FORM_REFERENCE) HIPCHK(c, hipMemsetAsync(w.xj, 0, vec64 * w.J, s));
    if (c->part_b.bytes < init_partials(w.N, w.sh.nslices, w.nsrc) * sizeof(double))
        return fail(c, OVL_E_STATE, "initialisation partials buffer too small");
    launch_init_state(w.st, w.b64, w.part_b, w.N, w.sh, s);
    HIPCHK(c, hipGetLastError());
    return OVL_OK;
}

// FP64 -> FP32 switch of one job at iteration k
void convert_job(ovl_ctx* c, Work& w, int k, hipStream_t s) {
    const int64_t n = (int64_t)w.nsrc * w.N;
    if (w.fused) {
        // the first FP32 kernel k reads r_{k-1} and q_{k-1}: slot k-1 (FP32
        // packed at its base from here on) or two-pass buffer (k-1)&1, and q[(k-1)&1]
        const int km = k - 1;
        launch_convert_64_to_32(w.q64 + (size_t)(km & 1) * w.qpp, w.q32 + (size_t)(km & 1) * w.qpp,
                                n, s);
        if (c->form == OVL_FORM_BASIS) {
            launch_convert_64_to_32(slot_ptr<double2>(w, km), w.r32, n, s);
            (void)hipMemcpyAsync(slot_ptr<float2>(w, km), w.r32, (size_t)n * sizeof(float2),
                                 hipMemcpyDeviceToDevice, s);
        } else {
            launch_convert_64_to_32(w.r64 + (size_t)(km & 1) * w.rpp, w.r32 + (size_t)(km & 1) * w.rpp,
                                    n, s);
        }
        return;
    }
    // the stencil of iteration k reads r_k and q_{k-1}
    launch_convert_64_to_32(w.q64, w.q32, n, s);
    if (c->form == OVL_FORM_BASIS) {
        launch_convert_64_to_32(slot_ptr<double2>(w, k), w.r32, n, s);
        (void)hipMemcpyAsync(slot_ptr<float2>(w, k), w.r32, (size_t)n * sizeof(float2),
                             hipMemcpyDeviceToDevice, s);
    } else if (c->form == OVL_FORM_TWOPASS) {
        launch_convert_64_to_32(w.r64 + (size_t)(k & 1) * w.rpp, w.r32 + (size_t)(k & 1) * w.rpp, n, s);
    } else {
        launch_convert_64_to_32(w.r64, w.r32, n, s);
        launch_convert_64_to_32(w.pj64, w.pj32, n * w.J, s);
    }
}

// Job i of the batch iterates in FP32 from iteration k on (its vectors
// converted after the work already queued).
void switch_job(Batch& B, size_t i, int k, hipStream_t s) {
    convert_job(B.ctx[i], *B.w[i], k, s);
    B.desc[i].phase = 1;
    launch_set_phase(B.desc_dev + i, 1, s);
}

// Parity of the newest active counts after `done` launches of the iteration:
// the two-kernel iteration k writes counts [(k+1)&1], the fused kernel k
// writes [k&1]; at the iteration limit the counts of the last live launch stay.
int count_parity(const Work& w, int done) {
    return w.fused ? std::min(done - 1, w.maxk) : std::min(done, w.maxk);
}

struct PollResult {
    int status = OVL_OK;
    bool all_done = true;
    double maxres = 0.0;
    int iters = 0, nact = 0;
    std::vector<double> job_res;  // per job: largest shifted residual estimate
    std::vector<char> job_done;   // per job: no live source
};

// Records ev after a chunk, whose last kernel has exported every job's state
// into pinned slot (chunk index & 1).
int post_state(Batch& B, hipStream_t s, hipEvent_t ev) {
    if (hipEventRecord(ev, s) != hipSuccess) return fail(B.ctx[0], OVL_E_HIP, "event record failed");
    return OVL_OK;
}

// Waits for ev (posted after the chunk that ends at iteration k_host) and
// evaluates the state copied into pinned slot `slot`.
PollResult read_state(Batch& B, int slot, int k_host, hipEvent_t ev, int* rc_out) {
    PollResult P;
    *rc_out = OVL_OK;
    if (hipEventSynchronize(ev) != hipSuccess) *rc_out = fail(B.ctx[0], OVL_E_HIP, "state wait failed");
    prof_collect(B.ctx[0]);
    P.job_res.assign(B.w.size(), 0.0);
    P.job_done.assign(B.w.size(), 1);
    for (size_t i = 0; i < B.w.size(); ++i) {
        ovl_ctx* c = B.ctx[i];
        Work& w = *B.w[i];
        const char* hb = host_slot(c, w, slot);
        const SrcState* hs = reinterpret_cast<const SrcState*>(hb);
        const int* hcnt = reinterpret_cast<const int*>(hb + state_cnt_off(w.nsrc)) +
                          (size_t)(count_parity(w, k_host) & 1) * w.nsrc * kMaxSlices;
        const double* hmres = reinterpret_cast<const double*>(hb + state_mres_off(w.nsrc));
        for (int n = 0; n < w.nsrc; ++n) {
            const SrcState& S = hs[n];
            if (S.status != OVL_OK && P.status == OVL_OK) P.status = S.status;
            int na = 0;
            for (int q = 0; q < w.sh.nslices; ++q) {
                na += hcnt[n * kMaxSlices + q];
                P.job_res[i] = std::max(P.job_res[i], hmres[n * kMaxSlices + q]);
            }
            const bool done = na == 0 || S.status != OVL_OK;
            P.job_done[i] = P.job_done[i] && done;
            P.all_done = P.all_done && done;
            P.iters = std::max(P.iters, S.iter);
            P.nact += na;
        }
        P.maxres = std::max(P.maxres, P.job_res[i]);
    }
    return P;
}

}  // namespace

// Profiling: algorithmic bytes of the stencil classes and of the r/p update
// of the basis and two-pass forms, from the sources' live iterations (the
// per-launch records cannot know them: a launch in which every source has
// finished returns at once and moves nothing).  A source live for iterations
// 0 .. iter-1 ran min(iter, k_switch) of them in FP64 and the rest in FP32,
// k_switch the iteration at which its job was converted (w.k_conv);
// a job's links are read once per launch in which any of its sources is live.
void credit_live_bytes(const Batch& B) {
    ovl_ctx* lead = B.ctx[0];
    if (!lead->prof_on) return;
    const bool sweep = B.form == OVL_FORM_FUSED || B.form == OVL_FORM_REFERENCE;
    for (size_t i = 0; i < B.w.size(); ++i) {
        const ovl_ctx* c = B.ctx[i];
        const Work& w = *B.w[i];
        const double V = (double)c->g.V;
        const SrcState* hs = reinterpret_cast<const SrcState*>(c->host_state);
        const int k_switch = w.k_conv;
        if (B.fused) {
            // kernel k is live for a source through k = iter (its last live
            // kernel records iter = k); FP64 below the first FP32 kernel
            // k_switch.  Per live source r_{k-1}, q_{k-1} read and r_k, q_k
            // written (kernel 0: b read, q_0 written), links once per launch.
            for (int f = 0; f < 2; ++f) {
                const double es = f ? (double)sizeof(float2) : (double)sizeof(double2);
                double vec = 0.0;
                int mx = 0;
                for (int n = 0; n < w.nsrc; ++n) {
                    const int last = std::min(hs[n].iter, w.maxk);  // kernels 0 .. last
                    const int ksw = k_switch < 0 ? last + 1 : std::min(k_switch, last + 1);
                    const int k0 = f ? ksw : 0, k1 = f ? last + 1 : ksw;  // [k0, k1)
                    if (k1 <= k0) continue;
                    vec += 48.0 * (k1 - k0) - (k0 == 0 ? 24.0 : 0.0);
                    mx = std::max(mx, k1 - k0);
                }
                lead->prof_bytes[8 + f] += V * es * (vec + (B.lnk[f] ? 24.0 : 36.0) * mx);
            }
            continue;
        }
        for (int f = 0; f < 2; ++f) {
            const double es = f ? (double)sizeof(float2) : (double)sizeof(double2);
            double sum = 0.0;
            int mx = 0;
            for (int n = 0; n < w.nsrc; ++n) {
                const int it = std::min(hs[n].iter, w.maxk);
                const int n64 = k_switch < 0 ? it : std::min(it, k_switch);
                const int itf = f ? it - n64 : n64;
                sum += itf;
                mx = std::max(mx, itf);
            }
            lead->prof_bytes[0 + f] += V * es * (36.0 * sum + (B.lnk[f] ? 24.0 : 36.0) * mx);
            if (!sweep) lead->prof_bytes[2 + f] += 3.0 * 12.0 * V * es * sum;
        }
    }
}

// Grid ranges of a batch: every job's blocks in the stencil grid of each
// precision and in the vector grid, in job order.  A retired job (every
// source finished) gets an empty range, so its blocks are no longer
// launched; a block never resolves to an empty range, whose job keeps its
// block counts.
static void layout_grids(Batch& B, const std::vector<char>& retired) {
    int sb[2] = {0, 0}, vb = 0;
    for (size_t i = 0; i < B.desc.size(); ++i) {
        JobDesc& d = B.desc[i];
        const bool live = retired.empty() || !retired[i];
        for (int f = 0; f < 2; ++f) {
            d.sten_b0[f] = sb[f];
            if (live) sb[f] += job_grid_blocks(d.sten_nb[f]);
        }
        d.vec_b0 = vb;
        if (live) vb += d.nbe * d.nsrc;
    }
    B.sten_total[0] = sb[0];
    B.sten_total[1] = sb[1];
    B.vec_total = vb;
}

// Builds the job table of a batch for its current variants and link formats
// (grid offsets per job and precision, state export slots), every job in
// precision phase `phase`, and uploads it.
static int build_desc(Batch& B, hipStream_t s, int phase = 0) {
    ovl_ctx* lead = B.ctx[0];
    B.maxJ = 0;
    B.desc.resize(B.w.size());
    int sb[2] = {0, 0}, vb = 0;
    const int vars[2] = {B.variant64, B.variant32};
    for (size_t i = 0; i < B.w.size(); ++i) {
        fill_desc(B.ctx[i], *B.w[i], B.desc[i], vars, B.lnk, sb, vb);
        B.maxJ = std::max(B.maxJ, B.w[i]->J);
        // the chunk kernels export the state into the pinned slots
        JobDesc& d = B.desc[i];
        void* hdev = nullptr;
        HIPCHK(lead, hipHostGetDevicePointer(&hdev, B.ctx[i]->host_state, 0));
        d.state_dev = reinterpret_cast<const char*>(B.w[i]->st);
        d.state_host = static_cast<char*>(hdev);
        d.state_bytes = (int)B.w[i]->state_bytes;
        d.state_stride = (int)state_slot_bytes(*B.w[i]);
        d.phase = phase;
    }
    B.sten_total[0] = sb[0];
    B.sten_total[1] = sb[1];
    B.vec_total = vb;
    const size_t dbytes = (B.desc.size() * sizeof(JobDesc) + 255) & ~(size_t)255;
    HIPCHK(lead, lead->jobs_dev.ensure(dbytes + 256));
    B.desc_dev = lead->jobs_dev.as<JobDesc>();
    B.kdev = reinterpret_cast<int*>(lead->jobs_dev.as<char>() + dbytes);
    HIPCHK(lead, hipMemcpyAsync(B.desc_dev, B.desc.data(), B.desc.size() * sizeof(JobDesc),
                                hipMemcpyHostToDevice, s));
    return OVL_OK;
}

// In-solver tuning of the two-kernel iteration's stencil (basis forms) in
// precision prec: every variant in every allowed link format runs one chunk
// of kChunk real iterations of this batch from its initial state (in FP32
// from iteration 0 for prec 1), timed with events on the solve stream; the
// four fastest run twice more, and the choice with the fastest run goes to
// *code.  The runs are discarded (the solve starts
// again from the initial state), so results do not depend on the tuning.  In
// the solver the stencil reads vectors the previous kernel has just written,
// which a stand-alone timing (cold caches, or warm from repeated launches on
// the same inputs) does not reproduce.
static int tune_solver_stencil(Batch& B, hipStream_t s, int prec, bool all12, int* code) {
    ovl_ctx* lead = B.ctx[0];
    const int nfmt = all12 ? 2 : 1;
    const char* vb = getenv("OVL_AUTOTUNE_VERBOSE");
    const bool verbose = vb && vb[0] == '1';
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(lead, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(lead, OVL_E_HIP, "event creation failed");
    }
    struct Ev {
        hipEvent_t a, b;
        ~Ev() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
    } evg{e0, e1};
    // one timed chunk of choice c (after an untimed one, from the initial state)
    auto time_choice = [&](int c, float* ms) -> int {
        const int v = c % kStencilVariants, lnk = c / kStencilVariants;
        if (prec) { B.variant32 = v; B.lnk[1] = lnk; } else { B.variant64 = v; B.lnk[0] = lnk; }
        int rc = build_desc(B, s, prec);
        if (rc) return rc;
        for (size_t i = 0; i < B.w.size(); ++i) {
            rc = init_job(B.ctx[i], *B.w[i], s);
            if (rc) return rc;
            // the two chunks below run iterations 0 .. 2 kChunk - 1, whose
            // updates write basis slots up to 2 kChunk: every slot chunk they
            // touch must exist and be published in the device table first
            if (B.ctx[i]->form == OVL_FORM_BASIS) {
                rc = ensure_slots(B.ctx[i], *B.w[i], 2 * kChunk + 1, s);
                if (rc) return rc;
            }
            if (prec) convert_job(B.ctx[i], *B.w[i], 0, s);
            if (B.ctx[i]->form == OVL_FORM_BASIS && !slots_cover(*B.w[i], 2 * kChunk))
                return fail(lead, OVL_E_STATE, "basis slots for the tuning chunks are missing");
        }
        HIPCHK(lead, hipMemsetAsync(B.kdev, 0, 2 * sizeof(int), s));
        enqueue_chunk(B, 1 << prec, kChunk, s, false, 0);
        HIPCHK(lead, hipEventRecord(e0, s));
        enqueue_chunk(B, 1 << prec, kChunk, s, false, 0);
        HIPCHK(lead, hipEventRecord(e1, s));
        HIPCHK(lead, hipEventSynchronize(e1));
        HIPCHK(lead, hipEventElapsedTime(ms, e0, e1));
        if (verbose)
            fprintf(stderr, "ovl in-solver tune %s: choice %d (variant %d, %s links) %.2f us/iteration\n",
                    prec ? "fp32" : "fp64", c, v, lnk ? "two-row" : "full", *ms * 1e3 / kChunk);
        return OVL_OK;
    };
    // every choice once, then the fastest few twice more each: a choice's
    // time is its fastest run, so one slow sample does not decide between
    // choices a few per cent apart
    const int nc = kStencilVariants * nfmt;
    std::vector<float> t(nc);
    for (int c = 0; c < nc; ++c) {
        int rc = time_choice(c, &t[c]);
        if (rc) return rc;
    }
    std::vector<int> order(nc);
    for (int c = 0; c < nc; ++c) order[c] = c;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return t[a] < t[b]; });
    constexpr int kFinalists = 4, kRepeats = 2;
    for (int rep = 0; rep < kRepeats; ++rep)
        for (int f = 0; f < kFinalists && f < nc; ++f) {
            float ms = 0.f;
            int rc = time_choice(order[f], &ms);
            if (rc) return rc;
            t[order[f]] = std::min(t[order[f]], ms);
        }
    int best = order[0];
    for (int f = 1; f < kFinalists && f < nc; ++f)
        if (t[order[f]] < t[best]) best = order[f];
    *code = best;
    return OVL_OK;
}

// Runs the shifted solver for every job of a batch (their sources packed in
// w->b64) and leaves s = sum_j c_j y_j in each w->s64.  Work is enqueued on
// the lead context's solve stream after its caller stream.  Returns a status
// and fills ctx->last of every context.
static int solve_batch_once(Batch& B) {
    ovl_ctx* lead = B.ctx[0];
    hipStream_t s;
    int rc = solve_stream(lead, &s);
    if (rc) return rc;
    HIPCHK(lead, hipEventRecord(lead->ev_in, lead->stream));
    HIPCHK(lead, hipStreamWaitEvent(s, lead->ev_in, 0));
    // On every return from here on, whether the solve succeeded or not, the
    // caller's stream waits for everything queued on the solve stream (so a
    // caller never reads buffers the solve may still write), and the timing
    // events are released.
    struct SolveScope {
        ovl_ctx* lead;
        hipStream_t s;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        ~SolveScope() {
            if (hipEventRecord(lead->ev_out, s) == hipSuccess)
                (void)hipStreamWaitEvent(lead->stream, lead->ev_out, 0);
            else
                (void)hipStreamSynchronize(s);
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
        }
    } scope{lead, s};
    const bool mixed = lead->precision == OVL_PREC_MIXED;
    const int form = lead->form;
    const bool graphs = graphs_enabled(lead);
    const int maxk = lead->maxiter;
    HIPCHK(lead, hipEventCreate(&scope.e0));
    HIPCHK(lead, hipEventCreate(&scope.e1));
    hipEvent_t e0 = scope.e0, e1 = scope.e1;
    HIPCHK(lead, hipEventRecord(e0, s));
    B.form = form;
    // stencil variants: those tuned for the largest job
    size_t big = 0;
    for (size_t i = 1; i < B.w.size(); ++i)
        if (B.ctx[i]->g.V * B.w[i]->nsrc > B.ctx[big]->g.V * B.w[big]->nsrc) big = i;
    // the two-row link form only where every job's field is SU(3)
    bool all12 = true;
    for (ovl_ctx* c : B.ctx) all12 = all12 && c->links12;
    B.fused = B.w[0]->fused;
    for (Work* w : B.w)
        if (w->fused != B.fused) return fail(lead, OVL_E_ARG, "mixed iteration kinds in one batch");
    if (B.fused) {
        // fused iteration: its own variants (hops per step, block order, LDS tile)
        const int c64 = iter_variant(B.ctx[big], B.w[big]->nsrc, 0);
        const int c32 = mixed ? iter_variant(B.ctx[big], B.w[big]->nsrc, 1) : 0;
        B.variant64 = c64 % kIterVariants;
        B.variant32 = c32 % kIterVariants;
        B.lnk[0] = all12 ? c64 / kIterVariants : 0;
        B.lnk[1] = all12 ? c32 / kIterVariants : 0;
        // the H_W stencil with the same hops per step, order and tile
        const int v = B.variant64;
        B.check_variant = (v & 1) + 4 * ((v >> 1) & 1) + 16 * ((v >> 2) & 1);
    } else {
        int c64 = stencil_lookup(B.ctx[big], B.w[big]->nsrc, 0, 1);
        int c32 = mixed ? stencil_lookup(B.ctx[big], B.w[big]->nsrc, 1, 1) : 0;
        const bool in_solver = form == OVL_FORM_BASIS || form == OVL_FORM_TWOPASS;
        if (c64 < 0 && in_solver) {
            rc = tune_solver_stencil(B, s, 0, all12, &c64);
            if (rc) return rc;
            stencil_store(B.ctx[big], B.w[big]->nsrc, 0, 1, c64);
        }
        if (c32 < 0 && in_solver) {
            rc = tune_solver_stencil(B, s, 1, all12, &c32);
            if (rc) return rc;
            stencil_store(B.ctx[big], B.w[big]->nsrc, 1, 1, c32);
        }
        if (c64 < 0) c64 = stencil_variant(B.ctx[big], B.w[big]->nsrc, 0, 1);
        if (c32 < 0) c32 = stencil_variant(B.ctx[big], B.w[big]->nsrc, 1, 1);
        B.variant64 = c64 % kStencilVariants;
        B.variant32 = c32 % kStencilVariants;
        B.lnk[0] = all12 ? c64 / kStencilVariants : 0;
        B.lnk[1] = all12 ? c32 / kStencilVariants : 0;
        B.check_variant = B.variant64;
    }
    B.check_lnk = B.lnk[0];
    rc = build_desc(B, s);
    if (rc) return rc;
    for (size_t i = 0; i < B.w.size(); ++i) {
        rc = init_job(B.ctx[i], *B.w[i], s);
        if (rc) return rc;
    }
    HIPCHK(lead, hipMemsetAsync(B.kdev, 0, 2 * sizeof(int), s));  // outside any captured graph

    int status = OVL_OK;
    for (Work* w : B.w) w->k_conv = -1;
    int k_host = 0;  // iterations whose state the host has read
    int k_enq = 0;   // iterations queued
    PollResult P;
    P.maxres = 1.0;
    int nact_known = 0;
    for (size_t i = 0; i < B.w.size(); ++i) nact_known += B.w[i]->J * B.w[i]->nsrc;
    std::vector<char>& retired = B.retired;
    retired.assign(B.w.size(), 0);
    hipEvent_t pev[2];
    HIPCHK(lead, hipEventCreateWithFlags(&pev[0], hipEventDisableTiming));
    HIPCHK(lead, hipEventCreateWithFlags(&pev[1], hipEventDisableTiming));
    struct EvGuard {
        hipEvent_t* e;
        ~EvGuard() { (void)hipEventDestroy(e[0]); (void)hipEventDestroy(e[1]); }
    } evg{pev};
    // one chunk of kChunk iterations, then the copy of its state into pinned
    // slot (chunk index & 1)
    auto queue_chunk = [&]() -> int {
        if (form == OVL_FORM_BASIS)
            for (size_t i = 0; i < B.w.size(); ++i) {
                const int r = ensure_slots(B.ctx[i], *B.w[i], k_enq + kChunk + 1, s);
                if (r) return r;
                if (!slots_cover(*B.w[i], k_enq + kChunk))
                    return fail(lead, OVL_E_STATE, "basis slots for iterations up to %d missing",
                                k_enq + kChunk);
            }
        int r = run_chunk(B, graphs, s, nact_known);
        if (r) return r;
        k_enq += kChunk;
        const int slot = (k_enq / kChunk) & 1;
        return post_state(B, s, pev[slot]);
    };
    // Look-ahead: while every job is far from its next decision point (its
    // own precision switch, then the tolerance), the chunk after the polled
    // one is queued before the host waits, so the device does not idle
    // through the poll.  Within a factor 10 of such a point the loop polls
    // each chunk before queueing the next, so every switch and the stop fall
    // on the same iteration as with one chunk in flight.  A chunk queued past
    // convergence finds no live source and returns at once.  Profiling keeps
    // one chunk in flight (its events are read at each poll).
    const bool may_look_ahead = !lead->prof_on;
    auto far_from_decisions = [&]() {
        if (!(P.maxres > 10.0 * lead->tol)) return false;
        if (!mixed) return true;
        if (P.job_res.empty()) return P.maxres > 10.0 * lead->switch_res;  // no poll yet
        for (size_t i = 0; i < B.w.size(); ++i)
            if (B.desc[i].phase == 0 && !P.job_done[i] && !(P.job_res[i] > 10.0 * lead->switch_res))
                return false;
        return true;
    };
    // launches the iteration may take: the two-kernel iteration k < maxk; the
    // fused kernel k <= maxk (kernel k advances the shifts by iteration k-1)
    const int klim = B.fused ? maxk + 1 : maxk;
    while (k_host < klim) {
        if (k_enq == k_host) {
            rc = queue_chunk();
            if (rc) return rc;
        }
        if (may_look_ahead && k_enq == k_host + kChunk && k_enq < klim && far_from_decisions()) {
            rc = queue_chunk();
            if (rc) return rc;
        }
        k_host += kChunk;
        int prc;
        const int slot = (k_host / kChunk) & 1;
        P = read_state(B, slot, k_host, pev[slot], &prc);
        if (prc) return prc;
        nact_known = P.nact;
        if (P.status != OVL_OK) { status = P.status; break; }
        if (P.all_done) break;
        if (mixed && k_host < klim) {
            // relaxed precision, job by job: once a job's largest shifted
            // residual is below switch_res the remaining corrections are small
            // enough that FP32 vectors perturb its result by ~eps32 * switch_res.
            // The conversion follows any chunk still queued; the other jobs
            // go on in their own precision.
            for (size_t i = 0; i < B.w.size(); ++i)
                if (B.desc[i].phase == 0 && !P.job_done[i] && P.job_res[i] < lead->switch_res) {
                    B.w[i]->k_conv = k_enq;
                    switch_job(B, i, k_enq, s);
                }
            HIPCHK(lead, hipGetLastError());
        }
        // a batch's finished jobs leave the grids (after any chunk still
        // queued); their active counts are cleared in both parities, so every
        // later read of their state finds them finished
        if (!B.fused && B.w.size() > 1) {
            bool change = false;
            for (size_t i = 0; i < B.w.size(); ++i)
                if (P.job_done[i] && !retired[i]) {
                    retired[i] = 1;
                    change = true;
                    HIPCHK(lead, hipMemsetAsync(B.w[i]->sh.cnt, 0,
                                                (size_t)2 * B.w[i]->nsrc * kMaxSlices * sizeof(int), s));
                }
            if (change) {
                layout_grids(B, retired);
                HIPCHK(lead, hipMemcpyAsync(B.desc_dev, B.desc.data(),
                                            B.desc.size() * sizeof(JobDesc), hipMemcpyHostToDevice, s));
            }
        }
    }
    // a chunk queued past the last poll: its state is the final one
    if (k_enq > k_host) {
        int prc;
        const int slot = (k_enq / kChunk) & 1;
        const PollResult Q = read_state(B, slot, k_enq, pev[slot], &prc);
        if (prc) return prc;
        if (status == OVL_OK) status = Q.status;
        P.all_done = P.all_done || Q.all_done;
        k_host = k_enq;
    }
    // the final state into slot 0, where the code below reads it
    if (((k_host / kChunk) & 1) != 0)
        for (size_t i = 0; i < B.w.size(); ++i)
            memcpy(B.ctx[i]->host_state, host_slot(B.ctx[i], *B.w[i], 1), B.w[i]->state_bytes);
    credit_live_bytes(B);
    const int k_run = k_host;
    if (status == OVL_OK && !P.all_done) status = OVL_NOT_CONVERGED;
    for (size_t i = 0; i < B.w.size(); ++i) {
        // first slot holding FP32 (the fused kernel k reads slot k-1, which the
        // switch to FP32 before kernel k converted)
        const int kc = B.w[i]->k_conv;
        B.w[i]->k_switch = kc < 0 ? -1 : (B.fused ? kc - 1 : kc);
        B.w[i]->K = 0;
        for (int n = 0; n < B.w[i]->nsrc; ++n) B.w[i]->K = std::max(B.w[i]->K, B.ctx[i]->host_state[n].iter);
    }
    if (status == OVL_OK || status == OVL_NOT_CONVERGED) {
        for (size_t i = 0; i < B.w.size(); ++i) {
            ovl_ctx* c = B.ctx[i];
            Work& w = *B.w[i];
            const int64_t N = w.N;
            const double Na = 12.0 * (double)c->g.V;  // algorithmic elements per source
            if (form == OVL_FORM_REFERENCE) {
                launch_sum_ref(w.xj, w.cj, w.s64, w.J, N, w.nsrc, s);
            } else if (form == OVL_FORM_BASIS || form == OVL_FORM_TWOPASS) {
                launch_basis_coef(w.h_a, w.h_b, w.h_pi, w.cj, w.st, w.W, w.h, w.J, w.maxk, w.nsrc, s);
            }
            if (form == OVL_FORM_BASIS) {
                // s = sum_i h_i r_i over every stored slot in one pass; FP64 slots
                // below k_switch, FP32 from it.  With the in-band check the same
                // pass rebuilds each source's checked shifted solution
                // x = sum_i u_i^j r_i into p64 (free after the solve).
                const int kend = w.K + 1;
                const int ksw = w.k_switch < 0 ? kend : w.k_switch;
                if (w.hx)
                    launch_pick_check(w.sh.res, w.W, w.zj, w.st, w.J, w.maxk, w.nsrc, w.hx, w.zc, s);
                {
                    // every stored slot in one launch, s (and x) written once; the
                    // device table must hold every chunk up to slot kend - 1
                    if (!slots_cover(w, kend - 1))
                        return fail(lead, OVL_E_STATE, "basis slots up to %d not in the table",
                                    kend - 1);
                    const int n64 = std::min(kend, ksw), n32 = kend - n64;
                    ProfScope ps(lead, s, 6, Na * w.nsrc * (16.0 * n64 + 8.0 * n32 + (w.hx ? 32.0 : 16.0)));
                    launch_basis_sum(w.slot_tab, w.slot_bytes, kend, ksw, w.h, w.hx, w.maxk, w.st,
                                     w.s64, w.p64, N, w.nsrc, s);
                }
                if (w.hx) {
                    // true residual of the rebuilt solution in FP64: H x (the FP64
                    // stencil of the solve, here as H_W alone), then per-block
                    // |b - (z x - H x)|^2 and |b|^2, copied to pinned host memory
                    // and summed on the host after the final synchronisation
                    launch_wilson<double>(0, w.p64, w.q64, stencil_links<double>(c, B.check_lnk),
                                          c->g, kappa_of(c->m0), make_double2(0, 0), nullptr,
                                          nullptr, nullptr, nullptr, 0, w.nsrc, s,
                                          B.check_variant, B.check_lnk);
                    launch_true_res_multi(w.b64, w.p64, w.q64, w.zc, w.cpart, kChkBlocks, N,
                                          w.nsrc, s);
                    HIPCHK(c, hipMemcpyAsync(w.chost, w.cpart,
                                             (size_t)w.nsrc * kChkBlocks * sizeof(double2),
                                             hipMemcpyDeviceToHost, s));
                }
            }
            HIPCHK(c, hipGetLastError());
        }
        if (form == OVL_FORM_TWOPASS) {
            // second pass: the same iterations again (bitwise identical, the
            // reductions being deterministic), now adding h_{k+1} r_{k+1} to s
            for (size_t i = 0; i < B.w.size(); ++i) {
                Work& w = *B.w[i];
                rc = init_job(B.ctx[i], w, s);
                if (rc) return rc;
                launch_s_init(w.b64, w.h, w.maxk, w.s64, w.N, w.nsrc, s);
                B.desc[i].h = w.h;
                B.desc[i].state_host = nullptr;  // the host keeps the first pass's final state
                B.desc[i].phase = 0;
            }
            std::fill(retired.begin(), retired.end(), 0);
            layout_grids(B, retired);
            HIPCHK(lead, hipMemcpyAsync(B.desc_dev, B.desc.data(), B.desc.size() * sizeof(JobDesc),
                                        hipMemcpyHostToDevice, s));
            HIPCHK(lead, hipMemsetAsync(B.kdev, 0, 2 * sizeof(int), s));
            for (int k2 = 0; k2 < k_run; k2 += kChunk) {
                // every job switches at the iteration of its first pass, and
                // leaves the grids once the iterations of its first pass are done
                bool change = false;
                for (size_t i = 0; i < B.w.size(); ++i) {
                    if (mixed && B.w[i]->k_conv == k2) switch_job(B, i, k2, s);
                    if (!B.fused && B.w.size() > 1 && !retired[i] && B.w[i]->K <= k2) {
                        retired[i] = 1;
                        change = true;
                    }
                }
                if (change) {
                    layout_grids(B, retired);
                    // every job done: the first pass's last chunks (queued
                    // ahead of its final poll) have nothing left to repeat
                    if (B.vec_total == 0) break;
                    HIPCHK(lead, hipMemcpyAsync(B.desc_dev, B.desc.data(),
                                                B.desc.size() * sizeof(JobDesc),
                                                hipMemcpyHostToDevice, s));
                }
                rc = run_chunk(B, graphs, s, nact_known);
                if (rc) return rc;
            }
            credit_live_bytes(B);  // the second pass repeats the same iterations
            HIPCHK(lead, hipGetLastError());
        }
    }
    // constant term of the rational function (single-contour form)
    if (lead->c0 != 0.0)
        for (size_t i = 0; i < B.w.size(); ++i)
            launch_axpy(B.w[i]->s64, B.w[i]->b64, lead->c0, (int64_t)B.w[i]->nsrc * B.w[i]->N, s);
    HIPCHK(lead, hipEventRecord(e1, s));
    HIPCHK(lead, hipEventSynchronize(e1));
    prof_collect(lead);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    // (the results go back to the caller's stream when `scope` ends)
    for (size_t i = 0; i < B.w.size(); ++i) {
        ovl_ctx* c = B.ctx[i];
        Work& w = *B.w[i];
        int na = 0;
        double mr = 0.0;
        const char* hb = reinterpret_cast<const char*>(c->host_state);
        const int* hcnt = reinterpret_cast<const int*>(hb + state_cnt_off(w.nsrc)) +
                          (size_t)(count_parity(w, k_run) & 1) * w.nsrc * kMaxSlices;
        const double* hmres = reinterpret_cast<const double*>(hb + state_mres_off(w.nsrc));
        for (int n = 0; n < w.nsrc; ++n)
            for (int q = 0; q < w.sh.nslices; ++q) {
                na += hcnt[n * kMaxSlices + q];
                mr = std::max(mr, hmres[n * kMaxSlices + q]);
            }
        // iteration counts per rhs, for ovl_spectral_bounds
        {
            const SrcState* hs = reinterpret_cast<const SrcState*>(c->host_state);
            c->last_iters.resize(w.nsrc);
            for (int n = 0; n < w.nsrc; ++n) c->last_iters[n] = std::min(hs[n].iter, w.maxk);
            c->last_maxk = w.maxk;
        }
        ovl_stats& L = c->last;
        std::memset(&L, 0, sizeof(L));
        L.iterations = w.K;
        L.fp32_iterations = w.k_switch < 0 ? 0 : std::max(0, w.K - w.k_switch);
        L.n_shifts = w.J;
        L.n_active_end = na;
        L.max_est_rel_res = mr;
        L.seconds = ms * 1e-3;
        if (B.fused) {
            L.stencil_variant64 = 1000 + B.variant64 + kIterVariants * B.lnk[0];
            L.stencil_variant32 = mixed ? 1000 + B.variant32 + kIterVariants * B.lnk[1] : -1;
        } else {
            L.stencil_variant64 = B.variant64 + kStencilVariants * B.lnk[0];
            L.stencil_variant32 = mixed ? B.variant32 + kStencilVariants * B.lnk[1] : -1;
        }
        L.max_true_rel_res = -1.0;
        L.mixed_true_rel_res = -1.0;
        if (w.hx && (status == OVL_OK || status == OVL_NOT_CONVERGED)) {
            // in-band check: the checked shift of every source, partials summed in order
            double worst = 0.0;
            for (int n = 0; n < w.nsrc; ++n) {
                double tt = 0.0, bb = 0.0;
                for (int b = 0; b < kChkBlocks; ++b) {
                    tt += w.chost[(size_t)n * kChkBlocks + b].x;
                    bb += w.chost[(size_t)n * kChkBlocks + b].y;
                }
                if (bb > 0.0) worst = std::max(worst, std::sqrt(tt / bb));
                else if (!(bb == 0.0)) worst = bb;  // NaN propagates
            }
            L.max_true_rel_res = worst;
        }
        if (status < 0) fail(c, status, "solver stopped: %s", ovl_status_string(status));
        if (status == OVL_NOT_CONVERGED)
            fail(c, status, "maxiter=%d reached with %d shifts above tol (max est. res %.3e)",
                 w.maxk, na, mr);
    }
    return status;
}

// The bound on the in-band true residual of a mixed-precision apply.  The
// FP32 phase of a job starts when its every shifted residual is below
// switch_res; from there on FP32 matvecs and vectors add to the true
// residual a drift of a few eps32 * switch_res (measured at 16^4 on the
// shift active longest: 1.9e-9, 1.3e-10 and 1.9e-11 at switch 1e-2, 1e-3
// and 1e-4, 2 to 3 eps32 switch_res), which the recurrence's estimates do
// not see.  Default: max(10 tol, 10 eps32 switch_res), so a repeat means
// more drift than that mechanism gives.
static double mixed_check_bound(const ovl_ctx* c) {
    if (c->check_bound > 0.0) return c->check_bound;
    const double eps32 = 5.960464477539063e-8;  // 2^-24
    return std::max(10.0 * c->tol, 10.0 * eps32 * c->switch_res);
}

// solve_batch_once, and in mixed precision its safeguard: when every shift
// met the tolerance by its residual estimate but the in-band FP64 check finds
// a true residual above the bound (mixed_check_bound) in some job, the whole
// batch is solved again in FP64 and the stats of every context say so; if
// that still misses 10 tol, the status is OVL_NOT_CONVERGED.
static int solve_batch(Batch& B) {
    int rc = solve_batch_once(B);
    ovl_ctx* lead = B.ctx[0];
    if (rc != OVL_OK || lead->precision != OVL_PREC_MIXED) return rc;
    double limit = mixed_check_bound(lead);
    auto failed = [&]() {
        for (ovl_ctx* c : B.ctx)
            if (!(c->last.max_true_rel_res <= limit) && c->last.max_true_rel_res != -1.0) return true;
        return false;
    };
    if (!failed()) return rc;
    std::vector<double> first(B.ctx.size());
    for (size_t i = 0; i < B.ctx.size(); ++i) {
        first[i] = B.ctx[i]->last.max_true_rel_res;
        B.ctx[i]->precision = OVL_PREC_FP64;
    }
    rc = solve_batch_once(B);
    for (size_t i = 0; i < B.ctx.size(); ++i) {
        B.ctx[i]->precision = OVL_PREC_MIXED;
        B.ctx[i]->last.fp64_repeat = 1;
        B.ctx[i]->last.mixed_true_rel_res = first[i];
    }
    limit = std::max(limit, 10.0 * lead->tol);
    if (rc == OVL_OK && failed()) {
        rc = OVL_NOT_CONVERGED;
        for (ovl_ctx* c : B.ctx)
            fail(c, rc, "true residual %.3e above %.3e after the FP64 repeat",
                 c->last.max_true_rel_res, limit);
    }
    return rc;
}

static int solve(ovl_ctx* ctx, Work& w) {
    Batch B;
    B.ctx.push_back(ctx);
    B.w.push_back(&w);
    return solve_batch(B);
}

static int materialize(ovl_ctx* ctx, const Work& w, int j0, int jn, double2* Y, int n, int K);

// True residuals ||b - (z_j - H) x_j|| / ||b|| of the last solve for the
// first ctx->check_n shifts of each source in the in-band check's order
// (active longest, then largest final estimate, then lower j; the reference
// form by the estimate alone).  x_j is stored by the reference form and
// rebuilt from the stored basis by the basis form; the fused and two-pass
// forms keep neither, and report -1.  Diagnostic: synchronous.
static int true_residuals(ovl_ctx* ctx, const Work& w) {
    if (ctx->check_n <= 0 || (ctx->form != OVL_FORM_BASIS && ctx->form != OVL_FORM_REFERENCE))
        return OVL_OK;
    hipStream_t s = ctx->stream;
    const int J = w.J;
    const int64_t N = w.N;
    const int nblk = 256;
    std::vector<double> est((size_t)w.nsrc * J);
    HIPCHK(ctx, hipStreamSynchronize(s));
    HIPCHK(ctx, hipMemcpy(est.data(), w.sh.res, est.size() * sizeof(double), hipMemcpyDeviceToHost));
    HIPCHK(ctx, ctx->chk.ensure((size_t)2 * N * sizeof(double2) + nblk * sizeof(double2)));
    double2* X = ctx->chk.as<double2>();
    double2* HX = X + N;
    double2* part = HX + N;
    const int code = stencil_variant(ctx, 1, 0, 0);
    const int var = code % kStencilVariants, lnk = code / kStencilVariants;
    const SrcState* hs = reinterpret_cast<const SrcState*>(ctx->host_state);
    std::vector<double2> hp(nblk);
    double worst = 0.0;
    for (int n = 0; n < w.nsrc; ++n) {
        std::vector<int> order(J);
        for (int j = 0; j < J; ++j) order[j] = j;
        const double* e = est.data() + (size_t)n * J;
        // basis form: shifts that stayed active longest first (last nonzero
        // coefficient u_i^j), as the in-band check picks them; then the
        // largest final estimate (the only order for the reference form)
        std::vector<int> last(J, 0);
        if (ctx->form == OVL_FORM_BASIS && w.W) {
            const int K = hs[n].iter;
            std::vector<double2> Wn((size_t)std::max(K, 1) * J);
            if (K > 0)
                HIPCHK(ctx, hipMemcpy(Wn.data(), w.W + (size_t)n * (w.maxk + 1) * J,
                                      (size_t)K * J * sizeof(double2), hipMemcpyDeviceToHost));
            for (int j = 0; j < J; ++j) {
                // the same bisection as the in-band pick (nonzero while active)
                int lo = -1, hi = K;
                while (hi - lo > 1) {
                    const int mid = (lo + hi) / 2;
                    const double2 u = Wn[(size_t)mid * J + j];
                    if (u.x != 0.0 || u.y != 0.0) lo = mid;
                    else hi = mid;
                }
                last[j] = lo;
            }
        }
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            return last[a] != last[b] ? last[a] > last[b] : e[a] > e[b];
        });
        const int m = std::min(ctx->check_n, J);
        for (int q = 0; q < m; ++q) {
            const int j = order[q];
            const double2* x;
            if (ctx->form == OVL_FORM_REFERENCE) {
                x = w.xj + ((size_t)n * J + j) * N;
            } else {
                const int rc = materialize(ctx, w, j, 1, X, n, hs[n].iter);
                if (rc) return rc;
                x = X;
            }
            launch_wilson<double>(0, x, HX, stencil_links<double>(ctx, lnk), ctx->g, kappa_of(ctx->m0),
                                  make_double2(0, 0), nullptr, nullptr, nullptr, nullptr, 0, 1, s,
                                  var, lnk);
            launch_true_res(w.b64 + (size_t)n * N, x, HX, ctx->z[j], part, nblk, N, s);
            HIPCHK(ctx, hipGetLastError());
            HIPCHK(ctx, hipMemcpyAsync(hp.data(), part, nblk * sizeof(double2),
                                       hipMemcpyDeviceToHost, s));
            HIPCHK(ctx, hipStreamSynchronize(s));
            double tt = 0.0, bb = 0.0;
            for (int b = 0; b < nblk; ++b) {
                tt += hp[b].x;
                bb += hp[b].y;
            }
            if (bb > 0.0) worst = std::max(worst, std::sqrt(tt / bb));
        }
    }
    ctx->last.max_true_rel_res = std::max(ctx->last.max_true_rel_res, worst);
    return OVL_OK;
}

extern "C" int ovl_set_check_bound(ovl_ctx* ctx, double bound) {
    if (!ctx) return OVL_E_ARG;
    if (!(bound >= 0.0) || !std::isfinite(bound))
        return fail(ctx, OVL_E_ARG, "the bound must be finite and >= 0");
    ctx->check_bound = bound;
    return OVL_OK;
}

extern "C" int ovl_set_residual_check(ovl_ctx* ctx, int32_t nsample) {
    if (!ctx) return OVL_E_ARG;
    if (nsample < -1 || nsample > 64) return fail(ctx, OVL_E_ARG, "nsample must be in [-1, 64]");
    ctx->check_n = nsample < 0 ? 0 : nsample;
    ctx->inband_check = nsample >= 0;
    return OVL_OK;
}

// ---------------------------------------------------------------------------
// spectral bounds from the seed recurrence and a contour suggestion
// ---------------------------------------------------------------------------
// The seed iteration is a Lanczos process on H: with A = z_s - H,
//   A r_k = -(beta_{k-1}/alpha_{k-1}) r_{k-1} + (1/alpha_k + beta_{k-1}/alpha_{k-1}) r_k
//           - (1/alpha_k) r_{k+1},
// so in the orthonormal basis v_k = r_k/||r_k|| the matrix of H is tridiagonal
// T with diagonal z_s - (1/alpha_k + beta_{k-1}/alpha_{k-1}) (real up to
// rounding) and off-diagonal moduli e_k = ||r_{k+1}|| / (|alpha_k| ||r_k||).
// Its eigenvalues (Ritz values) lie inside the spectrum's hull and converge
// to the extreme eigenvalues first.  Near zero, Ritz values of an indefinite
// H may fall into the gap; those of H^2 on the same space cannot: V^dag H^2 V
// = T^2 + e_K^2 u u^T (u the last unit vector) is positive, and its smallest
// eigenvalue bounds min |lambda|^2 from above.
namespace {
// number of eigenvalues below x of the symmetric tridiagonal (d, e) (Sturm)
int sturm_count(const std::vector<double>& d, const std::vector<double>& e, double x) {
    int cnt = 0;
    double q = 1.0;
    for (size_t i = 0; i < d.size(); ++i) {
        const double off = i ? e[i - 1] * e[i - 1] : 0.0;
        q = d[i] - x - (i ? off / q : 0.0);
        if (q == 0.0) q = -1e-300;
        if (q < 0.0) ++cnt;
    }
    return cnt;
}
// number of eigenvalues below x of the symmetric pentadiagonal matrix with
// diagonal a0, first and second superdiagonals a1, a2: negative pivots of
// the banded LDL^T of M - x I (Sylvester's law of inertia)
int penta_count(const std::vector<double>& a0, const std::vector<double>& a1,
                const std::vector<double>& a2, double x) {
    const size_t m = a0.size();
    int cnt = 0;
    double D1 = 0, D2 = 0;    // D_{i-1}, D_{i-2}
    double l1m = 0, l2m = 0;  // L_{i,i-1}, L_{i+1,i-1} (from row i-1's column)
    double l2mm = 0;          // L_{i,i-2}
    for (size_t i = 0; i < m; ++i) {
        double D = a0[i] - x - l1m * l1m * D1 - l2mm * l2mm * D2;
        if (D == 0.0) D = -1e-300;
        if (D < 0.0) ++cnt;
        // column i of L: L_{i+1,i} and L_{i+2,i}
        const double ai1 = i + 1 < m ? a1[i] : 0.0;
        const double ai2 = i + 2 < m ? a2[i] : 0.0;
        const double n1 = (ai1 - l2m * l1m * D1) / D;
        const double n2 = ai2 / D;
        l2mm = l2m;  // L_{i+1,i-1} becomes row i+1's L_{.,i-1}
        D2 = D1;
        D1 = D;
        l1m = n1;
        l2m = n2;
    }
    return cnt;
}
template <typename F>
double bisect(F count, int k, double lo, double hi) {  // the k-th (0-based) eigenvalue
    for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(1.0, std::fabs(lo) + std::fabs(hi));
         ++it) {
        const double mid = 0.5 * (lo + hi);
        if (count(mid) > k) hi = mid;
        else lo = mid;
    }
    return 0.5 * (lo + hi);
}
}  // namespace

extern "C" int ovl_spectral_bounds(ovl_ctx* ctx, int32_t src, double* bounds) {
    if (!ctx || !bounds) return OVL_E_ARG;
    if (src < 0 || (size_t)src >= ctx->last_iters.size())
        return fail(ctx, OVL_E_STATE, "no seed history for rhs %d (apply first)", src);
    const int K = ctx->last_iters[src];
    if (K < 2) return fail(ctx, OVL_E_STATE, "the last solve ran fewer than 2 iterations");
    DeviceGuard dg(ctx->device);
    std::vector<double2> h((size_t)K * 3);
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    HIPCHK(ctx, hipMemcpy(h.data(), ctx->seed.as<double2>() + (size_t)src * (ctx->last_maxk + 1) * 3,
                          h.size() * sizeof(double2), hipMemcpyDeviceToHost));
    const int m = K;
    std::vector<double> d(m), e(m);  // e[m-1]: coupling to the next (unbuilt) vector
    const double2 zs = ctx->zseed;
    for (int k = 0; k < m; ++k) {
        const double2 a = h[3 * k];
        const double aa = a.x * a.x + a.y * a.y;
        double2 dk = make_double2(a.x / aa, -a.y / aa);  // 1/alpha_k
        if (k > 0) {
            const double2 ap = h[3 * (k - 1)], bp = h[3 * (k - 1) + 1];
            const double apa = ap.x * ap.x + ap.y * ap.y;
            dk.x += (bp.x * ap.x + bp.y * ap.y) / apa;  // + beta_{k-1} / alpha_{k-1}
            dk.y += (bp.y * ap.x - bp.x * ap.y) / apa;
        }
        d[k] = zs.x - dk.x;
        e[k] = std::sqrt(h[3 * k + 2].y / h[3 * k + 2].x) / std::sqrt(aa);
    }
    std::vector<double> et(e.begin(), e.end() - 1);
    double lo = 1e300, hi = -1e300, emax = 0.0;
    for (int k = 0; k < m; ++k) {
        const double r = (k ? e[k - 1] : 0.0) + (k + 1 < m ? e[k] : 0.0);
        lo = std::min(lo, d[k] - r);
        hi = std::max(hi, d[k] + r);
        emax = std::max(emax, e[k]);
    }
    bounds[0] = bisect([&](double x) { return sturm_count(d, et, x); }, 0, lo, hi);
    bounds[1] = bisect([&](double x) { return sturm_count(d, et, x); }, m - 1, lo, hi);
    // M = T^2 + e_{m-1}^2 u u^T
    std::vector<double> a0(m), a1(m, 0.0), a2(m, 0.0);
    for (int i = 0; i < m; ++i) {
        a0[i] = d[i] * d[i] + (i ? e[i - 1] * e[i - 1] : 0.0) + e[i] * e[i];
        if (i + 1 < m) a1[i] = e[i] * (d[i] + d[i + 1]);
        if (i + 2 < m) a2[i] = e[i] * e[i + 1];
    }
    const double mhi = std::pow(std::max(std::fabs(lo), std::fabs(hi)) + 2.0 * emax, 2);
    const double mu = bisect([&](double x) { return penta_count(a0, a1, a2, x); }, 0, 0.0, mhi);
    bounds[2] = std::sqrt(std::max(mu, 0.0));
    return OVL_OK;
}

extern "C" int ovl_suggest_contour(double gap, double lmax, double target, int32_t* nq,
                                   double* gamma, double* rho) {
    if (!nq || !gamma || !rho) return OVL_E_ARG;
    if (!(gap > 0.0) || !(lmax > gap) || !(target > 0.0 && target < 1.0)) return OVL_E_ARG;
    // circle (alpha = 1) from a hair above 0 to 5% beyond lmax.  On a circle the
    // Gamma_+ filter is F(lam) = 1 / (1 + ((lam - gamma)/rho)^N), and the
    // two-contour error at |lam| is 1 - F(|lam|) + F(-|lam|); it is largest at
    // the ends |lam| = gap and |lam| = lmax, so take the smallest even N that
    // brings both under target
    const double eps = 1e-4 * gap;
    const double right = 1.05 * lmax;
    *rho = 0.5 * (right - eps);
    *gamma = eps + *rho;
    auto err = [&](double lam, int N) {
        const double a = std::pow(std::fabs((lam - *gamma) / *rho), N);
        const double b = std::pow((lam + *gamma) / *rho, N);
        return a / (1.0 + a) + 1.0 / (1.0 + b);
    };
    int n = 2;
    while (2 * n <= kMaxShifts && (err(gap, n) >= target || err(lmax, n) >= target)) n += 2;
    if (2 * n > kMaxShifts) return OVL_E_ARG;
    *nq = n;
    return OVL_OK;
}

static int apply_common(ovl_ctx* ctx, const void* in, void* out, int nrhs, ovl_stats* st,
                        bool dov) {
    if (!ctx) return OVL_E_ARG;
    DeviceGuard dg(ctx->device);
    int rc = check_apply_args(ctx, in, out, nrhs, true);
    if (rc) return rc;
    Work w;
    rc = prepare(ctx, nrhs, w);
    if (rc) return rc;
    launch_pack_spinor64(static_cast<const double2*>(in), w.b64, ctx->g.V, ctx->g.Vt, nrhs, ctx->stream);
    HIPCHK(ctx, hipGetLastError());
    rc = solve(ctx, w);
    if (rc < 0) return rc;
    const int rcc = true_residuals(ctx, w);
    if (rcc < 0) return rcc;
    if (dov)
        launch_unpack_dov(w.s64, static_cast<const double2*>(in), static_cast<double2*>(out),
                          0.5 * (1.0 + ctx->mq), 0.5 * (1.0 - ctx->mq), ctx->g.V, ctx->g.Vt, nrhs,
                          ctx->stream);
    else
        launch_unpack_spinor64(w.s64, static_cast<double2*>(out), ctx->g.V, ctx->g.Vt, nrhs, ctx->stream);
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (st) *st = ctx->last;
    return rc;
}

extern "C" int ovl_apply_sign(ovl_ctx* ctx, const void* in, void* out, int32_t nrhs,
                              ovl_stats* st) {
    return apply_common(ctx, in, out, nrhs, st, false);
}

extern "C" int ovl_apply_dov(ovl_ctx* ctx, const void* in, void* out, int32_t nrhs,
                             ovl_stats* st) {
    return apply_common(ctx, in, out, nrhs, st, true);
}

// Y[j] = sum_{i < K} u_i^j r_i for shifts [j0, j0+jn) of source n of the last
// basis solve, K being that source's iteration count
static int materialize(ovl_ctx* ctx, const Work& w, int j0, int jn, double2* Y, int n = 0,
                       int K = -1) {
    if (K < 0) K = w.K;
    const int ksw = w.k_switch < 0 ? K + 1 : w.k_switch;
    const double2* Wn = w.W + (size_t)n * (w.maxk + 1) * w.J;
    // on the caller's stream, after the solve's handoff; the slot table on the
    // device lists every chunk of this solve
    launch_materialize(w.slot_tab, w.slot_bytes, K, ksw, Wn, w.J, j0, jn, Y, w.N,
                       (int64_t)n * w.N, ctx->stream);
    HIPCHK(ctx, hipGetLastError());
    return OVL_OK;
}

extern "C" int ovl_force(ovl_ctx* ctx, const void* phi, void* grad, int32_t kind,
                         int32_t shift_chunk, double* action, ovl_stats* st) {
    if (!ctx) return OVL_E_ARG;
    DeviceGuard dg(ctx->device);
    if (kind != 0 && kind != 1 && kind != 2)
        return fail(ctx, OVL_E_ARG, "kind must be 0 (force), 1 (gradient) or 2 (action only)");
    if (!ctx->gauge_set || !ctx->masses_set || ctx->z.empty())
        return fail(ctx, OVL_E_STATE, "gauge, masses and nodes must be set before ovl_force");
    int rc = check_dev_ptr(ctx, phi, "phi");
    if (rc) return rc;
    if (kind != 2) {
        rc = check_dev_ptr(ctx, grad, "grad");
        if (rc) return rc;
        if (overlaps(phi, (size_t)12 * ctx->g.V * sizeof(double2), grad,
                     (size_t)36 * ctx->g.V * sizeof(double2)))
            return fail(ctx, OVL_E_ARG, "grad aliases phi");
    }
    const int saved_form = ctx->form;
    const std::vector<double2> z0 = ctx->z, c0 = ctx->c;
    const int J = (int)z0.size();
    const int64_t N = n12(ctx);
    const int C = (shift_chunk <= 0 || shift_chunk > J) ? J : shift_chunk;
    hipStream_t s = ctx->stream;
    bool swapped = false;
    // the first solve's basis, table and coefficients live in the force's
    // buffers while the second solve runs; afterwards the sets swap back
    auto swap_basis = [&]() {
        std::swap(ctx->slot_chunks, ctx->fslot_chunks);
        std::swap(ctx->slot_table, ctx->fslot_table);
        std::swap(ctx->W, ctx->fW);
        swapped = !swapped;
    };
    auto restore = [&]() {
        if (swapped) swap_basis();
        ctx->form = saved_form;
        ctx->z = z0;
        ctx->c = c0;
    };
    // 1. one basis-form solve for phi: s = sum c_j Y_j, with Y_j = (z_j - H)^-1 phi
    //    kept implicit in the stored basis and coefficients
    ctx->form = OVL_FORM_BASIS;
    Work w;
    rc = prepare(ctx, 1, w);
    if (rc) { restore(); return rc; }
    launch_pack_spinor64(static_cast<const double2*>(phi), w.b64, ctx->g.V, ctx->g.Vt, 1, s);
    const int rc1 = solve(ctx, w);
    if (rc1 < 0) { restore(); return rc1; }
    const ovl_stats st1 = ctx->last;
    if (ctx->fpsi.ensure((size_t)N * sizeof(double2)) != hipSuccess ||
        ctx->fpart.ensure(512 * sizeof(double)) != hipSuccess ||
        (kind != 2 && (ctx->fY.ensure((size_t)C * N * sizeof(double2)) != hipSuccess ||
                       ctx->fX.ensure((size_t)C * N * sizeof(double2)) != hipSuccess ||
                       ctx->facc.ensure((size_t)4 * ctx->g.V * 18 * sizeof(double2)) != hipSuccess ||
                       ctx->fc.ensure((size_t)J * sizeof(double2)) != hipSuccess))) {
        restore();
        return fail(ctx, OVL_E_OOM, "force work space allocation failed");
    }
    if (kind != 2)
        HIPCHK(ctx, hipMemcpyAsync(ctx->fc.p, w.cj, J * sizeof(double2), hipMemcpyDeviceToDevice, s));
    // 2. D_ov phi, psi = (1-mq)/2 gamma5 D_ov phi and S = |D_ov phi|^2
    const int npart = 256;
    launch_dov_psi(w.b64, w.s64, ctx->fpsi.as<double2>(), 0.5 * (1.0 + ctx->mq),
                   0.5 * (1.0 - ctx->mq), ctx->g.Vt, ctx->fpart.as<double>(), npart, s);
    std::vector<double> part(npart);
    HIPCHK(ctx, hipMemcpyAsync(part.data(), ctx->fpart.p, npart * sizeof(double),
                               hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    double S = 0.0;
    for (double v : part) S += v;
    if (kind == 2) {
        restore();
        ctx->last = st1;
        if (action) *action = S;
        if (st) *st = st1;
        return rc1 == OVL_NOT_CONVERGED ? OVL_NOT_CONVERGED : OVL_OK;
    }
    // 3. X_j = (conj(z_j) - H)^-1 psi from a second basis-form solve at the
    //    conjugate nodes, into a basis of its own
    swap_basis();
    for (int j = 0; j < J; ++j) ctx->z[j].y = -z0[j].y;
    Work w2;
    rc = prepare(ctx, 1, w2);
    if (rc) { restore(); return rc; }
    HIPCHK(ctx, hipMemcpyAsync(w2.b64, ctx->fpsi.p, N * sizeof(double2), hipMemcpyDeviceToDevice, s));
    const int rc2 = solve(ctx, w2);
    if (rc2 < 0) { restore(); return rc2; }
    const ovl_stats st2 = ctx->last;
    // 4. per link: sum_j c_j X_j^dag dH Y_j, C shifts at a time; Y_j and X_j of
    //    the chunk are rebuilt from their bases, so at most C of each exist
    for (int j0 = 0; j0 < J; j0 += C) {
        const int jn = std::min(C, J - j0);
        rc = materialize(ctx, w, j0, jn, ctx->fY.as<double2>());
        if (rc) { restore(); return rc; }
        rc = materialize(ctx, w2, j0, jn, ctx->fX.as<double2>());
        if (rc) { restore(); return rc; }
        launch_force(ctx->fX.as<double2>(), ctx->fY.as<double2>(), ctx->fc.as<double2>() + j0, jn,
                     ctx->g, ctx->U64.as<double2>(), ctx->bc, kappa_of(ctx->m0),
                     ctx->facc.as<double2>(), j0 == 0, j0 + jn >= J, kind,
                     static_cast<double2*>(grad), s);
        HIPCHK(ctx, hipGetLastError());
    }
    HIPCHK(ctx, hipStreamSynchronize(s));
    restore();
    ovl_stats& L = ctx->last;
    L = st1;
    L.iterations = std::max(st1.iterations, st2.iterations);
    L.fp32_iterations = std::max(st1.fp32_iterations, st2.fp32_iterations);
    L.n_active_end = st1.n_active_end + st2.n_active_end;
    L.max_est_rel_res = std::max(st1.max_est_rel_res, st2.max_est_rel_res);
    L.seconds = st1.seconds + st2.seconds;
    L.max_true_rel_res = std::max(st1.max_true_rel_res, st2.max_true_rel_res);
    L.fp64_repeat = st1.fp64_repeat | st2.fp64_repeat;
    L.mixed_true_rel_res = std::max(st1.mixed_true_rel_res, st2.mixed_true_rel_res);
    if (action) *action = S;
    if (st) *st = L;
    return (rc1 == OVL_NOT_CONVERGED || rc2 == OVL_NOT_CONVERGED) ? OVL_NOT_CONVERGED : OVL_OK;
}

extern "C" int ovl_apply_sign_batched(ovl_ctx* const* ctxs, int32_t nctx, const void* const* in,
                                      void* const* out, const int32_t* nrhs, ovl_stats* st) {
    if (!ctxs || nctx < 1 || nctx > kMaxJobs || !ctxs[0] || !in || !out || !nrhs) return OVL_E_ARG;
    ovl_ctx* lead = ctxs[0];
    DeviceGuard dg(lead->device);
    for (int i = 0; i < nctx; ++i) {
        if (!ctxs[i]) return fail(lead, OVL_E_ARG, "context %d is NULL", i);
        if (ctxs[i]->device != lead->device)
            return fail(lead, OVL_E_ARG, "context %d is on device %d, not %d", i, ctxs[i]->device,
                        lead->device);
        for (int k = 0; k < i; ++k)
            if (ctxs[k] == ctxs[i]) return fail(lead, OVL_E_ARG, "context %d appears twice", i);
    }
    if (lead->z.empty()) return fail(lead, OVL_E_STATE, "ovl_set_contour / ovl_set_nodes was not called");
    // every job takes the lead's nodes and solver settings for this call
    struct Saved {
        std::vector<double2> z, c;
        int precision, form, maxiter;
        double tol, switch_res;
        double2 zseed;
    };
    std::vector<Saved> saved(nctx);
    for (int i = 0; i < nctx; ++i) {
        ovl_ctx* c = ctxs[i];
        saved[i] = {c->z, c->c, c->precision, c->form, c->maxiter, c->tol, c->switch_res, c->zseed};
        c->z = lead->z;
        c->c = lead->c;
        c->precision = lead->precision;
        c->form = lead->form;
        c->maxiter = lead->maxiter;
        c->tol = lead->tol;
        c->switch_res = lead->switch_res;
        c->zseed = lead->zseed;
    }
    auto restore = [&]() {
        for (int i = 0; i < nctx; ++i) {
            ovl_ctx* c = ctxs[i];
            c->z = saved[i].z;
            c->c = saved[i].c;
            c->precision = saved[i].precision;
            c->form = saved[i].form;
            c->maxiter = saved[i].maxiter;
            c->tol = saved[i].tol;
            c->switch_res = saved[i].switch_res;
            c->zseed = saved[i].zseed;
        }
    };
    std::vector<Work> works(nctx);
    Batch B;
    int rc = OVL_OK;
    for (int i = 0; i < nctx && rc == OVL_OK; ++i) {
        rc = check_apply_args(ctxs[i], in[i], out[i], nrhs[i], true);
        if (rc == OVL_OK) rc = prepare(ctxs[i], nrhs[i], works[i]);
        if (rc != OVL_OK && ctxs[i] != lead) {
            fail(lead, rc, "context %d: %s", i, ctxs[i]->err);
        }
        B.ctx.push_back(ctxs[i]);
        B.w.push_back(&works[i]);
    }
    if (rc != OVL_OK) { restore(); return rc; }
    for (int i = 0; i < nctx; ++i)
        launch_pack_spinor64(static_cast<const double2*>(in[i]), works[i].b64, ctxs[i]->g.V, ctxs[i]->g.Vt, nrhs[i],
                             lead->stream);
    if (hipGetLastError() != hipSuccess) { restore(); return fail(lead, OVL_E_HIP, "pack failed"); }
    rc = solve_batch(B);
    if (rc >= 0) {
        for (int i = 0; i < nctx; ++i)
            launch_unpack_spinor64(works[i].s64, static_cast<double2*>(out[i]), ctxs[i]->g.V, ctxs[i]->g.Vt, nrhs[i],
                                   lead->stream);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(lead->stream) != hipSuccess)
            rc = fail(lead, OVL_E_HIP, "unpack failed");
    }
    restore();
    if (st) {
        ovl_stats a{};
        a.stencil_variant64 = lead->last.stencil_variant64;
        a.stencil_variant32 = lead->last.stencil_variant32;
        a.seconds = lead->last.seconds;
        for (int i = 0; i < nctx; ++i) {
            const ovl_stats& L = ctxs[i]->last;
            a.iterations = std::max(a.iterations, L.iterations);
            a.fp32_iterations = std::max(a.fp32_iterations, L.fp32_iterations);
            a.n_shifts = L.n_shifts;
            a.n_active_end += L.n_active_end;
            a.max_est_rel_res = std::max(a.max_est_rel_res, L.max_est_rel_res);
        }
        *st = a;
    }
    return rc;
}

// ============================================================================
// kernel timing
// ============================================================================
extern "C" int ovl_bench_kernel(ovl_ctx* ctx, int32_t which, int32_t nrhs, int32_t reps,
                                double* avg_ms, double* bytes) {
    if (!ctx || !avg_ms || !bytes) return OVL_E_ARG;
    // which 0/1: FP64/FP32 stencil with the autotuned choice; 100+c / 200+c: FP64/FP32
    // choice c = variant + kStencilVariants * (two-row links)
    const int nfmt = ctx->links12 ? 2 : 1;
    const bool explicit_v = (which >= 100 && which < 100 + kStencilVariants * nfmt) ||
                            (which >= 200 && which < 200 + kStencilVariants * nfmt);
    if (nrhs < 1 || reps < 1 || !(which == 0 || which == 1 || explicit_v))
        return fail(ctx, OVL_E_ARG, "bad bench arguments");
    if (!ctx->gauge_set || !ctx->masses_set) return fail(ctx, OVL_E_STATE, "gauge/masses not set");
    DeviceGuard dg(ctx->device);
    const int64_t N = n12(ctx);
    const bool f32 = which == 1 || which >= 200;
    const size_t es = f32 ? sizeof(float2) : sizeof(double2);
    const size_t nb = (size_t)nrhs * N * es;
    const int code = explicit_v ? which % 100 : stencil_variant(ctx, nrhs, f32 ? 1 : 0, 0);
    const int var = code % kStencilVariants, lnk = code / kStencilVariants;
    HIPCHK(ctx, ctx->bench_a.ensure(nb));
    HIPCHK(ctx, ctx->bench_b.ensure(nb));
    HIPCHK(ctx, hipMemsetAsync(ctx->bench_a.p, 0, nb, ctx->stream));
    auto launch = [&]() {
        if (f32)
            launch_wilson<float>(0, ctx->bench_a.as<float2>(), ctx->bench_b.as<float2>(),
                                 stencil_links<float>(ctx, lnk), ctx->g, kappa_of(ctx->m0),
                                 make_double2(0, 0), nullptr, nullptr, nullptr, nullptr, 0, nrhs,
                                 ctx->stream, var, lnk);
        else
            launch_wilson<double>(0, ctx->bench_a.as<double2>(), ctx->bench_b.as<double2>(),
                                  stencil_links<double>(ctx, lnk), ctx->g, kappa_of(ctx->m0),
                                  make_double2(0, 0), nullptr, nullptr, nullptr, nullptr, 0, nrhs,
                                  ctx->stream, var, lnk);
    };
    launch();
    HIPCHK(ctx, hipGetLastError());
    hipEvent_t e0, e1;
    HIPCHK(ctx, hipEventCreate(&e0));
    HIPCHK(ctx, hipEventCreate(&e1));
    HIPCHK(ctx, hipEventRecord(e0, ctx->stream));
    for (int i = 0; i < reps; ++i) launch();
    HIPCHK(ctx, hipEventRecord(e1, ctx->stream));
    HIPCHK(ctx, hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(ctx, hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *avg_ms = ms / reps;
    // algorithmic bytes: links once (36 complex per site), each spinor read once and
    // written once (12 complex per site per rhs)
    *bytes = (double)ctx->g.V * ((lnk ? 24.0 : 36.0) * es + 2.0 * 12.0 * es * nrhs);
    return OVL_OK;
}
