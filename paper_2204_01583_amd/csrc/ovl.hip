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

namespace {

// A device allocation that only grows.
struct DBuf {
    void* p = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t nb) {
        if (nb <= bytes) return hipSuccess;
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        hipError_t e = hipMalloc(&p, nb);
        if (e == hipSuccess) bytes = nb;
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
    // solver settings
    int precision = OVL_PREC_FP64;
    int form = OVL_FORM_FUSED;
    double tol = 1e-12;
    int maxiter = 4000;
    double2 zseed = make_double2(1.0, 0.05);
    double switch_res = 1e-4;
    int poll = 8;  // iterations between convergence polls
    // device buffers
    DBuf U64, U32;
    DBuf hw_in, hw_out;
    DBuf b64, r64, p64, q64, r32, p32, q32, s64, pj64, pj32, xj;
    std::vector<DBuf> slot_chunks;   // basis forms: kSlotChunk residual slots each
    size_t slot_chunk_bytes = 0;
    DBuf part_w, part_e, state, shifts, lists, nodes_dev, hist, W, h;
    SrcState* host_state = nullptr;  // pinned mirror
    int host_state_n = 0;
    DBuf bench_a, bench_b;
    DBuf fY, fX, fpsi, facc, fc, fpart;  // force work space
    // per-kernel-class event timing (ovl_set_profiling)
    static constexpr int kClasses = 8;
    bool prof_on = false;
    std::vector<hipEvent_t> ev_pool;
    struct ProfRec { int cls; int ev; double bytes; };
    std::vector<ProfRec> prof_pending;
    double prof_ms[kClasses] = {0};
    int64_t prof_n[kClasses] = {0};
    double prof_bytes[kClasses] = {0};
    // stencil variant chosen per (nrhs, precision) by the autotuner
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

int64_t n12(const ovl_ctx* ctx) { return 12 * ctx->g.V; }

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

// Brackets one launch of class `cls` with two events (profiling only).
struct ProfScope {
    ovl_ctx* ctx;
    int idx = -1;
    ProfScope(ovl_ctx* c, int cls, double bytes) : ctx(c) {
        if (!ctx->prof_on) return;
        const size_t need = 2 * (ctx->prof_pending.size() + 1);
        while (ctx->ev_pool.size() < need) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return;
            ctx->ev_pool.push_back(e);
        }
        idx = (int)ctx->prof_pending.size();
        ctx->prof_pending.push_back({cls, 2 * idx, bytes});
        (void)hipEventRecord(ctx->ev_pool[2 * idx], ctx->stream);
    }
    ~ProfScope() {
        if (idx >= 0) (void)hipEventRecord(ctx->ev_pool[2 * idx + 1], ctx->stream);
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
    }
    ctx->g.V = V;
    *out = ctx;
    return OVL_OK;
}

extern "C" int ovl_destroy(ovl_ctx* ctx) {
    if (!ctx) return OVL_OK;
    DeviceGuard dg(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    DBuf* bufs[] = {&ctx->U64,  &ctx->U32,   &ctx->hw_in,  &ctx->hw_out, &ctx->b64,   &ctx->r64,
                    &ctx->p64,  &ctx->q64,   &ctx->r32,    &ctx->p32,    &ctx->q32,   &ctx->s64,
                    &ctx->pj64, &ctx->pj32,  &ctx->xj,     &ctx->part_w, &ctx->part_e,
                    &ctx->state, &ctx->shifts, &ctx->lists, &ctx->nodes_dev, &ctx->hist, &ctx->W,
                    &ctx->h,    &ctx->bench_a, &ctx->bench_b, &ctx->fY, &ctx->fX, &ctx->fpsi,
                    &ctx->facc, &ctx->fc, &ctx->fpart};
    for (DBuf* b : bufs) b->release();
    for (DBuf& b : ctx->slot_chunks) b.release();
    for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    if (ctx->host_state) (void)hipHostFree(ctx->host_state);
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
    const size_t nl = (size_t)36 * ctx->g.V;
    HIPCHK(ctx, ctx->U64.ensure(nl * sizeof(double2)));
    HIPCHK(ctx, ctx->U32.ensure(nl * sizeof(float2)));
    launch_pack_gauge(static_cast<const double2*>(U), ctx->U64.as<double2>(),
                      ctx->U32.as<float2>(), ctx->g, ctx->bc, ctx->stream);
    HIPCHK(ctx, hipGetLastError());
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
    return OVL_OK;
}

extern "C" int ovl_set_solver(ovl_ctx* ctx, int32_t precision, int32_t form, double tol,
                              int32_t maxiter, double zr, double zi, double switch_res) {
    if (!ctx) return OVL_E_ARG;
    if (precision != OVL_PREC_FP64 && precision != OVL_PREC_MIXED)
        return fail(ctx, OVL_E_ARG, "unknown precision %d", precision);
    if (form < OVL_FORM_REFERENCE || form > OVL_FORM_BASIS)
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

std::string tune_key(const ovl_ctx* ctx, int nrhs, int prec) {
    hipDeviceProp_t prop;
    const char* arch = "gpu";
    if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) arch = prop.gcnArchName;
    int rt = 0;
    (void)hipRuntimeGetVersion(&rt);
    char buf[256];
    snprintf(buf, sizeof(buf), "%s|hip%d|%dx%dx%dx%d|n%d|%s", arch, rt, ctx->g.L[0], ctx->g.L[1],
             ctx->g.L[2], ctx->g.L[3], nrhs, prec ? "fp32" : "fp64");
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

template <typename R>
double time_variant(ovl_ctx* ctx, int v, int nrhs, C2<R>* a, C2<R>* b, const C2<R>* U) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return 1e30;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return 1e30;
    }
    auto run = [&]() {
        launch_wilson<R>(0, a, b, U, ctx->g, kappa_of(ctx->m0), make_double2(0, 0), nullptr, nullptr,
                         nullptr, nullptr, 0, nrhs, ctx->stream, v);
    };
    run();
    const int reps = 4;
    float best = 1e30f;
    for (int trial = 0; trial < 3; ++trial) {  // best of 3 trials damps timing noise
        (void)hipEventRecord(e0, ctx->stream);
        for (int i = 0; i < reps; ++i) run();
        (void)hipEventRecord(e1, ctx->stream);
        float ms = 1e30f;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            ms = 1e30f;
        best = std::min(best, ms);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return best / reps;
}

}  // namespace

// Variant of the stencil for nrhs right-hand sides in precision prec (0 FP64, 1 FP32).
static int stencil_variant(ovl_ctx* ctx, int nrhs, int prec) {
    const char* force = getenv("OVL_STENCIL_VARIANT");
    if (force && *force) {
        const int v = atoi(force);
        if (v >= 0 && v < kStencilVariants) return v;
    }
    const auto key = std::make_pair(nrhs, prec);
    auto it = ctx->stencil_variant.find(key);
    if (it != ctx->stencil_variant.end()) return it->second;
    const char* at = getenv("OVL_AUTOTUNE");
    if (at && at[0] == '0') return ctx->stencil_variant[key] = 0;
    const char* path = getenv("OVL_AUTOTUNE_CACHE");
    const std::string k = tune_key(ctx, nrhs, prec);
    if (path && *path) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto m = read_cache(path);
        auto f = m.find(k);
        if (f != m.end() && f->second >= 0 && f->second < kStencilVariants)
            return ctx->stencil_variant[key] = f->second;
    }
    const size_t es = prec ? sizeof(float2) : sizeof(double2);
    const size_t nb = (size_t)nrhs * n12(ctx) * es;
    int best = 0;
    if (ctx->bench_a.ensure(nb) == hipSuccess && ctx->bench_b.ensure(nb) == hipSuccess &&
        hipMemsetAsync(ctx->bench_a.p, 0, nb, ctx->stream) == hipSuccess) {
        double tbest = 1e30;
        for (int v = 0; v < kStencilVariants; ++v) {
            const double t = prec ? time_variant<float>(ctx, v, nrhs, ctx->bench_a.as<float2>(),
                                                        ctx->bench_b.as<float2>(), ctx->U32.as<float2>())
                                  : time_variant<double>(ctx, v, nrhs, ctx->bench_a.as<double2>(),
                                                         ctx->bench_b.as<double2>(), ctx->U64.as<double2>());
            if (t < tbest) {
                tbest = t;
                best = v;
            }
        }
    }
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
    const size_t bytes = (size_t)nrhs * n12(ctx) * sizeof(double2);
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
    launch_pack_spinor64(static_cast<const double2*>(in), ctx->hw_in.as<double2>(), ctx->g.V,
                         nrhs, ctx->stream);
    const int var = stencil_variant(ctx, nrhs, 0);
    launch_wilson<double>(0, ctx->hw_in.as<double2>(), ctx->hw_out.as<double2>(),
                          ctx->U64.as<double2>(), ctx->g, kappa_of(ctx->m0), make_double2(0, 0),
                          nullptr, nullptr, nullptr, nullptr, 0, nrhs, ctx->stream, var);
    launch_unpack_spinor64(ctx->hw_out.as<double2>(), static_cast<double2*>(out), ctx->g.V, nrhs,
                           ctx->stream);
    HIPCHK(ctx, hipGetLastError());
    return OVL_OK;
}

// ============================================================================
// shifted solver
// ============================================================================
namespace {

constexpr int kSlotChunk = 32;  // residual slots per basis allocation

struct Work {
    int nsrc, J, maxk;
    int64_t N;  // 12 V
    double2 *b64, *r64, *p64, *q64, *s64, *pj64, *xj;
    float2 *r32, *p32, *q32, *pj32;
    std::vector<char*> chunks;  // basis: slot i at chunks[i / kSlotChunk] + (i % kSlotChunk) * slot_bytes
    size_t slot_bytes;          // nsrc * N * sizeof(double2)
    double2* part_w;
    double* part_e;
    int nbw, nbe;          // partials per source of K1 and of the vector kernels
    SrcState* st;          // device state block: st | cnt | mres (one copy to the host)
    size_t state_bytes;
    ShiftDev sh;
    int var64, var32;      // stencil variants (autotuned)
    int k_switch;          // first FP32 iteration (mixed), or -1
    int K;                 // seed iterations of the last solve (max over sources)
    double2 *dz, *cj;
    double2 *h_a, *h_b, *h_pi, *W, *h;
};

// layout of the state block shared by the device and its pinned host mirror
size_t state_cnt_off(int nsrc) { return ((size_t)nsrc * sizeof(SrcState) + 255) & ~(size_t)255; }
size_t state_mres_off(int nsrc) {
    return (state_cnt_off(nsrc) + (size_t)2 * nsrc * kMaxSlices * sizeof(int) + 255) & ~(size_t)255;
}
size_t state_bytes_for(int nsrc) { return state_mres_off(nsrc) + (size_t)nsrc * kMaxSlices * sizeof(double); }

int prepare(ovl_ctx* ctx, int nsrc, Work& w) {
    const int J = (int)ctx->z.size();
    const int64_t N = n12(ctx);
    const bool mixed = ctx->precision == OVL_PREC_MIXED;
    const int form = ctx->form;
    w.nsrc = nsrc;
    w.J = J;
    w.N = N;
    w.maxk = ctx->maxiter;
    const size_t vec64 = (size_t)nsrc * N * sizeof(double2);
    const size_t vec32 = (size_t)nsrc * N * sizeof(float2);
    HIPCHK(ctx, ctx->b64.ensure(vec64));
    HIPCHK(ctx, ctx->r64.ensure(vec64));
    HIPCHK(ctx, ctx->p64.ensure(vec64));
    HIPCHK(ctx, ctx->q64.ensure(vec64));
    HIPCHK(ctx, ctx->s64.ensure(vec64));
    w.b64 = ctx->b64.as<double2>();
    w.r64 = ctx->r64.as<double2>();
    w.p64 = ctx->p64.as<double2>();
    w.q64 = ctx->q64.as<double2>();
    w.s64 = ctx->s64.as<double2>();
    w.r32 = w.p32 = w.q32 = w.pj32 = nullptr;
    w.pj64 = w.xj = nullptr;
    w.chunks.clear();
    w.slot_bytes = vec64;
    if (mixed) {
        HIPCHK(ctx, ctx->r32.ensure(vec32));
        HIPCHK(ctx, ctx->p32.ensure(vec32));
        HIPCHK(ctx, ctx->q32.ensure(vec32));
        w.r32 = ctx->r32.as<float2>();
        w.p32 = ctx->p32.as<float2>();
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
    if (basis && ctx->slot_chunk_bytes != vec64 * kSlotChunk) {
        // slot geometry changed: drop the old chunks
        for (DBuf& b : ctx->slot_chunks) b.release();
        ctx->slot_chunks.clear();
        ctx->slot_chunk_bytes = vec64 * kSlotChunk;
    }
    const int nslices = (J + 255) / 256;
    w.nbw = wilson_blocks(ctx->g);
    w.nbe = vec_blocks(N, nslices);
    HIPCHK(ctx, ctx->part_w.ensure((size_t)nsrc * w.nbw * sizeof(double2)));
    HIPCHK(ctx, ctx->part_e.ensure((size_t)nsrc * w.nbe * sizeof(double)));
    w.state_bytes = state_bytes_for(nsrc);
    HIPCHK(ctx, ctx->state.ensure(w.state_bytes));
    w.part_w = ctx->part_w.as<double2>();
    w.part_e = ctx->part_e.as<double>();
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
    HIPCHK(ctx, ctx->nodes_dev.ensure((size_t)2 * J * sizeof(double2)));
    w.dz = ctx->nodes_dev.as<double2>();
    w.cj = w.dz + J;
    sh.dz = w.dz;
    sh.c = w.cj;
    std::vector<double2> tab(2 * J);
    for (int j = 0; j < J; ++j) {
        tab[j] = make_double2(ctx->z[j].x - ctx->zseed.x, ctx->z[j].y - ctx->zseed.y);
        tab[J + j] = ctx->c[j];
    }
    HIPCHK(ctx, hipMemcpyAsync(w.dz, tab.data(), tab.size() * sizeof(double2),
                               hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));  // tab is pageable and goes out of scope
    w.h_a = w.h_b = w.h_pi = w.W = w.h = nullptr;
    if (basis) {
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
    if ((size_t)ctx->host_state_n < w.state_bytes) {
        if (ctx->host_state) (void)hipHostFree(ctx->host_state);
        ctx->host_state = nullptr;
        ctx->host_state_n = 0;
        HIPCHK(ctx, hipHostMalloc((void**)&ctx->host_state, w.state_bytes, hipHostMallocDefault));
        ctx->host_state_n = (int)w.state_bytes;
    }
    return OVL_OK;
}

template <typename R> R* slot_ptr(const Work& w, int i) {
    return reinterpret_cast<R*>(w.chunks[i / kSlotChunk] + (size_t)(i % kSlotChunk) * w.slot_bytes);
}

// make sure residual slots 0 .. upto exist
int ensure_slots(ovl_ctx* ctx, Work& w, int upto) {
    const int need = upto / kSlotChunk + 1;
    while ((int)ctx->slot_chunks.size() < need) {
        ctx->slot_chunks.emplace_back();
        HIPCHK(ctx, ctx->slot_chunks.back().ensure(ctx->slot_chunk_bytes));
    }
    w.chunks.clear();
    for (DBuf& b : ctx->slot_chunks) w.chunks.push_back(b.as<char>());
    return OVL_OK;
}

// One seed iteration k in precision R (double before the switch, float after):
// K1 stencil + <r,q>, K2 r update, K3 p update or shift sweep.
template <typename R>
void enqueue_iteration(ovl_ctx* ctx, const Work& w, int k, int form, hipStream_t s, C2<R>* r,
                       C2<R>* p, C2<R>* q, C2<R>* pj, const C2<R>* U, int nact_total) {
    const int64_t N = w.N;
    const bool basis = form == OVL_FORM_BASIS;
    const double es = sizeof(C2<R>);
    const int c32 = sizeof(R) == 4 ? 1 : 0;
    const double V = (double)ctx->g.V;
    // r_k: working vector, or basis slot k (FP32 slots are packed at the slot base)
    C2<R>* rk = basis ? slot_ptr<C2<R>>(w, k) : r;
    C2<R>* rk1 = basis ? slot_ptr<C2<R>>(w, k + 1) : r;
    {   // links once, p read, q written, r read for <r,q>
        ProfScope ps(ctx, 0 + c32, V * es * (36.0 + 36.0 * w.nsrc));
        launch_wilson<R>(1, p, q, U, ctx->g, kappa_of(ctx->m0), ctx->zseed, rk, w.part_w, w.st,
                         &w.sh, k, w.nsrc, s, c32 ? w.var32 : w.var64);
    }
    {
        ProfScope ps(ctx, 2 + c32, 3.0 * es * N * w.nsrc);
        launch_update_r<R>(rk, rk1, q, w.st, w.part_w, w.nbw, w.part_e, w.nbe, N, w.sh, k, s);
    }
    if (basis) {
        ProfScope ps(ctx, 2 + c32, 3.0 * es * N * w.nsrc);
        launch_update_p<R>(rk1, p, w.st, w.part_e, w.nbe, N, w.sh, k, s);
    } else {
        // r read, p read+write, s read+write (FP64) per source; p_j read+write
        // (and x_j read+write in FP64 for the reference form) per active shift
        const bool ref = form == OVL_FORM_REFERENCE;
        const double b = (double)N * (w.nsrc * (3.0 * es + (ref ? 0.0 : 32.0)) +
                                      nact_total * (2.0 * es + (ref ? 32.0 : 0.0)));
        ProfScope ps(ctx, 4 + c32, b);
        launch_sweep<R>(ref, r, p, pj, ref ? w.xj : w.s64, w.b64, w.st, w.part_e, w.nbe, N, w.sh,
                        k, s);
    }
}

}  // namespace

// Runs the shifted solver on nsrc sources packed in w.b64 and leaves
// s = sum_j c_j y_j in w.s64.  Returns a status; fills ctx->last.
static int solve(ovl_ctx* ctx, Work& w) {
    hipStream_t s = ctx->stream;
    const int form = ctx->form;
    const bool mixed = ctx->precision == OVL_PREC_MIXED;
    const int64_t N = w.N;
    const size_t vec64 = (size_t)w.nsrc * N * sizeof(double2);
    w.var64 = stencil_variant(ctx, w.nsrc, 0);
    w.var32 = mixed ? stencil_variant(ctx, w.nsrc, 1) : 0;
    hipEvent_t e0, e1;
    HIPCHK(ctx, hipEventCreate(&e0));
    HIPCHK(ctx, hipEventCreate(&e1));
    HIPCHK(ctx, hipEventRecord(e0, s));
    // r = p = b, s = 0 (fused), x_j = 0 (reference), slot 0 = b (basis)
    if (form == OVL_FORM_BASIS) {
        int rc = ensure_slots(ctx, w, std::min(w.maxk, ctx->poll) + 1);
        if (rc) return rc;
    }
    if (form == OVL_FORM_BASIS)
        HIPCHK(ctx, hipMemcpyAsync(slot_ptr<double2>(w, 0), w.b64, vec64,
                                   hipMemcpyDeviceToDevice, s));
    else
        HIPCHK(ctx, hipMemcpyAsync(w.r64, w.b64, vec64, hipMemcpyDeviceToDevice, s));
    HIPCHK(ctx, hipMemcpyAsync(w.p64, w.b64, vec64, hipMemcpyDeviceToDevice, s));
    if (form == OVL_FORM_FUSED) HIPCHK(ctx, hipMemsetAsync(w.s64, 0, vec64, s));
    if (form == OVL_FORM_REFERENCE) HIPCHK(ctx, hipMemsetAsync(w.xj, 0, vec64 * w.J, s));
    launch_init_state(w.st, w.b64, w.part_e, N, w.sh, s);
    HIPCHK(ctx, hipGetLastError());

    bool low = false;  // FP32 phase active
    int k_switch = -1;
    int k = 0;
    bool all_done = false;
    int status = OVL_OK;
    double maxres = 1.0;
    int iters = 0, nact = 0;
    int nact_known = w.J * w.nsrc;  // active shifts at the last poll (profiling bytes)
    while (k < w.maxk) {
        const int chunk = std::min(ctx->poll, w.maxk - k);
        if (form == OVL_FORM_BASIS) {
            int rc = ensure_slots(ctx, w, k + chunk + 1);
            if (rc) return rc;
        }
        for (int i = 0; i < chunk; ++i, ++k) {
            if (!low)
                enqueue_iteration<double>(ctx, w, k, form, s, w.r64, w.p64, w.q64, w.pj64,
                                          ctx->U64.as<double2>(), nact_known);
            else
                enqueue_iteration<float>(ctx, w, k, form, s, w.r32, w.p32, w.q32, w.pj32,
                                         ctx->U32.as<float2>(), nact_known);
        }
        HIPCHK(ctx, hipGetLastError());
        HIPCHK(ctx, hipMemcpyAsync(ctx->host_state, w.st, w.state_bytes, hipMemcpyDeviceToHost, s));
        HIPCHK(ctx, hipStreamSynchronize(s));
        prof_collect(ctx);
        all_done = true;
        maxres = 0.0;
        iters = 0;
        nact = 0;
        const char* hb = reinterpret_cast<const char*>(ctx->host_state);
        const int* hcnt = reinterpret_cast<const int*>(hb + state_cnt_off(w.nsrc)) +
                          (size_t)(k & 1) * w.nsrc * kMaxSlices;
        const double* hmres = reinterpret_cast<const double*>(hb + state_mres_off(w.nsrc));
        for (int n = 0; n < w.nsrc; ++n) {
            const SrcState& S = ctx->host_state[n];
            if (S.status != OVL_OK && status == OVL_OK) status = S.status;
            int na = 0;
            for (int i = 0; i < w.sh.nslices; ++i) {
                na += hcnt[n * kMaxSlices + i];
                maxres = std::max(maxres, hmres[n * kMaxSlices + i]);
            }
            all_done = all_done && (na == 0 || S.status != OVL_OK);
            iters = std::max(iters, S.iter);
            nact += na;
        }
        nact_known = nact;
        if (status != OVL_OK || all_done) break;
        if (mixed && !low && maxres < ctx->switch_res && k < w.maxk) {
            // relaxed precision: from here the remaining corrections are small
            // enough that FP32 vectors perturb the result by ~eps32 * switch_res
            low = true;
            k_switch = k;
            launch_convert_64_to_32(w.p64, w.p32, (int64_t)w.nsrc * N, s);
            if (form == OVL_FORM_BASIS) {
                launch_convert_64_to_32(slot_ptr<double2>(w, k), w.r32, (int64_t)w.nsrc * N, s);
                HIPCHK(ctx, hipMemcpyAsync(slot_ptr<float2>(w, k), w.r32,
                                           (size_t)w.nsrc * N * sizeof(float2),
                                           hipMemcpyDeviceToDevice, s));
            } else {
                launch_convert_64_to_32(w.r64, w.r32, (int64_t)w.nsrc * N, s);
                launch_convert_64_to_32(w.pj64, w.pj32, (int64_t)w.nsrc * N * w.J, s);
            }
            HIPCHK(ctx, hipGetLastError());
        }
    }
    w.k_switch = k_switch;
    w.K = iters;
    if (status == OVL_OK && !all_done) status = OVL_NOT_CONVERGED;
    if (status == OVL_OK || status == OVL_NOT_CONVERGED) {
        if (form == OVL_FORM_REFERENCE) {
            launch_sum_ref(w.xj, w.cj, w.s64, w.J, N, w.nsrc, s);
        } else if (form == OVL_FORM_BASIS) {
            launch_basis_coef(w.h_a, w.h_b, w.h_pi, w.cj, w.st, w.W, w.h, w.J, w.maxk, w.nsrc, s);
            // s = sum_i h_i r_i, chunk by chunk; FP64 slots below k_switch, FP32 from it
            const int kend = iters + 1;
            const int ksw = k_switch < 0 ? kend : k_switch;
            bool acc = false;
            for (int c0 = 0; c0 < kend; c0 += kSlotChunk) {
                const int c1 = std::min(kend, c0 + kSlotChunk);
                char* base = w.chunks[c0 / kSlotChunk];
                const int a0 = c0, a1 = std::min(c1, ksw);
                if (a1 > a0) {
                    ProfScope ps(ctx, 6, (double)N * w.nsrc * (16.0 * (a1 - a0) + 32.0));
                    launch_basis_gemv<double>(base, (int64_t)w.nsrc * N, N, w.h, w.maxk, w.st, c0,
                                              a0 - c0, a1 - c0, w.s64, acc, N, w.nsrc, s);
                    acc = true;
                }
                const int f0 = std::max(c0, ksw), f1 = c1;
                if (f1 > f0) {
                    ProfScope ps(ctx, 6, (double)N * w.nsrc * (8.0 * (f1 - f0) + 32.0));
                    launch_basis_gemv<float>(base, (int64_t)w.nsrc * N * 2, N, w.h, w.maxk, w.st,
                                             c0, f0 - c0, f1 - c0, w.s64, acc, N, w.nsrc, s);
                    acc = true;
                }
            }
        }
        HIPCHK(ctx, hipGetLastError());
    }
    HIPCHK(ctx, hipEventRecord(e1, s));
    HIPCHK(ctx, hipEventSynchronize(e1));
    prof_collect(ctx);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ovl_stats& L = ctx->last;
    std::memset(&L, 0, sizeof(L));
    L.iterations = iters;
    L.fp32_iterations = k_switch < 0 ? 0 : std::max(0, iters - k_switch);
    L.n_shifts = w.J;
    L.n_active_end = nact;
    L.max_est_rel_res = maxres;
    L.seconds = ms * 1e-3;
    L.stencil_variant64 = w.var64;
    L.stencil_variant32 = mixed ? w.var32 : -1;
    if (status < 0) fail(ctx, status, "solver stopped: %s", ovl_status_string(status));
    if (status == OVL_NOT_CONVERGED)
        fail(ctx, status, "maxiter=%d reached with %d shifts above tol (max est. res %.3e)",
             w.maxk, nact, maxres);
    return status;
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
    launch_pack_spinor64(static_cast<const double2*>(in), w.b64, ctx->g.V, nrhs, ctx->stream);
    HIPCHK(ctx, hipGetLastError());
    rc = solve(ctx, w);
    if (rc < 0) return rc;
    if (dov)
        launch_unpack_dov(w.s64, static_cast<const double2*>(in), static_cast<double2*>(out),
                          0.5 * (1.0 + ctx->mq), 0.5 * (1.0 - ctx->mq), ctx->g.V, nrhs,
                          ctx->stream);
    else
        launch_unpack_spinor64(w.s64, static_cast<double2*>(out), ctx->g.V, nrhs, ctx->stream);
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

// Y[j] = sum_i u_i^j r_i for shifts [j0, j0+jn) of the last basis solve (one source)
static int materialize(ovl_ctx* ctx, const Work& w, int j0, int jn, double2* Y) {
    const int K = w.K;
    const int ksw = w.k_switch < 0 ? K + 1 : w.k_switch;
    bool acc = false;
    for (int c0 = 0; c0 < K; c0 += kSlotChunk) {
        launch_materialize(w.chunks[c0 / kSlotChunk], w.slot_bytes, c0, kSlotChunk, ksw, w.W, w.J,
                           j0, jn, K, Y, w.N, acc, ctx->stream);
        acc = true;
    }
    if (!acc) HIPCHK(ctx, hipMemsetAsync(Y, 0, (size_t)jn * w.N * sizeof(double2), ctx->stream));
    HIPCHK(ctx, hipGetLastError());
    return OVL_OK;
}

extern "C" int ovl_force(ovl_ctx* ctx, const void* phi, void* grad, int32_t kind,
                         int32_t shift_chunk, double* action, ovl_stats* st) {
    if (!ctx) return OVL_E_ARG;
    DeviceGuard dg(ctx->device);
    if (kind != 0 && kind != 1) return fail(ctx, OVL_E_ARG, "kind must be 0 (force) or 1 (gradient)");
    if (!ctx->gauge_set || !ctx->masses_set || ctx->z.empty())
        return fail(ctx, OVL_E_STATE, "gauge, masses and nodes must be set before ovl_force");
    int rc = check_dev_ptr(ctx, phi, "phi");
    if (rc) return rc;
    rc = check_dev_ptr(ctx, grad, "grad");
    if (rc) return rc;
    if (overlaps(phi, (size_t)12 * ctx->g.V * sizeof(double2), grad,
                 (size_t)36 * ctx->g.V * sizeof(double2)))
        return fail(ctx, OVL_E_ARG, "grad aliases phi");
    const int saved_form = ctx->form;
    const std::vector<double2> z0 = ctx->z, c0 = ctx->c;
    const int J = (int)z0.size();
    const int64_t N = n12(ctx);
    const int C = (shift_chunk <= 0 || shift_chunk > J) ? J : shift_chunk;
    hipStream_t s = ctx->stream;
    auto restore = [&]() {
        ctx->form = saved_form;
        ctx->z = z0;
        ctx->c = c0;
    };
    // 1. Y_j = (z_j - H)^-1 phi and s = sum c_j Y_j from one basis-form solve
    ctx->form = OVL_FORM_BASIS;
    Work w;
    rc = prepare(ctx, 1, w);
    if (rc) { restore(); return rc; }
    launch_pack_spinor64(static_cast<const double2*>(phi), w.b64, ctx->g.V, 1, s);
    const int rc1 = solve(ctx, w);
    if (rc1 < 0) { restore(); return rc1; }
    const ovl_stats st1 = ctx->last;
    if (ctx->fY.ensure((size_t)J * N * sizeof(double2)) != hipSuccess ||
        ctx->fpsi.ensure((size_t)N * sizeof(double2)) != hipSuccess ||
        ctx->fX.ensure((size_t)C * N * sizeof(double2)) != hipSuccess ||
        ctx->facc.ensure((size_t)4 * ctx->g.V * 18 * sizeof(double2)) != hipSuccess ||
        ctx->fc.ensure((size_t)J * sizeof(double2)) != hipSuccess ||
        ctx->fpart.ensure(512 * sizeof(double)) != hipSuccess) {
        restore();
        return fail(ctx, OVL_E_OOM, "force work space allocation failed");
    }
    rc = materialize(ctx, w, 0, J, ctx->fY.as<double2>());
    if (rc) { restore(); return rc; }
    HIPCHK(ctx, hipMemcpyAsync(ctx->fc.p, w.cj, J * sizeof(double2), hipMemcpyDeviceToDevice, s));
    // 2. D_ov phi, psi = (1-mq)/2 gamma5 D_ov phi and S = |D_ov phi|^2
    const int npart = 256;
    launch_dov_psi(w.b64, w.s64, ctx->fpsi.as<double2>(), 0.5 * (1.0 + ctx->mq),
                   0.5 * (1.0 - ctx->mq), ctx->g.V, ctx->fpart.as<double>(), npart, s);
    std::vector<double> part(npart);
    HIPCHK(ctx, hipMemcpyAsync(part.data(), ctx->fpart.p, npart * sizeof(double),
                               hipMemcpyDeviceToHost, s));
    // 3. X_j = (conj(z_j) - H)^-1 psi from a second basis-form solve at the conjugate nodes
    for (int j = 0; j < J; ++j) ctx->z[j].y = -z0[j].y;
    Work w2;
    rc = prepare(ctx, 1, w2);  // synchronises the stream (so part[] is ready)
    if (rc) { restore(); return rc; }
    double S = 0.0;
    for (double v : part) S += v;
    HIPCHK(ctx, hipMemcpyAsync(w2.b64, ctx->fpsi.p, N * sizeof(double2), hipMemcpyDeviceToDevice, s));
    const int rc2 = solve(ctx, w2);
    if (rc2 < 0) { restore(); return rc2; }
    const ovl_stats st2 = ctx->last;
    // 4. per link: sum_j c_j X_j^dag dH Y_j, C shifts at a time
    for (int j0 = 0; j0 < J; j0 += C) {
        const int jn = std::min(C, J - j0);
        rc = materialize(ctx, w2, j0, jn, ctx->fX.as<double2>());
        if (rc) { restore(); return rc; }
        launch_force(ctx->fX.as<double2>(), ctx->fY.as<double2>() + (size_t)j0 * N,
                     ctx->fc.as<double2>() + j0, jn, ctx->g, ctx->U64.as<double2>(), ctx->bc,
                     kappa_of(ctx->m0), ctx->facc.as<double2>(), j0 == 0, j0 + jn >= J, kind,
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
    L.reserved[0] = st2.iterations;
    if (action) *action = S;
    if (st) *st = L;
    return (rc1 == OVL_NOT_CONVERGED || rc2 == OVL_NOT_CONVERGED) ? OVL_NOT_CONVERGED : OVL_OK;
}

extern "C" int ovl_apply_sign_batched(ovl_ctx* const* ctxs, int32_t nctx, const void* const*,
                                      void* const*, const int32_t*, ovl_stats*) {
    if (!ctxs || nctx < 1 || !ctxs[0]) return OVL_E_ARG;
    return fail(ctxs[0], OVL_E_STATE, "ovl_apply_sign_batched is not available in this build");
}

// ============================================================================
// kernel timing
// ============================================================================
extern "C" int ovl_bench_kernel(ovl_ctx* ctx, int32_t which, int32_t nrhs, int32_t reps,
                                double* avg_ms, double* bytes) {
    if (!ctx || !avg_ms || !bytes) return OVL_E_ARG;
    // which 0/1: FP64/FP32 stencil with the autotuned variant; 100+v / 200+v: FP64/FP32 variant v
    const bool explicit_v = (which >= 100 && which < 100 + kStencilVariants) ||
                            (which >= 200 && which < 200 + kStencilVariants);
    if (nrhs < 1 || reps < 1 || !(which == 0 || which == 1 || explicit_v))
        return fail(ctx, OVL_E_ARG, "bad bench arguments");
    if (!ctx->gauge_set || !ctx->masses_set) return fail(ctx, OVL_E_STATE, "gauge/masses not set");
    DeviceGuard dg(ctx->device);
    const int64_t N = n12(ctx);
    const bool f32 = which == 1 || which >= 200;
    const size_t es = f32 ? sizeof(float2) : sizeof(double2);
    const size_t nb = (size_t)nrhs * N * es;
    const int var = explicit_v ? which % 100 : stencil_variant(ctx, nrhs, f32 ? 1 : 0);
    HIPCHK(ctx, ctx->bench_a.ensure(nb));
    HIPCHK(ctx, ctx->bench_b.ensure(nb));
    HIPCHK(ctx, hipMemsetAsync(ctx->bench_a.p, 0, nb, ctx->stream));
    auto launch = [&]() {
        if (f32)
            launch_wilson<float>(0, ctx->bench_a.as<float2>(), ctx->bench_b.as<float2>(),
                                 ctx->U32.as<float2>(), ctx->g, kappa_of(ctx->m0),
                                 make_double2(0, 0), nullptr, nullptr, nullptr, nullptr, 0, nrhs, ctx->stream, var);
        else
            launch_wilson<double>(0, ctx->bench_a.as<double2>(), ctx->bench_b.as<double2>(),
                                  ctx->U64.as<double2>(), ctx->g, kappa_of(ctx->m0),
                                  make_double2(0, 0), nullptr, nullptr, nullptr, nullptr, 0, nrhs, ctx->stream, var);
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
    *bytes = (double)ctx->g.V * (36.0 * es + 2.0 * 12.0 * es * nrhs);
    return OVL_OK;
}
