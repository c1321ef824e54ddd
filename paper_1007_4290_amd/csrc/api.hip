// C-ABI of the sweeping preconditioner library: argument validation,
// context and device-memory management, the layer loop of the
// factorization (Alg. 2.3), the sweep (Alg. 2.4) and the flexible GMRES
// driver in FP64 (Sec. 2.4).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>
#include <algorithm>
#include <complex>
#include <string>
#include <vector>

#include <mutex>

#include "hsweep.h"
#include "internal.hpp"

// Device scratch of hsweep_apply_noalloc: the sweep's forward work vectors
// w_m (nrhs * n * n_p entries of the factor precision).  One copy per GPU,
// held until the process ends.  In host code `scratch` only names the
// symbol; its device address is looked up once per device (scratch_init).
static __device__ __align__(256) unsigned char scratch[HSWEEP_NOALLOC_SCRATCH_BYTES];

size_t factor_lds_bytes(const Plan& p, size_t elem);
bool factor_supported(const Plan& p);

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIPCHK(expr)                                                                   \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(e_ == hipErrorOutOfMemory ? HSWEEP_ENOMEM : HSWEEP_EDEVICE,    \
                        std::string(#expr) + ": " + hipGetErrorString(e_));            \
    } while (0)

constexpr size_t kMaxLds = 152 * 1024;   // dynamic LDS budget: 160 KiB minus static shared variables
constexpr int kAutoGroupRhs = 1 << 30;   // automatic grouping: right-hand sides from which G = 4

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    hipError_t ensure(size_t b) {
        if (b <= bytes && p) return hipSuccess;
        release();
        hipError_t e = hipMalloc(&p, b);
        if (e == hipSuccess) bytes = b;
        else p = nullptr;
        return e;
    }
};

struct HostBuf {
    void* p = nullptr;
    size_t bytes = 0;
    void release() {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        bytes = 0;
    }
    hipError_t ensure(size_t b) {
        if (b <= bytes && p) return hipSuccess;
        release();
        hipError_t e = hipHostMalloc(&p, b, hipHostMallocDefault);
        if (e == hipSuccess) bytes = b;
        else p = nullptr;
        return e;
    }
};

}  // namespace

int hsweep_report(int code, const std::string& msg) { return fail(code, msg); }
void hsweep_clear_error() { g_err.clear(); }

struct hsweep_ctx {
    int n = 0, pml = 0;
    double omega = 0.0;
    int device = 0;
    hsweep_opts opts{};
    Plan plan{};
    bool planned = false;
    bool factored = false;
    // coefficients (FP64)
    DevBuf c, isn1, sh1, isn2, sh2;     // velocity; stretching tables of the x1 and x2 axes
    // factorization (precision-typed)
    DevBuf dg, eo, cp, fac, Q, G, rank, status;
    // sweep work
    DevBuf sweep_w;
    // Krylov work
    DevBuf V, Z, w, r, hdev, partial, scale, active, y;
    // conj(g) of an adjoint solve
    DevBuf adj;
    // system offsets of the Krylov vectors; batched solves: concatenated
    // right-hand sides and solutions, sweep instance and task tables
    DevBuf offd, bf, bu, sinst, stask;
    HostBuf offh;
    HostBuf hhost, scalehost, activehost, yhost;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    double t_factor = 0, t_sweep = 0, t_stencil = 0, t_krylov = 0, n_apply = 0;
    // the layer loop of a single-context factorization, captured once as a
    // HIP graph (kernel nodes only) and replayed while its descriptor holds
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    DevBuf gdesc;
    std::vector<unsigned char> gkey;
    // strongly admissible factors (admissibility HSWEEP_ADM_STRONG)
    StrongFactors* strong = nullptr;
    AxisTables tables() const {
        AxisTables t;
        t.isn1 = (const c128*)isn1.p; t.sh1 = (const c128*)sh1.p;
        t.isn2 = (const c128*)isn2.p; t.sh2 = (const c128*)sh2.p;
        t.abc = 0;
        for (int k = 0; k < 4; ++k)
            if (opts.pml_sides[k] == HSWEEP_SIDE_ABC) t.abc |= 1 << k;
        return t;
    }
    void drop_graph() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        gexec = nullptr;
        graph = nullptr;
        gkey.clear();
    }
    ~hsweep_ctx() {
        strong_free(strong);
        drop_graph();
        if (cap) (void)hipStreamDestroy(cap);
        gdesc.release();
        DevBuf* bufs[] = {&c, &isn1, &sh1, &isn2, &sh2, &dg, &eo, &cp, &fac, &Q, &G, &rank, &status, &sweep_w,
                          &V, &Z, &w, &r, &hdev, &partial, &scale, &active, &y, &adj,
                          &offd, &bf, &bu, &sinst, &stask};
        for (DevBuf* b : bufs) b->release();
        HostBuf* hb[] = {&hhost, &scalehost, &activehost, &yhost, &offh};
        for (HostBuf* b : hb) b->release();
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

namespace {

// Per-device address of `scratch`, filled by scratch_init on the first
// hsweep_setup with that device current.
constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

int scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return fail(HSWEEP_EDEVICE, "device index out of range for the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return HSWEEP_OK;
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        return fail(HSWEEP_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    g_scratch_ptr[device] = ptr;
    return HSWEEP_OK;
}

int ilog2(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// Width in grid points of the absorbing layer on side k (x1 low, x1 high,
// x2 low, x2 high): the option if set, otherwise the width of hsweep_setup.
int side_width(const hsweep_ctx* ctx, const hsweep_opts& o, int k) {
    if (o.pml_sides[k] == HSWEEP_SIDE_ABC) return 0;
    return o.pml_sides[k] >= 0 ? o.pml_sides[k] : ctx->pml;
}

// Stretching tables of both axes (Sec. 2.1, eq. sigma) for the options `o`.
int build_tables(hsweep_ctx* ctx, const hsweep_opts& o) {
    const int n = ctx->n;
    const double h = 1.0 / (n + 1);
    launch_pml_1d(n, ctx->omega, side_width(ctx, o, 0) * h, side_width(ctx, o, 1) * h, o.pml_C, (c128*)ctx->isn1.p,
                  (c128*)ctx->sh1.p, 0);
    launch_pml_1d(n, ctx->omega, side_width(ctx, o, 2) * h, side_width(ctx, o, 3) * h, o.pml_C, (c128*)ctx->isn2.p,
                  (c128*)ctx->sh2.p, 0);
    HIPCHK(hipGetLastError());
    HIPCHK(hipDeviceSynchronize());
    return HSWEEP_OK;
}

int validate_opts(const hsweep_opts* o, int n) {
    if (!o) return fail(HSWEEP_EINVAL, "opts is NULL");
    if (!(o->precision == HSWEEP_C128 || o->precision == HSWEEP_C64))
        return fail(HSWEEP_EINVAL, "precision must be HSWEEP_C128 or HSWEEP_C64");
    if (!o->dense) {
        if (!is_pow2(o->leaf) || o->leaf < 4 || o->leaf > 64)
            return fail(HSWEEP_EINVAL, "leaf must be a power of two in [4, 64]");
        if (!is_pow2(o->rank) || o->rank < 2 || o->rank > 16)
            return fail(HSWEEP_EINVAL, "rank must be a power of two in [2, 16]");
    }
    if (!(o->rank_tol >= 0.0) || !isfinite(o->rank_tol) || o->rank_tol >= 1.0)
        return fail(HSWEEP_EINVAL, "rank_tol must be in [0, 1)");
    if (!(o->pml_C > 0.0) || !isfinite(o->pml_C)) return fail(HSWEEP_EINVAL, "pml_C must be finite and > 0");
    if (o->restart < 1 || o->restart > 200) return fail(HSWEEP_EINVAL, "restart must be in [1, 200]");
    if (!(o->rhs_group == 0 || o->rhs_group == 1 || o->rhs_group == 4))
        return fail(HSWEEP_EINVAL, "rhs_group must be 0 (automatic), 1 or 4");
    if (o->direction < 0 || o->direction > 3) return fail(HSWEEP_EINVAL, "direction must be one of HSWEEP_DIR_*");
    if (o->direction == HSWEEP_DIR_MX1)
        return fail(HSWEEP_EINVAL, "the leftward column sweep (-x1) is switched off: its first GPU run ended in a "
                                   "memory fault whose cause is not found");
    for (int k = 0; k < 4; ++k)
        if (o->pml_sides[k] < -1 && o->pml_sides[k] != HSWEEP_SIDE_ABC)
            return fail(HSWEEP_EINVAL, "pml_sides entries must be -1, HSWEEP_SIDE_ABC or >= 0");
    if (o->admissibility != HSWEEP_ADM_WEAK && o->admissibility != HSWEEP_ADM_STRONG)
        return fail(HSWEEP_EINVAL, "admissibility must be HSWEEP_ADM_WEAK or HSWEEP_ADM_STRONG");
    if (o->admissibility == HSWEEP_ADM_STRONG && (o->precision != HSWEEP_C128 || o->dense))
        return fail(HSWEEP_EINVAL, "the strongly admissible format runs in complex128 with compressed factors");
    (void)n;
    return HSWEEP_OK;
}

// Build the plan of the layer H-matrix; EINVAL if the kernels cannot hold it.
int make_plan(hsweep_ctx* ctx, Plan& p) {
    const hsweep_opts& o = ctx->opts;
    p.n = ctx->n;
    if (o.admissibility == HSWEEP_ADM_STRONG) {
        // no padding and none of the weak format's kernel limits
        p.np = ctx->n; p.b = o.leaf; p.L = (int)strong_layer_depth(ctx->n, o.leaf); p.r = o.rank; p.tol = o.rank_tol;
        plan_sizes(p);
        return HSWEEP_OK;
    }
    if (o.dense) {
        int np = 1 << ilog2(ctx->n);
        if (np < 4) np = 4;
        p.np = np; p.b = np; p.L = 0; p.r = 2; p.tol = 0.0;
        if (np > 64) return fail(HSWEEP_EINVAL, "dense Schur complements are limited to n <= 64");
    } else {
        p.b = o.leaf;
        p.L = 0;
        while ((p.b << p.L) < ctx->n) ++p.L;
        p.np = p.b << p.L;
        p.r = o.rank;
        p.tol = o.rank_tol;
    }
    if (p.np > 1024) return fail(HSWEEP_EINVAL, "padded layer width above 1024 (n > 1024) is not supported");
    if (1 + p.r * p.L > 64)
        return fail(HSWEEP_EINVAL, "rank * levels too large for the in-block recompression (reduce rank or raise leaf)");
    plan_sizes(p);
    if (!factor_supported(p)) return fail(HSWEEP_EINVAL, "unsupported leaf size or rank");
    if (!sweep_supported(p))
        return fail(HSWEEP_EINVAL, "no compiled sweep for this (leaf, rank, levels) combination");
    size_t elem = o.precision == HSWEEP_C64 ? sizeof(c64) : sizeof(c128);
    if (factor_lds_bytes(p, elem) > kMaxLds)
        return fail(HSWEEP_EINVAL, "layer too wide for this precision (LDS of the factorization kernels)");
    if (sweep_lds_bytes(p, elem, 1) > kMaxLds) return fail(HSWEEP_EINVAL, "layer too wide for the sweep kernel");
    return HSWEEP_OK;
}

// Allocate the factorization buffers of one context, build its layer
// coefficients (Sec. 2.1) and describe it for the factorization kernels.
template <typename T>
int prepare_factor(hsweep_ctx* ctx, hipStream_t s, InstDesc<T>& d) {
    const Plan& p = ctx->plan;
    const int n = p.n, np = p.np;
    const size_t E = sizeof(cpx<T>);
    HIPCHK(ctx->dg.ensure((size_t)n * np * E));
    HIPCHK(ctx->eo.ensure((size_t)n * np * E));
    HIPCHK(ctx->cp.ensure((size_t)(n > 1 ? n : 2) * np * E));
    HIPCHK(ctx->fac.ensure((size_t)n * p.eLayer * E));
    HIPCHK(ctx->Q.ensure((size_t)(p.L > 0 ? p.L : 1) * p.r * np * E));
    HIPCHK(ctx->G.ensure((size_t)(2 << p.L) * p.r * p.r * E));
    HIPCHK(ctx->rank.ensure((size_t)n * (1 << p.L) * sizeof(int)));
    HIPCHK(ctx->status.ensure(sizeof(int)));
    HIPCHK(hipMemsetAsync(ctx->status.p, 0, sizeof(int), s));
    HIPCHK(hipMemsetAsync(ctx->cp.p, 0, (size_t)(n > 1 ? n : 2) * np * E, s));
    launch_layer_coeffs<T>(n, np, ctx->opts.direction, ctx->omega, (const double*)ctx->c.p, ctx->tables(),
                           (cpx<T>*)ctx->dg.p, (cpx<T>*)ctx->eo.p, (cpx<T>*)ctx->cp.p, s);
    HIPCHK(hipGetLastError());
    d.p = p;
    d.fac = (cpx<T>*)ctx->fac.p;
    d.dg = (const cpx<T>*)ctx->dg.p;
    d.eo = (const cpx<T>*)ctx->eo.p;
    d.cp = (const cpx<T>*)ctx->cp.p;
    d.Q = (cpx<T>*)ctx->Q.p;
    d.G = (cpx<T>*)ctx->G.p;
    d.rank = (int*)ctx->rank.p;
    d.status = (int*)ctx->status.p;
    return HSWEEP_OK;
}

// Run the layer loop of Alg. 2.3 for `count` contexts of the same element
// type, leaf size and rank: layer step m of every context in one set of
// launches.  Synchronizes `s` and checks every context's pivot status.
template <typename T>
int do_factor_many(hsweep_ctx** ctxs, int count, hipStream_t s) {
    std::vector<InstDesc<T>> hd(count);
    std::vector<Plan> plans(count);
    int nmax = 0;
    for (int q = 0; q < count; ++q) {
        int rc = prepare_factor<T>(ctxs[q], s, hd[q]);
        if (rc) return rc;
        plans[q] = ctxs[q]->plan;
        nmax = std::max(nmax, plans[q].n);
    }
    DevBuf dd;
    HIPCHK(dd.ensure(count * sizeof(InstDesc<T>)));
    hipError_t e = hipMemcpyAsync(dd.p, hd.data(), count * sizeof(InstDesc<T>), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) { dd.release(); return fail(HSWEEP_EDEVICE, std::string("descriptor upload: ") + hipGetErrorString(e)); }
    int rc = HSWEEP_OK;
    for (int m = 0; m < nmax && rc == HSWEEP_OK; ++m)
        if (launch_factor_layer<T>((const InstDesc<T>*)dd.p, plans.data(), count, m, s) != 0)
            rc = fail(HSWEEP_EINVAL, "contexts of one batch need the same leaf size and rank");
    e = hipGetLastError();
    if (rc == HSWEEP_OK && e != hipSuccess) rc = fail(HSWEEP_EDEVICE, std::string("factor launch: ") + hipGetErrorString(e));
    e = hipStreamSynchronize(s);   // also keeps dd alive until the kernels are done
    dd.release();
    if (rc) return rc;
    if (e != hipSuccess) return fail(HSWEEP_EDEVICE, std::string("factor: ") + hipGetErrorString(e));
    for (int q = 0; q < count; ++q) {
        int st = 0;
        HIPCHK(hipMemcpy(&st, ctxs[q]->status.p, sizeof(int), hipMemcpyDeviceToHost));
        if (st) return fail(HSWEEP_ESINGULAR, "zero pivot in a leaf or core inverse");
    }
    return HSWEEP_OK;
}

// Single context: the coefficients are rebuilt on `s` (plain launches and
// memsets), then the layer loop runs as a HIP graph on `s`.  The graph holds
// kernel nodes only; it is captured on a private stream the first time and
// again whenever the descriptor (plan and buffers) changes.
template <typename T>
int do_factor_one(hsweep_ctx* ctx, hipStream_t s) {
    InstDesc<T> d;
    int rc = prepare_factor<T>(ctx, s, d);
    if (rc) return rc;
    const unsigned char* kb = reinterpret_cast<const unsigned char*>(&d);
    std::vector<unsigned char> key(kb, kb + sizeof(d));
    if (!ctx->gexec || key != ctx->gkey) {
        ctx->drop_graph();
        HIPCHK(ctx->gdesc.ensure(sizeof(d)));
        HIPCHK(hipMemcpy(ctx->gdesc.p, &d, sizeof(d), hipMemcpyHostToDevice));
        factor_kernels_init<T>();               // kernel attributes are set outside the capture
        if (!ctx->cap) HIPCHK(hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking));
        HIPCHK(hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeThreadLocal));
        const Plan plan = ctx->plan;
        bool ok = true;
        for (int m = 0; m < plan.n && ok; ++m)
            ok = launch_factor_layer<T>((const InstDesc<T>*)ctx->gdesc.p, &plan, 1, m, ctx->cap) == 0;
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(ctx->cap, &g);
        if (!ok || ec != hipSuccess || !g) {
            if (g) (void)hipGraphDestroy(g);
            (void)hipGetLastError();
            return fail(HSWEEP_EDEVICE, std::string("factor graph capture: ") + hipGetErrorString(ec));
        }
        ctx->graph = g;
        const hipError_t ei = hipGraphInstantiate(&ctx->gexec, g, nullptr, nullptr, 0);
        if (ei != hipSuccess) {
            ctx->drop_graph();
            return fail(HSWEEP_EDEVICE, std::string("factor graph instantiate: ") + hipGetErrorString(ei));
        }
        ctx->gkey = key;
    }
    HIPCHK(hipGraphLaunch(ctx->gexec, s));
    const hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(HSWEEP_EDEVICE, std::string("factor: ") + hipGetErrorString(e));
    int st = 0;
    HIPCHK(hipMemcpy(&st, ctx->status.p, sizeof(int), hipMemcpyDeviceToHost));
    if (st) return fail(HSWEEP_ESINGULAR, "zero pivot in a leaf or core inverse");
    return HSWEEP_OK;
}

// The factorization with HIP events around each kernel class, all layers
// queued before one synchronization (so no launch latency falls inside an
// interval): layer_ms sums the layer kernels (recompression and leaves),
// wood_ms the Woodbury kernels of every level.
template <typename T>
int do_factor_profile(hsweep_ctx* ctx, hipStream_t s, double* layer_ms, double* wood_ms) {
    InstDesc<T> d;
    int rc = prepare_factor<T>(ctx, s, d);
    if (rc) return rc;
    const Plan plan = ctx->plan;
    DevBuf dd;
    HIPCHK(dd.ensure(sizeof(d)));
    HIPCHK(hipMemcpyAsync(dd.p, &d, sizeof(d), hipMemcpyHostToDevice, s));
    factor_kernels_init<T>();
    std::vector<hipEvent_t> ev((size_t)3 * plan.n, nullptr);
    for (auto& e : ev) {
        if (hipEventCreate(&e) != hipSuccess) {
            for (auto& x : ev)
                if (x) (void)hipEventDestroy(x);
            dd.release();
            return fail(HSWEEP_EDEVICE, "event creation failed");
        }
    }
    for (int m = 0; m < plan.n && rc == HSWEEP_OK; ++m) {
        (void)hipEventRecord(ev[3 * m], s);
        if (launch_factor_layer<T>((const InstDesc<T>*)dd.p, &plan, 1, m, s, ev[3 * m + 1]) != 0)
            rc = fail(HSWEEP_EINVAL, "no factorization kernels for this plan");
        (void)hipEventRecord(ev[3 * m + 2], s);
    }
    const hipError_t e = hipStreamSynchronize(s);
    double tl = 0.0, tw = 0.0;
    if (rc == HSWEEP_OK && e == hipSuccess) {
        for (int m = 0; m < plan.n; ++m) {
            float a = 0.f, b = 0.f;
            (void)hipEventElapsedTime(&a, ev[3 * m], ev[3 * m + 1]);
            (void)hipEventElapsedTime(&b, ev[3 * m + 1], ev[3 * m + 2]);
            tl += a;
            tw += b;
        }
    }
    for (auto& x : ev) (void)hipEventDestroy(x);
    dd.release();
    if (rc) return rc;
    if (e != hipSuccess) return fail(HSWEEP_EDEVICE, std::string("factor: ") + hipGetErrorString(e));
    int st = 0;
    HIPCHK(hipMemcpy(&st, ctx->status.p, sizeof(int), hipMemcpyDeviceToHost));
    if (st) return fail(HSWEEP_ESINGULAR, "zero pivot in a leaf or core inverse");
    *layer_ms = tl;
    *wood_ms = tw;
    return HSWEEP_OK;
}

// Strongly admissible factors (complex128): the frame coefficients of every
// layer, then the layer loop of Alg. 2.3 in the strong format.
constexpr uint64_t kStrongSeed = 0x2545F4914F6CDD1Dull;

int do_factor_strong(hsweep_ctx* ctx, hipStream_t s) {
    const int n = ctx->n;
    const size_t E = sizeof(c128);
    strong_free(ctx->strong);
    ctx->strong = nullptr;
    HIPCHK(ctx->dg.ensure((size_t)n * n * E));
    HIPCHK(ctx->eo.ensure((size_t)n * n * E));
    HIPCHK(ctx->cp.ensure((size_t)(n > 1 ? n : 2) * n * E));
    HIPCHK(hipMemsetAsync(ctx->cp.p, 0, (size_t)(n > 1 ? n : 2) * n * E, s));
    launch_layer_coeffs<double>(n, n, ctx->opts.direction, ctx->omega, (const double*)ctx->c.p, ctx->tables(),
                                (c128*)ctx->dg.p, (c128*)ctx->eo.p, (c128*)ctx->cp.p, s);
    HIPCHK(hipGetLastError());
    std::string msg;
    const int rc = strong_factor(&ctx->strong, n, ctx->opts.leaf, ctx->opts.rank, ctx->opts.rank_tol, kStrongSeed,
                                 (const c128*)ctx->dg.p, (const c128*)ctx->eo.p, (const c128*)ctx->cp.p, s, &msg);
    if (rc) return fail(rc, msg);
    return HSWEEP_OK;
}

bool is_strong(const hsweep_ctx* ctx) { return ctx->opts.admissibility == HSWEEP_ADM_STRONG; }

// Right-hand sides per sweep workgroup: the option if set (4 only where a
// grouped kernel exists for the plan), otherwise 4 for many right-hand sides.
int sweep_group(const hsweep_ctx* ctx, int nrhs) {
    const int o = ctx->opts.rhs_group;
    const bool g4 = sweep_group_supported(ctx->plan);
    if (o == 1) return 1;
    if (o == 4) return g4 ? 4 : 1;
    return (g4 && nrhs >= kAutoGroupRhs) ? 4 : 1;
}

// Descriptor of this context's sweep over nrhs fields f -> u.
template <typename T>
SweepInst<T> sweep_inst(const hsweep_ctx* ctx, const c128* f, c128* u, void* work, const int* active, int nrhs) {
    const Plan& p = ctx->plan;
    SweepInst<T> in{};
    in.n = p.n; in.np = p.np; in.L = p.L; in.nrhs = nrhs;
    in.dir = ctx->opts.direction;
    in.eK = p.eK; in.eP = p.eP; in.eLayer = p.eLayer;
    in.fac = (const cpx<T>*)ctx->fac.p;
    in.cp = (const cpx<T>*)ctx->cp.p;
    in.f = f; in.u = u; in.w = (cpx<T>*)work;
    in.active = active;
    in.fstride = 0; in.ustride = 0;
    return in;
}

// The sweep's work vectors come from the context (allocated on demand) or,
// when `work` is given, from that buffer of at least nrhs * n * n_p entries.
template <typename T>
int do_apply(hsweep_ctx* ctx, const c128* f, c128* u, int nrhs, const int* active, hipStream_t s,
             void* work = nullptr) {
    const Plan& p = ctx->plan;
    if (!work) {
        HIPCHK(ctx->sweep_w.ensure((size_t)nrhs * p.n * p.np * sizeof(cpx<T>)));
        work = ctx->sweep_w.p;
    }
    SweepArgs<T> a{};
    a.one = sweep_inst<T>(ctx, f, u, work, active, nrhs);
    if (launch_sweep<T>(p, a, sweep_group(ctx, nrhs), s) != 0)
        return fail(HSWEEP_EINVAL, "no compiled sweep for this plan");
    HIPCHK(hipGetLastError());
    return HSWEEP_OK;
}

int apply_dispatch(hsweep_ctx* ctx, const c128* f, c128* u, int nrhs, const int* active, hipStream_t s) {
    if (is_strong(ctx)) {
        if (!ctx->strong) return fail(HSWEEP_ESTATE, "no strongly admissible factors");
        std::string msg;
        const int rc = strong_apply(ctx->strong, ctx->opts.direction, f, u, nrhs, active, s, &msg);
        return rc ? fail(rc, msg) : HSWEEP_OK;
    }
    if (ctx->opts.precision == HSWEEP_C64) return do_apply<float>(ctx, f, u, nrhs, active, s);
    return do_apply<double>(ctx, f, u, nrhs, active, s);
}

int check_ctx(const hsweep_ctx* ctx) {
    if (!ctx) return fail(HSWEEP_EINVAL, "context is NULL");
    return HSWEEP_OK;
}

int set_device(const hsweep_ctx* ctx) {
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return fail(HSWEEP_EDEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
    return HSWEEP_OK;
}

bool is_device_pointer(const void* ptr) {
    hipPointerAttribute_t attr;
    hipError_t e = hipPointerGetAttributes(&attr, ptr);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

// Givens rotation (c real, s complex) zeroing b in (a, b).
void givens(std::complex<double> a, std::complex<double> b, double& c, std::complex<double>& s) {
    if (b == 0.0) { c = 1.0; s = 0.0; return; }
    if (a == 0.0) { c = 0.0; s = std::conj(b) / std::abs(b); return; }
    double t = std::hypot(std::abs(a), std::abs(b));
    c = std::abs(a) / t;
    s = (a / std::abs(a)) * std::conj(b) / t;
}

// Host table of workgroup tasks for a multi-instance launch: group k of
// instance q (first right-hand side k*G) runs on XCD (running task index) % 8;
// table[slot * 8 + xcd] = (q << 16) | first right-hand side, -1 where idle.
std::vector<int> sweep_task_table(const int* nrhs, int ninst, int G) {
    std::vector<std::vector<int>> per(8);
    int t = 0;
    for (int q = 0; q < ninst; ++q)
        for (int r0 = 0; r0 < nrhs[q]; r0 += G, ++t) per[t % 8].push_back((q << 16) | r0);
    size_t slots = 0;
    for (auto& v : per) slots = v.size() > slots ? v.size() : slots;
    std::vector<int> table(8 * slots, -1);
    for (int x = 0; x < 8; ++x)
        for (size_t k = 0; k < per[x].size(); ++k) table[k * 8 + x] = per[x][k];
    return table;
}

// Flexible GMRES (right-preconditioned, FP64 Arnoldi with classical
// Gram-Schmidt applied twice, Givens rotations on the host) for the
// right-hand sides of `count` contexts: nr[q] fields of context q, f[q] ->
// u[q].  Every Krylov step is launched once for all of them: the vector
// kernels over the concatenation of all systems, the sweep as one launch per
// group of contexts with the same leaf size and rank (one launch for one
// context), the stencil once per context.  Each system stops on its own
// true residual ||f - A u|| <= tol ||f||.  The Krylov buffers live in
// ctxs[0] (its restart length is used).  Synchronizes `s`.
int solve_systems(hsweep_ctx** ctxs, int count, const int* nr, const c128* const* f_in, c128* const* u_out,
                  double tol, int maxit, int* iters, double* relres, hipStream_t s) {
    hsweep_ctx* c0 = ctxs[0];
    int rc = HSWEEP_OK;
    // systems and their offsets in the concatenated vectors
    std::vector<int> first(count + 1, 0);
    for (int q = 0; q < count; ++q) first[q + 1] = first[q] + nr[q];
    const int S = first[count];
    HIPCHK(c0->offh.ensure((size_t)(S + 1) * sizeof(size_t)));
    size_t* offh = (size_t*)c0->offh.p;
    size_t maxlen = 0;
    offh[0] = 0;
    for (int q = 0; q < count; ++q) {
        const size_t Nq = (size_t)ctxs[q]->n * ctxs[q]->n;
        maxlen = std::max(maxlen, Nq);
        for (int k = 0; k < nr[q]; ++k) offh[first[q] + k + 1] = offh[first[q] + k] + Nq;
    }
    const size_t Ntot = offh[S];
    const int m = c0->opts.restart;
    const int nblk = krylov_dot_blocks(maxlen);
    const int nvmax = m + 1;
    HIPCHK(c0->offd.ensure((size_t)(S + 1) * sizeof(size_t)));
    HIPCHK(c0->V.ensure((size_t)(m + 1) * Ntot * sizeof(c128)));
    HIPCHK(c0->Z.ensure((size_t)m * Ntot * sizeof(c128)));
    HIPCHK(c0->w.ensure(Ntot * sizeof(c128)));
    HIPCHK(c0->r.ensure(Ntot * sizeof(c128)));
    HIPCHK(c0->hdev.ensure((size_t)3 * nvmax * S * sizeof(c128)));
    HIPCHK(c0->partial.ensure((size_t)nblk * S * nvmax * sizeof(c128)));
    HIPCHK(c0->scale.ensure((size_t)S * sizeof(double)));
    HIPCHK(c0->active.ensure((size_t)S * sizeof(int)));
    HIPCHK(c0->y.ensure((size_t)m * S * sizeof(c128)));
    HIPCHK(c0->hhost.ensure((size_t)3 * nvmax * S * sizeof(c128)));
    HIPCHK(c0->scalehost.ensure((size_t)S * sizeof(double)));
    HIPCHK(c0->activehost.ensure((size_t)S * sizeof(int)));
    HIPCHK(c0->yhost.ensure((size_t)m * S * sizeof(c128)));
    HIPCHK(hipMemcpyAsync(c0->offd.p, offh, (size_t)(S + 1) * sizeof(size_t), hipMemcpyHostToDevice, s));
    const size_t* offd = (const size_t*)c0->offd.p;
    c128* V = (c128*)c0->V.p;
    c128* Z = (c128*)c0->Z.p;
    c128* w = (c128*)c0->w.p;
    c128* rr = (c128*)c0->r.p;
    c128* hd = (c128*)c0->hdev.p;
    c128* hd1 = hd;                          // first Gram-Schmidt pass
    c128* hd2 = hd + (size_t)nvmax * S;      // second pass
    c128* hd3 = hd2 + (size_t)nvmax * S;     // norms
    c128* part = (c128*)c0->partial.p;
    double* scd = (double*)c0->scale.p;
    int* actd = (int*)c0->active.p;
    c128* yd = (c128*)c0->y.p;
    std::complex<double>* hh = (std::complex<double>*)c0->hhost.p;
    double* sch = (double*)c0->scalehost.p;
    int* acth = (int*)c0->activehost.p;
    std::complex<double>* yh = (std::complex<double>*)c0->yhost.p;

    // right-hand sides and solutions: the caller's arrays for one context,
    // concatenated copies for several
    const c128* f = f_in[0];
    c128* u = u_out[0];
    if (count > 1) {
        HIPCHK(c0->bf.ensure(Ntot * sizeof(c128)));
        HIPCHK(c0->bu.ensure(Ntot * sizeof(c128)));
        for (int q = 0; q < count; ++q)
            HIPCHK(hipMemcpyAsync((c128*)c0->bf.p + offh[first[q]], f_in[q],
                                  (offh[first[q + 1]] - offh[first[q]]) * sizeof(c128), hipMemcpyDeviceToDevice, s));
        f = (const c128*)c0->bf.p;
        u = (c128*)c0->bu.p;
    }

    // sweep launches of a batch: one per (leaf, rank) group of contexts, with
    // device tables of instances (fields of column j at V + j Ntot -> Z + j Ntot)
    struct SweepGroup { std::vector<int> members; std::vector<Plan> plans; int G = 1, blocks = 0; size_t inst_off = 0, task_off = 0; };
    std::vector<SweepGroup> groups;
    const bool single_prec = c0->opts.precision == HSWEEP_C64;   // complex64 factors
    if (count > 1) {
        for (int q = 0; q < count; ++q) {
            const Plan& p = ctxs[q]->plan;
            const int rq = p.L > 0 ? p.r : 0;
            int gi = -1;
            for (size_t g = 0; g < groups.size(); ++g) {
                const Plan& p0 = ctxs[groups[g].members[0]]->plan;
                if (p0.b == p.b && (p0.L > 0 ? p0.r : 0) == rq) gi = (int)g;
            }
            if (gi < 0) { groups.emplace_back(); gi = (int)groups.size() - 1; }
            groups[gi].members.push_back(q);
            groups[gi].plans.push_back(p);
        }
        const size_t isz = single_prec ? sizeof(SweepInst<float>) : sizeof(SweepInst<double>);
        std::vector<unsigned char> itab;
        std::vector<int> ttab;
        for (auto& g : groups) {
            // the group's kernel: the largest level count of its members
            int lmax = 0, nrmax = 0;
            Plan pm = g.plans[0];
            std::vector<int> gnr;
            for (size_t k = 0; k < g.members.size(); ++k) {
                if (g.plans[k].L > lmax) { lmax = g.plans[k].L; pm = g.plans[k]; }
                nrmax = std::max(nrmax, nr[g.members[k]]);
                gnr.push_back(nr[g.members[k]]);
            }
            g.G = sweep_group(ctxs[g.members[0]], nrmax);
            if (g.G == 4 && !sweep_group_supported(pm)) g.G = 1;
            if (!(g.G == 1 ? sweep_supported(pm) : true)) return fail(HSWEEP_EINVAL, "no compiled sweep for a batch group");
            g.inst_off = itab.size();
            for (int q : g.members) {
                hsweep_ctx* cq = ctxs[q];
                const Plan& p = cq->plan;
                HIPCHK(cq->sweep_w.ensure((size_t)nr[q] * p.n * p.np * (single_prec ? sizeof(cpx<float>) : sizeof(cpx<double>))));
                const size_t o = offh[first[q]];
                if (single_prec) {
                    SweepInst<float> in = sweep_inst<float>(cq, V + o, Z + o, cq->sweep_w.p, actd + first[q], nr[q]);
                    in.fstride = Ntot; in.ustride = Ntot;
                    const unsigned char* b = (const unsigned char*)&in;
                    itab.insert(itab.end(), b, b + isz);
                } else {
                    SweepInst<double> in = sweep_inst<double>(cq, V + o, Z + o, cq->sweep_w.p, actd + first[q], nr[q]);
                    in.fstride = Ntot; in.ustride = Ntot;
                    const unsigned char* b = (const unsigned char*)&in;
                    itab.insert(itab.end(), b, b + isz);
                }
            }
            std::vector<int> t = sweep_task_table(gnr.data(), (int)gnr.size(), g.G);
            g.task_off = ttab.size();
            g.blocks = (int)t.size();
            ttab.insert(ttab.end(), t.begin(), t.end());
        }
        HIPCHK(c0->sinst.ensure(itab.size()));
        HIPCHK(c0->stask.ensure(ttab.size() * sizeof(int)));
        HIPCHK(hipMemcpy(c0->sinst.p, itab.data(), itab.size(), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(c0->stask.p, ttab.data(), ttab.size() * sizeof(int), hipMemcpyHostToDevice));
    }
    // u_j = M v_j for every active system: column j of V into column j of Z
    auto sweep_column = [&](int j) -> int {
        if (count == 1) return apply_dispatch(c0, V + (size_t)j * Ntot, Z + (size_t)j * Ntot, S, actd, s);
        for (auto& g : groups) {
            const int* tasks = (const int*)c0->stask.p + g.task_off;
            int e;
            if (single_prec)
                e = launch_sweep_multi_col<float>(g.plans.data(), (int)g.plans.size(),
                                                  (const SweepInst<float>*)((unsigned char*)c0->sinst.p + g.inst_off),
                                                  tasks, g.blocks, g.G, j, j, s);
            else
                e = launch_sweep_multi_col<double>(g.plans.data(), (int)g.plans.size(),
                                                   (const SweepInst<double>*)((unsigned char*)c0->sinst.p + g.inst_off),
                                                   tasks, g.blocks, g.G, j, j, s);
            if (e) return fail(HSWEEP_EINVAL, "no compiled sweep for a batch group");
        }
        HIPCHK(hipGetLastError());
        return HSWEEP_OK;
    };
    // y = A x (or y = f - A x) for every system, one launch per context
    auto stencil_all = [&](const c128* x, const c128* fv, c128* y, const int* act) {
        for (int q = 0; q < count; ++q) {
            hsweep_ctx* cq = ctxs[q];
            const size_t o = offh[first[q]];
            launch_stencil(cq->n, nr[q], cq->omega, (const double*)cq->c.p, cq->tables(), x + o, fv ? fv + o : nullptr,
                           y + o, act ? act + first[q] : nullptr, s);
        }
    };

    c0->t_sweep = c0->t_stencil = c0->t_krylov = 0.0;
    c0->n_apply = 0;
    auto sync = [&]() -> int {
        HIPCHK(hipStreamSynchronize(s));
        return HSWEEP_OK;
    };
    auto norms = [&](const c128* x, std::vector<double>& out) -> int {
        launch_multi_dot(x, 1, Ntot, x, offd, S, part, hd3, nblk, s);
        HIPCHK(hipMemcpyAsync(hh, hd3, (size_t)S * sizeof(c128), hipMemcpyDeviceToHost, s));
        rc = sync();
        if (rc) return rc;
        out.resize(S);
        for (int k = 0; k < S; ++k) out[k] = std::sqrt(std::max(0.0, hh[k].real()));
        return HSWEEP_OK;
    };

    std::vector<double> fnorm, beta;
    rc = norms(f, fnorm);
    if (rc) return rc;
    HIPCHK(hipMemsetAsync(u, 0, Ntot * sizeof(c128), s));
    std::vector<int> its(S, 0), done(S, 0);
    std::vector<double> res(S, 0.0);
    for (int k = 0; k < S; ++k) {
        if (fnorm[k] == 0.0) { done[k] = 1; res[k] = 0.0; }
        else res[k] = 1.0;
    }
    // first residual is f itself (x0 = 0)
    HIPCHK(hipMemcpyAsync(rr, f, Ntot * sizeof(c128), hipMemcpyDeviceToDevice, s));
    beta = fnorm;
    std::vector<std::vector<std::complex<double>>> H(S), g(S), sn(S);
    std::vector<std::vector<double>> cs(S);
    std::vector<int> kk(S, 0), incycle(S, 0);
    bool any_left = true;
    while (any_left) {
        // start a cycle for every unfinished right-hand side
        int ncyc = 0;
        for (int k = 0; k < S; ++k) {
            incycle[k] = (!done[k] && its[k] < maxit) ? 1 : 0;
            ncyc += incycle[k];
            sch[k] = incycle[k] && beta[k] > 0 ? 1.0 / beta[k] : 0.0;
            acth[k] = incycle[k];
            H[k].assign((size_t)(m + 1) * m, 0.0);
            g[k].assign(m + 1, 0.0);
            g[k][0] = beta[k];
            cs[k].assign(m, 0.0);
            sn[k].assign(m, 0.0);
            kk[k] = 0;
        }
        if (ncyc == 0) break;
        HIPCHK(hipMemcpyAsync(scd, sch, S * sizeof(double), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(actd, acth, S * sizeof(int), hipMemcpyHostToDevice, s));
        launch_scale(rr, scd, V, offd, S, maxlen, s);
        for (int j = 0; j < m; ++j) {
            HIPCHK(hipEventRecord(c0->ev[0], s));
            rc = sweep_column(j);
            if (rc) return rc;
            HIPCHK(hipEventRecord(c0->ev[1], s));
            stencil_all(Z + (size_t)j * Ntot, nullptr, w, actd);
            HIPCHK(hipEventRecord(c0->ev[2], s));
            // classical Gram-Schmidt, twice
            launch_multi_dot(V, j + 1, Ntot, w, offd, S, part, hd1, nblk, s);
            launch_multi_axpy(V, j + 1, Ntot, hd1, w, offd, S, maxlen, s);
            launch_multi_dot(V, j + 1, Ntot, w, offd, S, part, hd2, nblk, s);
            launch_multi_axpy(V, j + 1, Ntot, hd2, w, offd, S, maxlen, s);
            launch_multi_dot(w, 1, Ntot, w, offd, S, part, hd3, nblk, s);
            HIPCHK(hipEventRecord(c0->ev[3], s));
            HIPCHK(hipMemcpyAsync(hh, hd, (size_t)3 * nvmax * S * sizeof(c128), hipMemcpyDeviceToHost, s));
            rc = sync();
            if (rc) return rc;
            float t1 = 0, t2 = 0, t3 = 0;
            (void)hipEventElapsedTime(&t1, c0->ev[0], c0->ev[1]);
            (void)hipEventElapsedTime(&t2, c0->ev[1], c0->ev[2]);
            (void)hipEventElapsedTime(&t3, c0->ev[2], c0->ev[3]);
            c0->t_sweep += t1;
            c0->t_stencil += t2;
            c0->t_krylov += t3;
            c0->n_apply += 1;
            const std::complex<double>* h1 = hh;
            const std::complex<double>* h2 = hh + (size_t)nvmax * S;
            const std::complex<double>* h3 = hh + (size_t)2 * nvmax * S;
            int still = 0;
            for (int k = 0; k < S; ++k) {
                if (!incycle[k] || !acth[k]) { sch[k] = 0.0; continue; }
                its[k] += 1;
                std::complex<double>* col = &H[k][(size_t)j * (m + 1)];
                for (int i = 0; i <= j; ++i) col[i] = h1[(size_t)i * S + k] + h2[(size_t)i * S + k];
                double hn = std::sqrt(std::max(0.0, h3[k].real()));
                col[j + 1] = hn;
                for (int i = 0; i < j; ++i) {
                    std::complex<double> t = cs[k][i] * col[i] + sn[k][i] * col[i + 1];
                    col[i + 1] = -std::conj(sn[k][i]) * col[i] + cs[k][i] * col[i + 1];
                    col[i] = t;
                }
                givens(col[j], col[j + 1], cs[k][j], sn[k][j]);
                col[j] = cs[k][j] * col[j] + sn[k][j] * col[j + 1];
                col[j + 1] = 0.0;
                g[k][j + 1] = -std::conj(sn[k][j]) * g[k][j];
                g[k][j] = cs[k][j] * g[k][j];
                kk[k] = j + 1;
                double est = std::abs(g[k][j + 1]) / fnorm[k];
                bool stop = est <= tol || its[k] >= maxit || hn == 0.0;
                if (stop) {
                    acth[k] = 0;
                    sch[k] = 0.0;
                } else {
                    sch[k] = 1.0 / hn;
                    ++still;
                }
            }
            HIPCHK(hipMemcpyAsync(scd, sch, S * sizeof(double), hipMemcpyHostToDevice, s));
            HIPCHK(hipMemcpyAsync(actd, acth, S * sizeof(int), hipMemcpyHostToDevice, s));
            if (still == 0) break;
            launch_scale(w, scd, V + (size_t)(j + 1) * Ntot, offd, S, maxlen, s);
        }
        // solve the triangular systems and update x
        int kmax = 0;
        for (int k = 0; k < S; ++k) {
            for (int i = 0; i < m; ++i) yh[(size_t)i * S + k] = 0.0;
            if (!incycle[k] || kk[k] == 0) continue;
            int q = kk[k];
            std::vector<std::complex<double>> yy(q);
            for (int i = q - 1; i >= 0; --i) {
                std::complex<double> acc = g[k][i];
                for (int l = i + 1; l < q; ++l) acc -= H[k][(size_t)l * (m + 1) + i] * yy[l];
                yy[i] = acc / H[k][(size_t)i * (m + 1) + i];
            }
            for (int i = 0; i < q; ++i) yh[(size_t)i * S + k] = yy[i];
            kmax = std::max(kmax, q);
        }
        if (kmax > 0) {
            HIPCHK(hipMemcpyAsync(yd, yh, (size_t)m * S * sizeof(c128), hipMemcpyHostToDevice, s));
            launch_combine(Z, kmax, Ntot, yd, u, offd, S, maxlen, s);
        }
        // true residual
        stencil_all(u, f, rr, nullptr);
        rc = norms(rr, beta);
        if (rc) return rc;
        any_left = false;
        for (int k = 0; k < S; ++k) {
            if (done[k]) continue;
            res[k] = beta[k] / fnorm[k];
            if (res[k] <= tol) done[k] = 1;
            else if (its[k] < maxit) any_left = true;
        }
    }
    if (count > 1) {
        for (int q = 0; q < count; ++q)
            HIPCHK(hipMemcpyAsync(u_out[q], u + offh[first[q]], (offh[first[q + 1]] - offh[first[q]]) * sizeof(c128),
                                  hipMemcpyDeviceToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
    }
    HIPCHK(hipGetLastError());
    bool all = true;
    for (int k = 0; k < S; ++k) {
        if (iters) iters[k] = its[k];
        if (relres) relres[k] = res[k];
        if (!done[k]) all = false;
    }
    if (!all) return fail(HSWEEP_ENOCONV, "GMRES reached maxit before tol for some right-hand side");
    return HSWEEP_OK;
}

}  // namespace

extern "C" {

void hsweep_default_opts(hsweep_opts* o) {
    if (!o) return;
    o->leaf = 16;
    o->rank = 8;
    o->rank_tol = 1e-6;
    o->pml_C = 20.0;
    o->precision = HSWEEP_C128;
    o->dense = 0;
    o->restart = 40;
    o->rhs_group = 0;
    o->direction = HSWEEP_DIR_PX2;
    for (int k = 0; k < 4; ++k) o->pml_sides[k] = -1;
    o->admissibility = HSWEEP_ADM_WEAK;
}

const char* hsweep_last_error(void) { return g_err.c_str(); }

int hsweep_setup(const double* c, double omega, int pml, int n, hsweep_ctx** out) {
    g_err.clear();
    if (!out) return fail(HSWEEP_EINVAL, "out is NULL");
    *out = nullptr;
    if (!c) return fail(HSWEEP_EINVAL, "c is NULL");
    if (n < 3 || n > 8191) return fail(HSWEEP_EINVAL, "n must be in [3, 8191]");
    if (!(omega > 0.0) || !isfinite(omega)) return fail(HSWEEP_EINVAL, "omega must be finite and > 0");
    if (pml < 0 || 2 * pml >= n) return fail(HSWEEP_EINVAL, "pml must satisfy 0 <= pml and 2*pml < n");
    const size_t N = (size_t)n * n;
    std::vector<double> hc;
    const double* host_c = c;
    bool dev = is_device_pointer(c);
    if (dev) {
        hc.resize(N);
        hipError_t e = hipMemcpy(hc.data(), c, N * sizeof(double), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return fail(HSWEEP_EDEVICE, std::string("copy of c: ") + hipGetErrorString(e));
        host_c = hc.data();
    }
    for (size_t i = 0; i < N; ++i)
        if (!(host_c[i] > 0.0) || !isfinite(host_c[i]))
            return fail(HSWEEP_EINVAL, "c must be finite and > 0 everywhere");
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        return fail(HSWEEP_EDEVICE, "no HIP device available");
    }
    hsweep_ctx* ctx = new hsweep_ctx();
    ctx->n = n;
    ctx->pml = pml;
    ctx->omega = omega;
    if (hipGetDevice(&ctx->device) != hipSuccess) ctx->device = 0;
    hsweep_default_opts(&ctx->opts);
    auto bail = [&](int code) { delete ctx; return code; };
    int rc;
#define SETUPCHK(expr)                                                                     \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess) {                                                            \
            rc = fail(e_ == hipErrorOutOfMemory ? HSWEEP_ENOMEM : HSWEEP_EDEVICE,          \
                      std::string(#expr) + ": " + hipGetErrorString(e_));                  \
            return bail(rc);                                                               \
        }                                                                                  \
    } while (0)
    SETUPCHK(ctx->c.ensure(N * sizeof(double)));
    SETUPCHK(ctx->isn1.ensure((size_t)n * sizeof(c128)));
    SETUPCHK(ctx->sh1.ensure((size_t)(n + 1) * sizeof(c128)));
    SETUPCHK(ctx->isn2.ensure((size_t)n * sizeof(c128)));
    SETUPCHK(ctx->sh2.ensure((size_t)(n + 1) * sizeof(c128)));
    SETUPCHK(hipMemcpy(ctx->c.p, c, N * sizeof(double), dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice));
    for (int i = 0; i < 4; ++i) SETUPCHK(hipEventCreate(&ctx->ev[i]));
    rc = scratch_init(ctx->device);
    if (rc) return bail(rc);
    rc = build_tables(ctx, ctx->opts);
    if (rc) return bail(rc);
    SETUPCHK(hipGetLastError());
    SETUPCHK(hipDeviceSynchronize());
#undef SETUPCHK
    *out = ctx;
    return HSWEEP_OK;
}

int hsweep_set_opts(hsweep_ctx* ctx, const hsweep_opts* o) {
    g_err.clear();
    int rc = check_ctx(ctx);
    if (rc) return rc;
    rc = validate_opts(o, ctx->n);
    if (rc) return rc;
    for (int k = 0; k < 2; ++k)
        if (side_width(ctx, *o, 2 * k) + side_width(ctx, *o, 2 * k + 1) >= ctx->n)
            return fail(HSWEEP_EINVAL, "the two absorbing layers of an axis must leave interior points");
    bool pml_changed = o->pml_C != ctx->opts.pml_C;
    for (int k = 0; k < 4; ++k) pml_changed = pml_changed || side_width(ctx, *o, k) != side_width(ctx, ctx->opts, k);
    hsweep_opts old = ctx->opts;
    ctx->opts = *o;
    Plan p;
    rc = make_plan(ctx, p);
    if (rc) {
        ctx->opts = old;
        return rc;
    }
    ctx->plan = p;
    ctx->planned = true;
    ctx->factored = false;
    if (pml_changed) {
        rc = set_device(ctx);
        if (rc) return rc;
        rc = build_tables(ctx, *o);
        if (rc) return rc;
    }
    return HSWEEP_OK;
}

int hsweep_get_opts(const hsweep_ctx* ctx, hsweep_opts* o) {
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!o) return fail(HSWEEP_EINVAL, "opts is NULL");
    *o = ctx->opts;
    return HSWEEP_OK;
}

int hsweep_plan_info(const hsweep_ctx* ctx, int* n_p, int* levels, size_t* factor_bytes) {
    int rc = check_ctx(ctx);
    if (rc) return rc;
    Plan p = ctx->plan;
    if (!ctx->planned) {
        rc = make_plan(const_cast<hsweep_ctx*>(ctx), p);
        if (rc) return rc;
    }
    if (n_p) *n_p = p.np;
    if (levels) *levels = p.L;
    size_t elem = ctx->opts.precision == HSWEEP_C64 ? sizeof(c64) : sizeof(c128);
    if (factor_bytes)
        *factor_bytes = !ctx->factored ? 0 : is_strong(ctx) ? strong_bytes(ctx->strong) : (size_t)p.n * p.eLayer * elem;
    return HSWEEP_OK;
}

int hsweep_factor(hsweep_ctx* ctx, void* stream) {
    g_err.clear();
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!ctx->planned) {
        Plan p;
        rc = make_plan(ctx, p);
        if (rc) return rc;
        ctx->plan = p;
        ctx->planned = true;
    }
    rc = set_device(ctx);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    ctx->factored = false;
    HIPCHK(hipEventRecord(ctx->ev[0], s));
    if (is_strong(ctx)) {
        rc = do_factor_strong(ctx, s);
    } else {
        strong_free(ctx->strong);
        ctx->strong = nullptr;
        rc = ctx->opts.precision == HSWEEP_C64 ? do_factor_one<float>(ctx, s) : do_factor_one<double>(ctx, s);
    }
    if (rc) return rc;
    HIPCHK(hipEventRecord(ctx->ev[1], s));
    HIPCHK(hipEventSynchronize(ctx->ev[1]));
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]) == hipSuccess) ctx->t_factor = ms;
    ctx->factored = true;
    return HSWEEP_OK;
}

int hsweep_apply(hsweep_ctx* ctx, const void* f, void* u, int nrhs, void* stream) {
    g_err.clear();
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!f || !u) return fail(HSWEEP_EINVAL, "f and u must be device pointers");
    if (nrhs < 1 || nrhs > 65535) return fail(HSWEEP_EINVAL, "nrhs must be in [1, 65535]");
    if (f == u) return fail(HSWEEP_EINVAL, "f and u must not overlap");
    if (!ctx->factored) return fail(HSWEEP_ESTATE, "hsweep_apply before hsweep_factor");
    rc = set_device(ctx);
    if (rc) return rc;
    return apply_dispatch(ctx, (const c128*)f, (c128*)u, nrhs, nullptr, (hipStream_t)stream);
}

int hsweep_apply_noalloc(hsweep_ctx* ctx, const void* f, void* u, int nrhs, void* stream) {
    g_err.clear();
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!f || !u) return fail(HSWEEP_EINVAL, "f and u must be device pointers");
    if (nrhs < 1 || nrhs > 65535) return fail(HSWEEP_EINVAL, "nrhs must be in [1, 65535]");
    if (f == u) return fail(HSWEEP_EINVAL, "f and u must not overlap");
    if (is_strong(ctx)) return fail(HSWEEP_EINVAL, "hsweep_apply_noalloc serves the weak format only");
    if (!ctx->factored) return fail(HSWEEP_ESTATE, "hsweep_apply_noalloc before hsweep_factor");
    const Plan& p = ctx->plan;
    const size_t elem = ctx->opts.precision == HSWEEP_C64 ? sizeof(c64) : sizeof(c128);
    const size_t need = (size_t)nrhs * p.n * p.np * elem;
    if (need > (size_t)HSWEEP_NOALLOC_SCRATCH_BYTES)
        return fail(HSWEEP_EINVAL, "hsweep_apply_noalloc: nrhs * n * n_p work entries (" + std::to_string(need) +
                                       " bytes) exceed the static scratch of " +
                                       std::to_string((size_t)HSWEEP_NOALLOC_SCRATCH_BYTES) + " bytes");
    rc = set_device(ctx);
    if (rc) return rc;
    void* work = ctx->device < kMaxDevices ? g_scratch_ptr[ctx->device] : nullptr;
    if (!work) return fail(HSWEEP_EDEVICE, "scratch address of this device is unknown (no hsweep_setup on it)");
    const hipStream_t s = (hipStream_t)stream;
    if (ctx->opts.precision == HSWEEP_C64) return do_apply<float>(ctx, (const c128*)f, (c128*)u, nrhs, nullptr, s, work);
    return do_apply<double>(ctx, (const c128*)f, (c128*)u, nrhs, nullptr, s, work);
}

int hsweep_stencil(hsweep_ctx* ctx, const void* x, void* y, int nrhs, void* stream) {
    g_err.clear();
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!x || !y) return fail(HSWEEP_EINVAL, "x and y must be device pointers");
    if (nrhs < 1 || nrhs > 65535) return fail(HSWEEP_EINVAL, "nrhs must be in [1, 65535]");
    if (x == y) return fail(HSWEEP_EINVAL, "x and y must not overlap");
    rc = set_device(ctx);
    if (rc) return rc;
    launch_stencil(ctx->n, nrhs, ctx->omega, (const double*)ctx->c.p, ctx->tables(), (const c128*)x, nullptr, (c128*)y,
                   nullptr, (hipStream_t)stream);
    HIPCHK(hipGetLastError());
    return HSWEEP_OK;
}

int hsweep_dirichlet_forcing(hsweep_ctx* ctx, int edge, const void* b, void* f, int nrhs, void* stream) {
    g_err.clear();
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!b || !f) return fail(HSWEEP_EINVAL, "b and f must be device pointers");
    if (edge < 0 || edge > 3) return fail(HSWEEP_EINVAL, "edge must be one of HSWEEP_EDGE_*");
    if (nrhs < 1 || nrhs > 65535) return fail(HSWEEP_EINVAL, "nrhs must be in [1, 65535]");
    if ((ctx->tables().abc >> edge) & 1)
        return fail(HSWEEP_EINVAL, "Dirichlet data on an edge with the absorbing boundary condition");
    rc = set_device(ctx);
    if (rc) return rc;
    launch_dirichlet(ctx->n, nrhs, ctx->omega, (const double*)ctx->c.p, ctx->tables(), edge, (const c128*)b, (c128*)f,
                     (hipStream_t)stream);
    HIPCHK(hipGetLastError());
    return HSWEEP_OK;
}

int hsweep_grad_c(hsweep_ctx* ctx, const void* u, const void* mu, int nrhs, void* grad, void* stream) {
    g_err.clear();
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!u || !mu || !grad) return fail(HSWEEP_EINVAL, "u, mu and grad must be device pointers");
    if (nrhs < 1) return fail(HSWEEP_EINVAL, "nrhs must be >= 1");
    if (ctx->tables().abc)
        return fail(HSWEEP_EINVAL, "the velocity gradient is not available with the absorbing boundary condition");
    rc = set_device(ctx);
    if (rc) return rc;
    launch_grad(ctx->n, nrhs, ctx->omega, (const double*)ctx->c.p, ctx->tables(), (const c128*)u, (const c128*)mu,
                (double*)grad, (hipStream_t)stream);
    HIPCHK(hipGetLastError());
    return HSWEEP_OK;
}

int hsweep_solve(hsweep_ctx* ctx, const void* fv, void* uv, int nrhs, double tol, int maxit, int* iters,
                 double* relres, void* stream) {
    g_err.clear();
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!fv || !uv) return fail(HSWEEP_EINVAL, "f and u must be device pointers");
    if (fv == uv) return fail(HSWEEP_EINVAL, "f and u must not overlap");
    if (nrhs < 1 || nrhs > 65535) return fail(HSWEEP_EINVAL, "nrhs must be in [1, 65535]");
    if (!(tol > 0.0) || !isfinite(tol)) return fail(HSWEEP_EINVAL, "tol must be finite and > 0");
    if (maxit < 1) return fail(HSWEEP_EINVAL, "maxit must be >= 1");
    if (!ctx->factored) return fail(HSWEEP_ESTATE, "hsweep_solve before hsweep_factor");
    rc = set_device(ctx);
    if (rc) return rc;
    const c128* f = (const c128*)fv;
    c128* u = (c128*)uv;
    return solve_systems(&ctx, 1, &nrhs, &f, &u, tol, maxit, iters, relres, (hipStream_t)stream);
}

int hsweep_solve_adjoint(hsweep_ctx* ctx, const void* g, void* mu, void* grad_f, int nrhs, double tol, int maxit,
                         int* iters, double* relres, void* stream) {
    g_err.clear();
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!g || !mu) return fail(HSWEEP_EINVAL, "g and mu must be device pointers");
    if (g == mu || (grad_f && (grad_f == g || grad_f == mu)))
        return fail(HSWEEP_EINVAL, "g, mu and grad_f must not overlap");
    if (nrhs < 1 || nrhs > 65535) return fail(HSWEEP_EINVAL, "nrhs must be in [1, 65535]");
    if (!(tol > 0.0) || !isfinite(tol)) return fail(HSWEEP_EINVAL, "tol must be finite and > 0");
    if (maxit < 1) return fail(HSWEEP_EINVAL, "maxit must be >= 1");
    if (!ctx->factored) return fail(HSWEEP_ESTATE, "hsweep_solve_adjoint before hsweep_factor");
    rc = set_device(ctx);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const size_t tot = (size_t)nrhs * ctx->n * ctx->n;
    HIPCHK(ctx->adj.ensure(tot * sizeof(c128)));
    launch_conj((const c128*)g, (c128*)ctx->adj.p, tot, s);
    HIPCHK(hipGetLastError());
    rc = hsweep_solve(ctx, ctx->adj.p, mu, nrhs, tol, maxit, iters, relres, stream);
    if (rc != HSWEEP_OK && rc != HSWEEP_ENOCONV) return rc;
    if (grad_f) {
        launch_conj((const c128*)mu, (c128*)grad_f, tot, s);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(s));
    }
    return rc;
}

int hsweep_workspace_bytes(const hsweep_ctx* ctx, int nrhs, size_t* factor_bytes, size_t* solve_bytes) {
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (nrhs < 1 || nrhs > 65535) return fail(HSWEEP_EINVAL, "nrhs must be in [1, 65535]");
    Plan p = ctx->plan;
    if (!ctx->planned) {
        rc = make_plan(const_cast<hsweep_ctx*>(ctx), p);
        if (rc) return rc;
    }
    const size_t E = ctx->opts.precision == HSWEEP_C64 ? sizeof(c64) : sizeof(c128);
    const size_t n = (size_t)p.n, np = (size_t)p.np, N = n * n, K = (size_t)nrhs;
    const size_t m = (size_t)ctx->opts.restart;
    // coefficients of the setup: c, 1/s on the nodes and s on the half nodes of both axes
    size_t fb = N * sizeof(double) + 2 * (2 * n + 1) * sizeof(c128);
    size_t sb = 0;
    if (is_strong(ctx)) {
        // layer operators and the stored strong factors (known after hsweep_factor;
        // the factorization's own scratch is not counted); the sweep keeps w_m of
        // every layer and two layer vectors per right-hand side
        fb += 2 * n * n * sizeof(c128) + (n > 1 ? n : 2) * n * sizeof(c128);
        fb += ctx->factored ? strong_bytes(ctx->strong) : 0;
        sb = (n + 2) * n * K * sizeof(c128);
    } else {
        // layer operators, factor store and the per-layer work of the factorization
        fb += 2 * n * np * E + (n > 1 ? n : 2) * np * E + n * p.eLayer * E;
        fb += (size_t)(p.L > 0 ? p.L : 1) * p.r * np * E + ((size_t)2 << p.L) * p.r * p.r * E;
        fb += n * ((size_t)1 << p.L) * sizeof(int) + sizeof(int);
        sb = K * n * np * E;                    // sweep work vectors
    }
    // the flexible-GMRES basis, residuals and small arrays
    const size_t nblk = (size_t)krylov_dot_blocks(N);
    sb += (2 * m + 1) * K * N * sizeof(c128) + 2 * K * N * sizeof(c128);
    sb += 3 * (m + 1) * K * sizeof(c128) + nblk * K * (m + 1) * sizeof(c128);
    sb += K * (sizeof(double) + sizeof(int)) + m * K * sizeof(c128) + (K + 1) * sizeof(size_t);
    if (factor_bytes) *factor_bytes = fb;
    if (solve_bytes) *solve_bytes = sb;
    return HSWEEP_OK;
}

int hsweep_factor_batch(hsweep_ctx** ctxs, int count, void* stream) {
    g_err.clear();
    if (!ctxs || count < 1) return fail(HSWEEP_EINVAL, "ctxs must hold count >= 1 contexts");
    for (int q = 0; q < count; ++q) {
        int rc = check_ctx(ctxs[q]);
        if (rc) return rc;
        if (!ctxs[q]->planned) {
            Plan p;
            rc = make_plan(ctxs[q], p);
            if (rc) return rc;
            ctxs[q]->plan = p;
            ctxs[q]->planned = true;
        }
        if (ctxs[q]->opts.precision != ctxs[0]->opts.precision || ctxs[q]->device != ctxs[0]->device)
            return fail(HSWEEP_EINVAL, "contexts of one batch need the same precision and device");
        if (is_strong(ctxs[q])) return fail(HSWEEP_EINVAL, "batched factorization serves the weak format only");
    }
    int rc = set_device(ctxs[0]);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    for (int q = 0; q < count; ++q) ctxs[q]->factored = false;
    HIPCHK(hipEventRecord(ctxs[0]->ev[0], s));
    // one layer loop per group of contexts with the same leaf size and rank;
    // within a group every layer step is one set of launches for all of them
    std::vector<std::vector<hsweep_ctx*>> groups;
    for (int q = 0; q < count; ++q) {
        const Plan& a = ctxs[q]->plan;
        bool placed = false;
        for (auto& g : groups) {
            const Plan& b0 = g[0]->plan;
            if (a.b == b0.b && (a.L > 0 ? a.r : 2) == (b0.L > 0 ? b0.r : 2)) { g.push_back(ctxs[q]); placed = true; break; }
        }
        if (!placed) groups.push_back({ctxs[q]});
    }
    for (auto& g : groups) {
        rc = ctxs[0]->opts.precision == HSWEEP_C64 ? do_factor_many<float>(g.data(), (int)g.size(), s)
                                                   : do_factor_many<double>(g.data(), (int)g.size(), s);
        if (rc) return rc;
    }
    HIPCHK(hipEventRecord(ctxs[0]->ev[1], s));
    HIPCHK(hipEventSynchronize(ctxs[0]->ev[1]));
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ctxs[0]->ev[0], ctxs[0]->ev[1]);
    for (int q = 0; q < count; ++q) {
        ctxs[q]->t_factor = ms;
        ctxs[q]->factored = true;
    }
    return HSWEEP_OK;
}

int hsweep_solve_batch(hsweep_ctx** ctxs, int count, const void* const* f, void* const* u, double tol, int maxit,
                       int* iters, double* relres, void* stream) {
    g_err.clear();
    if (!ctxs || count < 1 || !f || !u) return fail(HSWEEP_EINVAL, "ctxs, f and u must hold count >= 1 entries");
    if (count > 4096) return fail(HSWEEP_EINVAL, "at most 4096 contexts per batch");
    if (!(tol > 0.0) || !isfinite(tol)) return fail(HSWEEP_EINVAL, "tol must be finite and > 0");
    if (maxit < 1) return fail(HSWEEP_EINVAL, "maxit must be >= 1");
    for (int q = 0; q < count; ++q) {
        int rc = check_ctx(ctxs[q]);
        if (rc) return rc;
        if (!f[q] || !u[q] || f[q] == u[q]) return fail(HSWEEP_EINVAL, "f[k] and u[k] must be distinct device pointers");
        if (is_strong(ctxs[q])) return fail(HSWEEP_EINVAL, "batched solves serve the weak format only");
        if (!ctxs[q]->factored) return fail(HSWEEP_ESTATE, "hsweep_solve_batch before the contexts are factored");
        if (ctxs[q]->opts.precision != ctxs[0]->opts.precision || ctxs[q]->device != ctxs[0]->device)
            return fail(HSWEEP_EINVAL, "contexts of one batch need the same precision and device");
        for (int p = 0; p < q; ++p)
            if (ctxs[p] == ctxs[q]) return fail(HSWEEP_EINVAL, "a context appears twice in the batch");
    }
    int rc = set_device(ctxs[0]);
    if (rc) return rc;
    std::vector<int> nr(count, 1);
    return solve_systems(ctxs, count, nr.data(), (const c128* const*)f, (c128* const*)u, tol, maxit, iters, relres,
                         (hipStream_t)stream);
}

void hsweep_destroy(hsweep_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    delete ctx;
}

int hsweep_factor_profile(hsweep_ctx* ctx, void* stream, double* out, int count) {
    g_err.clear();
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!out || count < 3) return fail(HSWEEP_EINVAL, "out must hold count >= 3 doubles");
    if (is_strong(ctx)) return fail(HSWEEP_EINVAL, "hsweep_factor_profile times the weak format's kernels only");
    if (!ctx->planned) {
        Plan p;
        rc = make_plan(ctx, p);
        if (rc) return rc;
        ctx->plan = p;
        ctx->planned = true;
    }
    rc = set_device(ctx);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    ctx->factored = false;
    double tl = 0.0, tw = 0.0;
    rc = ctx->opts.precision == HSWEEP_C64 ? do_factor_profile<float>(ctx, s, &tl, &tw)
                                           : do_factor_profile<double>(ctx, s, &tl, &tw);
    if (rc) return rc;
    ctx->factored = true;
    out[0] = tl;
    out[1] = tw;
    out[2] = (double)ctx->plan.n;
    return HSWEEP_OK;
}

int hsweep_timings(const hsweep_ctx* ctx, double* out, int count) {
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!out || count < 1) return fail(HSWEEP_EINVAL, "out must hold count >= 1 doubles");
    double v[5] = {ctx->t_factor, ctx->t_sweep, ctx->t_stencil, ctx->t_krylov, ctx->n_apply};
    for (int i = 0; i < count && i < 5; ++i) out[i] = v[i];
    return HSWEEP_OK;
}

}  // extern "C"
