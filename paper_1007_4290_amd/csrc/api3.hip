// C-ABI of the 3D sweeping preconditioner (Sec. 4): an n x n x n grid with
// absorbing layers on all six sides, swept face by face (faces x3 = const)
// with strongly admissible H-matrix factors on quadtree face clusters, and
// the flexible GMRES driver in FP64 around it.  Complex128 throughout.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <complex>
#include <string>
#include <vector>

#include "hsweep.h"
#include "internal.hpp"

namespace {

struct Buf {
    void* p = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t b) {
        if (b <= bytes && p) return hipSuccess;
        release();
        hipError_t e = hipMalloc(&p, b ? b : 1);
        if (e == hipSuccess) bytes = b;
        else p = nullptr;
        return e;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
};

#define CHK3(expr)                                                                                 \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return hsweep_report(e_ == hipErrorOutOfMemory ? HSWEEP_ENOMEM : HSWEEP_EDEVICE,       \
                                 std::string(#expr) + ": " + hipGetErrorString(e_));               \
    } while (0)

constexpr uint64_t kSeed3 = 0x9E6C63D0676A9A99ull;

}  // namespace

struct hsweep3_ctx {
    int n = 0, pml = 0, device = 0;
    double omega = 0.0;
    hsweep_opts opts{};
    Buf c, isn[3], sh[3], coef[7];
    StrongFactors* sf = nullptr;
    bool factored = false;
    // GMRES work
    Buf V, Z, w, r, hdev, partial, scale, active, y, offd;
    Coef3 cf() const {
        return Coef3{(c128*)coef[0].p, (c128*)coef[1].p, (c128*)coef[2].p, (c128*)coef[3].p,
                     (c128*)coef[4].p, (c128*)coef[5].p, (c128*)coef[6].p};
    }
    ~hsweep3_ctx() {
        strong_free(sf);
        Buf* all[] = {&c, &isn[0], &isn[1], &isn[2], &sh[0], &sh[1], &sh[2], &coef[0], &coef[1], &coef[2], &coef[3],
                      &coef[4], &coef[5], &coef[6], &V, &Z, &w, &r, &hdev, &partial, &scale, &active, &y, &offd};
        for (Buf* b : all) b->release();
    }
};

namespace {

int check3(const hsweep3_ctx* ctx) {
    if (!ctx) return hsweep_report(HSWEEP_EINVAL, "context is NULL");
    return HSWEEP_OK;
}

int device3(const hsweep3_ctx* ctx) {
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hsweep_report(HSWEEP_EDEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
    return HSWEEP_OK;
}

// Stretching tables of the three axes and the coefficient fields.
int build3(hsweep3_ctx* ctx) {
    const int n = ctx->n;
    const double h = 1.0 / (n + 1);
    const c128* isn[3];
    const c128* sh[3];
    for (int a = 0; a < 3; ++a) {
        launch_pml_1d(n, ctx->omega, ctx->pml * h, ctx->pml * h, ctx->opts.pml_C, (c128*)ctx->isn[a].p,
                      (c128*)ctx->sh[a].p, 0);
        isn[a] = (const c128*)ctx->isn[a].p;
        sh[a] = (const c128*)ctx->sh[a].p;
    }
    launch_coeff3(n, ctx->omega, (const double*)ctx->c.p, isn, sh, ctx->cf(), 0);
    CHK3(hipGetLastError());
    CHK3(hipDeviceSynchronize());
    return HSWEEP_OK;
}

void givens3(std::complex<double> a, std::complex<double> b, double& c, std::complex<double>& s) {
    if (b == 0.0) { c = 1.0; s = 0.0; return; }
    if (a == 0.0) { c = 0.0; s = std::conj(b) / std::abs(b); return; }
    const double t = std::hypot(std::abs(a), std::abs(b));
    c = std::abs(a) / t;
    s = (a / std::abs(a)) * std::conj(b) / t;
}

// Flexible GMRES (right preconditioner: the face-by-face sweep; FP64
// Arnoldi, classical Gram-Schmidt twice; Givens rotations on the host) for
// nrhs fields f -> u, each stopping on its own true residual.
int solve3(hsweep3_ctx* ctx, const c128* f, c128* u, int S, double tol, int maxit, int* iters, double* relres,
           hipStream_t s) {
    const size_t N3 = (size_t)ctx->n * ctx->n * ctx->n, Ntot = N3 * S;
    const int m = ctx->opts.restart, nv = m + 1;
    const int nblk = krylov_dot_blocks(N3);
    CHK3(ctx->V.ensure((size_t)nv * Ntot * sizeof(c128)));
    CHK3(ctx->Z.ensure((size_t)m * Ntot * sizeof(c128)));
    CHK3(ctx->w.ensure(Ntot * sizeof(c128)));
    CHK3(ctx->r.ensure(Ntot * sizeof(c128)));
    CHK3(ctx->hdev.ensure((size_t)3 * nv * S * sizeof(c128)));
    CHK3(ctx->partial.ensure((size_t)nblk * S * nv * sizeof(c128)));
    CHK3(ctx->scale.ensure((size_t)S * sizeof(double)));
    CHK3(ctx->active.ensure((size_t)S * sizeof(int)));
    CHK3(ctx->y.ensure((size_t)m * S * sizeof(c128)));
    CHK3(ctx->offd.ensure((size_t)(S + 1) * sizeof(size_t)));
    std::vector<size_t> off(S + 1);
    for (int k = 0; k <= S; ++k) off[k] = (size_t)k * N3;
    CHK3(hipMemcpyAsync(ctx->offd.p, off.data(), (S + 1) * sizeof(size_t), hipMemcpyHostToDevice, s));
    const size_t* offd = (const size_t*)ctx->offd.p;
    c128* V = (c128*)ctx->V.p;
    c128* Z = (c128*)ctx->Z.p;
    c128* w = (c128*)ctx->w.p;
    c128* rr = (c128*)ctx->r.p;
    c128* hd = (c128*)ctx->hdev.p;
    c128* hd1 = hd;
    c128* hd2 = hd + (size_t)nv * S;
    c128* hd3 = hd2 + (size_t)nv * S;
    c128* part = (c128*)ctx->partial.p;
    double* scd = (double*)ctx->scale.p;
    int* actd = (int*)ctx->active.p;
    c128* yd = (c128*)ctx->y.p;
    std::vector<std::complex<double>> hh((size_t)3 * nv * S), yh((size_t)m * S);
    std::vector<double> sch(S);
    std::vector<int> acth(S);
    const Coef3 cf = ctx->cf();
    int rc = HSWEEP_OK;
    auto norms = [&](const c128* x, std::vector<double>& out) -> int {
        launch_multi_dot(x, 1, Ntot, x, offd, S, part, hd3, nblk, s);
        CHK3(hipMemcpyAsync(hh.data(), hd3, (size_t)S * sizeof(c128), hipMemcpyDeviceToHost, s));
        CHK3(hipStreamSynchronize(s));
        out.resize(S);
        for (int k = 0; k < S; ++k) out[k] = std::sqrt(std::max(0.0, hh[k].real()));
        return HSWEEP_OK;
    };
    std::vector<double> fnorm, beta;
    rc = norms(f, fnorm);
    if (rc) return rc;
    CHK3(hipMemsetAsync(u, 0, Ntot * sizeof(c128), s));
    CHK3(hipMemcpyAsync(rr, f, Ntot * sizeof(c128), hipMemcpyDeviceToDevice, s));
    beta = fnorm;
    std::vector<int> its(S, 0), done(S, 0), kk(S, 0), incycle(S, 0);
    std::vector<double> res(S, 1.0);
    for (int k = 0; k < S; ++k)
        if (fnorm[k] == 0.0) { done[k] = 1; res[k] = 0.0; }
    std::vector<std::vector<std::complex<double>>> H(S), g(S), sn(S);
    std::vector<std::vector<double>> cs(S);
    std::string msg;
    bool any_left = true;
    while (any_left) {
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
        CHK3(hipMemcpyAsync(scd, sch.data(), S * sizeof(double), hipMemcpyHostToDevice, s));
        CHK3(hipMemcpyAsync(actd, acth.data(), S * sizeof(int), hipMemcpyHostToDevice, s));
        launch_scale(rr, scd, V, offd, S, N3, s);
        for (int j = 0; j < m; ++j) {
            rc = strong_apply3(ctx->sf, V + (size_t)j * Ntot, Z + (size_t)j * Ntot, S, actd, s, &msg);
            if (rc) return hsweep_report(rc, msg);
            launch_stencil3(ctx->n, S, cf, Z + (size_t)j * Ntot, nullptr, w, actd, s);
            launch_multi_dot(V, j + 1, Ntot, w, offd, S, part, hd1, nblk, s);
            launch_multi_axpy(V, j + 1, Ntot, hd1, w, offd, S, N3, s);
            launch_multi_dot(V, j + 1, Ntot, w, offd, S, part, hd2, nblk, s);
            launch_multi_axpy(V, j + 1, Ntot, hd2, w, offd, S, N3, s);
            launch_multi_dot(w, 1, Ntot, w, offd, S, part, hd3, nblk, s);
            CHK3(hipMemcpyAsync(hh.data(), hd, (size_t)3 * nv * S * sizeof(c128), hipMemcpyDeviceToHost, s));
            CHK3(hipStreamSynchronize(s));
            const std::complex<double>* h1 = hh.data();
            const std::complex<double>* h2 = h1 + (size_t)nv * S;
            const std::complex<double>* h3 = h2 + (size_t)nv * S;
            int still = 0;
            for (int k = 0; k < S; ++k) {
                if (!incycle[k] || !acth[k]) { sch[k] = 0.0; continue; }
                its[k] += 1;
                std::complex<double>* col = &H[k][(size_t)j * (m + 1)];
                for (int i = 0; i <= j; ++i) col[i] = h1[(size_t)i * S + k] + h2[(size_t)i * S + k];
                const double hn = std::sqrt(std::max(0.0, h3[k].real()));
                col[j + 1] = hn;
                for (int i = 0; i < j; ++i) {
                    const std::complex<double> t = cs[k][i] * col[i] + sn[k][i] * col[i + 1];
                    col[i + 1] = -std::conj(sn[k][i]) * col[i] + cs[k][i] * col[i + 1];
                    col[i] = t;
                }
                givens3(col[j], col[j + 1], cs[k][j], sn[k][j]);
                col[j] = cs[k][j] * col[j] + sn[k][j] * col[j + 1];
                col[j + 1] = 0.0;
                g[k][j + 1] = -std::conj(sn[k][j]) * g[k][j];
                g[k][j] = cs[k][j] * g[k][j];
                kk[k] = j + 1;
                const bool stop = std::abs(g[k][j + 1]) / fnorm[k] <= tol || its[k] >= maxit || hn == 0.0;
                if (stop) {
                    acth[k] = 0;
                    sch[k] = 0.0;
                } else {
                    sch[k] = 1.0 / hn;
                    ++still;
                }
            }
            CHK3(hipMemcpyAsync(scd, sch.data(), S * sizeof(double), hipMemcpyHostToDevice, s));
            CHK3(hipMemcpyAsync(actd, acth.data(), S * sizeof(int), hipMemcpyHostToDevice, s));
            if (still == 0) break;
            launch_scale(w, scd, V + (size_t)(j + 1) * Ntot, offd, S, N3, s);
        }
        int kmax = 0;
        for (int k = 0; k < S; ++k) {
            for (int i = 0; i < m; ++i) yh[(size_t)i * S + k] = 0.0;
            if (!incycle[k] || kk[k] == 0) continue;
            const int q = kk[k];
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
            CHK3(hipMemcpyAsync(yd, yh.data(), (size_t)m * S * sizeof(c128), hipMemcpyHostToDevice, s));
            launch_combine(Z, kmax, Ntot, yd, u, offd, S, N3, s);
        }
        launch_stencil3(ctx->n, S, cf, u, f, rr, nullptr, s);
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
    CHK3(hipGetLastError());
    bool all = true;
    for (int k = 0; k < S; ++k) {
        if (iters) iters[k] = its[k];
        if (relres) relres[k] = res[k];
        if (!done[k]) all = false;
    }
    if (!all) return hsweep_report(HSWEEP_ENOCONV, "GMRES reached maxit before tol for some right-hand side");
    return HSWEEP_OK;
}

}  // namespace

extern "C" {

int hsweep3_setup(const double* c, double omega, int pml, int n, hsweep3_ctx** out) {
    hsweep_clear_error();
    if (!out) return hsweep_report(HSWEEP_EINVAL, "out is NULL");
    *out = nullptr;
    if (!c) return hsweep_report(HSWEEP_EINVAL, "c is NULL");
    if (n < 3 || n > 255) return hsweep_report(HSWEEP_EINVAL, "n must be in [3, 255]");
    if (!(omega > 0.0) || !isfinite(omega)) return hsweep_report(HSWEEP_EINVAL, "omega must be finite and > 0");
    if (pml < 0 || 2 * pml >= n) return hsweep_report(HSWEEP_EINVAL, "pml must satisfy 0 <= pml and 2*pml < n");
    const size_t N3 = (size_t)n * n * n;
    hipPointerAttribute_t attr;
    const bool dev = hipPointerGetAttributes(&attr, c) == hipSuccess &&
                     (attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged);
    (void)hipGetLastError();
    std::vector<double> hc;
    const double* host_c = c;
    if (dev) {
        hc.resize(N3);
        CHK3(hipMemcpy(hc.data(), c, N3 * sizeof(double), hipMemcpyDeviceToHost));
        host_c = hc.data();
    }
    for (size_t i = 0; i < N3; ++i)
        if (!(host_c[i] > 0.0) || !isfinite(host_c[i]))
            return hsweep_report(HSWEEP_EINVAL, "c must be finite and > 0 everywhere");
    hsweep3_ctx* ctx = new hsweep3_ctx();
    ctx->n = n;
    ctx->pml = pml;
    ctx->omega = omega;
    if (hipGetDevice(&ctx->device) != hipSuccess) ctx->device = 0;
    hsweep_default_opts(&ctx->opts);
    ctx->opts.admissibility = HSWEEP_ADM_STRONG;
    ctx->opts.rank = 2;
    auto bail = [&](int rc) { delete ctx; return rc; };
    hipError_t e = ctx->c.ensure(N3 * sizeof(double));
    for (int a = 0; a < 3 && e == hipSuccess; ++a) {
        e = ctx->isn[a].ensure((size_t)n * sizeof(c128));
        if (e == hipSuccess) e = ctx->sh[a].ensure((size_t)(n + 1) * sizeof(c128));
    }
    for (int q = 0; q < 7 && e == hipSuccess; ++q) e = ctx->coef[q].ensure(N3 * sizeof(c128));
    if (e == hipSuccess) e = hipMemcpy(ctx->c.p, c, N3 * sizeof(double), dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice);
    if (e != hipSuccess)
        return bail(hsweep_report(e == hipErrorOutOfMemory ? HSWEEP_ENOMEM : HSWEEP_EDEVICE,
                                  std::string("3D setup: ") + hipGetErrorString(e)));
    const int rc = build3(ctx);
    if (rc) return bail(rc);
    *out = ctx;
    return HSWEEP_OK;
}

int hsweep3_set_opts(hsweep3_ctx* ctx, const hsweep_opts* o) {
    hsweep_clear_error();
    int rc = check3(ctx);
    if (rc) return rc;
    if (!o) return hsweep_report(HSWEEP_EINVAL, "opts is NULL");
    if (o->admissibility != HSWEEP_ADM_STRONG || o->precision != HSWEEP_C128 || o->dense)
        return hsweep_report(HSWEEP_EINVAL, "3D faces use strongly admissible complex128 factors");
    if (o->leaf < 1 || o->leaf > 1024) return hsweep_report(HSWEEP_EINVAL, "leaf must be in [1, 1024]");
    if (o->rank < 1 || o->rank > 64) return hsweep_report(HSWEEP_EINVAL, "rank must be in [1, 64]");
    if (!(o->rank_tol >= 0.0) || !isfinite(o->rank_tol) || o->rank_tol >= 1.0)
        return hsweep_report(HSWEEP_EINVAL, "rank_tol must be in [0, 1)");
    if (!(o->pml_C > 0.0) || !isfinite(o->pml_C)) return hsweep_report(HSWEEP_EINVAL, "pml_C must be finite and > 0");
    if (o->restart < 1 || o->restart > 200) return hsweep_report(HSWEEP_EINVAL, "restart must be in [1, 200]");
    const bool pml_changed = o->pml_C != ctx->opts.pml_C;
    ctx->opts = *o;
    ctx->factored = false;
    if (pml_changed) {
        rc = device3(ctx);
        if (rc) return rc;
        return build3(ctx);
    }
    return HSWEEP_OK;
}

int hsweep3_factor(hsweep3_ctx* ctx, void* stream) {
    hsweep_clear_error();
    int rc = check3(ctx);
    if (rc) return rc;
    rc = device3(ctx);
    if (rc) return rc;
    ctx->factored = false;
    strong_free(ctx->sf);
    ctx->sf = nullptr;
    const Coef3 cf = ctx->cf();
    std::string msg;
    rc = strong_factor3(&ctx->sf, ctx->n, ctx->opts.leaf, ctx->opts.rank, ctx->opts.rank_tol, kSeed3, cf.D, cf.X0,
                        cf.X1, cf.Y0, cf.Y1, cf.Z0, (hipStream_t)stream, &msg);
    if (rc) return hsweep_report(rc, msg);
    ctx->factored = true;
    return HSWEEP_OK;
}

int hsweep3_apply(hsweep3_ctx* ctx, const void* f, void* u, int nrhs, void* stream) {
    hsweep_clear_error();
    int rc = check3(ctx);
    if (rc) return rc;
    if (!f || !u) return hsweep_report(HSWEEP_EINVAL, "f and u must be device pointers");
    if (f == u) return hsweep_report(HSWEEP_EINVAL, "f and u must not overlap");
    if (nrhs < 1 || nrhs > 65535) return hsweep_report(HSWEEP_EINVAL, "nrhs must be in [1, 65535]");
    if (!ctx->factored) return hsweep_report(HSWEEP_ESTATE, "hsweep3_apply before hsweep3_factor");
    rc = device3(ctx);
    if (rc) return rc;
    std::string msg;
    rc = strong_apply3(ctx->sf, (const c128*)f, (c128*)u, nrhs, nullptr, (hipStream_t)stream, &msg);
    return rc ? hsweep_report(rc, msg) : HSWEEP_OK;
}

int hsweep3_stencil(hsweep3_ctx* ctx, const void* x, void* y, int nrhs, void* stream) {
    hsweep_clear_error();
    int rc = check3(ctx);
    if (rc) return rc;
    if (!x || !y) return hsweep_report(HSWEEP_EINVAL, "x and y must be device pointers");
    if (x == y) return hsweep_report(HSWEEP_EINVAL, "x and y must not overlap");
    if (nrhs < 1 || nrhs > 65535) return hsweep_report(HSWEEP_EINVAL, "nrhs must be in [1, 65535]");
    rc = device3(ctx);
    if (rc) return rc;
    launch_stencil3(ctx->n, nrhs, ctx->cf(), (const c128*)x, nullptr, (c128*)y, nullptr, (hipStream_t)stream);
    CHK3(hipGetLastError());
    return HSWEEP_OK;
}

int hsweep3_solve(hsweep3_ctx* ctx, const void* f, void* u, int nrhs, double tol, int maxit, int* iters,
                  double* relres, void* stream) {
    hsweep_clear_error();
    int rc = check3(ctx);
    if (rc) return rc;
    if (!f || !u) return hsweep_report(HSWEEP_EINVAL, "f and u must be device pointers");
    if (f == u) return hsweep_report(HSWEEP_EINVAL, "f and u must not overlap");
    if (nrhs < 1 || nrhs > 65535) return hsweep_report(HSWEEP_EINVAL, "nrhs must be in [1, 65535]");
    if (!(tol > 0.0) || !isfinite(tol)) return hsweep_report(HSWEEP_EINVAL, "tol must be finite and > 0");
    if (maxit < 1) return hsweep_report(HSWEEP_EINVAL, "maxit must be >= 1");
    if (!ctx->factored) return hsweep_report(HSWEEP_ESTATE, "hsweep3_solve before hsweep3_factor");
    rc = device3(ctx);
    if (rc) return rc;
    return solve3(ctx, (const c128*)f, (c128*)u, nrhs, tol, maxit, iters, relres, (hipStream_t)stream);
}

int hsweep3_plan_info(const hsweep3_ctx* ctx, int* levels, size_t* factor_bytes) {
    int rc = check3(ctx);
    if (rc) return rc;
    if (levels) *levels = (int)strong_face_depth(ctx->n, ctx->opts.leaf);
    if (factor_bytes) *factor_bytes = ctx->factored ? strong_bytes(ctx->sf) : 0;
    return HSWEEP_OK;
}

void hsweep3_destroy(hsweep3_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    delete ctx;
}

}  // extern "C"
