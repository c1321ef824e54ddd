// Host-logic check of the C-ABI without a GPU: the library's host code runs
// against a host-memory stand-in of the HIP runtime (fake_runtime.cpp), and
// every kernel launcher is replaced by a check that the device ranges the
// kernel would touch lie inside live allocations (stubs.cpp).  Covers the
// batched factorization and FGMRES over mixed grid sizes and leaf sizes, a
// multi-right-hand-side solve, the adjoint solve, the allocation-free apply,
// every sweep direction, absorbing-condition sides, the query entry points
// and argument errors.  The stand-in dot products return 1, so GMRES runs to maxit: the
// point is the ranges, not the numbers.
#include <math.h>
#include <stdio.h>
#include <vector>
#include "hsweep.h"
#include <hip/hip_runtime.h>

int multi_launches();

static int expect(int rc, int want, const char* what) {
    if (rc != want) {
        printf("%s: rc %d (%s), expected %d\n", what, rc, hsweep_last_error(), want);
        return 1;
    }
    return 0;
}

int main() {
    int bad = 0;
    // the mixed batch: 8 each of n = 127, 255 (leaf 16) and 511 (leaf 32)
    std::vector<int> ns, leaves;
    for (int k = 0; k < 8; ++k) { ns.push_back(127); leaves.push_back(16); }
    for (int k = 0; k < 8; ++k) { ns.push_back(255); leaves.push_back(16); }
    for (int k = 0; k < 8; ++k) { ns.push_back(511); leaves.push_back(32); }
    std::vector<hsweep_ctx*> ctx(ns.size());
    std::vector<void*> f(ns.size()), u(ns.size());
    for (size_t q = 0; q < ns.size(); ++q) {
        const int n = ns[q];
        std::vector<double> c((size_t)n * n, 1.0);
        if (expect(hsweep_setup(c.data(), 2 * M_PI * (n + 1) / 8, 16, n, &ctx[q]), 0, "setup")) return 1;
        hsweep_opts o;
        hsweep_default_opts(&o);
        o.leaf = leaves[q];
        o.precision = HSWEEP_C64;
        if (expect(hsweep_set_opts(ctx[q], &o), 0, "set_opts")) return 1;
        hipMalloc(&f[q], (size_t)n * n * 16);
        hipMalloc(&u[q], (size_t)n * n * 16);
    }
    bad += expect(hsweep_factor_batch(ctx.data(), (int)ctx.size(), nullptr), 0, "factor_batch");
    std::vector<int> its(ns.size());
    std::vector<double> res(ns.size());
    bad += expect(hsweep_solve_batch(ctx.data(), (int)ctx.size(), (const void* const*)f.data(), (void* const*)u.data(),
                                     1e-10, 60, its.data(), res.data(), nullptr),
                  HSWEEP_ENOCONV, "solve_batch");
    if (multi_launches() < 2) { printf("expected one sweep launch per leaf group and step\n"); ++bad; }
    // one context, 64 right-hand sides, then an adjoint solve and the allocation-free apply
    void *F, *U, *G;
    const size_t N = (size_t)511 * 511;
    hipMalloc(&F, 64 * N * 16);
    hipMalloc(&U, 64 * N * 16);
    hipMalloc(&G, 64 * N * 16);
    std::vector<int> it64(64);
    std::vector<double> r64(64);
    bad += expect(hsweep_solve(ctx[16], F, U, 64, 1e-10, 45, it64.data(), r64.data(), nullptr), HSWEEP_ENOCONV, "solve 64");
    bad += expect(hsweep_solve_adjoint(ctx[16], F, U, G, 2, 1e-10, 45, it64.data(), r64.data(), nullptr), HSWEEP_ENOCONV,
                  "adjoint");
    bad += expect(hsweep_apply_noalloc(ctx[16], F, U, 4, nullptr), 0, "apply_noalloc");
    bad += expect(hsweep_apply(ctx[0], F, U, 3, nullptr), 0, "apply");
    bad += expect(hsweep_dirichlet_forcing(ctx[16], HSWEEP_EDGE_X2_1, G, F, 2, nullptr), 0, "dirichlet");
    bad += expect(hsweep_grad_c(ctx[16], F, U, 2, G, nullptr), 0, "grad_c");
    // every sweep direction with its own layer widths
    for (int d = 0; d < 3; ++d) {
        hsweep_opts o;
        hsweep_get_opts(ctx[1], &o);
        o.direction = d;
        o.pml_sides[0] = 0; o.pml_sides[1] = 16; o.pml_sides[2] = 10; o.pml_sides[3] = 0;
        bad += expect(hsweep_set_opts(ctx[1], &o), 0, "set_opts direction");
        bad += expect(hsweep_factor(ctx[1], nullptr), 0, "factor direction");
        bad += expect(hsweep_solve(ctx[1], F, U, 2, 1e-10, 10, it64.data(), r64.data(), nullptr), HSWEEP_ENOCONV,
                      "solve direction");
    }
    {
        hsweep_opts o;
        hsweep_get_opts(ctx[1], &o);
        o.pml_sides[0] = 64; o.pml_sides[1] = 64;
        bad += expect(hsweep_set_opts(ctx[1], &o), HSWEEP_EINVAL, "layers wider than the axis");
        o.pml_sides[0] = -1; o.pml_sides[1] = -1; o.direction = 4;
        bad += expect(hsweep_set_opts(ctx[1], &o), HSWEEP_EINVAL, "direction out of range");
        o.direction = HSWEEP_DIR_MX1;
        bad += expect(hsweep_set_opts(ctx[1], &o), HSWEEP_EINVAL, "leftward column sweep switched off");
    }
    // absorbing boundary condition on two sides: factor and solve in every
    // direction; Dirichlet data on an absorbing edge and the gradient are refused
    for (int d = 0; d < 3; ++d) {
        hsweep_opts o;
        hsweep_get_opts(ctx[1], &o);
        o.direction = d;
        o.pml_sides[0] = HSWEEP_SIDE_ABC; o.pml_sides[1] = 4; o.pml_sides[2] = 0; o.pml_sides[3] = HSWEEP_SIDE_ABC;
        bad += expect(hsweep_set_opts(ctx[1], &o), 0, "set_opts abc");
        bad += expect(hsweep_factor(ctx[1], nullptr), 0, "factor abc");
        bad += expect(hsweep_solve(ctx[1], F, U, 2, 1e-10, 10, it64.data(), r64.data(), nullptr), HSWEEP_ENOCONV,
                      "solve abc");
    }
    bad += expect(hsweep_dirichlet_forcing(ctx[1], HSWEEP_EDGE_X1_0, G, F, 1, nullptr), HSWEEP_EINVAL,
                  "dirichlet on an absorbing edge");
    bad += expect(hsweep_dirichlet_forcing(ctx[1], HSWEEP_EDGE_X1_1, G, F, 1, nullptr), 0, "dirichlet on a layered edge");
    bad += expect(hsweep_grad_c(ctx[1], F, U, 1, G, nullptr), HSWEEP_EINVAL, "gradient with absorbing sides");
    // the remaining entry points and argument errors
    {
        int np = 0, lv = 0;
        size_t fb = 0, sb = 0;
        bad += expect(hsweep_plan_info(ctx[16], &np, &lv, &fb), 0, "plan_info");
        if (np != 512 || lv != 4 || fb == 0) { printf("plan_info: n_p %d levels %d bytes %zu\n", np, lv, fb); ++bad; }
        bad += expect(hsweep_workspace_bytes(ctx[16], 64, &fb, &sb), 0, "workspace_bytes");
        if (fb == 0 || sb == 0) { printf("workspace_bytes: %zu %zu\n", fb, sb); ++bad; }
        bad += expect(hsweep_stencil(ctx[16], F, U, 64, nullptr), 0, "stencil 64");
        std::vector<double> prof(4 * 511 + 8);
        int got = hsweep_factor_profile(ctx[16], nullptr, prof.data(), (int)prof.size());
        if (got < 0) { printf("factor_profile: %d (%s)\n", got, hsweep_last_error()); ++bad; }
        double tm[8];
        if (hsweep_timings(ctx[16], tm, 8) < 0) { printf("timings: %s\n", hsweep_last_error()); ++bad; }
        bad += expect(hsweep_apply(ctx[16], F, F, 1, nullptr), HSWEEP_EINVAL, "apply in place");
        bad += expect(hsweep_apply(ctx[16], F, U, 0, nullptr), HSWEEP_EINVAL, "apply nrhs 0");
        bad += expect(hsweep_solve(ctx[16], F, U, 1, 0.0, 10, it64.data(), r64.data(), nullptr), HSWEEP_EINVAL,
                      "solve tol 0");
        bad += expect(hsweep_dirichlet_forcing(ctx[16], 4, G, F, 1, nullptr), HSWEEP_EINVAL, "edge out of range");
        bad += expect(hsweep_apply(nullptr, F, U, 1, nullptr), HSWEEP_EINVAL, "null context");
        std::vector<hsweep_ctx*> two = {ctx[0], ctx[16]};      // leaf 16 and leaf 32 in one factor batch
        bad += expect(hsweep_factor_batch(two.data(), 2, nullptr), 0, "factor_batch of two leaf sizes");
    }
    // the strongly admissible format: complex128 and one context at a time
    {
        hsweep_opts o;
        hsweep_default_opts(&o);
        o.admissibility = HSWEEP_ADM_STRONG;
        o.precision = HSWEEP_C64;
        bad += expect(hsweep_set_opts(ctx[2], &o), HSWEEP_EINVAL, "strong in complex64");
        o.admissibility = 2;
        o.precision = HSWEEP_C128;
        bad += expect(hsweep_set_opts(ctx[2], &o), HSWEEP_EINVAL, "admissibility out of range");
        o.admissibility = HSWEEP_ADM_STRONG;
        bad += expect(hsweep_set_opts(ctx[2], &o), 0, "strong options");
        int np = 0, lv = 0;
        bad += expect(hsweep_plan_info(ctx[2], &np, &lv, nullptr), 0, "strong plan_info");
        if (np != 127 || lv != 3) { printf("strong plan: n_p %d levels %d\n", np, lv); ++bad; }
        std::vector<hsweep_ctx*> two = {ctx[2], ctx[3]};
        bad += expect(hsweep_factor_batch(two.data(), 2, nullptr), HSWEEP_EINVAL, "strong in a factor batch");
        double prof[4];
        bad += expect(hsweep_factor_profile(ctx[2], nullptr, prof, 4), HSWEEP_EINVAL, "strong factor_profile");
        bad += expect(hsweep_apply(ctx[2], F, U, 1, nullptr), HSWEEP_ESTATE, "strong apply before factor");
        bad += expect(hsweep_apply_noalloc(ctx[2], F, U, 1, nullptr), HSWEEP_EINVAL, "strong allocation-free apply");
        hsweep_ctx* one[1] = {ctx[2]};
        const void* fs[1] = {F};
        void* us[1] = {U};
        bad += expect(hsweep_solve_batch(one, 1, fs, us, 1e-6, 10, it64.data(), r64.data(), nullptr), HSWEEP_EINVAL,
                      "strong batched solve");
    }
    // a complex128 batch of two grid sizes with one leaf size (one sweep launch per step)
    std::vector<hsweep_ctx*> c2(2);
    std::vector<void*> f2(2), u2(2);
    const int n2[2] = {63, 31};
    for (int q = 0; q < 2; ++q) {
        std::vector<double> c((size_t)n2[q] * n2[q], 1.0);
        if (expect(hsweep_setup(c.data(), 20.0, 4, n2[q], &c2[q]), 0, "setup c128")) return 1;
        hsweep_opts o;
        hsweep_default_opts(&o);
        o.leaf = 8;
        if (expect(hsweep_set_opts(c2[q], &o), 0, "set_opts c128")) return 1;
        hipMalloc(&f2[q], (size_t)n2[q] * n2[q] * 16);
        hipMalloc(&u2[q], (size_t)n2[q] * n2[q] * 16);
    }
    bad += expect(hsweep_factor_batch(c2.data(), 2, nullptr), 0, "factor_batch c128");
    bad += expect(hsweep_solve_batch(c2.data(), 2, (const void* const*)f2.data(), (void* const*)u2.data(), 1e-10, 30,
                                     its.data(), res.data(), nullptr),
                  HSWEEP_ENOCONV, "solve_batch c128");
    for (auto* c : c2) hsweep_destroy(c);
    for (auto* c : ctx) hsweep_destroy(c);
    printf(bad ? "HOSTCHECK FAILED\n" : "HOSTCHECK OK\n");
    return bad ? 1 : 0;
}
