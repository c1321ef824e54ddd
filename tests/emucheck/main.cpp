// Driver of the emulated strong-format path: reads a problem from a binary
// file, runs hsweep_setup / set_opts (strong admissibility, complex128) /
// factor and then either one application of the preconditioner or a GMRES
// solve, and writes the result.
//
// Input (native byte order): int32 n, pml, leaf, rank, dir, nrhs, mode
// (0 apply, 1 solve, 2 the FP64 operator), maxit, sides[4]; float64 omega, rank_tol, gmres_tol;
// then c (n*n float64) and f (nrhs*n*n complex128).
// Output: int32 rc, plan n_p, levels, iters[nrhs]; float64 relres[nrhs];
// uint64 factor bytes; then u (nrhs*n*n complex128).
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <vector>
#include "hsweep.h"
#include <hip/hip_runtime.h>

static bool rd(FILE* fp, void* p, size_t b) { return fread(p, 1, b, fp) == b; }

int main(int argc, char** argv) {
    if (argc != 3) { fprintf(stderr, "usage: emu in.bin out.bin\n"); return 2; }
    fake_poison = true;
    FILE* fp = fopen(argv[1], "rb");
    if (!fp) return 2;
    int32_t hd[12];
    double dv[3];
    if (!rd(fp, hd, sizeof hd) || !rd(fp, dv, sizeof dv)) return 2;
    const int n = hd[0], pml = hd[1], leaf = hd[2], rank = hd[3], dir = hd[4], nrhs = hd[5], mode = hd[6], maxit = hd[7];
    const size_t N = (size_t)n * n;
    std::vector<double> c(N);
    std::vector<double> f(2 * N * nrhs);
    if (!rd(fp, c.data(), N * 8) || !rd(fp, f.data(), f.size() * 8)) return 2;
    fclose(fp);
    hsweep_ctx* ctx = nullptr;
    int rc = hsweep_setup(c.data(), dv[0], pml, n, &ctx);
    if (rc) { fprintf(stderr, "setup: %s\n", hsweep_last_error()); return 1; }
    hsweep_opts o;
    hsweep_default_opts(&o);
    o.leaf = leaf;
    o.rank = rank;
    o.rank_tol = dv[1];
    o.precision = HSWEEP_C128;
    o.direction = dir;
    o.admissibility = HSWEEP_ADM_STRONG;
    for (int k = 0; k < 4; ++k) o.pml_sides[k] = hd[8 + k];
    rc = hsweep_set_opts(ctx, &o);
    if (rc) { fprintf(stderr, "set_opts: %s\n", hsweep_last_error()); return 1; }
    rc = hsweep_factor(ctx, nullptr);
    if (rc) { fprintf(stderr, "factor: %s\n", hsweep_last_error()); return 1; }
    void *F, *U;
    hipMalloc(&F, N * nrhs * 16);
    hipMalloc(&U, N * nrhs * 16);
    hipMemcpy(F, f.data(), N * nrhs * 16, hipMemcpyHostToDevice);
    std::vector<int32_t> its(nrhs, 0);
    std::vector<double> res(nrhs, 0.0);
    if (mode == 0) rc = hsweep_apply(ctx, F, U, nrhs, nullptr);
    else if (mode == 1) rc = hsweep_solve(ctx, F, U, nrhs, dv[2], maxit, its.data(), res.data(), nullptr);
    else rc = hsweep_stencil(ctx, F, U, nrhs, nullptr);
    if (rc && rc != HSWEEP_ENOCONV) { fprintf(stderr, "apply/solve: %s\n", hsweep_last_error()); return 1; }
    int32_t np = 0, lv = 0;
    size_t fb = 0;
    hsweep_plan_info(ctx, &np, &lv, &fb);
    std::vector<double> u(2 * N * nrhs);
    hipMemcpy(u.data(), U, N * nrhs * 16, hipMemcpyDeviceToHost);
    fp = fopen(argv[2], "wb");
    if (!fp) return 2;
    int32_t head[3] = {rc, np, lv};
    uint64_t fb64 = fb;
    fwrite(head, 4, 3, fp);
    fwrite(its.data(), 4, nrhs, fp);
    fwrite(res.data(), 8, nrhs, fp);
    fwrite(&fb64, 8, 1, fp);
    fwrite(u.data(), 8, u.size(), fp);
    fclose(fp);
    hipFree(F);
    hipFree(U);
    hsweep_destroy(ctx);
    return 0;
}
