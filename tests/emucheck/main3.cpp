// Driver of the emulated 3D path: reads a problem from a binary file, runs
// hsweep3_setup / set_opts / factor and then one application of the
// face-by-face sweep, a GMRES solve or the FP64 operator, and writes the
// result.
//
// Input (native byte order): int32 n, pml, leaf, rank, nrhs, mode (0 apply,
// 1 solve, 2 the FP64 operator), maxit; float64 omega, rank_tol, gmres_tol;
// then c (n^3 float64) and f (nrhs*n^3 complex128).
// Output: int32 rc, levels, iters[nrhs]; float64 relres[nrhs]; uint64 factor
// bytes; then u (nrhs*n^3 complex128).
#include <stdint.h>
#include <stdio.h>
#include <vector>
#include "hsweep.h"
#include <hip/hip_runtime.h>

static bool rd(FILE* fp, void* p, size_t b) { return fread(p, 1, b, fp) == b; }

int main(int argc, char** argv) {
    if (argc != 3) { fprintf(stderr, "usage: emu3 in.bin out.bin\n"); return 2; }
    fake_poison = true;
    FILE* fp = fopen(argv[1], "rb");
    if (!fp) return 2;
    int32_t hd[7];
    double dv[3];
    if (!rd(fp, hd, sizeof hd) || !rd(fp, dv, sizeof dv)) return 2;
    const int n = hd[0], pml = hd[1], leaf = hd[2], rank = hd[3], nrhs = hd[4], mode = hd[5], maxit = hd[6];
    const size_t N3 = (size_t)n * n * n;
    std::vector<double> c(N3), f(2 * N3 * nrhs);
    if (!rd(fp, c.data(), N3 * 8) || !rd(fp, f.data(), f.size() * 8)) return 2;
    fclose(fp);
    hsweep3_ctx* ctx = nullptr;
    int rc = hsweep3_setup(c.data(), dv[0], pml, n, &ctx);
    if (rc) { fprintf(stderr, "setup: %s\n", hsweep_last_error()); return 1; }
    hsweep_opts o;
    hsweep_default_opts(&o);
    o.leaf = leaf;
    o.rank = rank;
    o.rank_tol = dv[1];
    o.precision = HSWEEP_C128;
    o.admissibility = HSWEEP_ADM_STRONG;
    rc = hsweep3_set_opts(ctx, &o);
    if (rc) { fprintf(stderr, "set_opts: %s\n", hsweep_last_error()); return 1; }
    void *F, *U;
    hipMalloc(&F, N3 * nrhs * 16);
    hipMalloc(&U, N3 * nrhs * 16);
    hipMemcpy(F, f.data(), N3 * nrhs * 16, hipMemcpyHostToDevice);
    std::vector<int32_t> its(nrhs, 0);
    std::vector<double> res(nrhs, 0.0);
    if (mode == 2) {
        rc = hsweep3_stencil(ctx, F, U, nrhs, nullptr);
    } else {
        rc = hsweep3_factor(ctx, nullptr);
        if (rc) { fprintf(stderr, "factor: %s\n", hsweep_last_error()); return 1; }
        if (mode == 0) rc = hsweep3_apply(ctx, F, U, nrhs, nullptr);
        else rc = hsweep3_solve(ctx, F, U, nrhs, dv[2], maxit, its.data(), res.data(), nullptr);
    }
    if (rc && rc != HSWEEP_ENOCONV) { fprintf(stderr, "apply/solve: %s\n", hsweep_last_error()); return 1; }
    int32_t lv = 0;
    size_t fb = 0;
    hsweep3_plan_info(ctx, &lv, &fb);
    std::vector<double> u(2 * N3 * nrhs);
    hipMemcpy(u.data(), U, N3 * nrhs * 16, hipMemcpyDeviceToHost);
    fp = fopen(argv[2], "wb");
    if (!fp) return 2;
    int32_t head[2] = {rc, lv};
    uint64_t fb64 = fb;
    fwrite(head, 4, 2, fp);
    fwrite(its.data(), 4, nrhs, fp);
    fwrite(res.data(), 8, nrhs, fp);
    fwrite(&fb64, 8, 1, fp);
    fwrite(u.data(), 8, u.size(), fp);
    fclose(fp);
    hipFree(F);
    hipFree(U);
    hsweep3_destroy(ctx);
    return 0;
}
