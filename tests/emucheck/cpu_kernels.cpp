// CPU versions of the launchers the emulated strong-format path needs
// besides the ones compiled from the library (coefficients, strong format):
// the FP64 Krylov vector operations in plain loops, and stand-ins for the
// weak format's factorization and sweep, which this check never calls.
#include <stdio.h>
#include <stdlib.h>
#include "internal.hpp"

static void never(const char* what) {
    fprintf(stderr, "weak-format launcher %s called in the strong-format check\n", what);
    abort();
}
template <typename T> int launch_factor_layer(const InstDesc<T>*, const Plan*, int, int, hipStream_t, hipEvent_t) { never("factor"); return -1; }
template int launch_factor_layer<float>(const InstDesc<float>*, const Plan*, int, int, hipStream_t, hipEvent_t);
template int launch_factor_layer<double>(const InstDesc<double>*, const Plan*, int, int, hipStream_t, hipEvent_t);
template <typename T> void factor_kernels_init() {}
template void factor_kernels_init<float>();
template void factor_kernels_init<double>();
size_t factor_lds_bytes(const Plan&, size_t) { return 0; }
bool factor_supported(const Plan&) { return true; }
size_t sweep_lds_bytes(const Plan&, size_t, int) { return 0; }
bool sweep_supported(const Plan&) { return true; }
bool sweep_group_supported(const Plan&) { return false; }
template <typename T> int launch_sweep(const Plan&, SweepArgs<T>, int, hipStream_t) { never("sweep"); return -1; }
template int launch_sweep<float>(const Plan&, SweepArgs<float>, int, hipStream_t);
template int launch_sweep<double>(const Plan&, SweepArgs<double>, int, hipStream_t);
template <typename T>
int launch_sweep_multi_col(const Plan*, int, const SweepInst<T>*, const int*, int, int, int, int, hipStream_t) {
    never("multi sweep");
    return -1;
}
template int launch_sweep_multi_col<float>(const Plan*, int, const SweepInst<float>*, const int*, int, int, int, int, hipStream_t);
template int launch_sweep_multi_col<double>(const Plan*, int, const SweepInst<double>*, const int*, int, int, int, int, hipStream_t);

int krylov_dot_blocks(size_t) { return 1; }
void launch_conj(const c128* x, c128* y, size_t n, hipStream_t) {
    for (size_t i = 0; i < n; ++i) y[i] = conj(x[i]);
}
void launch_multi_dot(const c128* V, int nv, size_t ld, const c128* w, const size_t* off, int S, c128*, c128* out, int,
                      hipStream_t) {
    for (int j = 0; j < nv; ++j)
        for (int k = 0; k < S; ++k) {
            c128 acc = czero<double>();
            for (size_t i = off[k]; i < off[k + 1]; ++i) cfma_conj(acc, V[j * ld + i], w[i]);
            out[(size_t)j * S + k] = acc;
        }
}
void launch_multi_axpy(const c128* V, int nv, size_t ld, const c128* h, c128* w, const size_t* off, int S, size_t,
                       hipStream_t) {
    for (int k = 0; k < S; ++k)
        for (size_t i = off[k]; i < off[k + 1]; ++i) {
            c128 acc = w[i];
            for (int j = 0; j < nv; ++j) acc -= h[(size_t)j * S + k] * V[j * ld + i];
            w[i] = acc;
        }
}
void launch_scale(const c128* w, const double* sc, c128* out, const size_t* off, int S, size_t, hipStream_t) {
    for (int k = 0; k < S; ++k)
        for (size_t i = off[k]; i < off[k + 1]; ++i) out[i] = sc[k] == 0.0 ? czero<double>() : sc[k] * w[i];
}
void launch_combine(const c128* Z, int nz, size_t ld, const c128* y, c128* x, const size_t* off, int S, size_t,
                    hipStream_t) {
    for (int k = 0; k < S; ++k)
        for (size_t i = off[k]; i < off[k + 1]; ++i)
            for (int j = 0; j < nz; ++j) x[i] += y[(size_t)j * S + k] * Z[j * ld + i];
}
