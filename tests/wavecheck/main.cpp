// Driver of the threaded check of the small dense launchers (k_dense.hip):
// reads one problem, runs the launcher, writes the results.
//
// Input: int32 op (0 QR, 1 SVD, 2 inverse), rows, cols, lda, rmax; float64
// tol; then the lda x cols complex128 matrix (column-major).
// Output: QR: Q (rows x kk), R (kk x cols); SVD: A after the call (lda x
// cols), V (cols x cols), sigma (cols float64), perm (cols int32), rank
// (int32); inverse: X (rows x rows), status (int32).
#include <stdint.h>
#include <stdio.h>
#include <vector>
#include <hip/hip_runtime.h>
#include "internal.hpp"

thread_local emu_index blockIdx, threadIdx;
thread_local dim3 blockDim, gridDim;
pthread_barrier_t wave_barrier;
unsigned long long wave_slot[1024];

static bool rd(FILE* fp, void* p, size_t b) { return fread(p, 1, b, fp) == b; }
template <typename T> static T* dev(size_t count) {
    void* p = nullptr;
    hipMalloc(&p, (count ? count : 1) * sizeof(T));
    return (T*)p;
}

int main(int argc, char** argv) {
    if (argc != 3) return 2;
    fake_poison = true;
    FILE* fp = fopen(argv[1], "rb");
    if (!fp) return 2;
    int32_t hd[5];
    double tol;
    if (!rd(fp, hd, sizeof hd) || !rd(fp, &tol, 8)) return 2;
    const int op = hd[0], p = hd[1], k = hd[2], lda = hd[3], rmax = hd[4];
    std::vector<c128> a((size_t)lda * k);
    if (!rd(fp, a.data(), a.size() * 16)) return 2;
    fclose(fp);
    c128* A = dev<c128>(a.size());
    hipMemcpy(A, a.data(), a.size() * 16, hipMemcpyHostToDevice);
    FILE* out = fopen(argv[2], "wb");
    if (op == 0) {
        const int kk = p < k ? p : k;
        c128 *W = dev<c128>((size_t)p * k), *Vh = dev<c128>((size_t)p * kk), *Q = dev<c128>((size_t)p * kk),
             *R = dev<c128>((size_t)kk * k);
        launch_small_qr(p, k, A, lda, W, Vh, Q, R, nullptr);
        fwrite(Q, 16, (size_t)p * kk, out);
        fwrite(R, 16, (size_t)kk * k, out);
    } else if (op == 1) {
        c128* V = dev<c128>((size_t)k * k);
        double* sig = dev<double>(k);
        int* perm = dev<int>(k);
        int* rank = dev<int>(1);
        launch_small_svd(p, k, A, lda, V, sig, perm, rank, tol, rmax, nullptr);
        fwrite(A, 16, a.size(), out);
        fwrite(V, 16, (size_t)k * k, out);
        fwrite(sig, 8, k, out);
        fwrite(perm, 4, k, out);
        fwrite(rank, 4, 1, out);
    } else {
        c128 *W = dev<c128>((size_t)p * (p + 1)), *X = dev<c128>((size_t)p * p);
        int* st = dev<int>(1);
        *st = 0;
        launch_small_inv(p, A, lda, W, X, st, nullptr);
        fwrite(X, 16, (size_t)p * p, out);
        fwrite(st, 4, 1, out);
    }
    fclose(out);
    return 0;
}
