// FP64 complex vector kernels of the flexible GMRES driver: batched inner
// products for classical Gram-Schmidt with reorthogonalization, batched
// axpy, scaling and the final combination x += Z y.  Reductions are
// deterministic: per-block partial sums are written out and summed in a
// fixed order by a second kernel (no floating-point atomics).
#include "internal.hpp"

namespace {

constexpr int kDotThreads = 256;
constexpr int kMaxDots = 64;     // inner products per pass (restart + 1 <= kMaxDots handled in chunks)

__device__ __forceinline__ c128 warp_sum(c128 v) {
    for (int off = 32; off > 0; off >>= 1) {
        v.re += __shfl_xor(v.re, off, 64);
        v.im += __shfl_xor(v.im, off, 64);
    }
    return v;
}

// grid (nblk, nrhs); partial[(blk * nrhs + k) * nv + j]
__global__ __launch_bounds__(kDotThreads) void multi_dot_kernel(const c128* __restrict__ V, int nv,
                                                              const c128* __restrict__ w, int nrhs, size_t N,
                                                              c128* __restrict__ partial) {
    __shared__ c128 red[kDotThreads / 64][kMaxDots];
    int blk = blockIdx.x, k = blockIdx.y, nblk = gridDim.x;
    size_t chunk = (N + nblk - 1) / nblk;
    size_t lo = blk * chunk, hi = lo + chunk < N ? lo + chunk : N;
    const c128* wk = w + (size_t)k * N;
    int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int j0 = 0; j0 < nv; j0 += kMaxDots) {
        int cnt = nv - j0 < kMaxDots ? nv - j0 : kMaxDots;
        for (int jj = 0; jj < cnt; ++jj) {
            const c128* vj = V + ((size_t)(j0 + jj) * nrhs + k) * N;
            c128 acc = czero<double>();
            for (size_t i = lo + threadIdx.x; i < hi; i += kDotThreads) cfma_conj(acc, vj[i], wk[i]);
            acc = warp_sum(acc);
            if (lane == 0) red[wv][jj] = acc;
        }
        __syncthreads();
        for (int jj = threadIdx.x; jj < cnt; jj += kDotThreads) {
            c128 s = czero<double>();
            for (int q = 0; q < kDotThreads / 64; ++q) s += red[q][jj];
            partial[((size_t)blk * nrhs + k) * nv + j0 + jj] = s;
        }
        __syncthreads();
    }
}

__global__ void dot_finish_kernel(const c128* __restrict__ partial, int nblk, int nv, int nrhs, c128* __restrict__ out) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nv * nrhs) return;
    int k = t / nv, j = t % nv;
    c128 s = czero<double>();
    for (int b = 0; b < nblk; ++b) s += partial[((size_t)b * nrhs + k) * nv + j];
    out[(size_t)j * nrhs + k] = s;
}

__global__ void multi_axpy_kernel(const c128* __restrict__ V, int nv, const c128* __restrict__ h,
                                  c128* __restrict__ w, int nrhs, size_t N) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    int k = blockIdx.y;
    if (i >= N) return;
    c128 acc = w[(size_t)k * N + i];
    for (int j = 0; j < nv; ++j) {
        c128 c = h[(size_t)j * nrhs + k];
        c128 v = V[((size_t)j * nrhs + k) * N + i];
        acc -= c * v;
    }
    w[(size_t)k * N + i] = acc;
}

__global__ void scale_kernel(const c128* __restrict__ w, const double* __restrict__ sc, c128* __restrict__ out,
                             size_t N) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    int k = blockIdx.y;
    if (i >= N) return;
    double s = sc[k];
    out[(size_t)k * N + i] = s == 0.0 ? czero<double>() : s * w[(size_t)k * N + i];
}

__global__ void combine_kernel(const c128* __restrict__ Z, int nz, const c128* __restrict__ y,
                               c128* __restrict__ x, int nrhs, size_t N) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    int k = blockIdx.y;
    if (i >= N) return;
    c128 acc = x[(size_t)k * N + i];
    for (int j = 0; j < nz; ++j) cfma(acc, y[(size_t)j * nrhs + k], Z[((size_t)j * nrhs + k) * N + i]);
    x[(size_t)k * N + i] = acc;
}

// y = conj(x) over n entries (x and y may be the same array).
__global__ void conj_kernel(const c128* __restrict__ x, c128* __restrict__ y, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    y[i] = conj(x[i]);
}

}  // namespace

void launch_conj(const c128* x, c128* y, size_t n, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(conj_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, y, n);
}

int krylov_dot_blocks(size_t N) {
    size_t b = (N + 8191) / 8192;
    if (b < 1) b = 1;
    if (b > 256) b = 256;
    return (int)b;
}

void launch_multi_dot(const c128* V, int nv, const c128* w, int nrhs, size_t N, c128* partial, c128* out,
                      int nblk, hipStream_t s) {
    hipLaunchKernelGGL(multi_dot_kernel, dim3(nblk, nrhs), dim3(kDotThreads), 0, s, V, nv, w, nrhs, N, partial);
    int tot = nv * nrhs;
    hipLaunchKernelGGL(dot_finish_kernel, dim3((tot + 255) / 256), dim3(256), 0, s, partial, nblk, nv, nrhs, out);
}

void launch_multi_axpy(const c128* V, int nv, const c128* h, c128* w, int nrhs, size_t N, hipStream_t s) {
    hipLaunchKernelGGL(multi_axpy_kernel, dim3((unsigned)((N + 255) / 256), nrhs), dim3(256), 0, s, V, nv, h, w, nrhs, N);
}

void launch_scale(const c128* w, const double* scale, c128* out, int nrhs, size_t N, hipStream_t s) {
    hipLaunchKernelGGL(scale_kernel, dim3((unsigned)((N + 255) / 256), nrhs), dim3(256), 0, s, w, scale, out, N);
}

void launch_combine(const c128* Z, int nz, const c128* y, c128* x, int nrhs, size_t N, hipStream_t s) {
    hipLaunchKernelGGL(combine_kernel, dim3((unsigned)((N + 255) / 256), nrhs), dim3(256), 0, s, Z, nz, y, x, nrhs, N);
}
