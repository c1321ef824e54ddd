// FP64 complex vector kernels of the flexible GMRES driver: batched inner
// products for classical Gram-Schmidt with reorthogonalization, batched
// axpy, scaling and the final combination x += Z y, each over a set of
// systems of possibly different lengths (several right-hand sides of one
// grid, or several grids) in one launch.  Reductions are
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

// Vectors are concatenations of S systems: system k occupies entries
// [off[k], off[k+1]) of every vector, and a set of vectors X_0, X_1, ...
// is stored with stride ld.

// grid (nblk, S); partial[(blk * S + k) * nv + j] = block partial of sum conj(V_j) w over system k
__global__ __launch_bounds__(kDotThreads) void multi_dot_kernel(const c128* __restrict__ V, int nv, size_t ld,
                                                              const c128* __restrict__ w,
                                                              const size_t* __restrict__ off, int S,
                                                              c128* __restrict__ partial) {
    __shared__ c128 red[kDotThreads / 64][kMaxDots];
    const int blk = blockIdx.x, k = blockIdx.y, nblk = gridDim.x;
    const size_t base = off[k], len = off[k + 1] - base;
    const size_t chunk = (len + nblk - 1) / nblk;
    const size_t lo = base + blk * chunk, hi = (size_t)blk * chunk + chunk < len ? lo + chunk : base + len;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int j0 = 0; j0 < nv; j0 += kMaxDots) {
        const int cnt = nv - j0 < kMaxDots ? nv - j0 : kMaxDots;
        for (int jj = 0; jj < cnt; ++jj) {
            const c128* vj = V + (size_t)(j0 + jj) * ld;
            c128 acc = czero<double>();
            for (size_t i = lo + threadIdx.x; i < hi; i += kDotThreads) cfma_conj(acc, vj[i], w[i]);
            acc = warp_sum(acc);
            if (lane == 0) red[wv][jj] = acc;
        }
        __syncthreads();
        for (int jj = threadIdx.x; jj < cnt; jj += kDotThreads) {
            c128 sacc = czero<double>();
            for (int q = 0; q < kDotThreads / 64; ++q) sacc += red[q][jj];
            partial[((size_t)blk * S + k) * nv + j0 + jj] = sacc;
        }
        __syncthreads();
    }
}

__global__ void dot_finish_kernel(const c128* __restrict__ partial, int nblk, int nv, int S, c128* __restrict__ out) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nv * S) return;
    int k = t / nv, j = t % nv;
    c128 sacc = czero<double>();
    for (int b = 0; b < nblk; ++b) sacc += partial[((size_t)b * S + k) * nv + j];
    out[(size_t)j * S + k] = sacc;
}

// grid (ceil(maxlen / 256), S): w_k -= sum_j h[j*S + k] V_j over system k
__global__ void multi_axpy_kernel(const c128* __restrict__ V, int nv, size_t ld, const c128* __restrict__ h,
                                  c128* __restrict__ w, const size_t* __restrict__ off, int S) {
    const int k = blockIdx.y;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t base = off[k];
    if (i >= off[k + 1] - base) return;
    const size_t e = base + i;
    c128 acc = w[e];
    for (int j = 0; j < nv; ++j) acc -= h[(size_t)j * S + k] * V[(size_t)j * ld + e];
    w[e] = acc;
}

__global__ void scale_kernel(const c128* __restrict__ w, const double* __restrict__ sc, c128* __restrict__ out,
                             const size_t* __restrict__ off) {
    const int k = blockIdx.y;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t base = off[k];
    if (i >= off[k + 1] - base) return;
    const double a = sc[k];
    out[base + i] = a == 0.0 ? czero<double>() : a * w[base + i];
}

__global__ void combine_kernel(const c128* __restrict__ Z, int nz, size_t ld, const c128* __restrict__ y,
                               c128* __restrict__ x, const size_t* __restrict__ off, int S) {
    const int k = blockIdx.y;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t base = off[k];
    if (i >= off[k + 1] - base) return;
    const size_t e = base + i;
    c128 acc = x[e];
    for (int j = 0; j < nz; ++j) cfma(acc, y[(size_t)j * S + k], Z[(size_t)j * ld + e]);
    x[e] = acc;
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

void launch_multi_dot(const c128* V, int nv, size_t ld, const c128* w, const size_t* off, int S, c128* partial,
                      c128* out, int nblk, hipStream_t s) {
    hipLaunchKernelGGL(multi_dot_kernel, dim3(nblk, S), dim3(kDotThreads), 0, s, V, nv, ld, w, off, S, partial);
    int tot = nv * S;
    hipLaunchKernelGGL(dot_finish_kernel, dim3((tot + 255) / 256), dim3(256), 0, s, partial, nblk, nv, S, out);
}

void launch_multi_axpy(const c128* V, int nv, size_t ld, const c128* h, c128* w, const size_t* off, int S,
                       size_t maxlen, hipStream_t s) {
    hipLaunchKernelGGL(multi_axpy_kernel, dim3((unsigned)((maxlen + 255) / 256), S), dim3(256), 0, s, V, nv, ld, h, w,
                       off, S);
}

void launch_scale(const c128* w, const double* scale, c128* out, const size_t* off, int S, size_t maxlen,
                  hipStream_t s) {
    hipLaunchKernelGGL(scale_kernel, dim3((unsigned)((maxlen + 255) / 256), S), dim3(256), 0, s, w, scale, out, off);
}

void launch_combine(const c128* Z, int nz, size_t ld, const c128* y, c128* x, const size_t* off, int S, size_t maxlen,
                    hipStream_t s) {
    hipLaunchKernelGGL(combine_kernel, dim3((unsigned)((maxlen + 255) / 256), S), dim3(256), 0, s, Z, nz, ld, y, x,
                       off, S);
}
