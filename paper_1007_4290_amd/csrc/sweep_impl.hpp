// The sweep of Alg. 2.4 (the preconditioner M), one workgroup per
// right-hand side, all 2n-1 layer steps inside one launch.
//
//   forward   x_m = f_m - A_{m,m-1} w_{m-1},  w_m = T_m x_m        (m = 1..n)
//   backward  u_n = w_n,  u_m = w_m - T_m (A_{m,m+1} u_{m+1})       (m = n-1..1)
//
// so that each T_m u_m of the paper's forward and diagonal loops is
// computed once.  T_m = blockdiag(K) - sum_nodes P X P^t is applied as
//   y = K x                                  (dense leaves)
//   g_c = P_c^t x[c]   for every non-root node c   (reductions over the node)
//   z_q = X_q [g_left; g_right]               (2r x 2r core per parent q)
//   y[c] -= P_c z_q(side of c)                (broadcast back)
// Thread i owns row i of the layer (the couplings A_{m,m+-1} are diagonal,
// so the vector updates between layers are thread-local).  Each thread
// keeps the factor data it needs for one layer step in registers:
//   its row of the dense leaf (b values), its row of P on every level
//   (L*r values), one contiguous chunk of r entries of P per level for the
//   reductions, and at most one row of a core X (2r values).
// None of it depends on the vector, so the loads of the next layer are
// issued before the barriers of the current one (double buffering): the
// memory latency of a layer step hides behind the previous step.
#pragma once
#include "internal.hpp"

namespace hsweep_sweep {

template <int B, int R> struct Chunk {
    static constexpr int CH = B < R ? B : R;   // chunk length (never longer than a leaf)
    static constexpr int NTQ = R / CH;         // reduction tasks per level and thread
};

template <typename T, int B, int R, int L>
struct LayerRegs {
    cpx<T> k[B];            // K[t][j][il], j < B
    cpx<T> pr[L > 0 ? L : 1][R];     // P[lvl][k][i]
    cpx<T> pc[L > 0 ? L : 1][R];     // NTQ chunks of CH entries of P per level (the reductions)
    cpx<T> x[2 * R];        // X[q][c][o], c < 2R (one core row per thread, if any)
};

template <typename T, int B, int R, int L>
__device__ __forceinline__ void load_layer(const Plan& p, const cpx<T>* __restrict__ lay, LayerRegs<T, B, R, L>& g) {
    const int np = p.np;
    const int i = threadIdx.x;
    if (i < np) {
        const int t = i / B, il = i % B;
        const cpx<T>* K = lay + (size_t)t * B * B + il;
#pragma unroll
        for (int j = 0; j < B; ++j) g.k[j] = K[(size_t)j * B];
        const cpx<T>* P = lay + p.eK;
        constexpr int CH = Chunk<B, R>::CH, NTQ = Chunk<B, R>::NTQ;
        const int nch = np / CH;                 // chunks of CH rows per column
#pragma unroll
        for (int l = 0; l < L; ++l) {
            {
                const cpx<T>* Pl = P + (size_t)l * R * np;
#pragma unroll
                for (int k = 0; k < R; ++k) g.pr[l][k] = Pl[(size_t)k * np + i];
#pragma unroll
                for (int tq = 0; tq < NTQ; ++tq) {
                    const int e = i + tq * np;   // task: (column kc, chunk ch) of this level
                    const int kc = e / nch, ch = e % nch;
                    const cpx<T>* Pc = Pl + (size_t)kc * np + ch * CH;
#pragma unroll
                    for (int j = 0; j < CH; ++j) g.pc[l][tq * CH + j] = Pc[j];
                }
            }
        }
    }
    const int npar = (1 << L) - 1;
    if (L > 0 && i < npar * 2 * R) {
        const int q = i / (2 * R), o = i % (2 * R);
        const cpx<T>* Xq = lay + p.eK + p.eP + (size_t)q * 4 * R * R + o;
#pragma unroll
        for (int c = 0; c < 2 * R; ++c) g.x[c] = Xq[(size_t)c * 2 * R];
    }
}

template <typename T>
struct SweepShared {
    cpx<T>* xs;    // np
    cpx<T>* part;  // L * r * np / CH  (per level: r columns x np/CH chunks)
    cpx<T>* gs;    // heap-indexed node reductions, (2^(L+1) - 1) * r
    cpx<T>* zs;    // (2^L - 1) * 2r
};

template <typename T, int B, int R, int L>
__device__ __forceinline__ cpx<T> apply_T(const Plan& p, const LayerRegs<T, B, R, L>& g, cpx<T> x,
                                          const SweepShared<T>& sh) {
    const int np = p.np;
    const int i = threadIdx.x;
    const bool row = i < np;
    __syncthreads();   // the previous step may still read xs / zs
    if (row) sh.xs[i] = x;
    __syncthreads();
    cpx<T> y = czero<T>();
    if (row) {
        const int t = i / B;
        const cpx<T>* xl = sh.xs + t * B;
#pragma unroll
        for (int j = 0; j < B; ++j) cfma(y, g.k[j], xl[j]);
        constexpr int CH = Chunk<B, R>::CH, NTQ = Chunk<B, R>::NTQ;
        const int nch = np / CH;
#pragma unroll
        for (int l = 0; l < L; ++l) {
            {
#pragma unroll
                for (int tq = 0; tq < NTQ; ++tq) {
                    const int e = i + tq * np;
                    const cpx<T>* xc = sh.xs + (e % nch) * CH;
                    cpx<T> acc = czero<T>();
#pragma unroll
                    for (int j = 0; j < CH; ++j) cfma(acc, g.pc[l][tq * CH + j], xc[j]);
                    sh.part[(size_t)l * R * nch + e] = acc;   // entry (kc * nch + ch) of level l
                }
            }
        }
    }
    if constexpr (L == 0) return y;
    __syncthreads();
    // node sums g_c for the nodes of levels 1..L (heap ids 1 .. 2^(L+1)-2)
    const int nch = np / Chunk<B, R>::CH;
    const int nnode = (1 << (L + 1)) - 2;
    for (int e = i; e < nnode * R; e += blockDim.x) {
        const int h = 1 + e / R, k = e % R;
        const int lvl = 31 - __clz(h + 1);
        const int idx = h - ((1 << lvl) - 1);
        const int cpn = nch >> lvl;   // chunks per node
        const cpx<T>* pp = sh.part + (size_t)(lvl - 1) * R * nch + k * nch + idx * cpn;
        cpx<T> acc = czero<T>();
        for (int q = 0; q < cpn; ++q) acc += pp[q];
        sh.gs[h * R + k] = acc;
    }
    __syncthreads();
    const int npar = (1 << L) - 1;
    if (i < npar * 2 * R) {
        const int q = i / (2 * R);
        const cpx<T>* gq = sh.gs + (size_t)(2 * q + 1) * R;   // children 2q+1, 2q+2 are contiguous
        cpx<T> acc = czero<T>();
#pragma unroll
        for (int c = 0; c < 2 * R; ++c) cfma(acc, g.x[c], gq[c]);
        sh.zs[i] = acc;
    }
    __syncthreads();
    if (row) {
        const int lnp = 31 - __clz(np);
#pragma unroll
        for (int l = 0; l < L; ++l) {
            {
                const int lvl = l + 1;
                const int c = i >> (lnp - lvl);   // node index at lvl
                const int q = (1 << (lvl - 1)) - 1 + (c >> 1);
                const cpx<T>* z = sh.zs + (size_t)q * 2 * R + (c & 1) * R;
                cpx<T> acc = czero<T>();
#pragma unroll
                for (int k = 0; k < R; ++k) cfma(acc, g.pr[l][k], z[k]);
                y -= acc;
            }
        }
    }
    return y;
}

template <typename T, int B, int R, int L, int NTHR>
__global__ __launch_bounds__(NTHR) void sweep_kernel(Plan p, SweepArgs<T> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int n = p.n, np = p.np;
    const int rhs = blockIdx.x;
    const int i = threadIdx.x;
    const size_t N = (size_t)n * n;
    const c128* f = a.f + rhs * N;
    c128* u = a.u + rhs * N;
    if (a.active && !a.active[rhs]) {
        for (size_t e = i; e < N; e += blockDim.x) u[e] = czero<double>();
        return;
    }
    SweepShared<T> sh;
    cpx<T>* base = (cpx<T>*)smem;
    sh.xs = base;
    sh.part = sh.xs + np;
    sh.gs = sh.part + (size_t)L * R * (np / Chunk<B, R>::CH);
    sh.zs = sh.gs + (size_t)((1 << (L + 1)) - 1) * R;
    cpx<T>* w = a.w + (size_t)rhs * n * np;
    const bool row = i < np;
    const bool real_row = i < n;
    // Double buffering when two layers of register tiles fit the registers a
    // thread has at this block size (512 per SIMD lane shared by the waves).
    constexpr int FOOT = (B + 2 * (L > 0 ? L : 1) * R + 2 * R) * (int)(2 * sizeof(T) / 4);
    constexpr int BUDGET = 131072 / NTHR < 512 ? 131072 / NTHR : 512;
    constexpr bool DB = 2 * FOOT + 48 <= BUDGET;
    LayerRegs<T, B, R, L> cur, nxt;
    if constexpr (DB) load_layer<T, B, R, L>(p, a.fac, cur);
    cpx<T> prev = czero<T>();
    for (int m = 0; m < n; ++m) {
        if constexpr (DB) {
            // next layer of the forward loop, or the first layer of the backward loop
            const int mn = (m + 1 < n) ? m + 1 : n - 2;
            load_layer<T, B, R, L>(p, a.fac + (size_t)mn * p.eLayer, nxt);
        } else {
            load_layer<T, B, R, L>(p, a.fac + (size_t)m * p.eLayer, cur);
        }
        cpx<T> x = czero<T>();
        if (real_row) x = ccast<T>(f[(size_t)m * n + i]);
        if (m > 0 && row) x -= a.cp[(size_t)(m - 1) * np + i] * prev;
        cpx<T> y = apply_T<T, B, R, L>(p, cur, x, sh);
        if (row) w[(size_t)m * np + i] = y;
        prev = y;
        if constexpr (DB) cur = nxt;
    }
    cpx<T> next = prev;
    if (real_row) u[(size_t)(n - 1) * n + i] = ccast<double>(next);
    for (int m = n - 2; m >= 0; --m) {
        if constexpr (DB) {
            if (m >= 1) load_layer<T, B, R, L>(p, a.fac + (size_t)(m - 1) * p.eLayer, nxt);
        } else {
            load_layer<T, B, R, L>(p, a.fac + (size_t)m * p.eLayer, cur);
        }
        cpx<T> x = czero<T>();
        if (row) x = a.cp[(size_t)m * np + i] * next;
        cpx<T> y = apply_T<T, B, R, L>(p, cur, x, sh);
        cpx<T> um = czero<T>();
        if (row) um = w[(size_t)m * np + i] - y;
        if (real_row) u[(size_t)m * n + i] = ccast<double>(um);
        next = um;
        if constexpr (DB) cur = nxt;
    }
}

template <typename T, int B, int R>
void launch_one(const Plan& p, const SweepArgs<T>& a, size_t lds, int threads, hipStream_t s) {
    static bool attr = false;
    if (!attr) {
        hipFuncAttributes fa;
        if (hipFuncGetAttributes(&fa, (const void*)sweep_kernel<T, B, R>) == hipSuccess)
            (void)hipFuncSetAttribute((const void*)sweep_kernel<T, B, R>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize,
                                      160 * 1024 - (int)fa.sharedSizeBytes);
        (void)hipGetLastError();
        attr = true;
    }
    hipLaunchKernelGGL((sweep_kernel<T, B, R>), dim3(a.nrhs), dim3(threads), lds, s, p, a);
}


// Launch one instantiation; the block has max(64, n_p, core rows) threads,
// rounded to whole wavefronts (NTHR is its upper bound).
template <typename T, int B, int R, int L, int NTHR>
void launch_inst(const Plan& p, const SweepArgs<T>& a, size_t lds, int threads, hipStream_t s) {
    static bool attr = false;
    if (!attr) {
        hipFuncAttributes fa;
        if (hipFuncGetAttributes(&fa, (const void*)sweep_kernel<T, B, R, L, NTHR>) == hipSuccess)
            (void)hipFuncSetAttribute((const void*)sweep_kernel<T, B, R, L, NTHR>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize,
                                      160 * 1024 - (int)fa.sharedSizeBytes);
        (void)hipGetLastError();
        attr = true;
    }
    hipLaunchKernelGGL((sweep_kernel<T, B, R, L, NTHR>), dim3(a.nrhs), dim3(threads), lds, s, p, a);
}

}  // namespace hsweep_sweep

// (leaf b, rank r, levels L) combinations with a compiled sweep.  The block
// size bound is b * 2^L rounded up to a wavefront.
#define HSWEEP_SWEEP_LIST_A(X)                                                        \
    X(4, 2, 0) X(8, 2, 0) X(16, 2, 0) X(32, 2, 0) X(64, 2, 0)                            \
    X(4, 8, 1) X(4, 8, 2) X(4, 16, 1) X(4, 16, 2) X(4, 16, 3)                            \
    X(8, 8, 1) X(8, 8, 2) X(8, 8, 3) X(8, 8, 4) X(8, 16, 2) X(8, 16, 3)
#define HSWEEP_SWEEP_LIST_B(X)                                                        \
    X(16, 8, 1) X(16, 8, 2) X(16, 8, 3) X(16, 8, 4) X(16, 8, 5) X(16, 8, 6)              \
    X(64, 8, 1) X(64, 8, 2) X(64, 8, 3) X(64, 8, 4)
#define HSWEEP_SWEEP_LIST_C(X)                                                        \
    X(32, 8, 1) X(32, 8, 2) X(32, 8, 3) X(32, 8, 4) X(32, 8, 5)                          \
    X(16, 16, 2) X(16, 16, 3) X(16, 16, 4)

#define HSWEEP_MAX2(a, b) ((a) > (b) ? (a) : (b))
#define HSWEEP_NTHR(BB, RR, LL) \
    ((HSWEEP_MAX2(HSWEEP_MAX2(64, (BB) << (LL)), ((1 << (LL)) - 1) * 2 * (RR)) + 63) / 64 * 64)

#define HSWEEP_SWEEP_NAME(TT, BB, RR, LL) sweep_launch_##TT##_##BB##_##RR##_##LL
#define HSWEEP_SWEEP_SIG(TT, CT, BB, RR, LL) \
    void HSWEEP_SWEEP_NAME(TT, BB, RR, LL)(const Plan& p, const SweepArgs<CT>& a, size_t lds, int th, hipStream_t s)

#define HSWEEP_SWEEP_DEFINE(BB, RR, LL)                                                             \
    HSWEEP_SWEEP_SIG(f, float, BB, RR, LL) {                                                        \
        hsweep_sweep::launch_inst<float, BB, RR, LL, HSWEEP_NTHR(BB, RR, LL)>(p, a, lds, th, s);    \
    }                                                                                               \
    HSWEEP_SWEEP_SIG(d, double, BB, RR, LL) {                                                       \
        hsweep_sweep::launch_inst<double, BB, RR, LL, HSWEEP_NTHR(BB, RR, LL)>(p, a, lds, th, s);   \
    }
