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
#include "wave_ops.hpp"

namespace hsweep_sweep {

template <int G, typename T>
__device__ __forceinline__ T seg_sum(T v) { return wops::gsum_ct<G>(v); }

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
    cpx<T>* gs;    // heap-indexed node reductions, (2^(L+1) - 1) * r
    cpx<T>* zs;    // (2^L - 1) * 2r
};

// Segmented sum for level l (0-based) of a node tree whose level-1 nodes
// span C1 lanes: segments of C1 >> l lanes.
template <int C1, typename T>
__device__ __forceinline__ T seg_sum_level(T v, int l) {
    if constexpr (C1 >= 64) { if (l == 0) return seg_sum<64>(v); }
    if constexpr (C1 >= 32) { if (l == (C1 >= 64 ? 1 : 0)) return seg_sum<32>(v); }
    const int g = C1 >> l;
    if (g >= 16) return seg_sum<16>(v);
    if (g >= 8) return seg_sum<8>(v);
    if (g >= 4) return seg_sum<4>(v);
    if (g >= 2) return seg_sum<2>(v);
    return v;
}

// y = T_m x for the row owned by this thread.  Three workgroup barriers per
// call when L > 0: after the vector is published, after the node reductions,
// after the cores.  The node reductions are segmented wavefront reductions of
// the per-thread chunk sums (each node's chunks are consecutive lanes).
template <typename T, int B, int R, int L>
__device__ __forceinline__ cpx<T> apply_T(const Plan& p, const LayerRegs<T, B, R, L>& g, cpx<T> x,
                                          const SweepShared<T>& sh) {
    const int np = p.np;
    const int i = threadIdx.x;
    const bool row = i < np;
    if constexpr (L == 0) __syncthreads();   // the previous step may still read xs
    if (row) sh.xs[i] = x;
    __syncthreads();
    cpx<T> y = czero<T>();
    if (row) {
        const int t = i / B;
        const cpx<T>* xl = sh.xs + t * B;
#pragma unroll
        for (int j = 0; j < B; ++j) cfma(y, g.k[j], xl[j]);
    }
    if constexpr (L > 0) {
        constexpr int CH = Chunk<B, R>::CH, NTQ = Chunk<B, R>::NTQ;
        const int nch = np / CH;
#pragma unroll
        for (int l = 0; l < L; ++l) {
            const int lvl = l + 1;
            const int cpn = nch >> lvl;           // chunks per node of this level
#pragma unroll
            for (int tq = 0; tq < NTQ; ++tq) {
                const int e = i + tq * np;        // (column kc, chunk ch) = (e / nch, e % nch)
                cpx<T> acc = czero<T>();
                if (row) {
                    const cpx<T>* xc = sh.xs + (e % nch) * CH;
#pragma unroll
                    for (int j = 0; j < CH; ++j) cfma(acc, g.pc[l][tq * CH + j], xc[j]);
                }
                // cpn = (B << L) / CH >> lvl is a compile-time power of two
                constexpr int NCH = (B << L) / CH;
                constexpr int CPN = (NCH >> 1) > 0 ? (NCH >> 1) : 1;
                acc.re = seg_sum_level<CPN>(acc.re, l);
                acc.im = seg_sum_level<CPN>(acc.im, l);
                if (row && (e % cpn) == 0) {
                    const int idx = (e % nch) / cpn, k = e / nch;
                    sh.gs[((1 << lvl) - 1 + idx) * R + k] = acc;
                }
            }
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

// Vector inputs of one layer step, loaded one step ahead: the loads are
// issued before the current step's stores, so waiting for them never waits
// for those stores (the vector memory counter retires in order).
template <typename T>
struct StepIn {
    c128 f;            // forward: f_m
    cpx<T> c;          // forward: A_{m,m-1} diagonal entry; backward: A_{m,m+1}
    cpx<T> w;          // backward: w_m
};

// State carried between the 2n-1 layer steps of one sweep.
template <typename T>
struct SweepState {
    const c128* f;
    c128* u;
    cpx<T>* w;
    const cpx<T>* cp;
    cpx<T> carry;      // forward: w_{m-1}; backward: u_{m+1}
    StepIn<T> pre;     // inputs of the next step
};

template <typename T>
__device__ __forceinline__ StepIn<T> fetch_in(const Plan& p, int s, const SweepState<T>& st) {
    const int n = p.n, np = p.np;
    const int i = threadIdx.x;
    const bool row = i < np, real_row = i < n;
    StepIn<T> in;
    in.f = czero<double>();
    in.c = czero<T>();
    in.w = czero<T>();
    if (s < n) {
        const int m = s;
        if (real_row) in.f = st.f[(size_t)m * n + i];
        if (m > 0 && row) in.c = st.cp[(size_t)(m - 1) * np + i];
    } else if (s < 2 * n - 1) {
        const int m = 2 * n - 2 - s;
        if (row) {
            in.c = st.cp[(size_t)m * np + i];
            in.w = st.w[(size_t)m * np + i];
        }
    }
    return in;
}

// Step s of the sweep: s < n is forward layer m = s, otherwise backward
// layer m = 2n-2-s.
template <typename T, int B, int R, int L>
__device__ __forceinline__ void sweep_step(const Plan& p, int s, const LayerRegs<T, B, R, L>& g,
                                           SweepState<T>& st, const SweepShared<T>& sh) {
    const int n = p.n, np = p.np;
    const int i = threadIdx.x;
    const bool row = i < np, real_row = i < n;
    const StepIn<T> in = st.pre;
    st.pre = fetch_in<T>(p, s + 1, st);          // before this step's stores
    if (s < n) {
        const int m = s;
        cpx<T> x = ccast<T>(in.f);
        if (m > 0) x -= in.c * st.carry;
        cpx<T> y = apply_T<T, B, R, L>(p, g, x, sh);
        if (row) st.w[(size_t)m * np + i] = y;
        st.carry = y;
        if (m == n - 1 && real_row) st.u[(size_t)m * n + i] = ccast<double>(y);
    } else {
        const int m = 2 * n - 2 - s;
        const cpx<T> x = in.c * st.carry;
        cpx<T> y = apply_T<T, B, R, L>(p, g, x, sh);
        const cpx<T> um = row ? in.w - y : czero<T>();
        if (real_row) st.u[(size_t)m * n + i] = ccast<double>(um);
        st.carry = um;
    }
}

__device__ __forceinline__ int layer_of_step(int s, int n) { return s < n ? s : 2 * n - 2 - s; }

template <typename T, int B, int R, int L, int NTHR>
__global__ __launch_bounds__(NTHR) void sweep_kernel(Plan p, SweepArgs<T> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int n = p.n, np = p.np;
    const int rhs = blockIdx.x;
    const int i = threadIdx.x;
    const size_t N = (size_t)n * n;
    SweepState<T> st;
    st.f = a.f + rhs * N;
    st.u = a.u + rhs * N;
    st.w = a.w + (size_t)rhs * n * np;
    st.cp = a.cp;
    st.carry = czero<T>();
    if (a.active && !a.active[rhs]) {
        for (size_t e = i; e < N; e += blockDim.x) st.u[e] = czero<double>();
        return;
    }
    st.pre = fetch_in<T>(p, 0, st);
    SweepShared<T> sh;
    cpx<T>* base = (cpx<T>*)smem;
    sh.xs = base;
    sh.gs = sh.xs + np;
    sh.zs = sh.gs + (size_t)((1 << (L + 1)) - 1) * R;
    const int steps = 2 * n - 1;
    // Double buffering when two layers of register tiles fit the registers a
    // thread has at this block size (512 per SIMD lane shared by the waves).
    constexpr int FOOT = (B + 2 * (L > 0 ? L : 1) * R + 2 * R) * (int)(2 * sizeof(T) / 4);
    constexpr int BUDGET = 131072 / NTHR < 512 ? 131072 / NTHR : 512;
    constexpr bool DB = 2 * FOOT + 48 <= BUDGET;
    if constexpr (DB) {
        // two register sets used alternately: no copies between steps
        LayerRegs<T, B, R, L> ga, gb;
        load_layer<T, B, R, L>(p, a.fac, ga);
        for (int s = 0; s < steps; s += 2) {
            if (s + 1 < steps) load_layer<T, B, R, L>(p, a.fac + (size_t)layer_of_step(s + 1, n) * p.eLayer, gb);
            sweep_step<T, B, R, L>(p, s, ga, st, sh);
            if (s + 1 < steps) {
                if (s + 2 < steps) load_layer<T, B, R, L>(p, a.fac + (size_t)layer_of_step(s + 2, n) * p.eLayer, ga);
                sweep_step<T, B, R, L>(p, s + 1, gb, st, sh);
            }
        }
    } else {
        LayerRegs<T, B, R, L> g;
        for (int s = 0; s < steps; ++s) {
            load_layer<T, B, R, L>(p, a.fac + (size_t)layer_of_step(s, n) * p.eLayer, g);
            sweep_step<T, B, R, L>(p, s, g, st, sh);
        }
    }
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
