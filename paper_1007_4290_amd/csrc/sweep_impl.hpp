// The sweep of Alg. 2.4 (the preconditioner M): all 2n-1 layer steps of one
// application inside one launch.  A workgroup runs the whole sweep for one
// instance and a group of G right-hand sides, so every layer's factor data
// that the workgroup loads serves G right-hand sides.
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
// Thread i owns row i of the layer for all G right-hand sides (the
// couplings A_{m,m+-1} are diagonal, so the vector updates between layers
// are thread-local).  Its factor data for a layer step: its row of the dense
// leaf (b values), its row of P on every level (L*r values), one chunk of r
// entries of P per level for the reductions, and at most one row of a core X
// (2r values).
//
// Three ways to hold that data, chosen at compile time from the register
// budget a thread has at this block size:
//   double buffered  two layers in registers, the next one loaded during the
//                    current step (small layers);
//   resident         one layer in registers, loaded at the start of a step;
//   phased           each phase's data loaded just before that phase, so no
//                    more than one phase's tiles are live (wide layers).
//
// G = 4 in complex64: the leaf, core and broadcast products run on the
// matrix cores.  Each is a row-times-block product y[i, g] = sum_k a[i, k]
// v[k, g], lane i holding its own matrix row a[i, :] and v in LDS.  With
// v_mfma_f32_4x4x1f32 (16 independent 4x4x1 blocks) a block of 4 lanes (4
// consecutive rows that share v) takes B = a[i, k] from each lane and A =
// the four real components (re v[k, 2p], im v[k, 2p], re v[k, 2p+1],
// im v[k, 2p+1]) of a pair p of right-hand sides, one per lane, and
// accumulates their products in the lane that owns the row.  Two products
// (real and imaginary part of a[i, k]) per pair and k give the complex
// results; FP32 accumulation.
#pragma once
#include "internal.hpp"
#include "wave_ops.hpp"

namespace hsweep_sweep {

typedef float v4f __attribute__((ext_vector_type(4)));

template <int B, int R> struct Chunk {
    static constexpr int CH = B < R ? B : R;   // chunk length (never longer than a leaf)
    static constexpr int NTQ = R / CH;         // reduction tasks per level and thread
};

template <typename T, int B, int R, int LM>
struct LayerRegs {
    cpx<T> k[B];                         // K[t][j][il], j < B
    cpx<T> pr[LM > 0 ? LM : 1][R];       // P[lvl][k][i]
    cpx<T> pc[LM > 0 ? LM : 1][R];       // NTQ chunks of CH entries of P per level
    cpx<T> x[2 * R];                     // X[q][c][o], c < 2R (one core row per thread, if any)
};

// Runtime geometry of the instance a workgroup works on.
struct Geo {
    int n, np, L, lnp, nch;   // grid, padded width, levels, log2(np), P chunks per column
    int dir;                  // sweep direction
    size_t eK, eP;
};

// Index in the natural grid order of position i (< n) of layer m in the
// frame of the sweep direction: rows upward or downward, columns rightward
// or leftward.
__device__ __forceinline__ size_t grid_index(const Geo& ge, int i, int m) {
    const int n = ge.n;
    if (ge.dir == 0) return (size_t)m * n + i;
    if (ge.dir == 1) return (size_t)(n - 1 - m) * n + i;
    if (ge.dir == 2) return (size_t)i * n + m;
    return (size_t)i * n + (n - 1 - m);
}

template <typename T, int B>
__device__ __forceinline__ void load_K(const Geo& ge, const cpx<T>* __restrict__ lay, cpx<T> (&k)[B]) {
    const int i = threadIdx.x;
    if (i < ge.np) {
        const cpx<T>* K = lay + (size_t)(i / B) * B * B + (i % B);
#pragma unroll
        for (int j = 0; j < B; ++j) k[j] = K[(size_t)j * B];
    } else {
#pragma unroll
        for (int j = 0; j < B; ++j) k[j] = czero<T>();
    }
}

template <typename T, int B, int R, int LM>
__device__ __forceinline__ void load_pc(const Geo& ge, const cpx<T>* __restrict__ lay, cpx<T> (&pc)[LM > 0 ? LM : 1][R]) {
    const int i = threadIdx.x, np = ge.np;
    constexpr int CH = Chunk<B, R>::CH, NTQ = Chunk<B, R>::NTQ;
    const cpx<T>* P = lay + ge.eK;
#pragma unroll
    for (int l = 0; l < LM; ++l) {
#pragma unroll
        for (int j = 0; j < R; ++j) pc[l][j] = czero<T>();
        if (l < ge.L && i < np) {
            const cpx<T>* Pl = P + (size_t)l * R * np;
#pragma unroll
            for (int tq = 0; tq < NTQ; ++tq) {
                const int e = i + tq * np;   // task: (column kc, chunk ch) of this level
                const int kc = e / ge.nch, ch = e % ge.nch;
                const cpx<T>* Pc = Pl + (size_t)kc * np + ch * CH;
#pragma unroll
                for (int j = 0; j < CH; ++j) pc[l][tq * CH + j] = Pc[j];
            }
        }
    }
}

// One level's chunk tile of load_pc (zero past the layer's levels or rows).
template <typename T, int B, int R>
__device__ __forceinline__ void load_pc_level(const Geo& ge, const cpx<T>* __restrict__ lay, int l, cpx<T> (&pc)[R]) {
    const int i = threadIdx.x, np = ge.np;
    constexpr int CH = Chunk<B, R>::CH, NTQ = Chunk<B, R>::NTQ;
#pragma unroll
    for (int j = 0; j < R; ++j) pc[j] = czero<T>();
    if (l < ge.L && i < np) {
        const cpx<T>* Pl = lay + ge.eK + (size_t)l * R * np;
#pragma unroll
        for (int tq = 0; tq < NTQ; ++tq) {
            const int e = i + tq * np;
            const int kc = e / ge.nch, ch = e % ge.nch;
            const cpx<T>* Pc = Pl + (size_t)kc * np + ch * CH;
#pragma unroll
            for (int j = 0; j < CH; ++j) pc[tq * CH + j] = Pc[j];
        }
    }
}

template <typename T, int B, int R, int LM>
__device__ __forceinline__ void load_pr(const Geo& ge, const cpx<T>* __restrict__ lay, cpx<T> (&pr)[LM > 0 ? LM : 1][R]) {
    const int i = threadIdx.x, np = ge.np;
    const cpx<T>* P = lay + ge.eK;
#pragma unroll
    for (int l = 0; l < LM; ++l) {
#pragma unroll
        for (int k = 0; k < R; ++k) pr[l][k] = czero<T>();
        if (l < ge.L && i < np) {
            const cpx<T>* Pl = P + (size_t)l * R * np;
#pragma unroll
            for (int k = 0; k < R; ++k) pr[l][k] = Pl[(size_t)k * np + i];
        }
    }
}

// One level's P row of load_pr.
template <typename T, int R>
__device__ __forceinline__ void load_pr_level(const Geo& ge, const cpx<T>* __restrict__ lay, int l, cpx<T> (&pr)[R]) {
    const int i = threadIdx.x, np = ge.np;
#pragma unroll
    for (int k = 0; k < R; ++k) pr[k] = czero<T>();
    if (l < ge.L && i < np) {
        const cpx<T>* Pl = lay + ge.eK + (size_t)l * R * np;
#pragma unroll
        for (int k = 0; k < R; ++k) pr[k] = Pl[(size_t)k * np + i];
    }
}

template <typename T, int R>
__device__ __forceinline__ void load_x(const Geo& ge, const cpx<T>* __restrict__ lay, cpx<T> (&x)[2 * R]) {
    const int i = threadIdx.x;
    const int npar = (1 << ge.L) - 1;
    if (ge.L > 0 && i < npar * 2 * R) {
        const int q = i / (2 * R), o = i % (2 * R);
        const cpx<T>* Xq = lay + ge.eK + ge.eP + (size_t)q * 4 * R * R + o;
#pragma unroll
        for (int c = 0; c < 2 * R; ++c) x[c] = Xq[(size_t)c * 2 * R];
    } else {
#pragma unroll
        for (int c = 0; c < 2 * R; ++c) x[c] = czero<T>();
    }
}

template <typename T, int B, int R, int LM>
__device__ __forceinline__ void load_layer(const Geo& ge, const cpx<T>* __restrict__ lay, LayerRegs<T, B, R, LM>& g) {
    load_K<T, B>(ge, lay, g.k);
    load_pr<T, B, R, LM>(ge, lay, g.pr);
    load_pc<T, B, R, LM>(ge, lay, g.pc);
    load_x<T, R>(ge, lay, g.x);
}

template <typename T>
struct SweepShared {
    cpx<T>* xs;    // np * G: the layer vectors, [row][g]
    cpx<T>* gs;    // (2^(L+1) - 1) * r * G: node reductions, heap-indexed, [node][k][g]
    cpx<T>* zs;    // (2^L - 1) * 2r * G: core products, [core row][g]
};

// One complex row-times-block product step on the matrix cores: for both
// pairs of right-hand sides, acc[2p] += A_p * re(a), acc[2p+1] += A_p * im(a)
// (see the file header for the lane layout).
__device__ __forceinline__ void mfma_row4(v4f (&acc)[4], const float* __restrict__ vrow, int m, cpx<float> a) {
    const float a0 = vrow[m], a1 = vrow[4 + m];
    acc[0] = __builtin_amdgcn_mfma_f32_4x4x1f32(a0, a.re, acc[0], 0, 0, 0);
    acc[1] = __builtin_amdgcn_mfma_f32_4x4x1f32(a0, a.im, acc[1], 0, 0, 0);
    acc[2] = __builtin_amdgcn_mfma_f32_4x4x1f32(a1, a.re, acc[2], 0, 0, 0);
    acc[3] = __builtin_amdgcn_mfma_f32_4x4x1f32(a1, a.im, acc[3], 0, 0, 0);
}

// The complex results of mfma_row4 for right-hand sides 0..3 of the lane's row.
__device__ __forceinline__ void mfma_row4_result(const v4f (&acc)[4], cpx<float> (&y)[4]) {
    y[0] = mk<float>(acc[0][0] - acc[1][1], acc[0][1] + acc[1][0]);
    y[1] = mk<float>(acc[0][2] - acc[1][3], acc[0][3] + acc[1][2]);
    y[2] = mk<float>(acc[2][0] - acc[3][1], acc[2][1] + acc[3][0]);
    y[3] = mk<float>(acc[2][2] - acc[3][3], acc[2][3] + acc[3][2]);
}

template <typename T, int G>
constexpr bool use_mfma() { return sizeof(T) == 4 && G == 4; }

// y_g = T_m x_g for the row owned by this thread and g < G.  Three
// workgroup barriers when L > 0: after the vector is published, after the
// node reductions, after the cores.  The node reductions are segmented
// wavefront reductions of the per-thread chunk sums (each node's chunks are
// consecutive lanes).  In the phased mode the tiles are loaded here, each
// just before its phase.
template <typename T, int B, int R, int LM, int G, bool PHASED>
__device__ __forceinline__ void apply_T(const Geo& ge, LayerRegs<T, B, R, LM>& g, const cpx<T>* __restrict__ lay,
                                        const cpx<T> (&x)[G], cpx<T> (&y)[G], const SweepShared<T>& sh) {
    const int np = ge.np, L = ge.L;
    const int i = threadIdx.x;
    const bool row = i < np;
    if (PHASED) load_K<T, B>(ge, lay, g.k);
    if (L == 0) __syncthreads();   // the previous step may still read xs
    if (row) {
#pragma unroll
        for (int q = 0; q < G; ++q) sh.xs[(size_t)i * G + q] = x[q];
    }
    __syncthreads();
    const int lane = i & 63, m4 = lane & 3;
    // ---- dense leaves
    if constexpr (use_mfma<T, G>()) {
        v4f acc[4] = {};
        const int t = row ? i / B : 0;
        const float* xf = (const float*)(sh.xs + (size_t)t * B * G);
#pragma unroll
        for (int j = 0; j < B; ++j) mfma_row4(acc, xf + (size_t)j * 2 * G, m4, row ? g.k[j] : czero<T>());
        mfma_row4_result(acc, y);
    } else {
#pragma unroll
        for (int q = 0; q < G; ++q) y[q] = czero<T>();
        if (row) {
            const cpx<T>* xl = sh.xs + (size_t)(i / B) * B * G;
#pragma unroll
            for (int j = 0; j < B; ++j) {
#pragma unroll
                for (int q = 0; q < G; ++q) cfma(y[q], g.k[j], xl[(size_t)j * G + q]);
            }
        }
    }
    if (L == 0) return;
    // ---- node reductions g_c = P_c^t x[c].  In the phased mode the chunk
    // tiles are streamed level by level, the next level's loads issued
    // before the current level's sums (two levels live instead of all).
    {
        constexpr int CH = Chunk<B, R>::CH, NTQ = Chunk<B, R>::NTQ;
        const int nch = ge.nch;
        cpx<T> pcb[2][PHASED ? R : 1];
        if constexpr (PHASED) load_pc_level<T, B, R>(ge, lay, 0, pcb[0]);
#pragma unroll
        for (int l = 0; l < LM; ++l) {
            if (l < L) {
                if constexpr (PHASED) {
                    if (l + 1 < LM) load_pc_level<T, B, R>(ge, lay, l + 1, pcb[(l + 1) & 1]);
                }
                const cpx<T>* tile = PHASED ? pcb[l & 1] : g.pc[l];
                const int lvl = l + 1;
                const int cpn = nch >> lvl;              // chunks per node of this level (<= 64)
#pragma unroll
                for (int tq = 0; tq < NTQ; ++tq) {
                    const int e = i + tq * np;           // (column kc, chunk ch) = (e / nch, e % nch)
                    cpx<T> acc[G];
#pragma unroll
                    for (int q = 0; q < G; ++q) acc[q] = czero<T>();
                    if (row) {
                        const cpx<T>* xc = sh.xs + (size_t)(e % nch) * CH * G;
#pragma unroll
                        for (int j = 0; j < CH; ++j) {
#pragma unroll
                            for (int q = 0; q < G; ++q) cfma(acc[q], tile[tq * CH + j], xc[(size_t)j * G + q]);
                        }
                    }
#pragma unroll
                    for (int q = 0; q < G; ++q) acc[q] = wops::gsum(acc[q], cpn);
                    if (row && (e % cpn) == 0) {
                        const int idx = (e % nch) / cpn, k = e / nch;
                        cpx<T>* gq = sh.gs + ((size_t)((1 << lvl) - 1 + idx) * R + k) * G;
#pragma unroll
                        for (int q = 0; q < G; ++q) gq[q] = acc[q];
                    }
                }
            }
        }
    }
    __syncthreads();
    if (PHASED) load_x<T, R>(ge, lay, g.x);
    // ---- cores z_q = X_q [g_left; g_right]
    {
        const int npar = (1 << L) - 1;
        const bool core = i < npar * 2 * R;
        if constexpr (use_mfma<T, G>()) {
            // whole waves past the last core row skip (wave-uniform test)
            if ((i & ~63) < npar * 2 * R) {
                v4f acc[4] = {};
                const int q = core ? i / (2 * R) : 0;
                const float* gf = (const float*)(sh.gs + (size_t)(2 * q + 1) * R * G);
#pragma unroll
                for (int c = 0; c < 2 * R; ++c) mfma_row4(acc, gf + (size_t)c * 2 * G, m4, core ? g.x[c] : czero<T>());
                cpx<T> z[4];
                mfma_row4_result(acc, z);
                if (core) {
#pragma unroll
                    for (int q2 = 0; q2 < 4; ++q2) sh.zs[(size_t)i * G + q2] = z[q2];
                }
            }
        } else if (core) {
            const int q = i / (2 * R);
            const cpx<T>* gq = sh.gs + (size_t)(2 * q + 1) * R * G;   // children 2q+1, 2q+2 are contiguous
            cpx<T> acc[G];
#pragma unroll
            for (int q2 = 0; q2 < G; ++q2) acc[q2] = czero<T>();
#pragma unroll
            for (int c = 0; c < 2 * R; ++c) {
#pragma unroll
                for (int q2 = 0; q2 < G; ++q2) cfma(acc[q2], g.x[c], gq[(size_t)c * G + q2]);
            }
#pragma unroll
            for (int q2 = 0; q2 < G; ++q2) sh.zs[(size_t)i * G + q2] = acc[q2];
        }
    }
    // phased: the P rows are streamed level by level like the chunk tiles,
    // the first level loaded here (the core rows are dead)
    cpx<T> prb[2][PHASED ? R : 1];
    if constexpr (PHASED) load_pr_level<T, R>(ge, lay, 0, prb[0]);
    __syncthreads();
    // ---- broadcast y[c] -= P_c z_q(side of c)
    if constexpr (use_mfma<T, G>()) {
        v4f acc[4] = {};
#pragma unroll
        for (int l = 0; l < LM; ++l) {
            if (l < L) {
                if constexpr (PHASED) {
                    if (l + 1 < LM) load_pr_level<T, R>(ge, lay, l + 1, prb[(l + 1) & 1]);
                }
                const cpx<T>* prl = PHASED ? prb[l & 1] : g.pr[l];
                const int lvl = l + 1;
                const int c = row ? i >> (ge.lnp - lvl) : 0;   // node index at lvl
                const int q = (1 << (lvl - 1)) - 1 + (c >> 1);
                const float* zf = (const float*)(sh.zs + ((size_t)q * 2 * R + (c & 1) * R) * G);
#pragma unroll
                for (int k = 0; k < R; ++k) mfma_row4(acc, zf + (size_t)k * 2 * G, m4, row ? prl[k] : czero<T>());
            }
        }
        cpx<T> d[4];
        mfma_row4_result(acc, d);
#pragma unroll
        for (int q = 0; q < 4; ++q) y[q] -= d[q];
    } else if (row) {
#pragma unroll
        for (int l = 0; l < LM; ++l) {
            if (l < L) {
                if constexpr (PHASED) {
                    if (l + 1 < LM) load_pr_level<T, R>(ge, lay, l + 1, prb[(l + 1) & 1]);
                }
                const cpx<T>* prl = PHASED ? prb[l & 1] : g.pr[l];
                const int lvl = l + 1;
                const int c = i >> (ge.lnp - lvl);   // node index at lvl
                const int q = (1 << (lvl - 1)) - 1 + (c >> 1);
                const cpx<T>* z = sh.zs + ((size_t)q * 2 * R + (c & 1) * R) * G;
                cpx<T> acc[G];
#pragma unroll
                for (int q2 = 0; q2 < G; ++q2) acc[q2] = czero<T>();
#pragma unroll
                for (int k = 0; k < R; ++k) {
#pragma unroll
                    for (int q2 = 0; q2 < G; ++q2) cfma(acc[q2], prl[k], z[(size_t)k * G + q2]);
                }
#pragma unroll
                for (int q2 = 0; q2 < G; ++q2) y[q2] -= acc[q2];
            }
        }
    }
}

// Vector inputs of one layer step, loaded one step ahead: the loads are
// issued before the current step's stores, so waiting for them never waits
// for those stores (the vector memory counter retires in order).
template <typename T, int G>
struct StepIn {
    c128 f[G];         // forward: f_m
    cpx<T> c;          // forward: A_{m,m-1} diagonal entry; backward: A_{m,m+1}
    cpx<T> w[G];       // backward: w_m
};

// State carried between the 2n-1 layer steps of one sweep.
template <typename T, int G>
struct SweepState {
    const c128* f[G];   // null for right-hand sides past the instance's last
    c128* u[G];
    cpx<T>* w[G];
    bool live[G];       // active right-hand side (inactive ones run with f = 0)
    const cpx<T>* cp;
    cpx<T> carry[G];    // forward: w_{m-1}; backward: u_{m+1}
    StepIn<T, G> pre;   // inputs of the next step
};

template <typename T, int G>
__device__ __forceinline__ StepIn<T, G> fetch_in(const Geo& ge, int s, const SweepState<T, G>& st) {
    const int n = ge.n, np = ge.np;
    const int i = threadIdx.x;
    const bool row = i < np, real_row = i < n;
    StepIn<T, G> in;
    in.c = czero<T>();
#pragma unroll
    for (int q = 0; q < G; ++q) {
        in.f[q] = czero<double>();
        in.w[q] = czero<T>();
    }
    if (s < n) {
        const int m = s;
#pragma unroll
        for (int q = 0; q < G; ++q)
            if (real_row && st.live[q]) in.f[q] = st.f[q][grid_index(ge, i, m)];
        if (m > 0 && row) in.c = st.cp[(size_t)(m - 1) * np + i];
    } else if (s < 2 * n - 1) {
        const int m = 2 * n - 2 - s;
        if (row) {
            in.c = st.cp[(size_t)m * np + i];
#pragma unroll
            for (int q = 0; q < G; ++q)
                if (st.w[q]) in.w[q] = st.w[q][(size_t)m * np + i];
        }
    }
    return in;
}

// Step s of the sweep: s < n is forward layer m = s, otherwise backward
// layer m = 2n-2-s.
template <typename T, int B, int R, int LM, int G, bool PHASED>
__device__ __forceinline__ void sweep_step(const Geo& ge, int s, LayerRegs<T, B, R, LM>& g, const cpx<T>* lay,
                                           SweepState<T, G>& st, const SweepShared<T>& sh) {
    const int n = ge.n, np = ge.np;
    const int i = threadIdx.x;
    const bool row = i < np, real_row = i < n;
    const StepIn<T, G> in = st.pre;
    st.pre = fetch_in<T, G>(ge, s + 1, st);      // before this step's stores
    cpx<T> x[G], y[G];
    if (s < n) {
        const int m = s;
#pragma unroll
        for (int q = 0; q < G; ++q) {
            x[q] = ccast<T>(in.f[q]);
            if (m > 0) x[q] -= in.c * st.carry[q];
        }
        apply_T<T, B, R, LM, G, PHASED>(ge, g, lay, x, y, sh);
#pragma unroll
        for (int q = 0; q < G; ++q) {
            if (row && st.w[q]) st.w[q][(size_t)m * np + i] = y[q];
            st.carry[q] = y[q];
            if (m == n - 1 && real_row && st.u[q]) st.u[q][grid_index(ge, i, m)] = ccast<double>(y[q]);
        }
    } else {
        const int m = 2 * n - 2 - s;
#pragma unroll
        for (int q = 0; q < G; ++q) x[q] = in.c * st.carry[q];
        apply_T<T, B, R, LM, G, PHASED>(ge, g, lay, x, y, sh);
#pragma unroll
        for (int q = 0; q < G; ++q) {
            const cpx<T> um = row ? in.w[q] - y[q] : czero<T>();
            if (real_row && st.u[q]) st.u[q][grid_index(ge, i, m)] = ccast<double>(um);
            st.carry[q] = um;
        }
    }
}

__device__ __forceinline__ int layer_of_step(int s, int n) { return s < n ? s : 2 * n - 2 - s; }

// Registers a thread may hold at this block size (512 per SIMD lane shared
// by the waves of the workgroup), in 32-bit registers.
template <typename T, int B, int R, int LM, int G, int NTHR>
struct Budget {
    static constexpr int C = (int)(2 * sizeof(T) / 4);              // registers per complex value
    static constexpr int FOOT = (B + 2 * (LM > 0 ? LM : 1) * R + 2 * R) * C;
    // per right-hand side: x, y, carry, the prefetched inputs (f in FP64, w)
    static constexpr int ACC = G * (8 + 5 * C) + (use_mfma<T, G>() ? 16 : 0) + 48;
    static constexpr int REG = 131072 / NTHR < 512 ? 131072 / NTHR : 512;
    static constexpr bool DB = 2 * FOOT + ACC <= REG;
    static constexpr bool PHASED = FOOT + ACC > REG;
};

template <typename T, int B, int R, int LM, int G, int NTHR>
__global__ __launch_bounds__(NTHR) void sweep_kernel(SweepArgs<T> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    // which instance and right-hand sides this workgroup runs
    int qi = 0, r0 = 0;
    if (!a.insts) {
        // one instance: its groups on a.nxcd XCDs (workgroup b runs on XCD b % 8)
        const int b = blockIdx.x, xcd = b & 7, slot = b >> 3;
        if (xcd >= a.nxcd) return;
        const int grp = slot * a.nxcd + xcd;
        if (grp >= a.ngroups) return;
        r0 = grp * G;
    } else {
        const int t = a.tasks[blockIdx.x];
        if (t < 0) return;
        qi = t >> 16;
        r0 = t & 0xffff;
    }
    const SweepInst<T> in = a.insts ? a.insts[qi] : a.one;
    Geo ge;
    ge.n = in.n; ge.np = in.np; ge.L = in.L; ge.lnp = 31 - __clz(in.np); ge.dir = in.dir;
    ge.nch = in.np / Chunk<B, R>::CH;
    ge.eK = in.eK; ge.eP = in.eP;
    const int n = in.n, np = in.np;
    const int i = threadIdx.x;
    const size_t N = (size_t)n * n;
    SweepState<T, G> st;
    st.cp = in.cp;
    bool any = false;
#pragma unroll
    for (int q = 0; q < G; ++q) {
        const int r = r0 + q;
        const bool exists = r < in.nrhs;
        st.f[q] = exists ? in.f + (size_t)a.jf * in.fstride + (size_t)r * N : nullptr;
        st.u[q] = exists ? in.u + (size_t)a.ju * in.ustride + (size_t)r * N : nullptr;
        st.w[q] = exists ? in.w + (size_t)r * n * np : nullptr;
        st.live[q] = exists && (!in.active || in.active[r]);
        st.carry[q] = czero<T>();
        any = any || st.live[q];
    }
    if (!any) {
        // every right-hand side of the group is inactive: u = 0
#pragma unroll
        for (int q = 0; q < G; ++q)
            if (st.u[q])
                for (size_t e = i; e < N; e += blockDim.x) st.u[q][e] = czero<double>();
        return;
    }
    st.pre = fetch_in<T, G>(ge, 0, st);
    SweepShared<T> sh;
    cpx<T>* base = (cpx<T>*)smem;
    sh.xs = base;
    sh.gs = sh.xs + (size_t)np * G;
    sh.zs = sh.gs + (size_t)((1 << (ge.L + 1)) - 1) * R * G;
    const int steps = 2 * n - 1;
    using BG = Budget<T, B, R, LM, G, NTHR>;
    if constexpr (BG::DB) {
        // two register sets used alternately: no copies between steps
        LayerRegs<T, B, R, LM> ga, gb;
        load_layer<T, B, R, LM>(ge, in.fac, ga);
        for (int s = 0; s < steps; s += 2) {
            if (s + 1 < steps) load_layer<T, B, R, LM>(ge, in.fac + (size_t)layer_of_step(s + 1, n) * in.eLayer, gb);
            sweep_step<T, B, R, LM, G, false>(ge, s, ga, nullptr, st, sh);
            if (s + 1 < steps) {
                if (s + 2 < steps) load_layer<T, B, R, LM>(ge, in.fac + (size_t)layer_of_step(s + 2, n) * in.eLayer, ga);
                sweep_step<T, B, R, LM, G, false>(ge, s + 1, gb, nullptr, st, sh);
            }
        }
    } else if constexpr (!BG::PHASED) {
        LayerRegs<T, B, R, LM> g;
        for (int s = 0; s < steps; ++s) {
            load_layer<T, B, R, LM>(ge, in.fac + (size_t)layer_of_step(s, n) * in.eLayer, g);
            sweep_step<T, B, R, LM, G, false>(ge, s, g, nullptr, st, sh);
        }
    } else {
        LayerRegs<T, B, R, LM> g;
        for (int s = 0; s < steps; ++s)
            sweep_step<T, B, R, LM, G, true>(ge, s, g, in.fac + (size_t)layer_of_step(s, n) * in.eLayer, st, sh);
    }
}

template <typename T, int B, int R, int LM, int G, int NTHR>
void launch_inst(const SweepArgs<T>& a, int blocks, size_t lds, hipStream_t s) {
    static bool attr = false;
    if (!attr) {
        hipFuncAttributes fa;
        if (hipFuncGetAttributes(&fa, (const void*)sweep_kernel<T, B, R, LM, G, NTHR>) == hipSuccess)
            (void)hipFuncSetAttribute((const void*)sweep_kernel<T, B, R, LM, G, NTHR>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize,
                                      160 * 1024 - (int)fa.sharedSizeBytes);
        (void)hipGetLastError();
        attr = true;
    }
    hipLaunchKernelGGL((sweep_kernel<T, B, R, LM, G, NTHR>), dim3(blocks), dim3(NTHR), lds, s, a);
}

}  // namespace hsweep_sweep

// (leaf b, rank r, levels L) combinations with a compiled sweep for one
// right-hand side per workgroup.  The block size is b * 2^L rounded up to a
// wavefront (or the core rows, if more).  Instances with fewer levels run on
// a kernel compiled for more (the levels are a runtime bound).
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
// Combinations with a compiled sweep for groups of 4 right-hand sides.
#define HSWEEP_SWEEP_LIST_G4(X)                                                       \
    X(16, 8, 3) X(16, 8, 4) X(16, 8, 5) X(32, 8, 3) X(32, 8, 4) X(32, 8, 5)

#define HSWEEP_MAX2(a, b) ((a) > (b) ? (a) : (b))
#define HSWEEP_NTHR(BB, RR, LL) \
    ((HSWEEP_MAX2(HSWEEP_MAX2(64, (BB) << (LL)), ((1 << (LL)) - 1) * 2 * (RR)) + 63) / 64 * 64)

#define HSWEEP_SWEEP_NAME(TT, BB, RR, LL, GG) sweep_launch_##TT##_##BB##_##RR##_##LL##_g##GG
#define HSWEEP_SWEEP_SIG(TT, CT, BB, RR, LL, GG) \
    void HSWEEP_SWEEP_NAME(TT, BB, RR, LL, GG)(const SweepArgs<CT>& a, int blocks, size_t lds, hipStream_t s)

#define HSWEEP_SWEEP_DEFINE_G(BB, RR, LL, GG)                                                          \
    HSWEEP_SWEEP_SIG(f, float, BB, RR, LL, GG) {                                                       \
        hsweep_sweep::launch_inst<float, BB, RR, LL, GG, HSWEEP_NTHR(BB, RR, LL)>(a, blocks, lds, s);  \
    }                                                                                                  \
    HSWEEP_SWEEP_SIG(d, double, BB, RR, LL, GG) {                                                      \
        hsweep_sweep::launch_inst<double, BB, RR, LL, GG, HSWEEP_NTHR(BB, RR, LL)>(a, blocks, lds, s); \
    }
#define HSWEEP_SWEEP_DEFINE(BB, RR, LL) HSWEEP_SWEEP_DEFINE_G(BB, RR, LL, 1)
#define HSWEEP_SWEEP_DEFINE4(BB, RR, LL) HSWEEP_SWEEP_DEFINE_G(BB, RR, LL, 4)
