// One layer of the approximate sweeping factorization (Alg. 2.3) on the GPU.
// Kernel templates; k_factor.hip instantiates them for complex64 and
// k_factor_f64.hip for complex128 (two translation units build in parallel).
//
// Given T_{m-1} in the form T = blockdiag(K) - sum_nodes P X P^t (the exact
// inverse of the H-matrix S_{m-1}), the step forms
//     S_m = A_{m,m} - D_m T_{m-1} D_m,       D_m = A_{m,m-1} (diagonal),
// as a weakly admissible H-matrix (Sec. 2.3): dense b x b diagonal leaves and,
// for each pair of sibling index sets (c1, c2), an off-diagonal block
// S(c1, c2) = Q_c1 Q_c2^t of rank <= r (S is complex symmetric, so
// S(c2, c1) = Q_c2 Q_c1^t and one factor per node suffices).  Then it inverts
// S_m level by level.  For a node c with children c1, c2,
//     S_c = blockdiag(S_c1, S_c2) + W [[0, I], [I, 0]] W^t,  W = blockdiag(Q_c1, Q_c2),
// so by the Sherman-Morrison-Woodbury identity
//     T_c = blockdiag(T_c1, T_c2) - P_c X_c P_c^t,
//     P_c = blockdiag(T_c1 Q_c1, T_c2 Q_c2),  X_c = [[Q_c1^t T_c1 Q_c1, I], [I, Q_c2^t T_c2 Q_c2]]^{-1}.
// This gives the same T_m as the paper's recursive 2x2 block inversion
// (hinv, Sec. 2.3) in exact arithmetic, with no truncation inside the
// inverse; truncation happens once per block when S_{m+1} is formed.
//
// Launches per layer (all on one stream):
//   layer_kernel       blocks [0, 2^L - 1): one per off-diagonal pair, build
//                      the stacked factors of S_m(c1, c2) (rank 1 + r*level),
//                      column-pivoted triangular factors of both (Householder
//                      QR, or in complex64 a pivoted Cholesky of the FP64 Gram
//                      matrix), one-sided Jacobi SVD of the small core,
//                      truncate (sigma > tol*sigma_1, at most r), write Q.
//                      blocks [2^L - 1, 2^(L+1) - 1): one per leaf, S_m leaf =
//                      A - D T_{m-1} D, Gauss-Jordan inverse -> K.
//   wood_pf_kernel(l)  levels l = L..1, one block per node: X_c from the
//                      children's G, then P_c = T_c Q_c and G_c = Q_c^t P_c
//                      (wood_kernel(l) where a node is too large for it).
//   wood_kernel(0)     the root core X_0.
#pragma once
#include "internal.hpp"
#include "wave_ops.hpp"

namespace {

constexpr int NT = 256;

template <typename T> __device__ __forceinline__ T eps_of();
template <> __device__ __forceinline__ float eps_of<float>() { return 1.1920929e-7f; }
template <> __device__ __forceinline__ double eps_of<double>() { return 2.220446049250313e-16; }

template <typename T> __device__ __forceinline__ T rsq(T x);
template <> __device__ __forceinline__ float rsq<float>(float x) { return sqrtf(x); }
template <> __device__ __forceinline__ double rsq<double>(double x) { return sqrt(x); }

__device__ __forceinline__ int heap_id(int lvl, int idx) { return (1 << lvl) - 1 + idx; }
// Reciprocal and reciprocal square root: the hardware approximations (about
// 1 ulp) in single precision, correctly rounded operations in double precision.
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double fast_rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float fast_rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double fast_rsq(double x) { return 1.0 / sqrt(x); }
// square root without the correctly rounded fix-up (about 1 ulp), for values
// that only set up a rotation
__device__ __forceinline__ float raw_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double raw_sqrt(double x) { return sqrt(x); }
// 1/sqrt(x) in FP64: the hardware estimate and one Newton step (relative
// error near 1e-14, far below what the pivoted Cholesky of a single-precision
// Gram matrix needs), in place of a correctly rounded sqrt and divide
__device__ __forceinline__ double rsq_nr(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    return y * (1.5 - 0.5 * x * y * y);
}
// 1 / a through one reciprocal of |a|^2 (pivots here are far from the
// overflow and underflow limits of |a|^2)
template <typename T> __device__ __forceinline__ cpx<T> cinv_fast(cpx<T> a) {
    const T r = fast_rcp(a.re * a.re + a.im * a.im);
    return mk<T>(a.re * r, -a.im * r);
}

// A wavefront executes in lockstep; wave_sync orders its LDS traffic and
// stops the compiler from moving memory operations across it.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ----------------------------------------------------------------------------
// Gauss-Jordan inversion with partial pivoting of a B x B matrix held in
// register tiles: thread (tr, tc) of a G x G grid (G = B / TS) owns rows
// tr*TS.. and columns tc*TS..  Pivots are chosen among the rows not yet used
// (no physical row swaps); the in-place result B satisfies
// inverse(perm^-1(i), perm(j)) = B(i, j).
template <int B> struct Tile {
    static constexpr int TS = B >= 16 ? B / 16 : 1;
    static constexpr int G = B / TS;
};

template <typename T, int B>
struct GJScratch {
    cpx<T> col[2][B];
    cpx<T> row[2][B];
    int used[B];
    int perm[B];
    int pinv[B];
};

template <typename T, int B>
__device__ __forceinline__ void gj_invert(cpx<T> (&M)[Tile<B>::TS][Tile<B>::TS], bool act, int tr, int tc,
                          GJScratch<T, B>& g, int* status) {
    constexpr int TS = Tile<B>::TS;
    for (int i = threadIdx.x; i < B; i += blockDim.x) g.used[i] = 0;
    __syncthreads();
    for (int k = 0; k < B; ++k) {
        cpx<T>* colk = g.col[k & 1];
        cpx<T>* rowp = g.row[k & 1];
        if (act && tc == k / TS) {
            const int kb = k % TS;
#pragma unroll
            for (int a = 0; a < TS; ++a)
#pragma unroll
                for (int bb = 0; bb < TS; ++bb)
                    if (bb == kb) colk[tr * TS + a] = M[a][bb];
        }
        __syncthreads();
        // pivot: largest |colk[i]| over the unused rows, by a wavefront argmax
        // (every wavefront computes the same result; ties -> lowest row)
        int p;
        T best;
        {
            const int lane = threadIdx.x & 63;
            best = T(-1);
            p = B;
            for (int i = lane; i < B; i += 64) {
                if (!g.used[i]) {
                    const T v = abs2(colk[i]);
                    if (v > best) { best = v; p = i; }
                }
            }
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                const T ob = __shfl_xor(best, off, 64);
                const int op = __shfl_xor(p, off, 64);
                if (ob > best || (ob == best && op < p)) { best = ob; p = op; }
            }
            if (p >= B) p = 0;
        }
        if (act && tr == p / TS) {
            const int pa = p % TS;
#pragma unroll
            for (int a = 0; a < TS; ++a)
#pragma unroll
                for (int bb = 0; bb < TS; ++bb)
                    if (a == pa) rowp[tc * TS + bb] = M[a][bb];
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            g.used[p] = 1;
            g.perm[k] = p;
            if (!(best > T(0))) *status = 1;
        }
        cpx<T> ipv = cinv(colk[p]);
        if (act) {
#pragma unroll
            for (int a = 0; a < TS; ++a) {
                int i = tr * TS + a;
                cpx<T> f = colk[i];
#pragma unroll
                for (int bb = 0; bb < TS; ++bb) {
                    int j = tc * TS + bb;
                    if (i == p) {
                        M[a][bb] = (j == k) ? ipv : rowp[j] * ipv;
                    } else {
                        M[a][bb] = (j == k) ? -(f * ipv) : M[a][bb] - f * (rowp[j] * ipv);
                    }
                }
            }
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < B; k += blockDim.x) g.pinv[g.perm[k]] = k;
    __syncthreads();
}

// ----------------------------------------------------------------------------
// Gauss-Jordan inversion with partial pivoting of a B x B matrix held in the
// registers of ONE wavefront (no LDS round trips, no workgroup barriers).
// Lane l holds row i = l % B and the CPL columns g*CPL .. g*CPL+CPL-1 of
// column group g = l / B.  Pivot rows are chosen among the rows not used yet
// (no physical swaps); if row i was the pivot of step k_i and perm[k] is the
// pivot row of step k, the inverse is inv(k_i, perm[j]) = M(i, j).
template <int B> struct WaveTile {
    static constexpr int NG = (64 / B) < B ? (64 / B) : B;   // column groups
    static constexpr int CPL = B / NG;                         // columns per lane
    static constexpr int LANES = B * NG;
};

template <typename T>
__device__ __forceinline__ cpx<T> shfl_c(cpx<T> v, int src) {
    return mk<T>(__shfl(v.re, src, 64), __shfl(v.im, src, 64));
}

// Runs on the lanes of one wavefront (all 64 must call it).  Min: column-major
// B x B input (ldi); Out: column-major inverse (ldo).  perm: B ints of LDS.
template <typename T, int B>
__device__ __forceinline__ void gj_wave(const cpx<T>* Min, int ldi, cpx<T>* Out, int ldo, int* perm,
                                        int* status) {
    constexpr int NG = WaveTile<B>::NG, CPL = WaveTile<B>::CPL, LANES = WaveTile<B>::LANES;
    const int lane = threadIdx.x & 63;
    const bool act = lane < LANES;
    const int i = lane % B, g = lane / B;
    cpx<T> M[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) M[c] = act ? Min[(size_t)(g * CPL + c) * ldi + i] : czero<T>();
    bool used = false;
    int mystep = 0;
    bool singular = false;
    for (int k = 0; k < B; ++k) {
        const int gk = k / CPL, kk = k % CPL;
        cpx<T> mine = czero<T>();
#pragma unroll
        for (int c = 0; c < CPL; ++c)
            if (c == kk) mine = M[c];
        const cpx<T> ci = shfl_c(mine, gk * B + i);          // this row's entry in column k
        // argmax of |ci|^2 over the unused rows of this column group
        T best = (act && !used) ? abs2(ci) : T(-1);
        int pr = act ? i : B;
#pragma unroll
        for (int off = 1; off < B; off <<= 1) {
            const T ob = __shfl_xor(best, off, 64);
            const int op = __shfl_xor(pr, off, 64);
            if (ob > best || (ob == best && op < pr)) { best = ob; pr = op; }
        }
        const int p = pr;                                    // same in every group
        const cpx<T> cp = shfl_c(ci, g * B + p);             // pivot value
        if (!(best > T(0))) singular = true;
        const cpx<T> ipv = cinv(cp);
        cpx<T> rowp[CPL];
#pragma unroll
        for (int c = 0; c < CPL; ++c) rowp[c] = shfl_c(M[c], g * B + p);
        if (i == p) { used = true; mystep = k; }
        if (lane == 0) perm[k] = p;
        if (act) {
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                const int j = g * CPL + c;
                if (i == p) M[c] = (j == k) ? ipv : rowp[c] * ipv;
                else M[c] = (j == k) ? -(ci * ipv) : M[c] - ci * (rowp[c] * ipv);
            }
        }
    }
    wave_sync();
    if (act) {
#pragma unroll
        for (int c = 0; c < CPL; ++c) Out[(size_t)perm[g * CPL + c] * ldo + mystep] = M[c];
    }
    if (lane == 0 && singular) *status = 1;
}

// Gauss-Jordan inversion with partial pivoting of a B x B matrix (B = 8, 16
// or 32) by one wavefront.  Lane l owns column j = l % B and the RPL = B*B/64
// rows rg*RPL .. rg*RPL + RPL-1 of row group rg = l / B.  A step fetches the
// pivot column's entries of its rows and, after a wave argmax, the pivot
// row's entry of its column, each with one ds_bpermute round trip.  Same
// pivot bookkeeping as gj_wave (no physical row swaps).
template <typename T>
__device__ __forceinline__ T bperm(T v, int src_lane);
template <>
__device__ __forceinline__ float bperm<float>(float v, int src) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v)));
}
template <>
__device__ __forceinline__ double bperm<double>(double v, int src) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_bpermute(src << 2, (int)(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_ds_bpermute(src << 2, (int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <typename T>
__device__ __forceinline__ cpx<T> bperm_c(cpx<T> v, int src) { return mk<T>(bperm(v.re, src), bperm(v.im, src)); }

__device__ __forceinline__ float readlane_f(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double readlane_f(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <typename T>
__device__ __forceinline__ cpx<T> readlane_c(cpx<T> v, int l) { return mk<T>(readlane_f(v.re, l), readlane_f(v.im, l)); }

template <typename T, int B>
__device__ __forceinline__ void gj_cols(const cpx<T>* Min, int ldi, cpx<T>* Out, int ldo, int* status) {
    static_assert(B == 8 || B == 16 || B == 32, "B * B must be a multiple of 64 lanes");
    constexpr int RPL = B * B / 64;
    const int lane = threadIdx.x & 63;
    const int j = lane % B, rg = lane / B;
    const int r0 = rg * RPL;
    cpx<T> M[RPL];
#pragma unroll
    for (int t = 0; t < RPL; ++t) M[t] = Min[(size_t)j * ldi + r0 + t];
    unsigned used = 0;              // rows of this lane already used as pivots (bit t)
    int mystep[RPL];
#pragma unroll
    for (int t = 0; t < RPL; ++t) mystep[t] = 0;
    int myperm = 0;                 // pivot row of step j
    bool singular = false;
    for (int k = 0; k < B; ++k) {
        // multipliers: column k's entries of this lane's rows
        cpx<T> ci[RPL];
#pragma unroll
        for (int t = 0; t < RPL; ++t) ci[t] = bperm_c(M[t], k + rg * B);
        // pivot: unused row of largest |entry| (lowest index among ties)
        T key = T(-1);
        int pr = 0x7fffffff;
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
            const T a = ((used >> t) & 1u) ? T(-1) : abs2(ci[t]);
            if (a > key) { key = a; pr = r0 + t; }
        }
        int p = wops::argmax_nonneg((float)key, pr & 63, key >= T(0));
        p = p < 0 ? 0 : p;                              // no unused row left: singular, flagged below
        const int tp = p % RPL, gp = p / RPL;           // pivot row's slot and row group
        // pivot row entry of this lane's column, and the pivot itself
        cpx<T> mine = M[0];
#pragma unroll
        for (int t = 1; t < RPL; ++t) mine = t == tp ? M[t] : mine;
        const cpx<T> rowp = bperm_c(mine, j + gp * B);
        const cpx<T> cp = readlane_c(rowp, k);          // pivot: column k's lane
        if (!(abs2(cp) > T(0))) singular = true;
        const cpx<T> ipv = cinv_fast(cp);
        const cpx<T> rs = rowp * ipv;                   // scaled pivot row entry
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
            const bool isp = r0 + t == p;
            if (j == k) M[t] = isp ? ipv : -(ci[t] * ipv);
            else M[t] = isp ? rs : M[t] - ci[t] * rs;
            if (isp) { used |= 1u << t; mystep[t] = k; }
        }
        if (j == k) myperm = p;
    }
#pragma unroll
    for (int t = 0; t < RPL; ++t) Out[(size_t)myperm * ldo + mystep[t]] = M[t];
    if (lane == 0 && singular) *status = 1;
}

// ----------------------------------------------------------------------------
// Leaf: S leaf of layer m, then its inverse K (column-major b x b).
//   S_leaf = A_leaf - D (K_prev - sum_lvl P_lvl X_lvl P_lvl^t) D   on the leaf rows.
// All factor data of the previous layer that the leaf needs is loaded in one
// phase (every load independent), then the update and the inverse run from
// registers and LDS.
template <typename T, int B, int R>
__device__ __forceinline__ void leaf_job(const Plan& p, const StepPtrs<T>& sp, int m, int t, unsigned char* smem) {
    constexpr int TS = Tile<B>::TS, G = Tile<B>::G;
    __shared__ int perm_w[B];
    const int tid = threadIdx.x;
    const bool act = tid < G * G;
    const int tr = tid % G, tc = tid / G;
    const int base = t * B;
    constexpr int r = R;
    const int L = p.L, np = p.np;
    cpx<T>* Pl = (cpx<T>*)smem;            // [lvl][i][k], L x B x r
    cpx<T>* Xb = Pl + (size_t)L * B * r;   // [lvl][k1][k2], L x r x r
    cpx<T>* Wl = Xb + (size_t)L * r * r;   // [lvl][i][k2], L x B x r

    cpx<T> M[TS][TS];
#pragma unroll
    for (int a = 0; a < TS; ++a)
#pragma unroll
        for (int bb = 0; bb < TS; ++bb) {
            int i = tr * TS + a, j = tc * TS + bb;
            M[a][bb] = (m > 0 && act) ? sp.Kp[(size_t)t * B * B + (size_t)j * B + i] : czero<T>();
        }
    if (m > 0 && L > 0) {
        for (int e = tid; e < L * B * r; e += NT) {
            int i = e % B, k = (e / B) % r, l = e / (B * r);
            Pl[((size_t)l * B + i) * r + k] = sp.Pp[((size_t)l * r + k) * np + base + i];
        }
        for (int e = tid; e < L * r * r; e += NT) {
            int k1 = e % r, k2 = (e / r) % r, l = e / (r * r);
            int anc = t >> (L - 1 - l);
            int q = anc >> 1, sg = anc & 1;
            const cpx<T>* Xq = sp.Xp + (size_t)heap_id(l, q) * 4 * r * r;
            Xb[((size_t)l * r + k1) * r + k2] = Xq[(size_t)(sg * r + k2) * 2 * r + sg * r + k1];
        }
        __syncthreads();
        for (int e = tid; e < L * B * r; e += NT) {
            int k2 = e % r, i = (e / r) % B, l = e / (B * r);
            const cpx<T>* pr = Pl + ((size_t)l * B + i) * r;
            const cpx<T>* xc = Xb + (size_t)l * r * r + k2;
            cpx<T> acc = czero<T>();
#pragma unroll
            for (int k1 = 0; k1 < r; ++k1) cfma(acc, pr[k1], xc[(size_t)k1 * r]);
            Wl[((size_t)l * B + i) * r + k2] = acc;
        }
        __syncthreads();
        if (act) {
#pragma unroll
            for (int a = 0; a < TS; ++a)
#pragma unroll
                for (int bb = 0; bb < TS; ++bb) {
                    int i = tr * TS + a, j = tc * TS + bb;
                    cpx<T> acc = czero<T>();
                    for (int l = 0; l < L; ++l) {
                        const cpx<T>* wr = Wl + ((size_t)l * B + i) * r;
                        const cpx<T>* pr = Pl + ((size_t)l * B + j) * r;
#pragma unroll
                        for (int k = 0; k < r; ++k) cfma(acc, wr[k], pr[k]);
                    }
                    M[a][bb] -= acc;
                }
        }
    }
    if (act) {
#pragma unroll
        for (int a = 0; a < TS; ++a)
#pragma unroll
            for (int bb = 0; bb < TS; ++bb) {
                int i = tr * TS + a, j = tc * TS + bb;
                int gi = base + i, gj = base + j;
                cpx<T> aij = czero<T>();
                if (i == j) aij = sp.dg[gi];
                else if (j == i + 1) aij = sp.eo[gi];
                else if (i == j + 1) aij = sp.eo[gj];
                M[a][bb] = (m > 0) ? aij - (sp.cp[gi] * sp.cp[gj]) * M[a][bb] : aij;
            }
    }
    // hand the leaf to one wavefront for the inverse (through LDS, column-major)
    __syncthreads();                       // Pl / Wl are no longer read
    cpx<T>* Ml = (cpx<T>*)smem;
    if (act) {
#pragma unroll
        for (int a = 0; a < TS; ++a)
#pragma unroll
            for (int bb = 0; bb < TS; ++bb) Ml[(size_t)(tc * TS + bb) * B + tr * TS + a] = M[a][bb];
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        if constexpr (B == 8 || B == 16 || B == 32) gj_cols<T, B>(Ml, B, sp.K + (size_t)t * B * B, B, sp.status);
        else gj_wave<T, B>(Ml, B, sp.K + (size_t)t * B * B, B, perm_w, sp.status);
    }
}

// ----------------------------------------------------------------------------
// Wavefront routines of the recompression.  One wavefront owns a problem; its
// 64 lanes form groups of G consecutive lanes (G a power of two), one group
// per column (or column pair), and lane g of a group handles the rows g,
// g + G, g + 2G, ...  Column sums are butterflies inside the group (DPP lane
// moves).  In the QR and in the application of Q each lane keeps its rows in
// registers (the first rrows of them; further rows stay in LDS and are
// streamed in chunks), so the only LDS traffic of a step is the reflector,
// which every group reads at the same addresses (broadcast, no conflicts).
// Pointers are cast to the LDS address space so that every access is a ds_*
// instruction; loads use clamped indices and selects instead of per-row
// branches, and the group geometry is kept in scalar registers.

template <typename X> using lds = __attribute__((address_space(3))) X;
template <typename X> __device__ __forceinline__ lds<X>* to_lds(X* p) { return (lds<X>*)p; }
template <typename X> __device__ __forceinline__ lds<X>* to_lds(const X* p) { return (lds<X>*)const_cast<X*>(p); }
template <typename T> __device__ __forceinline__ cpx<T> ldc(const lds<cpx<T>>* p) { return mk<T>(p->re, p->im); }
template <typename T> __device__ __forceinline__ void stc(lds<cpx<T>>* p, cpx<T> v) { p->re = v.re; p->im = v.im; }

// rows per lane held in registers (fewer in double precision, whose rows take
// twice the registers)
template <typename T> constexpr int rrows() { return sizeof(T) == 4 ? 32 : 16; }
constexpr int CHUNK = 8;    // rows per lane per chunk of LDS-resident rows

// Lane geometry for groups of G = 64 / 2^ceil(log2(ngroups)) lanes.
struct Groups {
    int lgG, G;   // log2 of the group size, group size (wave-uniform)
    int id, g;    // group index and lane within the group
};
__device__ __forceinline__ Groups make_groups(int ngroups) {
    Groups q;
    const int lgn = ngroups > 1 ? 32 - __clz(ngroups - 1) : 0;     // ceil(log2(ngroups))
    q.lgG = __builtin_amdgcn_readfirstlane(6 - lgn);
    q.G = 1 << q.lgG;
    const int lane = threadIdx.x & 63;
    q.id = lane >> q.lgG;
    q.g = lane & (q.G - 1);
    return q;
}
// rows g, g + G, ... below s: count for lane g, and for lane 0 (wave-uniform)
__device__ __forceinline__ int lane_rows(int s, const Groups& q) { return q.g < s ? ((s - 1 - q.g) >> q.lgG) + 1 : 0; }
__device__ __forceinline__ int max_rows(int s, const Groups& q) {
    return __builtin_amdgcn_readfirstlane((s + q.G - 1) >> q.lgG);
}

// Householder QR with column pivoting of the s x k column-major matrix A
// (leading dimension lda, k <= 64) in LDS, by one wavefront.  Columns stay in
// place: step j takes the remaining column p = perm[j] of largest norm, and
// the Hermitian reflector H_j = I - tau_j v_j v_j^H with
// v_j = (v0[j], A[j+1:, p]) maps it to beta_j e_j, stored in A[j, p].  Row j
// of every column not yet chosen then holds row j of R; pos[c] is the step at
// which column c was chosen (k if never), so R Pi^t has entry (j, c) equal to
// A[j, c] when j <= pos[c] and 0 otherwise.  Column norms are recomputed
// exactly from the updated rows at every step (no downdating).  The
// factorization stops at step kr when every remaining column norm is at most
// delta times the largest initial one.
template <typename T, int NR>
__device__ __forceinline__ int wave_qrcp_n(cpx<T>* Ag, int lda, int s, int k, int* permg, int* posg, cpx<T>* v0g,
                                           T* taug, T delta) {
    lds<cpx<T>>* A = to_lds(Ag);
    lds<int>* perm = to_lds(permg);
    lds<int>* pos = to_lds(posg);
    lds<cpx<T>>* v0 = to_lds(v0g);
    lds<T>* tau = to_lds(taug);
    const int lane = threadIdx.x & 63;
    const Groups gq = make_groups(k);
    const int G = gq.G, c = gq.id, g = gq.g;
    const bool col = c < k;
    lds<cpx<T>>* Ac = A + (size_t)(col ? c : 0) * lda;
    const int nrl = col ? lane_rows(s, gq) : 0;
    const int nmax = max_rows(s, gq);
    cpx<T> a[NR];
    // sums use four independent accumulators: with one wavefront per SIMD
    // nothing else hides the latency of a dependent chain
    T acc4[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int u = 0; u < NR; ++u) {
        const int i = g + G * u;
        a[u] = ldc(Ac + (i < s ? i : s - 1));
    }
    __builtin_amdgcn_sched_barrier(0);        // all loads in flight before the first use
#pragma unroll
    for (int u = 0; u < NR; ++u) {
        a[u] = u < nrl ? a[u] : czero<T>();
        acc4[u & 3] += abs2(a[u]);
    }
    T acc = (acc4[0] + acc4[1]) + (acc4[2] + acc4[3]);
    for (int u0 = NR; u0 < nmax; u0 += CHUNK) {
#pragma unroll
        for (int u = 0; u < CHUNK; ++u) {
            const int i = g + G * (u0 + u);
            const cpx<T> x = ldc(Ac + (i < s ? i : s - 1));
            acc += u0 + u < nrl ? abs2(x) : T(0);
        }
    }
    T nrm = wops::gsum(acc, G);
    T mx = col ? nrm : T(0);
    int unused = lane;
    wops::argmax(mx, unused);
    const T stop = delta * delta * mx;
    bool chosen = !col;
    const int kk = s < k ? s : k;
    int kr = kk;
    for (int j = 0; j < kk; ++j) {
        int p = wops::argmax_nonneg((float)nrm, c, !chosen);
        const T key = p >= 0 ? readlane_f(nrm, p * G) : T(-1);    // exact norm of the pivot column
        if (!(key > stop)) { kr = j; break; }
        // the pivot group publishes its register rows (rows beyond them are in LDS already)
        if (c == p) {
#pragma unroll
            for (int u = 0; u < NR; ++u)
                if (u < nrl) stc(Ac + (g + G * u), a[u]);
        }
        wave_sync();
        lds<cpx<T>>* Ap = A + (size_t)p * lda;
        const cpx<T> x0 = ldc(Ap + j);
        const T nx = sqrt(key), ax0 = sqrt(abs2(x0));
        const cpx<T> ph = ax0 > T(0) ? (T(1) / ax0) * x0 : mk<T>(T(1), T(0));
        const cpx<T> vv0 = (ax0 + nx) * ph;
        const T tj = T(1) / (nx * (nx + ax0));
        const bool act = !chosen && c != p;
        const int n_act = act ? nrl : 0;
        // reflector entries of this lane's rows: zero above row j, past the
        // column and on lanes that do not update
        cpx<T> d = czero<T>();
        cpx<T> v[NR];
#pragma unroll
        for (int u = 0; u < NR; ++u) {
            const int i = g + G * u;
            v[u] = ldc(Ap + (i < s ? i : s - 1));
        }
        __builtin_amdgcn_sched_barrier(0);
        cpx<T> d4[4] = {czero<T>(), czero<T>(), czero<T>(), czero<T>()};
#pragma unroll
        for (int u = 0; u < NR; ++u) {
            const int i = g + G * u;
            v[u] = (u < n_act && i >= j) ? (i == j ? vv0 : v[u]) : czero<T>();
            cfma_conj(d4[u & 3], v[u], a[u]);
        }
        d = (d4[0] + d4[1]) + (d4[2] + d4[3]);
        for (int u0 = NR; u0 < nmax; u0 += CHUNK) {
#pragma unroll
            for (int u = 0; u < CHUNK; ++u) {
                const int i = g + G * (u0 + u);
                const int ic = i < s ? i : s - 1;
                const cpx<T> lv = ldc(Ap + ic), x = ldc(Ac + ic);
                const bool in = u0 + u < n_act && i >= j;
                cfma_conj(d, in ? (i == j ? vv0 : lv) : czero<T>(), x);
            }
        }
        d = wops::gsum(d, G);
        const cpx<T> td = tj * d;
        T nn4[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int u = 0; u < NR; ++u) {
            const int i = g + G * u;
            a[u] -= v[u] * td;
            nn4[u & 3] += i > j ? abs2(a[u]) : T(0);
        }
        T nn = (nn4[0] + nn4[1]) + (nn4[2] + nn4[3]);
        for (int u0 = NR; u0 < nmax; u0 += CHUNK) {
            cpx<T> an[CHUNK];
#pragma unroll
            for (int u = 0; u < CHUNK; ++u) {
                const int i = g + G * (u0 + u);
                const int ic = i < s ? i : s - 1;
                const cpx<T> lv = ldc(Ap + ic), x = ldc(Ac + ic);
                an[u] = x - (i == j ? vv0 : lv) * td;
            }
#pragma unroll
            for (int u = 0; u < CHUNK; ++u) {
                const int i = g + G * (u0 + u);
                if (u0 + u < n_act && i >= j) {
                    stc(Ac + i, an[u]);
                    if (i > j) nn += abs2(an[u]);
                }
            }
        }
        nn = wops::gsum(nn, G);
        if (act) nrm = nn;
        if (c == p && g == (j & (G - 1))) stc(Ap + j, -nx * ph);
        if (lane == 0) {
            stc(v0 + j, vv0);
            tau[j] = tj;
            perm[j] = p;
            pos[p] = j;
        }
        if (c == p) chosen = true;
        wave_sync();
    }
    // columns never chosen: rows < kr hold R, the rest the dropped remainder
    if (!chosen) {
#pragma unroll
        for (int u = 0; u < NR; ++u)
            if (u < nrl) stc(Ac + (g + G * u), a[u]);
        if (g == 0) pos[c] = k;
    }
    wave_sync();
    return kr;
}

// Rows per lane held in registers: 4, 16 or rrows (beyond that they are streamed).
template <typename T>
__device__ __forceinline__ int wave_qrcp(cpx<T>* A, int lda, int s, int k, int* perm, int* pos, cpx<T>* v0, T* tau,
                                         T delta) {
    const int nmax = max_rows(s, make_groups(k));
    if (nmax <= 4) return wave_qrcp_n<T, 4>(A, lda, s, k, perm, pos, v0, tau, delta);
    if (nmax <= 16) return wave_qrcp_n<T, 16>(A, lda, s, k, perm, pos, v0, tau, delta);
    return wave_qrcp_n<T, rrows<T>()>(A, lda, s, k, perm, pos, v0, tau, delta);
}

// Y <- H_0 ... H_{kr-1} Y for the reflectors left in A by wave_qrcp (Y: s x
// ncol column-major, leading dimension ldy, ncol <= 64), by one wavefront.
template <typename T, int NR>
__device__ __forceinline__ void wave_apply_q_n(const cpx<T>* Ag, int lda, int s, int kr, const int* permg,
                                               const cpx<T>* v0g, const T* taug, cpx<T>* Yg, int ldy, int ncol) {
    lds<cpx<T>>* A = to_lds(Ag);
    lds<int>* perm = to_lds(permg);
    lds<cpx<T>>* v0 = to_lds(v0g);
    lds<T>* tau = to_lds(taug);
    const Groups gq = make_groups(ncol);
    const int G = gq.G, c = gq.id, g = gq.g;
    const bool act = c < ncol;
    lds<cpx<T>>* Yc = to_lds(Yg) + (size_t)(act ? c : 0) * ldy;
    const int nrl = act ? lane_rows(s, gq) : 0;
    const int nmax = max_rows(s, gq);
    cpx<T> y[NR];
#pragma unroll
    for (int u = 0; u < NR; ++u) {
        const int i = g + G * u;
        y[u] = ldc(Yc + (i < s ? i : s - 1));
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < NR; ++u) y[u] = u < nrl ? y[u] : czero<T>();
    for (int j = kr - 1; j >= 0; --j) {
        const T tj = tau[j];
        lds<cpx<T>>* Ap = A + (size_t)perm[j] * lda;
        const cpx<T> vv0 = ldc(v0 + j);
        cpx<T> d = czero<T>();
        cpx<T> v[NR];
#pragma unroll
        for (int u = 0; u < NR; ++u) {
            const int i = g + G * u;
            v[u] = ldc(Ap + (i < s ? i : s - 1));
        }
        __builtin_amdgcn_sched_barrier(0);
        cpx<T> d4[4] = {czero<T>(), czero<T>(), czero<T>(), czero<T>()};
#pragma unroll
        for (int u = 0; u < NR; ++u) {
            const int i = g + G * u;
            v[u] = (u < nrl && i >= j) ? (i == j ? vv0 : v[u]) : czero<T>();
            cfma_conj(d4[u & 3], v[u], y[u]);
        }
        d = (d4[0] + d4[1]) + (d4[2] + d4[3]);
        for (int u0 = NR; u0 < nmax; u0 += CHUNK) {
#pragma unroll
            for (int u = 0; u < CHUNK; ++u) {
                const int i = g + G * (u0 + u);
                const int ic = i < s ? i : s - 1;
                const cpx<T> lv = ldc(Ap + ic), x = ldc(Yc + ic);
                const bool in = u0 + u < nrl && i >= j;
                cfma_conj(d, in ? (i == j ? vv0 : lv) : czero<T>(), x);
            }
        }
        d = wops::gsum(d, G);
        const cpx<T> td = tj * d;
#pragma unroll
        for (int u = 0; u < NR; ++u) y[u] -= v[u] * td;
        for (int u0 = NR; u0 < nmax; u0 += CHUNK) {
            cpx<T> yn[CHUNK];
#pragma unroll
            for (int u = 0; u < CHUNK; ++u) {
                const int i = g + G * (u0 + u);
                const int ic = i < s ? i : s - 1;
                const cpx<T> lv = ldc(Ap + ic), x = ldc(Yc + ic);
                yn[u] = x - (i == j ? vv0 : lv) * td;
            }
#pragma unroll
            for (int u = 0; u < CHUNK; ++u) {
                const int i = g + G * (u0 + u);
                if (u0 + u < nrl && i >= j) stc(Yc + i, yn[u]);
            }
        }
    }
#pragma unroll
    for (int u = 0; u < NR; ++u)
        if (u < nrl) stc(Yc + (g + G * u), y[u]);
    wave_sync();
}

template <typename T>
__device__ __forceinline__ void wave_apply_q(const cpx<T>* A, int lda, int s, int kr, const int* perm,
                                             const cpx<T>* v0, const T* tau, cpx<T>* Y, int ldy, int ncol) {
    if (ncol <= 0) return;
    const int nmax = max_rows(s, make_groups(ncol));
    if (nmax <= 4) wave_apply_q_n<T, 4>(A, lda, s, kr, perm, v0, tau, Y, ldy, ncol);
    else if (nmax <= 16) wave_apply_q_n<T, 16>(A, lda, s, kr, perm, v0, tau, Y, ldy, ncol);
    else wave_apply_q_n<T, rrows<T>()>(A, lda, s, kr, perm, v0, tau, Y, ldy, ncol);
}

// One-sided Jacobi SVD by one wavefront of the P columns of N in LDS (P even,
// P <= 64; zero columns allowed).  The rotations of a round act on disjoint
// column pairs (round-robin order), one lane group of G lanes per pair.  N
// (nr rows) and J (P rows) are stored with NR * G rows per column, the rows
// past nr (past P for J) zero, so every lane loads and stores exactly NR rows
// of each column without predicates; a pair that needs no rotation applies the
// identity.  A pair is rotated when |a^H b| > thr |a| |b|, |a^H b| > gabs and
// both columns are above the negligible level tiny (squared norm).  Sweeps
// stop after one in which no pair was rotated by more than cos = sqrt(thr)
// (the next sweep, converging quadratically, would rotate none), or -- for up
// to JACOBI_CHECK_PMAX columns with a compile-time group size -- as soon as
// a test of all pairs finds none that a further sweep would rotate.  J
// (column-major, leading dimension NR * G) starts as the identity and
// accumulates the rotations, so that N_in J = N_out with nearly orthogonal
// columns; nrm2[c] is the squared norm of column c.  Since J is unitary,
// dropping columns of N_out changes N by exactly their norms, whatever their
// residual inner products.
// GT: the lane-group size when known at compile time (then the butterflies
// and the lane geometry are constants), 0 to take it from P at run time.
// NRJ: rows of J per lane (J has only P rows), at most NR.
// Largest column count for which a sweep's end is tested on all pairs at once
// (up to P (P - 1) / 2 <= 496 inner products, at most 8 per lane).
constexpr int JACOBI_CHECK_PMAX = 32;

// All inner products of the P columns of N (rows [0, ROWS), column-major,
// leading dimension ld) by one wavefront, after a sweep: writes every squared
// column norm to nrm2 and returns whether any pair still meets the rotation
// test of the sweeps.  When none does, a further sweep would rotate nothing,
// so this replaces that sweep.  P <= JACOBI_CHECK_PMAX.
template <typename CT, int ROWS>
__device__ __forceinline__ bool jacobi_pairs_left(const lds<cpx<CT>>* N, int P, int ld, lds<CT>* nrm2, CT thr,
                                                  CT gabs, CT tiny) {
    const int lane = threadIdx.x & 63;
    auto dot = [&](int a, int b) {
        const lds<cpx<CT>>* ca = N + (size_t)a * ld;
        const lds<cpx<CT>>* cb = N + (size_t)b * ld;
        cpx<CT> d0 = czero<CT>(), d1 = d0;
#pragma unroll
        for (int r = 0; r + 1 < ROWS; r += 2) {
            cfma_conj(d0, ldc(ca + r), ldc(cb + r));
            cfma_conj(d1, ldc(ca + r + 1), ldc(cb + r + 1));
        }
        if constexpr (ROWS & 1) cfma_conj(d0, ldc(ca + ROWS - 1), ldc(cb + ROWS - 1));
        return d0 + d1;
    };
    if (lane < P) nrm2[lane] = dot(lane, lane).re;
    wave_sync();
    // pairs a < b, row-major: index e = a (2P - a - 1) / 2 + (b - a - 1); a
    // from the float root of the quadratic, corrected by one step either way
    bool more = false;
    const int ne = P * (P - 1) / 2;
    const float tp = (float)(2 * P - 1);
    for (int e = lane; e < ne; e += 64) {
        int a = (int)((tp - __builtin_amdgcn_sqrtf(tp * tp - 8.0f * (float)e)) * 0.5f);
        a = a < 0 ? 0 : (a > P - 2 ? P - 2 : a);
        if (a * (2 * P - a - 1) / 2 > e) --a;
        else if ((a + 1) * (2 * P - a - 2) / 2 <= e) ++a;
        const int b = e - a * (2 * P - a - 1) / 2 + a + 1;
        const CT al = nrm2[a], be = nrm2[b];
        const CT ag2 = abs2(dot(a, b));
        more = more || (al > tiny && be > tiny && ag2 > thr * thr * (al * be) && ag2 > gabs * gabs);
    }
    return __ballot(more) != 0;
}

template <typename CT, int NR, int GT, int NRJ = NR>
__device__ __forceinline__ void wave_jacobi_n(cpx<CT>* Ng, int P, cpx<CT>* Jg, CT* nrm2g, CT thr, CT gabs, CT tiny,
                                              int max_sweeps) {
    static_assert(NRJ <= NR, "J has no more rows than N");
    lds<cpx<CT>>* N = to_lds(Ng);
    lds<cpx<CT>>* J = to_lds(Jg);
    lds<CT>* nrm2 = to_lds(nrm2g);
    const int lane = threadIdx.x & 63;
    const int npair = P / 2;
    const Groups gq = make_groups(npair);
    const int G = GT > 0 ? GT : gq.G;
    const int q = GT > 0 ? lane / GT : gq.id, g = GT > 0 ? lane % GT : gq.g;
    auto gs = [&](auto v) { if constexpr (GT > 0) return wops::gsum_ct<GT>(v); else return wops::gsum(v, G); };
    const int ld = (NR + 1) * G;                 // as jacobi_ld: one group of padding rows
    constexpr int CH = NR < 8 ? NR : 8;
    constexpr bool ONE = NR <= 8;
    const bool act = q < npair;
    for (int e = lane; e < ld * P; e += 64) {
        const int r = e % ld;
        stc(J + e, r == e / ld ? mk<CT>(CT(1), CT(0)) : czero<CT>());
    }
    wave_sync();
    const int P1 = P - 1;
    for (int sweep = 0; sweep <= max_sweeps; ++sweep) {
        const bool last = sweep == max_sweeps;
        CT mxc = CT(0);                       // largest squared cosine rotated in this sweep
        int nrot = 0;                         // pairs rotated in this sweep (wave-uniform)
        for (int rd = 0; rd < P1; ++rd) {
            // round-robin pairs: (rd, P-1) and ((rd + q) mod (P-1), (rd - q) mod (P-1))
            int a = rd + q, b = rd - q + P1;
            a = a >= P1 ? a - P1 : a;
            b = b >= P1 ? b - P1 : b;
            if (q == 0) { a = rd; b = P1; }
            if (!act) { a = 0; b = 0; }
            lds<cpx<CT>>* ca = N + (size_t)a * ld + g;
            lds<cpx<CT>>* cb = N + (size_t)b * ld + g;
            lds<cpx<CT>>* ja = J + (size_t)a * ld + g;
            lds<cpx<CT>>* jb = J + (size_t)b * ld + g;
            // rows in chunks of CH; with a single chunk the rows stay in registers
            cpx<CT> xa[CH], xb[CH], ya[CH], yb[CH];
            CT al = CT(0), be = CT(0);
            cpx<CT> ga = czero<CT>();
#pragma unroll
            for (int u0 = 0; u0 < NR; u0 += CH) {
#pragma unroll
                for (int u = 0; u < CH; ++u) {
                    xa[u] = ldc(ca + G * (u0 + u));
                    xb[u] = ldc(cb + G * (u0 + u));
                    if (ONE && u < NRJ) {
                        ya[u] = ldc(ja + G * u);
                        yb[u] = ldc(jb + G * u);
                    }
                }
                __builtin_amdgcn_sched_barrier(0);     // all loads in flight before the first use
#pragma unroll
                for (int u = 0; u < CH; ++u) {
                    al += abs2(xa[u]);
                    be += abs2(xb[u]);
                    cfma_conj(ga, xa[u], xb[u]);
                }
            }
            al = gs(al);
            be = gs(be);
            ga = gs(ga);
            const CT ag2 = abs2(ga);
            const CT ab = al * be;
            const bool doit = !last && act && al > tiny && be > tiny && ag2 > thr * thr * ab && ag2 > gabs * gabs;
            // rotation (identity when the pair is left alone)
            const CT iag = doit ? fast_rsq(ag2) : CT(0);              // 1 / |gamma|
            const CT zeta = CT(0.5) * (be - al) * iag;
            const CT tm = fast_rcp(fabs(zeta) + raw_sqrt(CT(1) + zeta * zeta));
            const CT t = doit ? (zeta >= CT(0) ? tm : -tm) : CT(0);
            const CT cs = fast_rsq(CT(1) + t * t);
            const CT sn = cs * t;
            const cpx<CT> em = doit ? iag * conj(ga) : mk<CT>(CT(1), CT(0));   // e^{-i phi}
            if (act && !last) {
#pragma unroll
                for (int u0 = 0; u0 < NR; u0 += CH) {
                    if (!ONE) {
                        // reload the chunk (the fence keeps the compiler from reusing pass-1 values)
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
                        for (int u = 0; u < CH; ++u) {
                            xa[u] = ldc(ca + G * (u0 + u));
                            xb[u] = ldc(cb + G * (u0 + u));
                            if (u0 + u < NRJ) {
                                ya[u] = ldc(ja + G * (u0 + u));
                                yb[u] = ldc(jb + G * (u0 + u));
                            }
                        }
                    }
#pragma unroll
                    for (int u = 0; u < CH; ++u) {
                        const cpx<CT> x2 = em * xb[u];
                        stc(ca + G * (u0 + u), cs * xa[u] - sn * x2);
                        stc(cb + G * (u0 + u), sn * xa[u] + cs * x2);
                        if (u0 + u < NRJ) {
                            const cpx<CT> y2 = em * yb[u];
                            stc(ja + G * (u0 + u), cs * ya[u] - sn * y2);
                            stc(jb + G * (u0 + u), sn * ya[u] + cs * y2);
                        }
                    }
                }
            }
            if (last && act && g == 0) {
                nrm2[a] = al;
                nrm2[b] = be;
            }
            if (doit) mxc = fmax(mxc, ag2 * fast_rcp(ab));
            nrot += __popcll(__ballot(doit && g == 0));
            wave_sync();
            if (last) break;
        }
        if (last) break;
        int unused = 0;
        wops::argmax(mxc, unused);
        if constexpr (GT > 0) {                       // compile-time group size
            if (P <= JACOBI_CHECK_PMAX && nrot <= P) {
                // after a sweep with few rotations (the last one before
                // convergence typically turns one or two pairs), one pass
                // over all pairs instead of a sweep that would find nothing
                // left to rotate; it also gives the norms
                const bool more = jacobi_pairs_left<CT, NR * GT>(N, P, ld, nrm2, thr, gabs, tiny);
                if (!more || !(mxc > thr) || sweep + 1 == max_sweeps) break;
                continue;
            }
        }
        if (!(mxc > thr)) sweep = max_sweeps - 1;   // converged: one more pass for the norms
    }
    wave_sync();
}

// Rows per lane (4, 8, 16 or 32) and leading dimension of N and J in the
// Jacobi for P columns of at most nr rows.
__host__ __device__ inline int jacobi_group(int P) {
    int np2 = 1;
    while (np2 < (P / 2 > 0 ? P / 2 : 1)) np2 <<= 1;
    return 64 / np2;
}
__host__ __device__ inline int jacobi_rows(int nr, int P) {
    const int G = jacobi_group(P);
    const int need = ((nr > P ? nr : P) + G - 1) / G;
    if (need == 3) return 3;
    int r = 1;
    while (r < need) r <<= 1;
    return r;
}
// (padded by one group so that columns do not start on the same LDS bank)
__host__ __device__ inline int jacobi_ld(int nr, int P) { return (jacobi_rows(nr, P) + 1) * jacobi_group(P); }

template <typename CT, int GT>
__device__ __forceinline__ void wave_jacobi_g(cpx<CT>* N, int P, int NRr, cpx<CT>* J, CT* nrm2, CT thr, CT gabs,
                                              CT tiny, int max_sweeps) {
    if (NRr == 1) wave_jacobi_n<CT, 1, GT>(N, P, J, nrm2, thr, gabs, tiny, max_sweeps);
    else if (NRr == 2) wave_jacobi_n<CT, 2, GT>(N, P, J, nrm2, thr, gabs, tiny, max_sweeps);
    else if (NRr == 3) wave_jacobi_n<CT, 3, GT>(N, P, J, nrm2, thr, gabs, tiny, max_sweeps);
    else if (NRr == 4) wave_jacobi_n<CT, 4, GT>(N, P, J, nrm2, thr, gabs, tiny, max_sweeps);
    else if (NRr == 8) wave_jacobi_n<CT, 8, GT>(N, P, J, nrm2, thr, gabs, tiny, max_sweeps);
    else if (NRr == 16) wave_jacobi_n<CT, 16, GT>(N, P, J, nrm2, thr, gabs, tiny, max_sweeps);
    else wave_jacobi_n<CT, 32, GT>(N, P, J, nrm2, thr, gabs, tiny, max_sweeps);
}

// Group sizes 4, 8 and 16 (P from 7 to 32 columns) are compiled as constants.
// With groups of 8 lanes (P from 9 to 16) J spans two rows per lane and with
// groups of 16 (P from 5 to 8) one, however many rows N has.
template <typename CT>
__device__ __forceinline__ void wave_jacobi(cpx<CT>* N, int P, int NRr, cpx<CT>* J, CT* nrm2, CT thr, CT gabs,
                                            CT tiny, int max_sweeps) {
    const int G = jacobi_group(P);
#define WJ(NRV, GV, NRJV) wave_jacobi_n<CT, NRV, GV, NRJV>(N, P, J, nrm2, thr, gabs, tiny, max_sweeps)
    if (G == 4 && NRr <= 16) wave_jacobi_g<CT, 4>(N, P, NRr, J, nrm2, thr, gabs, tiny, max_sweeps);
    else if (G == 8 && NRr >= 2 && NRr <= 8) {
        if (NRr == 2) WJ(2, 8, 2);
        else if (NRr == 3) WJ(3, 8, 2);
        else if (NRr == 4) WJ(4, 8, 2);
        else WJ(8, 8, 2);
    } else if (G == 16 && NRr <= 4) {
        if (NRr == 1) WJ(1, 16, 1);
        else if (NRr == 2) WJ(2, 16, 1);
        else if (NRr == 3) WJ(3, 16, 1);
        else WJ(4, 16, 1);
    } else wave_jacobi_g<CT, 0>(N, P, NRr, J, nrm2, thr, gabs, tiny, max_sweeps);
#undef WJ
}

// Gram matrices GA = A^H A and GB = B^H B (k x k, both triangles stored,
// column-major) of the s x k column-major A and B in LDS, accumulated in FP64
// (products of single-precision entries are exact), by all threads.
template <typename T>
__device__ __forceinline__ void gram_pair(const cpx<T>* A, const cpx<T>* B, int s, int lda, int k, c128* GA,
                                          c128* GB) {
    const int nt = k * (k + 1) / 2;
    for (int e = threadIdx.x; e < 2 * nt; e += NT) {
        const bool second = e >= nt;
        const int q = second ? e - nt : e;
        // column b, row a <= b of entry q = b (b + 1) / 2 + a: b from the
        // float root, corrected by one step either way (exact for k <= 64)
        int b = (int)((__builtin_amdgcn_sqrtf(8.0f * (float)q + 1.0f) - 1.0f) * 0.5f);
        b += (b + 1) * (b + 2) / 2 <= q ? 1 : 0;
        b -= b * (b + 1) / 2 > q ? 1 : 0;
        const int a = q - b * (b + 1) / 2;
        const lds<cpx<T>>* X = to_lds(second ? B : A);
        const lds<cpx<T>>* xa = X + (size_t)a * lda;
        const lds<cpx<T>>* xb = X + (size_t)b * lda;
        c128 g0 = czero<double>(), g1 = g0, g2 = g0, g3 = g0;     // independent chains
        int i = 0;
        for (; i + 4 <= s; i += 4) {
            cfma_conj(g0, ccast<double>(ldc(xa + i)), ccast<double>(ldc(xb + i)));
            cfma_conj(g1, ccast<double>(ldc(xa + i + 1)), ccast<double>(ldc(xb + i + 1)));
            cfma_conj(g2, ccast<double>(ldc(xa + i + 2)), ccast<double>(ldc(xb + i + 2)));
            cfma_conj(g3, ccast<double>(ldc(xa + i + 3)), ccast<double>(ldc(xb + i + 3)));
        }
        for (; i < s; ++i) cfma_conj(g0, ccast<double>(ldc(xa + i)), ccast<double>(ldc(xb + i)));
        const c128 g = (g0 + g1) + (g2 + g3);
        c128* G = second ? GB : GA;
        G[(size_t)b * k + a] = g;
        G[(size_t)a * k + b] = conj(g);
    }
}

// Pivoted Cholesky (Crout form) of the k x k Hermitian positive semidefinite
// G (column-major, k <= 64) by one wavefront; lane c owns column c (lanes
// 2c and 2c + 1 when k <= 32).  Step j
// takes the column p of largest Schur-complement diagonal d_p and forms row j
// of R:  R[j][c] = (G[p][c] - sum_{t<j} conj(R[t][p]) R[t][c]) / sqrt(d_p)
// for the columns not chosen yet, 0 for the others (so R holds R Pi^t, as the
// QR path's row j).  With G = A^H A this is the R of A's Householder QR with
// column pivoting (in exact arithmetic).  It stops at kr when every remaining
// d is at most delta^2 times the largest initial one; pos[c] is the step at
// which c was chosen (k if never), perm[j] the column of step j.
__device__ __forceinline__ int wave_pchol(const c128* Gg, int k, int kmax, c128* Rg, int* permg, int* posg,
                                          double delta) {
    lds<c128>* G = to_lds(const_cast<c128*>(Gg));
    lds<c128>* Rr = to_lds(Rg);
    lds<int>* perm = to_lds(permg);
    lds<int>* pos = to_lds(posg);
    const int lane = threadIdx.x & 63;
    // with k <= 32 two lanes share a column and split its dot products
    // (even and odd rows); both then hold the same values
    const bool two = k <= 32;
    const int c = two ? lane >> 1 : lane;
    const int h = two ? lane & 1 : 0;
    const int hs = two ? 2 : 1;
    const bool col = c < k;
    const int cc = col ? c : 0;
    double d = col ? ldc(G + (size_t)cc * k + cc).re : -1.0;
    double mx = d;
    int unused = lane;
    wops::argmax(mx, unused);
    const double stop = delta * delta * mx;
    bool chosen = !col;
    int kr = kmax;
    for (int j = 0; j < kmax; ++j) {
        const int p = wops::argmax_nonneg((float)d, c, !chosen && h == 0);
        const double key = p >= 0 ? readlane_f(d, p * hs) : -1.0;   // exact Schur diagonal of the pivot
        if (!(key > stop)) { kr = j; break; }
        const double ir = rsq_nr(key);
        const double rpp = key * ir;
        c128 val = ldc(G + (size_t)cc * k + p);          // G[p][c]
        // this lane's share of the dot over the rows so far (rows h, h + hs,
        // ...) in chunks of 4, one accumulator per chunk position; all 8 loads
        // are in flight before the first use.  Rows j and beyond are still
        // zero (cleared before the factorization, PCHOL_PAD rows of padding
        // past kmax), so a chunk that runs past row j - 1 adds nothing.
        c128 s0 = czero<double>(), s1 = s0, s2 = s0, s3 = s0;
        for (int t0 = h; t0 < j; t0 += 4 * hs) {
            c128 ap[4], ac[4];
            const lds<c128>* rt = Rr + (size_t)t0 * k;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                ap[u] = ldc(rt + (size_t)u * hs * k + p);
                ac[u] = ldc(rt + (size_t)u * hs * k + cc);
            }
            __builtin_amdgcn_sched_barrier(0);
            cfma_conj(s0, ap[0], ac[0]);
            cfma_conj(s1, ap[1], ac[1]);
            cfma_conj(s2, ap[2], ac[2]);
            cfma_conj(s3, ap[3], ac[3]);
        }
        c128 sd = (s0 + s1) + (s2 + s3);
        if (two) {
            // add the partner lane's share (the sum is the same on both lanes)
            sd.re += wops::dpp<wops::QP_XOR1>(sd.re, 0.0);
            sd.im += wops::dpp<wops::QP_XOR1>(sd.im, 0.0);
        }
        val -= sd;
        c128 r = chosen ? czero<double>() : (c == p ? mk(rpp, 0.0) : ir * val);
        if (!chosen && c != p) d -= abs2(r);
        if (col && h == 0) stc(Rr + (size_t)j * k + c, r);
        if (lane == 0) {
            perm[j] = p;
            pos[p] = j;
        }
        if (c == p) chosen = true;
        wave_sync();
    }
    if (col && h == 0 && !chosen) pos[c] = k;
    wave_sync();
    return kr;
}

// ----------------------------------------------------------------------------
// Recompression of the off-diagonal blocks of S_m.
struct RecompLayout {
    int s, k, kk, r;
    int lda, ldy;                                // padded leading dimensions of U, V and Y1, Y2
    size_t oU, oV, oY1, oY2, oV0u, oV0v, oEnd;   // cpx<T> units
    size_t dN, dJ, dS, dEnd;                     // cpx<CT> units (after oEnd)
    size_t gGu, gGv, gRu, gRv, gYu, gYv, gEnd;   // c128 units (after dEnd; Gram path only)
    size_t gTu, gTv;                             // inverses of R11 (Gram path, when they fit)
    bool tinv;
};

// LDS bound up to which the Gram path also keeps the two R11 inverses
constexpr size_t TINV_LDS_MAX = 150 * 1024;

// The Gram path (complex64 factors, truncation on, k <= GRAM_KMAX) replaces
// the Householder QR of the stacked factors by a pivoted Cholesky of their
// FP64 Gram matrices.
constexpr int GRAM_KMAX = 40;
// zero rows after the kmax Cholesky rows: the row loop reads up to 3 row
// strides (of at most 2 rows) past its last live row
constexpr int PCHOL_PAD = 8;
__host__ __device__ inline bool gram_path(size_t elem, double tol, int k) {
    return elem == sizeof(c64) && tol > 0.0 && k <= GRAM_KMAX;
}

// elem = sizeof(cpx<T>), celem = sizeof(cpx<CT>) of the core's type
__host__ __device__ inline RecompLayout recomp_layout(int s, int k, int r, int Xblocks, size_t elem, size_t celem,
                                                      bool gram) {
    RecompLayout l;
    l.s = s; l.k = k; l.r = r;
    l.kk = s < k ? s : k;
    // columns padded by the lane-group size of the wavefront routines, so the
    // groups' loads of one row fall on different LDS banks
    int pk = 1, pr = 1;
    while (pk < k) pk <<= 1;
    while (pr < (r / 2 > 0 ? r / 2 : 1)) pr <<= 1;
    l.lda = s + 64 / pk;
    l.ldy = s + 64 / pr;
    size_t o = 0;
    l.oU = o; o += (size_t)l.lda * k;
    l.oV = o; o += (size_t)l.lda * k;
    l.oY1 = o; o += (size_t)l.ldy * r;
    l.oY2 = o; o += (size_t)l.ldy * r;
    l.oV0u = o; o += l.kk;
    l.oV0v = o; o += l.kk;
    o += (size_t)Xblocks;                  // staged X blocks
    l.oEnd = o;
    // core N (nr <= kk rows) and rotations J, both P columns of jacobi_ld(nr, P)
    // entries (P <= kk + 1), then P squared norms
    size_t bytes = o * elem;
    bytes = (bytes + 15) / 16 * 16;
    size_t nj = 0;
    for (int P = 2; P <= l.kk + 1; P += 2) {
        const size_t e = (size_t)jacobi_ld(l.kk, P) * P;
        nj = e > nj ? e : nj;
    }
    l.dN = bytes / celem;
    l.dJ = l.dN + nj;
    l.dS = l.dJ + nj;
    l.dEnd = l.dS + (size_t)(l.kk + 2);
    // Gram path: the Gram matrices (k x k each) are dead once the Cholesky is
    // done and overlay the core area (N, J), which is written after it; the
    // dense pivot-ordered R11 blocks of the back substitution (kk x kk each)
    // overlay it again once the core is read.  Then Cholesky rows (kk x k)
    // and FP64 output blocks (kk x r).
    const size_t g0 = (bytes + 15) / 16;                          // start of the core area, c128 units
    size_t g = (l.dEnd * celem + 15) / 16;
    l.gGu = g0;
    l.gGv = g0 + (size_t)k * k;
    if (gram) {
        const size_t over = g0 + 2 * (size_t)k * k;
        g = over > g ? over : g;
    }
    // Cholesky rows, with PCHOL_PAD zero rows past the last so that the
    // row loop of wave_pchol reads in blocks without bounds tests
    l.gRu = g; if (gram) g += (size_t)(l.kk + PCHOL_PAD) * k;
    l.gRv = g; if (gram) g += (size_t)(l.kk + PCHOL_PAD) * k;
    l.gYu = g; if (gram) g += (size_t)l.kk * r;
    l.gYv = g; if (gram) g += (size_t)l.kk * r;
    l.tinv = gram && (g + 2 * (size_t)l.kk * l.kk) * sizeof(c128) <= TINV_LDS_MAX;
    l.gTu = g; if (l.tinv) g += (size_t)l.kk * l.kk;
    l.gTv = g; if (l.tinv) g += (size_t)l.kk * l.kk;
    l.gEnd = g;
    return l;
}

template <typename T, int R>
__device__ __forceinline__ void recompress_job(const Plan& p, const StepPtrs<T>& sp, int m, int pj,
                                               unsigned char* smem) {
    using CT = T;                                // core SVD in the factor precision
    __shared__ T tau_u[72], tau_v[72];
    __shared__ int perm_u[72], perm_v[72], pos_u[72], pos_v[72];
    __shared__ int order[72];
    __shared__ int rank_s, kr_u, kr_v;
    const int lp = 31 - __clz(pj + 1);           // pj: heap id of the parent node
    const int j = pj - ((1 << lp) - 1);
    const int lam = lp + 1;
    const int s = p.np >> lam;
    const int np = p.np;
    const int k = 1 + (m > 0 ? R * lam : 0);
    const int lo1 = 2 * j * s, lo2 = (2 * j + 1) * s;
    const int nX = m > 0 ? lam * R * R : 0;
    const bool gram = gram_path(sizeof(cpx<T>), p.tol, k);
    RecompLayout ly = recomp_layout(s, k, R, nX, sizeof(cpx<T>), sizeof(cpx<CT>), gram);
    cpx<T>* base = (cpx<T>*)smem;
    cpx<T>* Ut = base + ly.oU;
    cpx<T>* Vt = base + ly.oV;
    cpx<T>* Y1 = base + ly.oY1;
    cpx<T>* Y2 = base + ly.oY2;
    cpx<T>* Xs = base + ly.oEnd - nX;          // [blk][k1][k2]
    cpx<CT>* Nm = (cpx<CT>*)smem + ly.dN;
    cpx<CT>* Jm = (cpx<CT>*)smem + ly.dJ;
    CT* nrm2 = (CT*)((cpx<CT>*)smem + ly.dS);
    c128* GU = (c128*)smem + ly.gGu;
    c128* GV = (c128*)smem + ly.gGv;
    c128* RU = (c128*)smem + ly.gRu;
    c128* RV = (c128*)smem + ly.gRv;
    c128* YU = (c128*)smem + ly.gYu;
    c128* YV = (c128*)smem + ly.gYv;
    c128* TU = (c128*)smem + ly.gTu;
    c128* TV = (c128*)smem + ly.gTv;
    const int tid = threadIdx.x, wv = tid >> 6;
    const int lda = ly.lda, ldy = ly.ldy;

    // Stacked factors: S_m(c1, c2) = Ut Vt^t.
    //   column 0:          A_{m,m}(last of c1, first of c2) e_last e_first^t
    //   block 0 (cols 1..r): D P_lam[c1] X_pj(first block row, second block col) | D P_lam[c2]
    //   block b >= 1:      ancestor level l' = lam - b:  D P_l'[c1] X_q'(sg, sg)  | D P_l'[c2]
    for (int e = tid; e < nX; e += NT) {
        const int k2 = e % R, k1 = (e / R) % R, blk = e / (R * R);
        const cpx<T>* Xq;
        int rowoff, coloff;
        if (blk == 0) {
            Xq = sp.Xp + (size_t)pj * 4 * R * R;
            rowoff = 0; coloff = R;
        } else {
            const int lv = lam - blk;
            const int a = (2 * j) >> (lam - lv);
            Xq = sp.Xp + (size_t)heap_id(lv - 1, a >> 1) * 4 * R * R;
            rowoff = (a & 1) * R; coloff = rowoff;
        }
        Xs[e] = Xq[(size_t)(coloff + k2) * 2 * R + rowoff + k1];
    }
    for (int i = tid; i < s; i += NT) {
        Ut[i] = (i == s - 1) ? sp.eo[lo1 + s - 1] : czero<T>();
        Vt[i] = (i == 0) ? mk<T>(T(1), T(0)) : czero<T>();
    }
    __syncthreads();
    if (m > 0) {
        for (int e = tid; e < lam * s; e += NT) {
            const int i = e % s, blk = e / s;
            const int lv = lam - blk;
            const cpx<T>* Pv = sp.Pp + (size_t)(lv - 1) * R * np;
            cpx<T> pu[R], pv[R];
#pragma unroll
            for (int kk = 0; kk < R; ++kk) {
                pu[kk] = Pv[(size_t)kk * np + lo1 + i];
                pv[kk] = Pv[(size_t)kk * np + lo2 + i];
            }
            const cpx<T> d1 = sp.cp[lo1 + i], d2 = sp.cp[lo2 + i];
            const cpx<T>* xb = Xs + (size_t)blk * R * R;
#pragma unroll
            for (int k2 = 0; k2 < R; ++k2) {
                cpx<T> acc = czero<T>();
#pragma unroll
                for (int k1 = 0; k1 < R; ++k1) cfma(acc, pu[k1], xb[k1 * R + k2]);
                const int col = 1 + blk * R + k2;
                Ut[(size_t)col * lda + i] = d1 * acc;
                Vt[(size_t)col * lda + i] = d2 * pv[k2];
            }
        }
    }
    __syncthreads();

    // rank-revealing QR of both factors, one wavefront each, concurrently.
    // The cut is far below the truncation tolerance (none when nothing is
    // truncated); in complex64 at the level of the factors' own rounding.
    const T delta = p.tol <= 0.0 ? T(0) : (sizeof(T) == 4 ? T(4.0e-7) : T(1.0e-5 * p.tol < 1.0e-11 ? 1.0e-5 * p.tol : 1.0e-11));
    if (gram) {
        // Gram path: FP64 Gram matrices, then pivoted Cholesky (waves 0 and 1)
        gram_pair(Ut, Vt, s, lda, k, GU, GV);
        {
            // rows of R not yet formed read as zero in wave_pchol's dot products
            const int nz = (ly.kk + PCHOL_PAD) * k;
            for (int e = tid; e < 2 * nz; e += NT) (e < nz ? RU : RV)[e < nz ? e : e - nz] = czero<double>();
        }
        __syncthreads();
        if (wv < 2) {
            const bool w1 = wv == 1;
            const int kr = wave_pchol(w1 ? GV : GU, k, ly.kk, w1 ? RV : RU, w1 ? perm_v : perm_u,
                                      w1 ? pos_v : pos_u, (double)delta);
            if ((tid & 63) == 0) (w1 ? kr_v : kr_u) = kr;
        }
    } else if (wv < 2) {                        // one call site: wave 0 on Ut, wave 1 on Vt
        const bool w1 = wv == 1;
        const int kr = wave_qrcp(w1 ? Vt : Ut, lda, s, k, w1 ? perm_v : perm_u, w1 ? pos_v : pos_u,
                                 base + (w1 ? ly.oV0v : ly.oV0u), w1 ? tau_v : tau_u, delta);
        if ((tid & 63) == 0) (w1 ? kr_v : kr_u) = kr;
    }
    __syncthreads();
    const int k1 = kr_u, k2 = kr_v;

    // core M = (R1 Pi1^t)(R2 Pi2^t)^t (k1 x k2).  The SVD works on the
    // orientation with fewer columns: N = M (k2 <= k1) or N = M^H (k1 < k2).
    const bool tr = k1 < k2;
    const int nr = tr ? k2 : k1;
    const int ncl = tr ? k1 : k2;
    const int P = ncl + (ncl & 1);
    const int ldn = P > 0 ? jacobi_ld(nr, P) : 0;   // rows nr.. ldn-1 are zero padding
    for (int e = tid; e < ldn * P; e += NT) {
        const int row = e % ldn, col = e / ldn;
        cpx<CT> v = czero<CT>();
        if (gram && col < ncl && row < nr) {
            const int a = tr ? col : row;
            const int b = tr ? row : col;
            const lds<c128>* ra = to_lds(RU) + (size_t)a * k;
            const lds<c128>* rb = to_lds(RV) + (size_t)b * k;
            c128 w0 = czero<double>(), w1 = w0;
            int c = 0;
            for (; c + 2 <= k; c += 2) {
                cfma(w0, ldc(ra + c), ldc(rb + c));
                cfma(w1, ldc(ra + c + 1), ldc(rb + c + 1));
            }
            if (c < k) cfma(w0, ldc(ra + c), ldc(rb + c));
            const c128 w = w0 + w1;
            v = ccast<CT>(tr ? conj(w) : w);
        } else if (col < ncl && row < nr) {
            const int a = tr ? col : row;      // row of M (U side)
            const int b = tr ? row : col;      // column of M (V side)
            const lds<cpx<T>>* Ua = to_lds(Ut) + a;
            const lds<cpx<T>>* Vb = to_lds(Vt) + b;
#pragma unroll 8
            for (int c = 0; c < k; ++c) {            // branch-free so the loads pipeline
                const cpx<T> x = ldc(Ua + (size_t)c * lda), y = ldc(Vb + (size_t)c * lda);
                const bool on = pos_u[c] >= a && pos_v[c] >= b;
                cfma(v, on ? ccast<CT>(x) : czero<CT>(), ccast<CT>(y));
            }
            if (tr) v = conj(v);
        }
        Nm[(size_t)col * ldn + row] = v;
    }
    __syncthreads();
    if (wv == 0) {
        // Frobenius norm (fixed-order wave sum), then Jacobi
        CT f = CT(0);
        for (int e = tid; e < ldn * P; e += 64) f += abs2(Nm[e]);
        f = wops::sum(f);
        const CT eps = eps_of<CT>();
        const CT thr = sizeof(CT) == 4 ? CT(1.0e-6) : CT(1.0e-12);
        const CT tiny = f * eps * eps * CT(1e-2) + (sizeof(CT) == 4 ? CT(1e-37) : CT(1e-300));
        // inner products below a tenth of the truncation level of the squared
        // norms are left alone: they move no column norm by more than that
        const CT gabs = CT(0.1 * (p.tol > 0.0 ? p.tol : 0.0)) * f;
        if (P > 0) wave_jacobi<CT>(Nm, P, jacobi_rows(nr, P), Jm, nrm2, thr, gabs, tiny, 40);
        // selection: rank of each column by decreasing norm (ties: lower index first)
        const int lane = tid;
        CT mine = CT(-1);
        int rk = 64;
        if (lane < P) {
            mine = nrm2[lane];
            rk = 0;
            for (int c = 0; c < P; ++c) {
                const CT o = nrm2[c];
                rk += (o > mine || (o == mine && c < lane)) ? 1 : 0;
            }
            if (rk < R) order[rk] = lane;
        }
        CT s1 = mine;
        int unused = lane;
        wops::argmax(s1, unused);
        const CT t2 = CT(p.tol) * CT(p.tol);
        const bool keep = lane < P && rk < R && s1 > CT(0) && mine > t2 * s1 && mine > CT(0);
        const unsigned long long bal = __ballot(keep);
        if (lane == 0) rank_s = __popcll(bal);
    } else if (ly.tinv && wv <= 2) {
        // meanwhile waves 1 and 2 invert the triangular R11 of each side in
        // FP64 (R11(j, t) = R(j, perm(t)), t >= j; inverse upper triangular,
        // row-major, leading dimension kk): lane c forms column c, row by row
        // upwards from the diagonal, from its own earlier entries
        const bool sv = wv == 2;
        const int kr = sv ? k2 : k1;
        const int* pm = sv ? perm_v : perm_u;
        const lds<c128>* Rm = to_lds(sv ? RV : RU);
        lds<c128>* Tm = to_lds(sv ? TV : TU);
        const int c = tid & 63, kk = ly.kk;
        for (int jj = kr - 1; jj >= 0; --jj) {
            const double idg = 1.0 / ldc(Rm + (size_t)jj * k + pm[jj]).re;
            if (c >= jj && c < kr) {
                c128 a0 = c == jj ? mk<double>(1.0, 0.0) : czero<double>(), a1 = czero<double>();
                int mm = jj + 1;
                for (; mm + 2 <= c + 1; mm += 2) {
                    a0 -= ldc(Rm + (size_t)jj * k + pm[mm]) * ldc(Tm + (size_t)mm * kk + c);
                    a1 -= ldc(Rm + (size_t)jj * k + pm[mm + 1]) * ldc(Tm + (size_t)(mm + 1) * kk + c);
                }
                if (mm <= c) a0 -= ldc(Rm + (size_t)jj * k + pm[mm]) * ldc(Tm + (size_t)mm * kk + c);
                stc(Tm + (size_t)jj * kk + c, idg * (a0 + a1));
            }
        }
    }
    __syncthreads();
    const int rho = rank_s;

    // M = W S Z^H.  If N = M: N J = W S, Z = J.  If N = M^H: N J = Z S, W = J.
    // U = Q1 [W sqrt(S); 0],  V = Q2 [conj(Z) sqrt(S); 0]
    for (int e = tid; e < s * R; e += NT) {
        const int i = e % s, q = e / s;
        cpx<CT> u = czero<CT>(), v = czero<CT>();
        if (q < rho && (i < k1 || i < k2)) {
            const int c = order[q];
            const CT sq = sqrt(sqrt(nrm2[c]));            // sqrt of the singular value
            const CT isq = CT(1) / sq;
            if (i < k1) u = tr ? sq * Jm[(size_t)c * ldn + i] : isq * Nm[(size_t)c * ldn + i];
            if (i < k2) v = tr ? isq * conj(Nm[(size_t)c * ldn + i]) : sq * conj(Jm[(size_t)c * ldn + i]);
        }
        if (gram) {
            if (i < ly.kk) {
                YU[(size_t)q * ly.kk + i] = ccast<double>(u);
                YV[(size_t)q * ly.kk + i] = ccast<double>(v);
            }
        } else {
            Y1[(size_t)q * ldy + i] = ccast<T>(u);
            Y2[(size_t)q * ldy + i] = ccast<T>(v);
        }
    }
    __syncthreads();
    if (gram && ly.tinv) {
        // U_new = U Pi[:, :k1] (R11^-1 Y): Z = R11^-1 Y from the inverse formed
        // during the Jacobi (over the dead core area, same layout as Y), then
        // the product below
        for (int e = tid; e < 2 * R * ly.kk; e += NT) {
            const bool sv = e >= R * ly.kk;
            const int ee = sv ? e - R * ly.kk : e;
            const int q = ee / ly.kk, tt = ee % ly.kk;
            const int kr = sv ? k2 : k1;
            const lds<c128>* Tm = to_lds(sv ? TV : TU) + (size_t)tt * ly.kk;
            const lds<c128>* y = to_lds(sv ? YV : YU) + (size_t)q * ly.kk;
            c128 a0 = czero<double>(), a1 = czero<double>();
            if (q < rho && tt < kr) {
                int mm = tt;
                for (; mm + 2 <= kr; mm += 2) {
                    cfma(a0, ldc(Tm + mm), ldc(y + mm));
                    cfma(a1, ldc(Tm + mm + 1), ldc(y + mm + 1));
                }
                if (mm < kr) cfma(a0, ldc(Tm + mm), ldc(y + mm));
            }
            stc(to_lds(GU + (sv ? (size_t)R * ly.kk : 0)) + ee, a0 + a1);
        }
    } else if (gram) {
        // U_new = U Pi[:, :k1] R11^-1 Y: back substitution in place, then the
        // product with FP64 accumulation, which cancels the conditioning of R11
        // (U_new = Q1 Y with Q1 orthonormal).  R11 is first gathered densely in
        // pivot order (over the dead core area) so every load is independent.
        c128* D1 = GU;                                   // k1 x k1, row-major [jj][t]
        c128* D2 = GU + (size_t)ly.kk * ly.kk;           // k2 x k2
        for (int e = tid; e < k1 * k1 + k2 * k2; e += NT) {
            const bool sv = e >= k1 * k1;
            const int ee = sv ? e - k1 * k1 : e, kr = sv ? k2 : k1;
            const int jj = ee / kr, t = ee % kr;
            const int* pm = sv ? perm_v : perm_u;
            (sv ? D2 : D1)[(size_t)jj * kr + t] = (sv ? RV : RU)[(size_t)jj * k + pm[t]];
        }
        __syncthreads();
        if (tid < 2 * R) {
            const bool sv = tid >= R;
            const int q = tid % R;
            const int kr = sv ? k2 : k1;
            const lds<c128>* Dm = to_lds(sv ? D2 : D1);
            lds<c128>* z = to_lds((sv ? YV : YU) + (size_t)q * ly.kk);
            if (q < rho) {
                for (int jj = kr - 1; jj >= 0; --jj) {
                    c128 a0 = ldc(z + jj), a1 = czero<double>();
                    int t = jj + 1;
                    for (; t + 2 <= kr; t += 2) {
                        const c128 r0 = ldc(Dm + (size_t)jj * kr + t), r1 = ldc(Dm + (size_t)jj * kr + t + 1);
                        const c128 z0 = ldc(z + t), z1 = ldc(z + t + 1);
                        a0 -= r0 * z0;
                        a1 -= r1 * z1;
                    }
                    if (t < kr) a0 -= ldc(Dm + (size_t)jj * kr + t) * ldc(z + t);
                    stc(z + jj, (1.0 / ldc(Dm + (size_t)jj * kr + jj).re) * (a0 + a1));
                }
            }
        }
    }
    if (gram) {
        __syncthreads();
        // one thread per row and side, all output columns: the Z entries are
        // broadcast loads, the row's U entries one load per pivot
        for (int e = tid; e < 2 * s; e += NT) {
            const bool sv = e >= s;
            const int i = sv ? e - s : e;
            const int kr = sv ? k2 : k1;
            const int* pm = sv ? perm_v : perm_u;
            const lds<cpx<T>>* X = to_lds(sv ? Vt : Ut) + i;
            const lds<c128>* z = ly.tinv ? to_lds(GU + (sv ? (size_t)R * ly.kk : 0)) : to_lds(sv ? YV : YU);
            c128 acc[R];
#pragma unroll
            for (int q = 0; q < R; ++q) acc[q] = czero<double>();
            for (int t = 0; t < kr; ++t) {
                const c128 x = ccast<double>(ldc(X + (size_t)pm[t] * lda));
#pragma unroll
                for (int q = 0; q < R; ++q) cfma(acc[q], x, ldc(z + (size_t)q * ly.kk + t));
            }
            cpx<T>* Yo = sv ? Y2 : Y1;
#pragma unroll
            for (int q = 0; q < R; ++q) Yo[(size_t)q * ldy + i] = q < rho ? ccast<T>(acc[q]) : czero<T>();
        }
        __syncthreads();
    } else {
        // waves 0, 1: Q1 on the two halves of Y1's columns; waves 2, 3: Q2 on Y2
        constexpr int H = R / 2 > 0 ? R / 2 : 1;
        const int c0 = (wv & 1) * H;
        int nc = rho - c0;
        nc = nc < 0 ? 0 : (nc > H ? H : nc);
        const bool sv = wv >= 2;
        wave_apply_q(sv ? Vt : Ut, lda, s, sv ? k2 : k1, sv ? perm_v : perm_u, base + (sv ? ly.oV0v : ly.oV0u),
                     sv ? tau_v : tau_u, (sv ? Y2 : Y1) + (size_t)c0 * ldy, ldy, nc);
        __syncthreads();
    }
    cpx<T>* Qv = sp.Q + (size_t)(lam - 1) * R * np;
    for (int e = tid; e < s * R; e += NT) {
        const int i = e % s, q = e / s;
        Qv[(size_t)q * np + lo1 + i] = Y1[(size_t)q * ldy + i];
        Qv[(size_t)q * np + lo2 + i] = Y2[(size_t)q * ldy + i];
    }
    if (tid == 0) sp.rank[pj] = rho;
}

// One launch per layer for the two independent parts of forming S_m: blocks
// [0, 2^L - 1) recompress the off-diagonal blocks, the next 2^L blocks form
// and invert the dense leaves.
template <typename T>
__device__ __forceinline__ StepPtrs<T> step_ptrs(const InstDesc<T>& d, int m) {
    const Plan& p = d.p;
    StepPtrs<T> sp;
    cpx<T>* cur = d.fac + (size_t)m * p.eLayer;
    sp.K = cur; sp.P = cur + p.eK; sp.X = cur + p.eK + p.eP;
    if (m > 0) {
        const cpx<T>* prev = d.fac + (size_t)(m - 1) * p.eLayer;
        sp.Kp = prev; sp.Pp = prev + p.eK; sp.Xp = prev + p.eK + p.eP;
        sp.cp = d.cp + (size_t)(m - 1) * p.np;
    } else {
        sp.Kp = sp.Pp = sp.Xp = nullptr;
        sp.cp = nullptr;
    }
    sp.dg = d.dg + (size_t)m * p.np;
    sp.eo = d.eo + (size_t)m * p.np;
    sp.Q = d.Q;
    sp.G = d.G;
    sp.rank = d.rank + (size_t)m * (1 << p.L);
    sp.status = d.status;
    return sp;
}

template <typename T, int B, int R>
__global__ __launch_bounds__(NT) void layer_kernel(const InstDesc<T>* __restrict__ descs, int m) {
    extern __shared__ __align__(16) unsigned char smem[];
    const InstDesc<T> d = descs[blockIdx.y];
    const Plan& p = d.p;
    if (m >= p.n) return;
    const int nrec = p.L > 0 ? (1 << p.L) - 1 : 0;
    if ((int)blockIdx.x >= nrec + (1 << p.L)) return;
    const StepPtrs<T> sp = step_ptrs(d, m);
    if ((int)blockIdx.x < nrec) {
        if constexpr (R >= 2) recompress_job<T, R>(p, sp, m, blockIdx.x, smem);
    } else {
        leaf_job<T, B, R>(p, sp, m, blockIdx.x - nrec, smem);
    }
}

// ----------------------------------------------------------------------------
// Core inverse of a node from its children's G blocks, by one wavefront.
// With A = G_c1 and B = G_c2 (R x R, row-major),
//     [[A, I], [I, B]]^{-1} = [[-B W, I + B W A], [W, -W A]],  W = (I - A B)^{-1},
// which multiplies out to the identity directly; so one R x R Gauss-Jordan
// inverse (partial pivoting) replaces the 2R x 2R one, halving the pivot
// steps on the factorization's critical path.  Scratch: 5 R^2 LDS entries.
// Out receives the 2R x 2R inverse column-major.
template <typename T>
__device__ __forceinline__ void put_c(lds<cpx<T>>* p, cpx<T> v) { stc(p, v); }
template <typename T>
__device__ __forceinline__ void put_c(cpx<T>* p, cpx<T> v) { *p = v; }

template <typename T, int R, typename OutP>
__device__ __forceinline__ void wood_core(const cpx<T>* G1, const cpx<T>* G2, lds<cpx<T>>* scr, OutP Out,
                                          int* perm_w, int* status) {
    constexpr int RR = R * R, R2 = 2 * R;
    constexpr int NL = (2 * RR + 63) / 64;
    const int lane = threadIdx.x & 63;
    lds<cpx<T>>* A = scr;              // row-major A, then B
    lds<cpx<T>>* Bm = scr + RR;
    lds<cpx<T>>* E = scr + 2 * RR;     // I - A B (column-major), later B W (row-major)
    lds<cpx<T>>* Wc = scr + 3 * RR;    // W (column-major)
    lds<cpx<T>>* WA = scr + 4 * RR;    // W A (row-major)
    {
        cpx<T> v[NL];
#pragma unroll
        for (int u = 0; u < NL; ++u) {
            const int e = min(lane + 64 * u, 2 * RR - 1);
            v[u] = e < RR ? G1[e] : G2[e - RR];
        }
#pragma unroll
        for (int u = 0; u < NL; ++u)
            if (lane + 64 * u < 2 * RR) stc(A + lane + 64 * u, v[u]);
    }
    wave_sync();
    for (int e = lane; e < RR; e += 64) {
        const int r = e % R, c = e / R;
        cpx<T> a = mk<T>(r == c ? T(1) : T(0), T(0));
#pragma unroll
        for (int t = 0; t < R; ++t) a -= ldc(A + r * R + t) * ldc(Bm + t * R + c);
        stc(E + e, a);
    }
    wave_sync();
    if constexpr (R == 8 || R == 16 || R == 32) gj_cols<T, R>((const cpx<T>*)E, R, (cpx<T>*)Wc, R, status);
    else gj_wave<T, R>((const cpx<T>*)E, R, (cpx<T>*)Wc, R, perm_w, status);
    wave_sync();
    for (int e = lane; e < RR; e += 64) {
        const int r = e / R, c = e % R;
        cpx<T> bw = czero<T>(), wa = czero<T>();
#pragma unroll
        for (int t = 0; t < R; ++t) {
            cfma(bw, ldc(Bm + r * R + t), ldc(Wc + c * R + t));
            cfma(wa, ldc(Wc + t * R + r), ldc(A + t * R + c));
        }
        stc(E + e, bw);
        stc(WA + e, wa);
    }
    wave_sync();
    for (int e = lane; e < 4 * RR; e += 64) {
        const int r = e % R2, c = e / R2;
        cpx<T> x;
        if (r < R && c < R) x = -ldc(E + r * R + c);
        else if (r >= R && c < R) x = ldc(Wc + c * R + (r - R));
        else if (r >= R) x = -ldc(WA + (r - R) * R + (c - R));
        else {
            x = mk<T>(r == c - R ? T(1) : T(0), T(0));
#pragma unroll
            for (int t = 0; t < R; ++t) cfma(x, ldc(E + r * R + t), ldc(A + t * R + (c - R)));
        }
        put_c(Out + e, x);
    }
}

// ----------------------------------------------------------------------------
// Woodbury step for the nodes of level lam (lam = 0: root core only).
struct WoodLayout {
    size_t oQ, oY, oPart, oYs, oZs, oEnd;
};

__host__ __device__ inline WoodLayout wood_layout(int s, int r, int b, int L, int lam) {
    WoodLayout w;
    size_t o = 0;
    w.oQ = o; o += (size_t)s * r;
    w.oY = o; o += (size_t)s * r;
    w.oPart = o; o += (size_t)(s / b > 0 ? s / b : 1) * r * r;
    const int nodes = lam < L ? (1 << (L - lam)) : 1;   // children at the finest level inside the node
    w.oYs = o; o += (size_t)nodes * r * r;
    w.oZs = o; o += (size_t)nodes * r * r;
    w.oEnd = o;
    return w;
}

template <typename T, int B, int R>
__global__ __launch_bounds__(NT) void wood_kernel(const InstDesc<T>* __restrict__ descs, int m, int lam) {
    constexpr int R2 = 2 * R;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int perm_w[R2];
    const InstDesc<T> d = descs[blockIdx.y];
    const Plan& p = d.p;
    if (m >= p.n || p.L == 0 || lam > p.L || (int)blockIdx.x >= (1 << lam)) return;
    const StepPtrs<T> sp = step_ptrs(d, m);
    const int L = p.L, np = p.np;
    const int ci = blockIdx.x;
    const int node = heap_id(lam, ci);
    const int s = p.np >> lam;
    const int lo = ci * s;
    const int tid = threadIdx.x;

    // (a) core inverse of this node from its children's G blocks, by wavefront 0
    if (lam < L) {
        if (tid < 64)
            wood_core<T, R>(sp.G + (size_t)heap_id(lam + 1, 2 * ci) * R * R,
                            sp.G + (size_t)heap_id(lam + 1, 2 * ci + 1) * R * R, to_lds((cpx<T>*)smem),
                            sp.X + (size_t)node * 4 * R * R, perm_w, sp.status);
        __syncthreads();
    }
    if (lam == 0) return;

    WoodLayout wl = wood_layout(s, R, B, L, lam);
    cpx<T>* base = (cpx<T>*)smem;
    cpx<T>* Qc = base + wl.oQ;     // [i*R + k]
    cpx<T>* Y = base + wl.oY;      // [i*R + k]
    cpx<T>* part = base + wl.oPart;
    cpx<T>* ys = base + wl.oYs;
    cpx<T>* zs = base + wl.oZs;
    const cpx<T>* Qv = sp.Q + (size_t)(lam - 1) * R * np;
    for (int i = tid; i < s; i += NT) {
#pragma unroll
        for (int k = 0; k < R; ++k) Qc[i * R + k] = Qv[(size_t)k * np + lo + i];
    }
    __syncthreads();
    // (b1) leaf part: Y = K Qc, one row per thread
    for (int i = tid; i < s; i += NT) {
        const int gi = lo + i;
        const int il = gi % B;
        const cpx<T>* Kt = sp.K + (size_t)(gi / B) * B * B + il;
        cpx<T> kr[B];
#pragma unroll
        for (int jj = 0; jj < B; ++jj) kr[jj] = Kt[(size_t)jj * B];
        const cpx<T>* qb = Qc + (size_t)(i - il) * R;
        cpx<T> acc[R];
#pragma unroll
        for (int k = 0; k < R; ++k) acc[k] = czero<T>();
#pragma unroll
        for (int jj = 0; jj < B; ++jj)
#pragma unroll
            for (int k = 0; k < R; ++k) cfma(acc[k], kr[jj], qb[jj * R + k]);
#pragma unroll
        for (int k = 0; k < R; ++k) Y[i * R + k] = acc[k];
    }
    __syncthreads();
    // (b2) corrections of the nodes inside this node: child levels lc = lam+1 .. L
    const int nch = s / B;     // leaf-size chunks in the node
    for (int lc = lam + 1; lc <= L; ++lc) {
        const int sc = np >> lc;                  // child size
        const int ncn = s / sc;                   // children at level lc inside this node
        const int cpn = sc / B;                   // chunks per child
        const cpx<T>* Pv = sp.P + (size_t)(lc - 1) * R * np;
        // chunk partials of P^t Qc: task (chunk, k1) -> R outputs
        for (int e = tid; e < nch * R; e += NT) {
            const int ch = e % nch, k1 = e / nch;
            const cpx<T>* pc = Pv + (size_t)k1 * np + lo + ch * B;
            cpx<T> pv[B];
#pragma unroll
            for (int jj = 0; jj < B; ++jj) pv[jj] = pc[jj];
            cpx<T> acc[R];
#pragma unroll
            for (int k2 = 0; k2 < R; ++k2) acc[k2] = czero<T>();
#pragma unroll
            for (int jj = 0; jj < B; ++jj)
#pragma unroll
                for (int k2 = 0; k2 < R; ++k2) cfma(acc[k2], pv[jj], Qc[(ch * B + jj) * R + k2]);
#pragma unroll
            for (int k2 = 0; k2 < R; ++k2) part[(k1 * R + k2) * nch + ch] = acc[k2];
        }
        __syncthreads();
        for (int e = tid; e < ncn * R * R; e += NT) {
            const int c = e / (R * R), kk = e % (R * R);
            cpx<T> acc = czero<T>();
            for (int q = 0; q < cpn; ++q) acc += part[kk * nch + c * cpn + q];
            ys[c * R * R + kk] = acc;             // ys[c][k1][k2]
        }
        __syncthreads();
        // z_parent = X_parent [y_left; y_right]  (2R x R) for the parents at level lc-1
        const int npar = ncn / 2;
        for (int e = tid; e < npar * R2 * R; e += NT) {
            const int q = e / (R2 * R), o = (e / R) % R2, k2 = e % R;
            const int gq = (lo / (2 * sc)) + q;   // parent index at level lc-1
            const cpx<T>* Xq = sp.X + (size_t)heap_id(lc - 1, gq) * 4 * R * R + o;
            cpx<T> xr[R2];
#pragma unroll
            for (int c = 0; c < R2; ++c) xr[c] = Xq[(size_t)c * R2];
            cpx<T> acc = czero<T>();
#pragma unroll
            for (int c = 0; c < R2; ++c) cfma(acc, xr[c], ys[(2 * q + c / R) * R * R + (c % R) * R + k2]);
            zs[(q * R2 + o) * R + k2] = acc;
        }
        __syncthreads();
        for (int i = tid; i < s; i += NT) {
            const int c = i / sc;
            const int q = c >> 1, sg = c & 1;
            cpx<T> pr[R];
#pragma unroll
            for (int k1 = 0; k1 < R; ++k1) pr[k1] = Pv[(size_t)k1 * np + lo + i];
            const cpx<T>* z = zs + (size_t)(q * R2 + sg * R) * R;
#pragma unroll
            for (int k2 = 0; k2 < R; ++k2) {
                cpx<T> acc = czero<T>();
#pragma unroll
                for (int k1 = 0; k1 < R; ++k1) cfma(acc, pr[k1], z[k1 * R + k2]);
                Y[i * R + k2] -= acc;
            }
        }
        __syncthreads();
    }
    // (b3) P_c = Y ; G_c = Qc^t Y
    cpx<T>* Pw = sp.P + (size_t)(lam - 1) * R * np;
    for (int e = tid; e < s * R; e += NT) {
        const int i = e % s, k = e / s;
        Pw[(size_t)k * np + lo + i] = Y[i * R + k];
    }
    for (int e = tid; e < nch * R * R; e += NT) {
        const int ch = e % nch, k1 = (e / nch) % R, k2 = e / (nch * R);
        cpx<T> acc = czero<T>();
#pragma unroll
        for (int jj = 0; jj < B; ++jj) {
            const int i = ch * B + jj;
            cfma(acc, Qc[i * R + k1], Y[i * R + k2]);
        }
        part[(k1 * R + k2) * nch + ch] = acc;
    }
    __syncthreads();
    cpx<T>* Gw = sp.G + (size_t)node * R * R;
    for (int e = tid; e < R * R; e += NT) {
        cpx<T> acc = czero<T>();
        for (int ch = 0; ch < nch; ++ch) acc += part[e * nch + ch];
        Gw[e] = acc;                               // G[k1*R + k2]
    }
}

// ----------------------------------------------------------------------------
// The same Woodbury step (levels 1..L) organised for latency.  The step is a
// chain of small dependent products, so its time is the number of global
// round trips and barriers on that chain.  Here every input that earlier
// launches wrote (Q_c, the P columns and X cores of the nodes inside c, the
// leaf inverses) is fetched in one prologue, while wavefront 0 inverts the
// core of c; then the corrections of all inner levels run together:
//     T_c Q_c = K Q_c - sum_{levels lc > lam} P_lc z_lc,
//     z_lc = X_parent [P_left^t Q_c ; P_right^t Q_c]  (per parent at lc - 1),
// one barrier phase per product (chunk partials, child sums, z, update).
// Partial sums run over the same B-row chunks and in the same order as in
// wood_kernel.  Global memory is addressed through the global address space
// (so that LDS waits never wait on global stores) and LDS through the local
// one.  Used when the node has at most NT/2 rows and the layout fits in LDS.
struct WoodPfLayout {
    size_t oQ, oY, oP, oX, oC, oXo, oPart, oYs, oZs, oEnd;
};

__host__ __device__ inline WoodPfLayout wood_pf_layout(int s, int r, int b, int L, int lam) {
    const int nl = L - lam, nch = s / b;
    const size_t rr = (size_t)r * r;
    WoodPfLayout w;
    size_t o = 0;
    w.oQ = o; o += (size_t)s * r;                                  // Q_c rows   [i][k]
    w.oY = o; o += (size_t)s * r;                                  // T_c Q_c    [i][k]
    w.oP = o; o += (size_t)nl * r * (s + 2);                       // P levels lam+1..L  [l][k][i], ld s + 2
    w.oX = o; o += nl >= 1 ? ((size_t)(1 << nl) - 2) * 4 * rr : 0; // X of levels lam+1..L-1
    w.oC = o; o += nl >= 1 ? 5 * rr : 0;                           // core scratch
    w.oXo = o; o += nl >= 1 ? 4 * rr : 0;                          // core inverse X_c
    w.oPart = o; o += (size_t)(nl > 1 ? nl : 1) * rr * nch;        // chunk partials
    w.oYs = o; o += nl >= 1 ? ((size_t)(2 << nl) - 2) * rr : 0;    // child sums, all levels
    w.oZs = o; o += nl >= 1 ? ((size_t)(2 << nl) - 2) * rr : 0;    // z, all levels
    w.oEnd = o;
    return w;
}

template <typename X> using gbl = __attribute__((address_space(1))) X;
template <typename X> __device__ __forceinline__ gbl<X>* to_gbl(X* p) { return (gbl<X>*)p; }
template <typename X> __device__ __forceinline__ const gbl<X>* to_gbl(const X* p) { return (const gbl<X>*)p; }
template <typename T> __device__ __forceinline__ cpx<T> ldg(const gbl<cpx<T>>* p) { return mk<T>(p->re, p->im); }
template <typename T> __device__ __forceinline__ void stg(gbl<cpx<T>>* p, cpx<T> v) { p->re = v.re; p->im = v.im; }

template <typename T, int B, int R>
__global__ __launch_bounds__(NT) void wood_pf_kernel(const InstDesc<T>* __restrict__ descs, int m, int lam) {
    constexpr int R2 = 2 * R, RR = R * R;
    constexpr int KH = R > 1 ? R / 2 : 1;      // columns of T_c Q_c per thread
    constexpr int HPR = R / KH;                // threads per row
    constexpr int U = sizeof(T) == 4 ? 16 : 8; // loads in flight per thread and batch
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int perm_w[R];
    const InstDesc<T> d = descs[blockIdx.y];
    const Plan& p = d.p;
    if (m >= p.n || p.L == 0 || lam < 1 || lam > p.L || (int)blockIdx.x >= (1 << lam)) return;
    const StepPtrs<T> sp = step_ptrs(d, m);
    const int L = p.L, np = p.np, nl = L - lam;
    const int ci = blockIdx.x;
    const int node = heap_id(lam, ci);
    const int s = np >> lam, lo = ci * s, nch = s / B;
    // s and nch are powers of two: index arithmetic by shifts and masks
    const int ls = 31 - __clz(s), lnch = 31 - __clz(nch);
    constexpr int LR = R == 2 ? 1 : R == 4 ? 2 : R == 8 ? 3 : 4;
    static_assert((1 << LR) == R, "rank is a power of two");
    const int tid = threadIdx.x;
    const WoodPfLayout wl = wood_pf_layout(s, R, B, L, lam);
    lds<cpx<T>>* base = to_lds((cpx<T>*)smem);
    lds<cpx<T>>* Qc = base + wl.oQ;
    lds<cpx<T>>* Y = base + wl.oY;
    lds<cpx<T>>* Pc = base + wl.oP;
    lds<cpx<T>>* Xc = base + wl.oX;
    lds<cpx<T>>* Xo = base + wl.oXo;
    lds<cpx<T>>* part = base + wl.oPart;
    lds<cpx<T>>* ys = base + wl.oYs;
    lds<cpx<T>>* zs = base + wl.oZs;
    const bool has_core = nl >= 1;

    // T_c Q_c task of this thread: row i, columns k0 .. k0 + KH - 1
    const bool rowt = tid < s * HPR;
    const int i = rowt ? tid / HPR : 0;
    const int k0 = (tid % HPR) * KH;
    const int il = i % B;
    cpx<T> kr[B];
    {
        const gbl<cpx<T>>* Kt = to_gbl(sp.K) + (size_t)((lo + i) / B) * B * B + il;
#pragma unroll
        for (int jj = 0; jj < B; ++jj) kr[jj] = ldg(Kt + (size_t)jj * B);   // in range for every thread
    }

    if (has_core && tid < 64) {
        // (a) core of c from the children's G
        wood_core<T, R>(sp.G + (size_t)heap_id(lam + 1, 2 * ci) * RR, sp.G + (size_t)heap_id(lam + 1, 2 * ci + 1) * RR,
                        base + wl.oC, Xo, perm_w, sp.status);
    } else {
        // prologue: Q_c (transposed to rows), the P columns of levels
        // lam+1..L on the rows of c, and the X cores of levels lam+1..L-1
        // inside c; U independent loads per thread and batch, addresses
        // chosen by selects
        const int wt = has_core ? tid - 64 : tid, nw = has_core ? NT - 64 : NT;
        const int nQ = s * R, nP = nl * R * s;
        const int nX = nl >= 1 ? ((1 << nl) - 2) * 4 * RR : 0;
        const int ntot = nQ + nP + nX;
        const gbl<cpx<T>>* Qv = to_gbl(sp.Q) + (size_t)(lam - 1) * R * np + lo;
        const gbl<cpx<T>>* Pv = to_gbl(sp.P) + (size_t)lam * R * np + lo;
        const gbl<cpx<T>>* Xv = to_gbl(sp.X);
        for (int e0 = wt; e0 < ntot; e0 += U * nw) {
            cpx<T> v[U];
            int dst[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = min(e0 + u * nw, ntot - 1);
                // Q_c entry (row, column) -> row-major
                const int qi = e & (s - 1), qk = e >> ls;
                // P entry f = (l*R + k)*s + row: contiguous rows of each column
                const int f = e - nQ;
                const int fr = f & (s - 1), fc = f >> ls;        // stored with leading dimension s + 2
                // X entry g: node group j (level lam + j, 2^j nodes) found from g / (4 R^2) + 2
                const int g = e - nQ - nP;
                const int gn = (g >= 0 ? g : 0) / (4 * RR) + 2;
                const int j = 31 - __clz(gn);
                const int gl = (g >= 0 ? g : 0) - ((1 << j) - 2) * 4 * RR;
                const int first = heap_id(lam + j, ci << j);
                // the region is picked with bit masks (no branches)
                const bool isQ = e < nQ, isP = !isQ && e < nQ + nP;
                const uint64_t mQ = 0ull - (uint64_t)isQ, mP = 0ull - (uint64_t)isP, mX = ~(mQ | mP);
                const uint64_t aQ = (uint64_t)(Qv + (size_t)qk * np + qi);
                const uint64_t aP = (uint64_t)(Pv + (size_t)fc * np + fr);
                const uint64_t aX = (uint64_t)(Xv + (size_t)first * 4 * RR + gl);
                const gbl<cpx<T>>* src = (const gbl<cpx<T>>*)((aQ & mQ) | (aP & mP) | (aX & mX));
                dst[u] = (((int)wl.oQ + qi * R + qk) & (int)mQ) | (((int)wl.oP + fc * (s + 2) + fr) & (int)mP) |
                         (((int)wl.oX + g) & (int)mX);
                v[u] = ldg(src);
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (e0 + u * nw < ntot) stc(base + dst[u], v[u]);
        }
    }
    __syncthreads();

    // phase 1: K Q_c into registers; chunk partials of P_lc^t Q_c, all levels
    cpx<T> acc[KH];
#pragma unroll
    for (int k = 0; k < KH; ++k) acc[k] = czero<T>();
    if (rowt) {
        const lds<cpx<T>>* qb = Qc + (size_t)(i - il) * R + k0;
#pragma unroll
        for (int jj = 0; jj < B; ++jj)
#pragma unroll
            for (int k = 0; k < KH; ++k) cfma(acc[k], kr[jj], ldc(qb + jj * R + k));
    }
    // the partial tasks follow the row tasks in one list over the threads;
    // neighbouring threads take the same chunk (broadcast Q_c reads) and
    // different columns k1 (P rows padded to s + 2 entries: different banks)
    const int ldp = s + 2;
    const int nrt = s * HPR, npt = nl * nch * R;
    for (int v = tid; v < nrt + npt; v += NT) {
        if (v < nrt) continue;
        const int pe = v - nrt;
        const int lI = pe >> (lnch + LR), rem = pe & ((nch << LR) - 1);
        const int k1 = rem & (R - 1), ch = rem >> LR;
        const lds<cpx<T>>* pc = Pc + ((size_t)lI * R + k1) * ldp + ch * B;
        const lds<cpx<T>>* qc = Qc + (size_t)ch * B * R;
        cpx<T> a2[R];
#pragma unroll
        for (int k2 = 0; k2 < R; ++k2) a2[k2] = czero<T>();
#pragma unroll
        for (int jj = 0; jj < B; ++jj) {
            const cpx<T> pv = ldc(pc + jj);
#pragma unroll
            for (int k2 = 0; k2 < R; ++k2) cfma(a2[k2], pv, ldc(qc + jj * R + k2));
        }
#pragma unroll
        for (int k2 = 0; k2 < R; ++k2) stc(part + ((size_t)lI * nch + ch) * RR + k1 * R + k2, a2[k2]);
    }
    if (nl >= 1) {
        __syncthreads();
        // phase 2: per child sums ys[lI][c][k1*R + k2]
        const int nys = ((2 << nl) - 2) * RR;
        for (int e = tid; e < nys; e += NT) {
            const int lI = 30 - __clz(e / RR + 2);          // e / RR + 2 in [2^(lI+1), 2^(lI+2))
            const int el = e - ((2 << lI) - 2) * RR;
            const int c = el / RR, kk = el % RR;
            const int cpn = nch >> (lI + 1);
            const lds<cpx<T>>* pp = part + ((size_t)lI * nch + c * cpn) * RR + kk;
            cpx<T> a = czero<T>();
            for (int q = 0; q < cpn; ++q) a += ldc(pp + (size_t)q * RR);
            stc(ys + e, a);
        }
        __syncthreads();
        // phase 3: z = X_parent [y_left; y_right] for the parents at level lam + lI
        for (int e = tid; e < nys; e += NT) {
            const int lI = 30 - __clz(e / RR + 2);
            const int off = ((2 << lI) - 2) * RR;
            const int el = e - off;
            const int q = el / (R2 * R), o = (el / R) % R2, k2 = el % R;
            const lds<cpx<T>>* Xq = lI == 0 ? Xo : Xc + (((size_t)(1 << lI) - 2) + q) * 4 * RR;
            const lds<cpx<T>>* yq = ys + off + (size_t)2 * q * RR;
            cpx<T> a = czero<T>();
#pragma unroll
            for (int c = 0; c < R2; ++c) cfma(a, ldc(Xq + c * R2 + o), ldc(yq + (c / R) * RR + (c % R) * R + k2));
            stc(zs + e, a);
        }
        __syncthreads();
        // phase 4: subtract the corrections of every inner level from row i
        if (rowt) {
            for (int lI = 0; lI < nl; ++lI) {
                const int c = i >> (ls - lI - 1), q = c >> 1, sg = c & 1;
                const lds<cpx<T>>* z = zs + ((2 << lI) - 2) * RR + (size_t)(q * R2 + sg * R) * R + k0;
                cpx<T> pr[R];
#pragma unroll
                for (int k1 = 0; k1 < R; ++k1) pr[k1] = ldc(Pc + ((size_t)lI * R + k1) * ldp + i);
#pragma unroll
                for (int k = 0; k < KH; ++k) {
                    cpx<T> a = czero<T>();
#pragma unroll
                    for (int k1 = 0; k1 < R; ++k1) cfma(a, pr[k1], ldc(z + k1 * R + k));
                    acc[k] -= a;
                }
            }
        }
    }
    // (b3) P_c = T_c Q_c ; G_c = Q_c^t P_c.  Every global store waits until
    // the end: a store's data registers are not reused while it is in flight,
    // so a store followed by more work would stall that work.
    if (rowt) {
#pragma unroll
        for (int k = 0; k < KH; ++k) stc(Y + i * R + k0 + k, acc[k]);
    }
    __syncthreads();
    for (int e = tid; e < nch * RR; e += NT) {
        // neighbouring threads: same chunk and k1 (broadcast), consecutive k2
        const int k2 = e & (R - 1), k1 = (e >> LR) & (R - 1), ch = e >> (2 * LR);
        cpx<T> a = czero<T>();
#pragma unroll
        for (int jj = 0; jj < B; ++jj) {
            const int ii = ch * B + jj;
            cfma(a, ldc(Qc + ii * R + k1), ldc(Y + ii * R + k2));
        }
        stc(part + (size_t)ch * RR + k1 * R + k2, a);
    }
    __syncthreads();
    gbl<cpx<T>>* Gw = to_gbl(sp.G) + (size_t)node * RR;
    for (int e = tid; e < RR; e += NT) {
        cpx<T> a = czero<T>();
        for (int ch = 0; ch < nch; ++ch) a += ldc(part + (size_t)ch * RR + e);
        stg(Gw + e, a);
    }
    if (rowt) {
        gbl<cpx<T>>* Pw = to_gbl(sp.P) + (size_t)(lam - 1) * R * np + lo + i;
#pragma unroll
        for (int k = 0; k < KH; ++k) stg(Pw + (size_t)(k0 + k) * np, acc[k]);
    }
    if (has_core) {
        gbl<cpx<T>>* Xg = to_gbl(sp.X) + (size_t)node * 4 * RR;
        for (int e = tid; e < 4 * RR; e += NT) stg(Xg + e, ldc(Xo + e));
    }
}

constexpr size_t WOOD_PF_LDS_MAX = 156 * 1024;

template <typename T, int B, int R>
bool wood_pf_fits(const Plan& p, int lam, size_t* lds) {
    if (lam < 1 || lam > p.L) return false;
    const int s = p.np >> lam;
    if (s > NT / 2 || s < B) return false;
    const size_t l = wood_pf_layout(s, R, B, p.L, lam).oEnd * sizeof(cpx<T>);
    if (lds) *lds = l;
    return l <= WOOD_PF_LDS_MAX;
}

template <typename T, int R>
size_t recomp_lds(const Plan& p, int m) {
    size_t mx = 0;
    for (int lam = 1; lam <= p.L; ++lam) {
        int k = 1 + (m > 0 ? R * lam : 0);
        RecompLayout l = recomp_layout(p.np >> lam, k, R, m > 0 ? lam * R * R : 0, sizeof(cpx<T>), sizeof(cpx<T>),
                                       gram_path(sizeof(cpx<T>), p.tol, k));
        size_t b = l.gEnd * sizeof(c128);
        if (b > mx) mx = b;
    }
    return mx;
}

template <typename T, int B, int R>
size_t layer_lds(const Plan& p, int m) {
    size_t lds = (size_t)(2 * p.L * B * R + p.L * R * R + 1);
    if (lds < (size_t)B * B) lds = (size_t)B * B;
    lds *= sizeof(cpx<T>);
    if (p.L > 0) {
        size_t a = recomp_lds<T, R>(p, m);
        if (a > lds) lds = a;
    }
    return lds;
}

template <typename T, int B, int R>
size_t wood_lds(const Plan& p, int lam) {
    size_t lds = (size_t)5 * R * R;
    if (lam > 0 && lam <= p.L) {
        const size_t w = wood_layout(p.np >> lam, R, B, p.L, lam).oEnd;
        if (w > lds) lds = w;
    }
    return lds * sizeof(cpx<T>);
}

template <typename T, int B, int R>
void launch_layer(const InstDesc<T>* descs, const Plan* plans, int ninst, int m, hipStream_t s) {
    size_t lds = 0;
    int nblk = 0;
    for (int q = 0; q < ninst; ++q) {
        const Plan& p = plans[q];
        if (m >= p.n) continue;
        const size_t l = layer_lds<T, B, R>(p, m);
        if (l > lds) lds = l;
        const int nb = (p.L > 0 ? (1 << p.L) - 1 : 0) + (1 << p.L);
        if (nb > nblk) nblk = nb;
    }
    if (nblk == 0) return;
    hipLaunchKernelGGL((layer_kernel<T, B, R>), dim3(nblk, ninst), dim3(NT), lds, s, descs, m);
}

template <typename T, int B, int R>
void launch_wood(const InstDesc<T>* descs, const Plan* plans, int ninst, int m, int lam, hipStream_t s) {
    size_t lds = 0, lds_pf = 0;
    bool any = false, pf = lam >= 1;
    for (int q = 0; q < ninst; ++q) {
        const Plan& p = plans[q];
        if (m >= p.n || p.L == 0 || lam > p.L) continue;
        any = true;
        const size_t l = wood_lds<T, B, R>(p, lam);
        if (l > lds) lds = l;
        size_t lp = 0;
        if (pf && wood_pf_fits<T, B, R>(p, lam, &lp)) lds_pf = lp > lds_pf ? lp : lds_pf;
        else pf = false;
    }
    if (!any) return;
    if (pf)
        hipLaunchKernelGGL((wood_pf_kernel<T, B, R>), dim3(1 << lam, ninst), dim3(NT), lds_pf, s, descs, m, lam);
    else
        hipLaunchKernelGGL((wood_kernel<T, B, R>), dim3(1 << lam, ninst), dim3(NT), lds, s, descs, m, lam);
}

// Allow a kernel to use all LDS left after its static shared variables.
template <typename K>
void allow_lds(K kernel) {
    hipFuncAttributes a;
    if (hipFuncGetAttributes(&a, (const void*)kernel) == hipSuccess) {
        int dyn = 160 * 1024 - (int)a.sharedSizeBytes;
        (void)hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
    }
    (void)hipGetLastError();   // a refused attribute must not surface as a later launch error
}

#define FOR_LEAVES(X) X(4) X(8) X(16) X(32) X(64)
#define FOR_RANKS(X) X(2) X(4) X(8) X(16)
#define FOR_WOOD(X) \
    X(4, 2) X(4, 4) X(4, 8) X(4, 16) X(8, 2) X(8, 4) X(8, 8) X(8, 16) X(16, 2) X(16, 4) X(16, 8) X(16, 16) \
    X(32, 2) X(32, 4) X(32, 8) X(32, 16) X(64, 2) X(64, 4) X(64, 8) X(64, 16)

template <typename T>
void set_lds_limits() {
    static bool done = false;
    if (done) return;
    done = true;
#define A_WOOD(BB, RR) \
    allow_lds(wood_kernel<T, BB, RR>); allow_lds(wood_pf_kernel<T, BB, RR>); allow_lds(layer_kernel<T, BB, RR>);
    FOR_WOOD(A_WOOD)
#undef A_WOOD
}

}  // namespace

template <typename T>
int launch_factor_layer(const InstDesc<T>* descs, const Plan* plans, int ninst, int m, hipStream_t s,
                        hipEvent_t after_layer) {
    set_lds_limits<T>();
    const int b = plans[0].b, L0 = plans[0].L;
    const int rr = L0 > 0 ? plans[0].r : 2;   // dense leaves: no low-rank data
    int Lmax = 0;
    for (int q = 0; q < ninst; ++q) {
        if (plans[q].b != b || (plans[q].L > 0 ? plans[q].r : 2) != rr) return -1;
        if (plans[q].L > Lmax) Lmax = plans[q].L;
    }
    bool ok = false;
#define C_LAYER(BB, RR)                                                               \
    if (!ok && b == BB && rr == RR) {                                                 \
        launch_layer<T, BB, RR>(descs, plans, ninst, m, s);                           \
        if (after_layer) (void)hipEventRecord(after_layer, s);                        \
        for (int lam = Lmax; lam >= 0 && Lmax > 0; --lam)                             \
            launch_wood<T, BB, RR>(descs, plans, ninst, m, lam, s);                   \
        ok = true;                                                                    \
    }
    FOR_WOOD(C_LAYER)
#undef C_LAYER
    return ok ? 0 : -1;
}

template <typename T>
void factor_kernels_init() {
    set_lds_limits<T>();
}
