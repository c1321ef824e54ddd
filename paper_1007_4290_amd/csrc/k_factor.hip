// One layer of the approximate sweeping factorization (Alg. 2.3) on the GPU.
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
//   recompress_kernel  one block per off-diagonal pair: build the stacked
//                      factors of S_m(c1, c2) (rank 1 + r*level), Householder
//                      QR of both, one-sided Jacobi SVD of the small core,
//                      truncate (sigma > tol*sigma_1, at most r), write Q.
//   leaf_kernel        one block per leaf: S_m leaf = A - D T_{m-1} D, then
//                      Gauss-Jordan inverse with partial pivoting -> K.
//   wood_kernel(l)     levels l = L..1, one block per node: X_c from the
//                      children's G, then P_c = T_c Q_c and G_c = Q_c^t P_c.
//   wood_kernel(0)     the root core X_0.
#include "internal.hpp"

namespace {

constexpr int NT = 256;

template <typename T> __device__ __forceinline__ T eps_of();
template <> __device__ __forceinline__ float eps_of<float>() { return 1.1920929e-7f; }
template <> __device__ __forceinline__ double eps_of<double>() { return 2.220446049250313e-16; }

template <typename T> __device__ __forceinline__ T rsq(T x);
template <> __device__ __forceinline__ float rsq<float>(float x) { return sqrtf(x); }
template <> __device__ __forceinline__ double rsq<double>(double x) { return sqrt(x); }

__device__ __forceinline__ int heap_id(int lvl, int idx) { return (1 << lvl) - 1 + idx; }

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
        int p = 0;
        T best = T(-1);
        for (int i = 0; i < B; ++i) {
            if (!g.used[i]) {
                T v = abs2(colk[i]);
                if (v > best) { best = v; p = i; }
            }
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
// Leaf: S leaf of layer m, then its inverse K (column-major b x b).
template <typename T, int B>
__global__ __launch_bounds__(NT) void leaf_kernel(Plan p, StepPtrs<T> sp, int m) {
    constexpr int TS = Tile<B>::TS, G = Tile<B>::G;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ GJScratch<T, B> gjs;
    const int t = blockIdx.x;
    const int tid = threadIdx.x;
    const bool act = tid < G * G;
    const int tr = tid % G, tc = tid / G;
    const int base = t * B;
    const int r = p.r, L = p.L, np = p.np;
    cpx<T>* Pl = (cpx<T>*)smem;   // B x r, [i*r + k]
    cpx<T>* Wl = Pl + B * r;      // B x r
    cpx<T>* Xb = Wl + B * r;      // r x r, [k1*r + k2]

    cpx<T> M[TS][TS];
#pragma unroll
    for (int a = 0; a < TS; ++a)
#pragma unroll
        for (int bb = 0; bb < TS; ++bb) {
            int i = tr * TS + a, j = tc * TS + bb;
            M[a][bb] = (m > 0 && act) ? sp.Kp[(size_t)t * B * B + (size_t)j * B + i] : czero<T>();
        }
    if (m > 0) {
        for (int lvl = 1; lvl <= L; ++lvl) {
            int anc = t >> (L - lvl);
            int q = anc >> 1, sg = anc & 1;
            const cpx<T>* Pv = sp.Pp + (size_t)(lvl - 1) * r * np;
            const cpx<T>* Xq = sp.Xp + (size_t)heap_id(lvl - 1, q) * 4 * r * r;
            for (int e = tid; e < B * r; e += NT) {
                int i = e % B, k = e / B;
                Pl[i * r + k] = Pv[(size_t)k * np + base + i];
            }
            for (int e = tid; e < r * r; e += NT) {
                int k1 = e % r, k2 = e / r;
                Xb[k1 * r + k2] = Xq[(size_t)(sg * r + k2) * 2 * r + sg * r + k1];
            }
            __syncthreads();
            for (int e = tid; e < B * r; e += NT) {
                int i = e / r, k2 = e % r;
                cpx<T> acc = czero<T>();
                for (int k1 = 0; k1 < r; ++k1) cfma(acc, Pl[i * r + k1], Xb[k1 * r + k2]);
                Wl[i * r + k2] = acc;
            }
            __syncthreads();
            if (act) {
#pragma unroll
                for (int a = 0; a < TS; ++a)
#pragma unroll
                    for (int bb = 0; bb < TS; ++bb) {
                        int i = tr * TS + a, j = tc * TS + bb;
                        cpx<T> acc = czero<T>();
                        for (int k = 0; k < r; ++k) cfma(acc, Wl[i * r + k], Pl[j * r + k]);
                        M[a][bb] -= acc;
                    }
            }
            __syncthreads();
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
    gj_invert<T, B>(M, act, tr, tc, gjs, sp.status);
    if (act) {
#pragma unroll
        for (int a = 0; a < TS; ++a)
#pragma unroll
            for (int bb = 0; bb < TS; ++bb) {
                int i = tr * TS + a, j = tc * TS + bb;
                sp.K[(size_t)t * B * B + (size_t)gjs.perm[j] * B + gjs.pinv[i]] = M[a][bb];
            }
    }
}

// ----------------------------------------------------------------------------
// Block-level helpers for the recompression (all operands in LDS).
template <typename T>
__device__ T block_sum(T v, T* red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) red[wv] = v;
    __syncthreads();
    T s = T(0);
    for (int q = 0; q < NT / 64; ++q) s += red[q];
    __syncthreads();
    return s;
}

// dots[c - c0] = v^H A[j:, c] for c in [c0, ncol), where v = (v0, A[j+1:, j]).
// Work split: tasks (column, row-phase) with the rows of one task strided.
template <typename T>
__device__ void reflector_dots(const cpx<T>* A, int lda, int s, int j, cpx<T> v0, const cpx<T>* Y, int ldy,
                               int c0, int ncol, cpx<T>* part, cpx<T>* dots) {
    int nc = ncol - c0;
    if (nc <= 0) return;
    int nph = NT / nc;
    if (nph < 1) nph = 1;
    if (nph > 64) nph = 64;
    for (int task = threadIdx.x; task < nc * nph; task += NT) {
        int c = c0 + task % nc, ph = task / nc;
        cpx<T> acc = czero<T>();
        for (int i = j + ph; i < s; i += nph) {
            cpx<T> vi = (i == j) ? v0 : A[(size_t)j * lda + i];
            cfma_conj(acc, vi, Y[(size_t)c * ldy + i]);
        }
        part[task] = acc;
    }
    __syncthreads();
    for (int c = threadIdx.x; c < nc; c += NT) {
        cpx<T> acc = czero<T>();
        for (int ph = 0; ph < nph; ++ph) acc += part[ph * nc + c];
        dots[c] = acc;
    }
    __syncthreads();
}

// Y[j:, c] -= tau * v * dots[c - c0] for c in [c0, ncol).
template <typename T>
__device__ void reflector_update(const cpx<T>* A, int lda, int s, int j, cpx<T> v0, T tau, cpx<T>* Y, int ldy,
                                 int c0, int ncol, const cpx<T>* dots) {
    int nc = ncol - c0, nr = s - j;
    for (int e = threadIdx.x; e < nc * nr; e += NT) {
        int i = j + e % nr, c = c0 + e / nr;
        cpx<T> vi = (i == j) ? v0 : A[(size_t)j * lda + i];
        Y[(size_t)c * ldy + i] -= (tau * vi) * dots[c - c0];
    }
    __syncthreads();
}

// Householder QR of the s x k column-major matrix A (in LDS).  Hermitian
// reflectors H_j = I - tau_j v_j v_j^H with v_j = (v0_j, A[j+1:, j]); on exit
// A's upper triangle holds R (diagonal = beta_j) and Q = H_0 H_1 ... H_{kk-1}.
template <typename T>
__device__ void house_qr(cpx<T>* A, int s, int k, cpx<T>* v0, T* tau, T* redr, cpx<T>* part, cpx<T>* dots) {
    int kk = s < k ? s : k;
    for (int j = 0; j < kk; ++j) {
        T pr = T(0);
        for (int i = j + threadIdx.x; i < s; i += NT) pr += abs2(A[(size_t)j * s + i]);
        T nx2 = block_sum(pr, redr);
        cpx<T> x0 = A[(size_t)j * s + j];
        T nx = rsq(nx2), ax0 = rsq(abs2(x0));
        cpx<T> ph = ax0 > T(0) ? (T(1) / ax0) * x0 : mk<T>(T(1), T(0));
        cpx<T> vv0 = (ax0 + nx) * ph;
        T tj = nx > T(0) ? T(1) / (nx * (nx + ax0)) : T(0);
        reflector_dots(A, s, s, j, vv0, A, s, j + 1, k, part, dots);
        reflector_update(A, s, s, j, vv0, tj, A, s, j + 1, k, dots);
        if (threadIdx.x == 0) {
            A[(size_t)j * s + j] = -nx * ph;
            v0[j] = vv0;
            tau[j] = tj;
        }
        __syncthreads();
    }
}

// Y <- Q Y for the Q of house_qr (Y: s x ncol, column-major, ld s).
template <typename T>
__device__ void apply_q(const cpx<T>* A, int s, int kk, const cpx<T>* v0, const T* tau, cpx<T>* Y, int ncol,
                        cpx<T>* part, cpx<T>* dots) {
    for (int j = kk - 1; j >= 0; --j) {
        if (tau[j] == T(0)) continue;
        reflector_dots(A, s, s, j, v0[j], Y, s, 0, ncol, part, dots);
        reflector_update(A, s, s, j, v0[j], tau[j], Y, s, 0, ncol, dots);
    }
}

// One-sided Jacobi SVD of the P x P column-major matrix Mx (P even, columns
// beyond the true size are zero).  On exit the columns of Mx are W_c sigma_c
// and Z holds the accumulated unitary rotations (Mx_in Z = Mx_out).
template <typename T>
__device__ void jacobi_svd(cpx<T>* Mx, cpx<T>* Z, int P, int* flag) {
    const int npair = P / 2;
    const int grp = threadIdx.x >> 3, gl = threadIdx.x & 7;
    const T thr = T(P) * eps_of<T>();
    for (int e = threadIdx.x; e < P * P; e += NT) Z[e] = (e % P == e / P) ? mk<T>(T(1), T(0)) : czero<T>();
    __syncthreads();
    for (int sweep = 0; sweep < 60; ++sweep) {
        if (threadIdx.x == 0) *flag = 0;
        __syncthreads();
        for (int rd = 0; rd < P - 1; ++rd) {
            if (grp < npair) {
                int a, b;
                if (grp == 0) { a = rd; b = P - 1; }
                else { a = (rd + grp) % (P - 1); b = (rd - grp + P - 1) % (P - 1); }
                cpx<T>* ca = Mx + (size_t)a * P;
                cpx<T>* cb = Mx + (size_t)b * P;
                T al = T(0), be = T(0);
                cpx<T> ga = czero<T>();
                for (int i = gl; i < P; i += 8) {
                    al += abs2(ca[i]);
                    be += abs2(cb[i]);
                    cfma_conj(ga, ca[i], cb[i]);
                }
                for (int off = 1; off < 8; off <<= 1) {
                    al += __shfl_xor(al, off, 8);
                    be += __shfl_xor(be, off, 8);
                    ga.re += __shfl_xor(ga.re, off, 8);
                    ga.im += __shfl_xor(ga.im, off, 8);
                }
                T ag = rsq(abs2(ga));
                if (ag > thr * rsq(al * be) && ag > T(0)) {
                    T zeta = (be - al) / (T(2) * ag);
                    T t = (zeta >= T(0) ? T(1) : T(-1)) / (fabs(zeta) + rsq(T(1) + zeta * zeta));
                    T c = T(1) / rsq(T(1) + t * t);
                    T sn = c * t;
                    cpx<T> em = (T(1) / ag) * conj(ga);   // e^{-i phi}
                    for (int i = gl; i < P; i += 8) {
                        cpx<T> xa = ca[i], xb = cb[i];
                        ca[i] = c * xa - sn * (em * xb);
                        cb[i] = sn * xa + c * (em * xb);
                        cpx<T>* za = Z + (size_t)a * P;
                        cpx<T>* zb = Z + (size_t)b * P;
                        cpx<T> ya = za[i], yb = zb[i];
                        za[i] = c * ya - sn * (em * yb);
                        zb[i] = sn * ya + c * (em * yb);
                    }
                    if (gl == 0) *flag = 1;
                }
            }
            __syncthreads();
        }
        int f = *flag;
        __syncthreads();
        if (!f) break;
    }
}

// ----------------------------------------------------------------------------
// Recompression of the off-diagonal blocks of S_m.
struct RecompLayout {
    // element offsets (in cpx<T> units) inside dynamic LDS
    int s, k, kk, P, r;
    size_t oU, oV, oM, oZ, oY, oPart, oDots, oV0u, oV0v, oEnd;
};

__host__ __device__ inline RecompLayout recomp_layout(int s, int k, int r) {
    RecompLayout l;
    l.s = s; l.k = k; l.r = r;
    l.kk = s < k ? s : k;
    l.P = l.kk + (l.kk & 1);
    size_t o = 0;
    l.oU = o; o += (size_t)s * k;
    l.oV = o; o += (size_t)s * k;
    l.oM = o; o += (size_t)l.P * l.P;
    l.oZ = o; o += (size_t)l.P * l.P;
    l.oY = o; o += (size_t)s * r;
    l.oPart = o; o += NT;
    l.oDots = o; o += (k > r ? k : r);
    l.oV0u = o; o += l.kk;
    l.oV0v = o; o += l.kk;
    l.oEnd = o;
    return l;
}

template <typename T>
__global__ __launch_bounds__(NT) void recompress_kernel(Plan p, StepPtrs<T> sp, int m) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ T tau_u[64 * 2 + 8], tau_v[64 * 2 + 8], redr[NT / 64], sig[72];
    __shared__ int order[72];
    __shared__ int flag, rank_s;
    const int pj = blockIdx.x;                   // heap id of the parent node
    const int lp = 31 - __clz(pj + 1);
    const int j = pj - ((1 << lp) - 1);
    const int lam = lp + 1;
    const int s = p.np >> lam;
    const int r = p.r, np = p.np;
    const int k = 1 + (m > 0 ? r * lam : 0);
    const int lo1 = 2 * j * s, lo2 = (2 * j + 1) * s;
    RecompLayout ly = recomp_layout(s, k, r);
    cpx<T>* base = (cpx<T>*)smem;
    cpx<T>* Ut = base + ly.oU;
    cpx<T>* Vt = base + ly.oV;
    cpx<T>* Mx = base + ly.oM;
    cpx<T>* Z = base + ly.oZ;
    cpx<T>* Y = base + ly.oY;
    cpx<T>* part = base + ly.oPart;
    cpx<T>* dots = base + ly.oDots;
    cpx<T>* v0u = base + ly.oV0u;
    cpx<T>* v0v = base + ly.oV0v;
    const int tid = threadIdx.x;

    // Stacked factors: S_m(c1, c2) = Ut Vt^t.
    //   column 0:        A_{m,m}(last of c1, first of c2) e_last e_first^t
    //   columns 1..r:    D P_lam[c1] X_pj(0-block row, 1-block col) | D P_lam[c2]
    //   then for each ancestor level l' = lam-1 .. 1:
    //                    D P_l'[c1] X_q'(sigma, sigma)              | D P_l'[c2]
    for (int i = tid; i < s; i += NT) {
        Ut[i] = (i == s - 1) ? sp.eo[lo1 + s - 1] : czero<T>();
        Vt[i] = (i == 0) ? mk<T>(T(1), T(0)) : czero<T>();
    }
    if (m > 0) {
        for (int e = tid; e < lam * s * r; e += NT) {
            int i = e % s;
            int k2 = (e / s) % r;
            int blk = e / (s * r);          // 0: own pair, 1..lam-1: ancestors
            int lv, rowoff, coloff;
            const cpx<T>* Xq;
            if (blk == 0) {
                lv = lam;
                Xq = sp.Xp + (size_t)pj * 4 * r * r;
                rowoff = 0; coloff = r;
            } else {
                lv = lam - blk;
                int a = (2 * j) >> (lam - lv);
                int q = a >> 1, sg = a & 1;
                Xq = sp.Xp + (size_t)heap_id(lv - 1, q) * 4 * r * r;
                rowoff = sg * r; coloff = sg * r;
            }
            const cpx<T>* Pv = sp.Pp + (size_t)(lv - 1) * r * np;
            cpx<T> acc = czero<T>();
            for (int k1 = 0; k1 < r; ++k1)
                cfma(acc, Pv[(size_t)k1 * np + lo1 + i], Xq[(size_t)(coloff + k2) * 2 * r + rowoff + k1]);
            int col = 1 + blk * r + k2;
            Ut[(size_t)col * s + i] = sp.cp[lo1 + i] * acc;
            Vt[(size_t)col * s + i] = sp.cp[lo2 + i] * Pv[(size_t)k2 * np + lo2 + i];
        }
    }
    __syncthreads();

    house_qr(Ut, s, k, v0u, tau_u, redr, part, dots);
    house_qr(Vt, s, k, v0v, tau_v, redr, part, dots);

    // core Mx = R1 R2^t (kk x kk), padded to P x P with zeros
    const int kk = ly.kk, P = ly.P;
    for (int e = tid; e < P * P; e += NT) {
        int a = e % P, b = e / P;
        cpx<T> acc = czero<T>();
        if (a < kk && b < kk) {
            int c0 = a > b ? a : b;
            for (int c = c0; c < k; ++c) cfma(acc, Ut[(size_t)c * s + a], Vt[(size_t)c * s + b]);
        }
        Mx[(size_t)b * P + a] = acc;
    }
    __syncthreads();
    jacobi_svd(Mx, Z, P, &flag);

    // singular values and truncation
    for (int c = tid; c < P; c += NT) {
        T ss = T(0);
        for (int i = 0; i < P; ++i) ss += abs2(Mx[(size_t)c * P + i]);
        sig[c] = rsq(ss);
    }
    __syncthreads();
    if (tid == 0) {
        for (int c = 0; c < P; ++c) order[c] = c;
        for (int a = 0; a < P; ++a) {
            int best = a;
            for (int b2 = a + 1; b2 < P; ++b2)
                if (sig[order[b2]] > sig[order[best]]) best = b2;
            int tmp = order[a]; order[a] = order[best]; order[best] = tmp;
        }
        T s1 = sig[order[0]];
        int rho = 0;
        while (rho < P && rho < r && s1 > T(0) && sig[order[rho]] > T(p.tol) * s1 && sig[order[rho]] > T(0)) ++rho;
        rank_s = rho;
    }
    __syncthreads();
    const int rho = rank_s;

    // U = Q1 [W sqrt(S); 0]: W_c sqrt(s_c) = Mx_c / sqrt(s_c)
    for (int e = tid; e < s * r; e += NT) {
        int i = e % s, q = e / s;
        cpx<T> v = czero<T>();
        if (q < rho && i < kk) {
            int c = order[q];
            v = (T(1) / rsq(sig[c])) * Mx[(size_t)c * P + i];
        }
        Y[(size_t)q * s + i] = v;
    }
    __syncthreads();
    apply_q(Ut, s, kk, v0u, tau_u, Y, rho, part, dots);
    cpx<T>* Qv = sp.Q + (size_t)(lam - 1) * r * np;
    for (int e = tid; e < s * r; e += NT) {
        int i = e % s, q = e / s;
        Qv[(size_t)q * np + lo1 + i] = Y[(size_t)q * s + i];
    }
    __syncthreads();
    // V = Q2 [conj(Z) sqrt(S); 0]
    for (int e = tid; e < s * r; e += NT) {
        int i = e % s, q = e / s;
        cpx<T> v = czero<T>();
        if (q < rho && i < kk) {
            int c = order[q];
            v = rsq(sig[c]) * conj(Z[(size_t)c * P + i]);
        }
        Y[(size_t)q * s + i] = v;
    }
    __syncthreads();
    apply_q(Vt, s, kk, v0v, tau_v, Y, rho, part, dots);
    for (int e = tid; e < s * r; e += NT) {
        int i = e % s, q = e / s;
        Qv[(size_t)q * np + lo2 + i] = Y[(size_t)q * s + i];
    }
    if (tid == 0) sp.rank[pj] = rho;
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
    int nodes = lam < L ? (1 << (L - lam)) : 1;   // children at the finest level inside the node
    w.oYs = o; o += (size_t)nodes * r * r;
    w.oZs = o; o += (size_t)nodes * r * r;
    w.oEnd = o;
    return w;
}

template <typename T, int R2>
__global__ __launch_bounds__(NT) void wood_kernel(Plan p, StepPtrs<T> sp, int lam) {
    constexpr int TS = Tile<R2>::TS, G = Tile<R2>::G;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ GJScratch<T, R2> gjs;
    const int r = p.r, L = p.L, b = p.b, np = p.np;
    const int ci = blockIdx.x;
    const int node = heap_id(lam, ci);
    const int s = p.np >> lam;
    const int lo = ci * s;
    const int tid = threadIdx.x;

    // (a) core inverse of this node from its children's G blocks
    if (lam < L) {
        const bool act = tid < G * G;
        const int tr = tid % G, tc = tid / G;
        const cpx<T>* G1 = sp.G + (size_t)heap_id(lam + 1, 2 * ci) * r * r;
        const cpx<T>* G2 = sp.G + (size_t)heap_id(lam + 1, 2 * ci + 1) * r * r;
        cpx<T> M[TS][TS];
#pragma unroll
        for (int a = 0; a < TS; ++a)
#pragma unroll
            for (int bb = 0; bb < TS; ++bb) {
                int i = tr * TS + a, j = tc * TS + bb;
                cpx<T> v = czero<T>();
                if (act) {
                    if (i < r && j < r) v = G1[i * r + j];
                    else if (i >= r && j >= r) v = G2[(i - r) * r + (j - r)];
                    else if (i - j == r || j - i == r) v = mk<T>(T(1), T(0));
                }
                M[a][bb] = v;
            }
        gj_invert<T, R2>(M, act, tr, tc, gjs, sp.status);
        if (act) {
            cpx<T>* Xo = sp.X + (size_t)node * 4 * r * r;
#pragma unroll
            for (int a = 0; a < TS; ++a)
#pragma unroll
                for (int bb = 0; bb < TS; ++bb) {
                    int i = tr * TS + a, j = tc * TS + bb;
                    Xo[(size_t)gjs.perm[j] * R2 + gjs.pinv[i]] = M[a][bb];
                }
        }
        __syncthreads();
    }
    if (lam == 0) return;

    WoodLayout wl = wood_layout(s, r, b, L, lam);
    cpx<T>* base = (cpx<T>*)smem;
    cpx<T>* Qc = base + wl.oQ;     // [i*r + k]
    cpx<T>* Y = base + wl.oY;      // [i*r + k]
    cpx<T>* part = base + wl.oPart;
    cpx<T>* ys = base + wl.oYs;
    cpx<T>* zs = base + wl.oZs;
    const cpx<T>* Qv = sp.Q + (size_t)(lam - 1) * r * np;
    for (int e = tid; e < s * r; e += NT) {
        int i = e % s, k = e / s;
        Qc[i * r + k] = Qv[(size_t)k * np + lo + i];
    }
    __syncthreads();
    // (b1) leaf part: Y = K Qc
    for (int e = tid; e < s * r; e += NT) {
        int i = e % s, k = e / s;
        int gi = lo + i;
        int t = gi / b, il = gi % b;
        const cpx<T>* Kt = sp.K + (size_t)t * b * b;
        int lb = (gi - il) - lo;
        cpx<T> acc = czero<T>();
        for (int jj = 0; jj < b; ++jj) cfma(acc, Kt[(size_t)jj * b + il], Qc[(lb + jj) * r + k]);
        Y[i * r + k] = acc;
    }
    __syncthreads();
    // (b2) corrections of the nodes inside this node: levels lc = lam+1 .. L of children
    const int nch = s / b;     // leaf-size chunks in the node
    for (int lc = lam + 1; lc <= L; ++lc) {
        const int sc = np >> lc;                  // child size
        const int ncn = s / sc;                   // children at level lc inside this node
        const int cpn = sc / b;                   // chunks per child
        const cpx<T>* Pv = sp.P + (size_t)(lc - 1) * r * np;
        // chunk partials of P^t Qc
        for (int e = tid; e < nch * r * r; e += NT) {
            int ch = e % nch, k1 = (e / nch) % r, k2 = e / (nch * r);
            cpx<T> acc = czero<T>();
            for (int jj = 0; jj < b; ++jj) {
                int i = ch * b + jj;
                cfma(acc, Pv[(size_t)k1 * np + lo + i], Qc[i * r + k2]);
            }
            part[(k1 * r + k2) * nch + ch] = acc;
        }
        __syncthreads();
        for (int e = tid; e < ncn * r * r; e += NT) {
            int c = e / (r * r), kk = e % (r * r);
            cpx<T> acc = czero<T>();
            for (int q = 0; q < cpn; ++q) acc += part[kk * nch + c * cpn + q];
            ys[c * r * r + kk] = acc;             // ys[c][k1][k2]
        }
        __syncthreads();
        // z_parent = X_parent [y_left; y_right]  (2r x r) for the parents at level lc-1
        const int npar = ncn / 2;
        for (int e = tid; e < npar * 2 * r * r; e += NT) {
            int q = e / (2 * r * r), o = (e / r) % (2 * r), k2 = e % r;
            int gq = (lo / (2 * sc)) + q;         // parent index at level lc-1
            const cpx<T>* Xq = sp.X + (size_t)heap_id(lc - 1, gq) * 4 * r * r;
            cpx<T> acc = czero<T>();
            for (int c = 0; c < 2 * r; ++c) {
                cpx<T> yv = ys[(2 * q + c / r) * r * r + (c % r) * r + k2];
                cfma(acc, Xq[(size_t)c * 2 * r + o], yv);
            }
            zs[(q * 2 * r + o) * r + k2] = acc;
        }
        __syncthreads();
        for (int e = tid; e < s * r; e += NT) {
            int i = e % s, k2 = e / s;
            int c = i / sc;
            int q = c >> 1, sg = c & 1;
            cpx<T> acc = czero<T>();
            for (int k1 = 0; k1 < r; ++k1)
                cfma(acc, Pv[(size_t)k1 * np + lo + i], zs[(q * 2 * r + sg * r + k1) * r + k2]);
            Y[i * r + k2] -= acc;
        }
        __syncthreads();
    }
    // (b3) P_c = Y ; G_c = Qc^t Y
    cpx<T>* Pw = sp.P + (size_t)(lam - 1) * r * np;
    for (int e = tid; e < s * r; e += NT) {
        int i = e % s, k = e / s;
        Pw[(size_t)k * np + lo + i] = Y[i * r + k];
    }
    for (int e = tid; e < nch * r * r; e += NT) {
        int ch = e % nch, k1 = (e / nch) % r, k2 = e / (nch * r);
        cpx<T> acc = czero<T>();
        for (int jj = 0; jj < b; ++jj) {
            int i = ch * b + jj;
            cfma(acc, Qc[i * r + k1], Y[i * r + k2]);
        }
        part[(k1 * r + k2) * nch + ch] = acc;
    }
    __syncthreads();
    cpx<T>* Gw = sp.G + (size_t)node * r * r;
    for (int e = tid; e < r * r; e += NT) {
        cpx<T> acc = czero<T>();
        for (int ch = 0; ch < nch; ++ch) acc += part[e * nch + ch];
        Gw[e] = acc;                               // G[k1*r + k2]
    }
}

template <typename T, int B>
void launch_leaf(const Plan& p, int m, const StepPtrs<T>& sp, hipStream_t s) {
    size_t lds = (size_t)(2 * B * p.r + p.r * p.r) * sizeof(cpx<T>);
    hipLaunchKernelGGL((leaf_kernel<T, B>), dim3(1 << p.L), dim3(NT), lds, s, p, sp, m);
}

template <typename T, int R2>
void launch_wood(const Plan& p, int lam, const StepPtrs<T>& sp, hipStream_t s) {
    size_t lds = 0;
    if (lam > 0) lds = wood_layout(p.np >> lam, p.r, p.b, p.L, lam).oEnd * sizeof(cpx<T>);
    hipLaunchKernelGGL((wood_kernel<T, R2>), dim3(1 << lam), dim3(NT), lds, s, p, sp, lam);
}

template <typename T>
int set_lds_limits() {
    static bool done = false;
    if (done) return 0;
    done = true;
    const int mx = 160 * 1024;
    (void)hipFuncSetAttribute((const void*)recompress_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize, mx);
    (void)hipFuncSetAttribute((const void*)leaf_kernel<T, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, mx);
    (void)hipFuncSetAttribute((const void*)leaf_kernel<T, 8>, hipFuncAttributeMaxDynamicSharedMemorySize, mx);
    (void)hipFuncSetAttribute((const void*)leaf_kernel<T, 16>, hipFuncAttributeMaxDynamicSharedMemorySize, mx);
    (void)hipFuncSetAttribute((const void*)leaf_kernel<T, 32>, hipFuncAttributeMaxDynamicSharedMemorySize, mx);
    (void)hipFuncSetAttribute((const void*)leaf_kernel<T, 64>, hipFuncAttributeMaxDynamicSharedMemorySize, mx);
    (void)hipFuncSetAttribute((const void*)wood_kernel<T, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, mx);
    (void)hipFuncSetAttribute((const void*)wood_kernel<T, 8>, hipFuncAttributeMaxDynamicSharedMemorySize, mx);
    (void)hipFuncSetAttribute((const void*)wood_kernel<T, 16>, hipFuncAttributeMaxDynamicSharedMemorySize, mx);
    (void)hipFuncSetAttribute((const void*)wood_kernel<T, 32>, hipFuncAttributeMaxDynamicSharedMemorySize, mx);
    (void)hipFuncSetAttribute((const void*)wood_kernel<T, 64>, hipFuncAttributeMaxDynamicSharedMemorySize, mx);
    return 0;
}

}  // namespace

// Largest dynamic LDS (bytes) any factorization kernel needs for this plan.
size_t factor_lds_bytes(const Plan& p, size_t elem) {
    size_t mx = (size_t)(2 * p.b * p.r + p.r * p.r) * elem;
    for (int lam = 1; lam <= p.L; ++lam) {
        int s = p.np >> lam;
        size_t a = recomp_layout(s, 1 + p.r * lam, p.r).oEnd * elem;
        size_t w = wood_layout(s, p.r, p.b, p.L, lam).oEnd * elem;
        if (a > mx) mx = a;
        if (w > mx) mx = w;
    }
    return mx;
}

template <typename T>
int launch_factor_step(const Plan& p, int m, const StepPtrs<T>& sp, hipStream_t s) {
    set_lds_limits<T>();
    if (p.L > 0) {
        int kmax = 1 + (m > 0 ? p.r * 1 : 0);
        (void)kmax;
        size_t lds = 0;
        for (int lam = 1; lam <= p.L; ++lam) {
            size_t a = recomp_layout(p.np >> lam, 1 + (m > 0 ? p.r * lam : 0), p.r).oEnd;
            if (a > lds) lds = a;
        }
        hipLaunchKernelGGL(recompress_kernel<T>, dim3((1 << p.L) - 1), dim3(NT), lds * sizeof(cpx<T>), s, p, sp, m);
    }
    switch (p.b) {
        case 4: launch_leaf<T, 4>(p, m, sp, s); break;
        case 8: launch_leaf<T, 8>(p, m, sp, s); break;
        case 16: launch_leaf<T, 16>(p, m, sp, s); break;
        case 32: launch_leaf<T, 32>(p, m, sp, s); break;
        case 64: launch_leaf<T, 64>(p, m, sp, s); break;
        default: return -1;
    }
    for (int lam = p.L; lam >= 0 && p.L > 0; --lam) {
        switch (2 * p.r) {
            case 4: launch_wood<T, 4>(p, lam, sp, s); break;
            case 8: launch_wood<T, 8>(p, lam, sp, s); break;
            case 16: launch_wood<T, 16>(p, lam, sp, s); break;
            case 32: launch_wood<T, 32>(p, lam, sp, s); break;
            case 64: launch_wood<T, 64>(p, lam, sp, s); break;
            default: return -1;
        }
    }
    return 0;
}

template int launch_factor_step<float>(const Plan&, int, const StepPtrs<float>&, hipStream_t);
template int launch_factor_step<double>(const Plan&, int, const StepPtrs<double>&, hipStream_t);
