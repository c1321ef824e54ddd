// Small dense complex128 kernels of the strongly admissible H-arithmetic
// (Sec. 2.3, strongly admissible case):
//   block_jobs_kernel   a batch of block operations, one workgroup each: the
//                       recompression of a sum of two low-rank blocks (QRs
//                       of both stacked factors, SVD of the core, the kept
//                       columns), dense sums, low-rank updates, scalings and
//                       copies;
//   rsvd_tail_kernel    a batch of randomized-SVD tails (SVD of the projected
//                       block, the kept columns, U = Q conj(V_r));
//   hmatvec_kernel      one class of leaf blocks of an H-matrix product;
//   zqr_wave_kernel     the randomized SVD's sample QR;
//   zinv_wave_kernel    the inverse of a dense leaf;
//   zsvd_wave_kernel    the one-sided Jacobi SVD on its own (the recompression
//                       and the tail run the same code inside their kernels).
// One wavefront of 64 lanes works on one matrix: the blocks are at most a
// few hundred rows by a few dozen columns, and the factorization's critical
// path is a long chain of such small operations, so what counts is the
// length of each one's dependent chain, which the lanes shorten by
// splitting rows and columns between them.
//
// Matrices are column-major with the stated leading dimensions; every
// buffer is device memory owned by the caller.
#include <hip/hip_runtime.h>
#include <math.h>

#include "internal.hpp"

namespace {

constexpr int kWave = 64;
// A kernel whose working set fits in this much shared memory (LDS) works
// there, the inputs copied in and the results out; a larger one works in
// the caller's device buffers.  (64 KiB per workgroup in all, a few KiB
// left for the kernels' own shared arrays.)
constexpr size_t kLdsBytes = 60 * 1024;

// Copy of an m x n column-major block between leading dimensions.
__device__ __forceinline__ void wave_copy(int m, int n, const c128* src, int lds_, c128* dst, int ldd) {
    for (size_t e = threadIdx.x; e < (size_t)m * n; e += kWave) {
        const int i = (int)(e % m), j = (int)(e / m);
        dst[(size_t)j * ldd + i] = src[(size_t)j * lds_ + i];
    }
}

// Sum over all lanes; every lane gets lane 0's result (the butterfly leaves
// results that can differ in the last bit from lane to lane, and control
// flow that depends on them has to be uniform).
__device__ __forceinline__ double wave_sum(double x) {
    for (int m = kWave / 2; m > 0; m >>= 1) x += __shfl_xor(x, m);
    return __shfl(x, 0);
}
__device__ __forceinline__ int wave_sum_int(int x) {
    for (int m = kWave / 2; m > 0; m >>= 1) x += __shfl_xor(x, m);
    return __shfl(x, 0);
}

// Sum over an aligned group of g lanes (g a power of two), the group's first
// lane's result given to all of its lanes.
__device__ __forceinline__ double group_sum(double x, int g) {
    for (int m = g / 2; m > 0; m >>= 1) x += __shfl_xor(x, m);
    return __shfl(x, (int)(threadIdx.x & ~(unsigned)(g - 1)));
}

// M(:, j) -= (2 / vv) v (v^H M(:, j)) for j in [j0, j1): the Householder
// reflector I - 2 v v^H / vv, v zero above row c, applied to columns of the
// p-row matrix M.  The lanes form kc column slots (kc the power of two at
// or above the column count, at most 64) times 64 / kc row strides; a
// column's inner product is the sum over its slot's lanes.
__device__ void apply_reflector(int p, int c, const c128* __restrict__ v, double vv, c128* M, int j0, int j1) {
    const int lane = threadIdx.x;
    const double sc = 2.0 / vv;
    for (int jb = j0; jb < j1; jb += kWave) {
        const int nc = min(kWave, j1 - jb);
        int kc = 1;
        while (kc < nc) kc <<= 1;
        const int G = kWave / kc, col = lane & (kc - 1), rg = lane / kc;
        const bool act = col < nc;
        c128* Mj = M + (size_t)(jb + (act ? col : 0)) * p;
        c128 s = czero<double>();
        if (act)
            for (int i = c + rg; i < p; i += G) cfma_conj(s, v[i], Mj[i]);
        for (int m = kc; m < kWave; m <<= 1) {
            s.re += __shfl_xor(s.re, m);
            s.im += __shfl_xor(s.im, m);
        }
        s.re = __shfl(s.re, col);
        s.im = __shfl(s.im, col);
        const c128 f = sc * s;
        if (act)
            for (int i = c + rg; i < p; i += G) Mj[i] -= f * v[i];
    }
}

// Thin QR of the p x k matrix A, kk = min(p, k): Householder reflectors
// H_c = I - 2 v v^H / (v^H v) reduce a copy W (p x k) to R, the upper
// kk x k part of W; the reflectors are kept in Vh (p x kk) and Q = H_0 ...
// H_{kk-1} applied to the first kk columns of the identity (p x kk).
// The matrix is in W on entry (overwritten); ends after a barrier.
__device__ void wave_qr(int p, int k, c128* W, c128* Vh, c128* Q, c128* R) {
    const int lane = threadIdx.x;
    const int kk = min(p, k);
    for (size_t e = lane; e < (size_t)p * kk; e += kWave) Vh[e] = czero<double>();
    __syncthreads();
    for (int c = 0; c < kk; ++c) {
        c128* v = Vh + (size_t)c * p;
        const c128* w = W + (size_t)c * p;
        double part = 0.0;
        for (int i = c + lane; i < p; i += kWave) part += abs2(w[i]);
        const double nx = sqrt(wave_sum(part));
        if (nx == 0.0) continue;                     // column already zero: H_c = I, v stays zero
        const c128 x0 = w[c];
        const double a0 = hypot(x0.re, x0.im);
        const c128 ph = a0 > 0.0 ? mk(x0.re / a0, x0.im / a0) : mk(1.0, 0.0);
        // v = x + ph |x| e_c maps x to -ph |x| e_c without cancellation, and
        // v^H v = 2 |x| (|x| + |x_c|)
        for (int i = c + lane; i < p; i += kWave) v[i] = i == c ? x0 + nx * ph : w[i];
        const double vv = 2.0 * nx * (nx + a0);
        __syncthreads();
        apply_reflector(p, c, v, vv, W, c, k);
        __syncthreads();
    }
    for (size_t e = lane; e < (size_t)kk * k; e += kWave) {
        const int i = (int)(e % kk), j = (int)(e / kk);
        R[e] = i <= j ? W[(size_t)j * p + i] : czero<double>();
    }
    for (size_t e = lane; e < (size_t)p * kk; e += kWave) {
        const int i = (int)(e % p), j = (int)(e / p);
        Q[e] = mk(i == j ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    // backward accumulation: when H_c is applied, columns j < c of Q are
    // still e_j, zero on rows >= c, so only columns c.. change
    for (int c = kk - 1; c >= 0; --c) {
        const c128* v = Vh + (size_t)c * p;
        double part = 0.0;
        for (int i = c + lane; i < p; i += kWave) part += abs2(v[i]);
        const double vv = wave_sum(part);
        if (vv == 0.0) continue;
        apply_reflector(p, c, v, vv, Q, c, kk);
        __syncthreads();
    }
    __syncthreads();
}

// The two QRs of a recompression at once, one per half-wavefront (team t =
// lane / 32 factors the p_t x k matrix in W_t): both halves run the same
// instructions on their own matrix, every loop bound, shuffle and barrier
// taken by the whole wave (a half with nothing left to do idles), so the
// pair costs about one QR.  Same results as wave_qr on each matrix; ends
// after a barrier.
__device__ void wave_qr_pair(int k, int p0, c128* W0, c128* Vh0, c128* Q0, c128* R0, int p1, c128* W1, c128* Vh1,
                             c128* Q1, c128* R1) {
    constexpr int kHalf = kWave / 2;
    const int lane = threadIdx.x, team = lane / kHalf, tl = lane % kHalf, lead = team * kHalf;
    const int p = team ? p1 : p0;
    c128* W = team ? W1 : W0;
    c128* Vh = team ? Vh1 : Vh0;
    c128* Q = team ? Q1 : Q0;
    c128* R = team ? R1 : R0;
    const int kk = min(p, k);
    const int kk0 = min(p0, k), kk1 = min(p1, k), kmax = max(kk0, kk1);
    for (size_t e = tl; e < (size_t)p * kk; e += kHalf) Vh[e] = czero<double>();
    __syncthreads();
    // one reflector on columns [j0, j_t) of each half's matrix (j_t per half)
    auto reflect = [&](bool go, int c, const c128* v, double vv, c128* M, int j0, int j1, int j1max) {
        const double sc = go ? 2.0 / vv : 0.0;
        for (int jb = j0; jb < j1max; jb += kHalf) {
            const int nc = go ? max(0, min(kHalf, j1 - jb)) : 0;
            const int ncmax = min(kHalf, j1max - jb);
            int kc = 1;
            while (kc < ncmax) kc <<= 1;                // the same slot count in both halves
            const int G = kHalf / kc, col = tl & (kc - 1), rg = tl / kc;
            const bool act = col < nc;
            c128* Mj = M + (size_t)(jb + (act ? col : 0)) * p;
            c128 s = czero<double>();
            if (act)
                for (int i = c + rg; i < p; i += G) cfma_conj(s, v[i], Mj[i]);
            for (int m = kc; m < kHalf; m <<= 1) {
                s.re += __shfl_xor(s.re, m);
                s.im += __shfl_xor(s.im, m);
            }
            s.re = __shfl(s.re, lead + col);
            s.im = __shfl(s.im, lead + col);
            const c128 f = sc * s;
            if (act)
                for (int i = c + rg; i < p; i += G) Mj[i] -= f * v[i];
        }
    };
    auto half_sum = [&](double x) {
        for (int m = kHalf / 2; m > 0; m >>= 1) x += __shfl_xor(x, m);
        return __shfl(x, lead);
    };
    for (int c = 0; c < kmax; ++c) {
        const bool on = c < kk;
        c128* v = Vh + (size_t)(on ? c : 0) * p;
        const c128* w = W + (size_t)(on ? c : 0) * p;
        double part = 0.0;
        if (on)
            for (int i = c + tl; i < p; i += kHalf) part += abs2(w[i]);
        const double nx = sqrt(half_sum(part));
        const bool go = on && nx != 0.0;
        double vv = 1.0;
        if (go) {
            const c128 x0 = w[c];
            const double a0 = hypot(x0.re, x0.im);
            const c128 ph = a0 > 0.0 ? mk(x0.re / a0, x0.im / a0) : mk(1.0, 0.0);
            for (int i = c + tl; i < p; i += kHalf) v[i] = i == c ? x0 + nx * ph : w[i];
            vv = 2.0 * nx * (nx + a0);
        }
        __syncthreads();
        reflect(go, c, v, vv, W, c, k, k);
        __syncthreads();
    }
    for (size_t e = tl; e < (size_t)kk * k; e += kHalf) {
        const int i = (int)(e % kk), j = (int)(e / kk);
        R[e] = i <= j ? W[(size_t)j * p + i] : czero<double>();
    }
    for (size_t e = tl; e < (size_t)p * kk; e += kHalf) {
        const int i = (int)(e % p), j = (int)(e / p);
        Q[e] = mk(i == j ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    for (int c = kmax - 1; c >= 0; --c) {
        const bool on = c < kk;
        const c128* v = Vh + (size_t)(on ? c : 0) * p;
        double part = 0.0;
        if (on)
            for (int i = c + tl; i < p; i += kHalf) part += abs2(v[i]);
        const double vv = half_sum(part);
        const bool go = on && vv != 0.0;
        reflect(go, c, v, vv, Q, c, kk, kmax);
        __syncthreads();
    }
    __syncthreads();
}

__global__ void __launch_bounds__(kWave) zqr_wave_kernel(int p, int k, const c128* __restrict__ A, int lda, c128* W,
                                                         c128* Vh, c128* Q, c128* R, c128* Qc, int staged) {
    HIP_DYNAMIC_SHARED(c128, lds)
    const int kk = min(p, k);
    c128 *w = W, *vh = Vh, *q = Q, *r = R;
    if (staged) {
        w = lds;
        vh = w + (size_t)p * k;
        q = vh + (size_t)p * kk;
        r = q + (size_t)p * kk;
    }
    wave_copy(p, k, A, lda, w, p);
    __syncthreads();
    wave_qr(p, k, w, vh, q, r);
    if (staged) {
        wave_copy(p, kk, q, p, Q, p);
        wave_copy(kk, k, r, kk, R, kk);
    }
    if (Qc)
        for (size_t e = threadIdx.x; e < (size_t)p * kk; e += kWave) Qc[e] = conj(q[e]);
}

// Pair kp of round r of the circle-method round robin over B (even)
// players: player B - 1 stays, the others turn; over B - 1 rounds every
// pair meets once and each round's pairs are disjoint.  p < q.
__device__ __forceinline__ void round_robin_pair(int B, int r, int kp, int& p, int& q) {
    const int n1 = B - 1;
    if (kp == 0) {
        p = r;
        q = n1;
    } else {
        p = (r + kp) % n1;
        q = (r - kp + n1) % n1;
    }
    if (p > q) { const int t = p; p = q; q = t; }
}

// One-sided Jacobi SVD of the a x b matrix A (in place, A becomes A V): each
// round rotates a set of disjoint column pairs at once (round-robin order),
// a group of lanes per pair; a pair is rotated unless it is orthogonal to
// 1e-15 relative or one of its columns is below 1e-15 of the other's norm
// (with b > a the surplus columns shrink to rounding noise).  Sweeps of all
// pairs repeat until one rotates nothing (at most 80); a pair whose columns
// are both below 1e-15 of the matrix's Frobenius norm is left alone.  V (b x b) is the
// product of the rotations.  Then sigma_j = |column j|, perm lists the
// columns by decreasing sigma (ties by index; NaN last), and *rank is the
// number kept: sigma > tol * sigma_max (sigma > 0 when tol = 0), at most
// rmax.
__device__ void order_columns(int a, int b, const c128* A, int lda, double* sig, int* perm, int* rank, double tol,
                              int rmax);

// Ends after a barrier, *rank written.
__device__ void wave_svd(int a, int b, c128* A, int lda, c128* V, double* sig, int* perm, int* rank, double tol,
                         int rmax) {
    const int lane = threadIdx.x;
    for (size_t e = lane; e < (size_t)b * b; e += kWave) {
        const int i = (int)(e % b), j = (int)(e / b);
        V[e] = mk(i == j ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    // the squared Frobenius norm, which the rotations keep: pairs of columns
    // that are both below 1e-15 of it are rounding noise and stay as they are
    // (rotating them never converges once b > a, and their inner products
    // reach the subnormal range, where the phase below loses its modulus 1)
    double fro = 0.0;
    for (size_t e = lane; e < (size_t)a * b; e += kWave) fro += abs2(A[(e / a) * lda + e % a]);
    const double noise = 1e-30 * wave_sum(fro);
    const int B = b + (b & 1);                       // a dummy player when b is odd
    const int npair = B / 2;
    int g = 1;                                       // lanes per pair
    while (2 * g * npair <= kWave) g <<= 1;
    const int per = kWave / g;                       // pairs per pass
    const int gl = lane & (g - 1);
    for (int sweep = 0; sweep < 80 && B >= 2; ++sweep) {
        int rot = 0;
        for (int r = 0; r < B - 1; ++r) {
            for (int k0 = 0; k0 < npair; k0 += per) {
                const int kp = k0 + lane / g;
                int p = 0, q = 0;
                if (kp < npair) round_robin_pair(B, r, kp, p, q);
                const bool valid = kp < npair && q < b;
                c128* x = A + (size_t)(valid ? p : 0) * lda;
                c128* y = A + (size_t)(valid ? q : 0) * lda;
                double al = 0.0, be = 0.0;
                c128 ga = czero<double>();
                if (valid)
                    for (int i = gl; i < a; i += g) {
                        const c128 xi = x[i], yi = y[i];
                        al += abs2(xi);
                        be += abs2(yi);
                        cfma_conj(ga, xi, yi);
                    }
                al = group_sum(al, g);
                be = group_sum(be, g);
                ga.re = group_sum(ga.re, g);
                ga.im = group_sum(ga.im, g);
                // |ga| without squaring: a squared tiny inner product
                // underflows, and the phase below must have modulus 1
                const double gabs = hypot(ga.re, ga.im);
                bool turn = valid && gabs > 1e-15 * sqrt(al) * sqrt(be);
                if (be < 1e-30 * al || al < 1e-30 * be || (al <= noise && be <= noise)) turn = false;
                if (turn) {
                    if (gl == 0) ++rot;
                    // with w = e^{-i phi} y (phi = arg ga) the pair (x, w)
                    // has the real inner product |ga|; the real rotation that
                    // diagonalizes [[al, |ga|], [|ga|, be]] is applied to (x, w)
                    const c128 e = mk(ga.re / gabs, -ga.im / gabs);
                    const double zeta = (be - al) / (2.0 * gabs);
                    const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                    const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
                    for (int i = gl; i < a; i += g) {
                        const c128 xi = x[i], wi = e * y[i];
                        x[i] = cs * xi - sn * wi;
                        y[i] = sn * xi + cs * wi;
                    }
                    c128* vx = V + (size_t)p * b;
                    c128* vy = V + (size_t)q * b;
                    for (int i = gl; i < b; i += g) {
                        const c128 xi = vx[i], wi = e * vy[i];
                        vx[i] = cs * xi - sn * wi;
                        vy[i] = sn * xi + cs * wi;
                    }
                }
            }
            __syncthreads();
        }
        if (wave_sum_int(rot) == 0) break;
    }
    order_columns(a, b, A, lda, sig, perm, rank, tol, rmax);
}

// sigma_j = |column j| of the a x b matrix A, perm the columns by decreasing
// sigma (ties by index; NaN last), *rank the number kept: sigma > tol *
// sigma_max (sigma > 0 when tol = 0), at most rmax.  Ends after a barrier.
__device__ void order_columns(int a, int b, const c128* A, int lda, double* sig, int* perm, int* rank, double tol,
                              int rmax) {
    const int lane = threadIdx.x;
    for (int j = lane; j < b; j += kWave) {
        const c128* x = A + (size_t)j * lda;
        double s0 = 0.0, s1 = 0.0;
        int i = 0;
        for (; i + 1 < a; i += 2) {
            s0 += abs2(x[i]);
            s1 += abs2(x[i + 1]);
        }
        if (i < a) s0 += abs2(x[i]);
        sig[j] = sqrt(s0 + s1);
    }
    __syncthreads();
    // position of column j in decreasing order: the number of columns ahead
    // of it (larger sigma, or equal and a smaller index; NaN counts as -1,
    // so the order is total and perm a permutation)
    for (int j = lane; j < b; j += kWave) {
        const double sj = isnan(sig[j]) ? -1.0 : sig[j];
        int pos = 0;
        for (int i = 0; i < b; ++i) {
            const double si = isnan(sig[i]) ? -1.0 : sig[i];
            pos += (si > sj || (si == sj && i < j)) ? 1 : 0;
        }
        perm[pos] = j;
    }
    __syncthreads();
    if (lane == 0) {
        int r = 0;
        if (b > 0 && sig[perm[0]] > 0.0) {
            const double cut = tol > 0.0 ? tol * sig[perm[0]] : 0.0;
            for (int j = 0; j < b; ++j) r += sig[perm[j]] > cut ? 1 : 0;
            if (r > rmax) r = rmax;
        }
        *rank = r;
    }
    __syncthreads();
}

__global__ void __launch_bounds__(kWave) zsvd_wave_kernel(int a, int b, c128* A, int lda, c128* V, double* sig,
                                                          int* perm, int* rank, double tol, int rmax, int staged) {
    HIP_DYNAMIC_SHARED(c128, lds)
    if (!staged) {
        wave_svd(a, b, A, lda, V, sig, perm, rank, tol, rmax);
        return;
    }
    c128* As = lds;
    c128* Vs = As + (size_t)a * b;
    double* sg = (double*)(Vs + (size_t)b * b);
    int* pm = (int*)(sg + b);
    int* rk = pm + b;
    wave_copy(a, b, A, lda, As, a);
    __syncthreads();
    wave_svd(a, b, As, a, Vs, sg, pm, rk, tol, rmax);
    wave_copy(a, b, As, a, A, lda);
    wave_copy(b, b, Vs, b, V, b);
    for (int j = threadIdx.x; j < b; j += kWave) {
        sig[j] = sg[j];
        perm[j] = pm[j];
    }
    if (threadIdx.x == 0) *rank = *rk;
}

// Inverse X (m x m) of the m x m matrix A by Gauss-Jordan elimination with
// partial pivoting (the largest modulus, the first on ties), on a copy in W
// (m x m, followed by one column of m multipliers), the same row operations
// applied to X = I.  A lane owns columns of [W X].  A zero pivot sets
// *status to 1.
__global__ void __launch_bounds__(kWave) zinv_wave_kernel(int m, const c128* __restrict__ A, int lda, c128* Wg,
                                                          c128* Xg, int* status, int staged) {
    HIP_DYNAMIC_SHARED(c128, lds)
    const int lane = threadIdx.x;
    c128* W = staged ? lds : Wg;
    c128* X = staged ? lds + (size_t)m * (m + 1) : Xg;
    c128* F = W + (size_t)m * m;
    for (size_t e = lane; e < (size_t)m * m; e += kWave) {
        const int i = (int)(e % m), j = (int)(e / m);
        W[e] = A[(size_t)j * lda + i];
        X[e] = mk(i == j ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    for (int c = 0; c < m; ++c) {
        double best = -1.0;
        int p = m;
        for (int r = c + lane; r < m; r += kWave) {
            const double v = abs2(W[(size_t)c * m + r]);
            if (v > best) { best = v; p = r; }
        }
        for (int s = kWave / 2; s > 0; s >>= 1) {
            const double ob = __shfl_xor(best, s);
            const int op = __shfl_xor(p, s);
            if (ob > best || (ob == best && op < p)) { best = ob; p = op; }
        }
        best = __shfl(best, 0);
        p = __shfl(p, 0);
        if (!(best > 0.0)) {
            if (lane == 0) *status = 1;
            return;
        }
        if (p != c)
            for (int j = lane; j < 2 * m; j += kWave) {
                c128* M = j < m ? W + (size_t)j * m : X + (size_t)(j - m) * m;
                const c128 t = M[c];
                M[c] = M[p];
                M[p] = t;
            }
        __syncthreads();
        const c128 piv = cinv(W[(size_t)c * m + c]);
        for (int r = lane; r < m; r += kWave) F[r] = W[(size_t)c * m + r];
        __syncthreads();
        for (int j = lane; j < 2 * m; j += kWave) {
            c128* M = j < m ? W + (size_t)j * m : X + (size_t)(j - m) * m;
            const c128 t = piv * M[c];
            M[c] = t;
            for (int r = 0; r < m; ++r)
                if (r != c) M[r] -= F[r] * t;
        }
        __syncthreads();
    }
    if (staged) wave_copy(m, m, X, m, Xg, m);
}

// Block operations of one launch, one workgroup each, passed by value.
constexpr int kJobBatch = 32;
struct BlockJobBatch {
    BlockJob job[kJobBatch];
    double tol;
    int rmax;
    unsigned lds;          // shared-memory bytes of the launch
};

// The dense block operations of a batch (one workgroup, lanes over entries).
__device__ void dense_job(const BlockJob& J) {
    const int m = J.m, q = J.q;
    const size_t n = (size_t)m * q;
    const c128 alpha = J.alpha;
    for (size_t e = threadIdx.x; e < n; e += kWave) {
        const int i = (int)(e % m), j = (int)(e / m);
        c128 v;
        if (J.kind == JOB_SUM) {
            v = J.au[e] + alpha * J.av[e];
        } else if (J.kind == JOB_LOWRANK) {
            c128 a0 = czero<double>(), a1 = a0;
            int l = 0;
            for (; l + 1 < J.k2; l += 2) {
                cfma(a0, J.U[(size_t)l * J.ldu + i], J.V[(size_t)l * J.ldv + j]);
                cfma(a1, J.U[(size_t)(l + 1) * J.ldu + i], J.V[(size_t)(l + 1) * J.ldv + j]);
            }
            if (l < J.k2) cfma(a0, J.U[(size_t)l * J.ldu + i], J.V[(size_t)l * J.ldv + j]);
            v = J.ou[e] + alpha * (a0 + a1);
        } else if (J.kind == JOB_SCALE) {
            v = J.U[i] * J.au[e];
            if (J.V) v = v * J.V[j];
        } else {
            v = J.au[e];
        }
        J.ou[e] = v;
    }
}

// Job blockIdx.x: a dense block operation (dense_job), or the truncated
// product of [au, alpha U] (m x k) and [av, V] (q x k), k = k1 + k2: QR of
// both stacked factors, SVD of the core C = R1 R2^t, and the factors ou =
// Q1 (C V)_r (m x r) and ov = Q2 conj(V_r) (q x r), r = min(m, q, k, rmax)
// columns of which those past the kept rank are zero.
__global__ void __launch_bounds__(kWave) block_jobs_kernel(BlockJobBatch B) {
    HIP_DYNAMIC_SHARED(c128, lds)
    const BlockJob& J = B.job[blockIdx.x];
    if (J.kind != JOB_RECOMPRESS) {
        dense_job(J);
        return;
    }
    const int m = J.m, q = J.q, k1 = J.k1, k2 = J.k2, rmax = B.rmax;
    const int lane = threadIdx.x, k = k1 + k2;
    const int kk1 = min(m, k), kk2 = min(q, k), r = min(min(kk1, kk2), rmax);
    const RecompressLayout L = recompress_layout(m, q, k, rmax);
    c128* work = L.total * sizeof(c128) <= B.lds ? lds : J.work;
    c128 *W1 = work + L.W1, *Vh1 = work + L.Vh1, *Q1 = work + L.Q1, *R1 = work + L.R1;
    c128 *W2 = work + L.W2, *Vh2 = work + L.Vh2, *Q2 = work + L.Q2, *R2 = work + L.R2;
    c128 *C = work + L.C, *Vs = work + L.Vs, *Cg = work + L.Cg, *Vg = work + L.Vg;
    double* sig = (double*)(work + L.sig);
    int* perm = (int*)(work + L.perm);
    int* rank = (int*)(work + L.rank);
    const c128 alpha = J.alpha;
    for (size_t e = lane; e < (size_t)m * k; e += kWave) {
        const int i = (int)(e % m), j = (int)(e / m);
        W1[e] = j < k1 ? J.au[(size_t)j * m + i] : alpha * J.U[(size_t)(j - k1) * J.ldu + i];
    }
    for (size_t e = lane; e < (size_t)q * k; e += kWave) {
        const int i = (int)(e % q), j = (int)(e / q);
        W2[e] = j < k1 ? J.av[(size_t)j * q + i] : J.V[(size_t)(j - k1) * J.ldv + i];
    }
    __syncthreads();
    wave_qr_pair(k, m, W1, Vh1, Q1, R1, q, W2, Vh2, Q2, R2);
    for (size_t e = lane; e < (size_t)kk1 * kk2; e += kWave) {
        const int i = (int)(e % kk1), j = (int)(e / kk1);
        c128 acc = czero<double>();
        for (int l = j; l < k; ++l) cfma(acc, R1[(size_t)l * kk1 + i], R2[(size_t)l * kk2 + j]);   // R2 upper
        C[e] = acc;
    }
    __syncthreads();
    wave_svd(kk1, kk2, C, kk1, Vs, sig, perm, rank, B.tol, rmax);
    const int rk = *rank;
    for (size_t e = lane; e < (size_t)kk1 * r; e += kWave) {
        const int i = (int)(e % kk1), j = (int)(e / kk1);
        Cg[e] = j < rk ? C[(size_t)perm[j] * kk1 + i] : czero<double>();
    }
    for (size_t e = lane; e < (size_t)kk2 * r; e += kWave) {
        const int i = (int)(e % kk2), j = (int)(e / kk2);
        Vg[e] = j < rk ? conj(Vs[(size_t)perm[j] * kk2 + i]) : czero<double>();
    }
    __syncthreads();
    for (size_t e = lane; e < (size_t)m * r; e += kWave) {
        const int i = (int)(e % m), j = (int)(e / m);
        c128 acc = czero<double>();
        for (int l = 0; l < kk1; ++l) cfma(acc, Q1[(size_t)l * m + i], Cg[(size_t)j * kk1 + l]);
        J.ou[e] = acc;
    }
    for (size_t e = lane; e < (size_t)q * r; e += kWave) {
        const int i = (int)(e % q), j = (int)(e / q);
        c128 acc = czero<double>();
        for (int l = 0; l < kk2; ++l) cfma(acc, Q2[(size_t)l * q + i], Vg[(size_t)j * kk2 + l]);
        J.ov[e] = acc;
    }
}

// Products of leaf blocks with blocks of vectors, one workgroup each.
constexpr int kMvBatch = 64;
constexpr int kMvThreads = 128;
struct MatvecBatch {
    MatvecOp op[kMvBatch];
    const c128* X;
    c128* Y;
    c128* T;              // device temporaries of the factorized ops (or null: shared memory)
    c128 alpha;
    int ldx, ldy, ncol, trans, assign;
    size_t tstride;       // entries of T per op
};

// Y(yo + i, j) += alpha sum_l op(block)(i, l) X(xo + l, j) for op blockIdx.x
// (= instead of += when B.assign; kind 2 clears its rows).
// op(block) of a dense block is its entries (trans 0) or their transpose;
// of a factorized block U V^t it is U (V^t X) or V (U^t X), the r x ncol
// middle product in shared memory.
__global__ void __launch_bounds__(kMvThreads) hmatvec_kernel(MatvecBatch B) {
    HIP_DYNAMIC_SHARED(c128, lds)
    const MatvecOp& o = B.op[blockIdx.x];
    const int tid = threadIdx.x, ncol = B.ncol, tr = B.trans;
    const int out = tr ? o.q : o.m, in = tr ? o.m : o.q;
    const c128* X = B.X + o.xo;
    c128* Y = B.Y + o.yo;
    const c128 alpha = B.alpha;
    if (o.kind == 2) {
        for (int e = tid; e < o.m * ncol; e += kMvThreads) Y[(size_t)(e / o.m) * B.ldy + e % o.m] = czero<double>();
        return;
    }
    const bool add = !B.assign;
    if (o.kind == 0) {
        const c128* D = o.a;
        for (int e = tid; e < out * ncol; e += kMvThreads) {
            const int i = e % out, j = e / out;
            const c128* x = X + (size_t)j * B.ldx;
            c128 a0 = czero<double>(), a1 = a0;
            int l = 0;
            if (tr) {
                const c128* d = D + (size_t)i * o.m;            // column i of the block = row i of its transpose
                for (; l + 1 < in; l += 2) {
                    cfma(a0, d[l], x[l]);
                    cfma(a1, d[l + 1], x[l + 1]);
                }
                if (l < in) cfma(a0, d[l], x[l]);
            } else {
                for (; l + 1 < in; l += 2) {
                    cfma(a0, D[(size_t)l * o.m + i], x[l]);
                    cfma(a1, D[(size_t)(l + 1) * o.m + i], x[l + 1]);
                }
                if (l < in) cfma(a0, D[(size_t)l * o.m + i], x[l]);
            }
            const c128 v = alpha * (a0 + a1);
            Y[(size_t)j * B.ldy + i] = add ? Y[(size_t)j * B.ldy + i] + v : v;
        }
        return;
    }
    // factorized: P (in x r) applied first, then Q (out x r)
    const c128* P = tr ? o.a : o.b;
    const c128* Q = tr ? o.b : o.a;
    const int r = o.r;
    c128* T = B.T ? B.T + (size_t)blockIdx.x * B.tstride : lds;
    for (int e = tid; e < r * ncol; e += kMvThreads) {
        const int k = e % r, j = e / r;
        const c128* p = P + (size_t)k * in;
        const c128* x = X + (size_t)j * B.ldx;
        c128 a0 = czero<double>(), a1 = a0;
        int l = 0;
        for (; l + 1 < in; l += 2) {
            cfma(a0, p[l], x[l]);
            cfma(a1, p[l + 1], x[l + 1]);
        }
        if (l < in) cfma(a0, p[l], x[l]);
        T[e] = a0 + a1;
    }
    __syncthreads();
    for (int e = tid; e < out * ncol; e += kMvThreads) {
        const int i = e % out, j = e / out;
        c128 acc = czero<double>();
        for (int k = 0; k < r; ++k) cfma(acc, Q[(size_t)k * out + i], T[(size_t)j * r + k]);
        const c128 v = alpha * acc;
        Y[(size_t)j * B.ldy + i] = add ? Y[(size_t)j * B.ldy + i] + v : v;
    }
}

// The SVD of a tall a x b matrix A (b <= 64 columns) through its Gram
// matrix: G = A^H A in FP64, diagonalized by a parallel two-sided Jacobi
// (each round rotates a round-robin set of disjoint index pairs: the
// rotation's parameters are entries of G, so a round needs no cross-lane
// sums; the columns of G and V are rotated, then the rows of G), then W = A V
// and its columns ordered as wave_svd orders A V.  Squaring costs accuracy
// only for singular values far below the largest (relative error about
// 1e-16 (sigma_1 / sigma_j)^2), where the truncation cuts.  A pair is
// rotated unless its off-diagonal entry is below 1e-15 of the geometric
// mean of its diagonal, or one diagonal is below 1e-30 of the other, or both
// are below 1e-30 of the trace.  Ends after a barrier.
__device__ void wave_gram_svd(int a, int b, const c128* A, int lda, c128* G, c128* V, c128* W, double* sig, int* perm,
                              int* rank, double tol, int rmax) {
    __shared__ double pcs[32], psn[32];
    __shared__ c128 pe[32];
    __shared__ int pturn[32];
    const int lane = threadIdx.x;
    for (int e = lane; e < b * b; e += kWave) V[e] = mk(e % b == e / b ? 1.0 : 0.0, 0.0);
    // G (column-major, both triangles), entry (i, j) with i <= j by one lane
    for (int e = lane; e < b * (b + 1) / 2; e += kWave) {
        int j = 0;
        while ((j + 1) * (j + 2) / 2 <= e) ++j;
        const int i = e - j * (j + 1) / 2;
        const c128* x = A + (size_t)i * lda;
        const c128* y = A + (size_t)j * lda;
        c128 g0 = czero<double>(), g1 = g0;
        int l = 0;
        for (; l + 1 < a; l += 2) {
            cfma_conj(g0, x[l], y[l]);
            cfma_conj(g1, x[l + 1], y[l + 1]);
        }
        if (l < a) cfma_conj(g0, x[l], y[l]);
        const c128 g = g0 + g1;
        G[(size_t)j * b + i] = g;
        G[(size_t)i * b + j] = conj(g);
    }
    __syncthreads();
    double tr = 0.0;
    for (int j = lane; j < b; j += kWave) tr += G[(size_t)j * b + j].re;
    const double noise = 1e-30 * wave_sum(tr);
    const int B = b + (b & 1), npair = B / 2;
    for (int sweep = 0; sweep < 80 && B >= 2; ++sweep) {
        int rot = 0;
        for (int r = 0; r < B - 1; ++r) {
            for (int kp = lane; kp < npair; kp += kWave) {
                int p = 0, q = 0;
                round_robin_pair(B, r, kp, p, q);
                bool turn = q < b;
                double cs = 1.0, sn = 0.0;
                c128 e = mk(1.0, 0.0);
                if (turn) {
                    const double al = G[(size_t)p * b + p].re, be = G[(size_t)q * b + q].re;
                    const c128 ga = G[(size_t)q * b + p];
                    const double gabs = hypot(ga.re, ga.im);
                    turn = gabs > 1e-15 * sqrt(fabs(al)) * sqrt(fabs(be));
                    if (be < 1e-30 * al || al < 1e-30 * be || (al <= noise && be <= noise)) turn = false;
                    if (turn) {
                        ++rot;
                        e = mk(ga.re / gabs, -ga.im / gabs);
                        const double zeta = (be - al) / (2.0 * gabs);
                        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                        cs = 1.0 / sqrt(1.0 + t * t);
                        sn = cs * t;
                    }
                }
                pturn[kp] = turn;
                pcs[kp] = cs;
                psn[kp] = sn;
                pe[kp] = e;
            }
            __syncthreads();
            // columns p, q of G and V: x' = cs x - sn e y, y' = sn x + cs e y
            for (int e2 = lane; e2 < npair * 2 * b; e2 += kWave) {
                const int kp = e2 / (2 * b), i = e2 % b;
                const bool onv = (e2 / b) % 2 == 1;
                if (!pturn[kp]) continue;
                int p = 0, q = 0;
                round_robin_pair(B, r, kp, p, q);
                c128* M = onv ? V : G;
                const c128 x = M[(size_t)p * b + i], w = pe[kp] * M[(size_t)q * b + i];
                M[(size_t)p * b + i] = pcs[kp] * x - psn[kp] * w;
                M[(size_t)q * b + i] = psn[kp] * x + pcs[kp] * w;
            }
            __syncthreads();
            // rows p, q of G: row_p' = cs row_p - sn conj(e) row_q, row_q' = sn row_p + cs conj(e) row_q
            for (int e2 = lane; e2 < npair * b; e2 += kWave) {
                const int kp = e2 / b, j = e2 % b;
                if (!pturn[kp]) continue;
                int p = 0, q = 0;
                round_robin_pair(B, r, kp, p, q);
                const c128 x = G[(size_t)j * b + p], w = conj(pe[kp]) * G[(size_t)j * b + q];
                G[(size_t)j * b + p] = pcs[kp] * x - psn[kp] * w;
                G[(size_t)j * b + q] = psn[kp] * x + pcs[kp] * w;
            }
            __syncthreads();
        }
        if (wave_sum_int(rot) == 0) break;
    }
    // W = A V (a x b)
    for (size_t e2 = lane; e2 < (size_t)a * b; e2 += kWave) {
        const int i = (int)(e2 % a), j = (int)(e2 / a);
        c128 acc = czero<double>();
        for (int l = 0; l < b; ++l) cfma(acc, A[(size_t)l * lda + i], V[(size_t)j * b + l]);
        W[e2] = acc;
    }
    __syncthreads();
    order_columns(a, b, W, a, sig, perm, rank, tol, rmax);
}

// Randomized-SVD tails of one launch, one workgroup each, passed by value.
constexpr int kTailBatch = 32;
struct RsvdTailBatch {
    RsvdTail job[kTailBatch];
    double tol;
    int rmax;
    unsigned lds;          // shared-memory bytes of the launch
};

// Tail blockIdx.x: SVD of M (staged in shared memory with V when they fit),
// the kept columns, Uo = Q Vg.
__global__ void __launch_bounds__(kWave) rsvd_tail_kernel(RsvdTailBatch B) {
    HIP_DYNAMIC_SHARED(c128, lds)
    const RsvdTail& J = B.job[blockIdx.x];
    const int m = J.m, q = J.q, ell = J.ell, r = min(ell, B.rmax);
    const size_t qe = (size_t)q * ell, ee = (size_t)ell * ell;
    const bool staged = rsvd_tail_entries(q, ell) * sizeof(c128) <= B.lds;
    c128* A = staged ? lds : J.M;
    c128* V = staged ? lds + qe : J.V;
    if (staged) wave_copy(q, ell, J.M, q, A, q);
    __syncthreads();
    if (ell <= 64) {
        // through the ell x ell Gram matrix; A V lands in W
        c128* W = staged ? V + ee : J.work;
        c128* G = W + qe;
        wave_gram_svd(q, ell, A, q, G, V, W, J.sig, J.perm, J.rank, B.tol, B.rmax);
        A = W;
    } else {
        wave_svd(q, ell, A, q, V, J.sig, J.perm, J.rank, B.tol, B.rmax);
    }
    const int kept = *J.rank;
    for (size_t e = threadIdx.x; e < (size_t)ell * r; e += kWave) {
        const int i = (int)(e % ell), j = (int)(e / ell);
        J.Vg[e] = j < kept ? conj(V[(size_t)J.perm[j] * ell + i]) : czero<double>();
    }
    for (size_t e = threadIdx.x; e < (size_t)q * r; e += kWave) {
        const int i = (int)(e % q), j = (int)(e / q);
        J.Vo[e] = j < kept ? A[(size_t)J.perm[j] * q + i] : czero<double>();
    }
    __syncthreads();
    for (size_t e = threadIdx.x; e < (size_t)m * r; e += kWave) {
        const int i = (int)(e % m), j = (int)(e / m);
        c128 acc = czero<double>();
        for (int l = 0; l < ell; ++l) cfma(acc, J.Q[(size_t)l * m + i], J.Vg[(size_t)j * ell + l]);
        J.Uo[e] = acc;
    }
}

}  // namespace

void launch_block_jobs(const BlockJob* jobs, int count, int rmax, double tol, hipStream_t s) {
    for (int j0 = 0; j0 < count; j0 += kJobBatch) {
        BlockJobBatch B;
        const int nb = count - j0 < kJobBatch ? count - j0 : kJobBatch;
        size_t lds = 0;
        for (int j = 0; j < nb; ++j) {
            const BlockJob& J = jobs[j0 + j];
            B.job[j] = J;
            if (J.kind != JOB_RECOMPRESS) continue;
            const size_t bytes = recompress_layout(J.m, J.q, J.k1 + J.k2, rmax).total * sizeof(c128);
            if (bytes <= kLdsBytes && bytes > lds) lds = bytes;
        }
        B.tol = tol;
        B.rmax = rmax;
        B.lds = (unsigned)lds;
        hipLaunchKernelGGL(block_jobs_kernel, dim3(nb), dim3(kWave), lds, s, B);
    }
}

void launch_small_qr(int p, int k, const c128* A, int lda, c128* W, c128* Vh, c128* Q, c128* R, c128* Qc,
                     hipStream_t s) {
    const size_t kk = p < k ? p : k;
    const size_t bytes = ((size_t)p * k + 2 * (size_t)p * kk + kk * k) * sizeof(c128);
    const int staged = bytes <= kLdsBytes;
    hipLaunchKernelGGL(zqr_wave_kernel, dim3(1), dim3(kWave), staged ? bytes : 0, s, p, k, A, lda, W, Vh, Q, R, Qc,
                       staged);
}

void launch_small_svd(int a, int b, c128* A, int lda, c128* V, double* sig, int* perm, int* rank, double tol,
                      int rmax, hipStream_t s) {
    const size_t bytes = ((size_t)a * b + (size_t)b * b) * sizeof(c128) + (size_t)b * 12 + 16;
    const int staged = bytes <= kLdsBytes;
    hipLaunchKernelGGL(zsvd_wave_kernel, dim3(1), dim3(kWave), staged ? bytes : 0, s, a, b, A, lda, V, sig, perm,
                       rank, tol, rmax, staged);
}

void launch_small_inv(int m, const c128* A, int lda, c128* W, c128* X, int* status, hipStream_t s) {
    const size_t bytes = ((size_t)m * (m + 1) + (size_t)m * m) * sizeof(c128);
    const int staged = bytes <= kLdsBytes;
    hipLaunchKernelGGL(zinv_wave_kernel, dim3(1), dim3(kWave), staged ? bytes : 0, s, m, A, lda, W, X, status, staged);
}

void launch_hmatvec(const MatvecOp* ops, int count, int trans, int assign, const c128* X, int ldx, c128* Y, int ldy,
                    int ncol, c128 alpha, c128* tscratch, hipStream_t s) {
    const size_t need = hmatvec_scratch(ops, count, ncol);
    size_t mr = 0;
    for (int j = 0; j < count; ++j)
        if (ops[j].kind == 1 && (size_t)ops[j].r > mr) mr = ops[j].r;
    for (int j0 = 0; j0 < count; j0 += kMvBatch) {
        MatvecBatch B;
        const int nb = count - j0 < kMvBatch ? count - j0 : kMvBatch;
        for (int j = 0; j < nb; ++j) B.op[j] = ops[j0 + j];
        B.X = X;
        B.Y = Y;
        B.alpha = alpha;
        B.ldx = ldx;
        B.ldy = ldy;
        B.ncol = ncol;
        B.trans = trans;
        B.assign = assign;
        B.tstride = need ? mr * ncol : 0;
        B.T = need ? tscratch + (size_t)j0 * B.tstride : nullptr;
        const size_t lds = need ? 0 : mr * ncol * sizeof(c128);
        hipLaunchKernelGGL(hmatvec_kernel, dim3(nb), dim3(kMvThreads), lds, s, B);
    }
}

void launch_rsvd_tails(const RsvdTail* jobs, int count, int rmax, double tol, hipStream_t s) {
    for (int j0 = 0; j0 < count; j0 += kTailBatch) {
        RsvdTailBatch B;
        const int nb = count - j0 < kTailBatch ? count - j0 : kTailBatch;
        size_t lds = 0;
        for (int j = 0; j < nb; ++j) {
            const RsvdTail& J = jobs[j0 + j];
            B.job[j] = J;
            const size_t bytes = rsvd_tail_entries(J.q, J.ell) * sizeof(c128);
            if (bytes <= kLdsBytes && bytes > lds) lds = bytes;
        }
        B.tol = tol;
        B.rmax = rmax;
        B.lds = (unsigned)lds;
        hipLaunchKernelGGL(rsvd_tail_kernel, dim3(nb), dim3(kWave), lds, s, B);
    }
}
