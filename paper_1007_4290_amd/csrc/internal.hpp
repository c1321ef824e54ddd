// Internal declarations shared by the host orchestration and the kernels.
#pragma once
#include <stddef.h>
#include <stdint.h>
#include <string>
#include <vector>
#include "cplx.hpp"

// Plan of the layer H-matrix: the layer of n unknowns is padded to
// np = b * 2^L entries (the padding unknowns are decoupled, A entry 1), and
// bisected L times.  Node (level l, index i) covers rows [i*np>>l, (i+1)*np>>l)
// and has heap id (1<<l) - 1 + i.  Leaves are the 2^L nodes of level L.
struct Plan {
    int n;        // interior points per side = number of layers
    int np;       // padded layer width
    int b;        // leaf size
    int L;        // number of bisection levels (off-diagonal levels 1..L)
    int r;        // rank cap
    double tol;   // relative truncation threshold
    // complex entries per layer in the factor store
    size_t eK, eP, eX, eLayer;
};

inline void plan_sizes(Plan& p) {
    p.eK = (size_t)p.np * p.b;
    p.eP = (size_t)p.L * p.r * p.np;
    p.eX = (size_t)((1 << p.L) - 1) * 4 * p.r * p.r;
    p.eLayer = p.eK + p.eP + p.eX;
}

// Factor store layout of one layer (element type cpx<T>):
//   K[t*b*b + j*b + i]            leaf t inverse, entry (i, j) (column-major)
//   P[((lvl-1)*r + k)*np + i]     column k of P at level lvl (1..L), row i
//   X[node*4r^2 + col*2r + row]   Woodbury core inverse of non-leaf node (heap id)
// so that T_m = blockdiag(K) - sum_nodes P_node X_node P_node^t where
// P_node = blockdiag(P rows of the two children).

// Pointers of one factorization step (layer m).
template <typename T>
struct StepPtrs {
    cpx<T>* K; cpx<T>* P; cpx<T>* X;                  // layer m (written)
    const cpx<T>* Kp; const cpx<T>* Pp; const cpx<T>* Xp; // layer m-1 (null at m = 0)
    const cpx<T>* dg;   // np: diagonal of A_{m,m} (padding rows: 1)
    const cpx<T>* eo;   // np: eo[i] = A_{m,m}(i, i+1)
    const cpx<T>* cp;   // np: diagonal of A_{m,m-1} (null at m = 0)
    cpx<T>* Q;          // L*r*np: off-diagonal factors of S_m, [lvl-1][k][i]
    cpx<T>* G;          // heap-indexed r*r blocks Q_c^t P_c
    int* rank;          // 2^L - 1 ranks of the off-diagonal blocks of S_m
    int* status;        // set to nonzero on a zero pivot
};

// ---- coefficient kernels (FP64) ----
// Stretching tables of the two axes: 1/s on the n nodes and s on the n+1
// half nodes of x1 (isn1, sh1) and of x2 (isn2, sh2).
struct AxisTables {
    const c128* isn1; const c128* sh1;
    const c128* isn2; const c128* sh2;
    int abc;        // bit k set: side k (HSWEEP_EDGE_* order) has the absorbing boundary condition
};
void launch_pml_1d(int n, double omega, double eta_lo, double eta_hi, double C, c128* isn, c128* sh, hipStream_t s);
// Layer operators in the frame of sweep direction dir (0: +x2, 1: -x2, 2: +x1, 3: -x1).
template <typename T>
void launch_layer_coeffs(int n, int np, int dir, double omega, const double* c, const AxisTables& t, cpx<T>* dg,
                         cpx<T>* eo, cpx<T>* cp, hipStream_t s);
void launch_stencil(int n, int nrhs, double omega, const double* c, const AxisTables& t, const c128* x, const c128* f,
                    c128* y, const int* active, hipStream_t s);
void launch_grad(int n, int nrhs, double omega, const double* c, const AxisTables& t, const c128* u, const c128* mu,
                 double* grad, hipStream_t s);
// f -= coefficient * b for Dirichlet data b on an edge (0: x1=0, 1: x1=1, 2: x2=0, 3: x2=1).
void launch_dirichlet(int n, int nrhs, double omega, const double* c, const AxisTables& t, int edge, const c128* b,
                      c128* f, hipStream_t s);

// One problem instance of a (possibly batched) factorization: its plan and
// the device buffers of its layer coefficients and factor store.
template <typename T>
struct InstDesc {
    Plan p;
    cpx<T>* fac;        // n * eLayer
    const cpx<T>* dg;   // n * np
    const cpx<T>* eo;   // n * np
    const cpx<T>* cp;   // (n-1) * np
    cpx<T>* Q;          // L * r * np
    cpx<T>* G;          // 2^(L+1) * r * r
    int* rank;          // n * 2^L
    int* status;
};

// ---- factorization kernels ----
// Launches layer step m of every instance in `descs` (device array of ninst
// descriptors; `plans` are host copies of their plans).  All instances share
// the element type, leaf size and rank; instances with n <= m are skipped.
// If `after_layer` is given it is recorded on `s` between the layer kernel
// and the Woodbury kernels (for per-kernel timing).
template <typename T>
int launch_factor_layer(const InstDesc<T>* descs, const Plan* plans, int ninst, int m, hipStream_t s,
                        hipEvent_t after_layer = nullptr);
// Sets the kernels' LDS limits (done once; must precede a stream capture).
template <typename T>
void factor_kernels_init();

// ---- sweep (preconditioner application) ----
// One instance of a sweep launch.  For call column j, right-hand side r
// reads f + j*fstride + r*n*n and writes u + j*ustride + r*n*n (natural grid
// order; the sweep maps frame points to grid points by its direction); its
// forward work vectors are w + r*n*np.
template <typename T>
struct SweepInst {
    int n, np, L, nrhs;
    int dir;             // sweep direction: layer m, position i is grid point (see k_coeff.hip)
    size_t eK, eP, eLayer;
    const cpx<T>* fac;   // factor store base (n layers of eLayer entries)
    const cpx<T>* cp;    // (n-1)*np couplings, cp[m*np + i] = A_{m+1,m}(i, i)
    const c128* f;       // complex128 input fields
    c128* u;             // complex128 output fields
    cpx<T>* w;           // nrhs * n * np work
    const int* active;   // nrhs flags (null = all active); inactive ones get u = 0
    size_t fstride, ustride;
};
// Kernel argument of a sweep launch: one instance by value (insts null), or
// a device table of instances with a device table of workgroup tasks.
template <typename T>
struct SweepArgs {
    SweepInst<T> one;
    const SweepInst<T>* insts;
    const int* tasks;      // per workgroup: (instance << 16) | first right-hand side, -1 = idle
    int ngroups, nxcd;     // one instance: its right-hand-side groups and the XCDs they use
    int jf, ju;            // call column of the fields
};
// One instance, right-hand sides in groups of G (1 or 4) per workgroup.
template <typename T>
int launch_sweep(const Plan& p, SweepArgs<T> a, int G, hipStream_t s);
// Several instances (same leaf size and rank) in one launch of `blocks`
// workgroups; `tasks` is a device table of one entry per workgroup.
template <typename T>
int launch_sweep_multi_col(const Plan* plans, int ninst, const SweepInst<T>* insts, const int* tasks, int blocks,
                           int G, int jf, int ju, hipStream_t s);
size_t sweep_lds_bytes(const Plan& p, size_t elem, int G);
bool sweep_supported(const Plan& p);
bool sweep_group_supported(const Plan& p);

// ---- Krylov vector kernels (FP64 complex) ----
// S systems of lengths off[k+1] - off[k] (off: device array of S+1 offsets);
// system k occupies [off[k], off[k+1]) of every vector and vector j of a set
// starts at j * ld.  maxlen: the longest system.
// partial dots: out[j*S + k] = sum_i conj(V_j[i]) * w[i] over system k, j < nv
void launch_multi_dot(const c128* V, int nv, size_t ld, const c128* w, const size_t* off, int S, c128* partial,
                      c128* out, int nblk, hipStream_t s);
// w -= sum_j h[j*S + k] V_j on system k
void launch_multi_axpy(const c128* V, int nv, size_t ld, const c128* h, c128* w, const size_t* off, int S,
                       size_t maxlen, hipStream_t s);
// out = w * scale[k] on system k (scale 0 writes zeros)
void launch_scale(const c128* w, const double* scale, c128* out, const size_t* off, int S, size_t maxlen,
                  hipStream_t s);
// x += sum_j y[j*S + k] Z_j on system k
void launch_combine(const c128* Z, int nz, size_t ld, const c128* y, c128* x, const size_t* off, int S, size_t maxlen,
                    hipStream_t s);
int krylov_dot_blocks(size_t N);
// y = conj(x), n complex entries
void launch_conj(const c128* x, c128* y, size_t n, hipStream_t s);

// ---- small dense complex128 factorizations (k_dense.hip), one wavefront
// per matrix, column-major, all buffers device memory ----
// Thin QR of the p x k matrix A (leading dimension lda), kk = min(p, k):
// Q (p x kk), R (kk x k, upper), with W (p x k) and Vh (p x kk) as work;
// conj(Q) also into Qc (p x kk) when it is not null.
void launch_small_qr(int p, int k, const c128* A, int lda, c128* W, c128* Vh, c128* Q, c128* R, c128* Qc,
                     hipStream_t s);
// One-sided Jacobi SVD of the a x b matrix A in place (A becomes A V), V
// (b x b); sig (b) the column norms, perm (b) the columns by decreasing
// norm, *rank the count above tol * sigma_max (above 0 for tol = 0), at
// most rmax.
void launch_small_svd(int a, int b, c128* A, int lda, c128* V, double* sig, int* perm, int* rank, double tol,
                      int rmax, hipStream_t s);
// X = A^{-1} (m x m) by Gauss-Jordan with partial pivoting; W holds
// m (m + 1) entries of work; a zero pivot sets *status = 1.
void launch_small_inv(int m, const c128* A, int lda, c128* W, c128* X, int* status, hipStream_t s);
// Work layout of a recompression of m x k and q x k factors (offsets in
// complex128 entries, each piece on a 256-byte boundary): the two QRs
// (W, Vh, Q, R), the core C and its SVD (Vs, sigma, perm, rank), the kept
// columns Cg and Vg.
struct RecompressLayout {
    size_t W1, Vh1, Q1, R1, W2, Vh2, Q2, R2, C, Vs, sig, perm, rank, Cg, Vg, total;
};
__host__ __device__ inline RecompressLayout recompress_layout(int m, int q, int k, int rmax) {
    const int kk1 = m < k ? m : k, kk2 = q < k ? q : k;
    const int r0 = kk1 < kk2 ? kk1 : kk2, r = r0 < rmax ? r0 : rmax;
    RecompressLayout L;
    size_t o = 0;
    auto take = [&o](size_t n) {
        const size_t at = o;
        o += (n + 15) & ~(size_t)15;
        return at;
    };
    L.W1 = take((size_t)m * k);
    L.Vh1 = take((size_t)m * kk1);
    L.Q1 = take((size_t)m * kk1);
    L.R1 = take((size_t)kk1 * k);
    L.W2 = take((size_t)q * k);
    L.Vh2 = take((size_t)q * kk2);
    L.Q2 = take((size_t)q * kk2);
    L.R2 = take((size_t)kk2 * k);
    L.C = take((size_t)kk1 * kk2);
    L.Vs = take((size_t)kk2 * kk2);
    L.sig = take(((size_t)kk2 + 1) / 2);
    L.perm = take(((size_t)kk2 + 3) / 4);
    L.rank = take(1);
    L.Cg = take((size_t)kk1 * r);
    L.Vg = take((size_t)kk2 * r);
    L.total = o;
    return L;
}
// One block operation of a batch (kind):
//   JOB_RECOMPRESS  the truncated product of [au, alpha U] (m x k1 + k2) and
//                   [av, V] (q x k1 + k2) as ou (m x r) and ov (q x r), r =
//                   min(m, q, k1 + k2, rmax), the columns past the kept rank
//                   (singular values above tol * sigma_1, at most rmax) zero;
//                   work holds recompress_layout(m, q, k1 + k2, rmax).total
//                   entries; au, av have leading dimensions m and q;
//   JOB_SUM         ou = au + alpha av (m x q, leading dimension m);
//   JOB_LOWRANK     ou += alpha U V^t (ou m x q with leading dimension m; U
//                   m x k2, V q x k2 with ldu, ldv);
//   JOB_SCALE       ou(i, j) = U[i] au(i, j) (V ? V[j] : 1) (m x q, leading
//                   dimension m);
//   JOB_COPY        ou[e] = au[e], e < m q.
enum { JOB_RECOMPRESS = 0, JOB_SUM = 1, JOB_LOWRANK = 2, JOB_SCALE = 3, JOB_COPY = 4 };
struct BlockJob {
    const c128 *au, *av, *U, *V;
    c128 *work, *ou, *ov;
    c128 alpha;
    int kind, m, q, k1, k2, ldu, ldv;
};
// count independent block operations (host array), one workgroup each, in
// launches of up to 32; no job may read what another writes.
void launch_block_jobs(const BlockJob* jobs, int count, int rmax, double tol, hipStream_t s);

// The tail of a randomized SVD: the SVD of the projected block M (q x ell,
// overwritten with M V; right singular vectors in V, norms in sig, order in
// perm, kept count in *rank as launch_small_svd), then Vg = conj(V_r) (ell x
// r), Vo = (M V)_r (q x r) and Uo = Q Vg (m x r), r = min(ell, rmax), the
// columns past the kept rank zero.  Q is m x ell; work holds
// rsvd_tail_work(q, ell) entries.
struct RsvdTail {
    const c128* Q;
    c128 *M, *V, *Vg, *Uo, *Vo, *work;
    double* sig;
    int *perm, *rank;
    int m, q, ell;
};
// Device work of a tail (A V and the Gram matrix) and its whole working set,
// which is staged in shared memory when small enough.
inline size_t rsvd_tail_work(int q, int ell) { return (size_t)q * ell + (size_t)ell * ell; }
__host__ __device__ inline size_t rsvd_tail_entries(int q, int ell) {
    return 2 * ((size_t)q * ell + (size_t)ell * ell);
}
// count independent tails (host array), one workgroup each, in launches of up to 32.
void launch_rsvd_tails(const RsvdTail* jobs, int count, int rmax, double tol, hipStream_t s);

// One leaf block of an H-matrix product Y += alpha op(B) X: dense (kind 0,
// a = the m x q block) or factorized (kind 1, a = U (m x r), b = V (q x r),
// the block U V^t); op is the block (trans 0: X rows xo.., Y rows yo..) or
// its transpose (trans 1: q output rows).  Leading dimensions m and q.
// Kind 2 clears output rows yo.. (m = q = their count).
struct MatvecOp {
    const c128* a;
    const c128* b;
    int kind, m, q, r, yo, xo;
};
// The largest r * ncol of the factorized ops whose temporary fits in shared
// memory (4096 complex128 entries); past it each op takes max_r * ncol
// entries of device scratch.
inline size_t hmatvec_scratch(const MatvecOp* ops, int count, int ncol) {
    size_t mr = 0;
    for (int j = 0; j < count; ++j)
        if (ops[j].kind == 1 && (size_t)ops[j].r > mr) mr = ops[j].r;
    return mr * ncol <= 4096 ? 0 : mr * ncol * (size_t)count;
}
// Y += alpha op(block) X (Y = alpha op(block) X when assign) for count ops
// whose output rows are disjoint, one workgroup each (launches of up to 64);
// tscratch holds hmatvec_scratch(ops, count, ncol) entries (may be null
// when that is 0).
void launch_hmatvec(const MatvecOp* ops, int count, int trans, int assign, const c128* X, int ldx, c128* Y, int ldy,
                    int ncol, c128 alpha, c128* tscratch, hipStream_t s);

// ---- strongly admissible layer factors (complex128, strong.hip) ----
// Factors of the n layers in the strong format from the frame coefficients
// of layer_coeffs (dg, eo: n x n; cp: (n-1) x n, all with row stride n):
// leaf size `leaf`, rank cap rmax, relative truncation tol, randomized SVD
// test vectors drawn from `seed`.  On success *out owns the factors; on
// failure an HSWEEP_* code is returned and *msg says why.
struct StrongFactors;
int strong_factor(StrongFactors** out, int n, int leaf, int rmax, double tol, uint64_t seed, const c128* dg,
                  const c128* eo, const c128* cp, hipStream_t s, std::string* msg);
// The sweep with these factors for nrhs fields f -> u (natural grid order,
// frame of sweep direction dir); fields with active[r] == 0 get u = 0.
int strong_apply(StrongFactors* sf, int dir, const c128* f, c128* u, int nrhs, const int* active, hipStream_t s,
                 std::string* msg);
void strong_free(StrongFactors* sf);
size_t strong_bytes(const StrongFactors* sf);     // stored factor bytes
int strong_levels(const StrongFactors* sf);
int strong_max_rank(const StrongFactors* sf);
size_t strong_layer_depth(int n, int leaf);
// 3D (Sec. 4): factors of the n faces of an n x n x n grid in the strong
// format with quadtree face clusters, from the 7-point coefficient fields
// (n^3 each, x1 fastest, then x2, then x3), and their face-by-face sweep.
int strong_factor3(StrongFactors** out, int n, int leaf, int rmax, double tol, uint64_t seed, const c128* D,
                   const c128* X0, const c128* X1, const c128* Y0, const c128* Y1, const c128* Z0, hipStream_t s,
                   std::string* msg);
int strong_apply3(StrongFactors* sf, const c128* f, c128* u, int nrhs, const int* active, hipStream_t s,
                  std::string* msg);
size_t strong_face_depth(int n, int leaf);

// ---- 3D coefficients (k_coeff3.hip) ----
// The 7-point operator of Sec. 4 divided by s1 s2 s3: centre D and the
// couplings to (i-1), (i+1), (j-1), (j+1), (k-1), (k+1), each edge
// coefficient evaluated once for both rows it couples.  isn/sh: the
// stretching tables of the three axes (as in 2D).
struct Coef3 {
    c128 *D, *X0, *X1, *Y0, *Y1, *Z0, *Z1;
};
void launch_coeff3(int n, double omega, const double* c, const c128* const isn[3], const c128* const sh[3],
                   const Coef3& out, hipStream_t s);
// y = A x, or y = f - A x when f is given, for nrhs fields of n^3 points.
void launch_stencil3(int n, int nrhs, const Coef3& cf, const c128* x, const c128* f, c128* y, const int* active,
                     hipStream_t s);

// Error reporting shared by the entry points of the 2D and 3D contexts
// (sets the message hsweep_last_error returns and passes the code through).
int hsweep_report(int code, const std::string& msg);
void hsweep_clear_error();
