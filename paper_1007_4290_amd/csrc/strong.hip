// Strongly admissible H-matrix factors of the layer Schur complements and
// their sweep, in complex128 (Sec. 2.3, strongly admissible case; Alg. 2.3
// and Alg. 2.4 in that format).
//
// Format.  The n positions of a layer are bisected (lo, mid = lo + (hi-lo)/2,
// hi) to the depth L at which every cluster holds at most `leaf` positions,
// so every leaf is on level L.  Two clusters of one level are well
// separated when their distance (the smallest index difference) is at least
// their width (the larger size); for clusters of one level that means at
// least one cluster lies between them.  A block (t, s) of two clusters of
// one level is factorized, U V^t, when they are well separated (then their
// parents were not); dense when they are not and both are leaves; and split
// into its 2 x 2 children otherwise.  Every block row thus carries up to
// three factorized blocks per level and three dense leaves.
//
// Arithmetic, all in device kernels; the host walks the block tree and
// launches them:
//   S_m = A_mm - diag(a) T_{m-1} diag(a), a = diagonal of A_{m,m-1};
//   T_m = S_m^{-1} by 2 x 2 block inversion through the Schur complement of
//         the first diagonal block, recursively, with dense leaves inverted
//         by Gauss-Jordan elimination with partial pivoting;
//   every sum landing on a factorized block is recompressed: QR of both
//         stacked factors, SVD of the small core, singular values above
//         tol * sigma_1 kept (all nonzero ones for tol = 0), at most rmax;
//   a product of two non-factorized blocks landing on a factorized block
//         (F = H . H) is built by the randomized range finder of Halko,
//         Martinsson and Tropp (2011): rmax + 8 complex Gaussian test
//         vectors, QR of the sampled range, SVD of the projected block.
// The QR, SVD and inverse kernels (k_dense.hip) take one small matrix per
// wavefront, and so does the fused recompression (both QRs, the core SVD and
// the kept columns in one kernel); the recompressions of one tree walk share
// a launch, and a product of an H-matrix with a block of vectors goes out as
// one launch per class of leaf blocks with disjoint output rows (hprod).
// Blocks are at most a few hundred entries on a side and the factorization
// is bound by the dependent chain of the block recursion, not by arithmetic.
// No rank is read back: a factor's width is its kept rank's upper bound, so
// the launch sequence of a layer does not depend on the data.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <utility>
#include <vector>

#include "hsweep.h"
#include "internal.hpp"

namespace {

// ---------------------------------------------------------------- kernels

// op(M)(r, c) of a column-major matrix with leading dimension ld:
// 0 = M, 1 = M^t, 2 = conj(M), 3 = M^H.
__device__ __forceinline__ c128 op_el(const c128* M, int op, int r, int c, int ld) {
    c128 v = (op & 1) ? M[(size_t)r * ld + c] : M[(size_t)c * ld + r];
    return (op & 2) ? conj(v) : v;
}

// C = alpha op(A) op(B) + beta C; C is m x n, the inner dimension k.
__global__ void zgemm_kernel(int opa, int opb, int m, int n, int k, c128 alpha, const c128* A, int lda,
                             const c128* B, int ldb, c128 beta, c128* C, int ldc) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= m || j >= n) return;
    c128 a0 = czero<double>(), a1 = a0;
    int p = 0;
    for (; p + 1 < k; p += 2) {
        cfma(a0, op_el(A, opa, i, p, lda), op_el(B, opb, p, j, ldb));
        cfma(a1, op_el(A, opa, i, p + 1, lda), op_el(B, opb, p + 1, j, ldb));
    }
    if (p < k) cfma(a0, op_el(A, opa, i, p, lda), op_el(B, opb, p, j, ldb));
    c128 out = alpha * (a0 + a1);
    if (beta.re != 0.0 || beta.im != 0.0) out += beta * C[(size_t)j * ldc + i];
    C[(size_t)j * ldc + i] = out;
}

// C = alpha op(A) + beta B (op 0 or 2), elementwise; C may be A or B.
__global__ void zgeam_kernel(int m, int n, c128 alpha, int opa, const c128* A, int lda, c128 beta, const c128* B,
                             int ldb, c128* C, int ldc) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= m || j >= n) return;
    c128 out = alpha * op_el(A, opa, i, j, lda);
    if (B) out += beta * B[(size_t)j * ldb + i];
    C[(size_t)j * ldc + i] = out;
}

// C = 0 (m x n).
__global__ void zfill_kernel(int m, int n, c128* C, int ldc) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= m || j >= n) return;
    C[(size_t)j * ldc + i] = czero<double>();
}

// M(i, j) *= dl[i] (if dl) * dr[j] (if dr).
__global__ void zscale_kernel(int m, int n, c128* M, int ld, const c128* dl, const c128* dr) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= m || j >= n) return;
    c128 v = M[(size_t)j * ld + i];
    if (dl) v = v * dl[i];
    if (dr) v = v * dr[j];
    M[(size_t)j * ld + i] = v;
}

// The dense block (rows t0.., columns s0..) of the symmetric tridiagonal
// layer operator with diagonal dg and off-diagonal eo (eo[i] = A(i, i+1)).
__global__ void tridiag_block_kernel(int m, int q, int t0, int s0, const c128* dg, const c128* eo, c128* D) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= m || j >= q) return;
    const int r = t0 + i, c = s0 + j;
    c128 v = czero<double>();
    if (r == c) v = dg[r];
    else if (r == c + 1) v = eo[c];
    else if (c == r + 1) v = eo[r];
    D[(size_t)j * m + i] = v;
}


// Complex Gaussian entries (re + i im) / sqrt(2), re and im standard normal
// by the Box-Muller transform of two uniforms from the splitmix64 hash
// (Steele, Lea and Flood 2014) of the entry's counter.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}
__global__ void zrandn_kernel(size_t count, uint64_t seed, c128* out) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const uint64_t h1 = splitmix64(seed ^ splitmix64(2 * (uint64_t)i));
    const uint64_t h2 = splitmix64(seed ^ splitmix64(2 * (uint64_t)i + 1));
    const double u1 = ((double)(h1 >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    const double u2 = ((double)(h2 >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    const double r = sqrt(-2.0 * log(u1)) * 0.70710678118654752;
    const double th = 6.283185307179586477 * u2;
    out[i] = mk(r * cos(th), r * sin(th));
}

// Grid index of position i of frame layer m (sweep direction dir): rows
// upward or downward, columns rightward.
__device__ __forceinline__ size_t frame_index(int n, int dir, int i, int m) {
    if (dir == 0) return (size_t)m * n + i;
    if (dir == 1) return (size_t)(n - 1 - m) * n + i;
    return (size_t)i * n + m;
}

// L(i, r) = f_r(frame point (i, m)) - (a ? a[i] * Wp(i, r) : 0) for nrhs fields.
__global__ void gather_layer_kernel(int n, int nrhs, int dir, int m, const c128* f, const c128* a, const c128* Wp,
                                    c128* L) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (i >= n || r >= nrhs) return;
    c128 v = f[(size_t)r * n * n + frame_index(n, dir, i, m)];
    if (a) v -= a[i] * Wp[(size_t)r * n + i];
    L[(size_t)r * n + i] = v;
}

// u_r(frame point (i, m)) = L(i, r), or 0 for an inactive field.
__global__ void scatter_layer_kernel(int n, int nrhs, int dir, int m, const c128* L, const int* active, c128* u) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (i >= n || r >= nrhs) return;
    u[(size_t)r * n * n + frame_index(n, dir, i, m)] =
        (active && !active[r]) ? czero<double>() : L[(size_t)r * n + i];
}

// ---------------------------------------------------------------- host side

constexpr int kOversample = 8;
constexpr int kThreads = 64;

inline dim3 grid2(int m, int n) { return dim3((m + kThreads - 1) / kThreads, n); }

// Bump allocator over device chunks; reset() keeps the chunks for reuse.
struct Arena {
    std::vector<std::pair<char*, size_t>> chunks;
    size_t ci = 0, used = 0;
    size_t chunk = (size_t)16 << 20;
    hipError_t err = hipSuccess;
    c128* alloc(size_t count) {
        const size_t bytes = ((count ? count : 1) * sizeof(c128) + 255) & ~(size_t)255;
        while (ci < chunks.size() && used + bytes > chunks[ci].second) { ++ci; used = 0; }
        if (ci == chunks.size()) {
            size_t b = bytes > chunk ? bytes : chunk;
            void* p = nullptr;
            hipError_t e = hipMalloc(&p, b);
            if (e != hipSuccess) { err = e; return nullptr; }
            chunks.emplace_back((char*)p, b);
            used = 0;
        }
        char* p = chunks[ci].first + used;
        used += bytes;
        return (c128*)p;
    }
    void reset() { ci = 0; used = 0; }
    size_t reserved() const {
        size_t s = 0;
        for (auto& c : chunks) s += c.second;
        return s;
    }
    void release() {
        for (auto& c : chunks) (void)hipFree(c.first);
        chunks.clear();
        reset();
    }
};

// One block of an H-matrix.  Index ranges are absolute positions of the
// layer; d is m x q, u is m x rank, v is q x rank (column-major, leading
// dimension = row count).
struct Node {
    int t0, t1, s0, s1, level;
    char kind;          // 'D' dense, 'F' factorized, 'H' split
    int ch[4];          // children (row-major 2 x 2) of an 'H' block
    c128* d;
    c128* u;
    c128* v;
    int rank;
    int m() const { return t1 - t0; }
    int q() const { return s1 - s0; }
};

// An H-matrix (or a block of one): nodes[0] is its root.
struct HMat {
    std::vector<Node> nd;
};

int depth_for(int n, int leaf) {
    int L = 0;
    while ((n + (1 << L) - 1) / (1 << L) > leaf) ++L;
    return L;
}

bool well_separated(int t0, int t1, int s0, int s1) {
    int dist = 0;
    if (t1 <= s0) dist = s0 - (t1 - 1);
    else if (s1 <= t0) dist = t0 - (s1 - 1);
    const int w = std::max(t1 - t0, s1 - s0);
    return dist >= w;
}

// A cluster: the position range [lo, hi) of a layer.  On a face (Sec. 4)
// it is also a box [i0, i1) x [j0, j1) of face points at binary level `lev`
// with quadtree coordinates (qi, qj): boxes are bisected in x1 on even
// levels and in x2 on odd ones, and positions follow that bisection.
struct Cluster {
    int lo, hi, i0, i1, j0, j1, lev, qi, qj;
};

// Cluster geometry: the bisected line of a 2D layer, or the quadtree of a
// face, where two boxes of one quadtree level (an even binary level) are
// well separated when max(|qi - qi'|, |qj - qj'|) > 1; the half levels in
// between are always refined.
struct Geometry {
    bool face = false;
    int L = 0;
    bool admissible(const Cluster& t, const Cluster& s) const {
        if (!face) return well_separated(t.lo, t.hi, s.lo, s.hi);
        if (t.lev % 2) return false;
        return std::max(std::abs(t.qi - s.qi), std::abs(t.qj - s.qj)) > 1;
    }
    void split(const Cluster& c, Cluster& a, Cluster& b) const {
        a = c;
        b = c;
        a.lev = b.lev = c.lev + 1;
        if (!face) {
            const int mid = c.lo + (c.hi - c.lo) / 2;
            a.hi = mid;
            b.lo = mid;
            return;
        }
        if (c.lev % 2 == 0) {
            const int mid = c.i0 + (c.i1 - c.i0) / 2;
            a.i1 = mid; b.i0 = mid;
            a.qi = 2 * c.qi; b.qi = 2 * c.qi + 1;
        } else {
            const int mid = c.j0 + (c.j1 - c.j0) / 2;
            a.j1 = mid; b.j0 = mid;
            a.qj = 2 * c.qj; b.qj = 2 * c.qj + 1;
        }
        a.hi = c.lo + (a.i1 - a.i0) * (a.j1 - a.j0);
        b.lo = a.hi;
    }
};

int build_structure(HMat& M, const Geometry& geo, const Cluster& t, const Cluster& s, int level) {
    const int idx = (int)M.nd.size();
    Node b{};
    b.t0 = t.lo; b.t1 = t.hi; b.s0 = s.lo; b.s1 = s.hi; b.level = level;
    b.d = b.u = b.v = nullptr;
    b.rank = 0;
    b.ch[0] = b.ch[1] = b.ch[2] = b.ch[3] = -1;
    if (geo.admissible(t, s)) b.kind = 'F';
    else if (level == geo.L) b.kind = 'D';
    else b.kind = 'H';
    M.nd.push_back(b);
    if (b.kind == 'H') {
        Cluster tc[2], sc[2];
        geo.split(t, tc[0], tc[1]);
        geo.split(s, sc[0], sc[1]);
        for (int a = 0; a < 2; ++a)
            for (int c = 0; c < 2; ++c) {
                const int k = build_structure(M, geo, tc[a], sc[c], level + 1);
                M.nd[idx].ch[2 * a + c] = k;
            }
    }
    return idx;
}

// Face points in bisection order: perm[position] = natural face index j n + i.
void face_order(const Geometry& geo, const Cluster& c, int n, std::vector<int>& out) {
    if (c.lev == geo.L) {
        for (int j = c.j0; j < c.j1; ++j)
            for (int i = c.i0; i < c.i1; ++i) out.push_back(j * n + i);
        return;
    }
    Cluster a, b;
    geo.split(c, a, b);
    face_order(geo, a, n, out);
    face_order(geo, b, n, out);
}

}  // namespace

struct StrongFactors {
    int nl = 0;                   // layers (faces)
    int N = 0;                    // positions per layer (n on a line, n^2 on a face)
    int side = 0;                 // grid points per side
    int leaf = 0, L = 0, rmax = 0;
    double tol = 0.0;
    uint64_t seed = 0, draws = 0;
    Geometry geo;
    int* permd = nullptr;         // face: perm[position] = natural face index (device)
    HMat shape;                   // the block structure of a layer
    std::vector<HMat> T;          // T_m of every layer (device data in `keep`)
    Arena keep, tmp;
    int* dint = nullptr;          // device ints: [0] rank of the last SVD, [1] zero-pivot status
    c128* cpk = nullptr;          // couplings a_m = diagonal of A_{m+1,m}, (n-1) x n (in `keep`)
    hipStream_t s = nullptr;
    std::string err;
    int rc = HSWEEP_OK;
    // sweep work: W (n layers x n x nrhs), two layer vectors, product scratch
    c128* sw = nullptr;
    size_t sw_count = 0;
    int max_rank_seen = 0;
    std::vector<BlockJob> pend;   // recompressions not yet launched
    int defer = 0;                     // depth of walks whose recompressions wait in pend

    // ---- launch helpers
    bool ok() const { return rc == HSWEEP_OK; }
    void fail_with(int code, const std::string& m) {
        if (rc == HSWEEP_OK) { rc = code; err = m; }
    }
    c128* talloc(size_t count) {
        c128* p = tmp.alloc(count);
        if (!p) fail_with(HSWEEP_ENOMEM, "device memory for the strongly admissible factorization");
        return p;
    }
    void gemm(int opa, int opb, int m, int n, int k, c128 alpha, const c128* A, int lda, const c128* B, int ldb,
              c128 beta, c128* C, int ldc) {
        if (!ok() || m <= 0 || n <= 0) return;
        hipLaunchKernelGGL(zgemm_kernel, grid2(m, n), dim3(kThreads), 0, s, opa, opb, m, n, k, alpha, A, lda, B, ldb,
                           beta, C, ldc);
    }
    void geam(int m, int n, c128 alpha, int opa, const c128* A, int lda, c128 beta, const c128* B, int ldb, c128* C,
              int ldc) {
        if (!ok() || m <= 0 || n <= 0) return;
        hipLaunchKernelGGL(zgeam_kernel, grid2(m, n), dim3(kThreads), 0, s, m, n, alpha, opa, A, lda, beta, B, ldb,
                           C, ldc);
    }
    void zero(c128* C, int m, int n, int ldc) {
        if (!ok() || m <= 0 || n <= 0) return;
        hipLaunchKernelGGL(zfill_kernel, grid2(m, n), dim3(kThreads), 0, s, m, n, C, ldc);
    }

    // ---- structure
    // A zero H-matrix with the block structure of M's subtree idx: its dense
    // blocks share one allocation, cleared by one launch.
    HMat zeros_like(const HMat& M, int idx) {
        HMat R;
        copy_shape(R, M, idx, true);
        size_t tot = 0;
        for (const Node& b : R.nd)
            if (b.kind == 'D') tot += ((size_t)b.m() * b.q() + 15) & ~(size_t)15;
        if (tot == 0 || !ok()) return R;
        c128* base = talloc(tot);
        if (!base) return R;
        zero(base, (int)tot, 1, (int)tot);
        size_t at = 0;
        for (Node& b : R.nd)
            if (b.kind == 'D') {
                b.d = base + at;
                at += ((size_t)b.m() * b.q() + 15) & ~(size_t)15;
            }
        return R;
    }
    int copy_shape(HMat& R, const HMat& M, int idx, bool fresh) {
        const int k = (int)R.nd.size();
        Node b = M.nd[idx];
        if (fresh) {            // data pointers set by the caller
            b.u = b.v = nullptr;
            b.rank = 0;
            b.d = nullptr;
        }
        R.nd.push_back(b);
        if (b.kind == 'H')
            for (int c = 0; c < 4; ++c) {
                const int kc = copy_shape(R, M, M.nd[idx].ch[c], fresh);
                R.nd[k].ch[c] = kc;
            }
        return k;
    }
    // The block with root `top` (an 'H' node of `like`) assembled from four
    // finished H-matrices (shallow: their device data is shared).
    HMat assemble(const Node& top, const HMat* parts[4]) {
        HMat R;
        R.nd.push_back(top);
        for (int c = 0; c < 4; ++c) {
            const int k = copy_shape(R, *parts[c], 0, false);
            R.nd[0].ch[c] = k;
        }
        return R;
    }

    // ---- products with blocks of vectors (accumulating)
    // The leaves of B's subtree bi as product ops, offsets relative to the
    // subtree's corner (output rows along t for op = B, along s for B^t).
    void collect(const HMat& B, int bi, int trans, int rt, int rs, std::vector<MatvecOp>& ops) {
        const Node& b = B.nd[bi];
        if (b.kind == 'H') {
            for (int c = 0; c < 4; ++c) collect(B, b.ch[c], trans, rt, rs, ops);
            return;
        }
        if (b.kind == 'F' && b.rank == 0) return;
        MatvecOp o;
        o.kind = b.kind == 'D' ? 0 : 1;
        o.a = b.kind == 'D' ? b.d : b.u;
        o.b = b.kind == 'D' ? nullptr : b.v;
        o.m = b.m();
        o.q = b.q();
        o.r = b.kind == 'D' ? 0 : b.rank;
        const int to = b.t0 - rt, so = b.s0 - rs;
        o.yo = trans ? so : to;
        o.xo = trans ? to : so;
        ops.push_back(o);
    }
    // Y += alpha op(B) X over the subtree bi (op = B or B^t), or Y = alpha
    // op(B) X when assign: its leaves in classes of disjoint output rows
    // (intervals coloured greedily in order of their first row, which uses
    // the fewest classes), one launch per class, so each row sums its leaves
    // in a fixed order.  With assign the first class writes instead of adding
    // and clears the rows none of its leaves cover.
    void hprod(const HMat& B, int bi, int trans, const c128* X, int ldx, int ncol, c128* Y, int ldy, c128 alpha,
               bool assign = false) {
        if (!ok() || ncol <= 0) return;
        const Node& b = B.nd[bi];
        std::vector<MatvecOp> ops;
        collect(B, bi, trans, b.t0, b.s0, ops);
        std::vector<int> idx(ops.size());
        for (size_t i = 0; i < idx.size(); ++i) idx[i] = (int)i;
        std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return ops[x].yo < ops[y].yo; });
        std::vector<int> last_end;
        std::vector<std::vector<MatvecOp>> cls;
        for (int i : idx) {
            const int y0 = ops[i].yo, y1 = y0 + (trans ? ops[i].q : ops[i].m);
            size_t c = 0;
            while (c < last_end.size() && last_end[c] > y0) ++c;
            if (c == last_end.size()) {
                last_end.push_back(y1);
                cls.emplace_back();
            } else {
                last_end[c] = y1;
            }
            cls[c].push_back(ops[i]);
        }
        const int rows = trans ? b.q() : b.m();
        if (assign) {
            if (cls.empty()) cls.emplace_back();
            // the rows class 0 leaves uncovered (its intervals are sorted and disjoint)
            std::vector<MatvecOp> gaps;
            int at = 0;
            for (const MatvecOp& o : cls[0]) {
                if (o.yo > at) gaps.push_back(clear_op(at, o.yo - at));
                at = o.yo + (trans ? o.q : o.m);
            }
            if (at < rows) gaps.push_back(clear_op(at, rows - at));
            cls[0].insert(cls[0].end(), gaps.begin(), gaps.end());
        }
        for (size_t c = 0; c < cls.size(); ++c) {
            auto& cl = cls[c];
            const size_t need = hmatvec_scratch(cl.data(), (int)cl.size(), ncol);
            c128* T = need ? talloc(need) : nullptr;
            if (!ok()) return;
            launch_hmatvec(cl.data(), (int)cl.size(), trans, assign && c == 0, X, ldx, Y, ldy, ncol, alpha, T, s);
        }
    }
    static MatvecOp clear_op(int y0, int count) {
        MatvecOp o;
        o.a = o.b = nullptr;
        o.kind = 2;
        o.m = o.q = count;
        o.r = 0;
        o.yo = y0;
        o.xo = 0;
        return o;
    }
    // Y (B.m x ncol) = alpha B X and Y (B.q x ncol) = alpha B^t X
    void matvec_set(const HMat& B, int bi, const c128* X, int ldx, int ncol, c128* Y, int ldy, c128 alpha) {
        hprod(B, bi, 0, X, ldx, ncol, Y, ldy, alpha, true);
    }
    void matvec_t_set(const HMat& B, int bi, const c128* X, int ldx, int ncol, c128* Y, int ldy, c128 alpha) {
        hprod(B, bi, 1, X, ldx, ncol, Y, ldy, alpha, true);
    }
    // Y (B.m x ncol) += alpha B X
    void matvec(const HMat& B, int bi, const c128* X, int ldx, int ncol, c128* Y, int ldy, c128 alpha) {
        hprod(B, bi, 0, X, ldx, ncol, Y, ldy, alpha);
    }
    // Y (B.q x ncol) += alpha B^t X
    void matvec_t(const HMat& B, int bi, const c128* X, int ldx, int ncol, c128* Y, int ldy, c128 alpha) {
        hprod(B, bi, 1, X, ldx, ncol, Y, ldy, alpha);
    }

    // ---- small factorizations
    // Thin QR of A (p x k): Q (p x kk), R (kk x k), kk = min(p, k).
    void qr(int p, int k, const c128* A, int lda, c128*& Q, c128*& R, c128* Qc = nullptr) {
        const int kk = std::min(p, k);
        c128* W = talloc((size_t)p * k);
        c128* Vh = talloc((size_t)p * kk);
        Q = talloc((size_t)p * kk);
        R = talloc((size_t)kk * k);
        if (!ok()) return;
        launch_small_qr(p, k, A, lda, W, Vh, Q, R, Qc, s);
    }

    // out = trunc([a.u, alpha U] [a.v, V]^t): QR of both stacked factors,
    // SVD of the small core, the kept columns (one fused kernel); the width
    // is the kept rank's upper bound, the columns past the rank zero.  Inside
    // a walk over disjoint blocks (defer > 0) the job waits in `pend` and the
    // walk launches all of its jobs at once when it ends: the walk's other
    // launches neither read what the jobs write nor write what they read.
    void compress_sum(Node& out, const Node& a, c128 alpha, const c128* U, int ldu, const c128* V, int ldv, int k2) {
        const int m = out.m(), q = out.q(), k1 = a.rank, k = k1 + k2;
        out.u = out.v = nullptr;
        out.rank = 0;
        if (k == 0 || !ok()) return;
        const int r = std::min(std::min(std::min(m, k), std::min(q, k)), rmax);
        if (r == 0) return;
        c128* work = talloc(recompress_layout(m, q, k, rmax).total);
        out.u = talloc((size_t)m * r);
        out.v = talloc((size_t)q * r);
        if (!ok()) return;
        BlockJob J;
        J.kind = JOB_RECOMPRESS;
        J.au = a.u;
        J.av = a.v;
        J.U = U;
        J.V = V;
        J.work = work;
        J.ou = out.u;
        J.ov = out.v;
        J.alpha = alpha;
        J.m = m;
        J.q = q;
        J.k1 = k1;
        J.k2 = k2;
        J.ldu = ldu;
        J.ldv = ldv;
        job(J);
        out.rank = r;
        if (r > max_rank_seen) max_rank_seen = r;
    }
    // Queue a block operation; outside a walk it goes out at once.
    void job(const BlockJob& J) {
        pend.push_back(J);
        if (defer == 0) flush();
    }
    static BlockJob dense_job(int kind, int m, int q, const c128* src, c128* dst) {
        BlockJob J;
        J.kind = kind;
        J.au = src;
        J.av = J.U = J.V = nullptr;
        J.work = J.ov = nullptr;
        J.ou = dst;
        J.alpha = mk(1.0, 0.0);
        J.m = m;
        J.q = q;
        J.k1 = J.k2 = 0;
        J.ldu = J.ldv = m;
        return J;
    }
    // Launch the queued block operations (one workgroup each).
    void flush() {
        if (!pend.empty() && ok()) launch_block_jobs(pend.data(), (int)pend.size(), rmax, tol, s);
        pend.clear();
    }

    // Randomized SVD of the m x q product G H (G on (t, u), H on (u, s)):
    // Y = G (H Omega), Q = qr(Y), M = H^t (G^t conj(Q)) = (Q^H G H)^t, M V =
    // U S from the SVD of M, and G H ~ (Q conj(V_r)) ((M V)_r)^t.
    // The head of the randomized SVD of G H, up to the projected block M
    // (launched at once); the tail goes into `out` (its SVD, the kept
    // columns, Uo = Q Vg, launched with other tails by finish_rsvds).
    // Returns the factors' width r (0: nothing to add).
    int rsvd_begin(const HMat& G, int gi, const HMat& H, int hi, RsvdTail& out) {
        const Node& g = G.nd[gi];
        const Node& h = H.nd[hi];
        const int m = g.m(), q = h.q(), mid = g.q();
        const int ell = std::min(std::min(rmax + kOversample, m), q);
        if (ell <= 0 || !ok()) return 0;
        c128* Om = talloc((size_t)q * ell);
        c128* Y1 = talloc((size_t)mid * ell);
        c128* Y = talloc((size_t)m * ell);
        if (!ok()) return 0;
        const size_t cnt = (size_t)q * ell;
        hipLaunchKernelGGL(zrandn_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, cnt, seed + draws, Om);
        draws += 0x9E3779B97F4A7C15ull;
        matvec_set(H, hi, Om, q, ell, Y1, mid, mk(1.0, 0.0));
        matvec_set(G, gi, Y1, mid, ell, Y, m, mk(1.0, 0.0));
        c128 *Q, *R;
        c128* Qc = talloc((size_t)m * ell);
        qr(m, ell, Y, m, Q, R, Qc);                   // ell <= m: Q and conj(Q) are m x ell
        c128* M1 = talloc((size_t)mid * ell);
        c128* M = talloc((size_t)q * ell);
        if (!ok()) return 0;
        matvec_t_set(G, gi, Qc, m, ell, M1, mid, mk(1.0, 0.0));
        matvec_t_set(H, hi, M1, mid, ell, M, q, mk(1.0, 0.0));
        const int r = std::min(ell, rmax);               // width: the kept rank's bound
        if (r == 0) return 0;
        out.Q = Q;
        out.M = M;
        out.V = talloc((size_t)ell * ell);
        out.work = talloc(rsvd_tail_work(q, ell));
        out.sig = (double*)talloc(((size_t)ell + 1) / 2 + 1);
        out.perm = (int*)talloc(((size_t)ell + 3) / 4 + 1);
        out.rank = (int*)talloc(1);
        out.Vg = talloc((size_t)ell * r);
        out.Uo = talloc((size_t)m * r);
        out.Vo = talloc((size_t)q * r);
        out.m = m;
        out.q = q;
        out.ell = ell;
        return ok() ? r : 0;
    }
    // A randomized SVD waiting for its tail and its low-rank update of T's block ti.
    struct RsvdPending {
        RsvdTail tail;
        HMat* T;
        int ti, r;
        c128 alpha;
    };
    std::vector<RsvdPending> rpend;
    int phase = 0;                     // depth of product phases whose tails wait in rpend
    // The tails queued since `from` in one batch, then their updates.
    void finish_rsvds(size_t from) {
        if (rpend.size() > from && ok()) {
            std::vector<RsvdTail> tails;
            for (size_t i = from; i < rpend.size(); ++i) tails.push_back(rpend[i].tail);
            launch_rsvd_tails(tails.data(), (int)tails.size(), rmax, tol, s);
            for (size_t i = from; i < rpend.size() && ok(); ++i) {
                const RsvdPending& e = rpend[i];
                add_lowrank(*e.T, e.ti, e.tail.Uo, e.tail.m, e.tail.Vo, e.tail.q, e.r, e.alpha);
            }
        }
        rpend.resize(from);
    }

    // ---- H-arithmetic
    // T += U V^t along T's tree (U: T.m x k, V: T.q x k); the recompressions
    // of its factorized blocks go out as one batch
    void add_lowrank(HMat& T, int ti, const c128* U, int ldu, const c128* V, int ldv, int k, c128 alpha) {
        ++defer;
        add_lowrank_walk(T, ti, U, ldu, V, ldv, k, alpha);
        if (--defer == 0) flush();
    }
    void add_lowrank_walk(HMat& T, int ti, const c128* U, int ldu, const c128* V, int ldv, int k, c128 alpha) {
        if (k == 0 || !ok()) return;
        Node& b = T.nd[ti];
        if (b.kind == 'D') {                          // b.d += alpha U V^t
            BlockJob J = dense_job(JOB_LOWRANK, b.m(), b.q(), nullptr, b.d);
            J.U = U;
            J.V = V;
            J.ldu = ldu;
            J.ldv = ldv;
            J.k2 = k;
            J.alpha = alpha;
            job(J);
        } else if (b.kind == 'F') {
            Node old = b;
            Node out = b;
            compress_sum(out, old, alpha, U, ldu, V, ldv, k);
            T.nd[ti] = out;
        } else {
            for (int c = 0; c < 4; ++c) {
                const int ci = T.nd[ti].ch[c];
                const Node& h = T.nd[ci];
                add_lowrank_walk(T, ci, U + (h.t0 - T.nd[ti].t0), ldu, V + (h.s0 - T.nd[ti].s0), ldv, k, alpha);
            }
        }
    }
    // T += alpha G H (three blocks of one level)
    void mul_add(HMat& T, int ti, const HMat& G, int gi, const HMat& H, int hi, c128 alpha) {
        if (!ok()) return;
        const Node& g = G.nd[gi];
        const Node& h = H.nd[hi];
        const Node tb = T.nd[ti];
        if (g.kind == 'F') {                            // U_g (H^t V_g)^t
            if (g.rank == 0) return;
            c128* Vn = talloc((size_t)h.q() * g.rank);
            if (!ok()) return;
            matvec_t_set(H, hi, g.v, g.q(), g.rank, Vn, h.q(), mk(1.0, 0.0));
            add_lowrank(T, ti, g.u, g.m(), Vn, h.q(), g.rank, alpha);
        } else if (h.kind == 'F') {                     // (G U_h) V_h^t
            if (h.rank == 0) return;
            c128* Un = talloc((size_t)g.m() * h.rank);
            if (!ok()) return;
            matvec_set(G, gi, h.u, h.m(), h.rank, Un, g.m(), mk(1.0, 0.0));
            add_lowrank(T, ti, Un, g.m(), h.v, h.q(), h.rank, alpha);
        } else if (tb.kind == 'D') {
            gemm(0, 0, tb.m(), tb.q(), g.q(), alpha, g.d, g.m(), h.d, h.m(), mk(1.0, 0.0), T.nd[ti].d, tb.m());
        } else if (tb.kind == 'F') {                    // F = H . H
            RsvdPending e;
            e.r = rsvd_begin(G, gi, H, hi, e.tail);
            if (e.r == 0) return;
            e.T = &T;
            e.ti = ti;
            e.alpha = alpha;
            const size_t from = rpend.size();
            rpend.push_back(e);
            if (phase == 0) finish_rsvds(from);      // inside a phase: at the phase's end
        } else {
            // the four target blocks are independent, so the four products of
            // one b go out side by side (their block jobs share launches, and
            // so do the tails of their randomized SVDs);
            // the b = 1 products add to what b = 0 left, so a flush separates
            // them.  Launching queued jobs early is always safe.
            for (int b = 0; b < 2; ++b) {
                flush();
                const size_t from = rpend.size();
                ++defer;
                ++phase;
                for (int a = 0; a < 2; ++a)
                    for (int c = 0; c < 2; ++c)
                        mul_add(T, T.nd[ti].ch[2 * a + c], G, g.ch[2 * a + b], H, h.ch[2 * b + c], alpha);
                finish_rsvds(from);                    // the phase's randomized-SVD tails, side by side
                --phase;
                --defer;
                flush();
            }
        }
    }
    HMat mul(const HMat& G, int gi, const HMat& H, int hi, const HMat& like, int li, c128 alpha) {
        HMat T = zeros_like(like, li);
        if (ok()) mul_add(T, 0, G, gi, H, hi, alpha);
        return T;
    }
    // A + alpha B, two blocks of one structure
    int add_into(HMat& R, const HMat& A, int ai, const HMat& B, int bi, c128 alpha) {
        const int k = (int)R.nd.size();
        Node out = A.nd[ai];
        const Node& b = B.nd[bi];
        out.ch[0] = out.ch[1] = out.ch[2] = out.ch[3] = -1;
        if (out.kind == 'D') {                        // out.d = A.d + alpha b.d
            out.d = talloc((size_t)out.m() * out.q());
            if (ok()) {
                BlockJob J = dense_job(JOB_SUM, out.m(), out.q(), A.nd[ai].d, out.d);
                J.av = b.d;
                J.alpha = alpha;
                job(J);
            }
        } else if (out.kind == 'F') {
            compress_sum(out, A.nd[ai], alpha, b.u, b.m(), b.v, b.q(), b.rank);
        }
        R.nd.push_back(out);
        if (out.kind == 'H')
            for (int c = 0; c < 4; ++c) {
                const int kc = add_into(R, A, A.nd[ai].ch[c], B, b.ch[c], alpha);
                R.nd[k].ch[c] = kc;
            }
        return k;
    }
    HMat add(const HMat& A, int ai, const HMat& B, int bi, c128 alpha) {
        HMat R;
        ++defer;
        add_into(R, A, ai, B, bi, alpha);
        if (--defer == 0) flush();
        return R;
    }
    // G^{-1} by 2 x 2 block inversion: Y = G11^{-1}, Z = Y G12, X = G21 Y,
    // S = G22 - G21 Z, W = S^{-1}, T12 = -Z W, T21 = -W X, T11 = Y - Z T21.
    HMat inv(const HMat& G, int gi) {
        const Node& g = G.nd[gi];
        HMat R;
        if (!ok()) return R;
        if (g.kind == 'D') {
            Node out = g;
            const int m = g.m();
            c128* Wk = talloc((size_t)m * (m + 1));
            out.d = talloc((size_t)m * m);
            if (ok()) launch_small_inv(m, g.d, m, Wk, out.d, dint + 1, s);
            R.nd.push_back(out);
            return R;
        }
        const int g11 = g.ch[0], g12 = g.ch[1], g21 = g.ch[2], g22 = g.ch[3];
        const c128 one = mk(1.0, 0.0), mone = mk(-1.0, 0.0);
        HMat Y = inv(G, g11);
        HMat Z = mul(Y, 0, G, g12, G, g12, one);
        HMat X = mul(G, g21, Y, 0, G, g21, one);
        HMat P = mul(G, g21, Z, 0, G, g22, one);
        HMat S = add(G, g22, P, 0, mone);
        HMat W = inv(S, 0);
        HMat T12 = mul(Z, 0, W, 0, G, g12, mone);
        HMat T21 = mul(W, 0, X, 0, G, g21, mone);
        HMat Q = mul(Z, 0, T21, 0, G, g11, one);
        HMat T11 = add(Y, 0, Q, 0, mone);
        const HMat* parts[4] = {&T11, &T12, &T21, &W};
        Node top = g;
        return assemble(top, parts);
    }

    // A copy of M in the persistent arena.
    // (the block copies go out as one batch)
    HMat persist(const HMat& M) {
        HMat R = M;
        ++defer;
        for (auto& b : R.nd) {
            if (!ok()) break;
            if (b.kind == 'D') {
                c128* p = keep.alloc((size_t)b.m() * b.q());
                if (!p) { fail_with(HSWEEP_ENOMEM, "device memory for the strong factors"); break; }
                job(dense_job(JOB_COPY, b.m(), b.q(), b.d, p));
                b.d = p;
            } else if (b.kind == 'F' && b.rank > 0) {
                c128* pu = keep.alloc((size_t)b.m() * b.rank);
                c128* pv = keep.alloc((size_t)b.q() * b.rank);
                if (!pu || !pv) { fail_with(HSWEEP_ENOMEM, "device memory for the strong factors"); break; }
                job(dense_job(JOB_COPY, b.m(), b.rank, b.u, pu));
                job(dense_job(JOB_COPY, b.q(), b.rank, b.v, pv));
                b.u = pu;
                b.v = pv;
            } else if (b.kind == 'F') {
                b.u = b.v = nullptr;
            }
        }
        if (--defer == 0) flush();
        return R;
    }

    ~StrongFactors() {
        keep.release();
        tmp.release();
        if (dint) (void)hipFree(dint);
        if (sw) (void)hipFree(sw);
        if (permd) (void)hipFree(permd);
    }
};

// ---------------------------------------------------------------- interface

namespace {

// The dense block (rows t0.., columns s0.., positions in bisection order)
// of the face operator A_mm of the 7-point stencil: centre D and the
// couplings of point p = j n + i to (i-1, j), (i+1, j), (i, j-1), (i, j+1)
// (X0, X1, Y0, Y1, natural face order).
__global__ void face_block_kernel(int m, int q, int t0, int s0, int n, const int* perm, const c128* D, const c128* X0,
                                  const c128* X1, const c128* Y0, const c128* Y1, c128* out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= m || j >= q) return;
    const int p = perm[t0 + i], c = perm[s0 + j];
    const int ip = p % n, jp = p / n, ic = c % n, jc = c / n;
    c128 v = czero<double>();
    if (p == c) v = D[p];
    else if (jc == jp && ic == ip - 1) v = X0[p];
    else if (jc == jp && ic == ip + 1) v = X1[p];
    else if (ic == ip && jc == jp - 1) v = Y0[p];
    else if (ic == ip && jc == jp + 1) v = Y1[p];
    out[(size_t)j * m + i] = v;
}

// dst(r, pos) = src(r, perm[pos]) for `rows` rows of N entries.
__global__ void permute_rows_kernel(int rows, int N, const int* perm, const c128* src, c128* dst) {
    const int pos = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (pos >= N || r >= rows) return;
    dst[(size_t)r * N + pos] = src[(size_t)r * N + perm[pos]];
}

// L(pos, r) = f_r(face m, point perm[pos]) - (a ? a[pos] Wp(pos, r) : 0);
// field r holds nl faces of N points.
__global__ void gather_face_kernel(int N, int nl, int nrhs, int m, const int* perm, const c128* f, const c128* a,
                                   const c128* Wp, c128* L) {
    const int pos = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (pos >= N || r >= nrhs) return;
    c128 v = f[(size_t)r * nl * N + (size_t)m * N + perm[pos]];
    if (a) v -= a[pos] * Wp[(size_t)r * N + pos];
    L[(size_t)r * N + pos] = v;
}

__global__ void scatter_face_kernel(int N, int nl, int nrhs, int m, const int* perm, const c128* L, const int* active,
                                    c128* u) {
    const int pos = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (pos >= N || r >= nrhs) return;
    u[(size_t)r * nl * N + (size_t)m * N + perm[pos]] =
        (active && !active[r]) ? czero<double>() : L[(size_t)r * N + pos];
}

int fail_new(StrongFactors* sf, int code, const std::string& m, std::string* msg) {
    *msg = m;
    delete sf;
    return code;
}

// Alg. 2.3 in the strong format over sf->nl layers: fill(m, block) writes
// the dense blocks of A_mm, cp (device, (nl - 1) x N, position order) holds
// the diagonals of A_{m+1,m}.
template <typename Fill>
int factor_layers(StrongFactors* sf, Fill fill, const c128* cp, hipStream_t s, std::string* msg) {
    const int nl = sf->nl, N = sf->N;
    sf->s = s;
    hipError_t e = hipMalloc((void**)&sf->dint, 2 * sizeof(int));
    if (e == hipSuccess) e = hipMemsetAsync(sf->dint, 0, 2 * sizeof(int), s);
    if (e != hipSuccess)
        return fail_new(sf, e == hipErrorOutOfMemory ? HSWEEP_ENOMEM : HSWEEP_EDEVICE,
                        std::string("strong factorization: ") + hipGetErrorString(e), msg);
    if (nl > 1) {
        sf->cpk = sf->keep.alloc((size_t)(nl - 1) * N);
        if (!sf->cpk) return fail_new(sf, HSWEEP_ENOMEM, "device memory for the strong factors", msg);
        e = hipMemcpyAsync(sf->cpk, cp, (size_t)(nl - 1) * N * sizeof(c128), hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess)
            return fail_new(sf, HSWEEP_EDEVICE, std::string("strong factorization: ") + hipGetErrorString(e), msg);
    }
    const c128 mone = mk(-1.0, 0.0);
    for (int m = 0; m < nl && sf->ok(); ++m) {
        // A_mm in the format: all its entries lie in dense blocks
        HMat A = sf->zeros_like(sf->shape, 0);
        for (Node& b : A.nd)
            if (b.kind == 'D' && sf->ok()) fill(m, b);
        HMat S;
        if (m == 0) {
            S = A;
        } else {
            // diag(a) T_{m-1} diag(a), a = diagonal of A_{m,m-1}
            // (scaled copies of the blocks of T_{m-1}, one batch)
            const c128* a = sf->cpk + (size_t)(m - 1) * N;
            HMat D = sf->T[m - 1];
            ++sf->defer;
            for (Node& b : D.nd) {
                if (!sf->ok()) break;
                if (b.kind == 'D') {
                    c128* p = sf->talloc((size_t)b.m() * b.q());
                    if (!p) break;
                    BlockJob J = StrongFactors::dense_job(JOB_SCALE, b.m(), b.q(), b.d, p);
                    J.U = a + b.t0;
                    J.V = a + b.s0;
                    sf->job(J);
                    b.d = p;
                } else if (b.kind == 'F' && b.rank > 0) {
                    c128* pu = sf->talloc((size_t)b.m() * b.rank);
                    c128* pv = sf->talloc((size_t)b.q() * b.rank);
                    if (!pu || !pv) break;
                    BlockJob J = StrongFactors::dense_job(JOB_SCALE, b.m(), b.rank, b.u, pu);
                    J.U = a + b.t0;
                    sf->job(J);
                    J = StrongFactors::dense_job(JOB_SCALE, b.q(), b.rank, b.v, pv);
                    J.U = a + b.s0;
                    sf->job(J);
                    b.u = pu;
                    b.v = pv;
                }
            }
            if (--sf->defer == 0) sf->flush();
            S = sf->add(A, 0, D, 0, mone);
        }
        HMat Tm = sf->inv(S, 0);
        if (!sf->ok()) break;
        sf->T.push_back(sf->persist(Tm));
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) { sf->fail_with(HSWEEP_EDEVICE, std::string("strong factorization: ") + hipGetErrorString(e)); break; }
        if (sf->tmp.err != hipSuccess || sf->keep.err != hipSuccess) {
            sf->fail_with(HSWEEP_ENOMEM, "device memory for the strongly admissible factorization");
            break;
        }
        int st = 0;
        e = hipMemcpy(&st, sf->dint + 1, sizeof(int), hipMemcpyDeviceToHost);
        if (e != hipSuccess) { sf->fail_with(HSWEEP_EDEVICE, hipGetErrorString(e)); break; }
        if (st) { sf->fail_with(HSWEEP_ESINGULAR, "zero pivot in a dense leaf inverse (strong format)"); break; }
        sf->tmp.reset();
    }
    if (!sf->ok()) {
        const int rc = sf->rc;
        return fail_new(sf, rc, sf->err, msg);
    }
    sf->tmp.release();
    return HSWEEP_OK;
}

// Alg. 2.4 with T_m in the strong format for nrhs fields:
//   w_m = T_m (f_m - a_{m-1} w_{m-1}),  u_{nl-1} = w_{nl-1},
//   u_m = w_m - T_m (a_m u_{m+1}).
// gather(m, a, Wp, L) loads layer m of f (minus a * Wp when a is given) in
// position order, scatter(m, L) stores layer m of u.
template <typename Gather, typename Scatter>
int apply_layers(StrongFactors* sf, int nrhs, Gather gather, Scatter scatter, hipStream_t s, std::string* msg) {
    const int nl = sf->nl, N = sf->N;
    const size_t lay = (size_t)N * nrhs;
    const size_t need = lay * ((size_t)nl + 2);
    if (need > sf->sw_count) {
        if (sf->sw) (void)hipFree(sf->sw);
        sf->sw = nullptr;
        sf->sw_count = 0;
        hipError_t e = hipMalloc((void**)&sf->sw, need * sizeof(c128));
        if (e != hipSuccess) {
            *msg = std::string("strong sweep work: ") + hipGetErrorString(e);
            return e == hipErrorOutOfMemory ? HSWEEP_ENOMEM : HSWEEP_EDEVICE;
        }
        sf->sw_count = need;
    }
    c128* W = sf->sw;                          // w_m of every layer, N x nrhs each
    c128* L0 = W + lay * nl;                   // the current layer's fields
    c128* L1 = L0 + lay;                       // coupled fields a_m u_{m+1}
    sf->s = s;
    sf->rc = HSWEEP_OK;
    sf->err.clear();
    const dim3 g2 = grid2(N, nrhs);
    for (int m = 0; m < nl && sf->ok(); ++m) {
        gather(m, m > 0 ? sf->cpk + (size_t)(m - 1) * N : (const c128*)nullptr,
               m > 0 ? W + lay * (m - 1) : (const c128*)nullptr, L0);
        sf->matvec_set(sf->T[m], 0, L0, N, nrhs, W + lay * m, N, mk(1.0, 0.0));
        sf->tmp.reset();          // F-block scratch is reused in stream order
    }
    for (int m = nl - 1; m >= 0 && sf->ok(); --m) {
        if (m == nl - 1) {
            scatter(m, W + lay * m);
            sf->geam(N, nrhs, mk(1.0, 0.0), 0, W + lay * m, N, czero<double>(), nullptr, 0, L0, N);
            continue;
        }
        // L1 = a_m * u_{m+1} (u_{m+1} in L0), L0 = w_m - T_m L1
        hipLaunchKernelGGL(zscale_kernel, g2, dim3(kThreads), 0, s, N, nrhs, L0, N, sf->cpk + (size_t)m * N,
                           (const c128*)nullptr);
        sf->geam(N, nrhs, mk(1.0, 0.0), 0, L0, N, czero<double>(), nullptr, 0, L1, N);
        sf->geam(N, nrhs, mk(1.0, 0.0), 0, W + lay * m, N, czero<double>(), nullptr, 0, L0, N);
        sf->matvec(sf->T[m], 0, L1, N, nrhs, L0, N, mk(-1.0, 0.0));
        sf->tmp.reset();
        scatter(m, L0);
    }
    if (!sf->ok()) {
        *msg = sf->err;
        return sf->rc;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        *msg = std::string("strong sweep: ") + hipGetErrorString(e);
        return HSWEEP_EDEVICE;
    }
    return HSWEEP_OK;
}

int face_depth(int n, int leaf) {
    int Lq = 0;
    while (((n + (1 << Lq) - 1) >> Lq) * ((n + (1 << Lq) - 1) >> Lq) > leaf) ++Lq;
    return 2 * Lq;
}

}  // namespace

// ---------------------------------------------------------------- interface

size_t strong_layer_depth(int n, int leaf) { return (size_t)depth_for(n, leaf); }
size_t strong_face_depth(int n, int leaf) { return (size_t)face_depth(n, leaf); }

void strong_free(StrongFactors* sf) { delete sf; }

size_t strong_bytes(const StrongFactors* sf) {
    if (!sf) return 0;
    size_t e = 0;
    for (const HMat& M : sf->T)
        for (const Node& b : M.nd) {
            if (b.kind == 'D') e += (size_t)b.m() * b.q();
            else if (b.kind == 'F') e += (size_t)(b.m() + b.q()) * b.rank;
        }
    return e * sizeof(c128);
}

int strong_levels(const StrongFactors* sf) { return sf ? sf->L : 0; }
int strong_max_rank(const StrongFactors* sf) { return sf ? sf->max_rank_seen : 0; }

// 2D: the n layers of an n x n grid (frame coefficients dg, eo: n x n; cp:
// (n-1) x n, see layer_coeffs).
int strong_factor(StrongFactors** out, int n, int leaf, int rmax, double tol, uint64_t seed, const c128* dg,
                  const c128* eo, const c128* cp, hipStream_t s, std::string* msg) {
    *out = nullptr;
    StrongFactors* sf = new StrongFactors();
    sf->nl = n; sf->N = n; sf->side = n;
    sf->leaf = leaf; sf->rmax = rmax; sf->tol = tol; sf->seed = seed;
    sf->geo.face = false;
    sf->geo.L = sf->L = depth_for(n, leaf);
    const Cluster root{0, n, 0, n, 0, 1, 0, 0, 0};
    build_structure(sf->shape, sf->geo, root, root, 0);
    auto fill = [&](int m, Node& b) {
        hipLaunchKernelGGL(tridiag_block_kernel, grid2(b.m(), b.q()), dim3(kThreads), 0, s, b.m(), b.q(), b.t0, b.s0,
                           dg + (size_t)m * n, eo + (size_t)m * n, b.d);
    };
    const int rc = factor_layers(sf, fill, cp, s, msg);
    if (rc == HSWEEP_OK) *out = sf;
    return rc;
}

int strong_apply(StrongFactors* sf, int dir, const c128* f, c128* u, int nrhs, const int* active, hipStream_t s,
                 std::string* msg) {
    const int n = sf->side;
    const dim3 g2 = grid2(n, nrhs);
    auto gather = [&](int m, const c128* a, const c128* Wp, c128* L) {
        hipLaunchKernelGGL(gather_layer_kernel, g2, dim3(kThreads), 0, s, n, nrhs, dir, m, f, a, Wp, L);
    };
    auto scatter = [&](int m, const c128* L) {
        hipLaunchKernelGGL(scatter_layer_kernel, g2, dim3(kThreads), 0, s, n, nrhs, dir, m, L, active, u);
    };
    return apply_layers(sf, nrhs, gather, scatter, s, msg);
}

// 3D (Sec. 4): the n faces x3 = const of an n x n x n grid, face points in
// quadtree bisection order.  D, X0, X1, Y0, Y1, Z0: coefficient fields of
// the 7-point operator (n^3 each, x1 fastest, then x2, then x3; Z0 = the
// coupling to the face below).
int strong_factor3(StrongFactors** out, int n, int leaf, int rmax, double tol, uint64_t seed, const c128* D,
                   const c128* X0, const c128* X1, const c128* Y0, const c128* Y1, const c128* Z0, hipStream_t s,
                   std::string* msg) {
    *out = nullptr;
    StrongFactors* sf = new StrongFactors();
    const int N = n * n;
    sf->nl = n; sf->N = N; sf->side = n;
    sf->leaf = leaf; sf->rmax = rmax; sf->tol = tol; sf->seed = seed;
    sf->geo.face = true;
    sf->geo.L = sf->L = face_depth(n, leaf);
    const Cluster root{0, N, 0, n, 0, n, 0, 0, 0};
    build_structure(sf->shape, sf->geo, root, root, 0);
    std::vector<int> perm;
    face_order(sf->geo, root, n, perm);
    hipError_t e = hipMalloc((void**)&sf->permd, (size_t)N * sizeof(int));
    if (e == hipSuccess) e = hipMemcpy(sf->permd, perm.data(), (size_t)N * sizeof(int), hipMemcpyHostToDevice);
    if (e != hipSuccess)
        return fail_new(sf, e == hipErrorOutOfMemory ? HSWEEP_ENOMEM : HSWEEP_EDEVICE,
                        std::string("strong factorization: ") + hipGetErrorString(e), msg);
    // couplings a_m = Z0 of face m + 1, in position order
    c128* cp = nullptr;
    if (n > 1) {
        e = hipMalloc((void**)&cp, (size_t)(n - 1) * N * sizeof(c128));
        if (e != hipSuccess) return fail_new(sf, HSWEEP_ENOMEM, "device memory for the face couplings", msg);
        hipLaunchKernelGGL(permute_rows_kernel, grid2(N, n - 1), dim3(kThreads), 0, s, n - 1, N,
                           (const int*)sf->permd, Z0 + N, cp);
    }
    const int* perm_d = sf->permd;
    auto fill = [&](int m, Node& b) {
        const size_t o = (size_t)m * N;
        hipLaunchKernelGGL(face_block_kernel, grid2(b.m(), b.q()), dim3(kThreads), 0, s, b.m(), b.q(), b.t0, b.s0, n,
                           perm_d, D + o, X0 + o, X1 + o, Y0 + o, Y1 + o, b.d);
    };
    const int rc = factor_layers(sf, fill, cp, s, msg);
    if (cp) (void)hipFree(cp);
    if (rc == HSWEEP_OK) *out = sf;
    return rc;
}

int strong_apply3(StrongFactors* sf, const c128* f, c128* u, int nrhs, const int* active, hipStream_t s,
                  std::string* msg) {
    const int N = sf->N, nl = sf->nl;
    const dim3 g2 = grid2(N, nrhs);
    const int* perm = sf->permd;
    auto gather = [&](int m, const c128* a, const c128* Wp, c128* L) {
        hipLaunchKernelGGL(gather_face_kernel, g2, dim3(kThreads), 0, s, N, nl, nrhs, m, perm, f, a, Wp, L);
    };
    auto scatter = [&](int m, const c128* L) {
        hipLaunchKernelGGL(scatter_face_kernel, g2, dim3(kThreads), 0, s, N, nl, nrhs, m, perm, L, active, u);
    };
    return apply_layers(sf, nrhs, gather, scatter, s, msg);
}
