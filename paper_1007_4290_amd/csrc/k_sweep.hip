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
// Thread i owns row i of the layer; the couplings A_{m,m+-1} are diagonal,
// so the vector updates between layers are thread-local and only the
// matvec needs the workgroup.  The factor data of every layer is read once
// per layer step, with consecutive threads reading consecutive addresses.
#include "internal.hpp"

namespace {

template <typename T>
struct SweepShared {
    cpx<T>* xs;    // np
    cpx<T>* part;  // L * r * (np / b) chunk partials
    cpx<T>* gs;    // heap-indexed node reductions, (2^(L+1) - 1) * r
    cpx<T>* zs;    // (2^L - 1) * 2r
};

template <typename T>
__device__ cpx<T> apply_T(const Plan& p, const cpx<T>* __restrict__ lay, cpx<T> x, const SweepShared<T>& sh) {
    const int np = p.np, b = p.b, L = p.L, r = p.r;
    const int i = threadIdx.x;
    const bool row = i < np;
    const cpx<T>* K = lay;
    const cpx<T>* P = lay + p.eK;
    const cpx<T>* X = lay + p.eK + p.eP;
    __syncthreads();   // previous step may still read xs (L == 0 has no later barrier)
    if (row) sh.xs[i] = x;
    __syncthreads();
    cpx<T> y = czero<T>();
    if (row) {
        int t = i / b, il = i % b;
        const cpx<T>* Kt = K + (size_t)t * b * b + il;
        const cpx<T>* xl = sh.xs + t * b;
        for (int j = 0; j < b; ++j) cfma(y, Kt[(size_t)j * b], xl[j]);
    }
    if (L == 0) return y;
    const int nch = np / b;
    const int ntask = L * r * nch;
    for (int e = i; e < ntask; e += blockDim.x) {
        int ch = e % nch;
        int lk = e / nch;                       // (lvl-1)*r + k
        const cpx<T>* Pc = P + (size_t)lk * np + ch * b;
        const cpx<T>* xc = sh.xs + ch * b;
        cpx<T> acc = czero<T>();
        for (int j = 0; j < b; ++j) cfma(acc, Pc[j], xc[j]);
        sh.part[e] = acc;
    }
    __syncthreads();
    // node sums g_c for nodes of levels 1..L: heap id h in [1, 2^(L+1) - 1)
    const int nnode = (1 << (L + 1)) - 2;
    for (int e = i; e < nnode * r; e += blockDim.x) {
        int h = 1 + e / r, k = e % r;
        int lvl = 31 - __clz(h + 1);
        int idx = h - ((1 << lvl) - 1);
        int cpn = nch >> lvl;
        const cpx<T>* pp = sh.part + ((size_t)(lvl - 1) * r + k) * nch + idx * cpn;
        cpx<T> acc = czero<T>();
        for (int q = 0; q < cpn; ++q) acc += pp[q];
        sh.gs[h * r + k] = acc;
    }
    __syncthreads();
    const int npar = (1 << L) - 1;
    const int r2 = 2 * r;
    for (int e = i; e < npar * r2; e += blockDim.x) {
        int q = e / r2, o = e % r2;
        const cpx<T>* Xq = X + (size_t)q * r2 * r2 + o;
        const cpx<T>* g = sh.gs + (size_t)(2 * q + 1) * r;   // children 2q+1, 2q+2 are contiguous
        cpx<T> acc = czero<T>();
        for (int c = 0; c < r2; ++c) cfma(acc, Xq[(size_t)c * r2], g[c]);
        sh.zs[e] = acc;
    }
    __syncthreads();
    if (row) {
        for (int lvl = 1; lvl <= L; ++lvl) {
            int s = np >> lvl;
            int c = i / s;                      // node index at lvl
            int q = (1 << (lvl - 1)) - 1 + (c >> 1);
            const cpx<T>* z = sh.zs + (size_t)q * r2 + (c & 1) * r;
            const cpx<T>* Pl = P + (size_t)(lvl - 1) * r * np + i;
            cpx<T> acc = czero<T>();
            for (int k = 0; k < r; ++k) cfma(acc, Pl[(size_t)k * np], z[k]);
            y -= acc;
        }
    }
    return y;
}

template <typename T>
__global__ __launch_bounds__(1024) void sweep_kernel(Plan p, SweepArgs<T> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int n = p.n, np = p.np, b = p.b, L = p.L, r = p.r;
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
    sh.gs = sh.part + (size_t)L * r * (np / b);
    sh.zs = sh.gs + (size_t)((1 << (L + 1)) - 1) * r;
    cpx<T>* w = a.w + (size_t)rhs * n * np;
    const bool row = i < np;
    const bool real_row = i < n;
    cpx<T> prev = czero<T>();
    for (int m = 0; m < n; ++m) {
        cpx<T> x = czero<T>();
        if (real_row) x = ccast<T>(f[(size_t)m * n + i]);
        if (m > 0 && row) x -= a.cp[(size_t)(m - 1) * np + i] * prev;
        cpx<T> y = apply_T(p, a.fac + (size_t)m * p.eLayer, x, sh);
        if (row) w[(size_t)m * np + i] = y;
        prev = y;
    }
    cpx<T> next = prev;
    if (real_row) u[(size_t)(n - 1) * n + i] = ccast<double>(next);
    for (int m = n - 2; m >= 0; --m) {
        cpx<T> x = czero<T>();
        if (row) x = a.cp[(size_t)m * np + i] * next;
        cpx<T> y = apply_T(p, a.fac + (size_t)m * p.eLayer, x, sh);
        cpx<T> um = czero<T>();
        if (row) um = w[(size_t)m * np + i] - y;
        if (real_row) u[(size_t)m * n + i] = ccast<double>(um);
        next = um;
    }
}

}  // namespace

size_t sweep_lds_bytes(const Plan& p, size_t elem) {
    size_t e = (size_t)p.np + (size_t)p.L * p.r * (p.np / p.b) + (size_t)((1 << (p.L + 1)) - 1) * p.r +
               (size_t)((1 << p.L) - 1) * 2 * p.r;
    return e * elem;
}

int sweep_threads(const Plan& p) {
    int t = p.np < 64 ? 64 : p.np;
    return (t + 63) / 64 * 64;
}

template <typename T>
int launch_sweep(const Plan& p, const SweepArgs<T>& a, hipStream_t s) {
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void*)sweep_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        attr = true;
    }
    size_t lds = sweep_lds_bytes(p, sizeof(cpx<T>));
    hipLaunchKernelGGL(sweep_kernel<T>, dim3(a.nrhs), dim3(sweep_threads(p)), lds, s, p, a);
    return 0;
}

template int launch_sweep<float>(const Plan&, const SweepArgs<float>&, hipStream_t);
template int launch_sweep<double>(const Plan&, const SweepArgs<double>&, hipStream_t);
