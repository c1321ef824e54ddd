// PML profile, stencil coefficients, the FP64 5-point operator, the
// velocity gradient and Dirichlet edge data (Sec. 2.1, eqs. sigma and helmd;
// Sec. 2.5).
//
// The stretching s(t) = 1 / (1 + i sigma(t)/omega) is tabulated once per axis
// on the interior nodes x_i = (i+1) h and the half nodes x_{i+1/2} = (i+1/2) h
// (0-based i); each axis has its own layer widths at t = 0 and t = 1 (width
// 0: zero Dirichlet condition on that side, no layer).  Every edge
// coefficient of the stencil is then a product of two table entries:
//   horizontal edge between columns i and i+1 of row j:  s1(x_{i+1/2}) / s2(x_j) / h^2
//   vertical edge between rows j and j+1 of column i:    s2(x_{j+1/2}) / s1(x_i) / h^2
// and is evaluated by the same function for both rows it couples, so the
// operator is exactly symmetric.  1/s(x) = 1 + i sigma(x)/omega is stored
// directly to avoid a complex division.
//
// A side with the second-order absorbing boundary condition (Sec. 3, other
// boundary conditions) has no layer; its boundary value is eliminated,
// u_b = a u_0 + g D_tt u_0 with a = (2 + ikh)/(2 - ikh), g = ih/(k(2 - ikh)),
// k = omega/c at the first interior point: the row of u_0 gets e_b a on its
// diagonal (e_b its coupling to the boundary node) and e_b g D_tt u_0 as
// couplings along the side, in flux form with one weight per edge (the mean
// of w = e_b g / h^2 at its two points, symmetric again); at an end of the
// side the flux goes to the corner value, zero next to a side without the
// condition and dropped next to one with it.  Coef::exg, eyg and diagg are
// the couplings and diagonal with these closures; ex and ey stay the plain
// edge couplings (the ones to boundary nodes are what Dirichlet data and the
// closures multiply).
//
// The factorization works in the frame of its sweep direction (Sec. 2.4):
// frame point (i', m') (position i' along layer m') is the grid point
//   +x2: (i', m')   -x2: (i', n-1-m')   +x1: (m', i')   -x1: (n-1-m', i'),
// and the frame coefficients are the natural ones of the same grid points.
#include "internal.hpp"

namespace {

__device__ __forceinline__ double sigma_of(double t, double eta_lo, double eta_hi, double C) {
    if (eta_lo > 0.0 && t < eta_lo) { double q = (t - eta_lo) / eta_lo; return (C / eta_lo) * q * q; }
    if (eta_hi > 0.0 && t > 1.0 - eta_hi) { double q = (t - 1.0 + eta_hi) / eta_hi; return (C / eta_hi) * q * q; }
    return 0.0;
}

__global__ void pml_1d_kernel(int n, double omega, double eta_lo, double eta_hi, double C, c128* isn, c128* sh) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    double h = 1.0 / (n + 1);
    if (i <= n) {
        double t = (i + 0.5) * h;
        sh[i] = cinv(mk(1.0, sigma_of(t, eta_lo, eta_hi, C) / omega));
    }
    if (i < n) {
        double t = (i + 1) * h;
        isn[i] = mk(1.0, sigma_of(t, eta_lo, eta_hi, C) / omega);
    }
}

struct Coef {
    const double* c; AxisTables t; int n; double h; double ih2; double w; double w2;
    // edge between (i, j) and (i+1, j) for half index ih = i + 1 in 0..n (0-based nodes i)
    __device__ __forceinline__ c128 ex(int ih, int j) const { return ih2 * (t.sh1[ih] * t.isn2[j]); }
    // edge between (i, j) and (i, j+1) for half index jh = j + 1 in 0..n
    __device__ __forceinline__ c128 ey(int i, int jh) const { return ih2 * (t.sh2[jh] * t.isn1[i]); }
    __device__ __forceinline__ c128 diag(int i, int j) const {
        double cc = c[(size_t)j * n + i];
        c128 d = (w2 / (cc * cc)) * (t.isn1[i] * t.isn2[j]);
        return d - (ex(i, j) + ex(i + 1, j) + ey(i, j) + ey(i, j + 1));
    }
    // ---- absorbing boundary condition on the sides of t.abc (HSWEEP_EDGE_* bits)
    __device__ __forceinline__ bool abc(int sd) const { return (t.abc >> sd) & 1; }
    __device__ __forceinline__ double kw(int i, int j) const { return w / c[(size_t)j * n + i]; }
    __device__ __forceinline__ c128 abc_a(double k) const { return mk(2.0, k * h) * cinv(mk(2.0, -k * h)); }
    __device__ __forceinline__ c128 abc_g(double k) const { return mk(0.0, h) * cinv(mk(2.0 * k, -k * k * h)); }
    // coupling of the point next to side sd to its boundary node
    __device__ __forceinline__ c128 eb(int sd, int i, int j) const {
        return sd == 0 ? ex(0, j) : sd == 1 ? ex(n, j) : sd == 2 ? ey(i, 0) : ey(i, n);
    }
    // tangential weight w = e_b g / h^2 of that point
    __device__ __forceinline__ c128 abc_w(int sd, int i, int j) const {
        return ih2 * (eb(sd, i, j) * abc_g(kw(i, j)));
    }
    // couplings between two grid points (1 <= ih, jh <= n - 1)
    __device__ __forceinline__ c128 exg(int ih, int j) const {
        c128 e = ex(ih, j);
        if (t.abc) {
            if (j == 0 && abc(2)) e += 0.5 * (abc_w(2, ih - 1, 0) + abc_w(2, ih, 0));
            if (j == n - 1 && abc(3)) e += 0.5 * (abc_w(3, ih - 1, n - 1) + abc_w(3, ih, n - 1));
        }
        return e;
    }
    __device__ __forceinline__ c128 eyg(int i, int jh) const {
        c128 e = ey(i, jh);
        if (t.abc) {
            if (i == 0 && abc(0)) e += 0.5 * (abc_w(0, 0, jh - 1) + abc_w(0, 0, jh));
            if (i == n - 1 && abc(1)) e += 0.5 * (abc_w(1, n - 1, jh - 1) + abc_w(1, n - 1, jh));
        }
        return e;
    }
    // closure of side sd at a point next to it: position q along the side,
    // ends shared with sides lo and hi
    __device__ __forceinline__ c128 closure(int sd, int i, int j, int q, int lo, int hi) const {
        const bool along_x2 = sd < 2;                 // x1 sides run along x2
        c128 d = eb(sd, i, j) * abc_a(kw(i, j));
        const c128 wq = abc_w(sd, i, j);
        if (q > 0) d -= 0.5 * (wq + (along_x2 ? abc_w(sd, i, j - 1) : abc_w(sd, i - 1, j)));
        else if (!abc(lo)) d -= wq;
        if (q < n - 1) d -= 0.5 * (wq + (along_x2 ? abc_w(sd, i, j + 1) : abc_w(sd, i + 1, j)));
        else if (!abc(hi)) d -= wq;
        return d;
    }
    __device__ __forceinline__ c128 diagg(int i, int j) const {
        c128 d = diag(i, j);
        if (t.abc) {
            if (i == 0 && abc(0)) d += closure(0, i, j, j, 2, 3);
            if (i == n - 1 && abc(1)) d += closure(1, i, j, j, 2, 3);
            if (j == 0 && abc(2)) d += closure(2, i, j, i, 0, 1);
            if (j == n - 1 && abc(3)) d += closure(3, i, j, i, 0, 1);
        }
        return d;
    }
};

// Layer operators in the frame of the sweep direction: dg = diagonal of
// A_{m',m'}, eo[i'] = A_{m',m'}(i', i'+1), cp[i'] = A_{m'+1,m'}(i', i').
template <typename T>
__global__ void layer_coeffs_kernel(Coef cf, int np, int dir, cpx<T>* dg, cpx<T>* eo, cpx<T>* cp) {
    int ip = blockIdx.x * blockDim.x + threadIdx.x;
    int m = blockIdx.y;
    int n = cf.n;
    if (ip >= np) return;
    size_t o = (size_t)m * np + ip;
    const bool real = ip < n;
    // the grid point of frame point (ip, m); clamped for padding rows
    const int a = real ? ip : 0;
    int i, j;
    if (dir == 0) { i = a; j = m; }
    else if (dir == 1) { i = a; j = n - 1 - m; }
    else if (dir == 2) { i = m; j = a; }
    else { i = n - 1 - m; j = a; }
    dg[o] = real ? ccast<T>(cf.diagg(i, j)) : mk<T>(T(1), T(0));
    // along the layer: the next frame point is (i+1, j) for rows, (i, j+1) for columns
    c128 e = ip < n - 1 ? (dir < 2 ? cf.exg(i + 1, j) : cf.eyg(i, j + 1)) : czero<double>();
    eo[o] = ip < n - 1 ? ccast<T>(e) : czero<T>();
    if (m < n - 1) {
        // across layers: frame layer m+1 is row j+1, row j-1, column i+1 or column i-1
        c128 q = dir == 0 ? cf.eyg(i, j + 1) : dir == 1 ? cf.eyg(i, j) : dir == 2 ? cf.exg(i + 1, j) : cf.exg(i, j);
        cp[o] = real ? ccast<T>(q) : czero<T>();
    }
}

// y = A x, or y = f - A x when f is given; one thread per grid point.
__global__ void stencil_kernel(Coef cf, const c128* __restrict__ x, const c128* __restrict__ f,
                               c128* __restrict__ y, const int* __restrict__ active) {
    int n = cf.n;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y;
    int k = blockIdx.z;
    if (i >= n) return;
    size_t N = (size_t)n * n;
    size_t o = k * N + (size_t)j * n + i;
    if (active && !active[k]) { y[o] = czero<double>(); return; }
    const c128* xk = x + k * N;
    c128 acc = cf.diagg(i, j) * xk[(size_t)j * n + i];
    if (i > 0) acc += cf.exg(i, j) * xk[(size_t)j * n + i - 1];
    if (i < n - 1) acc += cf.exg(i + 1, j) * xk[(size_t)j * n + i + 1];
    if (j > 0) acc += cf.eyg(i, j) * xk[(size_t)(j - 1) * n + i];
    if (j < n - 1) acc += cf.eyg(i, j + 1) * xk[(size_t)(j + 1) * n + i];
    y[o] = f ? f[o] - acc : acc;
}

// grad[p] = sum_k Re(mu_k[p] u_k[p] * 2 omega^2 / ((s1 s2)[p] c[p]^3)); 1/(s1 s2) = isn1_i isn2_j.
__global__ void grad_kernel(int n, int nrhs, double w2, const double* __restrict__ c, AxisTables t,
                            const c128* __restrict__ u, const c128* __restrict__ mu, double* __restrict__ grad) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y;
    if (i >= n) return;
    size_t p = (size_t)j * n + i;
    size_t N = (size_t)n * n;
    double cc = c[p];
    c128 fac = (2.0 * w2 / (cc * cc * cc)) * (t.isn1[i] * t.isn2[j]);
    double g = 0.0;
    for (int k = 0; k < nrhs; ++k) {
        c128 z = mu[k * N + p] * u[k * N + p];
        g += (z * fac).re;
    }
    grad[p] = g;
}

// Dirichlet data b (nrhs x n values along one edge) moved to the right-hand
// side: the row next to the edge gets f -= (coefficient of its boundary
// neighbour) * b.  edge 0: x1 = 0, 1: x1 = 1, 2: x2 = 0, 3: x2 = 1.
__global__ void dirichlet_kernel(Coef cf, int edge, const c128* __restrict__ b, c128* __restrict__ f) {
    const int n = cf.n;
    const int k = blockIdx.y;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;   // position along the edge
    if (e >= n) return;
    int i, j;
    c128 coef;
    if (edge == 0) { i = 0; j = e; coef = cf.ex(0, j); }
    else if (edge == 1) { i = n - 1; j = e; coef = cf.ex(n, j); }
    else if (edge == 2) { i = e; j = 0; coef = cf.ey(i, 0); }
    else { i = e; j = n - 1; coef = cf.ey(i, n); }
    const size_t p = (size_t)k * n * n + (size_t)j * n + i;
    f[p] -= coef * b[(size_t)k * n + e];
}

Coef make_coef(int n, double omega, const double* c, const AxisTables& t) {
    Coef cf;
    cf.c = c; cf.t = t; cf.n = n;
    double h = 1.0 / (n + 1);
    cf.h = h;
    cf.ih2 = 1.0 / (h * h);
    cf.w = omega;
    cf.w2 = omega * omega;
    return cf;
}

}  // namespace

void launch_pml_1d(int n, double omega, double eta_lo, double eta_hi, double C, c128* isn, c128* sh, hipStream_t s) {
    int th = 256;
    hipLaunchKernelGGL(pml_1d_kernel, dim3((n + 1 + th - 1) / th), dim3(th), 0, s, n, omega, eta_lo, eta_hi, C, isn, sh);
}

template <typename T>
void launch_layer_coeffs(int n, int np, int dir, double omega, const double* c, const AxisTables& t, cpx<T>* dg,
                         cpx<T>* eo, cpx<T>* cp, hipStream_t s) {
    Coef cf = make_coef(n, omega, c, t);
    int th = 256;
    hipLaunchKernelGGL(layer_coeffs_kernel<T>, dim3((np + th - 1) / th, n), dim3(th), 0, s, cf, np, dir, dg, eo, cp);
}
template void launch_layer_coeffs<float>(int, int, int, double, const double*, const AxisTables&, c64*, c64*, c64*,
                                         hipStream_t);
template void launch_layer_coeffs<double>(int, int, int, double, const double*, const AxisTables&, c128*, c128*, c128*,
                                          hipStream_t);

void launch_stencil(int n, int nrhs, double omega, const double* c, const AxisTables& t, const c128* x, const c128* f,
                    c128* y, const int* active, hipStream_t s) {
    Coef cf = make_coef(n, omega, c, t);
    int th = n >= 256 ? 256 : 64;
    hipLaunchKernelGGL(stencil_kernel, dim3((n + th - 1) / th, n, nrhs), dim3(th), 0, s, cf, x, f, y, active);
}

void launch_grad(int n, int nrhs, double omega, const double* c, const AxisTables& t, const c128* u, const c128* mu,
                 double* grad, hipStream_t s) {
    int th = n >= 256 ? 256 : 64;
    hipLaunchKernelGGL(grad_kernel, dim3((n + th - 1) / th, n), dim3(th), 0, s, n, nrhs, omega * omega, c, t, u, mu, grad);
}

void launch_dirichlet(int n, int nrhs, double omega, const double* c, const AxisTables& t, int edge, const c128* b,
                      c128* f, hipStream_t s) {
    Coef cf = make_coef(n, omega, c, t);
    int th = n >= 256 ? 256 : 64;
    hipLaunchKernelGGL(dirichlet_kernel, dim3((n + th - 1) / th, nrhs), dim3(th), 0, s, cf, edge, b, f);
}
