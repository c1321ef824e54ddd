// PML profile, stencil coefficients, the FP64 5-point operator and the
// velocity gradient (Sec. 2.1, eqs. sigma and helmd).
//
// The stretching s(t) = 1 / (1 + i sigma(t)/omega) is tabulated once on the
// interior nodes x_i = (i+1) h and the half nodes x_{i+1/2} = (i+1/2) h
// (0-based i).  Every edge coefficient of the stencil is then a product of
// two table entries:
//   horizontal edge between columns i and i+1 of row j:  s(x_{i+1/2}) / s(x_j) / h^2
//   vertical edge between rows j and j+1 of column i:    s(x_{j+1/2}) / s(x_i) / h^2
// and is evaluated by the same function for both rows it couples, so the
// operator is exactly symmetric.  1/s(x) = 1 + i sigma(x)/omega is stored
// directly to avoid a complex division.
#include "internal.hpp"

namespace {

__device__ __forceinline__ double sigma_of(double t, double eta, double C) {
    if (eta <= 0.0) return 0.0;
    if (t < eta) { double q = (t - eta) / eta; return (C / eta) * q * q; }
    if (t > 1.0 - eta) { double q = (t - 1.0 + eta) / eta; return (C / eta) * q * q; }
    return 0.0;
}

__global__ void pml_1d_kernel(int n, double omega, double eta, double C, c128* sn, c128* isn, c128* sh) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    double h = 1.0 / (n + 1);
    if (i <= n) {
        double t = (i + 0.5) * h;
        sh[i] = cinv(mk(1.0, sigma_of(t, eta, C) / omega));
    }
    if (i < n) {
        double t = (i + 1) * h;
        c128 z = mk(1.0, sigma_of(t, eta, C) / omega);
        isn[i] = z;
        sn[i] = cinv(z);
    }
}

struct Coef {
    const double* c; const c128* isn; const c128* sh; int n; double ih2; double w2;
    // edge between (i, j) and (i+1, j) for half index ih = i + 1 in 0..n (0-based nodes i)
    __device__ __forceinline__ c128 ex(int ih, int j) const { return ih2 * (sh[ih] * isn[j]); }
    // edge between (i, j) and (i, j+1) for half index jh = j + 1 in 0..n
    __device__ __forceinline__ c128 ey(int i, int jh) const { return ih2 * (sh[jh] * isn[i]); }
    __device__ __forceinline__ c128 diag(int i, int j) const {
        double cc = c[(size_t)j * n + i];
        c128 d = (w2 / (cc * cc)) * (isn[i] * isn[j]);
        return d - (ex(i, j) + ex(i + 1, j) + ey(i, j) + ey(i, j + 1));
    }
};

template <typename T>
__global__ void layer_coeffs_kernel(Coef cf, int np, cpx<T>* dg, cpx<T>* eo, cpx<T>* cp) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int m = blockIdx.y;
    int n = cf.n;
    if (i >= np) return;
    size_t o = (size_t)m * np + i;
    dg[o] = i < n ? ccast<T>(cf.diag(i, m)) : mk<T>(T(1), T(0));
    eo[o] = i < n - 1 ? ccast<T>(cf.ex(i + 1, m)) : czero<T>();
    if (m < n - 1) cp[o] = i < n ? ccast<T>(cf.ey(i, m + 1)) : czero<T>();
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
    c128 acc = cf.diag(i, j) * xk[(size_t)j * n + i];
    if (i > 0) acc += cf.ex(i, j) * xk[(size_t)j * n + i - 1];
    if (i < n - 1) acc += cf.ex(i + 1, j) * xk[(size_t)j * n + i + 1];
    if (j > 0) acc += cf.ey(i, j) * xk[(size_t)(j - 1) * n + i];
    if (j < n - 1) acc += cf.ey(i, j + 1) * xk[(size_t)(j + 1) * n + i];
    y[o] = f ? f[o] - acc : acc;
}

// grad[p] = sum_k Re(mu_k[p] u_k[p] * 2 omega^2 / ((s1 s2)[p] c[p]^3)); 1/(s1 s2) = isn_i isn_j.
__global__ void grad_kernel(int n, int nrhs, double w2, const double* __restrict__ c,
                            const c128* __restrict__ isn, const c128* __restrict__ u,
                            const c128* __restrict__ mu, double* __restrict__ grad) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y;
    if (i >= n) return;
    size_t p = (size_t)j * n + i;
    size_t N = (size_t)n * n;
    double cc = c[p];
    c128 fac = (2.0 * w2 / (cc * cc * cc)) * (isn[i] * isn[j]);
    double g = 0.0;
    for (int k = 0; k < nrhs; ++k) {
        c128 z = mu[k * N + p] * u[k * N + p];
        g += (z * fac).re;
    }
    grad[p] = g;
}

Coef make_coef(int n, double omega, const double* c, const c128* isn, const c128* sh) {
    Coef cf;
    cf.c = c; cf.isn = isn; cf.sh = sh; cf.n = n;
    double h = 1.0 / (n + 1);
    cf.ih2 = 1.0 / (h * h);
    cf.w2 = omega * omega;
    return cf;
}

}  // namespace

void launch_pml_1d(int n, double omega, double eta, double C, c128* sn, c128* isn, c128* sh, hipStream_t s) {
    int th = 256;
    hipLaunchKernelGGL(pml_1d_kernel, dim3((n + 1 + th - 1) / th), dim3(th), 0, s, n, omega, eta, C, sn, isn, sh);
}

template <typename T>
void launch_layer_coeffs(int n, int np, double omega, const double* c, const c128* isn, const c128* sh,
                         cpx<T>* dg, cpx<T>* eo, cpx<T>* cp, hipStream_t s) {
    Coef cf = make_coef(n, omega, c, isn, sh);
    int th = 256;
    hipLaunchKernelGGL(layer_coeffs_kernel<T>, dim3((np + th - 1) / th, n), dim3(th), 0, s, cf, np, dg, eo, cp);
}
template void launch_layer_coeffs<float>(int, int, double, const double*, const c128*, const c128*, c64*, c64*, c64*, hipStream_t);
template void launch_layer_coeffs<double>(int, int, double, const double*, const c128*, const c128*, c128*, c128*, c128*, hipStream_t);

void launch_stencil(int n, int nrhs, double omega, const double* c, const c128* isn, const c128* sh,
                    const c128* x, const c128* f, c128* y, const int* active, hipStream_t s) {
    Coef cf = make_coef(n, omega, c, isn, sh);
    int th = n >= 256 ? 256 : 64;
    hipLaunchKernelGGL(stencil_kernel, dim3((n + th - 1) / th, n, nrhs), dim3(th), 0, s, cf, x, f, y, active);
}

void launch_grad(int n, int nrhs, double omega, const double* c, const c128* isn,
                 const c128* u, const c128* mu, double* grad, hipStream_t s) {
    int th = n >= 256 ? 256 : 64;
    hipLaunchKernelGGL(grad_kernel, dim3((n + th - 1) / th, n), dim3(th), 0, s, n, nrhs, omega * omega, c, isn, u, mu, grad);
}
