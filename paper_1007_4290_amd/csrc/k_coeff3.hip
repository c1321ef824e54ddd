// Coefficient fields and the FP64 7-point operator of the 3D problem
// (Sec. 4, discretization): the equation divided by s1 s2 s3,
//   d1((s1/(s2 s3)) d1 u) + d2((s2/(s1 s3)) d2 u) + d3((s3/(s1 s2)) d3 u)
//     + omega^2/(s1 s2 s3 c^2) u = f,
// with the stretching s_a = (1 + i sigma(x_a)/omega)^{-1} of each axis
// tabulated on nodes (as 1/s) and half nodes (as s), and the coupling of
// point (i, j, k) to (i+1, j, k) equal to s1(x_{i+1/2}) / (s2(x_j) s3(x_k)) / h^2
// (the same product for both rows it couples, so A = A^t exactly).  Points
// are ordered x1 fastest, then x2, then x3; zero Dirichlet values outside.
#include "internal.hpp"

namespace {

struct Tab3 {
    const c128 *isn1, *sh1, *isn2, *sh2, *isn3, *sh3;
};

__global__ void coeff3_kernel(int n, double w2, double ih2, const double* __restrict__ c, Tab3 t, Coef3 out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y, k = blockIdx.z;
    if (i >= n) return;
    const size_t p = ((size_t)k * n + j) * n + i;
    const c128 yz = t.isn2[j] * t.isn3[k], xz = t.isn1[i] * t.isn3[k], xy = t.isn1[i] * t.isn2[j];
    const c128 x0 = ih2 * (t.sh1[i] * yz), x1 = ih2 * (t.sh1[i + 1] * yz);
    const c128 y0 = ih2 * (t.sh2[j] * xz), y1 = ih2 * (t.sh2[j + 1] * xz);
    const c128 z0 = ih2 * (t.sh3[k] * xy), z1 = ih2 * (t.sh3[k + 1] * xy);
    const double cc = c[p];
    out.X0[p] = x0; out.X1[p] = x1;
    out.Y0[p] = y0; out.Y1[p] = y1;
    out.Z0[p] = z0; out.Z1[p] = z1;
    out.D[p] = (w2 / (cc * cc)) * (xy * t.isn3[k]) - (((x0 + x1) + (y0 + y1)) + (z0 + z1));
}

__global__ void stencil3_kernel(int n, Coef3 cf, const c128* __restrict__ x, const c128* __restrict__ f,
                                c128* __restrict__ y, const int* __restrict__ active) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int jk = blockIdx.y, r = blockIdx.z;
    if (i >= n) return;
    const int j = jk % n, k = jk / n;
    const size_t N3 = (size_t)n * n * n;
    const size_t p = ((size_t)k * n + j) * n + i;
    const size_t o = (size_t)r * N3 + p;
    if (active && !active[r]) { y[o] = czero<double>(); return; }
    const c128* xr = x + (size_t)r * N3;
    c128 acc = cf.D[p] * xr[p];
    if (i > 0) acc += cf.X0[p] * xr[p - 1];
    if (i < n - 1) acc += cf.X1[p] * xr[p + 1];
    if (j > 0) acc += cf.Y0[p] * xr[p - n];
    if (j < n - 1) acc += cf.Y1[p] * xr[p + n];
    if (k > 0) acc += cf.Z0[p] * xr[p - (size_t)n * n];
    if (k < n - 1) acc += cf.Z1[p] * xr[p + (size_t)n * n];
    y[o] = f ? f[o] - acc : acc;
}

}  // namespace

void launch_coeff3(int n, double omega, const double* c, const c128* const isn[3], const c128* const sh[3],
                   const Coef3& out, hipStream_t s) {
    const double h = 1.0 / (n + 1);
    const Tab3 t{isn[0], sh[0], isn[1], sh[1], isn[2], sh[2]};
    const int th = n >= 128 ? 128 : 64;
    hipLaunchKernelGGL(coeff3_kernel, dim3((n + th - 1) / th, n, n), dim3(th), 0, s, n, omega * omega, 1.0 / (h * h),
                       c, t, out);
}

void launch_stencil3(int n, int nrhs, const Coef3& cf, const c128* x, const c128* f, c128* y, const int* active,
                     hipStream_t s) {
    const int th = n >= 128 ? 128 : 64;
    hipLaunchKernelGGL(stencil3_kernel, dim3((n + th - 1) / th, n * n, nrhs), dim3(th), 0, s, n, cf, x, f, y, active);
}
