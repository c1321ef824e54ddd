// Complex arithmetic for device and host code, templated on the real type.
// Values are interleaved (re, im) pairs, so an array of cpx<double> has the
// same layout as a complex128 array and cpx<float> as complex64.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

template <typename T>
struct __align__(2 * sizeof(T)) cpx {
    T re, im;
};

using c64 = cpx<float>;
using c128 = cpx<double>;

#define HD __host__ __device__ __forceinline__

template <typename T> HD cpx<T> mk(T r, T i) { cpx<T> z; z.re = r; z.im = i; return z; }
template <typename T> HD cpx<T> czero() { return mk<T>(T(0), T(0)); }
template <typename T> HD cpx<T> operator+(cpx<T> a, cpx<T> b) { return mk<T>(a.re + b.re, a.im + b.im); }
template <typename T> HD cpx<T> operator-(cpx<T> a, cpx<T> b) { return mk<T>(a.re - b.re, a.im - b.im); }
template <typename T> HD cpx<T> operator-(cpx<T> a) { return mk<T>(-a.re, -a.im); }
template <typename T> HD cpx<T> operator*(cpx<T> a, cpx<T> b) {
    return mk<T>(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename T> HD cpx<T> operator*(T s, cpx<T> a) { return mk<T>(s * a.re, s * a.im); }
template <typename T> HD cpx<T>& operator+=(cpx<T>& a, cpx<T> b) { a.re += b.re; a.im += b.im; return a; }
template <typename T> HD cpx<T>& operator-=(cpx<T>& a, cpx<T> b) { a.re -= b.re; a.im -= b.im; return a; }
template <typename T> HD cpx<T> conj(cpx<T> a) { return mk<T>(a.re, -a.im); }
template <typename T> HD T abs2(cpx<T> a) { return a.re * a.re + a.im * a.im; }
// a += b * c
template <typename T> HD void cfma(cpx<T>& a, cpx<T> b, cpx<T> c) {
    a.re = fma(b.re, c.re, a.re); a.re = fma(-b.im, c.im, a.re);
    a.im = fma(b.re, c.im, a.im); a.im = fma(b.im, c.re, a.im);
}
// a += conj(b) * c
template <typename T> HD void cfma_conj(cpx<T>& a, cpx<T> b, cpx<T> c) {
    a.re = fma(b.re, c.re, a.re); a.re = fma(b.im, c.im, a.re);
    a.im = fma(b.re, c.im, a.im); a.im = fma(-b.im, c.re, a.im);
}
// 1 / a, scaled to avoid overflow of |a|^2
template <typename T> HD cpx<T> cinv(cpx<T> a) {
    T s = fabs(a.re) > fabs(a.im) ? fabs(a.re) : fabs(a.im);
    if (s == T(0)) return mk<T>(T(1) / s, T(0));
    T ar = a.re / s, ai = a.im / s;
    T d = (ar * ar + ai * ai) * s;
    return mk<T>(ar / d, -ai / d);
}
template <typename To, typename Ti> HD cpx<To> ccast(cpx<Ti> a) { return mk<To>(To(a.re), To(a.im)); }
