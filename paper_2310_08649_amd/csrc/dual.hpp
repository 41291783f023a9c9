// Forward-mode automatic differentiation on the device: a value with K
// directional derivatives.  Evaluating a right-hand side once on duals seeded
// with the unit vectors gives its whole state Jacobian (the forward-mode AD
// option of Section 2.2 for the Jacobian j), in registers.
#pragma once

#include <hip/hip_runtime.h>

namespace tvi {

template <int K>
struct Dual {
    double v;
    double d[K];
    __device__ __forceinline__ Dual() = default;
    __device__ __forceinline__ Dual(double x) : v(x)
    {
#pragma unroll
        for (int k = 0; k < K; ++k) d[k] = 0.0;
    }
};

__device__ __forceinline__ double val(double x) { return x; }
template <int K>
__device__ __forceinline__ double val(const Dual<K> &x) { return x.v; }

// derivative part scaled: r.d = a * x.d (+ b * y.d)
template <int K>
__device__ __forceinline__ Dual<K> lin1(double v, double a, const Dual<K> &x)
{
    Dual<K> r;
    r.v = v;
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = a * x.d[k];
    return r;
}
template <int K>
__device__ __forceinline__ Dual<K> lin2(double v, double a, const Dual<K> &x, double b, const Dual<K> &y)
{
    Dual<K> r;
    r.v = v;
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = fma(a, x.d[k], b * y.d[k]);
    return r;
}

template <int K>
__device__ __forceinline__ Dual<K> operator-(const Dual<K> &x) { return lin1(-x.v, -1.0, x); }
template <int K>
__device__ __forceinline__ Dual<K> operator+(const Dual<K> &x, const Dual<K> &y) { return lin2(x.v + y.v, 1.0, x, 1.0, y); }
template <int K>
__device__ __forceinline__ Dual<K> operator-(const Dual<K> &x, const Dual<K> &y) { return lin2(x.v - y.v, 1.0, x, -1.0, y); }
template <int K>
__device__ __forceinline__ Dual<K> operator*(const Dual<K> &x, const Dual<K> &y) { return lin2(x.v * y.v, y.v, x, x.v, y); }
template <int K>
__device__ __forceinline__ Dual<K> operator/(const Dual<K> &x, const Dual<K> &y)
{
    const double q = x.v / y.v;
    return lin2(q, 1.0 / y.v, x, -q / y.v, y);
}
template <int K>
__device__ __forceinline__ Dual<K> operator+(const Dual<K> &x, double c) { return lin1(x.v + c, 1.0, x); }
template <int K>
__device__ __forceinline__ Dual<K> operator+(double c, const Dual<K> &x) { return lin1(c + x.v, 1.0, x); }
template <int K>
__device__ __forceinline__ Dual<K> operator-(const Dual<K> &x, double c) { return lin1(x.v - c, 1.0, x); }
template <int K>
__device__ __forceinline__ Dual<K> operator-(double c, const Dual<K> &x) { return lin1(c - x.v, -1.0, x); }
template <int K>
__device__ __forceinline__ Dual<K> operator*(const Dual<K> &x, double c) { return lin1(x.v * c, c, x); }
template <int K>
__device__ __forceinline__ Dual<K> operator*(double c, const Dual<K> &x) { return lin1(c * x.v, c, x); }
template <int K>
__device__ __forceinline__ Dual<K> operator/(const Dual<K> &x, double c) { return lin1(x.v / c, 1.0 / c, x); }
template <int K>
__device__ __forceinline__ Dual<K> operator/(double c, const Dual<K> &x)
{
    const double q = c / x.v;
    return lin1(q, -q / x.v, x);
}
// fused multiply-add and absolute value for both plain and dual arguments
// (own names: overloads of fma / fabs here would hide the plain ones)
__device__ __forceinline__ double fma_t(double a, double b, double c) { return fma(a, b, c); }
template <int K>
__device__ __forceinline__ Dual<K> fma_t(double a, const Dual<K> &b, const Dual<K> &c)
{
    return lin2(fma(a, b.v, c.v), a, b, 1.0, c);
}
__device__ __forceinline__ double abs_t(double x) { return fabs(x); }
template <int K>
__device__ __forceinline__ Dual<K> abs_t(const Dual<K> &x) { return lin1(fabs(x.v), x.v < 0.0 ? -1.0 : 1.0, x); }
// x^e for x > 0 as x^(e-1) x (the callers guard the sign)
__device__ __forceinline__ double pow_pos(double x, double e) { return pow(x, e - 1.0) * x; }
template <int K>
__device__ __forceinline__ Dual<K> pow_pos(const Dual<K> &x, double e)
{
    const double pm1 = pow(x.v, e - 1.0);
    return lin1(pm1 * x.v, e * pm1, x);
}

// elementary functions for plain and dual arguments (the derivative rule of
// each applied to every direction), for right-hand sides written once for both
__device__ __forceinline__ double exp_t(double x) { return exp(x); }
template <int K>
__device__ __forceinline__ Dual<K> exp_t(const Dual<K> &x)
{
    const double e = exp(x.v);
    return lin1(e, e, x);
}
__device__ __forceinline__ double log_t(double x) { return log(x); }
template <int K>
__device__ __forceinline__ Dual<K> log_t(const Dual<K> &x) { return lin1(log(x.v), 1.0 / x.v, x); }
__device__ __forceinline__ double sqrt_t(double x) { return sqrt(x); }
template <int K>
__device__ __forceinline__ Dual<K> sqrt_t(const Dual<K> &x)
{
    const double r = sqrt(x.v);
    return lin1(r, 0.5 / r, x);
}
__device__ __forceinline__ double sin_t(double x) { return sin(x); }
template <int K>
__device__ __forceinline__ Dual<K> sin_t(const Dual<K> &x) { return lin1(sin(x.v), cos(x.v), x); }
__device__ __forceinline__ double cos_t(double x) { return cos(x); }
template <int K>
__device__ __forceinline__ Dual<K> cos_t(const Dual<K> &x) { return lin1(cos(x.v), -sin(x.v), x); }
__device__ __forceinline__ double tanh_t(double x) { return tanh(x); }
template <int K>
__device__ __forceinline__ Dual<K> tanh_t(const Dual<K> &x)
{
    const double th = tanh(x.v);
    return lin1(th, 1.0 - th * th, x);
}

} // namespace tvi
