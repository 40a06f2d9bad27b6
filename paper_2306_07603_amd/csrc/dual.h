// dual.h -- forward-mode (tangent-linear) arithmetic: a value and its
// derivatives with respect to N parameters, carried through every operation
// of the per-node IFDLBM arithmetic templates.
#pragma once

#include <hip/hip_runtime.h>

namespace ifd {

template <int N>
struct Dual {
    double v;
    double d[N];

    __host__ __device__ Dual() : v(0.0)
    {
        for (int i = 0; i < N; ++i) d[i] = 0.0;
    }
    __host__ __device__ Dual(double x) : v(x)
    {
        for (int i = 0; i < N; ++i) d[i] = 0.0;
    }
    __host__ __device__ static Dual make(double x, const double* dx)
    {
        Dual r(x);
        for (int i = 0; i < N; ++i) r.d[i] = dx[i];
        return r;
    }
    __host__ __device__ explicit operator double() const { return v; }
};

template <int N> __host__ __device__ inline Dual<N> operator+(const Dual<N>& a, const Dual<N>& b)
{
    Dual<N> r(a.v + b.v);
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i];
    return r;
}
template <int N> __host__ __device__ inline Dual<N> operator-(const Dual<N>& a, const Dual<N>& b)
{
    Dual<N> r(a.v - b.v);
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i];
    return r;
}
template <int N> __host__ __device__ inline Dual<N> operator-(const Dual<N>& a)
{
    Dual<N> r(-a.v);
    for (int i = 0; i < N; ++i) r.d[i] = -a.d[i];
    return r;
}
template <int N> __host__ __device__ inline Dual<N> operator*(const Dual<N>& a, const Dual<N>& b)
{
    Dual<N> r(a.v * b.v);
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
    return r;
}
template <int N> __host__ __device__ inline Dual<N> operator/(const Dual<N>& a, const Dual<N>& b)
{
    const double q = a.v / b.v;
    Dual<N> r(q);
    for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] - q * b.d[i]) / b.v;
    return r;
}
template <int N> __host__ __device__ inline Dual<N>& operator+=(Dual<N>& a, const Dual<N>& b) { return a = a + b; }
template <int N> __host__ __device__ inline Dual<N>& operator-=(Dual<N>& a, const Dual<N>& b) { return a = a - b; }
template <int N> __host__ __device__ inline Dual<N>& operator*=(Dual<N>& a, const Dual<N>& b) { return a = a * b; }
template <int N> __host__ __device__ inline bool operator>(const Dual<N>& a, const Dual<N>& b) { return a.v > b.v; }
template <int N> __host__ __device__ inline bool operator<(const Dual<N>& a, const Dual<N>& b) { return a.v < b.v; }
template <int N> __host__ __device__ inline bool operator>=(const Dual<N>& a, const Dual<N>& b) { return a.v >= b.v; }
template <int N> __host__ __device__ inline bool operator!=(const Dual<N>& a, const Dual<N>& b) { return a.v != b.v; }

// x^y for x > 0: d(x^y) = x^y (y dx / x + ln x dy)
template <int N> __host__ __device__ inline Dual<N> dual_pow(const Dual<N>& x, const Dual<N>& y)
{
    const double p = pow(x.v, y.v), lx = log(x.v);
    Dual<N> r(p);
    for (int i = 0; i < N; ++i) r.d[i] = p * (y.v * x.d[i] / x.v + lx * y.d[i]);
    return r;
}

template <int N> __device__ inline bool dual_isfinite(const Dual<N>& x)
{
    bool ok = isfinite(x.v);
    for (int i = 0; i < N; ++i) ok = ok && isfinite(x.d[i]);
    return ok;
}

}  // namespace ifd
