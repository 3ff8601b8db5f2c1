// kf_dual.hpp -- forward-mode dual numbers for the device code.
//
// A Dual carries a value and K directional derivatives.  The adjoint kernel
// runs the propagation (adaptive RKN stepping, the transport Jacobian it
// builds, landing, local<->global conversions) in this type to obtain the
// exact derivatives of the predicted state and of the transport Jacobian with
// respect to the start state and the two surfaces, and contracts them with
// the reverse-mode adjoints of the Kalman and smoother algebra.
// Discrete decisions (step acceptance, landing) look at the value only, so
// the derivative is that of the step sequence actually taken.
#pragma once
#include <hip/hip_runtime.h>

namespace kfm {

// the plain-number versions stay visible next to the dual overloads below
using ::sqrt;
using ::log;
using ::fabs;
using ::sincos;
using ::atan2;

template <int K>
struct Dual {
    double v;
    double d[K];
    __device__ Dual() : v(0.0) {
#pragma unroll
        for (int i = 0; i < K; ++i) d[i] = 0.0;
    }
    __device__ Dual(double x) : v(x) {
#pragma unroll
        for (int i = 0; i < K; ++i) d[i] = 0.0;
    }
};

// value part of any scalar used by the templated device code
__device__ inline double val(double x) { return x; }
__device__ inline float val(float x) { return x; }
template <int K> __device__ inline double val(const Dual<K>& x) { return x.v; }

// the plain type that holds a scalar's value (step-control bookkeeping)
template <class T> struct ValueOf { using type = T; };
template <int K> struct ValueOf<Dual<K>> { using type = double; };

template <int K>
__device__ inline Dual<K> operator+(const Dual<K>& a, const Dual<K>& b) {
    Dual<K> r(a.v + b.v);
#pragma unroll
    for (int i = 0; i < K; ++i) r.d[i] = a.d[i] + b.d[i];
    return r;
}
template <int K>
__device__ inline Dual<K> operator-(const Dual<K>& a, const Dual<K>& b) {
    Dual<K> r(a.v - b.v);
#pragma unroll
    for (int i = 0; i < K; ++i) r.d[i] = a.d[i] - b.d[i];
    return r;
}
template <int K>
__device__ inline Dual<K> operator-(const Dual<K>& a) {
    Dual<K> r(-a.v);
#pragma unroll
    for (int i = 0; i < K; ++i) r.d[i] = -a.d[i];
    return r;
}
template <int K>
__device__ inline Dual<K> operator*(const Dual<K>& a, const Dual<K>& b) {
    Dual<K> r(a.v * b.v);
#pragma unroll
    for (int i = 0; i < K; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
    return r;
}
template <int K>
__device__ inline Dual<K> operator/(const Dual<K>& a, const Dual<K>& b) {
    const double ib = 1.0 / b.v;
    Dual<K> r(a.v * ib);
#pragma unroll
    for (int i = 0; i < K; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) * ib;
    return r;
}
template <int K> __device__ inline Dual<K> operator+(const Dual<K>& a, double b) { return a + Dual<K>(b); }
template <int K> __device__ inline Dual<K> operator+(double a, const Dual<K>& b) { return Dual<K>(a) + b; }
template <int K> __device__ inline Dual<K> operator-(const Dual<K>& a, double b) { return a - Dual<K>(b); }
template <int K> __device__ inline Dual<K> operator-(double a, const Dual<K>& b) { return Dual<K>(a) - b; }
template <int K>
__device__ inline Dual<K> operator*(const Dual<K>& a, double b) {
    Dual<K> r(a.v * b);
#pragma unroll
    for (int i = 0; i < K; ++i) r.d[i] = a.d[i] * b;
    return r;
}
template <int K> __device__ inline Dual<K> operator*(double a, const Dual<K>& b) { return b * a; }
template <int K> __device__ inline Dual<K> operator/(const Dual<K>& a, double b) { return a * (1.0 / b); }
template <int K> __device__ inline Dual<K> operator/(double a, const Dual<K>& b) { return Dual<K>(a) / b; }
template <int K> __device__ inline Dual<K>& operator+=(Dual<K>& a, const Dual<K>& b) { a = a + b; return a; }
template <int K> __device__ inline Dual<K>& operator-=(Dual<K>& a, const Dual<K>& b) { a = a - b; return a; }
template <int K> __device__ inline bool operator<(const Dual<K>& a, const Dual<K>& b) { return a.v < b.v; }
template <int K> __device__ inline bool operator>(const Dual<K>& a, const Dual<K>& b) { return a.v > b.v; }
template <int K> __device__ inline bool operator<=(const Dual<K>& a, const Dual<K>& b) { return a.v <= b.v; }

template <int K>
__device__ inline Dual<K> chain(const Dual<K>& a, double f, double df) {
    Dual<K> r(f);
#pragma unroll
    for (int i = 0; i < K; ++i) r.d[i] = df * a.d[i];
    return r;
}
template <int K> __device__ inline Dual<K> sqrt(const Dual<K>& a) {
    const double s = ::sqrt(a.v);
    return chain(a, s, 0.5 / s);
}
template <int K> __device__ inline Dual<K> log(const Dual<K>& a) { return chain(a, ::log(a.v), 1.0 / a.v); }
template <int K> __device__ inline Dual<K> fabs(const Dual<K>& a) { return a.v < 0.0 ? -a : a; }
template <int K> __device__ inline void sincos(const Dual<K>& a, Dual<K>* s, Dual<K>* c) {
    double sv, cv;
    ::sincos(a.v, &sv, &cv);
    *s = chain(a, sv, cv);
    *c = chain(a, cv, -sv);
}
template <int K> __device__ inline Dual<K> atan2(const Dual<K>& y, const Dual<K>& x) {
    const double q = 1.0 / (x.v * x.v + y.v * y.v);
    Dual<K> r(::atan2(y.v, x.v));
#pragma unroll
    for (int i = 0; i < K; ++i) r.d[i] = (x.v * y.d[i] - y.v * x.d[i]) * q;
    return r;
}

}  // namespace kfm
