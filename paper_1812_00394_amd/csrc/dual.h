// Forward-mode dual numbers for the local Jacobians of the adjoint: value plus K directional
// derivatives.  Only the operations the step's cell-local algebra uses are provided; comparisons
// (max / min / branch tests) look at the value, so a derivative is that of the branch taken.
#pragma once

#include <hip/hip_runtime.h>

namespace fvlbm {

template <typename T, int K>
struct Dual {
    T v;
    T d[K];
    __device__ __forceinline__ Dual() : v(0) {
#pragma unroll
        for (int i = 0; i < K; ++i) d[i] = T(0);
    }
    __device__ __forceinline__ Dual(T x) : v(x) {
#pragma unroll
        for (int i = 0; i < K; ++i) d[i] = T(0);
    }
    // independent variable number i
    __device__ __forceinline__ static Dual var(T x, int i) {
        Dual r(x);
#pragma unroll
        for (int j = 0; j < K; ++j) r.d[j] = (j == i) ? T(1) : T(0);
        return r;
    }
};

template <typename T, int K>
__device__ __forceinline__ Dual<T, K> operator+(const Dual<T, K> &a, const Dual<T, K> &b) {
    Dual<T, K> r;
    r.v = a.v + b.v;
#pragma unroll
    for (int i = 0; i < K; ++i) r.d[i] = a.d[i] + b.d[i];
    return r;
}
template <typename T, int K>
__device__ __forceinline__ Dual<T, K> operator-(const Dual<T, K> &a, const Dual<T, K> &b) {
    Dual<T, K> r;
    r.v = a.v - b.v;
#pragma unroll
    for (int i = 0; i < K; ++i) r.d[i] = a.d[i] - b.d[i];
    return r;
}
template <typename T, int K>
__device__ __forceinline__ Dual<T, K> operator-(const Dual<T, K> &a) {
    Dual<T, K> r;
    r.v = -a.v;
#pragma unroll
    for (int i = 0; i < K; ++i) r.d[i] = -a.d[i];
    return r;
}
template <typename T, int K>
__device__ __forceinline__ Dual<T, K> operator*(const Dual<T, K> &a, const Dual<T, K> &b) {
    Dual<T, K> r;
    r.v = a.v * b.v;
#pragma unroll
    for (int i = 0; i < K; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
    return r;
}
template <typename T, int K>
__device__ __forceinline__ Dual<T, K> operator/(const Dual<T, K> &a, const Dual<T, K> &b) {
    Dual<T, K> r;
    const T ib = T(1) / b.v;
    r.v = a.v * ib;
#pragma unroll
    for (int i = 0; i < K; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) * ib;
    return r;
}
template <typename T, int K>
__device__ __forceinline__ Dual<T, K> operator+(const Dual<T, K> &a, T b) { return a + Dual<T, K>(b); }
template <typename T, int K>
__device__ __forceinline__ Dual<T, K> operator+(T a, const Dual<T, K> &b) { return Dual<T, K>(a) + b; }
template <typename T, int K>
__device__ __forceinline__ Dual<T, K> operator-(const Dual<T, K> &a, T b) { return a - Dual<T, K>(b); }
template <typename T, int K>
__device__ __forceinline__ Dual<T, K> operator-(T a, const Dual<T, K> &b) { return Dual<T, K>(a) - b; }
template <typename T, int K>
__device__ __forceinline__ Dual<T, K> operator*(const Dual<T, K> &a, T b) {
    Dual<T, K> r;
    r.v = a.v * b;
#pragma unroll
    for (int i = 0; i < K; ++i) r.d[i] = a.d[i] * b;
    return r;
}
template <typename T, int K>
__device__ __forceinline__ Dual<T, K> operator*(T a, const Dual<T, K> &b) { return b * a; }
template <typename T, int K>
__device__ __forceinline__ Dual<T, K> operator/(const Dual<T, K> &a, T b) { return a * (T(1) / b); }
template <typename T, int K>
__device__ __forceinline__ Dual<T, K> operator/(T a, const Dual<T, K> &b) { return Dual<T, K>(a) / b; }

template <typename T, int K>
__device__ __forceinline__ Dual<T, K> dsqrt(const Dual<T, K> &a) {
    Dual<T, K> r;
    r.v = sqrt(a.v);
    const T h = r.v > T(0) ? T(0.5) / r.v : T(0);
#pragma unroll
    for (int i = 0; i < K; ++i) r.d[i] = a.d[i] * h;
    return r;
}
// tanh' = sech^2 = 1 / cosh^2, evaluated directly: 1 - tanh^2 would keep rounding noise of a value
// just below 1 at saturation, where the exact derivative vanishes (cosh overflows to inf -> 0).
template <typename T, int K>
__device__ __forceinline__ Dual<T, K> dtanh(const Dual<T, K> &a) {
    Dual<T, K> r;
    r.v = tanh(a.v);
    const T ch = cosh(a.v);
    const T h = T(1) / (ch * ch);
#pragma unroll
    for (int i = 0; i < K; ++i) r.d[i] = a.d[i] * h;
    return r;
}
// max / min by value (first argument on ties, as the forward kernels' a >= b ? a : b)
template <typename T, int K>
__device__ __forceinline__ Dual<T, K> dmax(const Dual<T, K> &a, const Dual<T, K> &b) { return a.v >= b.v ? a : b; }
template <typename T, int K>
__device__ __forceinline__ Dual<T, K> dmin(const Dual<T, K> &a, const Dual<T, K> &b) { return a.v <= b.v ? a : b; }

}  // namespace fvlbm
