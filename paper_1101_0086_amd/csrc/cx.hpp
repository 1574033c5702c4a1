// Complex arithmetic on interleaved (re, im) pairs for device code.
#pragma once

#include <hip/hip_runtime.h>

namespace mpa {

template <typename T>
struct __align__(2 * sizeof(T)) cx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> mk(T re, T im) { return cx<T>{re, im}; }

template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }

template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }

template <typename T>
__device__ __forceinline__ cx<T> scale(cx<T> a, T s) { return {a.re * s, a.im * s}; }

// Products are written with explicit fused multiply-adds, so that which
// product of a sum is fused is fixed by the source rather than chosen by the
// compiler per call site: the same operation then rounds the same way in
// every kernel that uses it (the fused and node-parallel schedules rely on
// this to produce the same field).

// a * b
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return {fma(a.re, b.re, -(a.im * b.im)), fma(a.re, b.im, a.im * b.re)};
}

// a * conj(b)
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
    return {fma(a.re, b.re, a.im * b.im), fma(a.im, b.re, -(a.re * b.im))};
}

// multiply by +i (SIGN = +1) or -i (SIGN = -1)
template <int SIGN, typename T>
__device__ __forceinline__ cx<T> rot(cx<T> a) {
    if constexpr (SIGN > 0) return {-a.im, a.re};
    else return {a.im, -a.re};
}

template <typename T>
__device__ __forceinline__ T norm2(cx<T> a) { return fma(a.re, a.re, a.im * a.im); }

}  // namespace mpa
