// Shared device helpers of the DSBlockCG HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dsbcg {

// Complex number stored as two reals; 8-byte (float) or 16-byte (double)
// aligned so that one element is one vector load.
template <typename R>
struct alignas(2 * sizeof(R)) cx {
    R x, y;
};

template <typename R>
__device__ __host__ inline cx<R> mk(R a, R b) { return cx<R>{a, b}; }

template <typename R>
__device__ inline cx<R> operator+(cx<R> a, cx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ inline cx<R> operator-(cx<R> a, cx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__device__ inline cx<R> operator-(cx<R> a) { return {-a.x, -a.y}; }
template <typename R>
__device__ inline cx<R> operator*(cx<R> a, cx<R> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename R>
__device__ inline cx<R> operator*(R s, cx<R> a) { return {s * a.x, s * a.y}; }
template <typename R>
__device__ inline cx<R> conj(cx<R> a) { return {a.x, -a.y}; }
// i * a
template <typename R>
__device__ inline cx<R> mul_i(cx<R> a) { return {-a.y, a.x}; }
// acc += a * b
template <typename R>
__device__ inline void cmac(cx<R> &acc, cx<R> a, cx<R> b) {
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(a.y, b.x, acc.y);
}
// acc += conj(a) * b
template <typename R>
__device__ inline void cmac_conj(cx<R> &acc, cx<R> a, cx<R> b) {
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(-a.y, b.x, acc.y);
}
template <typename R>
__device__ inline R norm2(cx<R> a) { return a.x * a.x + a.y * a.y; }

template <typename To, typename From>
__device__ inline cx<To> cvt(cx<From> a) { return {static_cast<To>(a.x), static_cast<To>(a.y)}; }

typedef cx<double> zd;
typedef cx<float> zf;

}  // namespace dsbcg
