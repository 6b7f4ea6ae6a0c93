// Complex arithmetic for the device code (FP64 and FP32 storage types).
#pragma once
#include <hip/hip_runtime.h>

template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T re, im;
};

template <typename T>
__host__ __device__ __forceinline__ cx<T> mk(T a, T b) {
  cx<T> r;
  r.re = a;
  r.im = b;
  return r;
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return mk(a.re + b.re, a.im + b.im); }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return mk(a.re - b.re, a.im - b.im); }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator-(cx<T> a) { return mk(-a.re, -a.im); }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
  return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return mk(s * a.re, s * a.im); }
// conj(a) * b
template <typename T>
__host__ __device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return mk(a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re);
}
// i * a
template <typename T>
__host__ __device__ __forceinline__ cx<T> mul_i(cx<T> a) { return mk(-a.im, a.re); }
// -i * a
template <typename T>
__host__ __device__ __forceinline__ cx<T> mul_mi(cx<T> a) { return mk(a.im, -a.re); }
template <typename T>
__host__ __device__ __forceinline__ T abs2(cx<T> a) { return a.re * a.re + a.im * a.im; }
// a / b
template <typename T>
__host__ __device__ __forceinline__ cx<T> cdiv(cx<T> a, cx<T> b) {
  T d = b.re * b.re + b.im * b.im;
  return mk((a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d);
}
template <typename Tout, typename Tin>
__host__ __device__ __forceinline__ cx<Tout> cvt(cx<Tin> a) {
  return mk((Tout)a.re, (Tout)a.im);
}

using c128 = cx<double>;
using c64 = cx<float>;
