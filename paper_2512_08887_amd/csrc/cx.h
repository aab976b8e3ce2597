// Minimal complex arithmetic for host and device code (float and double).
// Interleaved (re, im), 8- or 16-byte aligned, layout-compatible with
// torch.complex64 / complex128 and std::complex.
#pragma once

#include <hip/hip_runtime.h>

namespace fbst {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T re, im;
};

using c32 = cx<float>;
using c64 = cx<double>;

template <typename T>
__host__ __device__ __forceinline__ cx<T> mk(T r, T i) { return cx<T>{r, i}; }

template <typename T>
__host__ __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator*(cx<T> a, T s) { return {a.re * s, a.im * s}; }

// a * b
template <typename T>
__host__ __device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a * b + c with one rounding
__host__ __device__ __forceinline__ float fmx(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__host__ __device__ __forceinline__ double fmx(double a, double b, double c) { return __builtin_fma(a, b, c); }
// a * conj(b)
template <typename T>
__host__ __device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
// a * b when DIR < 0, a * conj(b) when DIR > 0 (twiddles stored for the forward sign)
template <int DIR, typename T>
__host__ __device__ __forceinline__ cx<T> cmul_dir(cx<T> a, cx<T> b) {
  if constexpr (DIR < 0) return cmul(a, b);
  else return cmulc(a, b);
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> conjg(cx<T> a) { return {a.re, -a.im}; }

// multiply by -j (DIR < 0) or +j (DIR > 0): exp(DIR * j pi / 2)
template <int DIR, typename T>
__host__ __device__ __forceinline__ cx<T> rot90(cx<T> a) {
  if constexpr (DIR < 0) return {a.im, -a.re};
  else return {-a.im, a.re};
}

template <typename TO, typename TI>
__host__ __device__ __forceinline__ cx<TO> cvt(cx<TI> a) { return {static_cast<TO>(a.re), static_cast<TO>(a.im)}; }

}  // namespace fbst
