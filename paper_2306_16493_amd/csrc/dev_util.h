// Small device-side helpers shared by the rate kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace eph {

template <class T>
struct V2;
template <>
struct V2<double> {
  using t = double2;
};
template <>
struct V2<float> {
  using t = float2;
};

template <class T>
__device__ __forceinline__ typename V2<T>::t mk(T x, T y) {
  typename V2<T>::t r;
  r.x = x;
  r.y = y;
  return r;
}

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

// (a mod N) for |a| < 2^31, result in [0, N)
__device__ __forceinline__ int imod(int a, int N) {
  int r = a % N;
  return r < 0 ? r + N : r;
}

// (r, i) += a * b with four fused multiply-adds
template <class T>
__device__ __forceinline__ void cmac(T &r, T &i, T ar, T ai, T br, T bi) {
  r = fma(ar, br, r);
  r = fma(-ai, bi, r);
  i = fma(ar, bi, i);
  i = fma(ai, br, i);
}
// (r, i) += conj(a) * b
template <class T>
__device__ __forceinline__ void cmac_conj(T &r, T &i, T ar, T ai, T br, T bi) {
  r = fma(ar, br, r);
  r = fma(ai, bi, r);
  i = fma(ar, bi, i);
  i = fma(-ai, br, i);
}

}  // namespace eph
