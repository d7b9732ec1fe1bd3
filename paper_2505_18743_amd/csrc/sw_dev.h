// Device helpers shared by the element and face kernels.
#pragma once
#include "sw_internal.h"

namespace swk {

// Butterfly reductions over groups of P consecutive lanes (P a power of two);
// every lane of the group receives the result.
template <int P>
__device__ __forceinline__ double gsum(double v) {
#pragma unroll
  for (int m = P / 2; m >= 1; m >>= 1) v += __shfl_xor(v, m);
  return v;
}
template <int P>
__device__ __forceinline__ double gmin(double v) {
#pragma unroll
  for (int m = P / 2; m >= 1; m >>= 1) v = fmin(v, __shfl_xor(v, m));
  return v;
}
template <int P>
__device__ __forceinline__ int gand(int v) {
#pragma unroll
  for (int m = P / 2; m >= 1; m >>= 1) v &= __shfl_xor(v, m);
  return v;
}
template <int P>
__device__ __forceinline__ int gor(int v) {
#pragma unroll
  for (int m = P / 2; m >= 1; m >>= 1) v |= __shfl_xor(v, m);
  return v;
}

// 1/h_des of the desingularised velocity (eq:velocity)
__device__ __forceinline__ double inv_des(double h, double eps) {
  const double h4 = (h * h) * (h * h);
  const double e4 = (eps * eps) * (eps * eps);
  return 1.4142135623730951 * h / sqrt(fmax(h4, e4) + h4);
}

}  // namespace swk
