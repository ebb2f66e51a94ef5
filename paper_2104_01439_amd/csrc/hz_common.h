// Device helpers shared by the HIP kernels: complex arithmetic on interleaved pairs,
// compile-time loops and the P_p coupling pattern of the "/"-split lattice.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "hz_internal.h"

namespace hz {

__device__ __forceinline__ void cfma(double2& acc, double2 c, double2 v) {
  acc.x = fma(c.x, v.x, acc.x);
  acc.x = fma(-c.y, v.y, acc.x);
  acc.y = fma(c.x, v.y, acc.y);
  acc.y = fma(c.y, v.x, acc.y);
}
__device__ __forceinline__ void cfma(float2& acc, float2 c, float2 v) {
  acc.x = fmaf(c.x, v.x, acc.x);
  acc.x = fmaf(-c.y, v.y, acc.x);
  acc.y = fmaf(c.x, v.y, acc.y);
  acc.y = fmaf(c.y, v.x, acc.y);
}
// acc += conj(a) * b
__device__ __forceinline__ void cfma_conj(double2& acc, double2 a, double2 b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(-a.y, b.x, acc.y);
}
template <typename T> __device__ __forceinline__ V2<T> cmul(V2<T> a, V2<T> b) {
  V2<T> r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
template <typename T> __device__ __forceinline__ V2<T> csub(V2<T> a, V2<T> b) {
  V2<T> r;
  r.x = a.x - b.x;
  r.y = a.y - b.y;
  return r;
}
template <typename T> __device__ __forceinline__ V2<T> cadd(V2<T> a, V2<T> b) {
  V2<T> r;
  r.x = a.x + b.x;
  r.y = a.y + b.y;
  return r;
}
template <typename T> __device__ __forceinline__ V2<T> czero() {
  V2<T> r;
  r.x = T(0);
  r.y = T(0);
  return r;
}
template <typename T, typename S> __device__ __forceinline__ V2<T> cvt(S v) {
  V2<T> r;
  r.x = T(v.x);
  r.y = T(v.y);
  return r;
}

// Compile-time loop: f(std::integral_constant<int, i>) for i in [B, E).
template <int B, int E, typename F> __device__ __forceinline__ void sfor(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    sfor<B + 1, E>(static_cast<F&&>(f));
  }
}

// Lattice points (a0, b0) and (a1, b1) (lattice spacing h/p) share a closed triangle of the
// mesh whose cells (side p in lattice units) are split by the "/" diagonal:
// T_L = {0 <= y <= x <= p}, T_U = {0 <= x <= y <= p} in cell-local coordinates.
// (a0, b0) is taken in [0, p)^2, so only the cells with ci, cj in {-1, 0} can contain it.
constexpr bool in_tri(int p, int tri, int ci, int cj, int a, int b) {
  const int x = a - p * ci, y = b - p * cj;
  return tri == 0 ? (x <= p && y >= 0 && y <= x) : (x >= 0 && y <= p && x <= y);
}
constexpr bool couples(int p, int a0, int b0, int a1, int b1) {
  for (int cj = -1; cj <= 0; ++cj)
    for (int ci = -1; ci <= 0; ++ci)
      for (int tri = 0; tri < 2; ++tri)
        if (in_tri(p, tri, ci, cj, a0, b0) && in_tri(p, tri, ci, cj, a1, b1)) return true;
  return false;
}

// Wave-level reductions (64 lanes).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

}  // namespace hz
