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

// Sum over each row of 16 lanes (every lane of the row gets it): a butterfly of lane
// permutations within the row (mirror, half mirror, then the two quad exchanges), each step
// moving the two 32-bit halves of a value with DPP.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, int(bits), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, int(bits >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <typename T>
__device__ __forceinline__ T row16_sum(T v) {
  v += dpp_move<0x140>(v);   // row_mirror: lane i <- 15 - i
  v += dpp_move<0x141>(v);   // row_half_mirror: lane i <- 7 - i within each half row
  v += dpp_move<0x4E>(v);    // quad_perm [2, 3, 0, 1]
  v += dpp_move<0xB1>(v);    // quad_perm [1, 0, 3, 2]
  return v;
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
