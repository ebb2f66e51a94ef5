// Arnoldi kernels of the flexible GMRES outer iteration (Sec. 4, after Saad 1993).
//
// Classical Gram-Schmidt applied twice: each pass computes h = V^H w (mdot + reduce) and
// w -= V h (maxpy). Reductions are two-stage with a fixed order (per-workgroup partials,
// then a fixed-order sum), so results are bitwise reproducible and independent of how many
// solves share a launch. The batch index is blockIdx.y; every per-solve array has a stride.

#include "hz_common.h"

namespace hz {

namespace {

constexpr int EPT = 4;                 // elements per thread in the streaming kernels
constexpr int CHUNK = 256 * EPT;       // elements per workgroup
constexpr int MDOT_U = 2;              // basis vectors per step of k_mdot (4: no faster)

template <typename TV>
__global__ void __launch_bounds__(256)
k_mdot(const V2<TV>* __restrict__ V, Addr av, long ldv, int nv, const int* __restrict__ nvt,
       const double2* __restrict__ w, Addr aw, long N, double2* __restrict__ partial, int nblk) {
  __shared__ double red[2][64][4];
  const int bz = blockIdx.y;
  if (nvt) nv = nvt[bz];
  if (nv <= 0) return;
  V += av.at(bz);
  w += aw.at(bz);
  partial += long(bz) * nblk * 64;
  const long base = long(blockIdx.x) * CHUNK + threadIdx.x;
  double2 wv[EPT];
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const long k = base + q * 256;
    wv[q] = k < N ? w[k] : make_double2(0, 0);
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // MDOT_U basis vectors per step: their loads are in flight together
  for (int i0 = 0; i0 < nv; i0 += MDOT_U) {
    V2<TV> va[MDOT_U][EPT];
#pragma unroll
    for (int u = 0; u < MDOT_U; ++u)
#pragma unroll
      for (int q = 0; q < EPT; ++q) {
        const long k = base + q * 256;
        va[u][q] = (i0 + u < nv && k < N) ? V[(i0 + u) * ldv + k] : czero<TV>();
      }
#pragma unroll
    for (int u = 0; u < MDOT_U; ++u) {
      const int i = i0 + u;
      if (i >= nv) break;
      double2 acc = make_double2(0, 0);
#pragma unroll
      for (int q = 0; q < EPT; ++q) {
        const long k = base + q * 256;
        if (k < N) cfma_conj(acc, cvt<double>(va[u][q]), wv[q]);
      }
      acc.x = wave_sum(acc.x);
      acc.y = wave_sum(acc.y);
      if (lane == 0) { red[0][i][wave] = acc.x; red[1][i][wave] = acc.y; }
    }
  }
  __syncthreads();
  if (threadIdx.x < nv) {
    const int i = threadIdx.x;
    double2 s;
    s.x = ((red[0][i][0] + red[0][i][1]) + red[0][i][2]) + red[0][i][3];
    s.y = ((red[1][i][0] + red[1][i][1]) + red[1][i][2]) + red[1][i][3];
    partial[long(blockIdx.x) * 64 + i] = s;
  }
}

// out[i] = sum_b partial[b][i] in a fixed order, in two stages. First stage: workgroup g of
// instance bz sums block rows [g per, (g + 1) per) of every vector i < nv (1024 threads:
// vector t % 64, row lane t / 64 taking every 16th row in ascending order, so a row's
// vectors are read together), then its 16 row lanes in order, into work[bz][g][i].
__global__ void __launch_bounds__(1024)
k_reduce1(const double2* __restrict__ partial, int nblk, int nv, const int* __restrict__ nvt,
          double2* __restrict__ work) {
  __shared__ double sx[16][64], sy[16][64];
  const int bz = blockIdx.y;
  const int nvb = nvt ? nvt[bz] : nv;
  if (nvb <= 0) return;
  const int i = threadIdx.x & 63, rl = threadIdx.x >> 6;
  const int per = (nblk + kReduceGroups - 1) / kReduceGroups;
  const int b0 = blockIdx.x * per, b1 = min(nblk, b0 + per);
  const double2* __restrict__ pp = partial + long(bz) * nblk * 64;
  double ax = 0, ay = 0;
  if (i < nvb) {
#pragma unroll 4
    for (int b = b0 + rl; b < b1; b += 16) {
      const double2 v = pp[long(b) * 64 + i];
      ax += v.x;
      ay += v.y;
    }
  }
  sx[rl][i] = ax;
  sy[rl][i] = ay;
  __syncthreads();
  if (threadIdx.x < 64 && i < nvb) {
    double tx = 0, ty = 0;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      tx += sx[r][i];
      ty += sy[r][i];
    }
    work[(long(bz) * kReduceGroups + blockIdx.x) * 64 + i] = make_double2(tx, ty);
  }
}

// Second stage: out[i] = the kReduceGroups first-stage sums in a fixed order (16 row lanes of
// kReduceGroups / 16 sums each, then the lanes in order).
__global__ void __launch_bounds__(1024)
k_reduce2(const double2* __restrict__ work, int nv, const int* __restrict__ nvt,
          double2* __restrict__ out, long ostride) {
  __shared__ double sx[16][64], sy[16][64];
  const int bz = blockIdx.y;
  const int nvb = nvt ? nvt[bz] : nv;
  if (nvb <= 0) return;
  const int i = threadIdx.x & 63, rl = threadIdx.x >> 6;
  double ax = 0, ay = 0;
  if (i < nvb) {
#pragma unroll
    for (int g = rl; g < kReduceGroups; g += 16) {
      const double2 v = work[(long(bz) * kReduceGroups + g) * 64 + i];
      ax += v.x;
      ay += v.y;
    }
  }
  sx[rl][i] = ax;
  sy[rl][i] = ay;
  __syncthreads();
  if (threadIdx.x < 64 && i < nvb) {
    double tx = 0, ty = 0;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      tx += sx[r][i];
      ty += sy[r][i];
    }
    out[bz * ostride + i] = make_double2(tx, ty);
  }
}

// w -= sum_i V[i] h[i] (ascending i); optionally partial[b][0] = sum |w_new|^2 over the
// workgroup. One element per thread with its column of V (up to NVB basis vectors, NVB a
// multiple of 8 >= the largest basis size of the launch) in registers, every load issued
// before the barrier that stages h.
template <int NVB, bool NORM>
__global__ void __launch_bounds__(256, 1)
k_maxpy(const double2* __restrict__ V, Addr av, long ldv, int nv, const int* __restrict__ nvt,
        const double2* __restrict__ h, long hstride, double2* __restrict__ w, Addr aw, long N,
        double2* __restrict__ partial, int nblk) {
  __shared__ double2 hs[64];
  __shared__ double red[4];
  const int bz = blockIdx.y;
  if (nvt) nv = nvt[bz];
  if (nv <= 0) return;
  V += av.at(bz);
  w += aw.at(bz);
  h += bz * hstride;
  const long k = long(blockIdx.x) * 256 + threadIdx.x;
  const bool in = k < N;
  double2 vv[NVB];
#pragma unroll
  for (int i = 0; i < NVB; ++i) vv[i] = (i < nv && in) ? V[i * ldv + k] : make_double2(0, 0);
  double2 acc = in ? w[k] : make_double2(0, 0);
  if (threadIdx.x < nv) hs[threadIdx.x] = h[threadIdx.x];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NVB; ++i) {
    if (i < nv) {
      const double2 hh = hs[i];
      acc.x -= vv[i].x * hh.x - vv[i].y * hh.y;
      acc.y -= vv[i].x * hh.y + vv[i].y * hh.x;
    }
  }
  if (in) w[k] = acc;
  if (NORM) {
    double nrm = acc.x * acc.x + acc.y * acc.y;
    nrm = wave_sum(nrm);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nrm;
    __syncthreads();
    if (threadIdx.x == 0)
      partial[long(bz) * nblk * 64 + long(blockIdx.x) * 64] =
          make_double2(((red[0] + red[1]) + red[2]) + red[3], 0.0);
  }
}

// The first pass's update and the second pass's projection from one read of V:
// w' = w - V h (the same arithmetic as k_maxpy) and partial[b][i] = sum over the
// workgroup's elements of conj(V[i]) w'. One element per thread: its column of V (up to NVB
// basis vectors) stays in registers between the two. The per-vector sums over the workgroup
// run as DPP sums over rows of 16 lanes, then over the 16 row results in a fixed order.
template <int NVB>
__global__ void __launch_bounds__(256, 1)
k_maxpy_mdot(const double2* __restrict__ V, Addr av, long ldv, int nv, const int* __restrict__ nvt,
             const double2* __restrict__ h, long hstride, double2* __restrict__ w, Addr aw, long N,
             double2* __restrict__ partial, int nblk) {
  __shared__ double2 hs[64];
  __shared__ double red[2][64][16];
  const int bz = blockIdx.y;
  if (nvt) nv = nvt[bz];
  if (nv <= 0) return;
  V += av.at(bz);
  w += aw.at(bz);
  h += bz * hstride;
  partial += long(bz) * nblk * 64;
  if (threadIdx.x < nv) hs[threadIdx.x] = h[threadIdx.x];
  __syncthreads();
  const long k = long(blockIdx.x) * 256 + threadIdx.x;
  const bool in = k < N;
  double2 vv[NVB];
  double2 acc = in ? w[k] : make_double2(0, 0);
#pragma unroll
  for (int i = 0; i < NVB; ++i)
    vv[i] = (i < nv && in) ? V[i * ldv + k] : make_double2(0, 0);
#pragma unroll
  for (int i = 0; i < NVB; ++i) {
    if (i < nv) {
      const double2 hh = hs[i];
      acc.x -= vv[i].x * hh.x - vv[i].y * hh.y;
      acc.y -= vv[i].x * hh.y + vv[i].y * hh.x;
    }
  }
  if (in) w[k] = acc;
  const int row = threadIdx.x >> 4, lane16 = threadIdx.x & 15;
#pragma unroll
  for (int i = 0; i < NVB; ++i) {
    if (i < nv) {
      double2 d = make_double2(0, 0);
      cfma_conj(d, vv[i], acc);
      d.x = row16_sum(d.x);
      d.y = row16_sum(d.y);
      if (lane16 == 0) { red[0][i][row] = d.x; red[1][i][row] = d.y; }
    }
  }
  __syncthreads();
  if (threadIdx.x < nv) {
    const int i = threadIdx.x;
    double2 sm = make_double2(0, 0);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      sm.x += red[0][i][q];
      sm.y += red[1][i][q];
    }
    partial[long(blockIdx.x) * 64 + i] = sm;
  }
}

__global__ void k_scale(const double2* __restrict__ w, Addr aw, const double* __restrict__ s,
                        double2* __restrict__ v, Addr av, long N) {
  const long i = long(blockIdx.x) * 256 + threadIdx.x;
  const int bz = blockIdx.y;
  if (i >= N) return;
  const double a = s[bz];
  const double2 x = w[aw.at(bz) + i];
  v[av.at(bz) + i] = make_double2(a * x.x, a * x.y);
}

template <typename TZ>
__global__ void __launch_bounds__(256)
k_update(const V2<TZ>* __restrict__ Z, Addr az, long ldz, int nz, const int* __restrict__ nzt,
         const double2* __restrict__ y, long ystride, double2* __restrict__ u, Addr au, long N) {
  __shared__ double2 ys[64];
  const int bz = blockIdx.y;
  if (nzt) nz = nzt[bz];
  if (nz <= 0) return;
  Z += az.at(bz);
  y += bz * ystride;
  u += au.at(bz);
  if (threadIdx.x < nz) ys[threadIdx.x] = y[threadIdx.x];
  __syncthreads();
  const long k = long(blockIdx.x) * 256 + threadIdx.x;
  if (k >= N) return;
  double2 acc = u[k];
  for (int i = 0; i < nz; ++i) cfma(acc, cvt<double>(Z[i * ldz + k]), ys[i]);
  u[k] = acc;
}

__global__ void k_scale_arg(const double2* __restrict__ w, double a, double2* __restrict__ v,
                            long N) {
  const long i = long(blockIdx.x) * 256 + threadIdx.x;
  if (i >= N) return;
  const double2 x = w[i];
  v[i] = make_double2(a * x.x, a * x.y);
}

template <typename T> __global__ void k_zero(V2<T>* __restrict__ y, Addr ay, long N) {
  const long i = long(blockIdx.x) * 256 + threadIdx.x;
  if (i < N) y[ay.at(blockIdx.y) + i] = czero<T>();
}

__global__ void k_copy(const double2* __restrict__ x, Addr ax, double2* __restrict__ y, Addr ay,
                       long N) {
  const long i = long(blockIdx.x) * 256 + threadIdx.x;
  if (i < N) y[ay.at(blockIdx.y) + i] = x[ax.at(blockIdx.y) + i];
}

}  // namespace

int mdot_blocks(long N) { return int((N + CHUNK - 1) / CHUNK); }
int fused_blocks(long N) { return int((N + 255) / 256); }

// NVB bucket (a multiple of 8, at least nv) of a launch whose basis sizes are at most nv.
#define HZ_NVB(MACRO)                \
  if (nv <= 8) { MACRO(8); }         \
  else if (nv <= 16) { MACRO(16); }  \
  else if (nv <= 24) { MACRO(24); }  \
  else if (nv <= 32) { MACRO(32); }  \
  else if (nv <= 40) { MACRO(40); }  \
  else if (nv <= 48) { MACRO(48); }  \
  else if (nv <= 56) { MACRO(56); }  \
  else { MACRO(64); }

void launch_maxpy_mdot_b(const double2* V, Addr av, long ldv, int nv, const int* nvt,
                         const double2* h, long hs, double2* w, Addr aw, long N,
                         double2* partial, int nbatch, hipStream_t st) {
  if (nbatch <= 0) return;
  const dim3 g(unsigned(fused_blocks(N)), nbatch);
  const int nb = fused_blocks(N);
#define HZ_MM(B) k_maxpy_mdot<B><<<g, 256, 0, st>>>(V, av, ldv, nv, nvt, h, hs, w, aw, N, partial, nb)
  HZ_NVB(HZ_MM)
#undef HZ_MM
  HZ_HIP(hipGetLastError());
}

void launch_mdot_b(const double2* V, Addr av, long ldv, int nv, const int* nvt, const double2* w,
                   Addr aw, long N, double2* partial, int nblk, int nbatch, hipStream_t st) {
  if (nbatch <= 0) return;
  k_mdot<double><<<dim3(nblk, nbatch), 256, 0, st>>>(V, av, ldv, nv, nvt, w, aw, N, partial, nblk);
  HZ_HIP(hipGetLastError());
}

void launch_reduce_b(const double2* partial, int nblk, int nv, const int* nvt, double2* out,
                     long hs, int nbatch, double2* work, hipStream_t st) {
  if (nbatch <= 0 || nv <= 0) return;
  k_reduce1<<<dim3(kReduceGroups, nbatch), 1024, 0, st>>>(partial, nblk, nv, nvt, work);
  k_reduce2<<<dim3(1, nbatch), 1024, 0, st>>>(work, nv, nvt, out, hs);
  HZ_HIP(hipGetLastError());
}

void launch_maxpy_b(const double2* V, Addr av, long ldv, int nv, const int* nvt, const double2* h,
                    long hs, double2* w, Addr aw, long N, double2* norm_partial, int nbatch,
                    hipStream_t st) {
  if (nbatch <= 0) return;
  const int nb = fused_blocks(N);
  const dim3 g(unsigned(nb), nbatch);
#define HZ_MX(B)                                                                                \
  if (norm_partial)                                                                             \
    k_maxpy<B, true><<<g, 256, 0, st>>>(V, av, ldv, nv, nvt, h, hs, w, aw, N, norm_partial, nb); \
  else                                                                                          \
    k_maxpy<B, false><<<g, 256, 0, st>>>(V, av, ldv, nv, nvt, h, hs, w, aw, N, nullptr, nb);
  HZ_NVB(HZ_MX)
#undef HZ_MX
  HZ_HIP(hipGetLastError());
}

template <typename TZ>
void launch_update(const V2<TZ>* Z, long ldz, int nz, const double2* y, double2* u, long N,
                   hipStream_t st) {
  launch_update_b<TZ>(Z, Addr(), ldz, nz, nullptr, y, 0, u, Addr(), N, 1, st);
}
template void launch_update<double>(const double2*, long, int, const double2*, double2*, long,
                                    hipStream_t);
template void launch_update<float>(const float2*, long, int, const double2*, double2*, long,
                                   hipStream_t);

template <typename TZ>
void launch_update_b(const V2<TZ>* Z, Addr az, long ldz, int nz, const int* nzt, const double2* y,
                     long ys, double2* u, Addr au, long N, int nbatch, hipStream_t st) {
  if (nbatch <= 0) return;
  k_update<TZ><<<dim3(unsigned((N + 255) / 256), nbatch), 256, 0, st>>>(Z, az, ldz, nz, nzt, y, ys,
                                                                        u, au, N);
  HZ_HIP(hipGetLastError());
}
template void launch_update_b<double>(const double2*, Addr, long, int, const int*, const double2*,
                                      long, double2*, Addr, long, int, hipStream_t);
template void launch_update_b<float>(const float2*, Addr, long, int, const int*, const double2*,
                                     long, double2*, Addr, long, int, hipStream_t);

void launch_axpby_copy(const double2* x, double2* y, long N, hipStream_t st) {
  launch_copy_b(x, Addr(), y, Addr(), N, 1, st);
}

void launch_copy_b(const double2* x, Addr ax, double2* y, Addr ay, long N, int nbatch,
                   hipStream_t st) {
  if (N <= 0 || nbatch <= 0) return;
  k_copy<<<dim3(unsigned((N + 255) / 256), nbatch), 256, 0, st>>>(x, ax, y, ay, N);
  HZ_HIP(hipGetLastError());
}

// Scaling factor lives on the device (s_dev[0]) so that no host round trip is needed.
void launch_scale_dev(const double2* w, const double* s_dev, double2* v, long N, hipStream_t st) {
  launch_scale_b(w, Addr(), s_dev, v, Addr(), N, 1, st);
}

void launch_scale_b(const double2* w, Addr aw, const double* s_dev, double2* v, Addr av, long N,
                    int nbatch, hipStream_t st) {
  if (nbatch <= 0) return;
  k_scale<<<dim3(unsigned((N + 255) / 256), nbatch), 256, 0, st>>>(w, aw, s_dev, v, av, N);
  HZ_HIP(hipGetLastError());
}

void launch_scale(const double2* w, double s, double2* v, long N, hipStream_t st) {
  k_scale_arg<<<unsigned((N + 255) / 256), 256, 0, st>>>(w, s, v, N);
  HZ_HIP(hipGetLastError());
}

void launch_fill_zero(double2* y, long N, hipStream_t st) {
  if (N <= 0) return;
  k_zero<double><<<unsigned((N + 255) / 256), 256, 0, st>>>(y, Addr(), N);
  HZ_HIP(hipGetLastError());
}
void launch_fill_zero(float2* y, long N, hipStream_t st) {
  if (N <= 0) return;
  k_zero<float><<<unsigned((N + 255) / 256), 256, 0, st>>>(y, Addr(), N);
  HZ_HIP(hipGetLastError());
}
void launch_fill_zero_b(double2* y, Addr ay, long N, int nbatch, hipStream_t st) {
  if (N <= 0 || nbatch <= 0) return;
  k_zero<double><<<dim3(unsigned((N + 255) / 256), nbatch), 256, 0, st>>>(y, ay, N);
  HZ_HIP(hipGetLastError());
}

}  // namespace hz
