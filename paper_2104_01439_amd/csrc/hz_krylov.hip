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

template <typename TV>
__global__ void __launch_bounds__(256)
k_mdot(const V2<TV>* __restrict__ V, long ldv, int nv, const double2* __restrict__ w, long N,
       double2* __restrict__ partial, int nblk, long vstride, long wstride) {
  __shared__ double red[2][64][4];
  const long bo = blockIdx.y;
  V += bo * vstride;
  w += bo * wstride;
  partial += bo * long(nblk) * 64;
  const long base = long(blockIdx.x) * CHUNK + threadIdx.x;
  double2 wv[EPT];
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const long k = base + q * 256;
    wv[q] = k < N ? w[k] : make_double2(0, 0);
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int i = 0; i < nv; ++i) {
    const V2<TV>* vi = V + i * ldv;
    double2 acc = make_double2(0, 0);
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const long k = base + q * 256;
      if (k < N) cfma_conj(acc, cvt<double>(vi[k]), wv[q]);
    }
    acc.x = wave_sum(acc.x);
    acc.y = wave_sum(acc.y);
    if (lane == 0) { red[0][i][wave] = acc.x; red[1][i][wave] = acc.y; }
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

// out[i] = sum_b partial[b][i] in a fixed order; one workgroup per i.
__global__ void __launch_bounds__(256)
k_reduce(const double2* __restrict__ partial, int nblk, int nv, double2* __restrict__ out,
         long ostride) {
  __shared__ double sx[256], sy[256];
  const int i = blockIdx.x;
  const long bo = blockIdx.y;
  partial += bo * long(nblk) * 64;
  double ax = 0, ay = 0;
  for (int b = threadIdx.x; b < nblk; b += 256) {
    const double2 v = partial[long(b) * 64 + i];
    ax += v.x;
    ay += v.y;
  }
  sx[threadIdx.x] = ax;
  sy[threadIdx.x] = ay;
  __syncthreads();
  for (int s = 128; s >= 1; s >>= 1) {
    if (threadIdx.x < s) {
      sx[threadIdx.x] += sx[threadIdx.x + s];
      sy[threadIdx.x] += sy[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[bo * ostride + i] = make_double2(sx[0], sy[0]);
}

// w -= sum_i V[i] h[i]; optionally partial[blk][0] = sum |w_new|^2 over the chunk.
template <bool NORM>
__global__ void __launch_bounds__(256)
k_maxpy(const double2* __restrict__ V, long ldv, int nv, const double2* __restrict__ h,
        double2* __restrict__ w, long N, double2* __restrict__ partial, int nblk, long vstride,
        long wstride, long hstride) {
  __shared__ double2 hs[64];
  __shared__ double red[4];
  const long bo = blockIdx.y;
  V += bo * vstride;
  w += bo * wstride;
  h += bo * hstride;
  if (threadIdx.x < nv) hs[threadIdx.x] = h[threadIdx.x];
  __syncthreads();
  const long base = long(blockIdx.x) * CHUNK + threadIdx.x;
  double nrm = 0;
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const long k = base + q * 256;
    if (k >= N) continue;
    double2 acc = w[k];
    for (int i = 0; i < nv; ++i) {
      const double2 v = V[i * ldv + k];
      const double2 hh = hs[i];
      acc.x -= v.x * hh.x - v.y * hh.y;
      acc.y -= v.x * hh.y + v.y * hh.x;
    }
    w[k] = acc;
    if (NORM) nrm += acc.x * acc.x + acc.y * acc.y;
  }
  if (NORM) {
    nrm = wave_sum(nrm);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nrm;
    __syncthreads();
    if (threadIdx.x == 0)
      partial[bo * long(nblk) * 64 + long(blockIdx.x) * 64] =
          make_double2(((red[0] + red[1]) + red[2]) + red[3], 0.0);
  }
}

__global__ void k_scale(const double2* __restrict__ w, const double* __restrict__ s,
                        double2* __restrict__ v, long N, long wstride, long vstride) {
  const long i = long(blockIdx.x) * 256 + threadIdx.x;
  const long bo = blockIdx.y;
  if (i >= N) return;
  const double a = s[bo];
  const double2 x = w[bo * wstride + i];
  v[bo * vstride + i] = make_double2(a * x.x, a * x.y);
}

template <typename TZ>
__global__ void __launch_bounds__(256)
k_update(const V2<TZ>* __restrict__ Z, long ldz, int nz, const double2* __restrict__ y,
         double2* __restrict__ u, long N, long zstride, long ystride, long ustride) {
  __shared__ double2 ys[64];
  const long bo = blockIdx.y;
  Z += bo * zstride;
  y += bo * ystride;
  u += bo * ustride;
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

template <typename T> __global__ void k_zero(V2<T>* __restrict__ y, long N) {
  const long i = long(blockIdx.x) * 256 + threadIdx.x;
  if (i < N) y[i] = czero<T>();
}

__global__ void k_copy(const double2* __restrict__ x, double2* __restrict__ y, long N) {
  const long i = long(blockIdx.x) * 256 + threadIdx.x;
  if (i < N) y[i] = x[i];
}

}  // namespace

int mdot_blocks(long N) { return int((N + CHUNK - 1) / CHUNK); }

template <typename TV>
void launch_mdot(const V2<TV>* V, long ldv, int nv, const double2* w, long N, double2* partial,
                 int nblk, hipStream_t st) {
  k_mdot<TV><<<dim3(nblk, 1), 256, 0, st>>>(V, ldv, nv, w, N, partial, nblk, 0, 0);
  HZ_HIP(hipGetLastError());
}
template void launch_mdot<double>(const double2*, long, int, const double2*, long, double2*, int,
                                  hipStream_t);
template void launch_mdot<float>(const float2*, long, int, const double2*, long, double2*, int,
                                 hipStream_t);

void launch_reduce(const double2* partial, int nblk, int nv, double2* out, hipStream_t st) {
  k_reduce<<<dim3(nv, 1), 256, 0, st>>>(partial, nblk, nv, out, 0);
  HZ_HIP(hipGetLastError());
}

void launch_maxpy(const double2* V, long ldv, int nv, const double2* h, double2* w, long N,
                  double2* norm_partial, int nblk, hipStream_t st) {
  if (norm_partial)
    k_maxpy<true><<<dim3(nblk, 1), 256, 0, st>>>(V, ldv, nv, h, w, N, norm_partial, nblk, 0, 0, 0);
  else
    k_maxpy<false><<<dim3(nblk, 1), 256, 0, st>>>(V, ldv, nv, h, w, N, nullptr, nblk, 0, 0, 0);
  HZ_HIP(hipGetLastError());
}

template <typename TZ>
void launch_update(const V2<TZ>* Z, long ldz, int nz, const double2* y, double2* u, long N,
                   hipStream_t st) {
  k_update<TZ><<<dim3(unsigned((N + 255) / 256), 1), 256, 0, st>>>(Z, ldz, nz, y, u, N, 0, 0, 0);
  HZ_HIP(hipGetLastError());
}
template void launch_update<double>(const double2*, long, int, const double2*, double2*, long,
                                    hipStream_t);
template void launch_update<float>(const float2*, long, int, const double2*, double2*, long,
                                   hipStream_t);

void launch_axpby_copy(const double2* x, double2* y, long N, hipStream_t st) {
  k_copy<<<unsigned((N + 255) / 256), 256, 0, st>>>(x, y, N);
  HZ_HIP(hipGetLastError());
}

// Scaling factor lives on the device (s_dev[0]) so that no host round trip is needed.
void launch_scale_dev(const double2* w, const double* s_dev, double2* v, long N, hipStream_t st) {
  k_scale<<<dim3(unsigned((N + 255) / 256), 1), 256, 0, st>>>(w, s_dev, v, N, 0, 0);
  HZ_HIP(hipGetLastError());
}

void launch_scale(const double2* w, double s, double2* v, long N, hipStream_t st) {
  k_scale_arg<<<unsigned((N + 255) / 256), 256, 0, st>>>(w, s, v, N);
  HZ_HIP(hipGetLastError());
}

void launch_fill_zero(double2* y, long N, hipStream_t st) {
  if (N <= 0) return;
  k_zero<double><<<unsigned((N + 255) / 256), 256, 0, st>>>(y, N);
  HZ_HIP(hipGetLastError());
}
void launch_fill_zero(float2* y, long N, hipStream_t st) {
  if (N <= 0) return;
  k_zero<float><<<unsigned((N + 255) / 256), 256, 0, st>>>(y, N);
  HZ_HIP(hipGetLastError());
}

}  // namespace hz
