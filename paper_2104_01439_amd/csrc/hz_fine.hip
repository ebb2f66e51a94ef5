// Matrix-free lattice kernels of the twogrid method (Sec. 4, Algorithm 1; the fine level
// applies A_0 and A_eps without a stored matrix).
//
// Layout: a level vector holds M*M complex values, point (a, b) at index b*M + a.
// Work decomposition: one thread owns a "macro point", the p x p block of lattice points
// (p I + ca, p J + cb), ca, cb in [0, p), so that every lane of a wavefront applies the same
// p*p class stencils. The stencil coefficients are then wave-uniform (scalar loads) and the
// couplings that are structurally zero are removed at compile time. A workgroup stages its
// tile of the input, with a halo of p lattice points, in LDS with coalesced loads.

#include "hz_common.h"

namespace hz {

namespace {

constexpr int BX = 64;   // macro points per tile along x (one wavefront)
constexpr int BY = 4;    // macro rows per tile

__device__ __forceinline__ int region(int a, int M) { return a == 0 ? 0 : (a == M - 1 ? 2 : 1); }

template <int P, typename T, typename TX, typename TF, typename TY, int MODE>
__global__ void __launch_bounds__(256)
k_stencil(DevOp<T> op, const V2<TX>* __restrict__ x, Addr ax, const V2<TF>* __restrict__ f,
          Addr af, V2<TY>* __restrict__ y, Addr ay) {
  constexpr int W = 2 * P + 1, W2 = W * W;
  constexpr int LW = P * BX + 2 * P, LH = P * BY + 2 * P;
  __shared__ V2<T> tile[LH][LW];
  const int M = op.M;
  const int nmac = (M + P - 1) / P;
  const int bz = blockIdx.z;
  const V2<T>* __restrict__ coef = op.ctab ? op.ctab[bz] : op.coef;
  const V2<T>* __restrict__ wdinv = op.wtab ? op.wtab[bz] : op.wdinv;
  x += ax.at(bz);
  y += ay.at(bz);
  if (MODE != ST_APPLY) f += af.at(bz);
  const int I0 = blockIdx.x * BX, J0 = blockIdx.y * BY;
  const int ax0 = P * I0 - P, by0 = P * J0 - P;
  for (int idx = threadIdx.x; idx < LW * LH; idx += 256) {
    const int ly = idx / LW, lx = idx - ly * LW;
    const int a = ax0 + lx, b = by0 + ly;
    V2<T> v = czero<T>();
    if (a >= 0 && a < M && b >= 0 && b < M) v = cvt<T>(x[long(b) * M + a]);
    tile[ly][lx] = v;
  }
  __syncthreads();
  const int tx = threadIdx.x % BX, ty = threadIdx.x / BX;
  const int I = I0 + tx, J = J0 + ty;
  if (I >= nmac || J >= nmac) return;

  V2<T> acc[P][P];
#pragma unroll
  for (int i = 0; i < P; ++i)
#pragma unroll
    for (int j = 0; j < P; ++j) acc[i][j] = czero<T>();

  int reg[P][P];
#pragma unroll
  for (int cb = 0; cb < P; ++cb)
#pragma unroll
    for (int ca = 0; ca < P; ++ca) reg[cb][ca] = region(P * J + cb, M) * 3 + region(P * I + ca, M);

  const bool inner = I >= 1 && J >= 1 && P * I + P <= M - 1 && P * J + P <= M - 1;

  auto body = [&](auto uniform_tag) {
    constexpr bool UNIFORM = decltype(uniform_tag)::value;
    sfor<0, 3 * P>([&](auto wr_) {
      constexpr int wr = decltype(wr_)::value;  // lattice row P*J - P + wr
      V2<T> row[3 * P];
#pragma unroll
      for (int c = 0; c < 3 * P; ++c) row[c] = tile[P * ty + wr][P * tx + c];
      sfor<0, P>([&](auto cb_) {
        constexpr int cb = decltype(cb_)::value;
        constexpr int dy = wr - P - cb;
        if constexpr (dy >= -P && dy <= P) {
          sfor<0, P>([&](auto ca_) {
            constexpr int ca = decltype(ca_)::value;
            sfor<-P, P + 1>([&](auto dx_) {
              constexpr int dx = decltype(dx_)::value;
              if constexpr (couples(P, ca, cb, ca + dx, cb + dy)) {
                constexpr int off = (dy + P) * W + (dx + P);
                constexpr int cls = cb * P + ca;
                V2<T> c;
                if constexpr (UNIFORM) c = coef[(cls * 9 + 4) * W2 + off];
                else c = coef[(cls * 9 + reg[cb][ca]) * W2 + off];
                cfma(acc[cb][ca], c, row[P + ca + dx]);
              }
            });
          });
        }
      });
    });
  };
  if (__all(inner)) body(std::integral_constant<bool, true>{});
  else body(std::integral_constant<bool, false>{});

#pragma unroll
  for (int cb = 0; cb < P; ++cb) {
    const int b = P * J + cb;
#pragma unroll
    for (int ca = 0; ca < P; ++ca) {
      const int a = P * I + ca;
      if (a >= M || b >= M) continue;
      const long gi = long(b) * M + a;
      V2<T> out = acc[cb][ca];
      if constexpr (MODE == ST_RESID) {
        out = csub<T>(cvt<T>(f[gi]), out);
      } else if constexpr (MODE == ST_SMOOTH) {
        const V2<T> d = wdinv[(cb * P + ca) * 9 + reg[cb][ca]];
        const V2<T> rr = csub<T>(cvt<T>(f[gi]), out);
        out = cadd<T>(tile[P * ty + P + cb][P * tx + P + ca], cmul<T>(d, rr));
      }
      y[gi] = cvt<TY>(out);
    }
  }
}

template <int P, typename T, typename TF>
__global__ void __launch_bounds__(256)
k_jacobi0(DevOp<T> op, const V2<TF>* __restrict__ f, Addr af, V2<T>* __restrict__ y, Addr ay) {
  const int M = op.M;
  const long N = long(M) * M;
  const long i = long(blockIdx.x) * 256 + threadIdx.x;
  if (i >= N) return;
  const int bz = blockIdx.y;
  const int b = int(i / M), a = int(i - long(b) * M);
  const int cls = (b % P) * P + (a % P);
  const int reg = region(b, M) * 3 + region(a, M);
  const V2<T>* wd = op.wtab ? op.wtab[bz] : op.wdinv;
  y[ay.at(bz) + i] = cmul<T>(wd[cls * 9 + reg], cvt<T>(f[af.at(bz) + i]));
}

// yc(A, B) = sum over fine points (2A + dx, 2B + dy) of RW[cls(A,B)][dy][dx] r(...)
template <int P, typename T>
__global__ void __launch_bounds__(256)
k_restrict(int Mf, int Mc, const T* __restrict__ rw, const V2<T>* __restrict__ r,
           V2<T>* __restrict__ yc, Addr af, Addr ac) {
  constexpr int WR = 4 * P + 1;
  const long Nc = long(Mc) * Mc;
  const long i = long(blockIdx.x) * 256 + threadIdx.x;
  if (i >= Nc) return;
  r += af.at(blockIdx.y);
  yc += ac.at(blockIdx.y);
  const int B = int(i / Mc), A = int(i - long(B) * Mc);
  const int cls = (B % P) * P + (A % P);
  const T* w = rw + cls * WR * WR;
  V2<T> acc = czero<T>();
#pragma unroll
  for (int dy = -2 * P; dy <= 2 * P; ++dy) {
    const int b = 2 * B + dy;
    if (b < 0 || b >= Mf) continue;
#pragma unroll
    for (int dx = -2 * P; dx <= 2 * P; ++dx) {
      const int a = 2 * A + dx;
      if (a < 0 || a >= Mf) continue;
      const T wt = w[(dy + 2 * P) * WR + dx + 2 * P];
      if (wt != T(0)) {
        const V2<T> v = r[long(b) * Mf + a];
        acc.x += wt * v.x;
        acc.y += wt * v.y;
      }
    }
  }
  yc[i] = acc;
}

// yf(a, b) (+)= sum over coarse (A, B) with |a - 2A|, |b - 2B| <= 2P of RW[cls(A,B)][.][.] xc
template <int P, typename T, bool ADD>
__global__ void __launch_bounds__(256)
k_prolong(int Mf, int Mc, const T* __restrict__ rw, const V2<T>* __restrict__ xc,
          V2<T>* __restrict__ yf, Addr af, Addr ac) {
  constexpr int WR = 4 * P + 1;
  const long Nf = long(Mf) * Mf;
  const long i = long(blockIdx.x) * 256 + threadIdx.x;
  if (i >= Nf) return;
  xc += ac.at(blockIdx.y);
  yf += af.at(blockIdx.y);
  const int b = int(i / Mf), a = int(i - long(b) * Mf);
  V2<T> acc = czero<T>();
  const int A0 = (a - 2 * P + 1) >> 1, B0 = (b - 2 * P + 1) >> 1;   // ceil((a - 2P) / 2)
#pragma unroll
  for (int jb = 0; jb <= 2 * P; ++jb) {
    const int B = B0 + jb;
    const int dy = b - 2 * B;
    if (B < 0 || B >= Mc || dy < -2 * P || dy > 2 * P) continue;
#pragma unroll
    for (int ja = 0; ja <= 2 * P; ++ja) {
      const int A = A0 + ja;
      const int dx = a - 2 * A;
      if (A < 0 || A >= Mc || dx < -2 * P || dx > 2 * P) continue;
      const int cls = (B % P) * P + (A % P);
      const T wt = rw[(cls * WR + dy + 2 * P) * WR + dx + 2 * P];
      if (wt != T(0)) {
        const V2<T> v = xc[long(B) * Mc + A];
        acc.x += wt * v.x;
        acc.y += wt * v.y;
      }
    }
  }
  if (ADD) acc = cadd<T>(acc, yf[i]);
  yf[i] = acc;
}

struct PwParams {
  double t[10], w[10];     // Gauss-Legendre nodes and weights on [0, 1]
  double lag[4][10];       // equispaced Lagrange functions at the nodes
};

// Load vector of the plane-wave impedance data, one thread per lattice point: boundary
// points gather the integrals of g * phi over their boundary edges; interior points get 0.
__global__ void __launch_bounds__(256)
k_planewave(int p, int n, double k, double ct, double st, PwParams pw, double2* __restrict__ F) {
  const int M = p * n + 1;
  const long i = long(blockIdx.x) * 256 + threadIdx.x;
  if (i >= long(M) * M) return;
  const int b = int(i / M), a = int(i - long(b) * M);
  const double h = 1.0 / n;
  double2 acc = make_double2(0.0, 0.0);
  // sides: 0 bottom (y=0), 1 right (x=1), 2 top (y=1), 3 left (x=0)
  for (int side = 0; side < 4; ++side) {
    const bool on = side == 0 ? b == 0 : side == 1 ? a == M - 1 : side == 2 ? b == M - 1 : a == 0;
    if (!on) continue;
    const int c = (side == 0 || side == 2) ? a : b;      // lattice coordinate along the side
    double nx = 0, ny = 0;
    if (side == 0) ny = -1; else if (side == 1) nx = 1; else if (side == 2) ny = 1; else nx = -1;
    const double gfac = k * (nx * ct + ny * st - 1.0);  // g = i * gfac * u
    for (int e = c / p - 1; e <= c / p; ++e) {
      if (e < 0 || e >= n) continue;
      const int loc = c - p * e;
      if (loc < 0 || loc > p) continue;
      double sr = 0, si = 0;
      for (int q = 0; q < 10; ++q) {
        const double along = (e + pw.t[q]) * h;
        double x, y;
        if (side == 0) { x = along; y = 0; }
        else if (side == 1) { x = 1; y = along; }
        else if (side == 2) { x = along; y = 1; }
        else { x = 0; y = along; }
        double sn, cs;
        sincos(k * (x * ct + y * st), &sn, &cs);
        // i * gfac * (cs + i sn) = -gfac sn + i gfac cs
        const double wl = pw.w[q] * pw.lag[loc][q];
        sr += wl * (-gfac * sn);
        si += wl * (gfac * cs);
      }
      acc.x += h * sr;
      acc.y += h * si;
    }
  }
  F[i] = acc;
}

__global__ void k_d2f(const double2* __restrict__ x, Addr ax, float2* __restrict__ y, Addr ay,
                      long n) {
  const long i = long(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  const double2 v = x[ax.at(blockIdx.y) + i];
  y[ay.at(blockIdx.y) + i] = make_float2(float(v.x), float(v.y));
}
__global__ void k_f2d(const float2* __restrict__ x, double2* __restrict__ y, long n) {
  const long i = long(blockIdx.x) * 256 + threadIdx.x;
  if (i < n) y[i] = make_double2(double(x[i].x), double(x[i].y));
}

template <int P, typename T, typename TX, typename TF, typename TY>
void stencil_p(int mode, const DevOp<T>& op, const V2<TX>* x, Addr xs, const V2<TF>* f, Addr fs,
               V2<TY>* y, Addr ys, int nbatch, hipStream_t st) {
  const int nmac = (op.M + P - 1) / P;
  dim3 grid((nmac + BX - 1) / BX, (nmac + BY - 1) / BY, nbatch);
  if (mode == ST_APPLY)
    k_stencil<P, T, TX, TF, TY, ST_APPLY><<<grid, 256, 0, st>>>(op, x, xs, f, fs, y, ys);
  else if (mode == ST_RESID)
    k_stencil<P, T, TX, TF, TY, ST_RESID><<<grid, 256, 0, st>>>(op, x, xs, f, fs, y, ys);
  else
    k_stencil<P, T, TX, TF, TY, ST_SMOOTH><<<grid, 256, 0, st>>>(op, x, xs, f, fs, y, ys);
}

}  // namespace

template <typename T, typename TX, typename TF, typename TY>
void launch_stencil(int p, int mode, const DevOp<T>& op, const V2<TX>* x, Addr xs,
                    const V2<TF>* f, Addr fs, V2<TY>* y, Addr ys, int nbatch, hipStream_t st) {
  if (p == 1) stencil_p<1, T, TX, TF, TY>(mode, op, x, xs, f, fs, y, ys, nbatch, st);
  else if (p == 2) stencil_p<2, T, TX, TF, TY>(mode, op, x, xs, f, fs, y, ys, nbatch, st);
  else stencil_p<3, T, TX, TF, TY>(mode, op, x, xs, f, fs, y, ys, nbatch, st);
  HZ_HIP(hipGetLastError());
}

template <typename T, typename TF>
void launch_jacobi0(int p, const DevOp<T>& op, const V2<TF>* f, Addr fs, V2<T>* y, Addr ys,
                    int nbatch, hipStream_t st) {
  const long N = long(op.M) * op.M;
  dim3 grid(unsigned((N + 255) / 256), nbatch);
  if (p == 1) k_jacobi0<1, T, TF><<<grid, 256, 0, st>>>(op, f, fs, y, ys);
  else if (p == 2) k_jacobi0<2, T, TF><<<grid, 256, 0, st>>>(op, f, fs, y, ys);
  else k_jacobi0<3, T, TF><<<grid, 256, 0, st>>>(op, f, fs, y, ys);
  HZ_HIP(hipGetLastError());
}

template <typename T>
void launch_restrict(int p, int Mf, int Mc, const T* rw, const V2<T>* r, V2<T>* yc, int nbatch,
                     Addr fstride, Addr cstride, hipStream_t st) {
  const long Nc = long(Mc) * Mc;
  dim3 grid(unsigned((Nc + 255) / 256), nbatch);
  if (p == 1) k_restrict<1, T><<<grid, 256, 0, st>>>(Mf, Mc, rw, r, yc, fstride, cstride);
  else if (p == 2) k_restrict<2, T><<<grid, 256, 0, st>>>(Mf, Mc, rw, r, yc, fstride, cstride);
  else k_restrict<3, T><<<grid, 256, 0, st>>>(Mf, Mc, rw, r, yc, fstride, cstride);
  HZ_HIP(hipGetLastError());
}

template <typename T>
void launch_prolong(int p, int Mf, int Mc, const T* rw, const V2<T>* xc, V2<T>* yf, bool add,
                    int nbatch, Addr fstride, Addr cstride, hipStream_t st) {
  const long Nf = long(Mf) * Mf;
  dim3 grid(unsigned((Nf + 255) / 256), nbatch);
#define HZ_PRO(PP)                                                                             \
  if (add) k_prolong<PP, T, true><<<grid, 256, 0, st>>>(Mf, Mc, rw, xc, yf, fstride, cstride); \
  else k_prolong<PP, T, false><<<grid, 256, 0, st>>>(Mf, Mc, rw, xc, yf, fstride, cstride);
  if (p == 1) { HZ_PRO(1) } else if (p == 2) { HZ_PRO(2) } else { HZ_PRO(3) }
#undef HZ_PRO
  HZ_HIP(hipGetLastError());
}

void launch_planewave(int p, int n, double k, double theta, const double* gl_t,
                      const double* gl_w, const double* lag, double2* F, hipStream_t st) {
  PwParams pw;
  for (int q = 0; q < 10; ++q) {
    pw.t[q] = gl_t[q];
    pw.w[q] = gl_w[q];
    for (int l = 0; l < 4; ++l) pw.lag[l][q] = lag[l * 10 + q];
  }
  const long N = long(p * n + 1) * (p * n + 1);
  k_planewave<<<unsigned((N + 255) / 256), 256, 0, st>>>(p, n, k, std::cos(theta),
                                                         std::sin(theta), pw, F);
  HZ_HIP(hipGetLastError());
}

void launch_d2f(const double2* x, float2* y, long n, hipStream_t st) {
  if (n <= 0) return;
  k_d2f<<<unsigned((n + 255) / 256), 256, 0, st>>>(x, Addr(), y, Addr(), n);
  HZ_HIP(hipGetLastError());
}
void launch_d2f_b(const double2* x, Addr ax, float2* y, Addr ay, long n, int nbatch,
                  hipStream_t st) {
  if (n <= 0 || nbatch <= 0) return;
  k_d2f<<<dim3(unsigned((n + 255) / 256), nbatch), 256, 0, st>>>(x, ax, y, ay, n);
  HZ_HIP(hipGetLastError());
}
void launch_f2d(const float2* x, double2* y, long n, hipStream_t st) {
  if (n <= 0) return;
  k_f2d<<<unsigned((n + 255) / 256), 256, 0, st>>>(x, y, n);
  HZ_HIP(hipGetLastError());
}

// Instantiations used by the driver.
template void launch_stencil<double, double, double, double>(int, int, const DevOp<double>&,
    const double2*, Addr, const double2*, Addr, double2*, Addr, int, hipStream_t);
template void launch_stencil<double, float, double, double>(int, int, const DevOp<double>&,
    const float2*, Addr, const double2*, Addr, double2*, Addr, int, hipStream_t);
template void launch_stencil<float, float, float, float>(int, int, const DevOp<float>&,
    const float2*, Addr, const float2*, Addr, float2*, Addr, int, hipStream_t);
template void launch_jacobi0<double, double>(int, const DevOp<double>&, const double2*, Addr,
                                             double2*, Addr, int, hipStream_t);
template void launch_jacobi0<float, float>(int, const DevOp<float>&, const float2*, Addr, float2*,
                                           Addr, int, hipStream_t);
template void launch_restrict<double>(int, int, int, const double*, const double2*, double2*, int,
                                      Addr, Addr, hipStream_t);
template void launch_restrict<float>(int, int, int, const float*, const float2*, float2*, int,
                                     Addr, Addr, hipStream_t);
template void launch_prolong<double>(int, int, int, const double*, const double2*, double2*, bool,
                                     int, Addr, Addr, hipStream_t);
template void launch_prolong<float>(int, int, int, const float*, const float2*, float2*, bool, int,
                                    Addr, Addr, hipStream_t);

}  // namespace hz
