// Heterogeneous wavenumber (Sec. 6, the problem statement of the numerical results:
// k(x) = k_max mu(x), the point source f = 2 exp(-1000 |x - x_s|^2), g = 0).
//
// k and the shift multiplier s are constant on every fine cell. The operators then differ
// from point to point, so each level stores one stencil per lattice point, assembled on the
// device from the cell values: entry (i, j) of A_s is
//   sum over fine cells c around i of  K_c(i, j) - s_c k_c^2 M_c(i, j)
//   - i sum over fine boundary edges e of  k_e B_e(i, j),
// with K_c, M_c the integrals of the level's basis over cell c (exact, host tables) and k_e
// the k of the cell that e bounds. On the coarse level (r = 2 fine cells per coarse cell
// side) this is the coarse form with the fine coefficient integrated exactly, i.e. the
// Galerkin product P^T A_s P of nested spaces. The per-point stencils are stored
// offset-major, [(2p+1)^2][M*M], so that a wave reads each offset with one coalesced load.

#include <stdexcept>

#include "hz_common.h"

namespace hz {

namespace {

// One thread per lattice point: its (2p+1)^2 stencil entries from the cell tables.
template <int P, int R>
__global__ void __launch_bounds__(256)
k_assemble_cells(int M, const double* __restrict__ tK, const double* __restrict__ tM,
                 const double* __restrict__ tB, const double* __restrict__ kc,
                 const double2* __restrict__ sc, double omega, double2* __restrict__ A,
                 double2* __restrict__ wd) {
  constexpr int W = 2 * P + 1, W2 = W * W, NF = 4 * R * R;
  const long N = long(M) * M;
  const long i = long(blockIdx.x) * 256 + threadIdx.x;
  if (i >= N) return;
  const int nf = R * ((M - 1) / P);
  const int b = int(i / M), a = int(i - long(b) * M);
  const int A0 = a / P, B0 = b / P, ca = a - P * A0, cb = b - P * B0;
  const int cls = cb * P + ca;
  double2 center = make_double2(0.0, 0.0);
  for (int d = 0; d < W2; ++d) {
    const int dy = d / W - P, dx = d % W - P;
    double2 acc = make_double2(0.0, 0.0);
    const size_t t0 = (size_t(cls) * W2 + d) * NF;
    // volume: the fine cells around the point, in the order of f
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const int fx = R * A0 + f % (2 * R) - R, fy = R * B0 + f / (2 * R) - R;
      if (fx < 0 || fx >= nf || fy < 0 || fy >= nf) continue;
      const double kv = tK[t0 + f], mv = tM[t0 + f];
      if (kv == 0.0 && mv == 0.0) continue;
      const long c = long(fy) * nf + fx;
      const double k = kc[c];
      const double2 s = sc ? sc[c] : make_double2(1.0, 0.0);
      acc.x += kv - s.x * k * k * mv;
      acc.y -= s.y * k * k * mv;
    }
    // boundary: bottom (b = 0), top (b = M-1) along x; left (a = 0), right (a = M-1) along y
    for (int side = 0; side < 4; ++side) {
      const bool on = side == 0 ? b == 0 : side == 1 ? b == M - 1 : side == 2 ? a == 0 : a == M - 1;
      if (!on) continue;
      const bool along_x = side < 2;
      if (along_x ? dy != 0 : dx != 0) continue;
      const int pos = along_x ? a : b, e = along_x ? dx : dy;
      const int E0 = pos / P, cc = pos - P * E0;
      for (int fe = -R; fe < R; ++fe) {
        const int q = R * E0 + fe;
        if (q < 0 || q >= nf) continue;
        const double bv = tB[(size_t(cc) * W + (e + P)) * 2 * R + (fe + R)];
        if (bv == 0.0) continue;
        long c;
        if (side == 0) c = q;
        else if (side == 1) c = long(nf - 1) * nf + q;
        else if (side == 2) c = long(q) * nf;
        else c = long(q) * nf + nf - 1;
        acc.y -= kc[c] * bv;
      }
    }
    A[size_t(d) * N + i] = acc;
    if (d == (W2 - 1) / 2) center = acc;
  }
  if (wd) {
    const double den = center.x * center.x + center.y * center.y;
    wd[i] = den > 0.0 ? make_double2(omega * center.x / den, -omega * center.y / den)
                      : make_double2(0.0, 0.0);
  }
}

// Stencil application with per-point operators; one thread per lattice point, the rows of
// a workgroup's points banded per XCD (neighbouring rows read through one L2). Modes as for
// the class-table kernel: y = A x, y = f - A x, y = x + wd (f - A x), and the first two sweeps
// from zero in one pass (x = f; the neighbours' first iterates wd f are formed on the fly).
template <int P, typename T, typename TX, typename TF, typename TY, int MODE>
__global__ void __launch_bounds__(256)
k_stencil_pn(DevOp<T> op, const V2<TX>* __restrict__ x, Addr ax, const V2<TF>* __restrict__ f,
             Addr af, V2<TY>* __restrict__ y, Addr ay) {
  constexpr int W = 2 * P + 1, W2 = W * W;
  const int M = op.M;
  const long N = long(M) * M;
  const int nblocks = int((N + 255) / 256);
  const int per = (nblocks + 7) / 8;
  const long blk = long(blockIdx.x % 8) * per + blockIdx.x / 8;
  const long i = blk * 256 + threadIdx.x;
  if (i >= N) return;
  const int bz = blockIdx.y;
  const V2<T>* __restrict__ coef = op.ctab ? op.ctab[bz] : op.coef;
  const V2<T>* __restrict__ wdinv = op.wtab ? op.wtab[bz] : op.wdinv;
  x += ax.at(bz);
  y += ay.at(bz);
  if (MODE != ST_APPLY) f += af.at(bz);
  const int b = int(i / M), a = int(i - long(b) * M);
  V2<T> acc = czero<T>();
#pragma unroll
  for (int dy = -P; dy <= P; ++dy) {
    const int bb = b + dy;
    if (bb < 0 || bb >= M) continue;
#pragma unroll
    for (int dx = -P; dx <= P; ++dx) {
      if (P == 1 && !couples(1, 0, 0, dx, dy)) continue;   // structurally zero for P1
      const int aa = a + dx;
      if (aa < 0 || aa >= M) continue;
      const V2<T> c = coef[size_t((dy + P) * W + dx + P) * N + i];
      const long j = long(bb) * M + aa;
      V2<T> v = cvt<T>(x[j]);
      if constexpr (MODE == ST_SMOOTH0) v = cmul<T>(wdinv[j], v);
      cfma(acc, c, v);
    }
  }
  V2<T> out = acc;
  if constexpr (MODE == ST_RESID) {
    out = csub<T>(cvt<T>(f[i]), acc);
  } else if constexpr (MODE == ST_SMOOTH || MODE == ST_SMOOTH0) {
    const V2<T> d = wdinv[i];
    V2<T> u = cvt<T>(x[i]);
    if constexpr (MODE == ST_SMOOTH0) u = cmul<T>(d, u);
    out = cadd<T>(u, cmul<T>(d, csub<T>(cvt<T>(f[i]), acc)));
  }
  y[i] = cvt<TY>(out);
  (void)W2;
}

struct QuadArgs {
  const double *xi, *eta, *w, *phi;
  const int* loc;
  int nq;
};

// F_i = sum over the (up to six) triangles T around point i of h^2 sum_k w_k f(x_T(xi_k))
// phi_r(xi_k), r the local index of i in T; x_T(xi) = v0 + h (xi + eta, eta) for T_L and
// v0 + h (xi, xi + eta) for T_U (|det J| = h^2).
template <int P>
__global__ void __launch_bounds__(256)
k_gauss_rhs(int n, double sx, double sy, double amp, double width, QuadArgs q,
            double2* __restrict__ F) {
  const int M = P * n + 1;
  const long i = long(blockIdx.x) * 256 + threadIdx.x;
  if (i >= long(M) * M) return;
  const double h = 1.0 / n;
  const int b = int(i / M), a = int(i - long(b) * M);
  const int A0 = a / P, B0 = b / P, cls = (b - P * B0) * P + (a - P * A0);
  double acc = 0.0;
  for (int Bc = -1; Bc <= 0; ++Bc)
    for (int Ac = -1; Ac <= 0; ++Ac) {
      const int cx = A0 + Ac, cy = B0 + Bc;
      if (cx < 0 || cx >= n || cy < 0 || cy >= n) continue;
      for (int tri = 0; tri < 2; ++tri) {
        const int r = q.loc[cls * 8 + ((Bc + 1) * 2 + (Ac + 1)) * 2 + tri];
        if (r < 0) continue;
        const double x0 = cx * h, y0 = cy * h;
        double s = 0.0;
        for (int k = 0; k < q.nq; ++k) {
          const double xi = q.xi[k], et = q.eta[k];
          const double X = tri == 0 ? x0 + h * (xi + et) : x0 + h * xi;
          const double Y = tri == 0 ? y0 + h * et : y0 + h * (xi + et);
          const double r2 = (X - sx) * (X - sx) + (Y - sy) * (Y - sy);
          s += q.w[k] * (amp * exp(-width * r2)) * q.phi[size_t(r) * q.nq + k];
        }
        acc += h * h * s;
      }
    }
  F[i] = make_double2(acc, 0.0);
}

template <int P, typename T, typename TX, typename TF, typename TY>
void stencil_pn_p(int mode, const DevOp<T>& op, const V2<TX>* x, Addr xs, const V2<TF>* f,
                  Addr fs, V2<TY>* y, Addr ys, int nbatch, hipStream_t st) {
  const long N = long(op.M) * op.M;
  const int nblocks = int((N + 255) / 256);
  const dim3 grid(unsigned(8 * ((nblocks + 7) / 8)), nbatch);
  if (mode == ST_APPLY)
    k_stencil_pn<P, T, TX, TF, TY, ST_APPLY><<<grid, 256, 0, st>>>(op, x, xs, f, fs, y, ys);
  else if (mode == ST_RESID)
    k_stencil_pn<P, T, TX, TF, TY, ST_RESID><<<grid, 256, 0, st>>>(op, x, xs, f, fs, y, ys);
  else if (mode == ST_SMOOTH)
    k_stencil_pn<P, T, TX, TF, TY, ST_SMOOTH><<<grid, 256, 0, st>>>(op, x, xs, f, fs, y, ys);
  else
    k_stencil_pn<P, T, TX, TF, TY, ST_SMOOTH0><<<grid, 256, 0, st>>>(op, x, xs, f, fs, y, ys);
}

}  // namespace

template <typename T, typename TX, typename TF, typename TY>
void launch_stencil_pn(int p, int mode, const DevOp<T>& op, const V2<TX>* x, Addr xs,
                       const V2<TF>* f, Addr fs, V2<TY>* y, Addr ys, int nbatch, hipStream_t st) {
  if (p == 1) stencil_pn_p<1, T, TX, TF, TY>(mode, op, x, xs, f, fs, y, ys, nbatch, st);
  else if (p == 2) stencil_pn_p<2, T, TX, TF, TY>(mode, op, x, xs, f, fs, y, ys, nbatch, st);
  else stencil_pn_p<3, T, TX, TF, TY>(mode, op, x, xs, f, fs, y, ys, nbatch, st);
  HZ_HIP(hipGetLastError());
}

void launch_assemble_cells(int p, int r, int M, const double* tabK, const double* tabM,
                           const double* tabB, const double* kc, const double2* sc,
                           double omega, double2* A, double2* wd, hipStream_t st) {
  const long N = long(M) * M;
  const unsigned g = unsigned((N + 255) / 256);
#define HZ_ASM(PP, RR) \
  k_assemble_cells<PP, RR><<<g, 256, 0, st>>>(M, tabK, tabM, tabB, kc, sc, omega, A, wd)
  if (r == 1) {
    if (p == 1) HZ_ASM(1, 1); else if (p == 2) HZ_ASM(2, 1); else HZ_ASM(3, 1);
  } else if (r == 2) {
    if (p == 1) HZ_ASM(1, 2); else if (p == 2) HZ_ASM(2, 2); else HZ_ASM(3, 2);
  } else {
    throw std::runtime_error("cell tables: r must be 1 or 2");
  }
#undef HZ_ASM
  HZ_HIP(hipGetLastError());
}

void launch_gauss_rhs(int p, int n, double sx, double sy, double amp, double width,
                      const double* qxi, const double* qeta, const double* qw,
                      const double* qphi, const int* qloc, int nq, double2* F, hipStream_t st) {
  const long N = long(p * n + 1) * (p * n + 1);
  const unsigned g = unsigned((N + 255) / 256);
  const QuadArgs q{qxi, qeta, qw, qphi, qloc, nq};
  if (p == 1) k_gauss_rhs<1><<<g, 256, 0, st>>>(n, sx, sy, amp, width, q, F);
  else if (p == 2) k_gauss_rhs<2><<<g, 256, 0, st>>>(n, sx, sy, amp, width, q, F);
  else k_gauss_rhs<3><<<g, 256, 0, st>>>(n, sx, sy, amp, width, q, F);
  HZ_HIP(hipGetLastError());
}

template void launch_stencil_pn<double, double, double, double>(int, int, const DevOp<double>&,
    const double2*, Addr, const double2*, Addr, double2*, Addr, int, hipStream_t);
template void launch_stencil_pn<double, float, double, double>(int, int, const DevOp<double>&,
    const float2*, Addr, const double2*, Addr, double2*, Addr, int, hipStream_t);
template void launch_stencil_pn<float, float, float, float>(int, int, const DevOp<float>&,
    const float2*, Addr, const float2*, Addr, float2*, Addr, int, hipStream_t);

}  // namespace hz
