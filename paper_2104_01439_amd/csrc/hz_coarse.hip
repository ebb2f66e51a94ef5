// Exact coarse solve of the twogrid method (Sec. 4, Algorithm 1, the direct solve on the
// coarsest level; the paper factors it once, in the first FGMRES iteration, and reuses the
// factor). On the device the coarse operator A_eps^{2h} is treated as block tridiagonal in
// lattice rows: block j holds the p lattice rows p j .. p j + p - 1 (the last block the final
// row alone), so A_{j,j-1} and A_{j,j+1} are the sparse stencil couplings between adjacent
// blocks. Block LU without pivoting (justified: the Hermitian part of i A_eps is
// Im(s) k^2 M + k B, positive definite, so every Schur complement is nonsingular):
//     D_0 = A_00,   D_j = A_jj - A_{j,j-1} D_{j-1}^{-1} A_{j-1,j},   S_j := D_j^{-1}.
// S_j is formed explicitly by blocked Gauss-Jordan; the rank-NB updates run on FP64 MFMA.
// Solve:  g_j = S_j (b_j - A_{j,j-1} g_{j-1}),   x_j = g_j - S_j (A_{j,j+1} x_{j+1}).

#include "hz_common.h"

namespace hz {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int NB = 32;   // Gauss-Jordan panel width

__device__ __forceinline__ int region(int a, int M) { return a == 0 ? 0 : (a == M - 1 ? 2 : 1); }

__device__ __forceinline__ double2 crecip(double2 a) {
  const double d = a.x * a.x + a.y * a.y;
  return make_double2(a.x / d, -a.y / d);
}

// ------------------------------------------------------------------------------------------
// Schur complement assembly
// ------------------------------------------------------------------------------------------

// Tm[r'][c] = sum_{c' in block j-1} S_{j-1}[r'][c'] A[c'][c],  c in block j.
// A is symmetric, so A[c'][c] is the coefficient of the stencil of c at offset c' - c.
template <int P>
__global__ void __launch_bounds__(256)
k_schur_right(int j, int Mc, const double2* __restrict__ coef, const double2* __restrict__ Sprev,
              int nprev, int ncur, double2* __restrict__ Tm) {
  constexpr int W = 2 * P + 1, W2 = W * W;
  const int c = blockIdx.x * 256 + threadIdx.x;
  const int rp = blockIdx.y;
  if (c >= ncur) return;
  const int ac = c % Mc, bc = P * j + c / Mc;
  const int cls = (bc % P) * P + (ac % P);
  const int reg = region(bc, Mc) * 3 + region(ac, Mc);
  const double2* cc = coef + (cls * 9 + reg) * W2;
  const double2* srow = Sprev + size_t(rp) * nprev;
  double2 acc = make_double2(0, 0);
#pragma unroll
  for (int dy = -P; dy <= -1; ++dy) {
    const int bb = bc + dy;
    if (bb >= P * j) continue;
#pragma unroll
    for (int dx = -P; dx <= P; ++dx) {
      const int aa = ac + dx;
      if (aa < 0 || aa >= Mc) continue;
      const double2 cf = cc[(dy + P) * W + dx + P];
      if (cf.x == 0.0 && cf.y == 0.0) continue;
      const int col = (bb - P * (j - 1)) * Mc + aa;
      cfma(acc, cf, srow[col]);
    }
  }
  Tm[size_t(rp) * ncur + c] = acc;
}

// D[r][c] = A_jj[r][c] - sum_{r' in block j-1} A[r][r'] Tm[r'][c]   (Tm ignored for j = 0).
template <int P>
__global__ void __launch_bounds__(256)
k_schur_left(int j, int Mc, const double2* __restrict__ coef, const double2* __restrict__ Tm,
             int ncur, double2* __restrict__ D) {
  constexpr int W = 2 * P + 1, W2 = W * W;
  const int c = blockIdx.x * 256 + threadIdx.x;
  const int r = blockIdx.y;
  if (c >= ncur) return;
  const int ar = r % Mc, br = P * j + r / Mc;
  const int cls = (br % P) * P + (ar % P);
  const int reg = region(br, Mc) * 3 + region(ar, Mc);
  const double2* cr = coef + (cls * 9 + reg) * W2;
  double2 acc = make_double2(0, 0);
  const int ac = c % Mc, bc = P * j + c / Mc;
  const int dxa = ac - ar, dya = bc - br;
  if (dxa >= -P && dxa <= P && dya >= -P && dya <= P) acc = cr[(dya + P) * W + dxa + P];
  if (j > 0) {
#pragma unroll
    for (int dy = -P; dy <= -1; ++dy) {
      const int bb = br + dy;
      if (bb >= P * j) continue;
#pragma unroll
      for (int dx = -P; dx <= P; ++dx) {
        const int aa = ar + dx;
        if (aa < 0 || aa >= Mc) continue;
        const double2 cf = cr[(dy + P) * W + dx + P];
        if (cf.x == 0.0 && cf.y == 0.0) continue;
        const int rp = (bb - P * (j - 1)) * Mc + aa;
        const double2 tv = Tm[size_t(rp) * ncur + c];
        acc.x -= cf.x * tv.x - cf.y * tv.y;
        acc.y -= cf.x * tv.y + cf.y * tv.x;
      }
    }
  }
  D[size_t(r) * ncur + c] = acc;
}

// ------------------------------------------------------------------------------------------
// Blocked Gauss-Jordan inversion, in place. One panel K = [k0, k0 + w):
//   Pinv = X[K,K]^{-1};   X <- X - Wt Rt   with
//   Wt[i, :] = X[i, K] Pinv (i not in K),  Wt[K, :] = I - Pinv,
//   Rt[:, j] = X[K, j]      (j not in K),  Rt[:, K] = X[K, K] + I,
// which leaves X[K,K] = Pinv, X[K,j] = Pinv X[K,j], X[i,K] = -X[i,K] Pinv and the Schur
// update X[i,j] - X[i,K] Pinv X[K,j] elsewhere.
// ------------------------------------------------------------------------------------------

__global__ void __launch_bounds__(256)
k_gj_panel(const double2* __restrict__ X, int n, int k0, int w, double2* __restrict__ Wt,
           double2* __restrict__ Rt, int* __restrict__ flag) {
  __shared__ double2 Y[NB][NB + 1];
  __shared__ double2 rowt[NB], colt[NB];
  const int tid = threadIdx.x;
  for (int idx = tid; idx < NB * NB; idx += 256) {
    const int r = idx / NB, c = idx % NB;
    double2 v = make_double2(r == c ? 1.0 : 0.0, 0.0);
    if (r < w && c < w) v = X[size_t(k0 + r) * n + k0 + c];
    Y[r][c] = v;
  }
  __syncthreads();
  bool bad = false;
  for (int t = 0; t < w; ++t) {
    const double2 pv = Y[t][t];
    const double mag = pv.x * pv.x + pv.y * pv.y;
    if (!(mag > 0.0) || !isfinite(mag)) bad = true;
    const double2 pinv = crecip(pv);
    if (tid < NB) {
      rowt[tid] = cmul<double>(Y[t][tid], pinv);
      colt[tid] = Y[tid][t];
    }
    __syncthreads();
    for (int idx = tid; idx < NB * NB; idx += 256) {
      const int r = idx / NB, c = idx % NB;
      if (r == t) {
        Y[r][c] = (c == t) ? pinv : rowt[c];
      } else if (c == t) {
        const double2 v = cmul<double>(colt[r], pinv);
        Y[r][c] = make_double2(-v.x, -v.y);
      } else {
        const double2 a = colt[r], b = rowt[c];
        double2 v = Y[r][c];
        v.x -= a.x * b.x - a.y * b.y;
        v.y -= a.x * b.y + a.y * b.x;
        Y[r][c] = v;
      }
    }
    __syncthreads();
  }
  if (bad && tid == 0 && blockIdx.x == 0) *flag = 1;
  const int base = blockIdx.x * 64;
  for (int idx = tid; idx < 64 * NB; idx += 256) {
    const int i = base + idx / NB, kk = idx % NB;
    if (i >= n) continue;
    double2 v = make_double2(0, 0);
    if (kk < w) {
      if (i >= k0 && i < k0 + w) {
        const double2 y = Y[i - k0][kk];
        v = make_double2((i - k0 == kk ? 1.0 : 0.0) - y.x, -y.y);
      } else {
        const double2* xr = X + size_t(i) * n + k0;
        for (int t = 0; t < w; ++t) cfma(v, xr[t], Y[t][kk]);
      }
    }
    Wt[size_t(i) * NB + kk] = v;
  }
  for (int idx = tid; idx < 64 * NB; idx += 256) {
    const int jj = base + idx % 64, kk = idx / 64;
    if (jj >= n) continue;
    double2 v = make_double2(0, 0);
    if (kk < w) {
      v = X[size_t(k0 + kk) * n + jj];
      if (jj - k0 == kk) v.x += 1.0;
    }
    Rt[size_t(kk) * n + jj] = v;
  }
}

// X -= Wt (n x NB) * Rt (NB x n), complex FP64 on MFMA. Each wave owns a 32 x 32 tile
// (2 x 2 blocks of 16 x 16); operands are read straight from the (L2-resident) panels.
// v_mfma_f64_16x16x4: lane l holds A[l%16][l/16], B[l/16][l%16] and D[l/16 + 4r][l%16]
// (r = 0..3; the FP64 layout interleaves rows by 4, checked on the device).
__global__ void __launch_bounds__(256)
k_gj_update(double2* __restrict__ X, int n, const double2* __restrict__ Wt,
            const double2* __restrict__ Rt) {
  const int lane = threadIdx.x & 63;
  const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int tiles = (n + 31) / 32;
  if (wave >= tiles * tiles) return;
  const int ti = wave / tiles, tj = wave % tiles;
  const int i0 = ti * 32, j0 = tj * 32;
  const int li = lane & 15, lk = lane >> 4;
  v4d cre[2][2], cim[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = i0 + bi * 16 + lk + 4 * r, col = j0 + bj * 16 + li;
        double2 v = make_double2(0, 0);
        if (row < n && col < n) v = X[size_t(row) * n + col];
        cre[bi][bj][r] = v.x;
        cim[bi][bj][r] = v.y;
      }
#pragma unroll
  for (int k = 0; k < NB; k += 4) {
    double are[2], aim[2], bre[2], bim[2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) {
      const int row = i0 + bi * 16 + li;
      double2 a = make_double2(0, 0);
      if (row < n) a = Wt[size_t(row) * NB + k + lk];
      are[bi] = -a.x;
      aim[bi] = -a.y;
    }
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      const int col = j0 + bj * 16 + li;
      double2 b = make_double2(0, 0);
      if (col < n) b = Rt[size_t(k + lk) * n + col];
      bre[bj] = b.x;
      bim[bj] = b.y;
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) {
        // (-a)(b): re = -are*bre + aim*bim, im = -are*bim - aim*bre  (are, aim hold -a)
        cre[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(are[bi], bre[bj], cre[bi][bj], 0, 0, 0);
        cre[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(-aim[bi], bim[bj], cre[bi][bj], 0, 0, 0);
        cim[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(are[bi], bim[bj], cim[bi][bj], 0, 0, 0);
        cim[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(aim[bi], bre[bj], cim[bi][bj], 0, 0, 0);
      }
  }
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = i0 + bi * 16 + lk + 4 * r, col = j0 + bj * 16 + li;
        if (row < n && col < n) X[size_t(row) * n + col] = make_double2(cre[bi][bj][r], cim[bi][bj][r]);
      }
}

__global__ void k_factor_to_f32(const double2* __restrict__ S, float2* __restrict__ Sf, size_t n) {
  const size_t i = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (i < n) Sf[i] = make_float2(float(S[i].x), float(S[i].y));
}

// ------------------------------------------------------------------------------------------
// Block triangular solves (one launch per block row)
// ------------------------------------------------------------------------------------------

// LDS: t[rhs][c] = coupling term of block j (FWD: b_j - A_{j,j-1} g_{j-1};
// BWD: A_{j,j+1} x_{j+1}); then row r of block j: y_j[r] = S_j[r,:] t (FWD) or
// y_j[r] - S_j[r,:] t (BWD). One wavefront per row.
template <int P, typename T, bool FWD>
__global__ void __launch_bounds__(256)
k_csolve_step(int j, int nc, int Mc, const V2<T>* __restrict__ coef, const V2<T>* __restrict__ Sj,
              const V2<T>* __restrict__ b, V2<T>* __restrict__ y, int nrhs, long cstride) {
  constexpr int W = 2 * P + 1, W2 = W * W;
  extern __shared__ char smem[];
  V2<T>* t = reinterpret_cast<V2<T>*>(smem);
  const int nj = (j < nc ? P : 1) * Mc;
  const long dof0 = long(P) * j * Mc;
  for (int idx = threadIdx.x; idx < nj * nrhs; idx += 256) {
    const int rhs = idx / nj, c = idx - rhs * nj;
    const V2<T>* yv = y + rhs * cstride;
    const int ac = c % Mc, bc = P * j + c / Mc;
    const int cls = (bc % P) * P + (ac % P);
    const int reg = region(bc, Mc) * 3 + region(ac, Mc);
    const V2<T>* cc = coef + (cls * 9 + reg) * W2;
    V2<T> acc = FWD ? b[rhs * cstride + dof0 + c] : czero<T>();
#pragma unroll
    for (int dyi = 1; dyi <= P; ++dyi) {
      const int dy = FWD ? -dyi : dyi;
      const int bb = bc + dy;
      if (FWD ? (j == 0 || bb >= P * j) : (j == nc || bb < P * (j + 1) || bb >= Mc)) continue;
#pragma unroll
      for (int dx = -P; dx <= P; ++dx) {
        const int aa = ac + dx;
        if (aa < 0 || aa >= Mc) continue;
        const V2<T> cf = cc[(dy + P) * W + dx + P];
        const V2<T> v = yv[long(bb) * Mc + aa];
        if (FWD) {
          acc.x -= cf.x * v.x - cf.y * v.y;
          acc.y -= cf.x * v.y + cf.y * v.x;
        } else {
          cfma(acc, cf, v);
        }
      }
    }
    t[rhs * nj + c] = acc;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= nj) return;
  const V2<T>* srow = Sj + size_t(r) * nj;
  constexpr int MAXR = 4;
  T sr[MAXR], si[MAXR];
#pragma unroll
  for (int q = 0; q < MAXR; ++q) { sr[q] = T(0); si[q] = T(0); }
  for (int c = lane; c < nj; c += 64) {
    const V2<T> s = srow[c];
#pragma unroll
    for (int q = 0; q < MAXR; ++q) {
      if (q < nrhs) {
        const V2<T> tv = t[q * nj + c];
        sr[q] += s.x * tv.x - s.y * tv.y;
        si[q] += s.x * tv.y + s.y * tv.x;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < MAXR; ++q) {
    if (q < nrhs) {
      const T a = wave_sum(sr[q]), bq = wave_sum(si[q]);
      if (lane == 0) {
        V2<T>* yo = y + q * cstride + dof0 + r;
        if (FWD) {
          V2<T> o; o.x = a; o.y = bq;
          *yo = o;
        } else {
          V2<T> o = *yo;
          o.x -= a;
          o.y -= bq;
          *yo = o;
        }
      }
    }
  }
}

template <int P, typename T>
void csolve_p(const CoarseLayout& L, const DevOp<T>& cop, const V2<T>* S, const V2<T>* b, V2<T>* y,
              int nrhs, long cstride, hipStream_t st) {
  for (int r0 = 0; r0 < nrhs; r0 += 4) {
    const int nr = std::min(4, nrhs - r0);
    const V2<T>* bb = b + r0 * cstride;
    V2<T>* yy = y + r0 * cstride;
    for (int j = 0; j < L.nblocks(); ++j) {
      const int nj = int(L.size(j));
      const size_t lds = size_t(nj) * nr * sizeof(V2<T>);
      k_csolve_step<P, T, true><<<(nj + 3) / 4, 256, lds, st>>>(j, L.nc, L.Mc, cop.coef, S + L.off(j),
                                                                 bb, yy, nr, cstride);
    }
    for (int j = L.nblocks() - 2; j >= 0; --j) {
      const int nj = int(L.size(j));
      const size_t lds = size_t(nj) * nr * sizeof(V2<T>);
      k_csolve_step<P, T, false><<<(nj + 3) / 4, 256, lds, st>>>(j, L.nc, L.Mc, cop.coef, S + L.off(j),
                                                                  bb, yy, nr, cstride);
    }
  }
  HZ_HIP(hipGetLastError());
}

template <int P, typename T> void allow_lds() {
  HZ_HIP(hipFuncSetAttribute((const void*)k_csolve_step<P, T, true>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
  HZ_HIP(hipFuncSetAttribute((const void*)k_csolve_step<P, T, false>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
}

template <int P>
void factor_p(const CoarseLayout& L, const DevOp<double>& cop, double2* S,
              const CoarseFactorWork& w, hipStream_t st) {
  for (int j = 0; j < L.nblocks(); ++j) {
    const int n = int(L.size(j));
    double2* D = S + L.off(j);
    if (j > 0) {
      const int np = int(L.size(j - 1));
      k_schur_right<P><<<dim3((n + 255) / 256, np), 256, 0, st>>>(j, L.Mc, cop.coef, S + L.off(j - 1),
                                                                  np, n, w.T);
    }
    k_schur_left<P><<<dim3((n + 255) / 256, n), 256, 0, st>>>(j, L.Mc, cop.coef, w.T, n, D);
    const int tiles = (n + 31) / 32;
    const int upd_blocks = (tiles * tiles + 3) / 4;
    for (int k0 = 0; k0 < n; k0 += NB) {
      const int wdt = std::min(NB, n - k0);
      k_gj_panel<<<(n + 63) / 64, 256, 0, st>>>(D, n, k0, wdt, w.W, w.R, w.flag);
      k_gj_update<<<upd_blocks, 256, 0, st>>>(D, n, w.W, w.R);
    }
  }
  HZ_HIP(hipGetLastError());
}

}  // namespace

hz_status coarse_factor(const CoarseLayout& L, const DevOp<double>& cop, double2* S,
                        const CoarseFactorWork& w, hipStream_t st) {
  HZ_HIP(hipMemsetAsync(w.flag, 0, sizeof(int), st));
  if (L.p == 1) factor_p<1>(L, cop, S, w, st);
  else if (L.p == 2) factor_p<2>(L, cop, S, w, st);
  else factor_p<3>(L, cop, S, w, st);
  int flag = 0;
  HZ_HIP(hipMemcpyAsync(&flag, w.flag, sizeof(int), hipMemcpyDeviceToHost, st));
  HZ_HIP(hipStreamSynchronize(st));
  return flag ? HZ_ESINGULAR : HZ_OK;
}

template <typename T>
void coarse_solve(const CoarseLayout& L, const DevOp<T>& cop, const V2<T>* S, const V2<T>* b,
                  V2<T>* y, int nrhs, long cstride, hipStream_t st) {
  static bool once = false;
  if (!once) {
    allow_lds<1, double>(); allow_lds<2, double>(); allow_lds<3, double>();
    allow_lds<1, float>(); allow_lds<2, float>(); allow_lds<3, float>();
    once = true;
  }
  if (L.p == 1) csolve_p<1, T>(L, cop, S, b, y, nrhs, cstride, st);
  else if (L.p == 2) csolve_p<2, T>(L, cop, S, b, y, nrhs, cstride, st);
  else csolve_p<3, T>(L, cop, S, b, y, nrhs, cstride, st);
}

void launch_factor_to_f32(const double2* S, float2* Sf, size_t n, hipStream_t st) {
  k_factor_to_f32<<<unsigned((n + 255) / 256), 256, 0, st>>>(S, Sf, n);
  HZ_HIP(hipGetLastError());
}

template void coarse_solve<double>(const CoarseLayout&, const DevOp<double>&, const double2*,
                                   const double2*, double2*, int, long, hipStream_t);
template void coarse_solve<float>(const CoarseLayout&, const DevOp<float>&, const float2*,
                                  const float2*, float2*, int, long, hipStream_t);

}  // namespace hz
