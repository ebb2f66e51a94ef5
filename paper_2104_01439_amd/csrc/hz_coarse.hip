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
// Block triangular solves
// ------------------------------------------------------------------------------------------
//
// Step s of a solve is block j = s (forward sweep, s < nb) or j = 2 nb - 2 - s (backward
// sweep). Every workgroup first forms the coupling vector of block j in LDS,
//   FWD: t = b_j - A_{j,j-1} g_{j-1},   BWD: t = A_{j,j+1} x_{j+1},
// then computes its own balanced share of the rows of S_j t: the four waves split the
// columns, every lane issues all its loads of a row chunk at once, and the wave partial
// sums are combined in a fixed order. Steps are separated by a grid barrier when the
// kernel runs persistently (cooperative launch), or by kernel boundaries otherwise.

// Values that cross workgroups inside one launch (the block results g_j of the forward
// sweep and x_j of the backward sweep) are written and read with relaxed agent-scope
// atomics, which bypass the per-XCD L2 and are therefore coherent device-wide. Both result
// buffers are filled with a sentinel NaN (a payload no arithmetic produces) before the
// launch; a consumer polls the values it needs until none is the sentinel. This replaces a
// grid barrier: producers never wait, and a consumer waits exactly for its data. Every wait
// is bounded: on timeout it records an error and continues, so every wave terminates.
template <typename T> struct Sentinel;
template <> struct Sentinel<double> {
  using U = unsigned long long;
  static constexpr U bits = 0x7FFC0FFEE5AFE123ull;
};
template <> struct Sentinel<float> {
  using U = unsigned int;
  static constexpr U bits = 0x7FC0FEEDu;
};

template <typename T> __device__ __forceinline__ T ld_coh1(const T* q) {
  return __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T> __device__ __forceinline__ V2<T> ld_coh(const V2<T>* p) {
  const T* q = reinterpret_cast<const T*>(p);
  V2<T> r;
  r.x = ld_coh1(q);
  r.y = ld_coh1(q + 1);
  return r;
}
template <typename T> __device__ __forceinline__ void st_coh(V2<T>* p, V2<T> v) {
  T* q = reinterpret_cast<T*>(p);
  __hip_atomic_store(q, v.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(q + 1, v.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T> __device__ __forceinline__ bool is_sentinel(T v) {
  return __builtin_bit_cast(typename Sentinel<T>::U, v) == Sentinel<T>::bits;
}

template <typename T> __global__ void k_fill_sentinel(V2<T>* a, long n, long stride, int nrhs) {
  const long i = long(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  const T sv = __builtin_bit_cast(T, Sentinel<T>::bits);
  for (int h = 0; h < nrhs; ++h) {
    V2<T> v;
    v.x = sv;
    v.y = sv;
    a[h * stride + i] = v;
  }
}

// 256 threads: wave 0 gathers the neighbour block (polling until it is complete) and the
// right-hand side, combines the row sums and publishes the results; waves 1..3 stream the
// rows of S_j, prefetching the next block's rows as soon as their products are formed.
template <int P, typename T, int NR, int RCH, int QCH>
__global__ void __launch_bounds__(256)
k_csolve(int s_begin, int s_end, int nc, int Mc, const V2<T>* __restrict__ coef,
         const V2<T>* __restrict__ S, const V2<T>* __restrict__ b, V2<T>* __restrict__ y,
         V2<T>* __restrict__ gbuf, int nrhs, long cstride, int* __restrict__ err) {
  constexpr int W = 2 * P + 1, W2 = W * W, NCOEF = P * P * 9 * W2;
  constexpr int NCW = 3;                       // compute waves
  constexpr int ENT = 24;                      // neighbour entries per lane and round
  extern __shared__ char smem[];
  const int nmax = P * Mc;
  V2<T>* cl = reinterpret_cast<V2<T>*>(smem);  // coefficient table
  V2<T>* t = cl + NCOEF;                       // [NR][nmax] coupling vector of block j
  V2<T>* yn = t + NR * nmax;                   // [NR][nmax] neighbour block
  __shared__ T red[2][NCW][RCH][NR];
  const int nb = nc + 1;
  const int G = gridDim.x, g = blockIdx.x;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const size_t bsz = size_t(P * Mc) * size_t(P * Mc);
  const long Nc = long(Mc) * Mc;
  for (int i = threadIdx.x; i < NCOEF; i += 256) cl[i] = coef[i];

  V2<T> sv[RCH][QCH];
  bool have = false;                           // sv holds the first chunk of this step
  auto step_rows = [&](int s, int& nj, int& r0, int& r1, int& c0, int& c1, const V2<T>*& Sj) {
    const bool fwd = s < nb;
    const int j = fwd ? s : 2 * nb - 2 - s;
    nj = (j < nc ? P : 1) * Mc;
    r0 = int((long(nj) * g) / G);
    r1 = int((long(nj) * (g + 1)) / G);
    c0 = (nj * (wave - 1)) / NCW;
    c1 = (nj * wave) / NCW;
    Sj = S + size_t(j) * bsz;
  };
  auto load_chunk = [&](const V2<T>* Sj, int nj, int rb, int r1, int c0, int c1, int q0) {
#pragma unroll
    for (int rr = 0; rr < RCH; ++rr)
#pragma unroll
      for (int q = 0; q < QCH; ++q) {
        const int c = c0 + lane + 64 * (q0 + q);
        sv[rr][q] = (rb + rr < r1 && c < c1) ? Sj[size_t(rb + rr) * nj + c] : czero<T>();
      }
  };

  for (int s = s_begin; s < s_end; ++s) {
    const bool fwd = s < nb;
    const int j = fwd ? s : 2 * nb - 2 - s;
    const int nj = (j < nc ? P : 1) * Mc;
    const long dof0 = long(P) * j * Mc;
    // 1a. wave 0 gathers the neighbour block (g_{j-1} forward, x_{j+1} backward) and b_j
    const int jn = fwd ? j - 1 : j + 1;
    const bool has_n = fwd ? j > 0 : j < nc;
    const int nn = has_n ? (jn < nc ? P : 1) * Mc : 0;
    const long ndof0 = long(P) * jn * Mc;
    // backward neighbour x_{nc} is the forward result of the last block
    const V2<T>* src = fwd ? gbuf : (jn == nc ? gbuf : y);
    if (wave == 0) {
      for (int i0 = 0; i0 < nn * nrhs; i0 += 64 * ENT) {
        V2<T> v[ENT];
        unsigned pending = 0;
#pragma unroll
        for (int q = 0; q < ENT; ++q) {
          const int idx = i0 + lane + 64 * q;
          if (idx < nn * nrhs) pending |= 1u << q;
        }
        unsigned rounds = 0;
        while (pending) {
#pragma unroll
          for (int q = 0; q < ENT; ++q) {
            if (pending & (1u << q)) {
              const int idx = i0 + lane + 64 * q;
              const int h = idx / nn, c = idx - h * nn;
              v[q] = ld_coh<T>(src + h * (fwd || jn == nc ? Nc : cstride) + ndof0 + c);
            }
          }
#pragma unroll
          for (int q = 0; q < ENT; ++q)
            if ((pending & (1u << q)) && !is_sentinel(v[q].x) && !is_sentinel(v[q].y))
              pending &= ~(1u << q);
          if (pending) {
            ++rounds;
            if ((rounds & 255u) == 0) {   // rare checks: a timeout elsewhere, or our own
              if (rounds > (1u << 20)) {
                __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
              }
              if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
            }
            if (rounds > 8) __builtin_amdgcn_s_sleep(1);
          }
        }
#pragma unroll
        for (int q = 0; q < ENT; ++q) {
          const int idx = i0 + lane + 64 * q;
          if (idx < nn * nrhs) {
            const int h = idx / nn, c = idx - h * nn;
            yn[h * nmax + c] = v[q];
          }
        }
      }
      if (fwd)
        for (int idx = lane; idx < nj * nrhs; idx += 64) {
          const int h = idx / nj, c = idx - h * nj;
          t[h * nmax + c] = b[h * cstride + dof0 + c];
        }
    }
    __syncthreads();
    // 1b. coupling vector of block j, all waves, from LDS only (row by row: no divisions)
    {
      const int rows = nj / Mc;
      for (int h = 0; h < nrhs; ++h)
        for (int rl = 0; rl < rows; ++rl) {
          const int bc = P * j + rl;
          const int cb = (bc % P) * P, ry = region(bc, Mc) * 3;
          int bb_lo, bb_hi;                      // lattice rows of the neighbour block
          if (fwd) { bb_lo = P * j - P; bb_hi = P * j - 1; }
          else { bb_lo = P * (j + 1); bb_hi = min(P * (j + 1) + P - 1, Mc - 1); }
          for (int ac = threadIdx.x; ac < Mc; ac += 256) {
            const int c = rl * Mc + ac;
            const V2<T>* cc = cl + ((cb + ac % P) * 9 + ry + region(ac, Mc)) * W2;
            V2<T> acc = fwd ? t[h * nmax + c] : czero<T>();
            if (has_n) {
#pragma unroll
              for (int dyi = 1; dyi <= P; ++dyi) {
                const int dy = fwd ? -dyi : dyi;
                const int bb = bc + dy;
                if (bb < bb_lo || bb > bb_hi) continue;
                const V2<T>* ynr = yn + h * nmax + (bb - P * jn) * Mc;
#pragma unroll
                for (int dx = -P; dx <= P; ++dx) {
                  const int aa = ac + dx;
                  if (aa < 0 || aa >= Mc) continue;
                  const V2<T> cf = cc[(dy + P) * W + dx + P];
                  const V2<T> v = ynr[aa];
                  if (fwd) {
                    acc.x -= cf.x * v.x - cf.y * v.y;
                    acc.y -= cf.x * v.y + cf.y * v.x;
                  } else {
                    cfma(acc, cf, v);
                  }
                }
              }
            }
            t[h * nmax + c] = acc;
          }
        }
    }
    __syncthreads();
    // 2. rows [r0, r1) of S_j t in chunks of RCH rows
    int njs, r0, r1, c0, c1;
    const V2<T>* Sj;
    step_rows(s, njs, r0, r1, c0, c1, Sj);
    const int qn = wave > 0 ? (c1 - c0 + 63) / 64 : 0;
    const bool pre = have;   // sv was prefetched for this step
    have = false;
    for (int rb = r0; rb < r1; rb += RCH) {
      if (wave > 0) {
        T ar[RCH][NR], ai[RCH][NR];
#pragma unroll
        for (int rr = 0; rr < RCH; ++rr)
#pragma unroll
          for (int h = 0; h < NR; ++h) { ar[rr][h] = T(0); ai[rr][h] = T(0); }
        for (int q0 = 0; q0 < qn; q0 += QCH) {
          if (!(pre && rb == r0 && q0 == 0)) load_chunk(Sj, nj, rb, r1, c0, c1, q0);
#pragma unroll
          for (int q = 0; q < QCH; ++q) {
            const int c = c0 + lane + 64 * (q0 + q);
            if (c >= c1) continue;
#pragma unroll
            for (int h = 0; h < NR; ++h) {
              if (h >= nrhs) continue;
              const V2<T> tv = t[h * nmax + c];
#pragma unroll
              for (int rr = 0; rr < RCH; ++rr) {
                ar[rr][h] += sv[rr][q].x * tv.x - sv[rr][q].y * tv.y;
                ai[rr][h] += sv[rr][q].x * tv.y + sv[rr][q].y * tv.x;
              }
            }
          }
        }
        // prefetch the first chunk of the next step as soon as this one is consumed
        if (rb + RCH >= r1 && s + 1 < s_end) {
          int nj2, r02, r12, c02, c12;
          const V2<T>* Sj2;
          step_rows(s + 1, nj2, r02, r12, c02, c12, Sj2);
          load_chunk(Sj2, nj2, r02, r12, c02, c12, 0);
          have = true;
        }
#pragma unroll
        for (int rr = 0; rr < RCH; ++rr)
#pragma unroll
          for (int h = 0; h < NR; ++h) {
            const T sr = wave_sum(ar[rr][h]), si = wave_sum(ai[rr][h]);
            if (lane == 0) { red[0][wave - 1][rr][h] = sr; red[1][wave - 1][rr][h] = si; }
          }
      }
      __syncthreads();
      if (threadIdx.x < RCH * NR) {
        const int rr = threadIdx.x / NR, h = threadIdx.x % NR;
        const int r = rb + rr;
        if (r < r1 && h < nrhs) {
          const T sr = (red[0][0][rr][h] + red[0][1][rr][h]) + red[0][2][rr][h];
          const T si = (red[1][0][rr][h] + red[1][1][rr][h]) + red[1][2][rr][h];
          V2<T> o;
          if (fwd) {
            o.x = sr;
            o.y = si;
            st_coh<T>(gbuf + h * Nc + dof0 + r, o);
          } else {
            o = ld_coh<T>(gbuf + h * Nc + dof0 + r);
            o.x -= sr;
            o.y -= si;
            st_coh<T>(y + h * cstride + dof0 + r, o);
          }
        }
      }
      __syncthreads();
    }
  }
}

// Copies the forward result of the last block into the solution (x_{nc} = g_{nc}).
template <typename T>
__global__ void k_copy_last(const V2<T>* __restrict__ gbuf, V2<T>* __restrict__ y, long off,
                            long n, long Nc, long cstride, int nrhs) {
  const long i = long(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  for (int h = 0; h < nrhs; ++h) y[h * cstride + off + i] = gbuf[h * Nc + off + i];
}

template <int P, typename T, int NR, int RCH, int QCH>
void csolve_launch(const CoarseLayout& L, const DevOp<T>& cop, const V2<T>* S, const V2<T>* b,
                   V2<T>* y, int nrhs, long cstride, const CoarseSolveWork& w, hipStream_t st) {
  auto kern = k_csolve<P, T, NR, RCH, QCH>;
  const int nb = L.nblocks();
  const int nsteps = 2 * nb - 1;
  constexpr int NCOEF = P * P * 9 * (2 * P + 1) * (2 * P + 1);
  const size_t lds = (NCOEF + 2 * size_t(L.size(0)) * NR) * sizeof(V2<T>);
  // dynamic LDS beyond the default limit must be requested; the static part counts too
  static size_t configured = 0;
  if (lds > 48 * 1024 && lds > configured) {
    HZ_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                               int(lds)));
    configured = lds;
  }
  int dev = 0;
  HZ_HIP(hipGetDevice(&dev));
  int cus = 0, coop = 0;
  HZ_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  HZ_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
  int per_cu = 0;
  HZ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)kern, 256, lds));
  const int max_coresident = per_cu * cus;
  // balanced grid: R rows per workgroup, one workgroup per compute unit at most
  const int n0 = int(L.size(0));
  const int R = (n0 + cus - 1) / cus;
  int G = (n0 + R - 1) / R;
  const bool persistent = coop && w.persistent && max_coresident >= G && G > 0;
  int s_begin = 0, s_end = nsteps;
  V2<T>* gbuf = reinterpret_cast<V2<T>*>(w.g);
  int* err = w.err;
  int nr = nrhs;
  const long Nc = long(L.Mc) * L.Mc;
  const unsigned fb = unsigned((Nc + 255) / 256);
  k_fill_sentinel<T><<<fb, 256, 0, st>>>(gbuf, Nc, Nc, nrhs);
  k_fill_sentinel<T><<<fb, 256, 0, st>>>(y, Nc, cstride, nrhs);
  if (persistent) {
    void* args[] = {&s_begin, &s_end, (void*)&L.nc, (void*)&L.Mc, (void*)&cop.coef, (void*)&S,
                    (void*)&b, (void*)&y, &gbuf, &nr, (void*)&cstride, &err};
    HZ_HIP(hipLaunchCooperativeKernel((const void*)kern, dim3(G), dim3(256), args, lds, st));
  } else {
    for (int s = 0; s < nsteps; ++s)
      kern<<<G, 256, lds, st>>>(s, s + 1, L.nc, L.Mc, cop.coef, S, b, y, gbuf, nrhs, cstride, err);
  }
  const long off = long(L.p) * L.nc * L.Mc;
  k_copy_last<T><<<unsigned((L.Mc + 255) / 256), 256, 0, st>>>(gbuf, y, off, L.Mc, Nc, cstride, nrhs);
  HZ_HIP(hipGetLastError());
}

template <int P, typename T>
void csolve_p(const CoarseLayout& L, const DevOp<T>& cop, const V2<T>* S, const V2<T>* b, V2<T>* y,
              int nrhs, long cstride, const CoarseSolveWork& w, hipStream_t st) {
  if (nrhs == 1) {
    csolve_launch<P, T, 1, 5, 8>(L, cop, S, b, y, 1, cstride, w, st);
    return;
  }
  for (int r0 = 0; r0 < nrhs; r0 += 4) {
    const int nr = std::min(4, nrhs - r0);
    csolve_launch<P, T, 4, 2, 8>(L, cop, S, b + r0 * cstride, y + r0 * cstride, nr, cstride, w, st);
  }
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
                  V2<T>* y, int nrhs, long cstride, const CoarseSolveWork& w, hipStream_t st) {
  if (L.p == 1) csolve_p<1, T>(L, cop, S, b, y, nrhs, cstride, w, st);
  else if (L.p == 2) csolve_p<2, T>(L, cop, S, b, y, nrhs, cstride, w, st);
  else csolve_p<3, T>(L, cop, S, b, y, nrhs, cstride, w, st);
}

void launch_factor_to_f32(const double2* S, float2* Sf, size_t n, hipStream_t st) {
  k_factor_to_f32<<<unsigned((n + 255) / 256), 256, 0, st>>>(S, Sf, n);
  HZ_HIP(hipGetLastError());
}

template void coarse_solve<double>(const CoarseLayout&, const DevOp<double>&, const double2*,
                                   const double2*, double2*, int, long, const CoarseSolveWork&,
                                   hipStream_t);
template void coarse_solve<float>(const CoarseLayout&, const DevOp<float>&, const float2*,
                                  const float2*, float2*, int, long, const CoarseSolveWork&,
                                  hipStream_t);

}  // namespace hz
