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
// Blocked Gauss-Jordan inversion, in place. One panel K = [k0, k0 + w), w <= NB = 32, with
// Pinv = X[K,K]^{-1} and W[i,:] = X[i,K] Pinv:
//   X[K,K] <- Pinv,   X[i,K] <- -W[i,:],   X[K,j] <- Pinv X[K,j],   X[i,j] <- X[i,j] - W[i,:] X[K,j]
// for i, j outside K. Panels and 32 x 32 tiles are aligned, so every tile of the update is
// entirely in the pivot rows, the pivot columns, or neither (no cancellation-prone forms).
// The panel kernel writes Wt (rows outside K: W, rows in K: Pinv) and Rt = X[K, :].
// ------------------------------------------------------------------------------------------

__global__ void __launch_bounds__(256)
k_gj_panel(const double2* __restrict__ X, int n, int k0, int w, double2* __restrict__ Wt,
           double2* __restrict__ Rt, int* __restrict__ flag) {
  __shared__ double2 Y[2][NB][NB + 1];         // double-buffered Gauss-Jordan on X[K,K]
  __shared__ double2 Xp[32][NB + 1];            // this workgroup's rows of X[:, K]
  const int tid = threadIdx.x;
  const int base = blockIdx.x * 32;
  // coalesced staging, all loads in flight at once: the diagonal panel block, this
  // workgroup's rows of the column panel and its columns of the row panel
  {
    double2 vy[4], vx[4], vr[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = tid + 256 * q;
      const int r = idx / NB, c = idx % NB;
      vy[q] = make_double2(r == c ? 1.0 : 0.0, 0.0);
      if (r < w && c < w) vy[q] = X[size_t(k0 + r) * n + k0 + c];
      const int i = base + r;
      vx[q] = (i < n && c < w) ? X[size_t(i) * n + k0 + c] : make_double2(0, 0);
      const int jj = base + idx % 32, kk = idx / 32;
      vr[q] = (jj < n && kk < w) ? X[size_t(k0 + kk) * n + jj] : make_double2(0, 0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = tid + 256 * q;
      const int r = idx / NB, c = idx % NB;
      Y[0][r][c] = vy[q];
      Xp[r][c] = vx[q];
      const int jj = base + idx % 32, kk = idx / 32;
      if (jj < n) Rt[size_t(kk) * n + jj] = vr[q];
    }
  }
  __syncthreads();
  bool bad = false;
  int cur = 0;
  for (int t = 0; t < w; ++t) {
    const double2 pv = Y[cur][t][t];
    const double mag = pv.x * pv.x + pv.y * pv.y;
    if (!(mag > 0.0) || !isfinite(mag)) bad = true;
    // 1/mag: hardware reciprocal refined by two Newton steps (full double precision)
    double rm = __builtin_amdgcn_rcp(mag);
    rm = rm * (2.0 - mag * rm);
    rm = rm * (2.0 - mag * rm);
    const double2 pinv = make_double2(pv.x * rm, -pv.y * rm);
    double2 yrt[4], ytc[4], yrc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = tid + 256 * q;
      const int r = idx / NB, c = idx % NB;
      yrt[q] = Y[cur][r][t];
      ytc[q] = Y[cur][t][c];
      yrc[q] = Y[cur][r][c];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = tid + 256 * q;
      const int r = idx / NB, c = idx % NB;
      double2 v;
      if (r == t) {
        v = (c == t) ? pinv : cmul<double>(ytc[q], pinv);
      } else if (c == t) {
        const double2 a = cmul<double>(yrt[q], pinv);
        v = make_double2(-a.x, -a.y);
      } else {
        const double2 a = cmul<double>(yrt[q], pinv), b = ytc[q];
        v = yrc[q];
        v.x -= a.x * b.x - a.y * b.y;
        v.y -= a.x * b.y + a.y * b.x;
      }
      Y[cur ^ 1][r][c] = v;
    }
    cur ^= 1;
    __syncthreads();
  }
  if (bad && tid == 0 && blockIdx.x == 0) *flag = 1;
  for (int idx = tid; idx < 32 * NB; idx += 256) {
    const int r = idx / NB, kk = idx % NB;
    const int i = base + r;
    if (i >= n) continue;
    double2 v = make_double2(0, 0);
    if (kk < w) {
      if (i >= k0 && i < k0 + w) {
        v = Y[cur][i - k0][kk];
      } else {
#pragma unroll 8
        for (int t = 0; t < NB; ++t) cfma(v, Xp[r][t], Y[cur][t][kk]);
      }
    }
    Wt[size_t(i) * NB + kk] = v;
  }
}

// Tile update on FP64 MFMA. Each wave owns a 32 x 32 tile (2 x 2 blocks of 16 x 16);
// operands are read straight from the (L2-resident) panels.
// v_mfma_f64_16x16x4: lane l holds A[l%16][l/16], B[l/16][l%16] and D[l/16 + 4r][l%16]
// (r = 0..3; the FP64 layout interleaves rows by 4, checked on the device).
__global__ void __launch_bounds__(256)
k_gj_update(double2* __restrict__ X, int n, int k0, const double2* __restrict__ Wt,
            const double2* __restrict__ Rt) {
  const int lane = threadIdx.x & 63;
  const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int tiles = (n + 31) / 32;
  if (wave >= tiles * tiles) return;
  const int ti = wave / tiles, tj = wave % tiles;
  const int kt = k0 / 32;
  const int i0 = ti * 32, j0 = tj * 32;
  const int li = lane & 15, lk = lane >> 4;
  if (tj == kt) {
    // pivot columns: X[i,K] = -W[i,:] (i outside K), X[K,K] = Pinv
    for (int e = lane; e < 32 * 32; e += 64) {
      const int r = e / 32, c = e % 32;
      const int row = i0 + r, col = j0 + c;
      if (row < n && col < n) {
        double2 v = Wt[size_t(row) * NB + c];
        if (ti != kt) v = make_double2(-v.x, -v.y);
        X[size_t(row) * n + col] = v;
      }
    }
    return;
  }
  const bool pivot_rows = ti == kt;        // X[K,j] = Pinv X[K,j]; else X -= W X[K,j]
  v4d cre[2][2], cim[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = i0 + bi * 16 + lk + 4 * r, col = j0 + bj * 16 + li;
        double2 v = make_double2(0, 0);
        if (!pivot_rows && row < n && col < n) v = X[size_t(row) * n + col];
        cre[bi][bj][r] = v.x;
        cim[bi][bj][r] = v.y;
      }
  const double sg = pivot_rows ? 1.0 : -1.0;
#pragma unroll
  for (int k = 0; k < NB; k += 4) {
    double are[2], aim[2], bre[2], bim[2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) {
      const int row = i0 + bi * 16 + li;
      double2 a = make_double2(0, 0);
      if (row < n) a = Wt[size_t(row) * NB + k + lk];
      are[bi] = sg * a.x;
      aim[bi] = sg * a.y;
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
        // C += (sg a) b: re += are*bre - aim*bim, im += are*bim + aim*bre
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

// 512 threads. Waves 0-1 ("exchange waves") gather the neighbour block (polling until it is
// complete) and the right-hand side into LDS, combine the row sums and publish the results;
// they never hold prefetched data, so their loads are never ordered behind the stream.
// Waves 2-7 ("stream waves") split the columns of the workgroup's rows of S_j: each lane
// forms the coupling values of its own columns from LDS, accumulates partial row sums and,
// right after consuming a chunk, issues the loads of the next block's first chunk into the
// same registers.
constexpr int NSW = 6;   // stream waves

template <int P, typename T, int NR, int RCH, int QCH>
__global__ void __launch_bounds__(512)
k_csolve(int s_begin, int s_end, int nc, int Mc, const V2<T>* __restrict__ coef,
         const V2<T>* __restrict__ S, const V2<T>* __restrict__ b, V2<T>* __restrict__ y,
         V2<T>* __restrict__ gbuf, int nrhs, long cstride, int* __restrict__ err) {
  constexpr int W = 2 * P + 1, W2 = W * W, NCOEF = P * P * 9 * W2;
  constexpr int ENT = 12;                      // polled entries per lane and round
  extern __shared__ char smem[];
  const int nmax = P * Mc;
  V2<T>* cl = reinterpret_cast<V2<T>*>(smem);  // coefficient table
  V2<T>* t = cl + NCOEF;                       // [NR][nmax] right-hand side, then coupling vector
  V2<T>* yn = t + NR * nmax;                   // [NR][nmax] neighbour block
  __shared__ T red[2][NSW][RCH][NR];
  const int nb = nc + 1;
  const int G = gridDim.x, g = blockIdx.x;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int sw = wave - 2;                     // stream wave index (valid for wave >= 2)
  const size_t bsz = size_t(P * Mc) * size_t(P * Mc);
  const long Nc = long(Mc) * Mc;
  for (int i = threadIdx.x; i < NCOEF; i += 512) cl[i] = coef[i];

  V2<T> sv[RCH][QCH];
  bool have = false;                           // sv holds the first chunk of this step

  for (int s = s_begin; s < s_end; ++s) {
    const bool fwd = s < nb;
    const int j = fwd ? s : 2 * nb - 2 - s;
    const int nj = (j < nc ? P : 1) * Mc;
    const long dof0 = long(P) * j * Mc;
    const int jn = fwd ? j - 1 : j + 1;
    const bool has_n = fwd ? j > 0 : j < nc;
    const int nn = has_n ? (jn < nc ? P : 1) * Mc : 0;
    const long ndof0 = long(P) * jn * Mc;
    // backward: x_{nc} is the forward result of the last block (in gbuf)
    const bool from_g = fwd || jn == nc;
    const V2<T>* src = from_g ? gbuf : y;
    const long sstride = from_g ? Nc : cstride;
    // 1a. exchange waves: right-hand side block (forward) and the polled neighbour block
    if (wave < 2) {
      const int xl = threadIdx.x;              // 0..127
      if (fwd)
        for (int idx = xl; idx < nj * nrhs; idx += 128) {
          const int h = idx / nj, c = idx - h * nj;
          t[h * nmax + c] = b[h * cstride + dof0 + c];
        }
      for (int h = 0; h < nrhs; ++h) {
        const V2<T>* sh = src + h * sstride + ndof0;
        V2<T>* yh = yn + h * nmax;
        for (int i0 = 0; i0 < nn; i0 += 128 * ENT) {
          unsigned pending = 0;
#pragma unroll
          for (int q = 0; q < ENT; ++q)
            if (i0 + xl + 128 * q < nn) pending |= 1u << q;
          unsigned rounds = 0;
          while (pending) {
            V2<T> v[ENT];
#pragma unroll
            for (int q = 0; q < ENT; ++q)
              if (pending & (1u << q)) v[q] = ld_coh<T>(sh + i0 + xl + 128 * q);
#pragma unroll
            for (int q = 0; q < ENT; ++q)
              if ((pending & (1u << q)) && !is_sentinel(v[q].x) && !is_sentinel(v[q].y)) {
                yh[i0 + xl + 128 * q] = v[q];
                pending &= ~(1u << q);
              }
            if (pending) {
              ++rounds;
              if ((rounds & 255u) == 0) {
                if (rounds > (1u << 20)) {
                  __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                  break;
                }
                if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
              }
              if (rounds > 8) __builtin_amdgcn_s_sleep(1);
            }
          }
        }
      }
    }
    __syncthreads();
    // 2. rows [r0, r1) of S_j t in chunks of RCH rows; stream wave sw owns columns [c0, c1)
    const int r0 = int((long(nj) * g) / G), r1 = int((long(nj) * (g + 1)) / G);
    const int c0 = (nj * sw) / NSW, c1 = (nj * (sw + 1)) / NSW;
    const V2<T>* Sj = S + size_t(j) * bsz;
    int bb_lo, bb_hi;                          // lattice rows of the neighbour block
    if (fwd) { bb_lo = P * j - P; bb_hi = P * j - 1; }
    else { bb_lo = P * (j + 1); bb_hi = min(P * (j + 1) + P - 1, Mc - 1); }
    const bool pre = have;
    have = false;
    for (int rb = r0; rb < r1; rb += RCH) {
      if (wave >= 2) {
        T ar[RCH][NR], ai[RCH][NR];
#pragma unroll
        for (int rr = 0; rr < RCH; ++rr)
#pragma unroll
          for (int h = 0; h < NR; ++h) { ar[rr][h] = T(0); ai[rr][h] = T(0); }
        const int qn = (c1 - c0 + 63) / 64;
        for (int q0 = 0; q0 < qn; q0 += QCH) {
          if (!(pre && rb == r0 && q0 == 0)) {
#pragma unroll
            for (int rr = 0; rr < RCH; ++rr)
#pragma unroll
              for (int q = 0; q < QCH; ++q) {
                const int c = c0 + lane + 64 * (q0 + q);
                sv[rr][q] = (rb + rr < r1 && c < c1) ? Sj[size_t(rb + rr) * nj + c] : czero<T>();
              }
          }
#pragma unroll
          for (int q = 0; q < QCH; ++q) {
            const int c = c0 + lane + 64 * (q0 + q);
            if (c >= c1) continue;
            // coupling value of column c: t = b_j - A_{j,j-1} g_{j-1} (forward) or
            // A_{j,j+1} x_{j+1} (backward), from the neighbour block staged in LDS
            const int rl = c / Mc, ac = c - rl * Mc;
            const int bc = P * j + rl;
            const V2<T>* cc = cl + (((bc % P) * P + ac % P) * 9 + region(bc, Mc) * 3 + region(ac, Mc)) * W2;
#pragma unroll
            for (int h = 0; h < NR; ++h) {
              if (h >= nrhs) continue;
              V2<T> tv = fwd ? t[h * nmax + c] : czero<T>();
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
                      tv.x -= cf.x * v.x - cf.y * v.y;
                      tv.y -= cf.x * v.y + cf.y * v.x;
                    } else {
                      cfma(tv, cf, v);
                    }
                  }
                }
              }
#pragma unroll
              for (int rr = 0; rr < RCH; ++rr) {
                ar[rr][h] += sv[rr][q].x * tv.x - sv[rr][q].y * tv.y;
                ai[rr][h] += sv[rr][q].x * tv.y + sv[rr][q].y * tv.x;
              }
            }
          }
        }
        // next block's first chunk, issued as soon as this step's last chunk is consumed
        if (rb + RCH >= r1 && s + 1 < s_end) {
          const int s2 = s + 1;
          const bool fwd2 = s2 < nb;
          const int j2 = fwd2 ? s2 : 2 * nb - 2 - s2;
          const int nj2 = (j2 < nc ? P : 1) * Mc;
          const int r02 = int((long(nj2) * g) / G), r12 = int((long(nj2) * (g + 1)) / G);
          const int c02 = (nj2 * sw) / NSW, c12 = (nj2 * (sw + 1)) / NSW;
          const V2<T>* Sj2 = S + size_t(j2) * bsz;
#pragma unroll
          for (int rr = 0; rr < RCH; ++rr)
#pragma unroll
            for (int q = 0; q < QCH; ++q) {
              const int c = c02 + lane + 64 * q;
              sv[rr][q] = (r02 + rr < r12 && c < c12) ? Sj2[size_t(r02 + rr) * nj2 + c] : czero<T>();
            }
          have = true;
        }
#pragma unroll
        for (int rr = 0; rr < RCH; ++rr)
#pragma unroll
          for (int h = 0; h < NR; ++h) {
            const T sr = wave_sum(ar[rr][h]), si = wave_sum(ai[rr][h]);
            if (lane == 0) { red[0][sw][rr][h] = sr; red[1][sw][rr][h] = si; }
          }
      }
      __syncthreads();
      if (threadIdx.x < RCH * NR) {
        const int rr = threadIdx.x / NR, h = threadIdx.x % NR;
        const int r = rb + rr;
        if (r < r1 && h < nrhs) {
          T sr = red[0][0][rr][h], si = red[1][0][rr][h];
#pragma unroll
          for (int w2 = 1; w2 < NSW; ++w2) {
            sr += red[0][w2][rr][h];
            si += red[1][w2][rr][h];
          }
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
  HZ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)kern, 512, lds));
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
    HZ_HIP(hipLaunchCooperativeKernel((const void*)kern, dim3(G), dim3(512), args, lds, st));
  } else {
    for (int s = 0; s < nsteps; ++s)
      kern<<<G, 512, lds, st>>>(s, s + 1, L.nc, L.Mc, cop.coef, S, b, y, gbuf, nrhs, cstride, err);
  }
  const long off = long(L.p) * L.nc * L.Mc;
  k_copy_last<T><<<unsigned((L.Mc + 255) / 256), 256, 0, st>>>(gbuf, y, off, L.Mc, Nc, cstride, nrhs);
  HZ_HIP(hipGetLastError());
}

template <int P, typename T>
void csolve_p(const CoarseLayout& L, const DevOp<T>& cop, const V2<T>* S, const V2<T>* b, V2<T>* y,
              int nrhs, long cstride, const CoarseSolveWork& w, hipStream_t st) {
  if (nrhs == 1) {
    csolve_launch<P, T, 1, 5, 4>(L, cop, S, b, y, 1, cstride, w, st);
    return;
  }
  for (int r0 = 0; r0 < nrhs; r0 += 4) {
    const int nr = std::min(4, nrhs - r0);
    csolve_launch<P, T, 4, 2, 4>(L, cop, S, b + r0 * cstride, y + r0 * cstride, nr, cstride, w, st);
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
      k_gj_panel<<<(n + 31) / 32, 256, 0, st>>>(D, n, k0, wdt, w.W, w.R, w.flag);
      k_gj_update<<<upd_blocks, 256, 0, st>>>(D, n, k0, w.W, w.R);
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
