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

#include <map>
#include <mutex>
#include <stdexcept>
#include <type_traits>

#include "hz_common.h"

namespace hz {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));


__device__ __forceinline__ int region(int a, int M) { return a == 0 ? 0 : (a == M - 1 ? 2 : 1); }

__device__ __forceinline__ double2 crecip(double2 a) {
  const double d = a.x * a.x + a.y * a.y;
  return make_double2(a.x / d, -a.y / d);
}

// ------------------------------------------------------------------------------------------
// Schur complement assembly
// ------------------------------------------------------------------------------------------

// Schur complement of block j against one neighbour block jn = j -/+ 1 (its inverse Sn is
// stored): D_j -= A_{j,jn} Sn A_{jn,j}, done in two sparse-dense passes.
// Tm[r'][c] = sum_{c' in block jn} Sn[r'][c'] A[c'][c],  c in block j. A is symmetric, so
// A[c'][c] is the coefficient of the stencil of c at offset c' - c.
// Stencil of coarse point (a, b): the class table row, or with per-point operators (pn) the
// point's own entries at stride Nc; entry (dy, dx) is at cc[((dy + P) W + dx + P) * stride].
template <int P>
__device__ __forceinline__ const double2* stencil_of(const double2* coef, int pn, int a, int b,
                                                     int Mc, long& stride) {
  constexpr int W = 2 * P + 1, W2 = W * W;
  if (pn) {
    stride = long(Mc) * Mc;
    return coef + long(b) * Mc + a;
  }
  stride = 1;
  const int cls = (b % P) * P + (a % P);
  const int reg = region(b, Mc) * 3 + region(a, Mc);
  return coef + (cls * 9 + reg) * W2;
}

template <int P>
__global__ void __launch_bounds__(256)
k_schur_right(int j, int jn, int nc, int Mc, const double2* __restrict__ coef, int pn,
              const double2* __restrict__ Sn, int nn, int ncur, double2* __restrict__ Tm) {
  constexpr int W = 2 * P + 1;
  const int c = blockIdx.x * 256 + threadIdx.x;
  const int rp = blockIdx.y;
  if (c >= ncur) return;
  const int ac = c % Mc, bc = P * j + c / Mc;
  long cs;
  const double2* cc = stencil_of<P>(coef, pn, ac, bc, Mc, cs);
  const double2* srow = Sn + size_t(rp) * nn;
  const int lo = P * jn, hi = P * jn + (jn < nc ? P : 1);   // lattice rows of block jn
  double2 acc = make_double2(0, 0);
#pragma unroll
  for (int dy = -P; dy <= P; ++dy) {
    const int bb = bc + dy;
    if (bb < lo || bb >= hi) continue;
#pragma unroll
    for (int dx = -P; dx <= P; ++dx) {
      const int aa = ac + dx;
      if (aa < 0 || aa >= Mc) continue;
      const double2 cf = cc[((dy + P) * W + dx + P) * cs];
      if (cf.x == 0.0 && cf.y == 0.0) continue;
      cfma(acc, cf, srow[(bb - lo) * Mc + aa]);
    }
  }
  Tm[size_t(rp) * ncur + c] = acc;
}

// D[r][c] = (jn < 0 ? A_jj[r][c] : D[r][c]) - sum_{r' in block jn} A[r][r'] Tm[r'][c].
template <int P>
__global__ void __launch_bounds__(256)
k_schur_left(int j, int jn, int nc, int Mc, const double2* __restrict__ coef, int pn,
             const double2* __restrict__ Tm, int ncur, double2* __restrict__ D) {
  constexpr int W = 2 * P + 1;
  const int c = blockIdx.x * 256 + threadIdx.x;
  const int r = blockIdx.y;
  if (c >= ncur) return;
  const int ar = r % Mc, br = P * j + r / Mc;
  long cs;
  const double2* cr = stencil_of<P>(coef, pn, ar, br, Mc, cs);
  double2 acc;
  if (jn < 0) {
    acc = make_double2(0, 0);
    const int ac = c % Mc, bc = P * j + c / Mc;
    const int dxa = ac - ar, dya = bc - br;
    if (dxa >= -P && dxa <= P && dya >= -P && dya <= P) acc = cr[((dya + P) * W + dxa + P) * cs];
  } else {
    acc = D[size_t(r) * ncur + c];
    const int lo = P * jn, hi = P * jn + (jn < nc ? P : 1);
#pragma unroll
    for (int dy = -P; dy <= P; ++dy) {
      const int bb = br + dy;
      if (bb < lo || bb >= hi) continue;
#pragma unroll
      for (int dx = -P; dx <= P; ++dx) {
        const int aa = ar + dx;
        if (aa < 0 || aa >= Mc) continue;
        const double2 cf = cr[((dy + P) * W + dx + P) * cs];
        if (cf.x == 0.0 && cf.y == 0.0) continue;
        const double2 tv = Tm[size_t((bb - lo) * Mc + aa) * ncur + c];
        acc.x -= cf.x * tv.x - cf.y * tv.y;
        acc.y -= cf.x * tv.y + cf.y * tv.x;
      }
    }
  }
  D[size_t(r) * ncur + c] = acc;
}

// ------------------------------------------------------------------------------------------
// Block inversion by the symmetric Gauss-Jordan sweep. D_j is complex symmetric (A_eps is,
// and a Schur complement of a complex symmetric matrix with transposed couplings is too), so
// the sweep keeps every intermediate symmetric and only the upper 32 x 32 tiles are updated.
// One pass per pivot tile K (width w <= 32), with P = X[K,K]^{-1} and the pivot row panel
// R[t] = X[K,t] (taken from the upper tile (K,t), or transposed from (t,K) when t < K):
//   X[K,K] <- -P,   X[K,t] <- P R[t],   X[t,K] <- (P R[t])^T,
//   X[i,t] <- X[i,t] - (P R[i])^T R[t]                      for i, t != K.
// After every pivot the block holds -D^{-1}; a final pass negates it and mirrors the upper
// tiles into the lower ones, leaving S = D^{-1} dense and row-major for the solves.
// Without pivoting this is safe for the same reason as the block LU: every leading pivot
// block is a Schur complement of i D, whose Hermitian part is positive definite.
//
// Pass K is one launch. Workgroup 0 already forms the next pass's pivot block
// X[K+1,K+1] - (P R[K+1])^T R[K+1] and inverts it (32 Gauss-Jordan steps in LDS), so that no
// pass waits for a separate panel kernel; the other workgroups update one upper tile per
// wave on FP64 MFMA and write the next pivot row panel as they go. Panels and pivot inverses
// are double-buffered by pass parity.
// ------------------------------------------------------------------------------------------

constexpr int SB = 32;   // tile and pivot panel width

struct SweepPass {
  double2* X;            // the block, row-major n x n
  int n, T;              // size, tiles per side
  int K;                 // pivot tile of this pass
  const double2* Rc;     // this pass's pivot row panel [32][T*32] (zero beyond n)
  double2* Rn;           // the next pass's
  const double2* Pc;     // this pass's pivot inverse, 32 x 32 row-major (zero beyond w)
  double2* Pn;           // the next pass's
  int* flag;             // set on a zero or non-finite pivot
};

// Complex MFMA step C += (sa a) b on 16 x 16 blocks (a, b: this lane's operand values).
__device__ __forceinline__ void cmfma(v4d& cr, v4d& ci, double2 a, double2 b, double sa) {
  cr = __builtin_amdgcn_mfma_f64_16x16x4f64(sa * a.x, b.x, cr, 0, 0, 0);
  cr = __builtin_amdgcn_mfma_f64_16x16x4f64(-sa * a.y, b.y, cr, 0, 0, 0);
  ci = __builtin_amdgcn_mfma_f64_16x16x4f64(sa * a.x, b.y, ci, 0, 0, 0);
  ci = __builtin_amdgcn_mfma_f64_16x16x4f64(sa * a.y, b.x, ci, 0, 0, 0);
}

// Rs = P R[t] for the 16 x 16 output blocks (bp, bq), bq in [BQ0, BQ1). Lane l of block
// (bp, bq) holds Rs[16 bp + l/16 + 4 r][16 bq + l%16] in register r (the FP64 MFMA output
// layout), which is also the A-operand layout of Rs^T for the k-step 16 bp + 4 r.
template <int BQ0, int BQ1>
__device__ __forceinline__ void sweep_pr(const SweepPass& a, int t, v4d (&sr)[2][2],
                                         v4d (&si)[2][2]) {
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  const int ld = a.T * SB;
#pragma unroll
  for (int bp = 0; bp < 2; ++bp)
#pragma unroll
    for (int bq = BQ0; bq < BQ1; ++bq) { sr[bp][bq] = v4d{0, 0, 0, 0}; si[bp][bq] = v4d{0, 0, 0, 0}; }
#pragma unroll
  for (int k0 = 0; k0 < SB; k0 += 4) {
    double2 av[2], bv[2];
#pragma unroll
    for (int bp = 0; bp < 2; ++bp) av[bp] = a.Pc[(16 * bp + li) * SB + k0 + lk];
#pragma unroll
    for (int bq = BQ0; bq < BQ1; ++bq) bv[bq] = a.Rc[size_t(k0 + lk) * ld + t * SB + 16 * bq + li];
#pragma unroll
    for (int bp = 0; bp < 2; ++bp)
#pragma unroll
      for (int bq = BQ0; bq < BQ1; ++bq) cmfma(sr[bp][bq], si[bp][bq], av[bp], bv[bq], 1.0);
  }
}

// C -= Rs^T R[tj] for output blocks (bm, bn), bm in [BM0, BM1), bn in [BN0, BN1); Rs blocks
// (., bm) as left by sweep_pr.
template <int BM0, int BM1, int BN0, int BN1>
__device__ __forceinline__ void sweep_upd(const SweepPass& a, int tj, const v4d (&sr)[2][2],
                                          const v4d (&si)[2][2], v4d (&cr)[2][2],
                                          v4d (&ci)[2][2]) {
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  const int ld = a.T * SB;
#pragma unroll
  for (int k0 = 0; k0 < SB; k0 += 4) {
    double2 bv[2];
#pragma unroll
    for (int bn = BN0; bn < BN1; ++bn) bv[bn] = a.Rc[size_t(k0 + lk) * ld + tj * SB + 16 * bn + li];
#pragma unroll
    for (int bm = BM0; bm < BM1; ++bm) {
      const double2 av = make_double2(sr[k0 >> 4][bm][(k0 >> 2) & 3], si[k0 >> 4][bm][(k0 >> 2) & 3]);
#pragma unroll
      for (int bn = BN0; bn < BN1; ++bn) cmfma(cr[bm][bn], ci[bm][bn], av, bv[bn], -1.0);
    }
  }
}

// Loads the upper tile (ti, tj) into the MFMA output layout (zero beyond n). A diagonal
// tile is read from its upper triangle only (mirrored), so that every matrix the sweep works
// on is exactly symmetric: rounding differences between the two triangles of the diagonal
// tiles would otherwise be amplified from block to block along the factorisation chain.
__device__ __forceinline__ void sweep_load(const SweepPass& a, int ti, int tj, v4d (&cr)[2][2],
                                           v4d (&ci)[2][2]) {
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int bm = 0; bm < 2; ++bm)
#pragma unroll
    for (int bn = 0; bn < 2; ++bn)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int row = ti * SB + 16 * bm + lk + 4 * r, col = tj * SB + 16 * bn + li;
        if (row > col) { const int q = row; row = col; col = q; }   // diagonal tiles only
        double2 v = make_double2(0, 0);
        if (row < a.n && col < a.n) v = a.X[size_t(row) * a.n + col];
        cr[bm][bn][r] = v.x;
        ci[bm][bn][r] = v.y;
      }
}

// Inverts the w x w leading part of the 32 x 32 block in Y[0] by w Gauss-Jordan sweep steps
// (the rest is the identity) and writes P = its inverse (zero outside w x w) to dst. The
// block is first made exactly symmetric from its upper triangle, and P is written from the
// upper triangle of the result. 256 threads, double-buffered LDS, one barrier per step.
__device__ void sweep_invert(double2 (*Y)[SB][SB + 1], int w, double2* __restrict__ dst,
                             int* flag) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int idx = tid + 256 * q, r = idx / SB, c = idx % SB;
    if (r > c) Y[0][r][c] = Y[0][c][r];
  }
  __syncthreads();
  bool bad = false;
  int cur = 0;
  for (int t = 0; t < w; ++t) {
    const double2 pv = Y[cur][t][t];
    const double mag = pv.x * pv.x + pv.y * pv.y;
    if (!(mag > 0.0) || !isfinite(mag)) bad = true;
    // 1/mag: hardware reciprocal refined by two Newton steps (full double precision; shorter
    // than the IEEE division sequence on the step's critical path)
    double rm = __builtin_amdgcn_rcp(mag);
    rm = rm * (2.0 - mag * rm);
    rm = rm * (2.0 - mag * rm);
    const double2 pinv = make_double2(pv.x * rm, -pv.y * rm);
    double2 yrt[4], ytc[4], yrc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = tid + 256 * q, r = idx / SB, c = idx % SB;
      yrt[q] = Y[cur][r][t];
      ytc[q] = Y[cur][t][c];
      yrc[q] = Y[cur][r][c];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = tid + 256 * q, r = idx / SB, c = idx % SB;
      double2 v;
      if (r == t) {
        v = (c == t) ? make_double2(-pinv.x, -pinv.y) : cmul<double>(ytc[q], pinv);
      } else if (c == t) {
        v = cmul<double>(yrt[q], pinv);
      } else {
        const double2 g = cmul<double>(yrt[q], pinv);
        v = yrc[q];
        v.x -= g.x * ytc[q].x - g.y * ytc[q].y;
        v.y -= g.x * ytc[q].y + g.y * ytc[q].x;
      }
      Y[cur ^ 1][r][c] = v;
    }
    cur ^= 1;
    __syncthreads();
  }
  if (bad) atomicOr(flag, 1);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int idx = tid + 256 * q, r = idx / SB, c = idx % SB;
    const double2 v = Y[cur][min(r, c)][max(r, c)];
    dst[idx] = (r < w && c < w) ? make_double2(-v.x, -v.y) : make_double2(0, 0);
  }
}

// Before the first pass: the pivot row panel of tile 0 (workgroups 1..T) and the inverse of
// the first pivot block (workgroup 0).
__device__ __forceinline__ void sweep_first_body(const SweepPass& a) {
  __shared__ double2 Y[2][SB][SB + 1];
  const int tid = threadIdx.x;
  const int ld = a.T * SB;
  if (blockIdx.x == 0) {
    const int w = min(SB, a.n);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = tid + 256 * q, r = idx / SB, c = idx % SB;
      Y[0][r][c] = (r < w && c < w) ? a.X[size_t(r) * a.n + c]
                                    : make_double2(r == c ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    sweep_invert(Y, w, a.Pn, a.flag);
    return;
  }
  const int t = blockIdx.x - 1;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int idx = tid + 256 * q, r = idx / SB, c = idx % SB;
    const int col = t * SB + c;
    a.Rn[size_t(r) * ld + col] = (r < a.n && col < a.n) ? a.X[size_t(r) * a.n + col]
                                                        : make_double2(0, 0);
  }
}

// One pass of the sweep (pivot tile K). Workgroup 0 prepares the next pass's pivot inverse;
// every other wave owns one upper tile (ti <= tj).
__device__ __forceinline__ void sweep_pass_body(const SweepPass& a) {
  __shared__ double2 Y[2][SB][SB + 1];
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  const int wave = threadIdx.x >> 6;
  const int K = a.K, T = a.T, n = a.n, ld = T * SB;
  if (blockIdx.x == 0) {
    if (K + 1 >= T) return;
    // X[K+1,K+1] - (P R[K+1])^T R[K+1]: wave w forms output block (w/2, w%2)
    const int t1 = K + 1;
    v4d sr[2][2], si[2][2], cr[2][2], ci[2][2];
    sweep_load(a, t1, t1, cr, ci);
    const int bm = wave >> 1, bn = wave & 1;
    if (bm == 0) sweep_pr<0, 1>(a, t1, sr, si); else sweep_pr<1, 2>(a, t1, sr, si);
    if (bm == 0 && bn == 0) sweep_upd<0, 1, 0, 1>(a, t1, sr, si, cr, ci);
    else if (bm == 0) sweep_upd<0, 1, 1, 2>(a, t1, sr, si, cr, ci);
    else if (bn == 0) sweep_upd<1, 2, 0, 1>(a, t1, sr, si, cr, ci);
    else sweep_upd<1, 2, 1, 2>(a, t1, sr, si, cr, ci);
    const int w = min(SB, n - t1 * SB);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = 16 * bm + lk + 4 * r, c = 16 * bn + li;
      const double2 v = make_double2(cr[bm][bn][r], ci[bm][bn][r]);
      Y[0][m][c] = (m < w && c < w) ? v : make_double2(m == c ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    sweep_invert(Y, w, a.Pn, a.flag);
    return;
  }
  // tile of this wave (wave-uniform)
  int u = (blockIdx.x - 1) * 4 + wave;
  const int nu = T * (T + 1) / 2;
  if (u >= nu) return;
  int ti = 0;
  while (u >= T - ti) { u -= T - ti; ++ti; }
  const int tj = ti + u;
  if (ti == K + 1 && tj == K + 1) return;     // replaced by the next pass's pivot inverse
  v4d sr[2][2], si[2][2], cr[2][2], ci[2][2];
  bool transposed = false;                    // the result is Rs^T (pivot column tile)
  if (ti == K && tj == K) {
#pragma unroll
    for (int bm = 0; bm < 2; ++bm)
#pragma unroll
      for (int bn = 0; bn < 2; ++bn)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const double2 v = a.Pc[(16 * bm + lk + 4 * r) * SB + 16 * bn + li];
          cr[bm][bn][r] = -v.x;
          ci[bm][bn][r] = -v.y;
        }
  } else if (ti == K) {
    sweep_pr<0, 2>(a, tj, cr, ci);           // X[K,tj] = P R[tj]
  } else if (tj == K) {
    sweep_pr<0, 2>(a, ti, cr, ci);           // X[ti,K] = (P R[ti])^T
    transposed = true;
  } else {
    sweep_load(a, ti, tj, cr, ci);
    sweep_pr<0, 2>(a, ti, sr, si);
    sweep_upd<0, 2, 0, 2>(a, tj, sr, si, cr, ci);
  }
  // store (rows and columns beyond n are not stored); tiles in the next pivot row or column
  // also go to the next pass's panel: R'[t] = X[K+1, t]
  const bool nrow = ti == K + 1, ncol = tj == K + 1;
#pragma unroll
  for (int bm = 0; bm < 2; ++bm)
#pragma unroll
    for (int bn = 0; bn < 2; ++bn)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double2 v = make_double2(cr[bm][bn][r], ci[bm][bn][r]);
        // element (m, c) of the computed 32 x 32 result; transposed results land at (c, m)
        const int m = 16 * bm + lk + 4 * r, c = 16 * bn + li;
        const int tm = transposed ? c : m, tc = transposed ? m : c;   // position in the tile
        const int row = ti * SB + tm, col = tj * SB + tc;
        if (row < n && col < n) a.X[size_t(row) * n + col] = v;
        if (nrow) a.Rn[size_t(tm) * ld + tj * SB + tc] = v;
        if (ncol) a.Rn[size_t(tc) * ld + ti * SB + tm] = v;
      }
}

// Final pass: S = -X, the upper tiles negated in place and mirrored into the lower ones
// (diagonal tiles from their upper triangle).
__device__ __forceinline__ void sweep_last_body(double2* __restrict__ X, int n, int T) {
  __shared__ double2 L[SB][SB + 1];
  int u = blockIdx.x;
  int ti = 0;
  while (u >= T - ti) { u -= T - ti; ++ti; }
  const int tj = ti + u;
  const int tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int idx = tid + 256 * q, r = idx / SB, c = idx % SB;
    const int row = ti * SB + r, col = tj * SB + c;
    double2 v = make_double2(0, 0);
    if (row < n && col < n) {
      v = X[size_t(row) * n + col];
      v = make_double2(-v.x, -v.y);
    }
    L[r][c] = v;
  }
  __syncthreads();
  if (ti == tj) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = tid + 256 * q, r = idx / SB, c = idx % SB;
      const int row = ti * SB + r, col = tj * SB + c;
      if (row < n && col < n) X[size_t(row) * n + col] = L[min(r, c)][max(r, c)];
    }
    return;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int idx = tid + 256 * q, r = idx / SB, c = idx % SB;
    const int row = ti * SB + r, col = tj * SB + c;
    if (row < n && col < n) X[size_t(row) * n + col] = L[r][c];
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int idx = tid + 256 * q, r = idx / SB, c = idx % SB;
    const int row = tj * SB + r, col = ti * SB + c;
    if (row < n && col < n) X[size_t(row) * n + col] = L[c][r];
  }
}

// The sweep of one block: entry kernels over the bodies above.
__global__ void __launch_bounds__(256) k_sweep_first(SweepPass a) { sweep_first_body(a); }
__global__ void __launch_bounds__(256) k_sweep_pass(SweepPass a) { sweep_pass_body(a); }
__global__ void __launch_bounds__(256) k_sweep_last(double2* __restrict__ X, int n, int T) {
  sweep_last_body(X, n, T);
}

// The pass state of block z of a batch at pivot tile K: the block at base + xoff, its two
// alternating pivot row panels at W + woff and pivot inverses at R + roff.
__device__ __forceinline__ SweepPass sweep_pass_of(const SweepNode& z, double2* base, double2* W,
                                                   double2* R, int K, int* flag) {
  SweepPass a;
  const size_t ld = size_t(z.T) * SB;
  a.X = base + z.xoff;
  a.n = z.n;
  a.T = z.T;
  a.K = K;
  a.Rc = W + z.woff + size_t(K & 1) * SB * ld;
  a.Rn = W + z.woff + size_t((K + 1) & 1) * SB * ld;
  a.Pc = R + z.roff + size_t(K & 1) * SB * SB;
  a.Pn = R + z.roff + size_t((K + 1) & 1) * SB * SB;
  a.flag = flag;
  return a;
}

// Several blocks swept together, block blockIdx.y of the batch; workgroups beyond a block's
// own range (its pass count, tile count) leave at once.
__global__ void __launch_bounds__(256)
k_sweep_first_b(double2* base, double2* W, double2* R, const SweepNode* __restrict__ zs, int* flag) {
  const SweepNode z = zs[blockIdx.y];
  if (int(blockIdx.x) > z.T) return;
  sweep_first_body(sweep_pass_of(z, base, W, R, -1, flag));
}
__global__ void __launch_bounds__(256)
k_sweep_pass_b(double2* base, double2* W, double2* R, const SweepNode* __restrict__ zs, int K,
               int* flag) {
  const SweepNode z = zs[blockIdx.y];
  if (K >= z.T) return;
  if (blockIdx.x > 0 && int(blockIdx.x - 1) * 4 >= z.T * (z.T + 1) / 2) return;
  sweep_pass_body(sweep_pass_of(z, base, W, R, K, flag));
}
__global__ void __launch_bounds__(256)
k_sweep_last_b(double2* base, const SweepNode* __restrict__ zs) {
  const SweepNode z = zs[blockIdx.y];
  if (int(blockIdx.x) >= z.T * (z.T + 1) / 2) return;
  sweep_last_body(base + z.xoff, z.n, z.T);
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

// Result buffers of every job start as sentinels: gbuf (stride n) and y (stride cstride).
template <typename T>
__global__ void k_fill_sentinel(CsJobs<T> jobs, long n, long cstride) {
  const long i = long(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  const CoarseJob<T>* job = &jobs.j[blockIdx.y];
  const T sv = __builtin_bit_cast(T, Sentinel<T>::bits);
  V2<T> v;
  v.x = sv;
  v.y = sv;
  for (int h = 0; h < job->nrhs; ++h) {
    job->gbuf[h * n + i] = v;
    job->y[h * cstride + i] = v;
  }
}

// Twisted block solve. With m = nb / 2, the top chain runs blocks 0 .. m-1 and the bottom
// chain blocks nb-1 .. m+1 (their inverses were formed against j-1 and j+1 respectively):
//   forward   g_j = S_j (b_j - A_{j,j-1} g_{j-1})      (top)
//             h_j = S_j (b_j - A_{j,j+1} h_{j+1})      (bottom)
//   middle    x_m = S_m (b_m - A_{m,m-1} g_{m-1} - A_{m,m+1} h_{m+1})
//   backward  x_j = g_j - S_j A_{j,j+1} x_{j+1}        (top, j = m-1 .. 0)
//             x_j = h_j - S_j A_{j,j-1} x_{j-1}        (bottom, j = m+1 .. nb-1)
// so one solve is 2 F + 1 dependent steps, F = max(m, nb - 1 - m), each moving up to two
// blocks. The first half of the workgroups serves the top chain, the second half the bottom
// chain; all of them share the middle block.
struct StepPlan {
  int active, j, nj, r0, r1;
  int jpre, jfly;          // neighbour coupled in a pre-pass / on the fly (-1: none)
  int fwd, mid;            // fwd: out = S t (gbuf; y for the middle), else out = g_j - S t (y)
};

template <int P>
__device__ __forceinline__ StepPlan make_plan(int s, int g, int G, int nc, int Mc) {
  const int nb = nc + 1, m = nb / 2, nt = m, nbt = nb - 1 - m, F = max(nt, nbt);
  const int Gh = G / 2;
  const bool top = g < Gh;
  const int gl = top ? g : g - Gh;
  StepPlan p;
  p.active = 0; p.j = 0; p.jpre = -1; p.jfly = -1; p.fwd = 1; p.mid = 0;
  if (s < F) {
    if (top ? s < nt : s < nbt) {
      p.active = 1;
      p.j = top ? s : nb - 1 - s;
      p.jfly = top ? (p.j > 0 ? p.j - 1 : -1) : (p.j < nb - 1 ? p.j + 1 : -1);
    }
  } else if (s == F) {
    p.active = 1; p.mid = 1; p.j = m;
    p.jpre = m > 0 ? m - 1 : -1;
    p.jfly = m < nb - 1 ? m + 1 : -1;
  } else {
    const int q = s - F - 1;
    if (top ? q < nt : q < nbt) {
      p.active = 1; p.fwd = 0;
      p.j = top ? m - 1 - q : m + 1 + q;
      p.jfly = top ? p.j + 1 : p.j - 1;
    }
  }
  p.nj = (p.j < nc ? P : 1) * Mc;
  if (!p.active) { p.r0 = p.r1 = 0; }
  else if (p.mid) { p.r0 = int((long(p.nj) * g) / G); p.r1 = int((long(p.nj) * (g + 1)) / G); }
  else { p.r0 = int((long(p.nj) * gl) / Gh); p.r1 = int((long(p.nj) * (gl + 1)) / Gh); }
  return p;
}

// Sum over the couplings of column c of block j into block jn of coef * value (the values of
// block jn staged in LDS, row-major by lattice row).
template <int P, typename T>
__device__ __forceinline__ V2<T> coupling(int c, int j, int jn, int nc, int Mc,
                                          const V2<T>* __restrict__ cl, const V2<T>* yv) {
  constexpr int W = 2 * P + 1, W2 = W * W;
  // c = rl Mc + ac with rl < P (a block holds at most P lattice rows); the class row of
  // lattice row bc = P j + rl is rl
  int rl = 0;
  if constexpr (P >= 2) rl += c >= Mc;
  if constexpr (P >= 3) rl += c >= 2 * Mc;
  const int ac = c - rl * Mc;
  const int bc = P * j + rl;
  const int cls = rl * P + (P == 1 ? 0 : ac % P);
  const int ry = bc == 0 ? 0 : (bc == Mc - 1 ? 2 : 1);
  const int rx = ac == 0 ? 0 : (ac == Mc - 1 ? 2 : 1);
  const V2<T>* cc = cl + ((cls * 9 + ry * 3 + rx) * W2);
  const int lo = P * jn, hi = P * jn + (jn < nc ? P : 1);
  V2<T> acc = czero<T>();
#pragma unroll
  for (int dy = -P; dy <= P; ++dy) {
    const int bb = bc + dy;
    if (bb < lo || bb >= hi) continue;
    const V2<T>* yr = yv + (bb - lo) * Mc;
#pragma unroll
    for (int dx = -P; dx <= P; ++dx) {
      if (P == 1 && !couples(1, 0, 0, dx, dy)) continue;   // the P1 stencil has 7 points
      const int aa = ac + dx;
      if (aa < 0 || aa >= Mc) continue;
      cfma(acc, cc[(dy + P) * W + dx + P], yr[aa]);
    }
  }
  return acc;
}

// The same with per-point coefficients (the coarse point's own stencil, read from global
// memory at stride Nc, offset-major).
template <int P, typename T>
__device__ __forceinline__ V2<T> coupling_pn(int c, int j, int jn, int nc, int Mc,
                                             const V2<T>* __restrict__ coef, const V2<T>* yv) {
  constexpr int W = 2 * P + 1;
  int rl = 0;
  if constexpr (P >= 2) rl += c >= Mc;
  if constexpr (P >= 3) rl += c >= 2 * Mc;
  const int ac = c - rl * Mc;
  const int bc = P * j + rl;
  const long Nc = long(Mc) * Mc;
  const V2<T>* cc = coef + long(bc) * Mc + ac;
  const int lo = P * jn, hi = P * jn + (jn < nc ? P : 1);
  V2<T> acc = czero<T>();
#pragma unroll
  for (int dy = -P; dy <= P; ++dy) {
    const int bb = bc + dy;
    if (bb < lo || bb >= hi) continue;
    const V2<T>* yr = yv + (bb - lo) * Mc;
#pragma unroll
    for (int dx = -P; dx <= P; ++dx) {
      if (P == 1 && !couples(1, 0, 0, dx, dy)) continue;   // the P1 stencil has 7 points
      const int aa = ac + dx;
      if (aa < 0 || aa >= Mc) continue;
      cfma(acc, cc[long((dy + P) * W + dx + P) * Nc], yr[aa]);
    }
  }
  return acc;
}

// Polls lattice block jn of src (right-hand side h at src + h * sstride) until no value is
// the sentinel, staging it into yv[h * nmax + .]; executed by the 128 exchange threads. Entry
// (h, q) of a thread is column c0 + xl + 128 q of right-hand side h: every pending load of a
// slice of 128 * EH columns, for all right-hand sides, is in flight at once.
template <int P, typename T, int NR, int EH>
__device__ __forceinline__ void gather_block(const V2<T>* src, long sstride, int jn, int nc,
                                             int Mc, int nrhs, int nmax, V2<T>* yv, int xl,
                                             int* err) {
  const int nn = (jn < nc ? P : 1) * Mc;
  const long d0 = long(P) * jn * Mc;
  for (int c0 = 0; c0 < nn; c0 += 128 * EH) {
    unsigned long long pending = 0;
#pragma unroll
    for (int h = 0; h < NR; ++h)
#pragma unroll
      for (int q = 0; q < EH; ++q)
        if (h < nrhs && c0 + xl + 128 * q < nn) pending |= 1ull << (h * EH + q);
    unsigned rounds = 0;
    while (pending) {
      V2<T> v[NR][EH];
#pragma unroll
      for (int h = 0; h < NR; ++h)
#pragma unroll
        for (int q = 0; q < EH; ++q)
          if ((pending >> (h * EH + q)) & 1ull)
            v[h][q] = ld_coh<T>(src + h * sstride + d0 + c0 + xl + 128 * q);
#pragma unroll
      for (int h = 0; h < NR; ++h)
#pragma unroll
        for (int q = 0; q < EH; ++q)
          if (((pending >> (h * EH + q)) & 1ull) && !is_sentinel(v[h][q].x) &&
              !is_sentinel(v[h][q].y)) {
            yv[h * nmax + c0 + xl + 128 * q] = v[h][q];
            pending &= ~(1ull << (h * EH + q));
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

// 512 threads. Waves 0-1 ("exchange waves") gather neighbour results (polling) into LDS and
// publish the results; while a step computes they stage the next step's right-hand side
// (or zeros) into the LDS buffer the step no longer needs, so the two buffers swap roles from
// step to step. After a workgroup barrier all eight waves fold the coupling to the neighbour
// block into t. Waves 2-7 ("stream waves") form rows of S_j t: stream wave sw owns row group
// sw / CG (RW rows of each chunk of RG * RW rows) and column half sw % CG, each lane QW
// columns per chunk, so that one chunk covers the block rows of a workgroup and all of its
// factor loads are in flight at once. Factor loads are issued while the waves would wait for
// the exchange: right after the previous step's last chunk was consumed, and where a step is
// one chunk, a part of them two steps ahead. Per row the sum runs over the lane's columns in
// ascending order, then over each row of 16 lanes (row16_sum), then over the column halves
// and the four rows of lanes in order, for any number of right-hand sides.
constexpr int NSW = 6;                 // stream waves
constexpr int CSOL_CG = 2, CSOL_RG = 3, CSOL_RW = 3, CSOL_QW = 9;

// Column groups per chunk requested two steps ahead when a step is one chunk: as many as the
// registers left beside a chunk and the accumulators hold.
template <typename T, int NR>
constexpr bool csolve_one_ok() {   // registers for a chunk, the early columns and start values
  return !(sizeof(T) == 8 && NR >= 4);
}
template <typename T, int NR>
constexpr int csolve_early() {
  return sizeof(T) == 8 ? (NR == 1 ? 6 : 3) : (NR <= 2 ? 9 : 6);
}

template <int P, typename T, int NR>
__global__ void __launch_bounds__(512)
k_csolve(int s_begin, int s_end, int nc, int Mc, int Gp, CsJobs<T> jobs, long cstride,
         int one, int* __restrict__ err) {
  // workgroups [jb Gp, (jb + 1) Gp) serve job jb (one coarse system and its right-hand sides)
  const int jb = blockIdx.x / Gp;
  const CoarseJob<T>* job = &jobs.j[jb];
  const V2<T>* __restrict__ coef = job->coef;
  const V2<T>* __restrict__ S = job->S;
  const V2<T>* __restrict__ b = job->b;
  V2<T>* __restrict__ y = job->y;
  V2<T>* __restrict__ gbuf = job->gbuf;
  const int nrhs = job->nrhs;
  constexpr int W = 2 * P + 1, W2 = W * W, NCOEF = P * P * 9 * W2;
  constexpr int CG = CSOL_CG, RG = CSOL_RG, RW = CSOL_RW, QW = CSOL_QW;
  constexpr int RCH = RG * RW;                 // rows per chunk
  constexpr int EH = (sizeof(T) == 8 && NR >= 4) ? 5 : 9;   // polled columns per thread and slice
  extern __shared__ char smem[];
  const int nmax = P * Mc;
  V2<T>* cl = reinterpret_cast<V2<T>*>(smem);  // coefficient table
  V2<T>* buf0 = cl + NCOEF;                    // two [NR][nmax] buffers: t and neighbour
  V2<T>* buf1 = buf0 + NR * nmax;
  __shared__ T red[2][CG][4][RCH][NR];      // partial row sums per column half and row of 16 lanes
  const int G = Gp, g = blockIdx.x - jb * Gp;
  // wave-uniform (scalar) role index: the two roles run separate code
  const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  const int sw = wave - 2, rg = sw / CG, cg = sw - (sw / CG) * CG;
  const size_t bsz = size_t(P * Mc) * size_t(P * Mc);
  const long Nc = long(Mc) * Mc;
  const int pn = job->pn;   // per-point coefficients: read from global memory, not staged
  if (!pn)
    for (int i = threadIdx.x; i < NCOEF; i += 512) cl[i] = coef[i];

  // exchange waves: dst[h][c] = b_j (forward steps) or 0, c < nj, in slices of 128 EH
  auto stage = [&](const StepPlan& q, V2<T>* dst) __attribute__((always_inline)) {
    const long d0 = long(P) * q.j * Mc;
    for (int c0 = 0; c0 < q.nj; c0 += 128 * EH) {
      V2<T> v[NR][EH];
#pragma unroll
      for (int h = 0; h < NR; ++h)
#pragma unroll
        for (int e = 0; e < EH; ++e) {
          const int c = c0 + threadIdx.x + 128 * e;
          v[h][e] = (q.fwd && h < nrhs && c < q.nj) ? b[h * cstride + d0 + c] : czero<T>();
        }
#pragma unroll
      for (int h = 0; h < NR; ++h)
#pragma unroll
        for (int e = 0; e < EH; ++e) {
          const int c = c0 + threadIdx.x + 128 * e;
          if (h < nrhs && c < q.nj) dst[h * nmax + c] = v[h][e];
        }
    }
  };

  // t += sgn * A_{j,jn} y_jn for every right-hand side; run by all 512 threads (each role
  // calls it from its own loop, so that the two roles never share a code path: a wait for
  // outstanding loads at a shared join would hold the stream waves' prefetch)
  auto fold = [&](const StepPlan& pl, int jn, T sgn, V2<T>* t, const V2<T>* yn)
                  __attribute__((always_inline)) {
    for (int h = 0; h < nrhs; ++h)
      for (int c = threadIdx.x; c < pl.nj; c += 512) {
        const V2<T> cp = pn ? coupling_pn<P, T>(c, pl.j, jn, nc, Mc, coef, yn + h * nmax)
                            : coupling<P, T>(c, pl.j, jn, nc, Mc, cl, yn + h * nmax);
        V2<T> tv = t[h * nmax + c];
        tv.x += sgn * cp.x;
        tv.y += sgn * cp.y;
        t[h * nmax + c] = tv;
      }
  };

  if constexpr (csolve_one_ok<T, NR>()) {
  if (one) {
    // ---------------- every step is one chunk ----------------
    // The exchange waves request a step's start value (b_j or 0) into registers before they
    // poll for its neighbour rows and write it into t once the rows are in; the rows are
    // published by the first stream wave right after the row sums are complete, so the
    // exchange waves only poll. Columns q < QE of a chunk are requested two steps ahead,
    // while the previous step still waits for its neighbour; the other columns once the
    // previous step's product is formed. Early columns of even steps (counted from s_begin)
    // live in B, those of odd steps in A[.][q < QE]; late columns in A[.][q >= QE]. Both
    // roles pass the same barriers in the same order.
    V2<T>* t = buf0;
    V2<T>* yn = buf1;
    // the folds of a step, between the same barriers for both roles
    auto fold_step = [&](const StepPlan& pl, bool exch) __attribute__((always_inline)) {
      if (pl.jpre >= 0) {
        __syncthreads();
        fold(pl, pl.jpre, T(-1), t, yn);
        __syncthreads();
        if (exch && pl.active && pl.jfly >= 0)
          gather_block<P, T, NR, EH>(gbuf, Nc, pl.jfly, nc, Mc, nrhs, nmax, yn, threadIdx.x, err);
      }
      __syncthreads();
      if (pl.active) {
        if (pl.jfly >= 0) fold(pl, pl.jfly, pl.fwd ? T(-1) : T(1), t, yn);
        __syncthreads();
      }
    };
    if (wave < 2) {
      // ---- exchange waves: start values and neighbour rows of each step ----
      constexpr int NRE = NR <= 2 ? NR : 1, EHE = NR <= 2 ? EH : 1;   // registers permitting
      for (int s = s_begin; s < s_end; ++s) {
        const StepPlan pl = make_plan<P>(s, g, G, nc, Mc);
        const long d0 = long(P) * pl.j * Mc;
        V2<T> bv[NRE][EHE];
        if constexpr (NR <= 2) {
#pragma unroll
          for (int h = 0; h < NR; ++h)
#pragma unroll
            for (int e = 0; e < EH; ++e) {
              const int c = threadIdx.x + 128 * e;
              bv[h][e] = (pl.active && pl.fwd && h < nrhs && c < pl.nj)
                             ? b[h * cstride + d0 + c] : czero<T>();
            }
        }
        if (pl.active) {
          if (pl.jpre >= 0)
            gather_block<P, T, NR, EH>(gbuf, Nc, pl.jpre, nc, Mc, nrhs, nmax, yn, threadIdx.x,
                                       err);
          else if (pl.jfly >= 0)
            gather_block<P, T, NR, EH>(pl.fwd ? gbuf : y, pl.fwd ? Nc : cstride, pl.jfly, nc, Mc,
                                       nrhs, nmax, yn, threadIdx.x, err);
          if constexpr (NR <= 2) {
#pragma unroll
            for (int h = 0; h < NR; ++h)
#pragma unroll
              for (int e = 0; e < EH; ++e) {
                const int c = threadIdx.x + 128 * e;
                if (h < nrhs && c < pl.nj) t[h * nmax + c] = bv[h][e];
              }
          } else {
            stage(pl, t);
          }
        }
        fold_step(pl, true);
        __syncthreads();               // the row sums are complete
      }
    } else {
      // ---- stream waves ----
      constexpr int QE = csolve_early<T, NR>();
      V2<T> A[RW][QW];
      V2<T> B[RW][QE > 0 ? QE : 1];
      struct Tile { const V2<T>* Sj; int rw0, r1, nj, c0, c1; };
      auto tile_of = [&](int s2) __attribute__((always_inline)) {
        Tile tl{S, 0, 0, 0, 0, 0};
        if (s2 < s_end) {
          const StepPlan pn = make_plan<P>(s2, g, G, nc, Mc);
          if (pn.active && pn.r1 > pn.r0) {
            tl.Sj = S + size_t(pn.j) * bsz;
            tl.rw0 = pn.r0 + rg * RW;
            tl.r1 = pn.r1;
            tl.nj = pn.nj;
            tl.c0 = (pn.nj * cg) / CG;
            tl.c1 = (pn.nj * (cg + 1)) / CG;
          }
        }
        return tl;
      };
      // the publishing lanes: row rr = lane / NR of the chunk, right-hand side lane % NR
      const bool publisher = sw == 0 && lane < RCH * NR;
      // backwards, the forward result of the row this lane publishes, requested a step ahead
      V2<T> gprev = czero<T>();
      auto gprev_of = [&](int s2) __attribute__((always_inline)) {
        const StepPlan pn = make_plan<P>(s2, g, G, nc, Mc);
        const int r = pn.r0 + lane / NR, h = lane % NR;
        return (publisher && s2 < s_end && pn.active && !pn.fwd && r < pn.r1 && h < nrhs)
                   ? ld_coh<T>(gbuf + h * Nc + long(P) * pn.j * Mc + r) : czero<T>();
      };
#define HZ_LOAD_COLS(DST, QLO, QHI, TL)                                                      \
  _Pragma("unroll") for (int i = 0; i < RW; ++i)                                             \
  _Pragma("unroll") for (int q = QLO; q < QHI; ++q) {                                        \
    const int c = TL.c0 + lane + 64 * q;                                                     \
    DST[i][q] = (TL.rw0 + i < TL.r1 && c < TL.c1) ? TL.Sj[size_t(TL.rw0 + i) * TL.nj + c]    \
                                                   : czero<T>();                             \
  }
      gprev = gprev_of(s_begin);
      {
        const Tile t0 = tile_of(s_begin), t1 = tile_of(s_begin + 1);
        if constexpr (QE > 0) { HZ_LOAD_COLS(B, 0, QE, t0) }
        HZ_LOAD_COLS(A, QE, QW, t0)
        if constexpr (QE > 0) { HZ_LOAD_COLS(A, 0, QE, t1) }
      }
      // one step; the parity of the step decides which registers hold its early columns
      auto step = [&](int s, auto even_c) __attribute__((always_inline)) {
        constexpr bool EVEN = decltype(even_c)::value;
        const StepPlan pl = make_plan<P>(s, g, G, nc, Mc);
        const int nj = pl.nj;
        fold_step(pl, false);
        const int r0 = pl.r0, r1 = pl.r1;
        const int pr = r0 + lane / NR, ph = lane % NR;
        const bool pub = publisher && pr < r1 && ph < nrhs;
        if (r1 > r0) {
          const int c0 = (nj * cg) / CG, c1 = (nj * (cg + 1)) / CG;
          T ar[RW][NR], ai[RW][NR];
#pragma unroll
          for (int i = 0; i < RW; ++i)
#pragma unroll
            for (int h = 0; h < NR; ++h) { ar[i][h] = T(0); ai[i][h] = T(0); }
#pragma unroll
          for (int q = 0; q < QW; ++q) {
            const int c = c0 + lane + 64 * q;
            if (c >= c1) continue;
#pragma unroll
            for (int h = 0; h < NR; ++h) {
              if (h >= nrhs) continue;
              const V2<T> tv = t[h * nmax + c];
#pragma unroll
              for (int i = 0; i < RW; ++i) {
                const V2<T> sv = (EVEN && q < QE) ? B[i][q < QE ? q : 0] : A[i][q];
                ar[i][h] += sv.x * tv.x - sv.y * tv.y;
                ai[i][h] += sv.x * tv.y + sv.y * tv.x;
              }
            }
          }
#pragma unroll
          for (int i = 0; i < RW; ++i)
#pragma unroll
            for (int h = 0; h < NR; ++h) {
              const T sr = row16_sum(ar[i][h]), si = row16_sum(ai[i][h]);
              if ((lane & 15) == 0) {
                red[0][cg][lane >> 4][rg * RW + i][h] = sr;
                red[1][cg][lane >> 4][rg * RW + i][h] = si;
              }
            }
        }
        __syncthreads();                 // the row sums are complete
        if (pub) {
          const int rr = lane / NR;
          T sr = red[0][0][0][rr][ph], si = red[1][0][0][rr][ph];
#pragma unroll
          for (int k = 0; k < CG; ++k)
#pragma unroll
            for (int u = (k == 0 ? 1 : 0); u < 4; ++u) {
              sr += red[0][k][u][rr][ph];
              si += red[1][k][u][rr][ph];
            }
          // forward rows go to gbuf (the middle block's straight to y); backward rows are
          // the forward result minus the sum
          V2<T> o;
          o.x = pl.fwd ? sr : gprev.x - sr;
          o.y = pl.fwd ? si : gprev.y - si;
          V2<T>* dst = (pl.fwd && !pl.mid) ? gbuf + ph * Nc : y + ph * cstride;
          st_coh<T>(dst + long(P) * pl.j * Mc + pr, o);
        }
        // requests for the steps ahead, issued while the exchange waves poll: the next
        // step's forward result, the late columns of the next step and the early columns of
        // the one after, into the registers this step freed
        gprev = gprev_of(s + 1);
        {
          const Tile tn = tile_of(s + 1);
          HZ_LOAD_COLS(A, QE, QW, tn)
        }
        if constexpr (QE > 0) {
          const Tile tnn = tile_of(s + 2);
          if constexpr (EVEN) { HZ_LOAD_COLS(B, 0, QE, tnn) } else { HZ_LOAD_COLS(A, 0, QE, tnn) }
        }
      };
#undef HZ_LOAD_COLS
      for (int s = s_begin; s < s_end; s += 2) {
        step(s, std::true_type{});
        if (s + 1 < s_end) step(s + 1, std::false_type{});
      }
    }
    return;
  }
  }
  if (wave < 2) {
    // ---------------- exchange waves ----------------
    bool staged = false;             // t already holds this step's start value
    int par = 0;
    for (int s = s_begin; s < s_end; ++s) {
      const StepPlan pl = make_plan<P>(s, g, G, nc, Mc);
      const int j = pl.j;
      const long dof0 = long(P) * j * Mc;
      V2<T>* t = par ? buf1 : buf0;
      V2<T>* yn = par ? buf0 : buf1;
      // t = b_j (forward, middle) or 0 (backward) unless staged during the previous step;
      // the middle step couples two neighbours, the first folded between two barriers
      if (pl.active) {
        if (!staged) stage(pl, t);
        if (pl.jpre >= 0)
          gather_block<P, T, NR, EH>(gbuf, Nc, pl.jpre, nc, Mc, nrhs, nmax, yn, threadIdx.x, err);
      }
      if (pl.jpre >= 0) {
        __syncthreads();
        fold(pl, pl.jpre, T(-1), t, yn);
        __syncthreads();
      }
      if (pl.active && pl.jfly >= 0) {
        const bool from_g = pl.fwd;          // forward/middle neighbours are in gbuf
        gather_block<P, T, NR, EH>(from_g ? gbuf : y, from_g ? Nc : cstride, pl.jfly, nc, Mc,
                                   nrhs, nmax, yn, threadIdx.x, err);
      }
      __syncthreads();
      if (pl.active && pl.jfly >= 0) {
        fold(pl, pl.jfly, pl.fwd ? T(-1) : T(1), t, yn);
        __syncthreads();
      }
      // the neighbour buffer is free: stage the next step's start value into it
      staged = false;
      if (s + 1 < s_end) {
        const StepPlan pn = make_plan<P>(s + 1, g, G, nc, Mc);
        if (pn.active) {
          stage(pn, yn);
          staged = true;
        }
      }
      // combine the stream waves' partial row sums and publish the rows
      for (int rb = pl.r0; rb < pl.r1; rb += RCH) {
        __syncthreads();
        if (threadIdx.x < RCH * NR) {
          const int rr = threadIdx.x / NR, h = threadIdx.x % NR;
          const int r = rb + rr;
          if (r < pl.r1 && h < nrhs) {
            T sr = red[0][0][0][rr][h], si = red[1][0][0][rr][h];
#pragma unroll
            for (int k = 0; k < CG; ++k)
#pragma unroll
              for (int u = (k == 0 ? 1 : 0); u < 4; ++u) {
                sr += red[0][k][u][rr][h];
                si += red[1][k][u][rr][h];
              }
            V2<T> o;
            if (pl.fwd) {
              o.x = sr;
              o.y = si;
              st_coh<T>((pl.mid ? y + h * cstride : gbuf + h * Nc) + dof0 + r, o);
            } else {
              o = ld_coh<T>(gbuf + h * Nc + dof0 + r);
              o.x -= sr;
              o.y -= si;
              st_coh<T>(y + h * cstride + dof0 + r, o);
            }
          }
        }
        // red is rewritten by the next chunk; after the last chunk the next write to red
        // comes after this step's successor has passed two more barriers
        if (rb + RCH < pl.r1) __syncthreads();
      }
      // a step without rows of this workgroup still needs the staged buffer to be complete
      if (pl.r1 <= pl.r0) __syncthreads();
      par ^= 1;
    }
  } else {
    // ---------------- stream waves ----------------
    V2<T> sv[RW][QW];                  // factor entries of a chunk
    bool have = false;                 // sv holds the first chunk of this step
    int par = 0;
    for (int s = s_begin; s < s_end; ++s) {
      const StepPlan pl = make_plan<P>(s, g, G, nc, Mc);
      const int j = pl.j, nj = pl.nj;
      V2<T>* t = par ? buf1 : buf0;
      V2<T>* yn = par ? buf0 : buf1;
      if (pl.jpre >= 0) {
        __syncthreads();
        fold(pl, pl.jpre, T(-1), t, yn);
        __syncthreads();
      }
      __syncthreads();
      if (pl.active && pl.jfly >= 0) {
        fold(pl, pl.jfly, pl.fwd ? T(-1) : T(1), t, yn);
        __syncthreads();
      }
      // rows [r0, r1) of S_j t in chunks of RCH rows
      const int r0 = pl.r0, r1 = pl.r1;
      const int c0 = (nj * cg) / CG, c1 = (nj * (cg + 1)) / CG;
      const V2<T>* Sj = S + size_t(j) * bsz;
      const bool pre = have;
      have = false;
      for (int rb = r0; rb < r1; rb += RCH) {
        const int rw0 = rb + rg * RW;
        T ar[RW][NR], ai[RW][NR];
#pragma unroll
        for (int i = 0; i < RW; ++i)
#pragma unroll
          for (int h = 0; h < NR; ++h) { ar[i][h] = T(0); ai[i][h] = T(0); }
        const int qn = (c1 - c0 + 63) / 64;
        for (int q0 = 0; q0 < qn; q0 += QW) {
          if (!(pre && rb == r0 && q0 == 0)) {
#pragma unroll
            for (int i = 0; i < RW; ++i)
#pragma unroll
              for (int q = 0; q < QW; ++q) {
                const int c = c0 + lane + 64 * (q0 + q);
                sv[i][q] = (rw0 + i < r1 && c < c1) ? Sj[size_t(rw0 + i) * nj + c] : czero<T>();
              }
          }
#pragma unroll
          for (int q = 0; q < QW; ++q) {
            const int c = c0 + lane + 64 * (q0 + q);
            if (c >= c1) continue;
#pragma unroll
            for (int h = 0; h < NR; ++h) {
              if (h >= nrhs) continue;
              const V2<T> tv = t[h * nmax + c];
#pragma unroll
              for (int i = 0; i < RW; ++i) {
                ar[i][h] += sv[i][q].x * tv.x - sv[i][q].y * tv.y;
                ai[i][h] += sv[i][q].x * tv.y + sv[i][q].y * tv.x;
              }
            }
          }
        }
#pragma unroll
        for (int i = 0; i < RW; ++i)
#pragma unroll
          for (int h = 0; h < NR; ++h) {
            const T sr = row16_sum(ar[i][h]), si = row16_sum(ai[i][h]);
            if ((lane & 15) == 0) {
              red[0][cg][lane >> 4][rg * RW + i][h] = sr;
              red[1][cg][lane >> 4][rg * RW + i][h] = si;
            }
          }
        __syncthreads();                 // the exchange waves combine and publish ...
        const bool last = rb + RCH >= r1;
        // ... while the first chunk of the next step is requested (issuing the loads of a
        // whole chunk takes longer than the exchange, so it stays off the critical path)
        if (last && s + 1 < s_end) {
          const StepPlan pn = make_plan<P>(s + 1, g, G, nc, Mc);
          if (pn.active && pn.r1 > pn.r0) {
            const int nj2 = pn.nj;
            const int c02 = (nj2 * cg) / CG, c12 = (nj2 * (cg + 1)) / CG;
            const int rn0 = pn.r0 + rg * RW;
            const V2<T>* Sj2 = S + size_t(pn.j) * bsz;
#pragma unroll
            for (int i = 0; i < RW; ++i)
#pragma unroll
              for (int q = 0; q < QW; ++q) {
                const int c = c02 + lane + 64 * q;
                sv[i][q] = (rn0 + i < pn.r1 && c < c12) ? Sj2[size_t(rn0 + i) * nj2 + c]
                                                       : czero<T>();
              }
            have = true;
          }
        }
        if (!last) __syncthreads();      // red is rewritten by the next chunk
      }
      if (r1 <= r0) __syncthreads();
      par ^= 1;
    }
  }
}

constexpr size_t kLdsPerWorkgroup = 160 * 1024;   // gfx950

// The persistent solve spins on its peer workgroups, so two of its launches must never be
// resident at once: launches on one device run one after another whatever stream they are
// issued on. Each launch waits for an event recorded after the previous one (one event per
// device, re-recorded under a process-wide lock; a wait binds to the latest record at the
// time of the wait call).
std::mutex& order_mu() {
  static std::mutex m;
  return m;
}
// per device: the event recorded after its latest persistent launch (created on first use,
// or ahead of it by coarse_order_init); guarded by order_mu()
std::map<int, std::pair<hipEvent_t, bool>>& order_events() {
  static std::map<int, std::pair<hipEvent_t, bool>> m;
  return m;
}
std::pair<hipEvent_t, bool>& order_event_locked(int dev) {
  auto& m = order_events();
  auto it = m.find(dev);
  if (it == m.end()) {
    hipEvent_t e = nullptr;
    HZ_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    it = m.emplace(dev, std::make_pair(e, false)).first;
  }
  return it->second;
}
struct PersistentOrder {
  std::unique_lock<std::mutex> lk;
  std::pair<hipEvent_t, bool>* ev = nullptr;
  hipStream_t st;
  PersistentOrder(int dev, hipStream_t s) : lk(order_mu()), st(s) {
    ev = &order_event_locked(dev);
    if (ev->second) HZ_HIP(hipStreamWaitEvent(st, ev->first, 0));
  }
  // after the launch was issued
  ~PersistentOrder() { ev->second = hipEventRecord(ev->first, st) == hipSuccess; }
};

// Dynamic plus static LDS bytes of one k_csolve workgroup.
template <int P, typename T, int NR>
constexpr size_t csolve_lds(int Mc) {
  return (size_t(P * P * 9 * (2 * P + 1) * (2 * P + 1)) + 2 * size_t(P) * Mc * NR) * sizeof(V2<T>) +
         sizeof(T) * 2 * CSOL_CG * 4 * CSOL_RG * CSOL_RW * NR;
}

template <int P, typename T, int NR>
void csolve_launch(const CoarseLayout& L, const CsJobs<T>& jobs, int njobs, long cstride,
                   int* err, bool allow_persistent, hipStream_t st) {
  auto kern = k_csolve<P, T, NR>;
  const int nb = L.nblocks(), m = nb / 2;
  const int F = std::max(m, nb - 1 - m);
  const int nsteps = 2 * F + 1;
  constexpr int NCOEF = P * P * 9 * (2 * P + 1) * (2 * P + 1);
  const size_t lds = (NCOEF + 2 * size_t(L.size(0)) * NR) * sizeof(V2<T>);
  if (csolve_lds<P, T, NR>(L.Mc) > kLdsPerWorkgroup)
    throw std::runtime_error("coarse solve staging exceeds the LDS of a workgroup");
  int dev = 0;
  HZ_HIP(hipGetDevice(&dev));
  // dynamic LDS beyond the default limit must be requested (per device; the static part
  // counts too); several host threads may get here at once
  {
    static std::mutex mu;
    static std::map<int, size_t> configured;
    std::lock_guard<std::mutex> g(mu);
    size_t& c = configured[dev];
    if (lds > 48 * 1024 && lds > c) {
      HZ_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 int(lds)));
      c = lds;
    }
  }
  int cus = 0, coop = 0;
  HZ_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  HZ_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
  int per_cu = 0;
  HZ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)kern, 512, lds));
  const int max_coresident = per_cu * cus;
  // each job: two chains of Gh workgroups holding R rows of a block; all jobs together
  // occupy at most one workgroup per compute unit
  const int n0 = int(L.size(0));
  const int half = std::max(1, cus / 2 / njobs);
  const int R = (n0 + half - 1) / half;
  const int Gh = (n0 + R - 1) / R;
  int Gp = 2 * Gh;
  const int G = njobs * Gp;
  const bool persistent = coop && allow_persistent && max_coresident >= G;
  // every step's rows of a workgroup form one chunk of the stream waves
  constexpr int RCH = CSOL_RG * CSOL_RW;
  int one = csolve_one_ok<T, NR>() && (n0 + Gh - 1) / Gh <= RCH &&
            (n0 + CSOL_CG - 1) / CSOL_CG <= 64 * CSOL_QW;
  int s_begin = 0, s_end = nsteps;
  const long Nc = long(L.Mc) * L.Mc;
  const unsigned fb = unsigned((Nc + 255) / 256);
  k_fill_sentinel<T><<<dim3(fb, njobs), 256, 0, st>>>(jobs, Nc, cstride);
  if (persistent) {
    void* args[] = {&s_begin, &s_end, (void*)&L.nc, (void*)&L.Mc, &Gp, (void*)&jobs,
                    (void*)&cstride, &one, &err};
    PersistentOrder order(dev, st);
    HZ_HIP(hipLaunchCooperativeKernel((const void*)kern, dim3(G), dim3(512), args, lds, st));
  } else {
    for (int s = 0; s < nsteps; ++s)
      kern<<<G, 512, lds, st>>>(s, s + 1, L.nc, L.Mc, Gp, jobs, cstride, one, err);
  }
  HZ_HIP(hipGetLastError());
}

// Right-hand sides per job: groups of 4 share each factor read, or 2 / 1 where the group's
// staging does not fit in LDS.
template <int P, typename T>
int csolve_group(const CoarseLayout& L) {
  return csolve_lds<P, T, 4>(L.Mc) <= kLdsPerWorkgroup ? 4
         : csolve_lds<P, T, 2>(L.Mc) <= kLdsPerWorkgroup ? 2 : 1;
}

template <int P, typename T>
int csolve_jobs_p(const CoarseLayout& L, const CoarseJob<T>* jobs, int njobs, long cstride,
                  int* err, bool persistent, hipStream_t st) {
  int launches = 0;
  for (int j0 = 0; j0 < njobs; j0 += kMaxJobs) {
    const int nj = std::min(kMaxJobs, njobs - j0);
    CsJobs<T> t{};
    int nr = 1;
    for (int i = 0; i < nj; ++i) {
      t.j[i] = jobs[j0 + i];
      nr = std::max(nr, jobs[j0 + i].nrhs);
    }
    if (nr == 1) csolve_launch<P, T, 1>(L, t, nj, cstride, err, persistent, st);
    else if (nr == 2) csolve_launch<P, T, 2>(L, t, nj, cstride, err, persistent, st);
    else csolve_launch<P, T, 4>(L, t, nj, cstride, err, persistent, st);
    ++launches;
  }
  return launches;
}

// Twisted block LU: the top chain factors blocks 0 .. m-1 downwards (D_j against j-1), the
// bottom chain blocks nb-1 .. m+1 upwards (D_j against j+1), on two streams; the middle
// block m takes both Schur complements. Each inverse is stored in place of its block.
}  // namespace

size_t sweep_panel_elems(size_t nmax) { return 2 * size_t(SB) * ((nmax + SB - 1) / SB) * SB; }
size_t sweep_pinv_elems() { return 2 * size_t(SB) * SB; }

// Symmetric sweep of one block: first panel and pivot inverse, one launch per pivot tile,
// final mirror.
void sweep_inverse(double2* D, int n, double2* W, double2* R, int* flag, hipStream_t st) {
  const int nt = (n + SB - 1) / SB;
  const size_t ld = size_t(nt) * SB;
  SweepPass a;
  a.X = D;
  a.n = n;
  a.T = nt;
  a.flag = flag;
  a.K = -1;
  a.Rc = nullptr;
  a.Pc = nullptr;
  a.Rn = W;
  a.Pn = R;
  k_sweep_first<<<nt + 1, 256, 0, st>>>(a);
  const int nu = nt * (nt + 1) / 2;
  for (int K = 0; K < nt; ++K) {
    a.K = K;
    a.Rc = W + size_t(K & 1) * SB * ld;
    a.Rn = W + size_t((K + 1) & 1) * SB * ld;
    a.Pc = R + size_t(K & 1) * SB * SB;
    a.Pn = R + size_t((K + 1) & 1) * SB * SB;
    k_sweep_pass<<<1 + (nu + 3) / 4, 256, 0, st>>>(a);
  }
  k_sweep_last<<<nu, 256, 0, st>>>(D, n, nt);
}

void sweep_inverse_batch(double2* base, const SweepNode* zs, int nz, int maxT, double2* W,
                         double2* R, int* flag, hipStream_t st) {
  if (nz <= 0) return;
  const int maxnu = maxT * (maxT + 1) / 2;
  k_sweep_first_b<<<dim3(maxT + 1, nz), 256, 0, st>>>(base, W, R, zs, flag);
  for (int K = 0; K < maxT; ++K)
    k_sweep_pass_b<<<dim3(1 + (maxnu + 3) / 4, nz), 256, 0, st>>>(base, W, R, zs, K, flag);
  k_sweep_last_b<<<dim3(maxnu, nz), 256, 0, st>>>(base, zs);
  HZ_HIP(hipGetLastError());
}

namespace {

template <int P>
void factor_block(const CoarseLayout& L, const DevOp<double>& cop, double2* S, int j, int jn1,
                  int jn2, double2* T, double2* W, double2* R, int* flag, hipStream_t st) {
  const int n = int(L.size(j));
  double2* D = S + L.off(j);
  const dim3 g2((n + 255) / 256, n);
  k_schur_left<P><<<g2, 256, 0, st>>>(j, -1, L.nc, L.Mc, cop.coef, cop.pn, T, n, D);
  for (int jn : {jn1, jn2}) {
    if (jn < 0) continue;
    const int nn = int(L.size(jn));
    k_schur_right<P><<<dim3((n + 255) / 256, nn), 256, 0, st>>>(j, jn, L.nc, L.Mc, cop.coef,
                                                                cop.pn, S + L.off(jn), nn, n, T);
    k_schur_left<P><<<g2, 256, 0, st>>>(j, jn, L.nc, L.Mc, cop.coef, cop.pn, T, n, D);
  }
  sweep_inverse(D, n, W, R, flag, st);
}

template <int P>
void factor_p(const CoarseLayout& L, const DevOp<double>& cop, double2* S,
              const CoarseFactorWork& w, hipStream_t st) {
  const int nb = L.nblocks(), m = nb / 2;
  const size_t mb = size_t(L.size(0));
  hipStream_t s2 = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  HZ_HIP(hipStreamCreateWithFlags(&s2, hipStreamNonBlocking));
  HZ_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
  HZ_HIP(hipEventCreateWithFlags(&join, hipEventDisableTiming));
  HZ_HIP(hipEventRecord(fork, st));
  HZ_HIP(hipStreamWaitEvent(s2, fork, 0));
  // top chain on st, bottom chain on s2 (own temporaries)
  double2* T2 = w.T + mb * mb;
  double2* W2 = w.W + sweep_panel_elems(mb);
  double2* R2 = w.R + sweep_pinv_elems();
  int step = 0;
  for (int jt = 0, jb = nb - 1; jt < m || jb > m; ++jt, --jb, ++step) {
    if (jt < m) factor_block<P>(L, cop, S, jt, jt > 0 ? jt - 1 : -1, -1, w.T, w.W, w.R, w.flag, st);
    if (jb > m) factor_block<P>(L, cop, S, jb, jb < nb - 1 ? jb + 1 : -1, -1, T2, W2, R2, w.flag, s2);
  }
  HZ_HIP(hipEventRecord(join, s2));
  HZ_HIP(hipStreamWaitEvent(st, join, 0));
  factor_block<P>(L, cop, S, m, m > 0 ? m - 1 : -1, m < nb - 1 ? m + 1 : -1, w.T, w.W, w.R,
                  w.flag, st);
  HZ_HIP(hipGetLastError());
  HZ_HIP(hipStreamSynchronize(st));
  (void)hipEventDestroy(fork);
  (void)hipEventDestroy(join);
  (void)hipStreamDestroy(s2);
}

}  // namespace

void coarse_order_init(int dev) {
  std::lock_guard<std::mutex> g(order_mu());
  (void)order_event_locked(dev);
}

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
int coarse_group(const CoarseLayout& L) {
  if (L.p == 1) return csolve_group<1, T>(L);
  if (L.p == 2) return csolve_group<2, T>(L);
  return csolve_group<3, T>(L);
}

template <typename T>
int coarse_solve_jobs(const CoarseLayout& L, const CoarseJob<T>* jobs, int njobs, long cstride,
                      int* err, bool persistent, hipStream_t st) {
  if (njobs < 1) return 0;
  const int grp = coarse_group<T>(L);
  for (int i = 0; i < njobs; ++i)
    if (jobs[i].nrhs < 1 || jobs[i].nrhs > grp) throw std::runtime_error("bad coarse job size");
  if (L.p == 1) return csolve_jobs_p<1, T>(L, jobs, njobs, cstride, err, persistent, st);
  if (L.p == 2) return csolve_jobs_p<2, T>(L, jobs, njobs, cstride, err, persistent, st);
  return csolve_jobs_p<3, T>(L, jobs, njobs, cstride, err, persistent, st);
}

// One problem, nrhs right-hand sides with stride cstride: jobs of up to the LDS group size,
// one launch each (the jobs of one problem share its forward-sweep buffer).
template <typename T>
int coarse_solve(const CoarseLayout& L, const DevOp<T>& cop, const V2<T>* S, const V2<T>* b,
                 V2<T>* y, int nrhs, long cstride, const CoarseSolveWork& w, hipStream_t st) {
  if (nrhs < 1) return 0;
  if (nrhs > 1 && cstride < long(L.Mc) * L.Mc) throw std::runtime_error("coarse stride too small");
  const int grp = nrhs == 1 ? 1 : coarse_group<T>(L);
  int launches = 0;
  for (int r0 = 0; r0 < nrhs; r0 += grp) {
    CoarseJob<T> j;
    j.S = S;
    j.coef = cop.coef;
    j.pn = cop.pn;
    j.b = b + r0 * cstride;
    j.y = y + r0 * cstride;
    j.gbuf = reinterpret_cast<V2<T>*>(w.g);
    j.nrhs = std::min(grp, nrhs - r0);
    launches += coarse_solve_jobs<T>(L, &j, 1, cstride, w.err, w.persistent, st);
  }
  return launches;
}

void launch_factor_to_f32(const double2* S, float2* Sf, size_t n, hipStream_t st) {
  k_factor_to_f32<<<unsigned((n + 255) / 256), 256, 0, st>>>(S, Sf, n);
  HZ_HIP(hipGetLastError());
}

template int coarse_solve<double>(const CoarseLayout&, const DevOp<double>&, const double2*,
                                  const double2*, double2*, int, long, const CoarseSolveWork&,
                                  hipStream_t);
template int coarse_solve<float>(const CoarseLayout&, const DevOp<float>&, const float2*,
                                 const float2*, float2*, int, long, const CoarseSolveWork&,
                                 hipStream_t);
template int coarse_solve_jobs<double>(const CoarseLayout&, const CoarseJob<double>*, int, long,
                                       int*, bool, hipStream_t);
template int coarse_solve_jobs<float>(const CoarseLayout&, const CoarseJob<float>*, int, long,
                                      int*, bool, hipStream_t);
template int coarse_group<double>(const CoarseLayout&);
template int coarse_group<float>(const CoarseLayout&);

}  // namespace hz
