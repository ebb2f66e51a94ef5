// Matrix-free lattice kernels of the twogrid method (Sec. 4, Algorithm 1; the fine level
// applies A_0 and A_eps without a stored matrix).
//
// Layout: a level vector holds M*M complex values, point (a, b) at index b*M + a.
// Work decomposition: one thread owns a "macro point", the p x p block of lattice points
// (p I + ca, p J + cb), ca, cb in [0, p), so that every lane of a wavefront applies the same
// p*p class stencils. The stencil coefficients are then wave-uniform (scalar loads) and the
// couplings that are structurally zero are removed at compile time. A workgroup stages its
// tile of the input, with a halo of p lattice points, in LDS with coalesced loads.

#include <cstdio>
#include <cstdlib>
#include <functional>
#include <map>
#include <mutex>
#include <stdexcept>
#include <string>
#include <type_traits>

#include "hz_common.h"

namespace hz {

namespace {

constexpr int BX = 64;   // macro points per tile along x (one wavefront)

__device__ __forceinline__ int region(int a, int M) { return a == 0 ? 0 : (a == M - 1 ? 2 : 1); }

// Coarse-grid correction added while staging (ST_SMOOTH_PC): coarse vector, its batch
// offsets, coarse lattice size and prolongation weights.
template <typename T>
struct Corr {
  const V2<T>* ec = nullptr;
  Addr ac;
  int Mc = 0;
  const T* rw = nullptr;
};

// A tile is BX x BYT macro points (each p x p lattice points) plus a p-halo, staged in LDS;
// 256 threads = 64 columns x 4 rows, each thread BYT / 4 macro rows. XCD: the tiles are
// renumbered so that workgroup b (dispatched round-robin over the 8 XCDs, each with its own
// L2) takes the tiles of band b mod 8 in row order, so that the halo rows shared by
// vertically adjacent tiles are read through the same L2.
// ST_SMOOTH_PC first stages the coarse points whose prolongation reaches the tile (and the
// weight table), then stages v = x + P ec in 2 x 2 fine blocks: per fine point the coarse
// terms in ascending (B, A) order, as the prolongation kernel sums them, then the fine value
// added.
template <int P, typename T, typename TX, typename TF, typename TY, int MODE, int BYT, bool XCD>
__global__ void __launch_bounds__(256)
k_stencil(DevOp<T> op, const V2<TX>* __restrict__ x, Addr ax, const V2<TF>* __restrict__ f,
          Addr af, V2<TY>* __restrict__ y, Addr ay, Corr<T> cr) {
  constexpr int W = 2 * P + 1, W2 = W * W;
  constexpr int LW = P * BX + 2 * P, LH = P * BYT + 2 * P;
  constexpr bool PC = MODE == ST_SMOOTH_PC;
  constexpr int WR = 4 * P + 1;
  constexpr int CW = PC ? (LW + 4 * P + 3) / 2 + 1 : 1, CH = PC ? (LH + 4 * P + 3) / 2 + 1 : 1;
  __shared__ V2<T> tile[LH][LW];
  __shared__ V2<T> ctile[CH][CW];
  __shared__ T wl[PC && P > 1 ? P * P * WR * WR : 1];
  const int M = op.M;
  const int nmac = (M + P - 1) / P;
  const int ntx = (nmac + BX - 1) / BX, nty = (nmac + BYT - 1) / BYT;
  int tnum = blockIdx.x;
  if (XCD) {
    const int per = (ntx * nty + 7) / 8;
    tnum = (blockIdx.x % 8) * per + blockIdx.x / 8;
    if (tnum >= ntx * nty) return;             // whole workgroup, before any barrier
  }
  const int bz = blockIdx.y;
  const V2<T>* __restrict__ coef = op.ctab ? op.ctab[bz] : op.coef;
  const V2<T>* __restrict__ wdinv = op.wtab ? op.wtab[bz] : op.wdinv;
  x += ax.at(bz);
  y += ay.at(bz);
  if (MODE != ST_APPLY) f += af.at(bz);
  const int I0 = (tnum % ntx) * BX, J0 = (tnum / ntx) * BYT;
  const int ax0 = P * I0 - P, by0 = P * J0 - P;
  const int CA0 = (ax0 - 2 * P) >> 1, CB0 = (by0 - 2 * P) >> 1;   // floor
  if constexpr (PC) {
    // 2 x 2 fine blocks (2 At + i, 2 Bt + j): the (2P+1)^2 coarse points around (At, Bt) are
    // every coarse point whose prolongation reaches the block, and the weight offsets
    // (dx, dy) = (i + 2P - 2 ja, j + 2P - 2 jb) are compile-time constants. Every global load
    // of the staging (the coarse tile, the fine values) is issued before the one barrier.
    constexpr int NB = 2 * P + 1;
    constexpr int NBX = LW / 2 + 2, NBY = LH / 2 + 2;
    constexpr int NCT = (CW * CH + 255) / 256, NBL = (NBX * NBY + 255) / 256;
    const V2<T>* __restrict__ ec = cr.ec + cr.ac.at(bz);
    const int Mc = cr.Mc;
    const int bx0 = ax0 >> 1, by0c = by0 >> 1;
    V2<T> cl[NCT];
#pragma unroll
    for (int q = 0; q < NCT; ++q) {
      const int idx = threadIdx.x + 256 * q;
      const int cy = idx / CW, cx = idx - cy * CW;
      const int A = CA0 + cx, B = CB0 + cy;
      cl[q] = (idx < CW * CH && A >= 0 && A < Mc && B >= 0 && B < Mc) ? ec[long(B) * Mc + A]
                                                                      : czero<T>();
    }
    V2<T> xl[NBL][2][2];
#pragma unroll
    for (int q = 0; q < NBL; ++q) {
      const int idx = threadIdx.x + 256 * q;
      const int qy = idx / NBX, qx = idx - qy * NBX;
      const int At = bx0 + qx, Bt = by0c + qy;
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const int a = 2 * At + i, b = 2 * Bt + j;
          const int lx = a - ax0, ly = b - by0;
          const bool in = idx < NBX * NBY && lx >= 0 && lx < LW && ly >= 0 && ly < LH &&
                          a >= 0 && a < M && b >= 0 && b < M;
          xl[q][j][i] = in ? cvt<T>(x[long(b) * M + a]) : czero<T>();
        }
    }
#pragma unroll
    for (int q = 0; q < NCT; ++q) {
      const int idx = threadIdx.x + 256 * q;
      if (idx < CW * CH) ctile[idx / CW][idx % CW] = cl[q];
    }
    if (P > 1)
      for (int idx = threadIdx.x; idx < P * P * WR * WR; idx += 256) wl[idx] = cr.rw[idx];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NBL; ++q) {
      const int idx = threadIdx.x + 256 * q;
      if (idx >= NBX * NBY) continue;
      const int qy = idx / NBX, qx = idx - qy * NBX;
      const int At = bx0 + qx, Bt = by0c + qy;
      if (2 * At > ax0 + LW - 1 || 2 * Bt > by0 + LH - 1) continue;
      V2<T> cv[NB][NB];
#pragma unroll
      for (int jb = 0; jb < NB; ++jb)
#pragma unroll
        for (int ja = 0; ja < NB; ++ja) cv[jb][ja] = ctile[Bt - P + jb - CB0][At - P + ja - CA0];
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const int a = 2 * At + i, b = 2 * Bt + j;
          const int lx = a - ax0, ly = b - by0;
          if (lx < 0 || lx >= LW || ly < 0 || ly >= LH) continue;
          V2<T> v = czero<T>();
          if (a >= 0 && a < M && b >= 0 && b < M) {
            V2<T> pe = czero<T>();
            sfor<0, NB>([&](auto jb_) {
              constexpr int jb = decltype(jb_)::value;
              constexpr int dy0 = 2 * P - 2 * jb;           // dy = j + dy0
              const int B = Bt - P + jb;
              sfor<0, NB>([&](auto ja_) {
                constexpr int ja = decltype(ja_)::value;
                constexpr int dx0 = 2 * P - 2 * ja;
                const int A = At - P + ja;
                const int dy = j + dy0, dx = i + dx0;
                if (dy >= -2 * P && dy <= 2 * P && dx >= -2 * P && dx <= 2 * P && B >= 0 &&
                    B < Mc && A >= 0 && A < Mc) {
                  // P = 1: one class, the weight index is a constant (a wave-uniform load)
                  const int cls = P == 1 ? 0 : (B % P) * P + (A % P);
                  const int wi = (cls * WR + dy + 2 * P) * WR + dx + 2 * P;
                  const T wt = P == 1 ? cr.rw[wi] : wl[wi];
                  if (wt != T(0)) {
                    pe.x += wt * cv[jb][ja].x;
                    pe.y += wt * cv[jb][ja].y;
                  }
                }
              });
            });
            v = cadd<T>(pe, xl[q][j][i]);
          }
          tile[ly][lx] = v;
        }
    }
  } else {
    for (int idx = threadIdx.x; idx < LW * LH; idx += 256) {
      const int ly = idx / LW, lx = idx - ly * LW;
      const int a = ax0 + lx, b = by0 + ly;
      V2<T> v = czero<T>();
      if (a >= 0 && a < M && b >= 0 && b < M) {
        v = cvt<T>(x[long(b) * M + a]);
        if constexpr (MODE == ST_SMOOTH0)    // the first sweep from zero: u1 = wdinv f
          v = cmul<T>(wdinv[((b % P) * P + (a % P)) * 9 + region(b, M) * 3 + region(a, M)], v);
      }
      tile[ly][lx] = v;
    }
  }
  __syncthreads();
  const int tx = threadIdx.x % BX;
#pragma unroll
  for (int rr = 0; rr < BYT / 4; ++rr) {
  const int ty = threadIdx.x / BX + 4 * rr;
  const int I = I0 + tx, J = J0 + ty;
  if (I >= nmac || J >= nmac) continue;

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
      } else if constexpr (MODE == ST_SMOOTH || MODE == ST_SMOOTH0 || PC) {
        const V2<T> d = wdinv[(cb * P + ca) * 9 + reg[cb][ca]];
        const V2<T> rr = csub<T>(cvt<T>(f[gi]), out);
        out = cadd<T>(tile[P * ty + P + cb][P * tx + P + ca], cmul<T>(d, rr));
      }
      y[gi] = cvt<TY>(out);
    }
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
  const long wi = op.pn ? i : long(cls * 9 + reg);   // per point, or per (class, region)
  y[ay.at(bz) + i] = cmul<T>(wd[wi], cvt<T>(f[af.at(bz) + i]));
}

// Workgroups of a 1D launch over lattice points are dealt round-robin to the 8 XCDs (each
// with its own L2); renumbering them so that XCD x takes a contiguous band of 1/8 of the
// points keeps the lattice rows that neighbouring rows of outputs share in one L2.
__device__ __forceinline__ long xcd_band_block(int nblocks) {
  const int per = (nblocks + 7) / 8;
  return long(blockIdx.x % 8) * per + blockIdx.x / 8;
}
inline unsigned xcd_band_grid(long nblocks) { return unsigned(8 * ((nblocks + 7) / 8)); }

// yc(A, B) = sum over fine points (2A + dx, 2B + dy) of RW[cls(A,B)][dy][dx] r(...)
template <int P, typename T>
__global__ void __launch_bounds__(256)
k_restrict(int Mf, int Mc, const T* __restrict__ rw, const V2<T>* __restrict__ r,
           V2<T>* __restrict__ yc, Addr af, Addr ac) {
  constexpr int WR = 4 * P + 1;
  const long Nc = long(Mc) * Mc;
  const long i = xcd_band_block(int((Nc + 255) / 256)) * 256 + threadIdx.x;
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

// Residual and restriction in one pass, P1 (Alg. 1: restrict residual): r_c = P^T (f - A u).
// A workgroup owns RCX x RCY coarse points. It stages u on the fine points that the residuals
// of its restriction footprint read (the footprint, 2 fine points around the coarse tile's
// fine image, plus a 1-point halo), forms those residuals in registers with the stencil
// kernel's tap order (dy, then dx ascending; so bitwise its residual) and stores them over the
// staged u, then each thread restricts one coarse point from them in the restriction
// kernel's order. The residual never goes to
// memory; neighbouring tiles recompute their 3 shared footprint lines. Tiles in XCD bands as
// in the stencil kernel.
constexpr int RCX = 32, RCY = 8;
template <typename T>
__global__ void __launch_bounds__(256)
k_resid_restrict1(DevOp<T> op, const V2<T>* __restrict__ x, Addr ax, const V2<T>* __restrict__ f,
                  Addr af, int Mc, const T* __restrict__ rw, V2<T>* __restrict__ yc, Addr ac) {
  constexpr int W2 = 9;
  constexpr int RWD = 2 * RCX - 1 + 4, RHD = 2 * RCY - 1 + 4;   // residual region
  constexpr int UWD = RWD + 2, UHD = RHD + 2;                   // staged u
  __shared__ V2<T> ut[UHD][UWD];
  V2<T>* rt = &ut[0][0];      // the residuals (RHD x RWD) replace u once every wave has read it
  constexpr int NQ = (RWD * RHD + 255) / 256;
  const int M = op.M;
  const int ntx = (Mc + RCX - 1) / RCX, nty = (Mc + RCY - 1) / RCY;
  const int per = (ntx * nty + 7) / 8;
  const int tnum = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (tnum >= ntx * nty) return;               // whole workgroup, before any barrier
  const int bz = blockIdx.y;
  const V2<T>* __restrict__ coef = op.ctab ? op.ctab[bz] : op.coef;
  x += ax.at(bz);
  f += af.at(bz);
  yc += ac.at(bz);
  const int A0 = (tnum % ntx) * RCX, B0 = (tnum / ntx) * RCY;
  const int ra0 = 2 * A0 - 2, rb0 = 2 * B0 - 2;       // residual region origin
  const int ua0 = ra0 - 1, ub0 = rb0 - 1;             // staged u origin
  V2<T> fq[NQ];               // f at this thread's residual points, requested with u
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int idx = threadIdx.x + 256 * q;
    const int ly = idx / RWD, lx = idx - ly * RWD;
    const int a = ra0 + lx, b = rb0 + ly;
    fq[q] = (idx < RWD * RHD && a >= 0 && a < M && b >= 0 && b < M) ? f[long(b) * M + a]
                                                                    : czero<T>();
  }
  for (int idx = threadIdx.x; idx < UWD * UHD; idx += 256) {
    const int ly = idx / UWD, lx = idx - ly * UWD;
    const int a = ua0 + lx, b = ub0 + ly;
    ut[ly][lx] = (a >= 0 && a < M && b >= 0 && b < M) ? x[long(b) * M + a] : czero<T>();
  }
  __syncthreads();
  V2<T> rq[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int idx = threadIdx.x + 256 * q;
    const int ly = idx / RWD, lx = idx - ly * RWD;
    const int a = ra0 + lx, b = rb0 + ly;
    V2<T> r = czero<T>();
    if (idx < RWD * RHD && a >= 0 && a < M && b >= 0 && b < M) {
      const int reg = region(b, M) * 3 + region(a, M);
      V2<T> acc = czero<T>();
      sfor<-1, 2>([&](auto dy_) {
        constexpr int dy = decltype(dy_)::value;
        sfor<-1, 2>([&](auto dx_) {
          constexpr int dx = decltype(dx_)::value;
          if constexpr (couples(1, 0, 0, dx, dy)) {
            constexpr int off = (dy + 1) * 3 + (dx + 1);
            cfma(acc, coef[reg * W2 + off], ut[ly + 1 + dy][lx + 1 + dx]);
          }
        });
      });
      r = csub<T>(fq[q], acc);
    }
    rq[q] = r;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int idx = threadIdx.x + 256 * q;
    if (idx < RWD * RHD) rt[idx] = rq[q];
  }
  __syncthreads();
  const int A = A0 + int(threadIdx.x) % RCX, B = B0 + int(threadIdx.x) / RCX;
  if (A >= Mc || B >= Mc) return;
  V2<T> acc = czero<T>();
#pragma unroll
  for (int dy = -2; dy <= 2; ++dy) {
    const int b = 2 * B + dy;
    if (b < 0 || b >= M) continue;
#pragma unroll
    for (int dx = -2; dx <= 2; ++dx) {
      const int a = 2 * A + dx;
      if (a < 0 || a >= M) continue;
      const T wt = rw[(dy + 2) * 5 + dx + 2];
      if (wt != T(0)) {
        const V2<T> v = rt[(b - rb0) * RWD + (a - ra0)];
        acc.x += wt * v.x;
        acc.y += wt * v.y;
      }
    }
  }
  yc[long(B) * Mc + A] = acc;
}

// yf(a, b) (+)= sum over coarse (A, B) with |a - 2A|, |b - 2B| <= 2P of RW[cls(A,B)][.][.] xc.
// One thread per coarse point (At, Bt) forms the 2 x 2 fine points (2 At + i, 2 Bt + j): their
// coarse neighbourhoods are the same (2P+1)^2 points (held in registers for P <= 2), and a
// wave writes contiguous pairs of fine points. Per fine point the terms are summed in the
// order of ascending B, then A.
template <int P, typename T, bool ADD>
__global__ void __launch_bounds__(256)
k_prolong(int Mf, int Mc, const T* __restrict__ rw, const V2<T>* __restrict__ xc,
          V2<T>* __restrict__ yf, Addr af, Addr ac) {
  constexpr int WR = 4 * P + 1, NB = 2 * P + 1;
  constexpr bool CACHE = P <= 2;
  const long Nc = long(Mc) * Mc;
  const long t = xcd_band_block(int((Nc + 255) / 256)) * 256 + threadIdx.x;
  if (t >= Nc) return;
  xc += ac.at(blockIdx.y);
  yf += af.at(blockIdx.y);
  const int Bt = int(t / Mc), At = int(t - long(Bt) * Mc);
  V2<T> xv[CACHE ? NB : 1][CACHE ? NB : 1];
  if constexpr (CACHE) {
#pragma unroll
    for (int jb = 0; jb < NB; ++jb)
#pragma unroll
      for (int ja = 0; ja < NB; ++ja) {
        const int A = At - P + ja, B = Bt - P + jb;
        xv[jb][ja] = (A >= 0 && A < Mc && B >= 0 && B < Mc) ? xc[long(B) * Mc + A] : czero<T>();
      }
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int b = 2 * Bt + j;
    if (b >= Mf) continue;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int a = 2 * At + i;
      if (a >= Mf) continue;
      V2<T> acc = czero<T>();
#pragma unroll
      for (int jb = 0; jb < NB; ++jb) {
        const int B = Bt - P + jb;
        const int dy = b - 2 * B;
        if (B < 0 || B >= Mc || dy < -2 * P || dy > 2 * P) continue;
#pragma unroll
        for (int ja = 0; ja < NB; ++ja) {
          const int A = At - P + ja;
          const int dx = a - 2 * A;
          if (A < 0 || A >= Mc || dx < -2 * P || dx > 2 * P) continue;
          const int cls = (B % P) * P + (A % P);
          const T wt = rw[(cls * WR + dy + 2 * P) * WR + dx + 2 * P];
          if (wt != T(0)) {
            V2<T> v;
            if constexpr (CACHE) v = xv[jb][ja];
            else v = xc[long(B) * Mc + A];
            acc.x += wt * v.x;
            acc.y += wt * v.y;
          }
        }
      }
      const long gi = long(b) * Mf + a;
      if (ADD) acc = cadd<T>(acc, yf[gi]);
      yf[gi] = acc;
    }
  }
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

// Launch variants of the stencil (tile height, tile order). Every variant computes every
// output with the same arithmetic in the same order, so the choice never changes a result.
struct StencilVariant {
  int byt;
  bool xcd;
};
constexpr StencilVariant kVariants[] = {{4, false}, {4, true}, {8, false}, {8, true}, {16, true}};

template <int P, typename T, typename TX, typename TF, typename TY, int MODE, int BYT, bool XCD>
void stencil_launch(const DevOp<T>& op, const V2<TX>* x, Addr xs, const V2<TF>* f, Addr fs,
                    V2<TY>* y, Addr ys, int nbatch, hipStream_t st, const Corr<T>& cr) {
  const int nmac = (op.M + P - 1) / P;
  const int ntiles = ((nmac + BX - 1) / BX) * ((nmac + BYT - 1) / BYT);
  const int blocks = XCD ? 8 * ((ntiles + 7) / 8) : ntiles;
  k_stencil<P, T, TX, TF, TY, MODE, BYT, XCD><<<dim3(blocks, nbatch), 256, 0, st>>>(op, x, xs, f, fs, y, ys, cr);
}

template <int P, typename T, typename TX, typename TF, typename TY, int MODE>
void stencil_variant(int v, const DevOp<T>& op, const V2<TX>* x, Addr xs, const V2<TF>* f,
                     Addr fs, V2<TY>* y, Addr ys, int nbatch, hipStream_t st,
                     const Corr<T>& cr = Corr<T>()) {
  // taller tiles only where their LDS stays small (P <= 2)
  if (v == 1) stencil_launch<P, T, TX, TF, TY, MODE, 4, true>(op, x, xs, f, fs, y, ys, nbatch, st, cr);
  else if (v == 2 && P <= 2) stencil_launch<P, T, TX, TF, TY, MODE, (P <= 2 ? 8 : 4), false>(op, x, xs, f, fs, y, ys, nbatch, st, cr);
  else if (v == 3 && P <= 2) stencil_launch<P, T, TX, TF, TY, MODE, (P <= 2 ? 8 : 4), true>(op, x, xs, f, fs, y, ys, nbatch, st, cr);
  else if (v == 4 && P == 1) stencil_launch<P, T, TX, TF, TY, MODE, (P == 1 ? 16 : 4), true>(op, x, xs, f, fs, y, ys, nbatch, st, cr);
  else stencil_launch<P, T, TX, TF, TY, MODE, 4, false>(op, x, xs, f, fs, y, ys, nbatch, st, cr);
}

// Autotuner: the first launch of a (kernel, lattice size, batch bucket) times every variant
// on the stream with HIP events (the launch is a pure function of its inputs, so repeating
// it is harmless) and keeps the fastest for the rest of the process. HZ_TUNE=0 disables it.
std::mutex g_tune_mu;
std::map<std::string, int> g_tune;
thread_local bool tl_tune = true;

int tuned_variant(const std::string& key, int nvar,
                  const std::function<void(int)>& launch, hipStream_t st) {
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) return it->second;
  }
  static const bool enabled = [] {
    const char* e = std::getenv("HZ_TUNE");
    return !(e && e[0] == '0');
  }();
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (!enabled || !tl_tune || hipStreamIsCapturing(st, &cs) != hipSuccess ||
      cs != hipStreamCaptureStatusNone) {
    (void)hipGetLastError();
    return 0;
  }
  hipEvent_t a, b;
  HZ_HIP(hipEventCreate(&a));
  HZ_HIP(hipEventCreate(&b));
  int best = 0;
  float best_ms = 1e30f;
  for (int v = 0; v < nvar; ++v) {
    launch(v);                                 // warm
    float tmin = 1e30f;
    for (int r = 0; r < 3; ++r) {
      HZ_HIP(hipEventRecord(a, st));
      launch(v);
      HZ_HIP(hipEventRecord(b, st));
      HZ_HIP(hipEventSynchronize(b));
      float ms = 0;
      HZ_HIP(hipEventElapsedTime(&ms, a, b));
      tmin = std::min(tmin, ms);
    }
    if (tmin < best_ms) {
      best_ms = tmin;
      best = v;
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  static const bool verbose = [] {
    const char* e = std::getenv("HZ_TUNE_LOG");
    return e && e[0] == '1';
  }();
  if (verbose) std::fprintf(stderr, "hz tune %s: variant %d (%.3f ms)\n", key.c_str(), best, best_ms);
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune[key] = best;
  return best;
}

// HZ_STENCIL_VARIANT=v forces launch variant v (for checking every variant); unset or
// negative: the tuner's choice.
int forced_variant() {
  const char* e = std::getenv("HZ_STENCIL_VARIANT");
  return (e && *e) ? std::atoi(e) : -1;
}

// HZ_FUSE_RR=0: the residual and the restriction as two passes (for comparison).
bool resid_restrict_disabled() {
  static const bool off = [] {
    const char* e = std::getenv("HZ_FUSE_RR");
    return e && e[0] == '0';
  }();
  return off;
}

// HZ_FUSE_PC=0: the coarse correction as its own prolongation-add pass (for comparison).
bool smooth_pc_disabled() {
  static const bool off = [] {
    const char* e = std::getenv("HZ_FUSE_PC");
    return e && e[0] == '0';
  }();
  return off;
}

template <int P, typename T, typename TX, typename TF, typename TY>
void stencil_p(int mode, const DevOp<T>& op, const V2<TX>* x, Addr xs, const V2<TF>* f, Addr fs,
               V2<TY>* y, Addr ys, int nbatch, hipStream_t st, const Corr<T>& cr = Corr<T>()) {
  auto launch = [&](int v) {
    if (mode == ST_APPLY) stencil_variant<P, T, TX, TF, TY, ST_APPLY>(v, op, x, xs, f, fs, y, ys, nbatch, st);
    else if (mode == ST_RESID) stencil_variant<P, T, TX, TF, TY, ST_RESID>(v, op, x, xs, f, fs, y, ys, nbatch, st);
    else if (mode == ST_SMOOTH) stencil_variant<P, T, TX, TF, TY, ST_SMOOTH>(v, op, x, xs, f, fs, y, ys, nbatch, st);
    else if (mode == ST_SMOOTH0) stencil_variant<P, T, TX, TF, TY, ST_SMOOTH0>(v, op, x, xs, f, fs, y, ys, nbatch, st);
    else if constexpr (P <= 2 && std::is_same<T, TX>::value && std::is_same<T, TF>::value &&
                       std::is_same<T, TY>::value)
      stencil_variant<P, T, TX, TF, TY, ST_SMOOTH_PC>(v, op, x, xs, f, fs, y, ys, nbatch, st, cr);
    else throw std::runtime_error("stencil: mode not provided for this order or type");
  };
  const int nvar = P == 1 ? 5 : P == 2 ? 4 : 2;
  const int fv = forced_variant();
  if (fv >= 0) {
    if (fv >= nvar) throw std::runtime_error("HZ_STENCIL_VARIANT: no such variant for this order");
    launch(fv);
    return;
  }
  const int bucket = nbatch == 1 ? 1 : nbatch <= 4 ? 4 : nbatch <= 16 ? 16 : 64;
  const std::string key = "st" + std::to_string(P) + "/" + std::to_string(sizeof(T)) +
                          std::to_string(sizeof(TX)) + std::to_string(sizeof(TF)) +
                          std::to_string(sizeof(TY)) + "/" + std::to_string(mode) + "/" +
                          std::to_string(op.M) + "/" + std::to_string(bucket);
  launch(tuned_variant(key, nvar, launch, st));
}

}  // namespace

void set_stencil_tuning(bool on) { tl_tune = on; }

template <typename T, typename TX, typename TF, typename TY>
void launch_stencil(int p, int mode, const DevOp<T>& op, const V2<TX>* x, Addr xs,
                    const V2<TF>* f, Addr fs, V2<TY>* y, Addr ys, int nbatch, hipStream_t st) {
  if (op.pn) {
    launch_stencil_pn<T, TX, TF, TY>(p, mode, op, x, xs, f, fs, y, ys, nbatch, st);
    return;
  }
  if (p == 1) stencil_p<1, T, TX, TF, TY>(mode, op, x, xs, f, fs, y, ys, nbatch, st);
  else if (p == 2) stencil_p<2, T, TX, TF, TY>(mode, op, x, xs, f, fs, y, ys, nbatch, st);
  else stencil_p<3, T, TX, TF, TY>(mode, op, x, xs, f, fs, y, ys, nbatch, st);
  HZ_HIP(hipGetLastError());
}

template <typename T>
bool launch_smooth_pc(int p, const DevOp<T>& op, const V2<T>* x, Addr ax, const V2<T>* ec,
                      Addr ac, int Mc, const T* rw, const V2<T>* f, Addr af, V2<T>* y, Addr ay,
                      int nbatch, hipStream_t st) {
  if (op.pn || p > 2 || smooth_pc_disabled()) return false;
  if (op.M != 2 * (Mc - 1) + 1) throw std::runtime_error("smooth_pc: lattice sizes");
  Corr<T> cr;
  cr.ec = ec;
  cr.ac = ac;
  cr.Mc = Mc;
  cr.rw = rw;
  if (p == 1) stencil_p<1, T, T, T, T>(ST_SMOOTH_PC, op, x, ax, f, af, y, ay, nbatch, st, cr);
  else stencil_p<2, T, T, T, T>(ST_SMOOTH_PC, op, x, ax, f, af, y, ay, nbatch, st, cr);
  HZ_HIP(hipGetLastError());
  return true;
}

template <typename T>
bool launch_resid_restrict(int p, const DevOp<T>& op, const V2<T>* x, Addr ax, const V2<T>* f,
                           Addr af, int Mc, const T* rw, V2<T>* yc, Addr ac, int nbatch,
                           hipStream_t st) {
  if (op.pn || p != 1 || resid_restrict_disabled()) return false;
  if (op.M != 2 * (Mc - 1) + 1) throw std::runtime_error("resid_restrict: lattice sizes");
  const int ntiles = ((Mc + RCX - 1) / RCX) * ((Mc + RCY - 1) / RCY);
  k_resid_restrict1<T><<<dim3(8 * ((ntiles + 7) / 8), nbatch), 256, 0, st>>>(op, x, ax, f, af, Mc,
                                                                             rw, yc, ac);
  HZ_HIP(hipGetLastError());
  return true;
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
  dim3 grid(xcd_band_grid((Nc + 255) / 256), nbatch);
  if (p == 1) k_restrict<1, T><<<grid, 256, 0, st>>>(Mf, Mc, rw, r, yc, fstride, cstride);
  else if (p == 2) k_restrict<2, T><<<grid, 256, 0, st>>>(Mf, Mc, rw, r, yc, fstride, cstride);
  else k_restrict<3, T><<<grid, 256, 0, st>>>(Mf, Mc, rw, r, yc, fstride, cstride);
  HZ_HIP(hipGetLastError());
}

template <typename T>
void launch_prolong(int p, int Mf, int Mc, const T* rw, const V2<T>* xc, V2<T>* yf, bool add,
                    int nbatch, Addr fstride, Addr cstride, hipStream_t st) {
  const long Nc = long(Mc) * Mc;
  dim3 grid(xcd_band_grid((Nc + 255) / 256), nbatch);
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
template bool launch_resid_restrict<double>(int, const DevOp<double>&, const double2*, Addr,
    const double2*, Addr, int, const double*, double2*, Addr, int, hipStream_t);
template bool launch_resid_restrict<float>(int, const DevOp<float>&, const float2*, Addr,
    const float2*, Addr, int, const float*, float2*, Addr, int, hipStream_t);
template bool launch_smooth_pc<double>(int, const DevOp<double>&, const double2*, Addr,
    const double2*, Addr, int, const double*, const double2*, Addr, double2*, Addr, int, hipStream_t);
template bool launch_smooth_pc<float>(int, const DevOp<float>&, const float2*, Addr,
    const float2*, Addr, int, const float*, const float2*, Addr, float2*, Addr, int, hipStream_t);
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
