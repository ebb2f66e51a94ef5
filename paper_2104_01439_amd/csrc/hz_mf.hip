// Multifrontal direct solve of the coarse operator (the coarsest level of Sec. 4,
// Algorithm 1, factored once and reused as Sec. 6 does with its multifrontal LU).
//
// Nested dissection of the coarse lattice: a region is cut by a lattice line at a cell
// boundary (multiple of p) across its longer side; points on the two sides of such a line
// never share an element, so the line separates the region. Regions of at most kMfLeaf
// points are leaves. Node v owns the points I_v of its line (or of its leaf region) and
// couples to B_v, the ancestors' line points on the ring around its region.
//
// Factorisation, bottom-up by tree height: the front F_v on I_v + B_v holds the rows of A_c at
// I_v (and their transposes) plus the children's update matrices (extend-add); then
//   S_v = F_II^{-1},  G_v = S_v F_IB,  G_v^T,  U_v = F_BB - F_BI G_v  (passed to the parent).
// Solve: forward (heights ascending) f = [b_I; 0] + children's u, z_I = S_v f_I,
// u_v = f_B - G_v^T f_I; backward (heights descending) x_I = z_I - G_v x_B.
// The factor is explicit (inverses and products), so each pass is a set of independent
// matrix-vector products per height: at most 2 H + 1 dependent launches per solve, fewer with
// the bottom subtrees (heights 0 .. T) in one launch per pass.

#include <algorithm>
#include <cstring>
#include <map>
#include <memory>
#include <tuple>
#include <mutex>
#include <stdexcept>
#include <unordered_map>

#include "hz_common.h"

namespace hz {

// ------------------------------------------------------------------------------------------
// Symbolic analysis (host)
// ------------------------------------------------------------------------------------------

namespace {

struct Builder {
  int p, Mc;
  MfSym* S;
  std::vector<std::vector<int>> Ipts, Bpts;
  std::vector<std::pair<int, int>> ch;

  int cut(int lo, int hi) const {   // cell line strictly inside (lo, hi) nearest the middle
    const double mid = 0.5 * (lo + hi);
    int best = -1;
    for (int c = lo + 1; c < hi; ++c)
      if (c % p == 0 && (best < 0 || std::abs(c - mid) < std::abs(best - mid))) best = c;
    return best;
  }

  std::vector<int> ring(int a0, int a1, int b0, int b1) const {
    std::vector<int> r;
    for (int b = b0 - 1; b <= b1 + 1; ++b)
      for (int a = a0 - 1; a <= a1 + 1; ++a) {
        if (a >= a0 && a <= a1 && b >= b0 && b <= b1) continue;
        if (a < 0 || a >= Mc || b < 0 || b >= Mc) continue;
        r.push_back(b * Mc + a);
      }
    return r;
  }

  int add(std::vector<int>&& I, std::vector<int>&& B, int c0, int c1, int h) {
    Ipts.push_back(std::move(I));
    Bpts.push_back(std::move(B));
    ch.push_back({c0, c1});
    S->height.push_back(h);
    return int(Ipts.size()) - 1;
  }

  int rec(int a0, int a1, int b0, int b1) {
    const int w = a1 - a0 + 1, hgt = b1 - b0 + 1;
    int c = -1;
    bool vert = true;
    if (w * hgt > kMfLeaf) {
      if (w >= hgt) {
        c = cut(a0, a1);
        if (c < 0) { c = cut(b0, b1); vert = false; }
      } else {
        c = cut(b0, b1);
        vert = false;
        if (c < 0) { c = cut(a0, a1); vert = true; }
      }
    }
    if (c < 0) {
      std::vector<int> I;
      for (int b = b0; b <= b1; ++b)
        for (int a = a0; a <= a1; ++a) I.push_back(b * Mc + a);
      return add(std::move(I), ring(a0, a1, b0, b1), -1, -1, 0);
    }
    int k1, k2;
    std::vector<int> I;
    if (vert) {
      k1 = rec(a0, c - 1, b0, b1);
      k2 = rec(c + 1, a1, b0, b1);
      for (int b = b0; b <= b1; ++b) I.push_back(b * Mc + c);
    } else {
      k1 = rec(a0, a1, b0, c - 1);
      k2 = rec(a0, a1, c + 1, b1);
      for (int a = a0; a <= a1; ++a) I.push_back(c * Mc + a);
    }
    const int h = 1 + std::max(S->height[k1], S->height[k2]);
    return add(std::move(I), ring(a0, a1, b0, b1), k1, k2, h);
  }
};

// Rows of one wave-per-row solve task: about 32 KB of the matrix, a multiple of the four
// waves, 4 .. 64.
int task_rows(int len) {
  int r = (32768 / 16 + len - 1) / std::max(len, 1);
  r = (r + 3) / 4 * 4;
  return std::min(64, std::max(4, r));
}

void build_symbolic(MfSym& S, int p, int nc) {
  S.p = p;
  S.nc = nc;
  S.Mc = p * nc + 1;
  Builder b{p, S.Mc, &S, {}, {}, {}};
  const int root = b.rec(0, S.Mc - 1, 0, S.Mc - 1);
  const int nn = int(b.Ipts.size());
  if (root != nn - 1) throw std::runtime_error("multifrontal: root is not last");
  S.nodes.assign(nn, MfNode());
  S.parent.assign(nn, -1);
  S.H = S.height[root];
  long Io = 0, Bo = 0, F = 0, U = 0;
  for (int v = 0; v < nn; ++v) {
    MfNode& nd = S.nodes[v];
    nd.s = int(b.Ipts[v].size());
    nd.m = int(b.Bpts[v].size());
    nd.ch0 = b.ch[v].first;
    nd.ch1 = b.ch[v].second;
    if (nd.ch0 >= 0) S.parent[nd.ch0] = v;
    if (nd.ch1 >= 0) S.parent[nd.ch1] = v;
    nd.Ioff = Io;
    nd.Boff = Bo;
    Io += nd.s;
    Bo += nd.m;
    nd.Soff = F;
    F += long(nd.s) * nd.s;
    nd.Goff = F;
    F += long(nd.s) * nd.m;
    nd.GToff = F;
    F += long(nd.s) * nd.m;
    nd.uoff = U;
    U += nd.m;
    S.maxf = std::max(S.maxf, nd.s + nd.m);
    {
      const double ds = nd.s, dm = nd.m;
      S.flop += 8.0 * (ds * ds * ds + 2.0 * ds * ds * dm + dm * dm * ds);
    }
    S.I.insert(S.I.end(), b.Ipts[v].begin(), b.Ipts[v].end());
    S.B.insert(S.B.end(), b.Bpts[v].begin(), b.Bpts[v].end());
  }
  S.numel = F;
  S.uel = U;
  if (Io != long(S.Mc) * S.Mc) throw std::runtime_error("multifrontal: points not partitioned");
  // front positions of each child's B points in its parent
  for (int v = 0; v < nn; ++v) {
    const MfNode& nd = S.nodes[v];
    if (nd.ch0 < 0) continue;
    std::unordered_map<int, int> pos;
    pos.reserve(size_t(nd.s + nd.m) * 2);
    for (int i = 0; i < nd.s; ++i) pos[b.Ipts[v][i]] = i;
    for (int k = 0; k < nd.m; ++k) pos[b.Bpts[v][k]] = nd.s + k;
    const long inv0 = long(S.inv.size());
    S.inv.resize(S.inv.size() + 2 * size_t(nd.s + nd.m), -1);
    S.nodes[v].invoff = inv0;
    int slot = 0;
    for (int c : {nd.ch0, nd.ch1}) {
      MfNode& cn = S.nodes[c];
      cn.mapoff = long(S.map.size());
      int j = 0;
      for (int g : b.Bpts[c]) {
        auto it = pos.find(g);
        if (it == pos.end()) throw std::runtime_error("multifrontal: ring point not in parent front");
        S.map.push_back(it->second);
        S.inv[inv0 + 2 * it->second + slot] = j++;
      }
      ++slot;
    }
  }
  // nodes by height (also flat, for the small-node tasks), solve tasks by height
  S.at.assign(S.H + 1, {});
  for (int v = 0; v < nn; ++v) S.at[S.height[v]].push_back(v);
  auto is_small = [&](int v) { return S.nodes[v].s + S.nodes[v].m <= 64; };
  for (int h = 0; h <= S.H; ++h) {   // small nodes first within a height
    std::stable_partition(S.at[h].begin(), S.at[h].end(), is_small);
    S.hn.insert(S.hn.end(), S.at[h].begin(), S.at[h].end());
  }
  S.fwd0.assign(S.H + 2, 0);
  S.bwd0.assign(S.H + 2, 0);
  int hbase = 0;
  for (int h = 0; h <= S.H; ++h) {
    S.fwd0[h] = int(S.fwd.size());
    S.bwd0[h] = int(S.bwd.size());
    std::vector<int> small;   // positions in hn
    for (size_t q = 0; q < S.at[h].size(); ++q) {
      const int v = S.at[h][q];
      const MfNode& nd = S.nodes[v];
      if (is_small(v)) {
        small.push_back(hbase + int(q));
        continue;
      }
      if (nd.s <= 64) {
        // short rows: thread per row over [S; G^T] rows, 256 rows per task
        for (int r = 0; r < nd.s + nd.m; r += 256)
          S.fwd.push_back({v, 5, r, std::min(nd.s + nd.m, r + 256)});
      } else {
        const int R = task_rows(nd.s);
        for (int r = 0; r < nd.s; r += R) S.fwd.push_back({v, 0, r, std::min(nd.s, r + R)});
        for (int r = 0; r < nd.m; r += R) S.fwd.push_back({v, 1, r, std::min(nd.m, r + R)});
      }
      if (nd.m > 0) {
        const int R = task_rows(nd.m);
        for (int r = 0; r < nd.s; r += R) S.bwd.push_back({v, 2, r, std::min(nd.s, r + R)});
      }
    }
    // small nodes (s + m <= 64): one wave each, four to a workgroup; r0 .. r1 is a range of
    // consecutive positions in hn (the small nodes of a height are consecutive there)
    for (size_t i = 0; i < small.size(); i += 4) {
      const int n4 = int(std::min<size_t>(4, small.size() - i));
      if (small[i + n4 - 1] - small[i] != n4 - 1) throw std::runtime_error("multifrontal: task");
      S.fwd.push_back({-1, 3, small[i], small[i] + n4});
      S.bwd.push_back({-1, 4, small[i], small[i] + n4});
    }
    hbase += int(S.at[h].size());
  }
  S.fwd0[S.H + 1] = int(S.fwd.size());
  S.bwd0[S.H + 1] = int(S.bwd.size());
  // bottom subtrees: T = the largest height up to which every node is small, at most 3 (a
  // workgroup walks up to 15 nodes; taller subtrees would serialise more than the launches
  // they save)
  {
    int T = -1;
    for (int h = 0; h <= std::min(S.H, 3); ++h) {
      bool all = true;
      for (int v : S.at[h]) all = all && is_small(v);
      if (!all) break;
      T = h;
    }
    if (T == S.H) T = S.H - 1;          // keep the root out (it has no parent to hand u to)
    S.T = T;
    std::vector<int> size(nn, 1);       // subtree sizes: a subtree is [v - size + 1, v]
    for (int v = 0; v < nn; ++v)
      if (S.nodes[v].ch0 >= 0) size[v] += size[S.nodes[v].ch0] + size[S.nodes[v].ch1];
    MfSubHdr& mx = S.sub_max;
    for (int v = 0; T >= 0 && v < nn; ++v) {
      if (S.height[v] > T) continue;
      const int pa = S.parent[v];
      if (pa >= 0 && S.height[pa] <= T) continue;   // not a subtree root
      const int v0 = v - size[v] + 1;
      std::vector<int> list;
      for (int x = v0; x <= v; ++x) list.push_back(x);
      std::stable_sort(list.begin(), list.end(),
                       [&](int a, int c) { return S.height[a] < S.height[c]; });
      MfSubHdr hd;
      hd.q0 = int(S.sub_node.size());
      hd.nrec = int(list.size());
      hd.i0 = S.nodes[v0].Ioff;
      hd.np = int(S.nodes[v].Ioff + S.nodes[v].s - hd.i0);
      hd.b0 = S.nodes[v0].Boff;
      hd.nbm = int(S.nodes[v].Boff + S.nodes[v].m - hd.b0);
      hd.mroot = S.nodes[v].m;
      hd.uoff_root = S.nodes[v].uoff;
      hd.bl0 = long(S.sub_bloc.size());
      hd.inv0 = -1;
      long inv1 = 0;
      for (int x = v0; x <= v; ++x)
        if (S.nodes[x].invoff >= 0) {
          if (hd.inv0 < 0) hd.inv0 = S.nodes[x].invoff;
          inv1 = S.nodes[x].invoff + 2 * (S.nodes[x].s + S.nodes[x].m);
        }
      if (hd.inv0 < 0) hd.inv0 = 0;
      hd.ninv = int(std::max<long>(0, inv1 - hd.inv0));
      std::map<int, int> lu;                          // LDS offset of each node's u
      int lds = 0;
      for (int x : list) {
        lu[x] = x == v ? -1 : lds;
        if (x != v) lds += S.nodes[x].m;
      }
      S.sub_lds = std::max(S.sub_lds, lds);
      for (int x : list) {
        const MfNode& nd = S.nodes[x];
        MfSubNode r;
        r.so = nd.Soff;
        r.go = nd.Goff;
        r.gto = nd.GToff;
        r.s = nd.s;
        r.m = nd.m;
        r.pI = int(nd.Ioff - hd.i0);
        r.pinv = nd.invoff >= 0 ? int(nd.invoff - hd.inv0) : -1;
        r.pB = int(nd.Boff - hd.b0);
        r.lu0 = nd.ch0 >= 0 ? lu[nd.ch0] : -1;
        r.lu1 = nd.ch1 >= 0 ? lu[nd.ch1] : -1;
        r.lu = lu[x];
        S.sub_node.push_back(r);
      }
      // local indices of the ring entries: the subtree's points, then the root's ring
      std::unordered_map<int, int> loc;
      for (int t = 0; t < hd.np; ++t) loc[S.I[hd.i0 + t]] = t;
      for (int t = 0; t < hd.mroot; ++t) loc[S.B[hd.b0 + hd.nbm - hd.mroot + t]] = hd.np + t;
      for (int t = 0; t < hd.nbm; ++t) {
        auto it = loc.find(S.B[hd.b0 + t]);
        if (it == loc.end()) throw std::runtime_error("multifrontal: subtree ring point");
        S.sub_bloc.push_back(it->second);
      }
      int q = 0;
      for (int h = 0; h <= T + 1; ++h) {
        while (q < int(list.size()) && S.height[list[q]] < h) ++q;
        S.sub_lev.push_back(hd.q0 + q);
      }
      mx.nrec = std::max(mx.nrec, hd.nrec);
      mx.np = std::max(mx.np, hd.np);
      mx.ninv = std::max(mx.ninv, hd.ninv);
      mx.nbm = std::max(mx.nbm, hd.nbm);
      mx.mroot = std::max(mx.mroot, hd.mroot);
      S.sub_hdr.push_back(hd);
    }
  }
  S.fmax.assign(S.H + 1, 0);
  S.bmax.assign(S.H + 1, 0);
  S.fbig.assign(S.H + 1, 1);
  S.bbig.assign(S.H + 1, 1);
  for (int v = 0; v < nn; ++v) {
    const MfNode& nd = S.nodes[v];
    if (is_small(v) || nd.s <= 64) S.fbig[S.height[v]] = 0;
    if (is_small(v)) S.bbig[S.height[v]] = 0;
  }
  // the row prefetch costs occupancy (about 180 registers): worth it only where a height has
  // few workgroups to overlap (at most 3 per compute unit)
  for (int h = 0; h <= S.H; ++h) {
    if (S.fwd0[h + 1] - S.fwd0[h] > 768) S.fbig[h] = 0;
    if (S.bwd0[h + 1] - S.bwd0[h] > 768) S.bbig[h] = 0;
  }
  for (int v = 0; v < nn; ++v) {
    const MfNode& nd = S.nodes[v];
    if (is_small(v)) continue;
    S.fmax[S.height[v]] = std::max(S.fmax[S.height[v]], nd.s + nd.m);
    S.bmax[S.height[v]] = std::max(S.bmax[S.height[v]], nd.m);
  }
}

std::mutex g_sym_mu;
std::map<std::pair<int, int>, std::unique_ptr<MfSym>> g_sym;

}  // namespace

// ------------------------------------------------------------------------------------------
// Factorisation kernels
// ------------------------------------------------------------------------------------------

namespace {

__device__ __forceinline__ int mf_region(int a, int M) { return a == 0 ? 0 : (a == M - 1 ? 2 : 1); }

// A_c(g1, g2): the stencil of g1 at offset g2 - g1 (class tables or per-point), zero beyond it.
template <int P>
__device__ __forceinline__ double2 coarse_entry(const double2* __restrict__ coef, int pn, int Mc,
                                                int g1, int g2) {
  constexpr int W = 2 * P + 1, W2 = W * W;
  const int b1 = g1 / Mc, a1 = g1 - b1 * Mc, b2 = g2 / Mc, a2 = g2 - b2 * Mc;
  const int dx = a2 - a1, dy = b2 - b1;
  if (dx < -P || dx > P || dy < -P || dy > P) return make_double2(0.0, 0.0);
  const int d = (dy + P) * W + dx + P;
  if (pn) return coef[long(d) * Mc * Mc + g1];
  const int cls = (b1 % P) * P + (a1 % P);
  const int reg = mf_region(b1, Mc) * 3 + mf_region(a1, Mc);
  return coef[(cls * 9 + reg) * W2 + d];
}

// Row r of the front of node v: F[r][c] = A_c(I/B point r, I/B point c) when r or c is in I
// (the row of the point in I, so that F_BI = F_IB^T exactly), zero in the F_BB part.
template <int P>
__global__ void __launch_bounds__(256)
k_mf_front(MfView mv, const double2* __restrict__ coef, int pn, int Mc, const int2* __restrict__ rows,
           double2* __restrict__ arena, const long* __restrict__ foff) {
  const int2 t = rows[blockIdx.x];
  const MfNode nd = mv.nodes[t.x];
  const int s = nd.s, w = nd.s + nd.m, r = t.y;
  double2* Fr = arena + foff[t.x] + long(r) * w;
  const int gr = r < s ? mv.I[nd.Ioff + r] : mv.B[nd.Boff + r - s];
  for (int c = threadIdx.x; c < w; c += 256) {
    double2 v = make_double2(0.0, 0.0);
    if (r < s || c < s) {
      const int gc = c < s ? mv.I[nd.Ioff + c] : mv.B[nd.Boff + c - s];
      v = r < s ? coarse_entry<P>(coef, pn, Mc, gr, gc) : coarse_entry<P>(coef, pn, Mc, gc, gr);
    }
    Fr[c] = v;
  }
}

// Extend-add of row j of child c's update matrix U_c = F_c[s_c:, s_c:] into its parent's front.
// One child slot per launch (the two children of a node may hit the same entries).
__global__ void __launch_bounds__(256)
k_mf_extend(MfView mv, const int* __restrict__ parent, const int2* __restrict__ rows,
            double2* __restrict__ arena, const long* __restrict__ foff) {
  const int2 t = rows[blockIdx.x];
  const int c = t.x, j = t.y, v = parent[c];
  const MfNode cn = mv.nodes[c], pnd = mv.nodes[v];
  const int wc = cn.s + cn.m, wp = pnd.s + pnd.m;
  const double2* U = arena + foff[c] + long(cn.s + j) * wc + cn.s;
  const int* map = mv.map + cn.mapoff;
  double2* Fp = arena + foff[v] + long(map[j]) * wp;
  for (int k = threadIdx.x; k < cn.m; k += 256) {
    const double2 u = U[k];
    double2 f = Fp[map[k]];
    f.x += u.x;
    f.y += u.y;
    Fp[map[k]] = f;
  }
}

// S_v = F_II^{-1} for s <= 64, one workgroup per node: the symmetric Gauss-Jordan sweep in LDS
// on the upper triangle mirrored (every pivot X[t][t] -> -1/p, row and column t scaled by 1/p,
// the rest X[r][c] -= X[r][t] X[t][c] / p), leaving -F_II^{-1}.
__global__ void __launch_bounds__(256)
k_mf_gj(MfView mv, const int* __restrict__ list, const double2* __restrict__ arena,
        const long* __restrict__ foff, double2* __restrict__ Fac, int* flag) {
  extern __shared__ double2 X[];
  __shared__ double2 rowt[64], colt[64];
  const int v = list[blockIdx.x];
  const MfNode nd = mv.nodes[v];
  const int s = nd.s, w = nd.s + nd.m, ld = s + 1;
  const double2* Fv = arena + foff[v];
  for (int idx = threadIdx.x; idx < s * s; idx += 256) {
    const int r = idx / s, c = idx - r * s;
    X[r * ld + c] = Fv[long(min(r, c)) * w + max(r, c)];
  }
  __syncthreads();
  bool bad = false;
  for (int t = 0; t < s; ++t) {
    const double2 pv = X[t * ld + t];
    const double mag = pv.x * pv.x + pv.y * pv.y;
    if (!(mag > 0.0) || !isfinite(mag)) bad = true;
    const double2 pinv = make_double2(pv.x / mag, -pv.y / mag);
    for (int i = threadIdx.x; i < s; i += 256) {
      rowt[i] = X[t * ld + i];
      colt[i] = X[i * ld + t];
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < s * s; idx += 256) {
      const int r = idx / s, c = idx - r * s;
      double2 v;
      if (r == t) {
        v = (c == t) ? make_double2(-pinv.x, -pinv.y) : cmul<double>(rowt[c], pinv);
      } else if (c == t) {
        v = cmul<double>(colt[r], pinv);
      } else {
        const double2 g = cmul<double>(colt[r], pinv);
        v = X[r * ld + c];
        v.x -= g.x * rowt[c].x - g.y * rowt[c].y;
        v.y -= g.x * rowt[c].y + g.y * rowt[c].x;
      }
      X[r * ld + c] = v;
    }
    __syncthreads();
  }
  if (bad && threadIdx.x == 0) atomicOr(flag, 1);
  double2* Sv = Fac + nd.Soff;
  for (int idx = threadIdx.x; idx < s * s; idx += 256) {
    const int r = idx / s, c = idx - r * s;
    const double2 x = X[min(r, c) * ld + max(r, c)];
    Sv[idx] = make_double2(-x.x, -x.y);
  }
}

// F_II of a large node into its S slot (row-major s x s), for the in-place sweep inverse.
__global__ void __launch_bounds__(256)
k_mf_copy_ii(const double2* __restrict__ Fv, int s, int w, double2* __restrict__ Sv) {
  const long idx = long(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= long(s) * s) return;
  const int r = int(idx / s), c = int(idx - long(r) * s);
  Sv[idx] = Fv[long(r) * w + c];
}

// Batched complex GEMM of varying sizes: C = A B (sub = 0) or C -= A B (sub = 1), all row-major.
// 64 x 64 output tiles, 256 threads in a 16 x 16 grid with 4 x 4 outputs each, k in steps of 8
// staged in LDS; each output sums its k terms in ascending order.
// Operands are offsets into the factor (F) or the front arena (W): flags bit 0 / 1 / 2 set
// when A / B / C lie in the arena, bit 3 for C -= A B.
struct GemmDesc {
  long a, b, c;
  int lda, ldb, ldc, M, N, K, flags;
  long tile0;
};

__global__ void __launch_bounds__(256)
k_mf_gemm(const GemmDesc* __restrict__ descs, const int* __restrict__ tdesc, double2* Fbase,
          double2* Wbase) {
  __shared__ double2 As[8][65], Bs[8][65];
  const GemmDesc gd = descs[tdesc[blockIdx.x]];
  struct {
    const double2* A;
    const double2* B;
    double2* C;
    int lda, ldb, ldc, M, N, K, sub;
    long tile0;
  } g{(gd.flags & 1 ? Wbase : Fbase) + gd.a, (gd.flags & 2 ? Wbase : Fbase) + gd.b,
      (gd.flags & 4 ? Wbase : Fbase) + gd.c, gd.lda, gd.ldb, gd.ldc, gd.M, gd.N, gd.K,
      (gd.flags >> 3) & 1, gd.tile0};
  const long t = long(blockIdx.x) - g.tile0;
  const int tn = (g.N + 63) / 64;
  const int row0 = int(t / tn) * 64, col0 = int(t % tn) * 64;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double2 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = make_double2(0.0, 0.0);
  for (int k0 = 0; k0 < g.K; k0 += 8) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int idx = threadIdx.x + 256 * q;
      const int ra = idx >> 3, ka = idx & 7;
      As[ka][ra] = (row0 + ra < g.M && k0 + ka < g.K) ? g.A[long(row0 + ra) * g.lda + k0 + ka]
                                                     : make_double2(0.0, 0.0);
      const int kb = idx >> 6, cb = idx & 63;
      Bs[kb][cb] = (k0 + kb < g.K && col0 + cb < g.N) ? g.B[long(k0 + kb) * g.ldb + col0 + cb]
                                                     : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      double2 a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[k][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[k][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) cfma(acc[i][j], a[i], b[j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = row0 + ty + 16 * i, c = col0 + tx + 16 * j;
      if (r >= g.M || c >= g.N) continue;
      double2* cp = g.C + long(r) * g.ldc + c;
      if (g.sub) {
        double2 v = *cp;
        v.x -= acc[i][j].x;
        v.y -= acc[i][j].y;
        *cp = v;
      } else {
        *cp = acc[i][j];
      }
    }
}

template <int P>
void launch_front(const MfView& mv, const DevOp<double>& cop, int Mc, const int2* rows, int nrows,
                  double2* arena, const long* foff, hipStream_t st) {
  k_mf_front<P><<<nrows, 256, 0, st>>>(mv, cop.coef, cop.pn, Mc, rows, arena, foff);
}

// Everything of a factorisation and a solve that depends only on the mesh class, on one
// device: the symbolic view (node table, point lists, maps, node order, tasks) and the
// factorisation's launch tables (front offsets in the arena, front rows, extend-add rows,
// small inversions, parents, GEMM descriptors and tile maps, per height). Built once per
// (device, p, n_c) and kept until the process ends.
struct MfHeightLaunch {
  size_t r0, r1, e0[2], e1[2], g0, g1, d0[2], d1[2], t0[2], t1[2];
  int smax;                     // largest separator of the small inversions
  std::vector<int> big;         // nodes inverted by the sweep
  std::vector<long> bigoff;     // their fronts' offsets in the arena
  size_t z0 = 0, z1 = 0;        // their sweep descriptors
  int maxT = 0;                 // largest tile count among them
};
struct MfPlan {
  MfView view;                  // device pointers
  MfView* dview = nullptr;      // the same struct on the device
  long arena = 0;               // front arena elements
  size_t maxbig = 0;
  std::vector<MfHeightLaunch> hl;
  const long* foff = nullptr;
  const int2 *rows = nullptr, *ext = nullptr;
  const int *gj = nullptr, *parent = nullptr, *td = nullptr;
  const GemmDesc* gd = nullptr;
  const SweepNode* zn = nullptr;   // sweep descriptors of the large separators, by height
  long zw = 0, zr = 0;             // panel and pivot-inverse work of the largest height's batch
};

std::mutex g_plan_mu;
std::map<std::tuple<int, int, int>, std::unique_ptr<MfPlan>> g_plans;

const MfPlan& mf_plan(const MfSym& sym, hipStream_t st) {
  int dev = 0;
  HZ_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> guard(g_plan_mu);
  auto& slot = g_plans[std::make_tuple(dev, sym.p, sym.nc)];
  if (slot) return *slot;
  std::unique_ptr<MfPlan> P(new MfPlan());
  const int nn = int(sym.nodes.size());
  // front arena: the fronts of height h live until their parents (at heights up to
  // last[h]) have taken their update matrices; first fit over the heights' intervals
  std::vector<int> last(sym.H + 1, 0);
  for (int v = 0; v < nn; ++v)
    if (sym.parent[v] >= 0)
      last[sym.height[v]] = std::max(last[sym.height[v]], sym.height[sym.parent[v]]);
  std::vector<long> hsize(sym.H + 1, 0), hoff(sym.H + 1, 0);
  for (int h = 0; h <= sym.H; ++h)
    for (int v : sym.at[h]) hsize[h] += long(sym.nodes[v].s + sym.nodes[v].m) * (sym.nodes[v].s + sym.nodes[v].m);
  std::vector<std::pair<long, long>> live;   // (offset, size) of live heights' blocks
  std::vector<int> live_h;
  for (int h = 0; h <= sym.H; ++h) {
    for (size_t i = 0; i < live.size();) {     // heights whose parents all precede h
      if (last[live_h[i]] < h) { live.erase(live.begin() + i); live_h.erase(live_h.begin() + i); }
      else ++i;
    }
    std::vector<std::pair<long, long>> sorted = live;
    std::sort(sorted.begin(), sorted.end());
    long off = 0;
    for (auto& b : sorted) {
      if (b.first - off >= hsize[h]) break;
      off = std::max(off, b.first + b.second);
    }
    hoff[h] = off;
    P->arena = std::max(P->arena, off + hsize[h]);
    live.push_back({off, hsize[h]});
    live_h.push_back(h);
  }
  std::vector<long> fo(nn, 0);
  for (int h = 0; h <= sym.H; ++h) {
    long o = hoff[h];
    for (int v : sym.at[h]) {
      fo[v] = o;
      o += long(sym.nodes[v].s + sym.nodes[v].m) * (sym.nodes[v].s + sym.nodes[v].m);
    }
  }
  std::vector<int2> rows, ext;
  std::vector<int> gj, parent(sym.parent.begin(), sym.parent.end());
  std::vector<GemmDesc> gd;
  std::vector<int> td;
  std::vector<SweepNode> zn;
  P->hl.assign(sym.H + 1, MfHeightLaunch());
  for (int h = 0; h <= sym.H; ++h) {
    MfHeightLaunch& L = P->hl[h];
    L.r0 = rows.size();
    for (int v : sym.at[h])
      for (int r = 0; r < sym.nodes[v].s + sym.nodes[v].m; ++r) rows.push_back(make_int2(v, r));
    L.r1 = rows.size();
    for (int slot = 0; slot < 2; ++slot) {
      L.e0[slot] = ext.size();
      for (int v : sym.at[h]) {
        const int c = slot == 0 ? sym.nodes[v].ch0 : sym.nodes[v].ch1;
        if (c < 0) continue;
        for (int j = 0; j < sym.nodes[c].m; ++j) ext.push_back(make_int2(c, j));
      }
      L.e1[slot] = ext.size();
    }
    L.g0 = gj.size();
    L.smax = 0;
    for (int v : sym.at[h]) {
      if (sym.nodes[v].s <= 64) {
        gj.push_back(v);
        L.smax = std::max(L.smax, sym.nodes[v].s);
      } else {
        L.big.push_back(v);
        L.bigoff.push_back(fo[v]);
        P->maxbig = std::max(P->maxbig, size_t(sym.nodes[v].s));
      }
    }
    L.g1 = gj.size();
    {
      // the large separators of this height, swept together
      L.z0 = zn.size();
      long w = 0, r = 0;
      for (int v : L.big) {
        const MfNode& nd = sym.nodes[v];
        SweepNode z;
        z.xoff = nd.Soff;
        z.woff = w;
        z.roff = r;
        z.n = nd.s;
        z.T = (nd.s + 31) / 32;
        w += long(sweep_panel_elems(size_t(nd.s)));
        r += long(sweep_pinv_elems());
        L.maxT = std::max(L.maxT, z.T);
        zn.push_back(z);
      }
      L.z1 = zn.size();
      P->zw = std::max(P->zw, w);
      P->zr = std::max(P->zr, r);
    }
    for (int phase = 0; phase < 2; ++phase) {
      L.d0[phase] = gd.size();
      L.t0[phase] = td.size();
      for (int v : sym.at[h]) {
        const MfNode& nd = sym.nodes[v];
        if (nd.m == 0) continue;
        const int s = nd.s, m = nd.m, w = s + m;
        const long F = fo[v];
        std::vector<GemmDesc> add;
        if (phase == 0) {
          add.push_back({nd.Soff, F + s, nd.Goff, s, w, m, s, m, s, 2, 0});                // G = S F_IB
          add.push_back({F + long(s) * w, nd.Soff, nd.GToff, w, s, s, m, s, s, 1, 0});     // G^T = F_BI S
        } else {
          add.push_back({F + long(s) * w, nd.Goff, F + long(s) * w + s, w, m, w, m, m, s,
                         1 | 4 | 8, 0});                                                   // U
        }
        for (GemmDesc d : add) {
          d.tile0 = long(td.size() - L.t0[phase]);
          const long nt = long((d.M + 63) / 64) * ((d.N + 63) / 64);
          for (long q = 0; q < nt; ++q) td.push_back(int(gd.size() - L.d0[phase]));
          gd.push_back(d);
        }
      }
      L.d1[phase] = gd.size();
      L.t1[phase] = td.size();
    }
  }
  // one device buffer: the symbolic arrays and view, then the factorisation's tables
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  std::vector<std::pair<const void*, size_t>> parts = {
      {sym.nodes.data(), sym.nodes.size() * sizeof(MfNode)}, {sym.I.data(), sym.I.size() * 4},
      {sym.B.data(), sym.B.size() * 4}, {sym.map.data(), sym.map.size() * 4},
      {sym.hn.data(), sym.hn.size() * 4}, {sym.fwd.data(), sym.fwd.size() * sizeof(MfTask)},
      {sym.bwd.data(), sym.bwd.size() * sizeof(MfTask)}, {sym.inv.data(), sym.inv.size() * 4},
      {sym.sub_hdr.data(), sym.sub_hdr.size() * sizeof(MfSubHdr)},
      {sym.sub_node.data(), sym.sub_node.size() * sizeof(MfSubNode)},
      {sym.sub_lev.data(), sym.sub_lev.size() * 4},
      {sym.sub_bloc.data(), sym.sub_bloc.size() * 4},
      {nullptr, sizeof(MfView)},
      {fo.data(), fo.size() * 8}, {rows.data(), rows.size() * 8}, {ext.data(), ext.size() * 8},
      {gj.data(), gj.size() * 4}, {parent.data(), parent.size() * 4},
      {gd.data(), gd.size() * sizeof(GemmDesc)}, {td.data(), td.size() * 4},
      {zn.data(), zn.size() * sizeof(SweepNode)}};
  size_t tot = 0;
  for (auto& q : parts) tot += al(q.second);
  char* d = nullptr;
  HZ_HIP(hipMalloc(reinterpret_cast<void**>(&d), std::max<size_t>(tot, 256)));
  std::vector<char> h(tot, 0);
  std::vector<char*> at;
  size_t o = 0;
  for (auto& q : parts) {
    if (q.first) std::memcpy(h.data() + o, q.first, q.second);
    at.push_back(d + o);
    o += al(q.second);
  }
  MfView& v = P->view;
  v.nodes = reinterpret_cast<const MfNode*>(at[0]);
  v.I = reinterpret_cast<const int*>(at[1]);
  v.B = reinterpret_cast<const int*>(at[2]);
  v.map = reinterpret_cast<const int*>(at[3]);
  v.hn = reinterpret_cast<const int*>(at[4]);
  v.fwd = reinterpret_cast<const MfTask*>(at[5]);
  v.bwd = reinterpret_cast<const MfTask*>(at[6]);
  v.inv = reinterpret_cast<const int*>(at[7]);
  v.sub_hdr = reinterpret_cast<const MfSubHdr*>(at[8]);
  v.sub_node = reinterpret_cast<const MfSubNode*>(at[9]);
  v.sub_lev = reinterpret_cast<const int*>(at[10]);
  v.sub_bloc = reinterpret_cast<const int*>(at[11]);
  P->dview = reinterpret_cast<MfView*>(at[12]);
  std::memcpy(h.data() + (at[12] - d), &v, sizeof(MfView));
  P->foff = reinterpret_cast<const long*>(at[13]);
  P->rows = reinterpret_cast<const int2*>(at[14]);
  P->ext = reinterpret_cast<const int2*>(at[15]);
  P->gj = reinterpret_cast<const int*>(at[16]);
  P->parent = reinterpret_cast<const int*>(at[17]);
  P->gd = reinterpret_cast<const GemmDesc*>(at[18]);
  P->td = reinterpret_cast<const int*>(at[19]);
  P->zn = reinterpret_cast<const SweepNode*>(at[20]);
  HZ_HIP(hipMemcpyAsync(d, h.data(), tot, hipMemcpyHostToDevice, st));
  HZ_HIP(hipStreamSynchronize(st));   // h is local
  slot = std::move(P);
  return *slot;
}

}  // namespace

MfView* mf_device_view(const MfSym& sym, MfView* host_copy, hipStream_t st) {
  const MfPlan& P = mf_plan(sym, st);
  if (host_copy) *host_copy = P.view;
  return P.dview;
}

hz_status mf_factor(const MfSym& sym, const DevOp<double>& cop, double2* Fac, int* flag,
                    hipStream_t st) {
  const MfPlan& P = mf_plan(sym, st);
  const MfView& mv = P.view;
  double2* ws = nullptr;
  HZ_HIP(hipMallocAsync(reinterpret_cast<void**>(&ws), size_t(std::max<long>(P.arena, 1)) * 16, st));
  // sweep work for the large inversions of one height (all swept together)
  double2 *W = nullptr, *R = nullptr;
  if (P.zw > 0) {
    HZ_HIP(hipMallocAsync(reinterpret_cast<void**>(&W), size_t(P.zw) * 16, st));
    HZ_HIP(hipMallocAsync(reinterpret_cast<void**>(&R), size_t(P.zr) * 16, st));
  }
  HZ_HIP(hipMemsetAsync(flag, 0, sizeof(int), st));
  const int p = sym.p, Mc = sym.Mc;
  for (int h = 0; h <= sym.H; ++h) {
    const MfHeightLaunch& L = P.hl[h];
    const int nr = int(L.r1 - L.r0);
    if (nr > 0) {
      if (p == 1) launch_front<1>(mv, cop, Mc, P.rows + L.r0, nr, ws, P.foff, st);
      else if (p == 2) launch_front<2>(mv, cop, Mc, P.rows + L.r0, nr, ws, P.foff, st);
      else launch_front<3>(mv, cop, Mc, P.rows + L.r0, nr, ws, P.foff, st);
      HZ_HIP(hipGetLastError());
    }
    for (int slot = 0; slot < 2; ++slot) {
      const int ne = int(L.e1[slot] - L.e0[slot]);
      if (ne > 0) k_mf_extend<<<ne, 256, 0, st>>>(mv, P.parent, P.ext + L.e0[slot], ws, P.foff);
    }
    const int ng = int(L.g1 - L.g0);
    if (ng > 0) {
      static std::once_flag once;
      std::call_once(once, [] {
        HZ_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mf_gj),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, 64 * 65 * 16));
      });
      k_mf_gj<<<ng, 256, size_t(L.smax) * (L.smax + 1) * 16, st>>>(mv, P.gj + L.g0, ws, P.foff,
                                                                    Fac, flag);
    }
    for (size_t q = 0; q < L.big.size(); ++q) {
      const MfNode& nd = sym.nodes[L.big[q]];
      const long n2 = long(nd.s) * nd.s;
      k_mf_copy_ii<<<unsigned((n2 + 255) / 256), 256, 0, st>>>(ws + L.bigoff[q], nd.s,
                                                              nd.s + nd.m, Fac + nd.Soff);
    }
    if (L.z1 > L.z0)
      sweep_inverse_batch(Fac, P.zn + L.z0, int(L.z1 - L.z0), L.maxT, W, R, flag, st);
    for (int phase = 0; phase < 2; ++phase) {
      const int nt = int(L.t1[phase] - L.t0[phase]);
      if (nt > 0) k_mf_gemm<<<nt, 256, 0, st>>>(P.gd + L.d0[phase], P.td + L.t0[phase], Fac, ws);
    }
    HZ_HIP(hipGetLastError());
  }
  int hflag = 0;
  HZ_HIP(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  HZ_HIP(hipStreamSynchronize(st));
  if (W) (void)hipFreeAsync(W, st);
  if (R) (void)hipFreeAsync(R, st);
  (void)hipFreeAsync(ws, st);
  return hflag ? HZ_ESINGULAR : HZ_OK;
}

// ------------------------------------------------------------------------------------------
// Solve kernels
// ------------------------------------------------------------------------------------------

namespace {

// Column groups of 64 requested ahead per wave on the large-node heights (rows up to 1536).
constexpr int kMfPf = 24;

template <typename T> __device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// One launch per tree height and pass; workgroup (task, job, right-hand-side group). Large
// nodes: the workgroup assembles the node's front vector in LDS and each wave forms rows of
// one matrix (lanes over the columns, then a butterfly sum); with PF > 0 (heights whose tasks
// are all of that kind) each wave requests the first PF column groups of its first row before
// the front vector is gathered, so that the row streams in while the gather waits. Small nodes
// (s + m <= 64): one wave per node, lane r forms row r (lanes read consecutive entries of a
// stored row). The front vector is f_i = (b at I_v, or 0) + child 0's u + child 1's u at
// position i, in that order, through the node's inverse maps.
template <typename T, int NR, bool FWD, int PF>
__global__ void __launch_bounds__(256)
k_mf_solve(CsJobs<T> jobs, int task0, long cstride) {
  extern __shared__ char smem[];
  V2<T>* f = reinterpret_cast<V2<T>*>(smem);
  const CoarseJob<T>* job = &jobs.j[blockIdx.y];
  const int hb = blockIdx.z * NR;
  const int nr = min(NR, job->nrhs - hb);
  if (nr <= 0) return;
  const MfView mv = *job->mf;
  const MfTask t = (FWD ? mv.fwd : mv.bwd)[task0 + blockIdx.x];
  const V2<T>* __restrict__ Fac = job->S;
  const V2<T>* b = job->b + long(hb) * cstride;
  V2<T>* y = job->y + long(hb) * cstride;
  V2<T>* u = job->gbuf + long(hb) * job->ustride;
  const long us = job->ustride;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (t.kind <= 2 || t.kind == 5) {
    const MfNode nd = mv.nodes[t.v];
    const int s = nd.s, m = nd.m, w = s + m;
    const V2<T>* X = Fac + (t.kind == 0 ? nd.Soff : t.kind == 1 ? nd.GToff : nd.Goff);
    const int len = t.kind == 2 ? m : s;                // row length of the matrix
    const int vl = FWD ? w : m;                          // LDS vector per right-hand side
    V2<T> pre[PF > 0 ? PF : 1];
    if constexpr (PF > 0) {
      const int r = t.r0 + wave;
      const V2<T>* xr = X + long(r) * len;
#pragma unroll
      for (int q = 0; q < PF; ++q) {
        const int k = lane + 64 * q;
        pre[q] = (r < t.r1 && k < len) ? xr[k] : czero<T>();
      }
    }
    if (FWD) {
      // the task's rows read f_I and, for rows of G^T f_I, f_B at those rows only: gather
      // positions [0, s) and [lo, hi)
      const bool kids = nd.invoff >= 0;
      const long u0 = kids ? mv.nodes[nd.ch0].uoff : 0, u1 = kids ? mv.nodes[nd.ch1].uoff : 0;
      const int lo = t.kind == 1 ? s + t.r0 : t.kind == 5 ? max(s, t.r0) : s;
      const int hi = t.kind == 1 ? s + t.r1 : t.kind == 5 ? max(s, t.r1) : s;
      const int ng = s + (hi - lo);
      for (int q = threadIdx.x; q < ng; q += 256) {
        const int i = q < s ? q : lo + (q - s);
        const int j0 = kids ? mv.inv[nd.invoff + 2 * i] : -1;
        const int j1 = kids ? mv.inv[nd.invoff + 2 * i + 1] : -1;
        const int gi = i < s ? mv.I[nd.Ioff + i] : 0;
        for (int h = 0; h < nr; ++h) {
          V2<T> v = i < s ? b[h * cstride + gi] : czero<T>();
          if (j0 >= 0) {
            const V2<T> a = u[h * us + u0 + j0];
            v.x += a.x;
            v.y += a.y;
          }
          if (j1 >= 0) {
            const V2<T> a = u[h * us + u1 + j1];
            v.x += a.x;
            v.y += a.y;
          }
          f[h * w + i] = v;
        }
      }
    } else {
      for (int k = threadIdx.x; k < m; k += 256)
        for (int h = 0; h < nr; ++h) f[h * m + k] = y[h * cstride + mv.B[nd.Boff + k]];
    }
    __syncthreads();
    if (FWD && t.kind == 5) {
      // thread per row: rows r < s of S (symmetric: walk row k, entry r), rows s + r' of
      // G^T f_I (walk row i of G, entry r'); consecutive threads read consecutive entries
      const int r = t.r0 + int(threadIdx.x);
      if (r < t.r1) {
        V2<T> acc[NR];
#pragma unroll
        for (int h = 0; h < NR; ++h) acc[h] = czero<T>();
        const bool zr = r < s;
        const V2<T>* Xc = zr ? Fac + nd.Soff + r : Fac + nd.Goff + (r - s);
        const int ld = zr ? s : m;
#pragma unroll 4
        for (int k = 0; k < s; ++k) {
          const V2<T> xv = Xc[long(k) * ld];
#pragma unroll
          for (int h = 0; h < NR; ++h)
            if (h < nr) cfma(acc[h], xv, f[h * w + k]);
        }
#pragma unroll
        for (int h = 0; h < NR; ++h) {
          if (h >= nr) continue;
          if (zr) {
            y[h * cstride + mv.I[nd.Ioff + r]] = acc[h];
          } else {
            const V2<T> fb = f[h * w + r];
            V2<T> o;
            o.x = fb.x - acc[h].x;
            o.y = fb.y - acc[h].y;
            u[h * us + nd.uoff + (r - s)] = o;
          }
        }
      }
      return;
    }
    bool first = true;
    for (int r = t.r0 + wave; r < t.r1; r += 4) {
      V2<T> acc[NR];
#pragma unroll
      for (int h = 0; h < NR; ++h) acc[h] = czero<T>();
      const V2<T>* xr = X + long(r) * len;
      int k0 = lane;
      if constexpr (PF > 0) {
#pragma unroll
        for (int q = 0; q < PF; ++q) {
          const int k = lane + 64 * q;
          if (k < len) {
            const V2<T> xv = first ? pre[q] : xr[k];
#pragma unroll
            for (int h = 0; h < NR; ++h)
              if (h < nr) cfma(acc[h], xv, f[h * vl + k]);
          }
        }
        k0 = lane + 64 * PF;
      }
#pragma unroll 4
      for (int k = k0; k < len; k += 64) {
        const V2<T> xv = xr[k];
#pragma unroll
        for (int h = 0; h < NR; ++h)
          if (h < nr) cfma(acc[h], xv, f[h * vl + k]);
      }
      first = false;
#pragma unroll
      for (int h = 0; h < NR; ++h) {
        acc[h].x = wave_sum(acc[h].x);
        acc[h].y = wave_sum(acc[h].y);
      }
      if (lane == 0)
#pragma unroll
        for (int h = 0; h < NR; ++h) {
          if (h >= nr) continue;
          if (!FWD) {
            const long gi = h * cstride + mv.I[nd.Ioff + r];
            V2<T> z = y[gi];
            z.x -= acc[h].x;
            z.y -= acc[h].y;
            y[gi] = z;
          } else if (t.kind == 0) {
            y[h * cstride + mv.I[nd.Ioff + r]] = acc[h];
          } else {
            const V2<T> fb = f[h * w + s + r];
            V2<T> o;
            o.x = fb.x - acc[h].x;
            o.y = fb.y - acc[h].y;
            u[h * us + nd.uoff + r] = o;
          }
        }
    }
    return;
  }
  // small nodes: wave `wave` takes node hn[r0 + wave]; every thread passes every barrier
  const bool has = t.r0 + wave < t.r1;
  const int v = has ? mv.hn[t.r0 + wave] : 0;
  const MfNode nd = mv.nodes[v];
  const int s = nd.s, m = nd.m;
  V2<T>* fw = f + wave * (NR * 64);
  if (FWD) {
    if (has && lane < s + m)
      for (int h = 0; h < nr; ++h)
        fw[h * 64 + lane] = lane < s ? b[h * cstride + mv.I[nd.Ioff + lane]] : czero<T>();
    __syncthreads();
    for (int slot = 0; slot < 2; ++slot) {
      const int c = slot == 0 ? nd.ch0 : nd.ch1;
      if (has && c >= 0) {
        const MfNode cn = mv.nodes[c];
        if (lane < cn.m) {
          const int pos = mv.map[cn.mapoff + lane];
          for (int h = 0; h < nr; ++h) {
            const V2<T> uv = u[h * us + cn.uoff + lane];
            fw[h * 64 + pos].x += uv.x;
            fw[h * 64 + pos].y += uv.y;
          }
        }
      }
      __syncthreads();
    }
    if (has && lane < s + m) {
      V2<T> acc[NR];
#pragma unroll
      for (int h = 0; h < NR; ++h) acc[h] = czero<T>();
      if (lane < s) {
        const V2<T>* Sv = Fac + nd.Soff;     // symmetric: row k, entry lane = S[lane][k]
#pragma unroll 4
        for (int k = 0; k < s; ++k) {
          const V2<T> xv = Sv[long(k) * s + lane];
#pragma unroll
          for (int h = 0; h < NR; ++h)
            if (h < nr) cfma(acc[h], xv, fw[h * 64 + k]);
        }
#pragma unroll
        for (int h = 0; h < NR; ++h)
          if (h < nr) y[h * cstride + mv.I[nd.Ioff + lane]] = acc[h];
      } else {
        const int rr = lane - s;
        const V2<T>* Gv = Fac + nd.Goff;     // (G^T f_I)[rr] = sum_i G[i][rr] f[i]
#pragma unroll 4
        for (int i = 0; i < s; ++i) {
          const V2<T> xv = Gv[long(i) * m + rr];
#pragma unroll
          for (int h = 0; h < NR; ++h)
            if (h < nr) cfma(acc[h], xv, fw[h * 64 + i]);
        }
#pragma unroll
        for (int h = 0; h < NR; ++h) {
          if (h >= nr) continue;
          const V2<T> fb = fw[h * 64 + s + rr];
          V2<T> o;
          o.x = fb.x - acc[h].x;
          o.y = fb.y - acc[h].y;
          u[h * us + nd.uoff + rr] = o;
        }
      }
    }
  } else {
    if (has && lane < m)
      for (int h = 0; h < nr; ++h) fw[h * 64 + lane] = y[h * cstride + mv.B[nd.Boff + lane]];
    __syncthreads();
    if (has && m > 0 && lane < s) {
      V2<T> acc[NR];
#pragma unroll
      for (int h = 0; h < NR; ++h) acc[h] = czero<T>();
      const V2<T>* GTv = Fac + nd.GToff;     // (G x_B)[lane] = sum_k G^T[k][lane] x_B[k]
#pragma unroll 4
      for (int k = 0; k < m; ++k) {
        const V2<T> xv = GTv[long(k) * s + lane];
#pragma unroll
        for (int h = 0; h < NR; ++h)
          if (h < nr) cfma(acc[h], xv, fw[h * 64 + k]);
      }
#pragma unroll
      for (int h = 0; h < NR; ++h) {
        if (h >= nr) continue;
        const long gi = h * cstride + mv.I[nd.Ioff + lane];
        V2<T> z = y[gi];
        z.x -= acc[h].x;
        z.y -= acc[h].y;
        y[gi] = z;
      }
    }
  }
}

// Orders a wave's LDS writes before its reads of other lanes' entries: a wave's LDS operations
// complete in issue order, and the fences keep the compiler from moving them across.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Matrix entries a lane requests before it reads its front entries.
constexpr int kMfSubPf = 8;

// LDS extents of the bottom-subtree launch (largest over the subtrees): records, points, the
// inverse-map (forward) or ring-index (backward) entries, the local vector per right-hand
// side (points; backward also the root's ring) and the update storage.
struct MfSubDims {
  int nrec, np, nint, xs, ulds;
};

__host__ __device__ inline size_t mf_sub_vec_offset(const MfSubDims& d) {
  return (32 + size_t(d.nrec) * sizeof(MfSubNode) + size_t(d.np + d.nint) * 4 + 15) / 16 * 16;
}

// The bottom subtrees (heights 0 .. T, every node small) in one launch per pass: workgroup
// (subtree, job, right-hand-side group). The workgroup first copies the subtree's node
// records, point indices and inverse maps (forward) or ring indices (backward) into LDS with
// b (forward) or z (backward, y at the subtree's points and at the root's ring); then, one
// height at a time with a barrier between heights, the four waves take the height's nodes in
// turn, one wave per node, so that a node waits only for its own matrix rows.
// Forward, heights ascending: lane r < s + m forms row r of [S; G^T] (as the small-node tasks
// do) from f_r = (b at I_v, or 0) + child 0's u + child 1's u; the update vectors stay in LDS,
// only the subtree root's goes to memory. Backward, heights descending: x_B from the local
// vector; the rows of G x_B are split over 64 / RW lane groups (RW = 16, 32 or 64 >= s) that
// each take a contiguous part of the m columns, then summed across the groups; x_I goes to the
// local vector and to y.
template <typename T, int NR, bool FWD>
__global__ void __launch_bounds__(256)
k_mf_sub(CsJobs<T> jobs, int TT, long cstride, MfSubDims dm) {
  extern __shared__ __align__(16) char smem[];
  int* lev = reinterpret_cast<int*>(smem);
  MfSubNode* rl = reinterpret_cast<MfSubNode*>(smem + 32);
  int* il = reinterpret_cast<int*>(rl + dm.nrec);
  int* ml = il + dm.np;
  V2<T>* vl = reinterpret_cast<V2<T>*>(smem + mf_sub_vec_offset(dm));
  const CoarseJob<T>* job = &jobs.j[blockIdx.y];
  const int hb = blockIdx.z * NR;
  const int nr = min(NR, job->nrhs - hb);
  if (nr <= 0) return;
  const MfView mv = *job->mf;
  const V2<T>* __restrict__ Fac = job->S;
  const V2<T>* b = job->b + long(hb) * cstride;
  V2<T>* y = job->y + long(hb) * cstride;
  V2<T>* u = job->gbuf + long(hb) * job->ustride;
  const long us = job->ustride;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const MfSubHdr hd = mv.sub_hdr[blockIdx.x];
  const int xs = dm.xs;
  V2<T>* ub = vl + NR * xs;                                   // forward: update vectors
  V2<T>* fw = (FWD ? ub + NR * dm.ulds : ub) + wave * (NR * 64);   // the wave's f_I or x_B
  // prologue
  if (tid <= TT + 1) lev[tid] = mv.sub_lev[long(blockIdx.x) * (TT + 2) + tid] - hd.q0;
  {
    const long* src = reinterpret_cast<const long*>(mv.sub_node + hd.q0);
    long* dst = reinterpret_cast<long*>(rl);
    constexpr int W8 = int(sizeof(MfSubNode) / 8);
    for (int t = tid; t < hd.nrec * W8; t += 256) dst[t] = src[t];
  }
  if (FWD) {
    for (int t = tid; t < hd.ninv; t += 256) ml[t] = mv.inv[hd.inv0 + t];
  } else {
    for (int t = tid; t < hd.nbm; t += 256) ml[t] = mv.sub_bloc[hd.bl0 + t];
  }
  for (int t = tid; t < hd.np; t += 256) {
    const int gi = mv.I[hd.i0 + t];
    il[t] = gi;
#pragma unroll
    for (int h = 0; h < NR; ++h)
      if (h < nr) vl[h * xs + t] = FWD ? b[h * cstride + gi] : y[h * cstride + gi];
  }
  if (!FWD) {
    for (int t = tid; t < hd.mroot; t += 256) {
      const int gb = mv.B[hd.b0 + hd.nbm - hd.mroot + t];
#pragma unroll
      for (int h = 0; h < NR; ++h)
        if (h < nr) vl[h * xs + hd.np + t] = y[h * cstride + gb];
    }
  }
  __syncthreads();
  for (int step = 0; step <= TT; ++step) {
    const int ht = FWD ? step : TT - step;
    const int q1 = lev[ht + 1];
    for (int q = lev[ht] + wave; q < q1; q += 4) {
      const MfSubNode r = rl[q];
      const int s = r.s, m = r.m, w = s + m;
      if (FWD) {
        const bool row = lane < w;
        const V2<T>* col = lane < s ? Fac + r.so + lane : Fac + r.go + (lane - s);
        const int ld = lane < s ? s : m;
        V2<T> xr[kMfSubPf];
#pragma unroll
        for (int k = 0; k < kMfSubPf; ++k) xr[k] = (row && k < s) ? col[long(k) * ld] : czero<T>();
        V2<T> fl[NR];
#pragma unroll
        for (int h = 0; h < NR; ++h) fl[h] = czero<T>();
        if (row) {
          const int j0 = r.lu0 >= 0 ? ml[r.pinv + 2 * lane] : -1;
          const int j1 = r.lu1 >= 0 ? ml[r.pinv + 2 * lane + 1] : -1;
#pragma unroll
          for (int h = 0; h < NR; ++h) {
            if (h >= nr) continue;
            V2<T> v = lane < s ? vl[h * xs + r.pI + lane] : czero<T>();
            if (j0 >= 0) {
              const V2<T> a = ub[h * dm.ulds + r.lu0 + j0];
              v.x += a.x;
              v.y += a.y;
            }
            if (j1 >= 0) {
              const V2<T> a = ub[h * dm.ulds + r.lu1 + j1];
              v.x += a.x;
              v.y += a.y;
            }
            fl[h] = v;
            if (lane < s) fw[h * 64 + lane] = v;
          }
        }
        wave_sync();
        if (row) {
          V2<T> acc[NR];
#pragma unroll
          for (int h = 0; h < NR; ++h) acc[h] = czero<T>();
#pragma unroll
          for (int k = 0; k < kMfSubPf; ++k)
            if (k < s)
#pragma unroll
              for (int h = 0; h < NR; ++h)
                if (h < nr) cfma(acc[h], xr[k], fw[h * 64 + k]);
          for (int k = kMfSubPf; k < s; ++k) {
            const V2<T> xv = col[long(k) * ld];
#pragma unroll
            for (int h = 0; h < NR; ++h)
              if (h < nr) cfma(acc[h], xv, fw[h * 64 + k]);
          }
#pragma unroll
          for (int h = 0; h < NR; ++h) {
            if (h >= nr) continue;
            if (lane < s) {
              y[h * cstride + il[r.pI + lane]] = acc[h];
            } else {
              V2<T> o;
              o.x = fl[h].x - acc[h].x;
              o.y = fl[h].y - acc[h].y;
              if (r.lu >= 0) ub[h * dm.ulds + r.lu + (lane - s)] = o;
              else u[h * us + hd.uoff_root + (lane - s)] = o;
            }
          }
        }
        wave_sync();     // fw is the wave's next node's
      } else {
        if (m == 0) continue;
        const int RW = s <= 16 ? 16 : (s <= 32 ? 32 : 64);
        const int i = lane & (RW - 1), c = lane / RW;
        const int kc = (m + 64 / RW - 1) / (64 / RW);
        const int k0 = c * kc, k1 = min(m, k0 + kc);
        const V2<T>* col = Fac + r.gto + i;              // G^T[k][i] = G[i][k]
        const bool act = i < s;
        V2<T> xr[kMfSubPf];
#pragma unroll
        for (int t = 0; t < kMfSubPf; ++t)
          xr[t] = (act && k0 + t < k1) ? col[long(k0 + t) * s] : czero<T>();
        if (lane < m) {
          const int lb = ml[r.pB + lane];
#pragma unroll
          for (int h = 0; h < NR; ++h)
            if (h < nr) fw[h * 64 + lane] = vl[h * xs + lb];
        }
        wave_sync();
        V2<T> acc[NR];
#pragma unroll
        for (int h = 0; h < NR; ++h) acc[h] = czero<T>();
        if (act) {
#pragma unroll
          for (int t = 0; t < kMfSubPf; ++t)
            if (k0 + t < k1)
#pragma unroll
              for (int h = 0; h < NR; ++h)
                if (h < nr) cfma(acc[h], xr[t], fw[h * 64 + k0 + t]);
          for (int k = k0 + kMfSubPf; k < k1; ++k) {
            const V2<T> xv = col[long(k) * s];
#pragma unroll
            for (int h = 0; h < NR; ++h)
              if (h < nr) cfma(acc[h], xv, fw[h * 64 + k]);
          }
        }
#pragma unroll
        for (int h = 0; h < NR; ++h)
          for (int o = RW; o < 64; o <<= 1) {
            acc[h].x += __shfl_xor(acc[h].x, o, 64);
            acc[h].y += __shfl_xor(acc[h].y, o, 64);
          }
        if (act && c == 0)
#pragma unroll
          for (int h = 0; h < NR; ++h) {
            if (h >= nr) continue;
            V2<T> z = vl[h * xs + r.pI + i];
            z.x -= acc[h].x;
            z.y -= acc[h].y;
            vl[h * xs + r.pI + i] = z;
            y[h * cstride + il[r.pI + i]] = z;
          }
        wave_sync();
      }
    }
    __syncthreads();
  }
}

MfSubDims mf_sub_dims(const MfSym& sym, bool fwd) {
  const MfSubHdr& mx = sym.sub_max;
  MfSubDims d;
  d.nrec = mx.nrec;
  d.np = mx.np;
  d.nint = fwd ? mx.ninv : mx.nbm;
  d.xs = fwd ? mx.np : mx.np + mx.mroot;
  d.ulds = sym.sub_lds;
  return d;
}

size_t mf_sub_lds(const MfSym& sym, bool fwd, int NR, size_t item) {
  const MfSubDims d = mf_sub_dims(sym, fwd);
  return mf_sub_vec_offset(d) + size_t(NR) * (d.xs + (fwd ? d.ulds : 0) + 4 * 64) * item;
}

template <typename T, int NR>
int mf_launch_all(const MfSym& sym, const CsJobs<T>& jj, int njobs, int maxr, long cstride,
                  hipStream_t st) {
  const size_t item = sizeof(V2<T>);
  const unsigned gz = unsigned((maxr + NR - 1) / NR);
  int launches = 0;
  // LDS of a height: its largest front vector (forward) or ring (backward), or the small
  // nodes' wave regions; small requests keep more workgroups resident per CU
  auto lds_of = [&](int h, bool fwd) {
    const int mx = fwd ? sym.fmax[h] : sym.bmax[h];
    return std::max<size_t>(size_t(NR) * mx, 4 * size_t(NR) * 64) * item;
  };
  const int nsub = int(sym.sub_hdr.size());
  if (nsub > 0) {
    k_mf_sub<T, NR, true><<<dim3(nsub, njobs, gz), 256, mf_sub_lds(sym, true, NR, item), st>>>(
        jj, sym.T, cstride, mf_sub_dims(sym, true));
    ++launches;
  }
  for (int h = sym.T + 1; h <= sym.H; ++h) {
    const int n = sym.fwd0[h + 1] - sym.fwd0[h];
    if (n > 0) {
      const dim3 g(n, njobs, gz);
      if (sym.fbig[h]) k_mf_solve<T, NR, true, kMfPf><<<g, 256, lds_of(h, true), st>>>(jj, sym.fwd0[h], cstride);
      else k_mf_solve<T, NR, true, 0><<<g, 256, lds_of(h, true), st>>>(jj, sym.fwd0[h], cstride);
      ++launches;
    }
  }
  for (int h = sym.H; h > sym.T; --h) {
    const int n = sym.bwd0[h + 1] - sym.bwd0[h];
    if (n > 0) {
      const dim3 g(n, njobs, gz);
      if (sym.bbig[h]) k_mf_solve<T, NR, false, kMfPf><<<g, 256, lds_of(h, false), st>>>(jj, sym.bwd0[h], cstride);
      else k_mf_solve<T, NR, false, 0><<<g, 256, lds_of(h, false), st>>>(jj, sym.bwd0[h], cstride);
      ++launches;
    }
  }
  if (nsub > 0) {
    k_mf_sub<T, NR, false><<<dim3(nsub, njobs, gz), 256, mf_sub_lds(sym, false, NR, item), st>>>(
        jj, sym.T, cstride, mf_sub_dims(sym, false));
    ++launches;
  }
  HZ_HIP(hipGetLastError());
  return launches;
}

template <typename T, int NR>
void mf_set_lds(size_t bytes) {
  static std::mutex mu;
  static size_t done = 0;
  std::lock_guard<std::mutex> g(mu);
  if (bytes <= done) return;
  HZ_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mf_solve<T, NR, true, 0>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes)));
  HZ_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mf_solve<T, NR, false, 0>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes)));
  HZ_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mf_solve<T, NR, true, kMfPf>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes)));
  HZ_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mf_solve<T, NR, false, kMfPf>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes)));
  HZ_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mf_sub<T, NR, true>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes)));
  HZ_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mf_sub<T, NR, false>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes)));
  done = bytes;
}

}  // namespace

template <typename T>
int mf_solve_jobs(const MfSym& sym, const CoarseJob<T>* jobs, int njobs, long cstride,
                  hipStream_t st) {
  int launches = 0;
  const size_t item = sizeof(V2<T>);
  for (int j0 = 0; j0 < njobs; j0 += kMaxJobs) {
    const int nj = std::min(kMaxJobs, njobs - j0);
    CsJobs<T> jj;
    int maxr = 0;
    for (int i = 0; i < nj; ++i) {
      jj.j[i] = jobs[j0 + i];
      maxr = std::max(maxr, jobs[j0 + i].nrhs);
    }
    // right-hand sides per workgroup: as many as the front vectors' LDS allows (<= 4)
    const size_t per = std::max<size_t>(sym.maxf, 4 * 64) * item;
    auto need = [&](int nr) {
      return std::max({size_t(nr) * per, mf_sub_lds(sym, true, nr, item), mf_sub_lds(sym, false, nr, item)});
    };
    int NR = 4;
    while (NR > 1 && need(NR) > 128 * 1024) NR /= 2;
    if (need(NR) > 160 * 1024) throw std::runtime_error("multifrontal: front exceeds LDS");
    if (maxr == 1) NR = 1;
    if (NR == 4) { mf_set_lds<T, 4>(need(4)); launches += mf_launch_all<T, 4>(sym, jj, nj, maxr, cstride, st); }
    else if (NR == 2) { mf_set_lds<T, 2>(need(2)); launches += mf_launch_all<T, 2>(sym, jj, nj, maxr, cstride, st); }
    else { mf_set_lds<T, 1>(need(1)); launches += mf_launch_all<T, 1>(sym, jj, nj, maxr, cstride, st); }
  }
  return launches;
}

template int mf_solve_jobs<double>(const MfSym&, const CoarseJob<double>*, int, long, hipStream_t);
template int mf_solve_jobs<float>(const MfSym&, const CoarseJob<float>*, int, long, hipStream_t);

const MfSym& mf_symbolic(int p, int nc) {
  std::lock_guard<std::mutex> g(g_sym_mu);
  auto& slot = g_sym[{p, nc}];
  if (!slot) {
    std::unique_ptr<MfSym> s(new MfSym());
    build_symbolic(*s, p, nc);
    slot = std::move(s);
  }
  return *slot;
}

}  // namespace hz
