// Host-side construction of the stencil and transfer tables.
//
// The fine and coarse operators of the twogrid method (Sec. 4, Algorithm 1) act on a
// uniform lattice with constant k, so every row of K, M and B (Sec. 2, system matrix) is one
// of a few stencils: it depends only on the class (a mod p, b mod p) of the lattice point
// and on whether the point lies on the left/right and bottom/top boundary lines. This file
// computes those stencils from the P_p element integrals, plus the weights of the canonical
// FE prolongation (coarse basis functions evaluated at fine lattice points).
//
// Element integrals are exact: the Lagrange basis is expanded in monomials and integrated
// with  int_T xi^a eta^b = a! b! / (a+b+2)!  on the reference triangle.

#include "hz_internal.h"

#include <cmath>
#include <cstring>
#include <stdexcept>

namespace hz {

namespace {

double fact(int n) {
  double r = 1.0;
  for (int i = 2; i <= n; ++i) r *= i;
  return r;
}

// Dense solve of a small system by Gauss-Jordan with partial pivoting (in place).
void invert_small(std::vector<double>& A, int n) {
  std::vector<double> I(n * n, 0.0);
  for (int i = 0; i < n; ++i) I[i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
    for (int j = 0; j < n; ++j) {
      std::swap(A[c * n + j], A[piv * n + j]);
      std::swap(I[c * n + j], I[piv * n + j]);
    }
    double d = A[c * n + c];
    for (int j = 0; j < n; ++j) { A[c * n + j] /= d; I[c * n + j] /= d; }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      double f = A[r * n + c];
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) { A[r * n + j] -= f * A[c * n + j]; I[r * n + j] -= f * I[c * n + j]; }
    }
  }
  A = I;
}

}  // namespace

// ------------------------------------------------------------------------------------------
// Reference element
// ------------------------------------------------------------------------------------------

RefElement::RefElement(int p_) : p(p_) {
  nloc = (p + 1) * (p + 2) / 2;
  int r = 0;
  for (int j = 0; j <= p; ++j)
    for (int i = 0; i + j <= p; ++i) { ni[r] = i; nj[r] = j; ++r; }
  int m = 0;
  for (int a = 0; a <= p; ++a)
    for (int b = 0; a + b <= p; ++b) { ma[m] = a; mb[m] = b; ++m; }
  std::vector<double> V(nloc * nloc);
  for (int row = 0; row < nloc; ++row) {
    double x = double(ni[row]) / p, y = double(nj[row]) / p;
    for (int c = 0; c < nloc; ++c) V[row * nloc + c] = std::pow(x, ma[c]) * std::pow(y, mb[c]);
  }
  invert_small(V, nloc);  // V^{-1}: column k holds the monomial coefficients of phi_k
  for (int mm = 0; mm < nloc; ++mm)
    for (int k = 0; k < nloc; ++k) C[mm][k] = V[mm * nloc + k];
}

double RefElement::phi(int k, double x, double y) const {
  double s = 0.0;
  for (int mm = 0; mm < nloc; ++mm) s += C[mm][k] * std::pow(x, ma[mm]) * std::pow(y, mb[mm]);
  return s;
}

// Exact reference integrals of products of basis functions and of their derivatives.
static void reference_integrals(const RefElement& el, double Mref[10][10], double Gxx[10][10],
                                double Gxy[10][10], double Gyy[10][10]) {
  const int n = el.nloc;
  auto I = [](int a, int b) { return (a < 0 || b < 0) ? 0.0 : fact(a) * fact(b) / fact(a + b + 2); };
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < n; ++c) {
      double m = 0, xx = 0, xy = 0, yy = 0;
      for (int m1 = 0; m1 < n; ++m1)
        for (int m2 = 0; m2 < n; ++m2) {
          const double w = el.C[m1][r] * el.C[m2][c];
          if (w == 0.0) continue;
          const int a1 = el.ma[m1], b1 = el.mb[m1], a2 = el.ma[m2], b2 = el.mb[m2];
          m += w * I(a1 + a2, b1 + b2);
          if (a1 && a2) xx += w * a1 * a2 * I(a1 + a2 - 2, b1 + b2);
          if (a1 && b2) xy += w * a1 * b2 * I(a1 + a2 - 1, b1 + b2 - 1);
          if (b1 && b2) yy += w * b1 * b2 * I(a1 + a2, b1 + b2 - 2);
        }
      Mref[r][c] = m; Gxx[r][c] = xx; Gxy[r][c] = xy; Gyy[r][c] = yy;
    }
}

// ------------------------------------------------------------------------------------------
// Level tables
// ------------------------------------------------------------------------------------------

// Lattice offsets of local node r inside cell (0,0): T_L = {(0,0),(1,0),(1,1)} maps the
// reference node (i, j) to (i + j, j); T_U = {(0,0),(1,1),(0,1)} maps it to (i, i + j).
static inline void local_offset(const RefElement& el, int tri, int r, int& da, int& db) {
  if (tri == 0) { da = el.ni[r] + el.nj[r]; db = el.nj[r]; }
  else          { da = el.ni[r];            db = el.ni[r] + el.nj[r]; }
}

LevelTables build_level_tables(int p, int n, double h) {
  LevelTables t;
  t.p = p; t.n = n; t.h = h; t.M = p * n + 1;
  const int W = 2 * p + 1, W2 = W * W;
  const int ncls = p * p;
  t.K.assign(size_t(ncls) * 9 * W2, 0.0);
  t.Mm.assign(t.K.size(), 0.0);
  t.B.assign(t.K.size(), 0.0);

  RefElement el(p);
  double Mref[10][10], Gxx[10][10], Gxy[10][10], Gyy[10][10];
  reference_integrals(el, Mref, Gxx, Gxy, Gyy);
  // Element matrices of the two triangle types. x = v0 + J (xi, eta); grad = J^{-T} grad_ref.
  double Ke[2][10][10], Me[2][10][10];
  for (int tri = 0; tri < 2; ++tri) {
    double J[2][2];
    if (tri == 0) { J[0][0] = h; J[0][1] = h; J[1][0] = 0; J[1][1] = h; }
    else          { J[0][0] = h; J[0][1] = 0; J[1][0] = h; J[1][1] = h; }
    const double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    const double Ji[2][2] = {{J[1][1] / det, -J[0][1] / det}, {-J[1][0] / det, J[0][0] / det}};
    // S = J^{-1} J^{-T}: metric applied to reference gradients
    double S[2][2];
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) S[a][b] = Ji[a][0] * Ji[b][0] + Ji[a][1] * Ji[b][1];
    for (int r = 0; r < el.nloc; ++r)
      for (int c = 0; c < el.nloc; ++c) {
        Ke[tri][r][c] = std::fabs(det) * (S[0][0] * Gxx[r][c] + S[0][1] * Gxy[r][c] +
                                          S[1][0] * Gxy[c][r] + S[1][1] * Gyy[r][c]);
        Me[tri][r][c] = std::fabs(det) * Mref[r][c];
      }
  }
  // 1D edge mass of the p+1 equispaced Lagrange functions on an edge of length h:
  // expand each cardinal polynomial in monomials, integrate exactly.
  double E[4][4];
  {
    double coef[4][4] = {{0}};
    for (int s = 0; s <= p; ++s) {
      double c[4] = {1, 0, 0, 0};
      double den = 1.0;
      for (int q = 0; q <= p; ++q) {
        if (q == s) continue;
        const double tq = double(q) / p;
        double nc[4] = {0, 0, 0, 0};
        for (int d = 3; d >= 0; --d) {
          if (d > 0) nc[d] += c[d - 1];
          nc[d] -= tq * c[d];
        }
        std::memcpy(c, nc, sizeof(c));
        den *= (double(s) / p - tq);
      }
      for (int d = 0; d < 4; ++d) coef[s][d] = c[d] / den;
    }
    for (int s = 0; s <= p; ++s)
      for (int q = 0; q <= p; ++q) {
        double v = 0;
        for (int d1 = 0; d1 <= p; ++d1)
          for (int d2 = 0; d2 <= p; ++d2) v += coef[s][d1] * coef[q][d2] / (d1 + d2 + 1);
        E[s][q] = h * v;
      }
  }
  // Representative mesh of NR x NR cells: assemble the row of one point per (class, region).
  const int NR = 4, MR = p * NR + 1;
  auto coord = [&](int cls, int reg) -> int {
    if (reg == 0) return cls == 0 ? 0 : -1;
    if (reg == 2) return cls == 0 ? MR - 1 : -1;
    return p * (NR / 2) + cls;
  };
  for (int cb = 0; cb < p; ++cb)
    for (int ca = 0; ca < p; ++ca)
      for (int ry = 0; ry < 3; ++ry)
        for (int rx = 0; rx < 3; ++rx) {
          const int a0 = coord(ca, rx), b0 = coord(cb, ry);
          if (a0 < 0 || b0 < 0) continue;
          const size_t base = (size_t(cb * p + ca) * 9 + ry * 3 + rx) * W2;
          // volume terms
          for (int cj = 0; cj < NR; ++cj)
            for (int ci = 0; ci < NR; ++ci)
              for (int tri = 0; tri < 2; ++tri)
                for (int r = 0; r < el.nloc; ++r) {
                  int da, db;
                  local_offset(el, tri, r, da, db);
                  if (p * ci + da != a0 || p * cj + db != b0) continue;
                  for (int c = 0; c < el.nloc; ++c) {
                    int ea, eb;
                    local_offset(el, tri, c, ea, eb);
                    const int ox = p * ci + ea - a0, oy = p * cj + eb - b0;
                    const size_t o = base + (oy + p) * W + (ox + p);
                    t.K[o] += Ke[tri][r][c];
                    t.Mm[o] += Me[tri][r][c];
                  }
                }
          // boundary edges: bottom, top (along x), left, right (along y)
          for (int side = 0; side < 4; ++side)
            for (int e = 0; e < NR; ++e)
              for (int s = 0; s <= p; ++s) {
                int a, b;
                if (side == 0)      { a = p * e + s; b = 0; }
                else if (side == 1) { a = p * e + s; b = MR - 1; }
                else if (side == 2) { a = 0; b = p * e + s; }
                else                { a = MR - 1; b = p * e + s; }
                if (a != a0 || b != b0) continue;
                for (int q = 0; q <= p; ++q) {
                  int a2, b2;
                  if (side < 2) { a2 = p * e + q; b2 = b; }
                  else          { a2 = a; b2 = p * e + q; }
                  const size_t o = base + (b2 - b0 + p) * W + (a2 - a0 + p);
                  t.B[o] += E[s][q];
                }
              }
        }

  // Prolongation weights: value of the coarse basis function of a coarse node of class
  // (ca, cb) at the fine lattice point offset (dx, dy) in [-2p, 2p]^2 from the fine point
  // coinciding with that node. Evaluated on a representative coarse mesh (coarse lattice
  // units); the containing coarse triangle is any one holding the point (continuity).
  const int WR = 4 * p + 1;
  t.RW.assign(size_t(ncls) * WR * WR, 0.0);
  for (int cb = 0; cb < p; ++cb)
    for (int ca = 0; ca < p; ++ca) {
      const int A = p * 2 + ca, Bc = p * 2 + cb;           // coarse lattice coordinates
      for (int dy = -2 * p; dy <= 2 * p; ++dy)
        for (int dx = -2 * p; dx <= 2 * p; ++dx) {
          const double X = (2.0 * A + dx) / 2.0, Y = (2.0 * Bc + dy) / 2.0;  // coarse units
          const int I = int(std::floor(X / p)), Jc = int(std::floor(Y / p));
          const double lx = X / p - I, ly = Y / p - Jc;
          const int tri = (ly <= lx) ? 0 : 1;
          double xi, eta;
          if (tri == 0) { xi = lx - ly; eta = ly; }
          else          { xi = lx;      eta = ly - lx; }
          double val = 0.0;
          for (int r = 0; r < el.nloc; ++r) {
            int da, db;
            local_offset(el, tri, r, da, db);
            if (p * I + da == A && p * Jc + db == Bc) val = el.phi(r, xi, eta);
          }
          if (std::fabs(val) < 1e-14) val = 0.0;
          t.RW[(size_t(cb * p + ca) * WR + (dy + 2 * p)) * WR + (dx + 2 * p)] = val;
        }
    }
  return t;
}

// ------------------------------------------------------------------------------------------
// Per-cell coefficient tables (heterogeneous k)
// ------------------------------------------------------------------------------------------

namespace {

// Bivariate polynomial of total degree <= 6: c[a][b] multiplies x^a y^b.
struct Poly2 {
  double c[7][7];
  Poly2() { std::memset(c, 0, sizeof(c)); }
};

Poly2 pmul(const Poly2& A, const Poly2& B) {
  Poly2 r;
  for (int a1 = 0; a1 <= 6; ++a1)
    for (int b1 = 0; a1 + b1 <= 6; ++b1) {
      if (A.c[a1][b1] == 0.0) continue;
      for (int a2 = 0; a1 + a2 <= 6; ++a2)
        for (int b2 = 0; a1 + b1 + a2 + b2 <= 6; ++b2) r.c[a1 + a2][b1 + b2] += A.c[a1][b1] * B.c[a2][b2];
    }
  return r;
}

Poly2 paffine(double c0, double cx, double cy) {
  Poly2 r;
  r.c[0][0] = c0;
  r.c[1][0] = cx;
  r.c[0][1] = cy;
  return r;
}

Poly2 ppow(const Poly2& A, int e) {
  Poly2 r;
  r.c[0][0] = 1.0;
  for (int i = 0; i < e; ++i) r = pmul(r, A);
  return r;
}

// Integral over the reference triangle {x, y >= 0, x + y <= 1}.
double pint(const Poly2& A) {
  double s = 0.0;
  for (int a = 0; a <= 6; ++a)
    for (int b = 0; a + b <= 6; ++b)
      if (A.c[a][b] != 0.0) s += A.c[a][b] * fact(a) * fact(b) / fact(a + b + 2);
  return s;
}

// sum_m coef[m] x^ma y^mb (monomials of the element, exponents shifted by (-dx, -dy) and
// scaled for a derivative), composed with x = lx(xi, eta), y = ly(xi, eta).
Poly2 compose(const RefElement& el, const double* coef, int der, const Poly2& lx,
              const Poly2& ly) {
  Poly2 r;
  for (int m = 0; m < el.nloc; ++m) {
    if (coef[m] == 0.0) continue;
    int a = el.ma[m], b = el.mb[m];
    double f = coef[m];
    if (der == 1) { if (a == 0) continue; f *= a; --a; }
    if (der == 2) { if (b == 0) continue; f *= b; --b; }
    const Poly2 t = pmul(ppow(lx, a), ppow(ly, b));
    for (int i = 0; i <= 6; ++i)
      for (int j = 0; i + j <= 6; ++j) r.c[i][j] += f * t.c[i][j];
  }
  return r;
}

// 1D polynomial coefficients (degree <= p) of the p + 1 equispaced cardinal functions on [0, 1].
void cardinal_1d(int p, double coef[4][4]) {
  for (int s = 0; s <= p; ++s) {
    double c[4] = {1, 0, 0, 0};
    double den = 1.0;
    for (int q = 0; q <= p; ++q) {
      if (q == s) continue;
      const double tq = double(q) / p;
      double nc[4] = {0, 0, 0, 0};
      for (int d = 3; d >= 0; --d) {
        if (d > 0) nc[d] += c[d - 1];
        nc[d] -= tq * c[d];
      }
      std::memcpy(c, nc, sizeof(c));
      den *= (double(s) / p - tq);
    }
    for (int d = 0; d < 4; ++d) coef[s][d] = c[d] / den;
  }
}

}  // namespace

CellTables build_cell_tables(int p, int r, double hf) {
  CellTables t;
  t.p = p;
  t.r = r;
  const int W = 2 * p + 1, W2 = W * W, NF = 4 * r * r;
  t.K.assign(size_t(p) * p * W2 * NF, 0.0);
  t.Mm.assign(t.K.size(), 0.0);
  t.B.assign(size_t(p) * W * 2 * r, 0.0);
  RefElement el(p);
  // Level triangle T of a level cell of side r (fine-cell units): x = J_T xi.
  // Fine triangle t of sub-cell (sx, sy): x = (sx, sy) + J_t xi.
  const double JL[2][2] = {{1, 1}, {0, 1}}, JU[2][2] = {{1, 0}, {1, 1}};
  for (int cb = 0; cb < p; ++cb)
    for (int ca = 0; ca < p; ++ca) {
      const int cls = cb * p + ca;
      for (int Bc = -1; Bc <= 0; ++Bc)
        for (int Ac = -1; Ac <= 0; ++Ac)
          for (int tri = 0; tri < 2; ++tri) {
            int rl = -1;
            for (int q = 0; q < el.nloc; ++q) {
              int da, db;
              local_offset(el, tri, q, da, db);
              if (p * Ac + da == ca && p * Bc + db == cb) rl = q;
            }
            if (rl < 0) continue;
            const double(*JT)[2] = tri == 0 ? JL : JU;
            // J_T^{-1} for J_T = r * JT (det JT = 1)
            const double Ti[2][2] = {{JT[1][1] / r, -JT[0][1] / r}, {-JT[1][0] / r, JT[0][0] / r}};
            for (int sy = 0; sy < r; ++sy)
              for (int sx = 0; sx < r; ++sx)
                for (int ft = 0; ft < 2; ++ft) {
                  // the fine triangle lies in T when its centroid does
                  const double gx = sx + (ft == 0 ? 2.0 : 1.0) / 3.0;
                  const double gy = sy + (ft == 0 ? 1.0 : 2.0) / 3.0;
                  if (tri == 0 ? !(gy < gx) : !(gy > gx)) continue;
                  const double(*Jt)[2] = ft == 0 ? JL : JU;
                  // xi_T = Ti (v0_t + Jt xi) = G xi + g
                  double G[2][2], g[2];
                  for (int i = 0; i < 2; ++i) {
                    g[i] = Ti[i][0] * sx + Ti[i][1] * sy;
                    for (int j = 0; j < 2; ++j) G[i][j] = Ti[i][0] * Jt[0][j] + Ti[i][1] * Jt[1][j];
                  }
                  const Poly2 lx = paffine(g[0], G[0][0], G[0][1]);
                  const Poly2 ly = paffine(g[1], G[1][0], G[1][1]);
                  double ci[10], cj[10];
                  for (int m = 0; m < el.nloc; ++m) ci[m] = el.C[m][rl];
                  const Poly2 phi_i = compose(el, ci, 0, lx, ly);
                  // physical gradient (fine units): grad_x = T^{-T} grad_xi
                  const Poly2 di0 = compose(el, ci, 1, lx, ly), di1 = compose(el, ci, 2, lx, ly);
                  const int fx = r * Ac + sx, fy = r * Bc + sy;
                  const int f = (fy + r) * 2 * r + (fx + r);
                  for (int q = 0; q < el.nloc; ++q) {
                    int ea, eb;
                    local_offset(el, tri, q, ea, eb);
                    const int ox = p * Ac + ea - ca, oy = p * Bc + eb - cb;
                    for (int m = 0; m < el.nloc; ++m) cj[m] = el.C[m][q];
                    const Poly2 phi_j = compose(el, cj, 0, lx, ly);
                    const Poly2 dj0 = compose(el, cj, 1, lx, ly), dj1 = compose(el, cj, 2, lx, ly);
                    double kv = 0.0;
                    for (int k = 0; k < 2; ++k) {
                      // (grad_x phi)_k = Ti[0][k] d/dxi + Ti[1][k] d/deta
                      Poly2 gi, gj;
                      for (int a = 0; a <= 6; ++a)
                        for (int b = 0; a + b <= 6; ++b) {
                          gi.c[a][b] = Ti[0][k] * di0.c[a][b] + Ti[1][k] * di1.c[a][b];
                          gj.c[a][b] = Ti[0][k] * dj0.c[a][b] + Ti[1][k] * dj1.c[a][b];
                        }
                      kv += pint(pmul(gi, gj));
                    }
                    const double mv = hf * hf * pint(pmul(phi_i, phi_j));
                    const size_t o = (size_t(cls) * W2 + (oy + p) * W + (ox + p)) * NF + f;
                    t.K[o] += kv;     // |det J_t| = 1 in fine units; stiffness is scale-free
                    t.Mm[o] += mv;
                  }
                }
          }
    }
  // boundary: node at position c = p E0 + cc along a side; level edges E0 - 1, E0 (length
  // r hf) with local nodes q = 0..p; fine sub-edge s of a level edge covers t in [s/r, (s+1)/r]
  double coef[4][4];
  cardinal_1d(p, coef);
  for (int cc = 0; cc < p; ++cc)
    for (int erel = -1; erel <= 0; ++erel) {
      const int qi = cc - p * erel;
      if (qi < 0 || qi > p) continue;
      for (int d = -p; d <= p; ++d) {
        const int qj = cc + d - p * erel;
        if (qj < 0 || qj > p) continue;
        double prod[7] = {0, 0, 0, 0, 0, 0, 0};
        for (int a = 0; a <= p; ++a)
          for (int b = 0; b <= p; ++b) prod[a + b] += coef[qi][a] * coef[qj][b];
        for (int s = 0; s < r; ++s) {
          const double t0 = double(s) / r, t1 = double(s + 1) / r;
          double v = 0.0;
          for (int e = 0; e <= 2 * p; ++e)
            v += prod[e] * (std::pow(t1, e + 1) - std::pow(t0, e + 1)) / (e + 1);
          const int fe = r * erel + s;
          t.B[(size_t(cc) * W + (d + p)) * 2 * r + (fe + r)] += r * hf * v;
        }
      }
    }
  return t;
}

// Collapsed Gauss-Legendre rule on the reference triangle: xi = u, eta = (1 - u) v with
// weight w_u w_v (1 - u), q Gauss points per direction on [0, 1]; plus the basis values at
// the points and, per class and neighbouring triangle, the local index of the point.
QuadTables build_quad_tables(int p, int q) {
  QuadTables t;
  t.p = p;
  t.nq = q * q;
  std::vector<double> x(q), w(q);
  for (int i = 0; i < q; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (q + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1, p1 = z;
      for (int kk = 2; kk <= q; ++kk) {
        const double p2 = ((2 * kk - 1) * z * p1 - (kk - 1) * p0) / kk;
        p0 = p1;
        p1 = p2;
      }
      dp = q * (z * p1 - p0) / (z * z - 1);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = 0.5 * (z + 1);
    w[i] = 1.0 / ((1 - z * z) * dp * dp);
  }
  RefElement el(p);
  t.xi.resize(t.nq);
  t.eta.resize(t.nq);
  t.w.resize(t.nq);
  t.phi.assign(size_t(el.nloc) * t.nq, 0.0);
  for (int a = 0; a < q; ++a)
    for (int b = 0; b < q; ++b) {
      const int k = a * q + b;
      t.xi[k] = x[a];
      t.eta[k] = (1 - x[a]) * x[b];
      t.w[k] = w[a] * w[b] * (1 - x[a]);
      for (int r = 0; r < el.nloc; ++r) t.phi[size_t(r) * t.nq + k] = el.phi(r, t.xi[k], t.eta[k]);
    }
  t.loc.assign(size_t(p) * p * 8, -1);
  for (int cb = 0; cb < p; ++cb)
    for (int ca = 0; ca < p; ++ca)
      for (int Bc = -1; Bc <= 0; ++Bc)
        for (int Ac = -1; Ac <= 0; ++Ac)
          for (int tri = 0; tri < 2; ++tri)
            for (int r = 0; r < el.nloc; ++r) {
              int da, db;
              local_offset(el, tri, r, da, db);
              if (p * Ac + da == ca && p * Bc + db == cb)
                t.loc[size_t(cb * p + ca) * 8 + ((Bc + 1) * 2 + (Ac + 1)) * 2 + tri] = r;
            }
  return t;
}

std::vector<cd> combine_operator(const LevelTables& t, double k, cd s) {
  std::vector<cd> c(t.K.size());
  const cd k2s = s * (k * k);
  for (size_t i = 0; i < c.size(); ++i)
    c[i] = cd(t.K[i], 0.0) - k2s * t.Mm[i] - cd(0.0, k) * t.B[i];
  return c;
}

}  // namespace hz
