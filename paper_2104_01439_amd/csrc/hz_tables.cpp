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

std::vector<cd> combine_operator(const LevelTables& t, double k, cd s) {
  std::vector<cd> c(t.K.size());
  const cd k2s = s * (k * k);
  for (size_t i = 0; i < c.size(); ++i)
    c[i] = cd(t.K[i], 0.0) - k2s * t.Mm[i] - cd(0.0, k) * t.B[i];
  return c;
}

}  // namespace hz
