"""P_p Lagrange finite elements on the uniform right-triangle mesh of the unit square.

Test infrastructure (see the package header): a plain assembled-matrix discretisation.

Follows Sec. 2 of the paper: the sesquilinear form
    a_eps(u, v) = int grad u . grad conj(v) - int (k^2 + i eps) u conj(v) - i int_{dOmega} k u conj(v)
and the linear form F(v) = int f conj(v) + int_{dOmega} g conj(v), which give the
system matrix A(k, eps) = K - M(k, eps) - i B(k) with K_ij = a(phi_j, phi_i),
M_ij = m(phi_j, phi_i; k, eps), B_ij = b(phi_j, phi_i; k) and F_i = F(phi_i).

Readings taken where the paper is silent or uses another element:

* element: P_p (p = 1, 2, 3) Lagrange triangles with equispaced nodes; every square
  cell (i, j) of side h is split by its "/" diagonal into
  T_L = {(i,j), (i+1,j), (i+1,j+1)} and T_U = {(i,j), (i+1,j+1), (i,j+1)};
* the shift is written eps = beta k^2, i.e. the volume mass term is multiplied by a
  complex s = 1 + i beta; the boundary term keeps k (the shifted problem of Sec. 2
  keeps the impedance condition unchanged);
* dofs sit on the lattice (a h/p, b h/p), a, b = 0..p n, and are numbered b*M + a
  with M = p n + 1.

Element integrals use a collapsed (Duffy) Gauss-Legendre rule on the reference
triangle, exact for the polynomial degrees involved.
"""

import numpy as np
import scipy.sparse as sp


# --------------------------------------------------------------------------------------
# Reference element
# --------------------------------------------------------------------------------------

def _monomials(p):
    return [(a, b) for a in range(p + 1) for b in range(p + 1 - a)]


def _eval_monomials(p, x, y):
    """Rows: points, columns: monomials x^a y^b with a + b <= p."""
    x = np.asarray(x, float)
    y = np.asarray(y, float)
    return np.stack([x ** a * y ** b for a, b in _monomials(p)], axis=-1)


def _eval_monomial_grads(p, x, y):
    x = np.asarray(x, float)
    y = np.asarray(y, float)
    gx, gy = [], []
    for a, b in _monomials(p):
        gx.append(a * x ** max(a - 1, 0) * y ** b if a > 0 else np.zeros_like(x))
        gy.append(b * x ** a * y ** max(b - 1, 0) if b > 0 else np.zeros_like(x))
    return np.stack(gx, axis=-1), np.stack(gy, axis=-1)


def triangle_rule(q=6):
    """Collapsed Gauss-Legendre rule on {xi, eta >= 0, xi + eta <= 1}.

    xi = u, eta = (1 - u) v with Jacobian (1 - u); exact for total degree <= 2q - 2.
    """
    t, w = np.polynomial.legendre.leggauss(q)
    t = 0.5 * (t + 1.0)
    w = 0.5 * w
    U, V = np.meshgrid(t, t, indexing="ij")
    WU, WV = np.meshgrid(w, w, indexing="ij")
    xi = U.ravel()
    eta = ((1.0 - U) * V).ravel()
    wt = (WU * WV * (1.0 - U)).ravel()
    return xi, eta, wt


class ref_element:
    """Equispaced P_p Lagrange element on the reference triangle (0,0), (1,0), (0,1).

    ``nodes`` holds the integer lattice offsets (i, j) of the local nodes; the node
    sits at (i/p, j/p).
    """

    def __init__(self, p):
        assert p in (1, 2, 3)
        self.p = p
        self.nodes = np.array([(i, j) for j in range(p + 1) for i in range(p + 1 - j)])
        V = _eval_monomials(p, self.nodes[:, 0] / p, self.nodes[:, 1] / p)
        self.coef = np.linalg.inv(V)            # phi_k = sum_m coef[m, k] * mono_m

    def phi(self, x, y):
        return _eval_monomials(self.p, x, y) @ self.coef

    def grad(self, x, y):
        gx, gy = _eval_monomial_grads(self.p, x, y)
        return gx @ self.coef, gy @ self.coef


def element_matrices(p, h):
    """Stiffness and mass matrices of the two triangle types of one mesh cell.

    Returns dict with K_L, K_U, M_L, M_U (nloc x nloc) and the local lattice offsets
    of each local node for both types.
    """
    el = ref_element(p)
    xi, eta, wt = triangle_rule(6)
    Phi = el.phi(xi, eta)                   # (nq, nloc)
    Gx, Gy = el.grad(xi, eta)               # (nq, nloc)
    out = {}
    # T_L: v0 = (0,0), v1 = (h,0), v2 = (h,h)  ->  J = [[h, h], [0, h]]
    # T_U: v0 = (0,0), v1 = (h,h), v2 = (0,h)  ->  J = [[h, 0], [h, h]]
    for name, J in (("L", np.array([[h, h], [0.0, h]])), ("U", np.array([[h, 0.0], [h, h]]))):
        detJ = abs(np.linalg.det(J))
        G = np.linalg.inv(J).T              # physical grad = G @ reference grad
        px = G[0, 0] * Gx + G[0, 1] * Gy
        py = G[1, 0] * Gx + G[1, 1] * Gy
        out["K_" + name] = detJ * (px.T @ (wt[:, None] * px) + py.T @ (wt[:, None] * py))
        out["M_" + name] = detJ * (Phi.T @ (wt[:, None] * Phi))
    i, j = el.nodes[:, 0], el.nodes[:, 1]
    out["off_L"] = np.stack([i + j, j], axis=1)     # lattice offset (da, db) within the cell
    out["off_U"] = np.stack([i, i + j], axis=1)
    return out


def edge_mass(p, h):
    """1D mass matrix of the p+1 equispaced Lagrange functions on an edge of length h."""
    t = np.linspace(0.0, 1.0, p + 1)
    s, w = np.polynomial.legendre.leggauss(8)
    s = 0.5 * (s + 1.0)
    w = 0.5 * w
    L = _lagrange_1d(t, s)                  # (nq, p+1)
    return h * (L.T @ (w[:, None] * L))


def _lagrange_1d(t, s):
    s = np.asarray(s, float)
    out = np.ones((s.size, t.size))
    for a in range(t.size):
        for b in range(t.size):
            if a != b:
                out[:, a] *= (s - t[b]) / (t[a] - t[b])
    return out


# --------------------------------------------------------------------------------------
# Mesh-level assembly
# --------------------------------------------------------------------------------------

class Discretisation:
    """P_p space on the n x n "/"-split mesh of the unit square (h = 1/n)."""

    def __init__(self, n, p):
        assert n >= 1 and p in (1, 2, 3)
        self.n, self.p = n, p
        self.h = 1.0 / n
        self.M = p * n + 1
        self.N = self.M * self.M
        self._em = element_matrices(p, self.h)
        self._K = self._M = self._B = None

    # -- element connectivity ---------------------------------------------------------
    def element_dofs(self, kind):
        """(n*n, nloc) global dof numbers of every triangle of type ``kind`` ('L'/'U')."""
        n, p, M = self.n, self.p, self.M
        ci, cj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        ci, cj = ci.ravel(), cj.ravel()
        off = self._em["off_" + kind]
        a = p * ci[:, None] + off[None, :, 0]
        b = p * cj[:, None] + off[None, :, 1]
        return b * M + a

    def _assemble_volume(self, key):
        rows, cols, vals = [], [], []
        for kind in ("L", "U"):
            dofs = self.element_dofs(kind)
            Ae = self._em[key + "_" + kind]
            nloc = Ae.shape[0]
            rows.append(np.repeat(dofs, nloc, axis=1).ravel())
            cols.append(np.tile(dofs, (1, nloc)).ravel())
            vals.append(np.broadcast_to(Ae.ravel(), (dofs.shape[0], nloc * nloc)).ravel())
        A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(self.N, self.N))
        return A.tocsr()

    def boundary_edges(self):
        """(4n, p+1) global dofs along every boundary edge, with side labels 0..3
        (0: y=0, 1: x=1, 2: y=1, 3: x=0), nodes ordered by increasing coordinate."""
        n, p, M = self.n, self.p, self.M
        t = np.arange(p + 1)
        i = np.arange(n)
        along = p * i[:, None] + t[None, :]
        bottom = along                      # b = 0
        top = (M - 1) * M + along           # b = M-1
        left = along * M                    # a = 0
        right = along * M + (M - 1)         # a = M-1
        dofs = np.concatenate([bottom, right, top, left])
        side = np.repeat(np.arange(4), n)
        return dofs, side

    def _assemble_boundary(self):
        E = edge_mass(self.p, self.h)
        dofs, _ = self.boundary_edges()
        q = self.p + 1
        rows = np.repeat(dofs, q, axis=1).ravel()
        cols = np.tile(dofs, (1, q)).ravel()
        vals = np.broadcast_to(E.ravel(), (dofs.shape[0], q * q)).ravel()
        return sp.coo_matrix((vals, (rows, cols)), shape=(self.N, self.N)).tocsr()

    @property
    def K(self):
        if self._K is None:
            self._K = self._assemble_volume("K")
        return self._K

    @property
    def Mass(self):
        if self._M is None:
            self._M = self._assemble_volume("M")
        return self._M

    @property
    def B1(self):
        """Boundary mass with unit weight: B(k) = k * B1 for constant k."""
        if self._B is None:
            self._B = self._assemble_boundary()
        return self._B

    def operator(self, k, s=1.0):
        """A_s = K - s k^2 M - i k B1 (s = 1 + i beta; s = 1 gives A_0), CSR complex."""
        A = self.K.astype(complex) - (s * k * k) * self.Mass - (1j * k) * self.B1
        return A.tocsr()

    # -- coordinates, interpolation -------------------------------------------------
    def coords(self):
        a = np.arange(self.M)
        X, Y = np.meshgrid(a * self.h / self.p, a * self.h / self.p, indexing="xy")
        return X.ravel(), Y.ravel()         # index b*M + a -> (x_a, y_b)

    def interpolate(self, fun):
        x, y = self.coords()
        return fun(x, y)

    # -- right-hand side: plane-wave impedance data ---------------------------------
    def planewave_rhs(self, k, theta, q=10):
        """F_i = int_{dOmega} g phi_i ds for g = du/dn - i k u of u = exp(ik(x cos + y sin)).

        Per side: outward normal n, g = i k (n . d - 1) u with d = (cos, sin); each
        boundary edge is integrated with a q-point Gauss-Legendre rule (f = 0).
        """
        c, s_ = np.cos(theta), np.sin(theta)
        normals = {0: (0.0, -1.0), 1: (1.0, 0.0), 2: (0.0, 1.0), 3: (-1.0, 0.0)}
        dofs, side = self.boundary_edges()
        n, h, p = self.n, self.h, self.p
        tq, wq = np.polynomial.legendre.leggauss(q)
        tq = 0.5 * (tq + 1.0)
        wq = 0.5 * wq
        L = _lagrange_1d(np.linspace(0.0, 1.0, p + 1), tq)      # (q, p+1)
        F = np.zeros(self.N, complex)
        i = np.arange(n)
        for sd in range(4):
            idx = side == sd
            along = (i[:, None] + tq[None, :]) * h               # (n, q)
            if sd == 0:
                x, y = along, np.zeros_like(along)
            elif sd == 1:
                x, y = np.ones_like(along), along
            elif sd == 2:
                x, y = along, np.ones_like(along)
            else:
                x, y = np.zeros_like(along), along
            nx, ny = normals[sd]
            u = np.exp(1j * k * (x * c + y * s_))
            g = 1j * k * (nx * c + ny * s_ - 1.0) * u             # (n, q)
            contrib = h * (g * wq[None, :]) @ L                   # (n, p+1)
            np.add.at(F, dofs[idx].ravel(), contrib.ravel())
        return F


def planewave(k, theta):
    c, s = np.cos(theta), np.sin(theta)
    return lambda x, y: np.exp(1j * k * (x * c + y * s))


# --------------------------------------------------------------------------------------
# Prolongation between the 2h and h meshes
# --------------------------------------------------------------------------------------

def prolongation(fine, coarse):
    """P_{iJ} = phi^{2h}_J(x_i): the coarse basis evaluated at the fine nodes.

    The canonical FE interpolation V_{2h} -> V_h (Sec. 4: nested spaces by uniform
    refinement). Each fine node is located in a coarse triangle; the coarse basis of
    that triangle is evaluated there (continuity makes the choice of triangle on a
    shared edge irrelevant).
    """
    assert fine.p == coarse.p and fine.n == 2 * coarse.n
    p, nc = coarse.p, coarse.n
    el = ref_element(p)
    x, y = fine.coords()
    H = coarse.h
    I = np.minimum(np.floor(x / H + 1e-12).astype(int), nc - 1)
    J = np.minimum(np.floor(y / H + 1e-12).astype(int), nc - 1)
    lx = x / H - I                          # local cell coordinates in [0, 1]
    ly = y / H - J
    lower = ly <= lx + 1e-12
    # T_L: (lx, ly) = xi (1,0) + eta (1,1) -> eta = ly, xi = lx - ly
    # T_U: (lx, ly) = xi (1,1) + eta (0,1) -> xi = lx, eta = ly - lx
    xi = np.where(lower, lx - ly, lx)
    eta = np.where(lower, ly, ly - lx)
    vals = el.phi(xi, eta)                  # (Nf, nloc)
    i, j = el.nodes[:, 0], el.nodes[:, 1]
    offa = np.where(lower[:, None], (i + j)[None, :], i[None, :])
    offb = np.where(lower[:, None], j[None, :], (i + j)[None, :])
    A = p * I[:, None] + offa
    B = p * J[:, None] + offb
    cols = (B * coarse.M + A).ravel()
    rows = np.repeat(np.arange(fine.N), vals.shape[1])
    vals = vals.ravel()
    keep = np.abs(vals) > 1e-13
    return sp.csr_matrix((vals[keep], (rows[keep], cols[keep])), shape=(fine.N, coarse.N))
