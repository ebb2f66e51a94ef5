"""Pins of the oracle's discretisation against closed forms, invariants and brute force.

Each test fixes a fact of the mathematics that a plausible mistake in ``oracle/fem.py``
(a wrong sign, a dropped term, a transposed index, a wrong quadrature) would break.
"""

import math
import os

import numpy as np
import pytest

from oracle.fem import Discretisation, element_matrices, ref_element, prolongation, edge_mass

HERE = os.path.dirname(os.path.abspath(__file__))


# ---------------------------------------------------------------------------------------
# P1: textbook closed forms
# ---------------------------------------------------------------------------------------

def _row(A, M, a, b, r=2):
    """Stencil of row (a, b) as a (2r+1)^2 array indexed [db + r, da + r]."""
    row = A[b * M + a]
    out = np.zeros((2 * r + 1, 2 * r + 1), dtype=row.dtype)
    for db in range(-r, r + 1):
        for da in range(-r, r + 1):
            aa, bb = a + da, b + db
            if 0 <= aa < M and 0 <= bb < M:
                out[db + r, da + r] = row[bb * M + aa]
    return out


def test_p1_interior_stencils_closed_form():
    n = 6
    d = Discretisation(n, 1)
    h = d.h
    K = _row(d.K.toarray(), d.M, 3, 3, 1)
    Mm = _row(d.Mass.toarray(), d.M, 3, 3, 1)
    # five-point Laplacian; the diagonal edge of a right triangle carries no stiffness
    np.testing.assert_allclose(K, [[0, -1, 0], [-1, 4, -1], [0, -1, 0]], atol=1e-14)
    # mass: h^2/12 * (6 at the centre, 1 at N, S, E, W, NE, SW)
    ref = h * h / 12 * np.array([[1, 1, 0], [1, 6, 1], [0, 1, 1]])
    np.testing.assert_allclose(Mm, ref, atol=1e-16)


def test_p1_boundary_stencils_closed_form():
    n = 6
    d = Discretisation(n, 1)
    h = d.h
    K = _row(d.K.toarray(), d.M, 3, 0, 1)      # bottom edge node
    np.testing.assert_allclose(K[1:], [[-0.5, 2, -0.5], [0, -1, 0]], atol=1e-14)
    B = d.B1.toarray()
    # P1 edge mass h/6 [2 1; 1 2]: boundary diagonal 2h/3, neighbours h/6 (corners too)
    for a, b in [(3, 0), (0, 0), (6, 6), (0, 4), (6, 2)]:
        i = b * d.M + a
        assert B[i, i] == pytest.approx(2 * h / 3, rel=1e-13)
    i = 3
    assert B[i, i + 1] == pytest.approx(h / 6, rel=1e-13)
    assert B[i, i - 1] == pytest.approx(h / 6, rel=1e-13)
    assert abs(B[3 * d.M + 3]).max() == 0.0     # interior rows carry no boundary term


def test_p1_system_matrix_combination():
    """A_s = K - s k^2 M - i k B: interior centre 4 - s k^2 h^2/2, N -1 - s k^2 h^2/12."""
    n, k, s = 8, 7.0, 1 + 0.3j
    d = Discretisation(n, 1)
    h = d.h
    A = d.operator(k, s).toarray()
    c = 4 * d.M + 4
    assert A[c, c] == pytest.approx(4 - s * k * k * h * h / 2, rel=1e-13)
    assert A[c, c + d.M] == pytest.approx(-1 - s * k * k * h * h / 12, rel=1e-13)
    assert A[c, c + d.M + 1] == pytest.approx(-s * k * k * h * h / 12, rel=1e-13)
    assert A[c, c + d.M - 1] == 0
    b = 4                                            # bottom node: - i k (2h/3) on the diagonal
    Ab = A[b, b]
    assert Ab == pytest.approx(2 - s * k * k * h * h / 4 - 1j * k * 2 * h / 3, rel=1e-13)


# ---------------------------------------------------------------------------------------
# P2 / P3: invariants that hold exactly for polynomial integrands
# ---------------------------------------------------------------------------------------

def _monos(p):
    return [(a, b) for a in range(p + 1) for b in range(p + 1 - a)]


def _sq(a, b):
    """int_{(0,1)^2} x^a y^b."""
    if a < 0 or b < 0:
        return 0.0
    return 1.0 / ((a + 1) * (b + 1))


def _bd(a, b):
    """oint_{boundary of (0,1)^2} x^a y^b ds."""
    bottom = (1.0 / (a + 1)) if b == 0 else 0.0
    top = 1.0 / (a + 1)
    left = (1.0 / (b + 1)) if a == 0 else 0.0
    right = 1.0 / (b + 1)
    return bottom + top + left + right


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("n", [1, 3, 4])
def test_polynomial_reproduction(p, n):
    d = Discretisation(n, p)
    x, y = d.coords()
    K, Mm, B = d.K, d.Mass, d.B1
    for (a1, b1) in _monos(p):
        q = x ** a1 * y ** b1
        for (a2, b2) in _monos(p):
            r = x ** a2 * y ** b2
            assert q @ (Mm @ r) == pytest.approx(_sq(a1 + a2, b1 + b2), rel=1e-12, abs=1e-14)
            gk = a1 * a2 * _sq(a1 + a2 - 2, b1 + b2) + b1 * b2 * _sq(a1 + a2, b1 + b2 - 2)
            assert q @ (K @ r) == pytest.approx(gk, rel=1e-12, abs=1e-12)
            assert q @ (B @ r) == pytest.approx(_bd(a1 + a2, b1 + b2), rel=1e-12, abs=1e-14)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_row_sums_and_symmetry(p):
    d = Discretisation(5, p)
    one = np.ones(d.N)
    np.testing.assert_allclose(d.K @ one, 0.0, atol=1e-12)
    assert one @ (d.Mass @ one) == pytest.approx(1.0, rel=1e-13)
    assert one @ (d.B1 @ one) == pytest.approx(4.0, rel=1e-13)
    A = d.operator(11.0, 1 + 0.7j)
    assert abs(A - A.T).max() < 1e-13                # complex symmetric, not Hermitian
    assert abs(A - A.conj().T).max() > 1e-3


@pytest.mark.parametrize("p", [1, 2, 3])
def test_nodal_basis(p):
    el = ref_element(p)
    V = el.phi(el.nodes[:, 0] / p, el.nodes[:, 1] / p)
    np.testing.assert_allclose(V, np.eye(len(el.nodes)), atol=1e-12)


def _exact_tri_monomial(a, b):
    """int over the reference triangle of xi^a eta^b = a! b! / (a+b+2)!."""
    return math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_bruteforce_assembly(p):
    """Element-by-element loop with exact monomial integration == vectorised assembly."""
    n = 3
    h = 1.0 / n
    d = Discretisation(n, p)
    el = ref_element(p)
    monos = _monos(p)
    C = el.coef                                      # phi_k = sum_m C[m,k] mono_m
    nl = len(el.nodes)
    # reference mass and gradient products by exact integration
    Mref = np.zeros((nl, nl))
    Gxx = np.zeros((nl, nl)); Gxy = np.zeros((nl, nl)); Gyy = np.zeros((nl, nl))
    for m1, (a1, b1) in enumerate(monos):
        for m2, (a2, b2) in enumerate(monos):
            w = _exact_tri_monomial(a1 + a2, b1 + b2)
            Mref += w * np.outer(C[m1], C[m2])
            if a1 and a2:
                Gxx += a1 * a2 * _exact_tri_monomial(a1 + a2 - 2, b1 + b2) * np.outer(C[m1], C[m2])
            if b1 and b2:
                Gyy += b1 * b2 * _exact_tri_monomial(a1 + a2, b1 + b2 - 2) * np.outer(C[m1], C[m2])
            if a1 and b2:
                Gxy += a1 * b2 * _exact_tri_monomial(a1 + a2 - 1, b1 + b2 - 1) * np.outer(C[m1], C[m2])
    K = np.zeros((d.N, d.N)); M = np.zeros((d.N, d.N))
    for ci in range(n):
        for cj in range(n):
            for kind in ("L", "U"):
                if kind == "L":
                    J = np.array([[h, h], [0, h]])
                    loc = [(p * ci + i + j, p * cj + j) for i, j in el.nodes]
                else:
                    J = np.array([[h, 0], [h, h]])
                    loc = [(p * ci + i, p * cj + i + j) for i, j in el.nodes]
                G = np.linalg.inv(J).T
                det = abs(np.linalg.det(J))
                S = G.T @ G                           # metric for reference gradients
                Ke = det * (S[0, 0] * Gxx + S[0, 1] * Gxy + S[1, 0] * Gxy.T + S[1, 1] * Gyy)
                Me = det * Mref
                idx = [b * d.M + a for a, b in loc]
                for r_, I in enumerate(idx):
                    for c_, Jd in enumerate(idx):
                        K[I, Jd] += Ke[r_, c_]
                        M[I, Jd] += Me[r_, c_]
    np.testing.assert_allclose(d.K.toarray(), K, atol=1e-12)
    np.testing.assert_allclose(d.Mass.toarray(), M, atol=1e-15)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_edge_mass_exact(p):
    h = 0.25
    E = edge_mass(p, h)
    assert E.sum() == pytest.approx(h, rel=1e-14)
    t = np.linspace(0, 1, p + 1)
    for a in range(p + 1):
        for b in range(p + 1):
            if a + b <= 2 * p:
                assert (t ** a) @ E @ (t ** b) == pytest.approx(h / (a + b + 1), rel=1e-13)


# ---------------------------------------------------------------------------------------
# Transfers and the coarse operator
# ---------------------------------------------------------------------------------------

@pytest.mark.parametrize("p", [1, 2, 3])
def test_prolongation_reproduces_coarse_polynomials(p):
    f, c = Discretisation(8, p), Discretisation(4, p)
    P = prolongation(f, c)
    np.testing.assert_allclose(P @ np.ones(c.N), 1.0, atol=1e-13)
    xf, yf = f.coords()
    xc, yc = c.coords()
    for (a, b) in _monos(p):
        np.testing.assert_allclose(P @ (xc ** a * yc ** b), xf ** a * yf ** b, atol=1e-13)
    # a coarse function that is only piecewise polynomial: nodal values at coincident nodes
    rng = np.random.default_rng(5)
    xcv = rng.standard_normal(c.N)
    coincide = [(2 * A, 2 * B) for B in range(c.M) for A in range(c.M)]
    fine_vals = (P @ xcv).reshape(f.M, f.M)
    for J, (a2, b2) in enumerate(coincide):
        assert fine_vals[b2, a2] == pytest.approx(xcv[J], abs=1e-13)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_restriction_is_transpose(p):
    f, c = Discretisation(6, p), Discretisation(3, p)
    P = prolongation(f, c)
    rng = np.random.default_rng(1)
    xc = rng.standard_normal(c.N) + 1j * rng.standard_normal(c.N)
    y = rng.standard_normal(f.N) + 1j * rng.standard_normal(f.N)
    lhs = np.vdot(y, P @ xc)
    rhs = np.vdot(P.T @ y, xc)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_galerkin_equals_rediscretised(p):
    """Nested spaces, constant k, nested boundary edges: P^T A_h P == A_2h exactly."""
    k, s = 9.0, 1 + 0.5j
    f, c = Discretisation(8, p), Discretisation(4, p)
    P = prolongation(f, c)
    G = (P.T @ f.operator(k, s) @ P).toarray()
    A2 = c.operator(k, s).toarray()
    assert abs(G - A2).max() <= 1e-13 * abs(A2).max()


# ---------------------------------------------------------------------------------------
# Right-hand side: moments against closed-form boundary integrals
# ---------------------------------------------------------------------------------------

def _I0(al):
    """int_0^1 exp(i al t) dt."""
    return 1.0 if al == 0 else (np.exp(1j * al) - 1) / (1j * al)


def _I1(al):
    """int_0^1 t exp(i al t) dt."""
    if al == 0:
        return 0.5
    return np.exp(1j * al) / (1j * al) + (np.exp(1j * al) - 1) / al ** 2


def _boundary_moments(k, th):
    """(oint g, oint g x, oint g y) for the plane-wave impedance data."""
    c, s = np.cos(th), np.sin(th)
    gb = 1j * k * (-s - 1)          # y = 0, normal (0,-1): u = e^{ikcx}
    gr = 1j * k * (c - 1)           # x = 1, normal (1, 0): u = e^{ikc} e^{iksy}
    gt = 1j * k * (s - 1)           # y = 1: u = e^{iks} e^{ikcx}
    gl = 1j * k * (-c - 1)          # x = 0: u = e^{iksy}
    ec, es = np.exp(1j * k * c), np.exp(1j * k * s)
    m0 = gb * _I0(k * c) + gr * ec * _I0(k * s) + gt * es * _I0(k * c) + gl * _I0(k * s)
    mx = gb * _I1(k * c) + gr * ec * _I0(k * s) + gt * es * _I1(k * c) + 0.0
    my = 0.0 + gr * ec * _I1(k * s) + gt * es * _I0(k * c) + gl * _I1(k * s)
    return m0, mx, my


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("theta", [np.pi / 7, 2.1, 4.0])
def test_planewave_rhs_moments(p, theta):
    k = 13.0
    d = Discretisation(16, p)
    F = d.planewave_rhs(k, theta)
    x, y = d.coords()
    m0, mx, my = _boundary_moments(k, theta)
    assert F.sum() == pytest.approx(m0, rel=1e-12)
    assert F @ x == pytest.approx(mx, rel=1e-12)
    assert F @ y == pytest.approx(my, rel=1e-12)
    interior = (x > 0) & (x < 1) & (y > 0) & (y < 1)
    assert np.all(F[interior] == 0)


def test_dof_counts_golden():
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "dof_counts.txt"))
            if l.strip() and not l.startswith("#")]
    for p, l, real in rows:
        n = 2 ** int(l)
        assert 2 * (int(p) * n + 1) ** 2 == int(real)
        if int(p) == 1:
            assert 2 * Discretisation(n, 1).N == int(real)
