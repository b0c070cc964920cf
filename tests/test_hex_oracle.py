"""Pins of the oracle's hexahedral element (Table 1's tensor-product element):
tensor Gauss rule, tensor-product Gauss-Lobatto Lagrange basis, trilinear
geometry and the element loop on it, checked against closed forms (monomial
integrals, the textbook Q1 unit-cube matrices built from the 1D linear-element
matrices), exact symbolic integrals (volume of a distorted hexahedron, the
bilinear form on a parallelepiped), invariants and over-integration."""
from fractions import Fraction

import numpy as np
import pytest

import oracle

CUBE = np.array([[(v & 1), (v >> 1) & 1, (v >> 2) & 1] for v in range(8)], dtype=float)   # [0,1]^3, v = i+2j+4k


def coeffs(seed):
    rng = np.random.default_rng(seed)
    L = rng.normal(0, 0.3, (3, 3))
    return L @ L.T + np.eye(3), rng.normal(0, 1, 3), rng.uniform(0, 1), rng.uniform(-1, 1)


def distorted_hex(seed, amp=0.2):
    rng = np.random.default_rng(seed)
    M = np.array([[1.0, 0.15, -0.1], [0.05, 0.9, 0.1], [-0.1, 0.05, 1.1]])
    return CUBE @ M.T + amp * rng.uniform(-0.5, 0.5, (8, 3))


def hex1(p, X, D, beta, c, f, n1=0):
    A, b, fl = oracle.integrate_hex(p, X[None], D[None], np.asarray(beta, float)[None], np.array([c], float),
                                    np.array([f], float), n1=n1)
    return A[0], b[0], int(fl[0])


def line_moment(g):
    return Fraction(0) if g % 2 else Fraction(2, g + 1)


@pytest.mark.parametrize("p", range(1, 8))
def test_hex_rule_exact(p):
    pts, w = oracle.hex_rule(p + 1)
    worst = 0.0
    for a in (0, 1, 2 * p, 2 * p + 1):
        for b in (0, 2, 2 * p + 1):
            for g in (0, 1, 2 * p):
                exact = float(line_moment(a) * line_moment(b) * line_moment(g))
                worst = max(worst, abs(np.sum(w * pts[:, 0] ** a * pts[:, 1] ** b * pts[:, 2] ** g) - exact))
    assert worst < 1e-14
    # discriminating: degree 2p+2 in one variable is not exact
    assert abs(np.sum(w * pts[:, 0] ** (2 * p + 2)) - 8 * float(line_moment(2 * p + 2)) / 2) > 1e-8


@pytest.mark.parametrize("p", range(1, 8))
def test_hex_basis_kronecker_and_partition(p):
    nodes = oracle.hex_nodes(p)
    n = oracle.hex_nshp(p)
    V = np.array([oracle.hex_basis(p, x)[0] for x in nodes])
    assert np.abs(V - np.eye(n)).max() < 1e-12
    rng = np.random.default_rng(p)
    for xi in rng.uniform(-1, 1, (5, 3)):
        phi, dphi = oracle.hex_basis(p, xi)
        assert abs(phi.sum() - 1.0) < 1e-12 and np.abs(dphi.sum(axis=0)).max() < 1e-10


@pytest.mark.parametrize("p", [1, 2, 3, 5])
def test_hex_basis_reproduces_qp(p):
    """Interpolation at the nodes reproduces every polynomial of degree <= p in
    each variable, values and gradients."""
    rng = np.random.default_rng(10 + p)
    C = rng.normal(0, 1, (p + 1, p + 1, p + 1))

    def g(x):
        v = 0.0; gr = np.zeros(3)
        for i in range(p + 1):
            for j in range(p + 1):
                for k in range(p + 1):
                    m = x[0] ** i * x[1] ** j * x[2] ** k
                    v += C[i, j, k] * m
                    gr += C[i, j, k] * np.array([i * x[0] ** max(i - 1, 0) * x[1] ** j * x[2] ** k,
                                                  j * x[0] ** i * x[1] ** max(j - 1, 0) * x[2] ** k,
                                                  k * x[0] ** i * x[1] ** j * x[2] ** max(k - 1, 0)])
        return v, gr

    u = np.array([g(x)[0] for x in oracle.hex_nodes(p)])
    for xi in rng.uniform(-1, 1, (4, 3)):
        phi, dphi = oracle.hex_basis(p, xi)
        v, gr = g(xi)
        assert abs(phi @ u - v) < 1e-10 * max(1, abs(v))
        assert np.abs(dphi.T @ u - gr).max() < 1e-9 * max(1, np.abs(gr).max())


def test_hex_p1_basis_is_geometry_basis():
    rng = np.random.default_rng(3)
    for xi in rng.uniform(-1, 1, (4, 3)):
        phi, _ = oracle.hex_basis(1, xi)
        N = np.array([np.prod([(1 + s * x) / 2 for s, x in zip(2 * CUBE[v] - 1, xi)]) for v in range(8)])
        assert np.abs(phi - N).max() < 1e-15


def test_hex_geometry_reference_and_affine():
    ref = 2 * CUBE - 1
    J, det, K, x = oracle.hex_geometry(ref, [0.3, -0.2, 0.7])
    assert np.abs(J - np.eye(3)).max() < 1e-15 and abs(det - 1) < 1e-15 and np.abs(x - [0.3, -0.2, 0.7]).max() < 1e-15
    M = np.array([[1.2, 0.3, -0.1], [0.1, 0.8, 0.2], [0.0, -0.3, 1.5]])
    t = np.array([0.5, -1.0, 2.0])
    X = ref @ M.T + t
    xi = np.array([-0.4, 0.6, 0.1])
    J, det, K, x = oracle.hex_geometry(X, xi)
    assert np.abs(J - M).max() < 1e-14 and abs(det - np.linalg.det(M)) < 1e-13
    assert np.abs(K - np.linalg.inv(M)).max() < 1e-13 and np.abs(x - (M @ xi + t)).max() < 1e-14


def test_hex_q1_unit_cube_textbook():
    """Unit cube, p = 1: the element matrices are Kronecker products of the 1D
    linear-element matrices on [0, 1] (x the fastest index)."""
    K1 = np.array([[1.0, -1.0], [-1.0, 1.0]])
    M1 = np.array([[1 / 3, 1 / 6], [1 / 6, 1 / 3]])
    C1 = np.array([[-0.5, 0.5], [-0.5, 0.5]])            # int phi_a phi_b'
    kr = lambda z, y, x: np.kron(np.kron(z, y), x)
    D, be, c, f = np.diag([1.0, 2.0, 3.0]), np.array([0.7, -0.4, 1.1]), 0.6, 1.3
    A, b, fl = hex1(1, CUBE, D, be, c, f)
    ref = (1.0 * kr(M1, M1, K1) + 2.0 * kr(M1, K1, M1) + 3.0 * kr(K1, M1, M1)
           + be[0] * kr(M1, M1, C1) + be[1] * kr(M1, C1, M1) + be[2] * kr(C1, M1, M1) + c * kr(M1, M1, M1))
    assert fl == 0
    assert np.abs(A - ref).max() < 1e-14
    assert np.abs(b - f * kr(M1, M1, M1).sum(axis=1)).max() < 1e-15
    # the classical Laplacian entries: 1/3 on the diagonal, 0 along edges, -1/12 across faces and the body
    Al, _, _ = hex1(1, CUBE, np.eye(3), np.zeros(3), 0.0, 0.0)
    diff = np.array([[bin(a ^ b2).count("1") for b2 in range(8)] for a in range(8)])
    assert np.allclose(Al[diff == 0], 1 / 3) and np.allclose(Al[diff == 1], 0.0, atol=1e-15)
    assert np.allclose(Al[diff == 2], -1 / 12) and np.allclose(Al[diff == 3], -1 / 12)


def exact_hex_volume(X):
    import sympy as sp
    a, b, z = sp.symbols("a b z")
    Xr = [[sp.Rational(float(v)) for v in row] for row in X]
    N = [sp.Rational(1, 8) * (1 + (2 * (v & 1) - 1) * a) * (1 + (2 * ((v >> 1) & 1) - 1) * b)
         * (1 + (2 * ((v >> 2) & 1) - 1) * z) for v in range(8)]
    x = [sum(N[v] * Xr[v][d] for v in range(8)) for d in range(3)]
    J = sp.Matrix([[sp.diff(x[d], s) for s in (a, b, z)] for d in range(3)])
    return float(sp.integrate(sp.expand(J.det()), (a, -1, 1), (b, -1, 1), (z, -1, 1)))


@pytest.mark.parametrize("p", [1, 2, 4])
def test_hex_mass_sum_is_exact_volume(p):
    X = distorted_hex(20 + p, amp=0.3)
    vol = exact_hex_volume(X)
    A, b, fl = hex1(p, X, np.zeros((3, 3)), np.zeros(3), 1.0, 0.7)
    assert fl == 0
    assert abs(A.sum() - vol) < 1e-13 * vol and abs(b.sum() - 0.7 * vol) < 1e-13 * vol


@pytest.mark.parametrize("p", [1, 3, 5])
def test_hex_invariants(p):
    X = distorted_hex(30 + p, amp=0.3)
    D, be, c, f = coeffs(30 + p)
    Ad, _, _ = hex1(p, X, D, np.zeros(3), 0.0, 0.0)
    assert np.abs(Ad.sum(axis=1)).max() < 1e-12 * np.abs(Ad).max()        # constants in the null space
    assert np.abs(Ad - Ad.T).max() < 1e-12 * np.abs(Ad).max()
    Ac, _, _ = hex1(p, X, np.zeros((3, 3)), be, 0.0, 0.0)
    assert np.abs(Ac.sum(axis=1)).max() < 1e-12 * np.abs(Ac).max()        # beta . grad 1 = 0
    A, _, _ = hex1(p, X, D, be, c, f)
    assert np.abs(A - (Ad + Ac + c * hex1(p, X, np.zeros((3, 3)), np.zeros(3), 1.0, 0.0)[0])).max() \
        < 1e-12 * np.abs(A).max()                                           # linear in the coefficients


@pytest.mark.parametrize("p", [1, 2])
def test_hex_affine_exact_bilinear_form(p):
    """v^T A u equals the exact integral of D grad u . grad v + v beta . grad u
    + c u v over a parallelepiped for physical polynomials u, v of degree p."""
    import sympy as sp
    x, y, zz = sp.symbols("x y z")
    a, b, z = sp.symbols("a b zeta")
    M = sp.Matrix([[1, sp.Rational(1, 4), 0], [sp.Rational(-1, 8), sp.Rational(3, 4), sp.Rational(1, 8)],
                   [sp.Rational(1, 8), 0, sp.Rational(5, 4)]])
    t = sp.Matrix([sp.Rational(1, 3), sp.Rational(-1, 5), sp.Rational(2, 7)])
    Dm = sp.Matrix([[2, sp.Rational(1, 3), 0], [sp.Rational(1, 4), 1, sp.Rational(-1, 5)], [0, sp.Rational(1, 6), sp.Rational(3, 2)]])
    bv = sp.Matrix([sp.Rational(1, 2), -1, sp.Rational(3, 4)])
    cc = sp.Rational(2, 3)
    rng = np.random.default_rng(40 + p)

    def rand_poly():
        e = 1
        for _ in range(5):
            i = int(rng.integers(0, p + 1)); j = int(rng.integers(0, p + 1 - i)); k = int(rng.integers(0, p + 1 - i - j))
            e += int(rng.integers(-4, 5)) * x ** i * y ** j * zz ** k
        return e

    u, v = rand_poly(), rand_poly()
    gu = [sp.diff(u, s) for s in (x, y, zz)]
    gv = [sp.diff(v, s) for s in (x, y, zz)]
    integrand = sum(gv[i] * Dm[i, j] * gu[j] for i in range(3) for j in range(3)) \
        + v * sum(bv[i] * gu[i] for i in range(3)) + cc * u * v
    xm = M * sp.Matrix([a, b, z]) + t
    integrand = sp.expand(integrand.subs({x: xm[0], y: xm[1], zz: xm[2]}, simultaneous=True))
    exact = sp.integrate(integrand, (a, -1, 1), (b, -1, 1), (z, -1, 1)) * M.det()
    Mf = np.array(M.tolist(), dtype=float); tf = np.array(t.tolist(), dtype=float).ravel()
    X = (2 * CUBE - 1) @ Mf.T + tf
    nodes = oracle.hex_nodes(p) @ Mf.T + tf
    un = np.array([float(u.subs({x: n[0], y: n[1], zz: n[2]})) for n in nodes])
    vn = np.array([float(v.subs({x: n[0], y: n[1], zz: n[2]})) for n in nodes])
    A, _, _ = hex1(p, X, np.array(Dm.tolist(), dtype=float), np.array(bv.tolist(), dtype=float).ravel(), float(cc), 0.0)
    assert abs(vn @ A @ un - float(exact)) < 1e-12 * max(1.0, abs(float(exact)))


@pytest.mark.parametrize("p", [2, 4])
def test_hex_over_integration_converges(p):
    X = distorted_hex(50 + p, amp=0.3)
    D, be, c, f = coeffs(50 + p)
    Ar, _, _ = hex1(p, X, D, be, c, f, n1=p + 10)
    errs = [np.linalg.norm(hex1(p, X, D, be, c, f, n1=m)[0] - Ar) / np.linalg.norm(Ar) for m in (p + 1, p + 3, p + 5)]
    assert errs[0] < 1e-2 and errs[2] < errs[1] < errs[0]


def test_hex_inverted_flagged():
    X = CUBE[[4, 5, 6, 7, 0, 1, 2, 3]]             # top and bottom swapped: det J < 0
    D, be, c, f = coeffs(1)
    _, _, fl = hex1(2, X, D, be, c, f)
    assert fl == 1
