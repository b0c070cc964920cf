"""Pins of the oracle's tetrahedral element (Table 1's complete-basis 3D
element): collapsed Gauss rule, Lagrange basis on the tetrahedral lattice,
affine geometry and the element loop on it, checked against closed forms
(monomial integrals a! b! c! / (a+b+c+3)!, the textbook P1 matrices of the
reference tetrahedron), exact symbolic integrals (the bilinear form on an
affine tetrahedron) and invariants."""
import math

import numpy as np
import pytest

import oracle

REF = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=float)


def coeffs(seed):
    rng = np.random.default_rng(seed)
    L = rng.normal(0, 0.3, (3, 3))
    return L @ L.T + np.eye(3), rng.normal(0, 1, 3), rng.uniform(0, 1), rng.uniform(-1, 1)


def tet1(p, X, D, beta, c, f, n1=0):
    A, b, fl = oracle.integrate_tet(p, X[None], D[None], np.asarray(beta, float)[None], np.array([c], float),
                                    np.array([f], float), n1=n1)
    return A[0], b[0], int(fl[0])


def tet_monomial(a, b, c):
    return math.factorial(a) * math.factorial(b) * math.factorial(c) / math.factorial(a + b + c + 3)


def some_tet(seed):
    rng = np.random.default_rng(seed)
    X = REF @ np.array([[1.1, 0.2, -0.1], [0.1, 0.9, 0.2], [-0.2, 0.1, 1.2]]).T + rng.uniform(-0.1, 0.1, (4, 3))
    return X + np.array([0.3, -0.2, 0.5])


@pytest.mark.parametrize("p", range(1, 8))
def test_tet_rule_exact_to_degree_2p(p):
    pts, w = oracle.tet_rule(p + 2)
    assert (w > 0).all() and abs(w.sum() - 1 / 6) < 1e-15
    worst = 0.0
    for a in range(2 * p + 1):
        for b in range(2 * p + 1 - a):
            for c in range(2 * p + 1 - a - b):
                ex = tet_monomial(a, b, c)
                worst = max(worst, abs(np.sum(w * pts[:, 0] ** a * pts[:, 1] ** b * pts[:, 2] ** c) - ex) / ex)
    assert worst < 1e-13
    # discriminating: with p+1 points per direction the rule is not exact at degree 2p in zeta
    pts1, w1 = oracle.tet_rule(p + 1)
    assert abs(np.sum(w1 * pts1[:, 2] ** (2 * p)) - tet_monomial(0, 0, 2 * p)) > 1e-10 * tet_monomial(0, 0, 2 * p)


@pytest.mark.parametrize("p", range(1, 8))
def test_tet_basis_kronecker_and_partition(p):
    nodes = oracle.tet_nodes(p)
    n = oracle.tet_nshp(p)
    assert n == (p + 1) * (p + 2) * (p + 3) // 6          # Table 1, tetrahedral row
    V = np.array([oracle.tet_basis(p, x)[0] for x in nodes])
    assert np.abs(V - np.eye(n)).max() < 1e-12
    rng = np.random.default_rng(p)
    for xi in rng.dirichlet([1, 1, 1, 1], 5)[:, 1:]:
        phi, dphi = oracle.tet_basis(p, xi)
        assert abs(phi.sum() - 1) < 1e-12 and np.abs(dphi.sum(axis=0)).max() < 1e-9


@pytest.mark.parametrize("p", [1, 2, 4, 6])
def test_tet_basis_reproduces_pp(p):
    rng = np.random.default_rng(20 + p)
    terms = [(a, b, c, rng.normal()) for a in range(p + 1) for b in range(p + 1 - a) for c in range(p + 1 - a - b)]

    def g(x):
        v = sum(k * x[0] ** a * x[1] ** b * x[2] ** c for a, b, c, k in terms)
        gr = np.array([sum(k * a * x[0] ** max(a - 1, 0) * x[1] ** b * x[2] ** c for a, b, c, k in terms),
                       sum(k * b * x[0] ** a * x[1] ** max(b - 1, 0) * x[2] ** c for a, b, c, k in terms),
                       sum(k * c * x[0] ** a * x[1] ** b * x[2] ** max(c - 1, 0) for a, b, c, k in terms)])
        return v, gr

    u = np.array([g(x)[0] for x in oracle.tet_nodes(p)])
    for xi in rng.dirichlet([1, 1, 1, 1], 4)[:, 1:]:
        phi, dphi = oracle.tet_basis(p, xi)
        v, gr = g(xi)
        assert abs(phi @ u - v) < 1e-9 * max(1, abs(v))
        assert np.abs(dphi.T @ u - gr).max() < 1e-8 * max(1, np.abs(gr).max())


def test_tet_p1_basis_is_barycentric():
    xi = np.array([0.2, 0.3, 0.1])
    phi, dphi = oracle.tet_basis(1, xi)
    assert np.abs(phi - [0.4, 0.2, 0.3, 0.1]).max() < 1e-15
    assert np.abs(dphi - np.array([[-1, -1, -1], [1, 0, 0], [0, 1, 0], [0, 0, 1]])).max() < 1e-15


def test_tet_geometry_affine():
    X = some_tet(1)
    J, det, K, x = oracle.tet_geometry(X, [0.2, 0.3, 0.1])
    M = (X[1:] - X[0]).T
    assert np.abs(J - M).max() < 1e-15 and abs(det - np.linalg.det(M)) < 1e-14
    assert np.abs(K - np.linalg.inv(M)).max() < 1e-13 and np.abs(x - (X[0] + M @ [0.2, 0.3, 0.1])).max() < 1e-15


def test_tet_p1_reference_textbook():
    """Reference tetrahedron, p = 1: stiffness (1/6) grad l_a . D grad l_b,
    mass (1/120)(1 + delta_ab), convection (1/24) beta . grad l_b."""
    G = np.array([[-1, -1, -1], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=float)
    D, be, c, f = np.diag([1.0, 2.0, 0.5]), np.array([0.3, -0.7, 1.2]), 0.8, 1.5
    A, b, fl = tet1(1, REF, D, be, c, f)
    ref = G @ D @ G.T / 6 + np.tile(G @ be, (4, 1)) / 24 + c * (np.ones((4, 4)) + np.eye(4)) / 120
    assert fl == 0 and np.abs(A - ref).max() < 1e-15
    assert np.abs(b - f / 24).max() < 1e-16


@pytest.mark.parametrize("p", [1, 3, 5])
def test_tet_mass_sum_volume_and_invariants(p):
    X = some_tet(10 + p)
    vol = abs(np.linalg.det(X[1:] - X[0])) / 6
    A, b, fl = tet1(p, X, np.zeros((3, 3)), np.zeros(3), 1.0, 0.7)
    assert fl == 0 and abs(A.sum() - vol) < 1e-13 * vol and abs(b.sum() - 0.7 * vol) < 1e-13 * vol
    D, be, _, _ = coeffs(10 + p)
    Ad, _, _ = tet1(p, X, D, np.zeros(3), 0.0, 0.0)
    assert np.abs(Ad.sum(axis=1)).max() < 1e-11 * np.abs(Ad).max()
    assert np.abs(Ad - Ad.T).max() < 1e-12 * np.abs(Ad).max()
    Ac, _, _ = tet1(p, X, np.zeros((3, 3)), be, 0.0, 0.0)
    assert np.abs(Ac.sum(axis=1)).max() < 1e-11 * np.abs(Ac).max()


@pytest.mark.parametrize("p", [1, 2, 3])
def test_tet_exact_bilinear_form(p):
    """v^T A u equals the exact integral over an affine tetrahedron for
    physical polynomials u, v of degree p."""
    import sympy as sp
    x, y, z = sp.symbols("x y z")
    a, b, c = sp.symbols("a b c")
    X = sp.Matrix([[0, 0, 0], [sp.Rational(5, 4), sp.Rational(1, 8), 0], [sp.Rational(-1, 8), 1, sp.Rational(1, 4)],
                   [sp.Rational(1, 4), sp.Rational(1, 8), sp.Rational(9, 8)]]) + sp.ones(4, 1) * sp.Matrix([[sp.Rational(1, 3), 0, sp.Rational(-1, 2)]])
    M = (X[1:, :] - sp.ones(3, 1) * X[0, :]).T
    Dm = sp.Matrix([[2, sp.Rational(1, 3), 0], [sp.Rational(1, 4), 1, sp.Rational(-1, 5)], [0, sp.Rational(1, 6), sp.Rational(3, 2)]])
    bv = sp.Matrix([sp.Rational(1, 2), -1, sp.Rational(3, 4)])
    cc = sp.Rational(2, 3)
    rng = np.random.default_rng(60 + p)

    def rand_poly():
        e = 1
        for _ in range(5):
            i = int(rng.integers(0, p + 1)); j = int(rng.integers(0, p + 1 - i)); k = int(rng.integers(0, p + 1 - i - j))
            e += int(rng.integers(-4, 5)) * x ** i * y ** j * z ** k
        return e

    u, v = rand_poly(), rand_poly()
    gu = [sp.diff(u, s) for s in (x, y, z)]
    gv = [sp.diff(v, s) for s in (x, y, z)]
    integrand = sum(gv[i] * Dm[i, j] * gu[j] for i in range(3) for j in range(3)) \
        + v * sum(bv[i] * gu[i] for i in range(3)) + cc * u * v
    xm = M * sp.Matrix([a, b, c]) + X[0, :].T
    integrand = sp.expand(integrand.subs({x: xm[0], y: xm[1], z: xm[2]}, simultaneous=True))
    exact = sp.integrate(integrand, (a, 0, 1 - b - c), (b, 0, 1 - c), (c, 0, 1)) * M.det()
    Xf = np.array(X.tolist(), dtype=float)
    Mf = np.array(M.tolist(), dtype=float)
    nodes = oracle.tet_nodes(p) @ Mf.T + Xf[0]
    un = np.array([float(u.subs({x: n[0], y: n[1], z: n[2]})) for n in nodes])
    vn = np.array([float(v.subs({x: n[0], y: n[1], z: n[2]})) for n in nodes])
    A, _, _ = tet1(p, Xf, np.array(Dm.tolist(), dtype=float), np.array(bv.tolist(), dtype=float).ravel(), float(cc), 0.0)
    assert abs(vn @ A @ un - float(exact)) < 1e-12 * max(1.0, abs(float(exact)))


def test_tet_inverted_flagged():
    D, be, c, f = coeffs(3)
    _, _, fl = tet1(2, REF[[0, 2, 1, 3]], D, be, c, f)
    assert fl == 1
