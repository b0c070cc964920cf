"""Pins of the FP64 CPU oracle against what the mathematics fixes.

Every function of the oracle is checked here against something other than
itself: library routines (numpy's Gauss-Legendre), closed forms (Gauss-Lobatto
nodes, monomial integrals, textbook P1 prism matrices), exact symbolic
integrals (sympy), invariants of the element matrices, and finite
differences for the adjoint.  A dropped term, a wrong sign or index, or a
transposed operand in the oracle fails at least one test below.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1310_1194_amd import meshgen

REF = np.array([[0, 0, -1], [1, 0, -1], [0, 1, -1], [0, 0, 1], [1, 0, 1], [0, 1, 1]], dtype=float)


def affine_prism(M, t):
    return REF @ np.asarray(M, float).T + np.asarray(t, float)


def distorted_prism(seed=0, amp=0.15):
    rng = np.random.default_rng(seed)
    M = np.array([[0.9, 0.2, 0.1], [-0.1, 1.1, 0.05], [0.15, -0.05, 0.45]])
    X = affine_prism(M, [0.3, -0.2, 0.1])
    return X + amp * rng.uniform(-1, 1, X.shape) * 0.5


def coeffs(seed=0):
    rng = np.random.default_rng(seed)
    L = rng.normal(0, 0.3, (3, 3))
    D = L @ L.T + np.eye(3)
    return D, rng.normal(0, 1, 3), rng.uniform(0, 1), rng.uniform(-1, 1)


def integrate1(p, X, D, beta, c, f, n1=0):
    A, b, fl = oracle.integrate(p, X[None], D[None], np.asarray(beta, float)[None],
                                np.array([c], float), np.array([f], float), n1=n1)
    return A[0], b[0], int(fl[0])


# --------------------------------------------------------------------------
# quadrature
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", range(1, 21))
def test_gauss_legendre_matches_numpy(n):
    x, w = oracle.gauss_legendre(n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    assert np.allclose(x, xr, rtol=0, atol=2e-15)
    assert np.allclose(w, wr, rtol=0, atol=2e-15)


def test_gauss_closed_forms():
    x, w = oracle.gauss_legendre(2)
    assert np.allclose(x, [-1 / math.sqrt(3), 1 / math.sqrt(3)], atol=1e-16)
    assert np.allclose(w, [1, 1], atol=1e-15)
    x, w = oracle.gauss_legendre(3)
    assert np.allclose(x, [-math.sqrt(0.6), 0, math.sqrt(0.6)], atol=1e-16)
    assert np.allclose(w, [5 / 9, 8 / 9, 5 / 9], atol=1e-15)


def test_gll_closed_forms():
    assert np.allclose(oracle.gll_nodes(1), [-1, 1], atol=0)
    assert np.allclose(oracle.gll_nodes(2), [-1, 0, 1], atol=1e-16)
    assert np.allclose(oracle.gll_nodes(3), [-1, -1 / math.sqrt(5), 1 / math.sqrt(5), 1], atol=1e-16)
    s = math.sqrt(3 / 7)
    assert np.allclose(oracle.gll_nodes(4), [-1, -s, 0, s, 1], atol=1e-16)


@pytest.mark.parametrize("p", range(1, 8))
def test_gll_interior_nodes_are_roots_of_dP(p):
    r = np.sort(np.polynomial.legendre.Legendre.basis(p).deriv().roots().real)
    x = oracle.gll_nodes(p)
    assert x[0] == -1 and x[-1] == 1
    assert np.allclose(x[1:-1], r, atol=1e-13)


def tri_monomial(a, b):
    """int over the unit triangle of xi1^a xi2^b = a! b! / (a+b+2)!."""
    return Fraction(math.factorial(a) * math.factorial(b), math.factorial(a + b + 2))


def line_monomial(g):
    return Fraction(0) if g % 2 else Fraction(2, g + 1)


@pytest.mark.parametrize("p", range(1, 8))
def test_rule_exact_on_monomials(p):
    pts, w = oracle.rule(p + 1)
    assert abs(w.sum() - 1.0) < 1e-14          # |reference prism| = 1/2 * 2
    worst = 0.0
    for a in range(2 * p + 1):
        for b in range(2 * p + 1 - a):
            for g in (0, 1, 2 * p, 2 * p + 1):
                exact = float(tri_monomial(a, b) * line_monomial(g))
                q = np.sum(w * pts[:, 0] ** a * pts[:, 1] ** b * pts[:, 2] ** g)
                worst = max(worst, abs(q - exact))
    assert worst < 1e-14


def test_rule_is_not_exact_beyond_its_degree():
    # the check above is discriminating: degree 2p+2 on the triangle fails
    p = 2
    pts, w = oracle.rule(p + 1)
    exact = float(tri_monomial(2 * p + 2, 0) * 2)
    assert abs(np.sum(w * pts[:, 0] ** (2 * p + 2)) - exact) > 1e-6


# --------------------------------------------------------------------------
# basis
# --------------------------------------------------------------------------

@pytest.mark.parametrize("p", range(1, 8))
def test_basis_kronecker(p):
    nodes = oracle.nodes(p)
    n = oracle.nshp(p)
    V = np.array([oracle.basis(p, x)[0] for x in nodes])
    assert np.abs(V - np.eye(n)).max() < 1e-12


@pytest.mark.parametrize("p", range(1, 8))
def test_basis_partition_of_unity(p):
    rng = np.random.default_rng(p)
    for _ in range(5):
        a, b = rng.uniform(0, 1, 2)
        if a + b > 1:
            a, b = 1 - a, 1 - b
        phi, dphi = oracle.basis(p, [a, b, rng.uniform(-1, 1)])
        assert abs(phi.sum() - 1) < 1e-12
        assert np.abs(dphi.sum(axis=0)).max() < 1e-10


def _poly_terms(p, rng, k=8):
    terms = []
    for _ in range(k):
        a = rng.integers(0, p + 1); b = rng.integers(0, p + 1 - a); g = rng.integers(0, p + 1)
        terms.append((rng.normal(), int(a), int(b), int(g)))
    return terms


def _poly_eval(terms, x):
    v = 0.0; d = np.zeros(3)
    for cf, a, b, g in terms:
        v += cf * x[0] ** a * x[1] ** b * x[2] ** g
        if a: d[0] += cf * a * x[0] ** (a - 1) * x[1] ** b * x[2] ** g
        if b: d[1] += cf * b * x[0] ** a * x[1] ** (b - 1) * x[2] ** g
        if g: d[2] += cf * g * x[0] ** a * x[1] ** b * x[2] ** (g - 1)
    return v, d


@pytest.mark.parametrize("p", range(1, 8))
def test_basis_reproduces_element_space(p):
    """sum_a u(node_a) phi_a = u and the same for gradients, for u in P_p(T) x P_p."""
    rng = np.random.default_rng(100 + p)
    terms = _poly_terms(p, rng)
    nodes = oracle.nodes(p)
    un = np.array([_poly_eval(terms, x)[0] for x in nodes])
    scale = sum(abs(t[0]) for t in terms) * (p + 1) ** 2
    for _ in range(6):
        a, b = rng.uniform(0, 1, 2)
        if a + b > 1:
            a, b = 1 - a, 1 - b
        x = np.array([a, b, rng.uniform(-1, 1)])
        phi, dphi = oracle.basis(p, x)
        u, du = _poly_eval(terms, x)
        assert abs(phi @ un - u) < 1e-12 * scale
        assert np.abs(dphi.T @ un - du).max() < 1e-11 * scale


def test_basis_p1_is_the_vertex_basis():
    rng = np.random.default_rng(7)
    for _ in range(5):
        a, b = rng.uniform(0, 0.5, 2); z = rng.uniform(-1, 1)
        lam = [1 - a - b, a, b]
        expect = [lam[i] * (1 - z) / 2 for i in range(3)] + [lam[i] * (1 + z) / 2 for i in range(3)]
        phi, _ = oracle.basis(1, [a, b, z])
        assert np.allclose(phi, expect, atol=1e-15)
    assert np.allclose(oracle.nodes(1), REF)


# --------------------------------------------------------------------------
# geometry
# --------------------------------------------------------------------------

def test_geometry_reference_prism_is_identity():
    J, det, K, x = oracle.geometry(REF, [0.2, 0.3, -0.4])
    assert np.allclose(J, np.eye(3), atol=1e-15) and abs(det - 1) < 1e-15
    assert np.allclose(K, np.eye(3), atol=1e-15) and np.allclose(x, [0.2, 0.3, -0.4])


def test_geometry_affine():
    M = np.array([[1.3, 0.2, -0.4], [0.1, 0.7, 0.3], [-0.2, 0.5, 0.9]])
    t = np.array([0.5, -1.0, 2.0])
    X = affine_prism(M, t)
    for xi in ([0.1, 0.1, 0.0], [0.6, 0.2, 0.9], [0.0, 1.0, -1.0]):
        J, det, K, x = oracle.geometry(X, xi)
        assert np.allclose(J, M, atol=1e-14)
        assert abs(det - np.linalg.det(M)) < 1e-14
        assert np.allclose(K, np.linalg.inv(M), atol=1e-13)
        assert np.allclose(x, M @ xi + t, atol=1e-14)


def test_mapped_points_on_distorted_prism():
    X = distorted_prism(3)
    pts, _ = oracle.rule(3)
    D, be, c, f = coeffs(3)
    _, _, _, xq = oracle.integrate(2, X[None], D[None], be[None], np.array([c]), np.array([f]), want_xq=True)
    for q, (a, b, z) in enumerate(pts):
        bot = (1 - a - b) * X[0] + a * X[1] + b * X[2]
        top = (1 - a - b) * X[3] + a * X[4] + b * X[5]
        assert np.allclose(xq[0, q], (1 - z) / 2 * bot + (1 + z) / 2 * top, atol=1e-15)


def test_inverted_element_is_flagged():
    D, be, c, f = coeffs(0)
    X = distorted_prism(0)
    assert integrate1(1, X, D, be, c, f)[2] == 0
    Xbad = X[[3, 4, 5, 0, 1, 2]]        # top and bottom swapped: det J < 0
    assert integrate1(1, Xbad, D, be, c, f)[2] == 1


# --------------------------------------------------------------------------
# element matrices
# --------------------------------------------------------------------------

@pytest.mark.parametrize("p", range(1, 6))
def test_symmetry_without_convection(p):
    X = distorted_prism(p)
    D, _, c, f = coeffs(p)
    A, _, _ = integrate1(p, X, D, np.zeros(3), c, f)
    assert np.abs(A - A.T).max() < 1e-14 * np.abs(A).max()
    Am, _, _ = integrate1(p, X, np.zeros((3, 3)), np.zeros(3), 1.0, f)
    assert np.abs(Am - Am.T).max() < 1e-14 * np.abs(Am).max()


@pytest.mark.parametrize("p", range(1, 7))
def test_zero_row_sums(p):
    X = distorted_prism(10 + p)
    D, be, _, _ = coeffs(p)
    Ad, _, _ = integrate1(p, X, D, np.zeros(3), 0.0, 0.0)
    s = np.abs(Ad).max()
    assert np.abs(Ad.sum(axis=1)).max() < 1e-12 * s
    assert np.abs(Ad.sum(axis=0)).max() < 1e-12 * s     # diffusion: columns too
    Ac, _, _ = integrate1(p, X, np.zeros((3, 3)), be, 0.0, 0.0)
    assert np.abs(Ac.sum(axis=1)).max() < 1e-12 * np.abs(Ac).max()
    # the convection column sums are not zero: the test above is discriminating
    assert np.abs(Ac.sum(axis=0)).max() > 1e-3 * np.abs(Ac).max()


def exact_volume(X):
    """Volume of the bilinear prism by exact symbolic integration of det(dx/dxi)."""
    import sympy as sp
    a, b, z = sp.symbols("a b z")
    Xr = [[sp.Rational(float(v)) for v in row] for row in X]
    lam = [1 - a - b, a, b]
    x = [sum(lam[i] * (1 - z) / 2 * Xr[i][d] + lam[i] * (1 + z) / 2 * Xr[i + 3][d] for i in range(3))
         for d in range(3)]
    J = sp.Matrix([[sp.diff(x[d], v) for v in (a, b, z)] for d in range(3)])
    det = sp.expand(J.det())
    vol = sp.integrate(sp.integrate(sp.integrate(det, (a, 0, 1 - b)), (b, 0, 1)), (z, -1, 1))
    return float(vol)


@pytest.mark.parametrize("p", range(1, 5))
def test_mass_sum_equals_exact_volume(p):
    X = distorted_prism(20 + p, amp=0.3)
    vol = exact_volume(X)
    A, b, _ = integrate1(p, X, np.zeros((3, 3)), np.zeros(3), 1.0, 0.7)
    assert abs(A.sum() - vol) < 1e-14 * abs(vol) * 10
    assert abs(b.sum() - 0.7 * vol) < 1e-14 * abs(vol) * 10


@pytest.mark.parametrize("p", [1, 3, 5])
def test_linearity_in_coefficients(p):
    X = distorted_prism(30 + p)
    D, be, c, f = coeffs(p)
    A, _, _ = integrate1(p, X, D, be, c, f)
    A1, _, _ = integrate1(p, X, D, np.zeros(3), 0.0, f)
    A2, _, _ = integrate1(p, X, np.zeros((3, 3)), be, 0.0, f)
    A3, _, _ = integrate1(p, X, np.zeros((3, 3)), np.zeros(3), c, f)
    assert np.abs(A - (A1 + A2 + A3)).max() < 1e-14 * np.abs(A).max() * 10


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_diffusion_psd_with_constant_nullspace(p):
    X = distorted_prism(40 + p)
    D, _, _, _ = coeffs(p)
    A, _, _ = integrate1(p, X, D, np.zeros(3), 0.0, 0.0)
    ev = np.linalg.eigvalsh(A)
    assert ev[0] > -1e-13 * ev[-1] and abs(ev[0]) < 1e-12 * ev[-1]
    assert ev[1] > 1e-6 * ev[-1]


def test_translation_and_scaling():
    p = 3
    X = distorted_prism(50)
    D, be, c, f = coeffs(50)
    parts = [(D, np.zeros(3), 0.0, 0.0, 1), (np.zeros((3, 3)), be, 0.0, 0.0, 2),
             (np.zeros((3, 3)), np.zeros(3), c, 0.0, 3)]
    for Dk, bk, ck, _, power in parts:
        A, _, _ = integrate1(p, X, Dk, bk, ck, f)
        At, _, _ = integrate1(p, X + np.array([3.0, -2.0, 5.0]), Dk, bk, ck, f)
        assert np.abs(At - A).max() < 1e-12 * np.abs(A).max()
        s = 1.7
        As, bs, _ = integrate1(p, s * X, Dk, bk, ck, f)
        assert np.abs(As - s ** power * A).max() < 1e-13 * np.abs(As).max()
    _, b, _ = integrate1(p, X, D, be, c, f)
    _, bs, _ = integrate1(p, 1.7 * X, D, be, c, f)
    assert np.abs(bs - 1.7 ** 3 * b).max() < 1e-13 * np.abs(bs).max()


def test_rotation_covariance():
    p = 2
    X = distorted_prism(60)
    D, be, c, f = coeffs(60)
    th = 0.7
    R1 = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]])
    R2 = np.array([[1, 0, 0], [0, math.cos(1.1), -math.sin(1.1)], [0, math.sin(1.1), math.cos(1.1)]])
    R = R2 @ R1
    A, b, _ = integrate1(p, X, D, be, c, f)
    Ar, br, _ = integrate1(p, X @ R.T, R @ D @ R.T, R @ be, c, f)
    assert np.abs(Ar - A).max() < 1e-13 * np.abs(A).max()
    assert np.abs(br - b).max() < 1e-13 * np.abs(b).max()


@pytest.mark.parametrize("p", [1, 2, 3])
def test_affine_prism_exact_bilinear_form(p):
    """v^T A u equals the exact integral of D grad u . grad v + v beta.grad u + c u v
    for physical polynomials u, v of degree p on an affine prism."""
    import sympy as sp
    x, y, zz = sp.symbols("x y z")
    a, b, z = sp.symbols("a b zeta")
    rng = np.random.default_rng(70 + p)
    Mq = [[Fraction(int(rng.integers(-3, 4)), 8) for _ in range(3)] for _ in range(3)]
    for i in range(3):
        Mq[i][i] += Fraction(1)
    M = sp.Matrix([[sp.Rational(v.numerator, v.denominator) for v in row] for row in Mq])
    if M.det() <= 0:
        M[:, 2] = -M[:, 2]
    t = sp.Matrix([sp.Rational(1, 3), sp.Rational(-1, 5), sp.Rational(2, 7)])
    Dm = sp.Matrix([[2, sp.Rational(1, 3), 0], [sp.Rational(1, 4), 1, sp.Rational(-1, 5)], [0, sp.Rational(1, 6), sp.Rational(3, 2)]])
    bv = sp.Matrix([sp.Rational(1, 2), -1, sp.Rational(3, 4)])
    cc = sp.Rational(2, 3)

    def rand_poly():
        e = 0
        for _ in range(6):
            i = int(rng.integers(0, p + 1)); j = int(rng.integers(0, p + 1 - i)); k = int(rng.integers(0, p + 1 - i - j))
            e += int(rng.integers(-4, 5)) * x ** i * y ** j * zz ** k
        return e + 1

    u, v = rand_poly(), rand_poly()
    gu = [sp.diff(u, s) for s in (x, y, zz)]
    gv = [sp.diff(v, s) for s in (x, y, zz)]
    integrand = sum(gv[i] * Dm[i, j] * gu[j] for i in range(3) for j in range(3)) \
        + v * sum(bv[i] * gu[i] for i in range(3)) + cc * u * v
    xmap = M * sp.Matrix([a, b, z]) + t
    integrand = sp.expand(integrand.subs({x: xmap[0], y: xmap[1], zz: xmap[2]}, simultaneous=True))
    exact = sp.integrate(sp.integrate(sp.integrate(integrand, (a, 0, 1 - b)), (b, 0, 1)), (z, -1, 1)) * M.det()

    Mf = np.array(M.tolist(), dtype=float); tf = np.array(t.tolist(), dtype=float).ravel()
    X = affine_prism(Mf, tf)
    nodes = oracle.nodes(p) @ Mf.T + tf
    un = np.array([float(u.subs({x: n[0], y: n[1], zz: n[2]})) for n in nodes])
    vn = np.array([float(v.subs({x: n[0], y: n[1], zz: n[2]})) for n in nodes])
    A, _, _ = integrate1(p, X, np.array(Dm.tolist(), dtype=float), np.array(bv.tolist(), dtype=float).ravel(),
                         float(cc), 0.0)
    got = vn @ A @ un
    assert abs(got - float(exact)) < 1e-12 * max(1.0, abs(float(exact)))


def test_right_prism_p1_textbook():
    """p=1 on T x [z0, z0+H] with D = diag(d1,d2,dz): the tensor-product form of the
    textbook P1 triangle and linear 1D matrices."""
    P = np.array([[0.1, 0.2], [0.9, 0.3], [0.4, 1.1]])
    z0, H = 0.25, 0.6
    X = np.array([[*P[i], z0] for i in range(3)] + [[*P[i], z0 + H] for i in range(3)])
    d1, d2, dz = 1.3, 0.7, 2.1
    bx, by, bz = 0.4, -1.2, 0.9
    c = 0.8
    area = 0.5 * ((P[1, 0] - P[0, 0]) * (P[2, 1] - P[0, 1]) - (P[2, 0] - P[0, 0]) * (P[1, 1] - P[0, 1]))
    bb = np.array([P[(i + 1) % 3, 1] - P[(i + 2) % 3, 1] for i in range(3)])
    cc = np.array([P[(i + 2) % 3, 0] - P[(i + 1) % 3, 0] for i in range(3)])
    KT = (d1 * np.outer(bb, bb) + d2 * np.outer(cc, cc)) / (4 * area)
    MT = area / 12 * (np.ones((3, 3)) + np.eye(3))
    CT = np.tile(area / 3 * (bx * bb + by * cc) / (2 * area), (3, 1))
    Mz = H / 6 * np.array([[2, 1], [1, 2]])
    Kz = np.array([[1, -1], [-1, 1]]) / H
    Cz = np.array([[-0.5, 0.5], [-0.5, 0.5]])
    expect = np.kron(Mz, KT) + dz * np.kron(Kz, MT) + np.kron(Mz, CT) + bz * np.kron(Cz, MT) + c * np.kron(Mz, MT)
    A, b, _ = integrate1(1, X, np.diag([d1, d2, dz]), [bx, by, bz], c, 0.5)
    assert np.abs(A - expect).max() < 1e-14 * np.abs(expect).max() * 10
    assert np.allclose(b, 0.5 * area * H / 6 * np.ones(6), atol=1e-15)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_over_integration(p):
    D, be, c, f = coeffs(80 + p)
    # affine: the standard rule is already exact
    Xa = affine_prism([[1.0, 0.3, 0.1], [0.0, 0.8, -0.2], [0.1, 0.0, 0.5]], [0, 0, 0])
    A0, b0, _ = integrate1(p, Xa, D, be, c, f)
    A1, b1, _ = integrate1(p, Xa, D, be, c, f, n1=p + 13)
    assert np.abs(A0 - A1).max() < 1e-13 * np.abs(A1).max()
    # distorted: over-integrated rules converge; the standard rule differs at the
    # quadrature-error level
    Xd = distorted_prism(90 + p, amp=0.3)
    A9, _, _ = integrate1(p, Xd, D, be, c, f, n1=p + 9)
    A13, _, _ = integrate1(p, Xd, D, be, c, f, n1=p + 13)
    As, _, _ = integrate1(p, Xd, D, be, c, f)
    ref = np.linalg.norm(A13)
    assert np.linalg.norm(A9 - A13) < 1e-12 * ref
    assert 1e-9 * ref < np.linalg.norm(As - A13) < 1e-1 * ref


# --------------------------------------------------------------------------
# adjoint
# --------------------------------------------------------------------------

def _loss(p, X, D, be, c, f, G, g):
    A, b, _ = integrate1(p, X, D, be, c, f)
    return float(np.sum(G * A) + np.sum(g * b))


def _adj_case(p, seed):
    X = distorted_prism(seed)
    D, be, c, f = coeffs(seed)
    D = D + np.array([[0, 0.2, 0], [-0.1, 0, 0], [0, 0.05, 0]])  # nonsymmetric D is allowed
    rng = np.random.default_rng(seed)
    n = oracle.nshp(p)
    return X, D, be, c, f, rng.normal(0, 1, (n, n)), rng.normal(0, 1, n)


def _adjoint1(p, X, D, be, c, f, G, g):
    out = oracle.adjoint(p, X[None], D[None], np.asarray(be)[None], np.array([c]), np.array([f]), G[None], g[None])
    return [o[0] for o in out]


@pytest.mark.parametrize("p", [1, 2, 3])
def test_adjoint_central_differences(p):
    X, D, be, c, f, G, g = _adj_case(p, 200 + p)
    dX, dD, db, dc, df, Le = _adjoint1(p, X, D, be, c, f, G, g)
    assert abs(Le - _loss(p, X, D, be, c, f, G, g)) < 1e-12 * abs(Le)
    h = 1e-6
    fd = []
    for k in range(18):
        e = np.zeros(18); e[k] = h
        fd.append((_loss(p, X + e.reshape(6, 3), D, be, c, f, G, g)
                   - _loss(p, X - e.reshape(6, 3), D, be, c, f, G, g)) / (2 * h))
    fdX = np.array(fd).reshape(6, 3)
    assert np.abs(fdX - dX).max() < 1e-6 * np.abs(dX).max()
    fdD = np.zeros((3, 3))
    for i in range(3):
        for j in range(3):
            E = np.zeros((3, 3)); E[i, j] = h
            fdD[i, j] = (_loss(p, X, D + E, be, c, f, G, g) - _loss(p, X, D - E, be, c, f, G, g)) / (2 * h)
    assert np.abs(fdD - dD).max() < 1e-6 * np.abs(dD).max()
    fdb = np.array([(_loss(p, X, D, be + h * np.eye(3)[k], c, f, G, g)
                     - _loss(p, X, D, be - h * np.eye(3)[k], c, f, G, g)) / (2 * h) for k in range(3)])
    assert np.abs(fdb - db).max() < 1e-6 * np.abs(db).max()
    fdc = (_loss(p, X, D, be, c + h, f, G, g) - _loss(p, X, D, be, c - h, f, G, g)) / (2 * h)
    fdf = (_loss(p, X, D, be, c, f + h, G, g) - _loss(p, X, D, be, c, f - h, G, g)) / (2 * h)
    assert abs(fdc - dc) < 1e-6 * abs(dc) and abs(fdf - df) < 1e-6 * abs(df)


@pytest.mark.parametrize("p", [1, 2, 4])
def test_adjoint_coefficient_identities(p):
    """Linearity in (D, beta, c, f): each coefficient gradient is <G, A(unit coefficient)>."""
    X, D, be, c, f, G, g = _adj_case(p, 300 + p)
    dX, dD, db, dc, df, Le = _adjoint1(p, X, D, be, c, f, G, g)
    Z = np.zeros((3, 3)); z = np.zeros(3)
    for i in range(3):
        for j in range(3):
            E = Z.copy(); E[i, j] = 1
            A, _, _ = integrate1(p, X, E, z, 0.0, 0.0)
            assert abs(np.sum(G * A) - dD[i, j]) < 1e-12 * np.abs(dD).max()
    for k in range(3):
        A, _, _ = integrate1(p, X, Z, np.eye(3)[k], 0.0, 0.0)
        assert abs(np.sum(G * A) - db[k]) < 1e-12 * np.abs(db).max()
    A, _, _ = integrate1(p, X, Z, z, 1.0, 0.0)
    assert abs(np.sum(G * A) - dc) < 1e-12 * abs(dc)
    _, b, _ = integrate1(p, X, Z, z, 0.0, 1.0)
    assert abs(np.sum(g * b) - df) < 1e-12 * abs(df)


@pytest.mark.parametrize("p", [1, 3])
def test_adjoint_translation_and_homogeneity(p):
    X, D, be, c, f, G, g = _adj_case(p, 400 + p)
    dX, *_ = _adjoint1(p, X, D, be, c, f, G, g)
    assert np.abs(dX.sum(axis=0)).max() < 1e-11 * np.abs(dX).max()
    Z = np.zeros((3, 3)); z = np.zeros(3)
    Ld = _loss(p, X, D, z, 0.0, 0.0, G, g)
    Lc = _loss(p, X, Z, be, 0.0, 0.0, G, g)
    Lm = _loss(p, X, Z, z, c, 0.0, G, g)
    Ll = _loss(p, X, Z, z, 0.0, f, G, g)
    assert abs(np.sum(X * dX) - (Ld + 2 * Lc + 3 * Lm + 3 * Ll)) < 1e-11 * np.abs(X * dX).sum()


# --------------------------------------------------------------------------
# meshes
# --------------------------------------------------------------------------

def test_mesh_volume_and_validity():
    b = meshgen.make_batch(6, 5, 4, amp=0.2, seed=1)
    A, _, flags = oracle.integrate(1, b.coords, np.zeros_like(b.D), np.zeros_like(b.beta),
                                   np.ones(b.ne), np.zeros(b.ne))
    assert abs(A.sum() - 1.0) < 1e-13
    assert flags.sum() == 0


def test_mesh_is_seeded_and_perturbs_interior_only():
    b1 = meshgen.make_batch(4, 4, 2, 0.2, seed=5, with_conn=True)
    b2 = meshgen.make_batch(4, 4, 2, 0.2, seed=5)
    assert np.array_equal(b1.coords, b2.coords) and np.array_equal(b1.D, b2.D)
    v = b1.meta["verts"]
    on_boundary = np.any((np.isclose(v, 0) | np.isclose(v, 1)), axis=1)
    assert on_boundary.sum() >= 2 * 25   # top and bottom faces at least
    assert np.all(np.abs(b1.D - np.transpose(b1.D, (0, 2, 1))) == 0)
    assert np.all(np.linalg.eigvalsh(b1.D) >= 1 - 1e-12)


# ---- spatially varying coefficients (vertex fields) -------------------------

def _vertex_fields(batch):
    """Per-vertex copies of the element constants (the constant field)."""
    rep = lambda a: np.repeat(a[:, None], 6, axis=1)
    return rep(batch.D), rep(batch.beta), rep(batch.c), rep(batch.f)


def test_fields_constant_reduce_to_element_constants():
    from paper_1310_1194_amd import meshgen
    for p in (1, 3):
        batch = meshgen.make_batch(2, 2, 1, amp=0.25, seed=50 + p)
        A0, b0, _ = oracle.integrate(p, batch.coords, batch.D, batch.beta, batch.c, batch.f)
        A1, b1, _ = oracle.integrate_fields(p, batch.coords, *_vertex_fields(batch))
        assert np.abs(A1 - A0).max() <= 1e-14 * np.abs(A0).max()
        assert np.abs(b1 - b0).max() <= 1e-14 * np.abs(b0).max()


def test_fields_affine_reaction_and_source_integrate_the_field():
    """c(x), f(x) affine, given by their vertex values: the mass sum and the
    load sum equal the rule applied to c and f evaluated at the mapped points
    (geometry only, no coefficient interpolation), which the rule integrates
    exactly (degree <= 3 per direction at p >= 2)."""
    from paper_1310_1194_amd import meshgen
    p = 2
    batch = meshgen.make_batch(2, 2, 2, amp=0.25, seed=61)
    ne = batch.ne
    g_c, c0 = np.array([0.7, -0.4, 1.3]), 0.9
    g_f, f0 = np.array([-1.1, 0.5, 0.2]), -0.3
    cv = c0 + batch.coords @ g_c          # [ne, 6]
    fv = f0 + batch.coords @ g_f
    Dv = np.zeros((ne, 6, 3, 3)); bv = np.zeros((ne, 6, 3))
    A, b, _ = oracle.integrate_fields(p, batch.coords, Dv, bv, cv, fv)
    pts, w = oracle.rule(p + 1)
    for e in range(ne):
        sc = sf = 0.0
        for q in range(len(w)):
            J, det, K, x = oracle.geometry(batch.coords[e], pts[q])
            sc += w[q] * det * (c0 + x @ g_c)
            sf += w[q] * det * (f0 + x @ g_f)
        assert abs(A[e].sum() - sc) <= 1e-13 * abs(sc) + 1e-16
        assert abs(b[e].sum() - sf) <= 1e-13 * abs(sf) + 1e-16


def test_fields_are_linear():
    from paper_1310_1194_amd import meshgen
    p = 2
    batch = meshgen.make_batch(2, 1, 1, amp=0.2, seed=62)
    rng = np.random.default_rng(3)
    ne = batch.ne
    F1 = [rng.normal(size=(ne, 6, 3, 3)), rng.normal(size=(ne, 6, 3)), rng.normal(size=(ne, 6)), rng.normal(size=(ne, 6))]
    F2 = [rng.normal(size=a.shape) for a in F1]
    A1, b1, _ = oracle.integrate_fields(p, batch.coords, *F1)
    A2, b2, _ = oracle.integrate_fields(p, batch.coords, *F2)
    A3, b3, _ = oracle.integrate_fields(p, batch.coords, *[2.0 * x - 3.0 * y for x, y in zip(F1, F2)])
    assert np.abs(A3 - (2 * A1 - 3 * A2)).max() <= 1e-13 * np.abs(A3).max()
    assert np.abs(b3 - (2 * b1 - 3 * b2)).max() <= 1e-13 * np.abs(b3).max()


def test_laplace_right_prism_p1_textbook():
    """The Laplace-only oracle (the paper's eq. (1)) on its symmetric rule, p=1,
    right prism: M_z (x) K_T + K_z (x) M_T with the textbook P1 triangle and
    linear 1D matrices (the rule is exact on affine prisms)."""
    import oracle
    P = np.array([[0.1, 0.2], [0.9, 0.3], [0.4, 1.1]])
    z0, H = 0.25, 0.6
    X = np.array([[*P[i], z0] for i in range(3)] + [[*P[i], z0 + H] for i in range(3)])
    area = 0.5 * ((P[1, 0] - P[0, 0]) * (P[2, 1] - P[0, 1]) - (P[2, 0] - P[0, 0]) * (P[1, 1] - P[0, 1]))
    bb = np.array([P[(i + 1) % 3, 1] - P[(i + 2) % 3, 1] for i in range(3)])
    cc = np.array([P[(i + 2) % 3, 0] - P[(i + 1) % 3, 0] for i in range(3)])
    KT = (np.outer(bb, bb) + np.outer(cc, cc)) / (4 * area)
    MT = area / 12 * (np.ones((3, 3)) + np.eye(3))
    Mz = H / 6 * np.array([[2, 1], [1, 2]])
    Kz = np.array([[1, -1], [-1, 1]]) / H
    expect = np.kron(Mz, KT) + np.kron(Kz, MT)
    A, flags = oracle.integrate_laplace(1, X[None])
    assert flags[0] == 0
    assert np.abs(A[0] - expect).max() < 1e-14 * np.abs(expect).max() * 10


def test_det_condition_helper_matches_oracle_jacobian():
    """The conditioning estimate the FP64 GPU tolerances use takes J from the
    prism map; it must agree with the oracle's Jacobian (det and columns) on a
    distorted mesh, including an element with an inverted corner."""
    import sys
    from pathlib import Path
    sys.path.insert(0, str(Path(__file__).parent))
    from gpu_util import det_condition
    from paper_1310_1194_amd import meshgen
    b = meshgen.make_batch(3, 2, 2, amp=0.3, seed=4)
    pts, _ = oracle.prism_rule(3, "collapsed")
    kap = det_condition(b.coords, pts)
    for e in (0, 5, b.ne - 1):
        ref = 0.0
        for q in range(pts.shape[0]):
            J, det, K, x = oracle.geometry(b.coords[e], pts[q])
            ref = max(ref, np.prod(np.linalg.norm(J, axis=0)) / abs(det))
        assert abs(kap[e] - ref) <= 1e-9 * ref
    assert (kap >= 1.0 - 1e-12).all()
