"""Pins of the oracle's symmetric prism rule (fully symmetric triangle rule of
degree 2p x (p+1) Gauss points in zeta) and of the element loop on a rule
given by the caller.

The rule is pinned by the point counts the paper prints (Table 3), exact
monomial integrals over the triangle and the prism (closed form i! j! /
(i+j+2)!), positivity, interior points and invariance under permutations of
the barycentric coordinates.  The element loop on it is pinned by exactness
where both rules are exact (affine prisms, constant coefficients), by the
exact volume of distorted prisms, by zero diffusion row sums and by the
plumbing reproducing the built-in collapsed rule bit for bit.
"""
import itertools
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import rules
from test_costmodel import golden
from test_oracle_pins import affine_prism, coeffs, distorted_prism, exact_volume, integrate1, tri_monomial

P = range(1, 8)


def sym(p):
    return oracle.prism_rule(p, "symmetric")


def integrate_sym(p, X, D, beta, c, f):
    A, b, fl = oracle.integrate(p, X[None], D[None], np.asarray(beta, float)[None], np.array([c], float),
                                np.array([f], float), rule="symmetric")
    return A[0], b[0], int(fl[0])


def test_point_counts_match_paper_table3():
    g = golden()
    for p in P:
        pts, w = sym(p)
        assert 4 * len(w) == g["table3_quadrature"][p - 1]          # 4 scalars per point
        assert len(w) * g["table3_shape_at_point"][p - 1] == g["table3_shape_all_points"][p - 1]


@pytest.mark.parametrize("p", P)
def test_triangle_rule_exact_to_degree_2p(p):
    xi, w = rules.triangle_rule(p)
    assert (w > 0).all()
    lam = np.c_[1 - xi.sum(1), xi]
    assert (lam > 0).all()                                            # strictly interior
    worst = 0.0
    for i in range(2 * p + 1):
        for j in range(2 * p + 1 - i):
            exact = float(tri_monomial(i, j))
            worst = max(worst, abs(np.sum(w * xi[:, 0] ** i * xi[:, 1] ** j) - exact) / exact)
    assert worst < 5e-15


@pytest.mark.parametrize("p", P)
def test_triangle_rule_not_exact_beyond(p):
    """The exactness check is discriminating: some monomial of degree 2p+1 or
    2p+2 is not integrated exactly."""
    xi, w = rules.triangle_rule(p)
    worst = 0.0
    for d in (2 * p + 1, 2 * p + 2):
        for i in range(d + 1):
            exact = float(tri_monomial(i, d - i))
            worst = max(worst, abs(np.sum(w * xi[:, 0] ** i * xi[:, 1] ** (d - i)) - exact) / exact)
    assert worst > 1e-8


@pytest.mark.parametrize("p", P)
def test_triangle_rule_fully_symmetric(p):
    xi, w = rules.triangle_rule(p)
    lam = np.c_[1 - xi.sum(1), xi]
    key = lambda L, W: sorted(zip(np.round(L[:, 0], 13), np.round(L[:, 1], 13), np.round(W, 15)))
    ref = key(lam, w)
    for perm in itertools.permutations(range(3)):
        assert key(lam[:, perm], w) == ref


@pytest.mark.parametrize("p", P)
def test_prism_rule_exact(p):
    pts, w = sym(p)
    assert abs(w.sum() - 1.0) < 1e-14
    worst = 0.0
    for i in range(2 * p + 1):
        for j in range(2 * p + 1 - i):
            for g in (0, 1, 2, 2 * p, 2 * p + 1):
                exact = float(tri_monomial(i, j) * (Fraction(0) if g % 2 else Fraction(2, g + 1)))
                got = np.sum(w * pts[:, 0] ** i * pts[:, 1] ** j * pts[:, 2] ** g)
                worst = max(worst, abs(got - exact))
    assert worst < 1e-15


@pytest.mark.parametrize("p", [1, 3, 6])
def test_rule_plumbing_reproduces_builtin(p):
    X = distorted_prism(40 + p)
    D, be, c, f = coeffs(40 + p)
    A0, b0, _ = integrate1(p, X, D, be, c, f)
    pts, w = oracle.rule(p + 1)
    A1, b1, _ = oracle.integrate_rule(p, pts, w, X[None], D[None], be[None], np.array([c]), np.array([f]))
    assert np.array_equal(A0, A1[0]) and np.array_equal(b0, b1[0])


@pytest.mark.parametrize("p", P)
def test_symmetric_equals_collapsed_on_affine_prisms(p):
    """Constant coefficients on an affine prism: the integrand is a polynomial
    both rules integrate exactly, so the two element matrices agree."""
    M = np.array([[1.1, 0.2, -0.1], [0.1, 0.9, 0.05], [-0.2, 0.1, 0.6]])
    X = affine_prism(M, [0.2, -0.3, 0.5])
    D, be, c, f = coeffs(50 + p)
    A0, b0, _ = integrate1(p, X, D, be, c, f)
    A1, b1, fl = integrate_sym(p, X, D, be, c, f)
    assert fl == 0
    assert np.abs(A1 - A0).max() < 1e-13 * np.abs(A0).max()
    assert np.abs(b1 - b0).max() < 1e-13 * np.abs(b0).max()


@pytest.mark.parametrize("p", [1, 2, 4])
def test_symmetric_mass_sum_is_exact_volume(p):
    """det J of a bilinear prism has degree 2 in xi and 2 in zeta: integrated
    exactly by the rule, so the mass entries sum to the exact volume."""
    X = distorted_prism(60 + p, amp=0.3)
    vol = exact_volume(X)
    A, b, _ = integrate_sym(p, X, np.zeros((3, 3)), np.zeros(3), 1.0, 0.7)
    assert abs(A.sum() - vol) < 1e-13 * abs(vol)
    assert abs(b.sum() - 0.7 * vol) < 1e-13 * abs(vol)


@pytest.mark.parametrize("p", [2, 5])
def test_symmetric_diffusion_rows_sum_to_zero(p):
    X = distorted_prism(70 + p, amp=0.3)
    D, _, _, _ = coeffs(70 + p)
    A, _, _ = integrate_sym(p, X, D, np.zeros(3), 0.0, 0.0)
    assert np.abs(A.sum(axis=1)).max() < 1e-12 * np.abs(A).max()
    assert np.abs(A - A.T).max() < 1e-12 * np.abs(A).max()


@pytest.mark.parametrize("p", [2, 4])
def test_symmetric_close_to_overintegrated_on_distorted(p):
    """Distorted prisms: both rules approximate the same integral; against a
    heavily over-integrated collapsed rule the symmetric rule's error is small
    and of the order of the default collapsed rule's."""
    X = distorted_prism(80 + p, amp=0.3)
    D, be, c, f = coeffs(80 + p)
    Ar, _, _ = integrate1(p, X, D, be, c, f, n1=p + 9)
    A0, _, _ = integrate1(p, X, D, be, c, f)
    A1, _, _ = integrate_sym(p, X, D, be, c, f)
    e0 = np.linalg.norm(A0 - Ar) / np.linalg.norm(Ar)
    e1 = np.linalg.norm(A1 - Ar) / np.linalg.norm(Ar)
    assert e1 < 1e-2 and e1 < 50 * e0


@pytest.mark.parametrize("p", [3])
def test_fields_on_rule_reduce_to_element_constants(p):
    X = distorted_prism(90 + p)
    D, be, c, f = coeffs(90 + p)
    rep = lambda a: np.repeat(np.asarray(a, float)[None, None], 6, axis=1)
    A0, b0, _ = integrate_sym(p, X, D, be, c, f)
    A1, b1, _ = oracle.integrate_fields(p, X[None], rep(D), rep(be), rep(c), rep(f), rule="symmetric")
    assert np.abs(A1[0] - A0).max() < 1e-14 * np.abs(A0).max()
    assert np.abs(b1[0] - b0).max() < 1e-14 * np.abs(b0).max()


@pytest.mark.parametrize("p", [1, 3])
def test_adjoint_on_symmetric_rule_central_differences(p):
    """The oracle's adjoint on the symmetric rule against central differences
    of its forward integration on the same rule (h = 1e-6)."""
    rng = np.random.default_rng(300 + p)
    X = distorted_prism(300 + p, amp=0.3)
    D, be, c, f = coeffs(300 + p)
    n = oracle.nshp(p)
    G = rng.normal(0, 1, (n, n)); g = rng.normal(0, 1, n)

    def loss(Xv, Dv, bv, cv, fv):
        A, b, _ = integrate_sym(p, Xv, Dv, bv, cv, fv)
        return float(np.sum(G * A) + g @ b)

    dX, dD, db, dc, df, Le = oracle.adjoint(p, X[None], D[None], be[None], np.array([c]), np.array([f]),
                                            G[None], g[None], rule="symmetric")
    assert abs(Le[0] - loss(X, D, be, c, f)) < 1e-12 * abs(Le[0])
    h = 1e-6
    fdX = np.zeros(18)
    for k in range(18):
        e = np.zeros(18); e[k] = h
        fdX[k] = (loss(X + e.reshape(6, 3), D, be, c, f) - loss(X - e.reshape(6, 3), D, be, c, f)) / (2 * h)
    assert np.abs(fdX.reshape(6, 3) - dX[0]).max() < 1e-6 * np.abs(dX).max()
    fdD = np.array([[(loss(X, D + h * np.outer(np.eye(3)[i], np.eye(3)[j]), be, c, f)
                      - loss(X, D - h * np.outer(np.eye(3)[i], np.eye(3)[j]), be, c, f)) / (2 * h)
                     for j in range(3)] for i in range(3)])
    assert np.abs(fdD - dD[0]).max() < 1e-6 * np.abs(dD).max()
    fdb = np.array([(loss(X, D, be + h * np.eye(3)[k], c, f) - loss(X, D, be - h * np.eye(3)[k], c, f)) / (2 * h)
                    for k in range(3)])
    assert np.abs(fdb - db[0]).max() < 1e-6 * np.abs(db).max()
    assert abs((loss(X, D, be, c + h, f) - loss(X, D, be, c - h, f)) / (2 * h) - dc[0]) < 1e-6 * abs(dc[0])
    assert abs((loss(X, D, be, c, f + h) - loss(X, D, be, c, f - h)) / (2 * h) - df[0]) < 1e-6 * abs(df[0])
