"""ctypes binding of the plain FP64 CPU oracle (``feint_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
benchmark's CPU-baseline leg.  The product library never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from pathlib import Path

import numpy as np

HERE = Path(__file__).resolve().parent
SRC = HERE / "feint_oracle.c"
LIB = HERE / "liboracle.so"

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


def build(force: bool = True) -> Path:
    """Compile the oracle with gcc: -O2, no FMA contraction, no fast-math, OpenMP."""
    if force or not LIB.exists() or LIB.stat().st_mtime < SRC.stat().st_mtime:
        tmp = LIB.with_suffix(".so.tmp")
        cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-Wall", "-o", str(tmp), str(SRC), "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not LIB.exists():
            build()
        L = ctypes.CDLL(str(LIB))
        L.oracle_gauss_legendre.argtypes = [ctypes.c_int, _dp, _dp]
        L.oracle_gll_nodes.argtypes = [ctypes.c_int, _dp]
        L.oracle_rule.argtypes = [ctypes.c_int, _dp, _dp]
        L.oracle_nodes.argtypes = [ctypes.c_int, _dp]
        L.oracle_basis.argtypes = [ctypes.c_int, _dp, _dp, _dp]
        L.oracle_geometry.argtypes = [_dp, _dp, _dp, _dp, _dp, _dp]
        L.oracle_integrate.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64] + [_dp] * 8 + [_ip]
        L.oracle_integrate_fields.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64] + [_dp] * 8 + [_ip]
        L.oracle_integrate_rule.argtypes = ([ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_int64, ctypes.c_int]
                                            + [_dp] * 8 + [_ip])
        L.oracle_tet_rule.argtypes = [ctypes.c_int, _dp, _dp]
        L.oracle_tet_nodes.argtypes = [ctypes.c_int, _dp]
        L.oracle_tet_basis.argtypes = [ctypes.c_int, _dp, _dp, _dp]
        L.oracle_tet_geometry.argtypes = [_dp, _dp, _dp, _dp, _dp, _dp]
        L.oracle_integrate_tet.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64] + [_dp] * 8 + [_ip]
        L.oracle_hex_rule.argtypes = [ctypes.c_int, _dp, _dp]
        L.oracle_hex_nodes.argtypes = [ctypes.c_int, _dp]
        L.oracle_hex_basis.argtypes = [ctypes.c_int, _dp, _dp, _dp]
        L.oracle_hex_geometry.argtypes = [_dp, _dp, _dp, _dp, _dp, _dp]
        L.oracle_integrate_hex.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64] + [_dp] * 8 + [_ip]
        L.oracle_adjoint.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64] + [_dp] * 13
        L.oracle_adjoint_rule.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_int64] + [_dp] * 13
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _c(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def nshp(p):
    return (p + 1) * (p + 1) * (p + 2) // 2


def gauss_legendre(n):
    x = np.zeros(n); w = np.zeros(n)
    assert lib().oracle_gauss_legendre(n, _p(x), _p(w)) == 0
    return x, w


def gll_nodes(p):
    x = np.zeros(p + 1)
    assert lib().oracle_gll_nodes(p, _p(x)) == 0
    return x


def rule(n1):
    pts = np.zeros((n1 ** 3, 3)); w = np.zeros(n1 ** 3)
    assert lib().oracle_rule(n1, _p(pts), _p(w)) == n1 ** 3
    return pts, w


def nodes(p):
    out = np.zeros((nshp(p), 3))
    assert lib().oracle_nodes(p, _p(out)) == nshp(p)
    return out


def basis(p, xi):
    """phi [n], reference gradients [n,3] at one point xi = (xi1, xi2, zeta)."""
    xi = _c(xi)
    n = nshp(p)
    phi = np.zeros(n); dphi = np.zeros((n, 3))
    assert lib().oracle_basis(p, _p(xi), _p(phi), _p(dphi)) == 0
    return phi, dphi


def geometry(X, xi):
    """J [3,3], det, K = J^{-1} [3,3], mapped point x [3]."""
    X = _c(X); xi = _c(xi)
    J = np.zeros((3, 3)); K = np.zeros((3, 3)); x = np.zeros(3); det = np.zeros(1)
    lib().oracle_geometry(_p(X), _p(xi), _p(J), _p(det), _p(K), _p(x))
    return J, float(det[0]), K, x


def prism_rule(p, rule):
    """(pts [nq,3], w [nq]) of a named rule: "collapsed" ((p+1)^3-point
    collapsed Gauss) or "symmetric" (symmetric triangle rule of degree 2p x
    (p+1) Gauss points in zeta, ``oracle/rules.py``)."""
    if rule == "collapsed":
        return globals()["rule"](p + 1)
    if rule == "symmetric":
        from . import rules
        return rules.prism_rule(p, gauss_legendre)
    raise ValueError(f"unknown rule {rule!r}")


def _integrate_on(p, pts, w, nv, coords, D, beta, c, f, want_xq):
    coords = _c(coords); D = _c(D); beta = _c(beta); c = _c(c); f = _c(f)
    pts = _c(pts); w = _c(w)
    ne, n, nq = coords.shape[0], nshp(p), w.shape[0]
    A = np.zeros((ne, n, n)); b = np.zeros((ne, n))
    flags = np.zeros(ne, dtype=np.int32)
    xq = np.zeros((ne, nq, 3)) if want_xq else None
    rc = lib().oracle_integrate_rule(p, nq, _p(pts), _p(w), ne, nv, _p(coords), _p(D), _p(beta), _p(c), _p(f),
                                     _p(A), _p(b), _p(xq), flags.ctypes.data_as(_ip))
    assert rc == 0, rc
    return (A, b, flags, xq) if want_xq else (A, b, flags)


def integrate_rule(p, pts, w, coords, D, beta, c, f, want_xq=False):
    """Element-constant coefficients on the caller's rule (pts [nq,3], w [nq])."""
    return _integrate_on(p, pts, w, 1, coords, D, beta, c, f, want_xq)


def integrate_fields_rule(p, pts, w, coords, Dv, betav, cv, fv, want_xq=False):
    """Vertex coefficient fields on the caller's rule."""
    return _integrate_on(p, pts, w, 6, coords, Dv, betav, cv, fv, want_xq)


def integrate(p, coords, D, beta, c, f, n1=0, want_xq=False, rule=None):
    """A [ne,n,n], b [ne,n], flags [ne] (and xq [ne,nq,3] when asked).
    rule=None: collapsed Gauss with n1 (default p+1) points per direction;
    rule="symmetric": the symmetric prism rule."""
    if rule is not None:
        return integrate_rule(p, *prism_rule(p, rule), coords, D, beta, c, f, want_xq)
    coords = _c(coords); D = _c(D); beta = _c(beta); c = _c(c); f = _c(f)
    ne = coords.shape[0]
    n = nshp(p)
    nqq = (n1 if n1 > 0 else p + 1) ** 3
    A = np.zeros((ne, n, n)); b = np.zeros((ne, n))
    flags = np.zeros(ne, dtype=np.int32)
    xq = np.zeros((ne, nqq, 3)) if want_xq else None
    rc = lib().oracle_integrate(p, n1, ne, _p(coords), _p(D), _p(beta), _p(c), _p(f),
                                _p(A), _p(b), _p(xq), flags.ctypes.data_as(_ip))
    assert rc == 0, rc
    if want_xq:
        return A, b, flags, xq
    return A, b, flags


def integrate_laplace(p, coords, rule="symmetric"):
    """The paper's own term (its eq. (1)): A_ab = sum_q w_q det J_q grad phi_a .
    grad phi_b on the given rule (default: the symmetric rule, the paper's
    N_I points), i.e. the element loop above with D = I and no convection,
    reaction or source.  Returns A [ne,n,n] and the det J <= 0 flags."""
    coords = _c(coords)
    ne = coords.shape[0]
    D = np.repeat(np.eye(3)[None], ne, axis=0)
    z3, z1 = np.zeros((ne, 3)), np.zeros(ne)
    A, _, flags = integrate(p, coords, D, z3, z1, z1, rule=rule)
    return A, flags


def integrate_fields(p, coords, Dv, betav, cv, fv, n1=0, want_xq=False, rule=None):
    """Coefficients given at the six vertices (Dv [ne,6,3,3], betav [ne,6,3],
    cv [ne,6], fv [ne,6]) and evaluated at each point with the geometry shape
    functions.  Returns A, b, flags (and xq)."""
    if rule is not None:
        return integrate_fields_rule(p, *prism_rule(p, rule), coords, Dv, betav, cv, fv, want_xq)
    coords = _c(coords); Dv = _c(Dv); betav = _c(betav); cv = _c(cv); fv = _c(fv)
    ne = coords.shape[0]
    n = nshp(p)
    nqq = (n1 if n1 > 0 else p + 1) ** 3
    A = np.zeros((ne, n, n)); b = np.zeros((ne, n))
    flags = np.zeros(ne, dtype=np.int32)
    xq = np.zeros((ne, nqq, 3)) if want_xq else None
    rc = lib().oracle_integrate_fields(p, n1, ne, _p(coords), _p(Dv), _p(betav), _p(cv), _p(fv),
                                       _p(A), _p(b), _p(xq), flags.ctypes.data_as(_ip))
    assert rc == 0, rc
    if want_xq:
        return A, b, flags, xq
    return A, b, flags


def adjoint(p, coords, D, beta, c, f, G, g, n1=0, rule=None):
    """Gradients of sum_e <G_e,A_e> + <g_e,b_e>: dcoords, dD, dbeta, dc, df, per-element loss.
    rule=None: collapsed Gauss with n1 points per direction; rule="symmetric": the symmetric rule."""
    coords = _c(coords); D = _c(D); beta = _c(beta); c = _c(c); f = _c(f); G = _c(G); g = _c(g)
    ne = coords.shape[0]
    dX = np.zeros_like(coords); dD = np.zeros_like(D); db = np.zeros_like(beta)
    dc = np.zeros(ne); df = np.zeros(ne); Le = np.zeros(ne)
    if rule is not None:
        pts, w = prism_rule(p, rule)
        pts = _c(pts); w = _c(w)
        rc = lib().oracle_adjoint_rule(p, w.shape[0], _p(pts), _p(w), ne, _p(coords), _p(D), _p(beta), _p(c), _p(f),
                                       _p(G), _p(g), _p(dX), _p(dD), _p(db), _p(dc), _p(df), _p(Le))
        assert rc == 0, rc
        return dX, dD, db, dc, df, Le
    rc = lib().oracle_adjoint(p, n1, ne, _p(coords), _p(D), _p(beta), _p(c), _p(f), _p(G), _p(g),
                              _p(dX), _p(dD), _p(db), _p(dc), _p(df), _p(Le))
    assert rc == 0, rc
    return dX, dD, db, dc, df, Le


def assemble(dofs, ndof, A, b):
    """Global assembly (Sec. 2: the element matrices are summed into the global
    matrix through the element-to-global numbering), plain FP64.

    Every element contributes A_e[a, b] to entry (dofs[e, a], dofs[e, b]) and
    b_e[a] to rhs[dofs[e, a]].  Entries are grouped by a stable sort of their
    (row, col) key, so each global entry is the sum of its contributions in
    element order.  Returns (row_ptr [ndof+1], cols [nnz], vals [nnz], rhs
    [ndof]) with columns ascending within a row."""
    dofs = np.asarray(dofs, dtype=np.int64)
    ne, n = dofs.shape
    A = np.asarray(A, dtype=np.float64).reshape(ne, n, n)
    b = np.asarray(b, dtype=np.float64).reshape(ne, n)
    rows = np.repeat(dofs[:, :, None], n, axis=2).ravel()
    cols = np.repeat(dofs[:, None, :], n, axis=1).ravel()
    key = rows * ndof + cols
    order = np.argsort(key, kind="stable")
    key_s = key[order]
    vals_s = A.ravel()[order]
    start = np.flatnonzero(np.r_[True, key_s[1:] != key_s[:-1]])
    uniq = key_s[start]
    vals = np.empty(len(start))
    for m in range(len(start)):                      # contributions in element order
        stop = start[m + 1] if m + 1 < len(start) else len(key_s)
        acc = 0.0
        for v in vals_s[start[m]:stop]:
            acc += v
        vals[m] = acc
    r = uniq // ndof
    row_ptr = np.zeros(ndof + 1, dtype=np.int64)
    np.add.at(row_ptr, r + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    rhs = np.zeros(ndof)
    for e in range(ne):                              # dofs of one element are distinct
        rhs[dofs[e]] += b[e]
    return row_ptr, (uniq % ndof).astype(np.int64), vals, rhs


def hex_nshp(p):
    return (p + 1) ** 3


def hex_rule(n1):
    """n1^3 Gauss points on [-1,1]^3 (pts [nq,3], w [nq]), q = (k n1 + j) n1 + i."""
    pts = np.zeros((n1 ** 3, 3)); w = np.zeros(n1 ** 3)
    assert lib().oracle_hex_rule(n1, _p(pts), _p(w)) == n1 ** 3
    return pts, w


def hex_nodes(p):
    out = np.zeros((hex_nshp(p), 3))
    assert lib().oracle_hex_nodes(p, _p(out)) == hex_nshp(p)
    return out


def hex_basis(p, xi):
    """Tensor-product Gauss-Lobatto Lagrange basis: phi [n], gradients [n,3]."""
    xi = _c(xi)
    n = hex_nshp(p)
    phi = np.zeros(n); dphi = np.zeros((n, 3))
    assert lib().oracle_hex_basis(p, _p(xi), _p(phi), _p(dphi)) == 0
    return phi, dphi


def hex_geometry(X, xi):
    """Trilinear hexahedron X [8,3]: J [3,3], det, K = J^{-1}, mapped point."""
    X = _c(X); xi = _c(xi)
    J = np.zeros((3, 3)); K = np.zeros((3, 3)); x = np.zeros(3); det = np.zeros(1)
    lib().oracle_hex_geometry(_p(X), _p(xi), _p(J), _p(det), _p(K), _p(x))
    return J, float(det[0]), K, x


def integrate_hex(p, coords, D, beta, c, f, n1=0, want_xq=False):
    """Hexahedra (coords [ne,8,3]): A [ne,n,n], b [ne,n], flags (and xq)."""
    coords = _c(coords); D = _c(D); beta = _c(beta); c = _c(c); f = _c(f)
    ne, n = coords.shape[0], hex_nshp(p)
    nqq = (n1 if n1 > 0 else p + 1) ** 3
    A = np.zeros((ne, n, n)); b = np.zeros((ne, n))
    flags = np.zeros(ne, dtype=np.int32)
    xq = np.zeros((ne, nqq, 3)) if want_xq else None
    rc = lib().oracle_integrate_hex(p, n1, ne, _p(coords), _p(D), _p(beta), _p(c), _p(f),
                                    _p(A), _p(b), _p(xq), flags.ctypes.data_as(_ip))
    assert rc == 0, rc
    return (A, b, flags, xq) if want_xq else (A, b, flags)


def tet_nshp(p):
    return (p + 1) * (p + 2) * (p + 3) // 6


def tet_rule(n1):
    """n1^3 collapsed Gauss points on the reference tetrahedron (pts, w)."""
    pts = np.zeros((n1 ** 3, 3)); w = np.zeros(n1 ** 3)
    assert lib().oracle_tet_rule(n1, _p(pts), _p(w)) == n1 ** 3
    return pts, w


def tet_nodes(p):
    out = np.zeros((tet_nshp(p), 3))
    assert lib().oracle_tet_nodes(p, _p(out)) == tet_nshp(p)
    return out


def tet_basis(p, xi):
    xi = _c(xi)
    n = tet_nshp(p)
    phi = np.zeros(n); dphi = np.zeros((n, 3))
    assert lib().oracle_tet_basis(p, _p(xi), _p(phi), _p(dphi)) == 0
    return phi, dphi


def tet_geometry(X, xi):
    X = _c(X); xi = _c(xi)
    J = np.zeros((3, 3)); K = np.zeros((3, 3)); x = np.zeros(3); det = np.zeros(1)
    lib().oracle_tet_geometry(_p(X), _p(xi), _p(J), _p(det), _p(K), _p(x))
    return J, float(det[0]), K, x


def integrate_tet(p, coords, D, beta, c, f, n1=0, want_xq=False):
    """Tetrahedra (coords [ne,4,3]): A [ne,n,n], b [ne,n], flags (and xq)."""
    coords = _c(coords); D = _c(D); beta = _c(beta); c = _c(c); f = _c(f)
    ne, n = coords.shape[0], tet_nshp(p)
    nqq = (n1 if n1 > 0 else p + 2) ** 3
    A = np.zeros((ne, n, n)); b = np.zeros((ne, n))
    flags = np.zeros(ne, dtype=np.int32)
    xq = np.zeros((ne, nqq, 3)) if want_xq else None
    rc = lib().oracle_integrate_tet(p, n1, ne, _p(coords), _p(D), _p(beta), _p(c), _p(f),
                                    _p(A), _p(b), _p(xq), flags.ctypes.data_as(_ip))
    assert rc == 0, rc
    return (A, b, flags, xq) if want_xq else (A, b, flags)


def set_threads(nt: int):
    lib().oracle_set_threads(int(nt))


def max_threads() -> int:
    return int(lib().oracle_max_threads())
