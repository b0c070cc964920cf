"""Sizes, work and traffic of per-element integration on prisms.

Two counting conventions live here:

* the paper's own (Sec. 2.2 "Computational and memory complexity", Tables 1-3):
  N_sh shape functions, N_I points of its symmetric triangle rule of degree
  2p times p+1 line points, 7 operations per matrix entry per point (Laplace
  term), 220 per point for the Jacobian, and 3(p+1)(p+2)/2 + 6(p+1) + 19 N_sh
  for the shape functions at one point;
* this library's: the convection-diffusion-reaction contraction
  A_e = sum_q B_q^T W_q B_q costs 4 FMAs = 8 flops per entry per point on the
  (p+1)^3-point collapsed rule, so F_dom = 8 n^2 nq per element.
"""
from __future__ import annotations

# Points of the symmetric triangle rule of degree 2p that the paper's point
# counts imply (Table 3 "xi, w" row / 4 / (p+1)).
PAPER_TRIANGLE_POINTS = {1: 3, 2: 6, 3: 12, 4: 16, 5: 25, 6: 33, 7: 42}


def nshp(p: int) -> int:
    return (p + 1) * (p + 1) * (p + 2) // 2


def ntri(p: int) -> int:
    return (p + 1) * (p + 2) // 2


def nq(p: int, rule: str = "collapsed") -> int:
    """Points of the collapsed Gauss rule ((p+1)^3) or of the symmetric rule
    (the paper's N_I)."""
    return (p + 1) ** 3 if rule == "collapsed" else paper_nI(p)


def paper_nI(p: int) -> int:
    return PAPER_TRIANGLE_POINTS[p] * (p + 1)


def paper_shape_ops_per_point(p: int) -> int:
    return 3 * (p + 1) * (p + 2) // 2 + 6 * (p + 1) + 19 * nshp(p)


PAPER_JACOBIAN_OPS = 220


def paper_matrix_ops_per_point(p: int) -> int:
    return 7 * nshp(p) ** 2


def paper_total_ops(p: int) -> int:
    return paper_nI(p) * (paper_shape_ops_per_point(p) + PAPER_JACOBIAN_OPS
                          + paper_matrix_ops_per_point(p))


def laplace_paper_ops_per_point(p: int) -> int:
    """Work of the Laplace kernel (the paper's term on its rule) at one point,
    counted the paper's way: shape functions, Jacobian, 7 per matrix entry."""
    return paper_shape_ops_per_point(p) + PAPER_JACOBIAN_OPS + paper_matrix_ops_per_point(p)


def laplace_paper_ops(p: int, points: int) -> int:
    """The Laplace kernel's work per element in the paper's convention, for a
    rule of `points` points (the kernel's rule has the paper's N_I)."""
    return points * laplace_paper_ops_per_point(p)


def f_dom(p: int, rule: str = "collapsed") -> int:
    """Algorithmic flops of the contraction per element: 8 n^2 nq."""
    return 8 * nshp(p) ** 2 * nq(p, rule)


def f_factored(n: int, nk: int, nq_: int) -> int:
    """Flops per element of the contraction factorised along the third
    coordinate (the rule is nij plane points times nk line points, the basis
    n = nk * nt plane factors times line factors): the GEMM over (plane point,
    derivative row), 8 n^2 nij; forming Z_k from the nk line points,
    8 nk^2 nij n; forming Y from the point blocks and the factors,
    24 nq nt + 12 nq n."""
    nij, nt = nq_ // nk, n // nk
    return 8 * n * n * nij + 8 * nk * nk * nij * n + 24 * nq_ * nt + 12 * nq_ * n


def f_factored_zfirst(n: int, nk: int, nq_: int) -> int:
    """Flops per element of the factorised contraction with the line-point
    sums taken first: the GEMM over (plane point, derivative row), 8 n^2 nij;
    per (plane point, k, k') the 13 nonzero entries of
    G[r][s] = sum_m lam_r(k, m) lam_s(k', m) W_m[r][s], 26 nk^3 nij; and each of
    the 4 nk n nij Z values as four products with the plane factors,
    32 nk n nij."""
    nij = nq_ // nk
    return 8 * n * n * nij + 26 * nk ** 3 * nij + 32 * nk * n * nij


def is_zfirst_tile(desc: str) -> bool:
    """Tiles "KxTNfz" (FP64, FP32) and "KxTNfwg" (split), optionally "o" and
    the waves per SIMD, take the line-point sums first."""
    import re
    return re.fullmatch(r"\d+x\d+f(z|wg)(o\d)?", desc) is not None


def f_kf(p: int, rule: str = "collapsed") -> int:
    """f_factored for prisms: ntri triangle functions times p+1 line functions."""
    return f_factored(nshp(p), p + 1, nq(p, rule))


def kf_mfma_flops(p: int, rule: str = "collapsed", n: int = 0, nq_: int = 0) -> int:
    """Hardware MFMA flops per element of the factorised contraction: one
    16x16x4 product per (row block, column block) pair of 16-padded plane
    tiles and line indices, per plane point (prisms by default; n and nq_
    give another element's shape-function and point counts)."""
    nk = p + 1
    n, nq_ = n or nshp(p), nq_ or nq(p, rule)
    tt = -(-(n // nk) // 16)
    return 2 * 16 * 16 * 4 * (nq_ // nk) * (nk * tt) ** 2


def f_adjoint_factored(p: int, rule: str = "collapsed") -> int:
    """Flops per element of the adjoint factorised along zeta: H_k = G^T tau
    (8 n^2 nij), Hh = sum_k lam H_k (8 (p+1)^2 nij n), and per point the 16
    sums over b of Hh B (32 nq n) with B's factor products (4 nq n)."""
    n, nk, q = nshp(p), p + 1, nq(p, rule)
    nij = q // nk
    return 8 * n * n * nij + 8 * nk * nk * nij * n + 36 * q * n


def f_hex_sumfact(p: int) -> int:
    """Flops per element of the hexahedral contraction factorised in all three
    directions (n = p+1 points and 1D factors per direction; an FMA counts 2):
    the xi1 pass, per (a1, q3, b1) and q1, 4 products of the a1 and b1 factors
    and 13 FMAs per q2 (the nonzero entries of W_q): n^4 (4 + 26 n); the xi2
    pass, per (a1, q3, b1), a2 and q2, 6 products and 3 FMAs folding the a2
    factors and 6 n FMAs with the b2 factors: n^5 (12 + 12 n); the xi3 pass, per
    (a1, a2, b2, b1) and a3, 2 n products and 2 n FMAs folding the a3 factors and
    2 n^2 FMAs with the b3 factors: n^6 (6 + 4 n); the load vector, three
    passes of n FMAs per output: 6 n^4.  Total 10 n^4 + 38 n^5 + 18 n^6 + 4 n^7."""
    n = p + 1
    return 10 * n ** 4 + 38 * n ** 5 + 18 * n ** 6 + 4 * n ** 7


def f_tet_reference(n: int) -> int:
    """Flops per element of the tetrahedral reference-matrix GEMM: the element
    matrix as a combination of 13 reference matrices (13 multiply-adds per
    entry) and the load vector as a multiple of one reference vector."""
    return 26 * n * n + n


def tet_reference_mfma_flops(n: int) -> int:
    """Issued 16x16x4 MFMA flops per element of that GEMM: K = 13 slots padded
    to 16, n^2 entries padded to a multiple of 16 (full waves of elements)."""
    return 2 * 16 * ((n * n + 15) // 16 * 16)


def is_tet_ref_tile(desc: str) -> bool:
    """Tile descriptions "refR" (optionally "s", "eE", "oK") name the tetrahedral
    reference-matrix GEMM."""
    import re
    return re.fullmatch(r"ref\d+s?(e\d+)?(o\d)?", desc) is not None


def is_sf_tile(desc: str) -> bool:
    """Tile descriptions "sfWw..." name the hexahedral sum factorisation."""
    import re
    return re.fullmatch(r"sf\d+w(x\d+)?[rl]?(o\d)?", desc) is not None


def is_kf_tile(desc: str) -> bool:
    """Tile descriptions "KxTNf", "KxTNfw", "KxTNfz" and (split forms)
    "KxTNfwg", optionally "o" and the waves per SIMD, name the triangle-point
    contraction."""
    import re
    return re.fullmatch(r"\d+x\d+f(wg?|z)?(o\d)?", desc) is not None


def f_kernel(p: int, rule: str, desc: str) -> int:
    """Algorithmic flops per element of the algorithm the tile runs."""
    return f_kf(p, rule) if is_kf_tile(desc) else f_dom(p, rule)


def f_full(p: int) -> int:
    """F_dom + load vector and gradient transform (28 n nq) + geometry (220 nq)."""
    n, q = nshp(p), nq(p)
    return f_dom(p) + 28 * n * q + 220 * q


INPUT_BYTES = 8 * (18 + 9 + 3 + 1 + 1)   # coords, D, beta, c, f in FP64 = 256


def out_bytes(p: int, elem_size: int) -> int:
    n = nshp(p)
    return (n * n + n) * elem_size


def bytes_per_element(p: int, elem_size: int) -> int:
    """Algorithmic HBM bytes of the forward pass per element."""
    return INPUT_BYTES + out_bytes(p, elem_size)


# coords + the coefficients at the six vertices (D, beta, c, f) in FP64 = 816
FIELD_INPUT_BYTES = 8 * (18 + 6 * (9 + 3 + 1 + 1))


def fields_bytes_per_element(p: int, elem_size: int) -> int:
    """Algorithmic HBM bytes of the forward pass with vertex coefficient fields."""
    return FIELD_INPUT_BYTES + out_bytes(p, elem_size)


def adjoint_bytes_per_element(p: int, elem_size: int) -> int:
    """Adjoint: read G, g (elem_size each) + the 256 B of inputs, write 32 FP64 gradients."""
    return out_bytes(p, elem_size) + INPUT_BYTES + 32 * 8
