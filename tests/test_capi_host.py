"""CPU tests of the C-ABI library: it loads, exports every declared symbol, and
rejects bad arguments on the host before any device work."""
import ctypes
import re
from pathlib import Path

import pytest

from paper_1310_1194_amd import native

ROOT = Path(__file__).resolve().parent.parent


def declared_symbols():
    hdr = (ROOT / "include" / "feint.h").read_text()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    return sorted(set(re.findall(r"\b(feint_[a-z0-9_]+)\s*\(", hdr)))


def test_header_and_binding_agree():
    assert declared_symbols() == sorted(native.EXPORTS)


def test_library_exports_every_symbol():
    L = native.lib()
    for name in declared_symbols():
        assert hasattr(L, name), name


def test_counts():
    L = native.lib()
    assert [L.feint_nshp(p) for p in range(0, 9)] == [-1, 6, 18, 40, 75, 126, 196, 288, -1]
    assert [L.feint_nq(p) for p in range(1, 8)] == [(p + 1) ** 3 for p in range(1, 8)]
    assert L.feint_elem_size(0) == 8 and L.feint_elem_size(2) == 4 and L.feint_elem_size(9) == 0


def _el(ne, null=False):
    v = 0 if null else 0x1000
    return native.Elements(v, v, v, v, v, ne)


def test_host_validation_before_device_work():
    L = native.lib()
    el = _el(4)
    A = ctypes.c_void_p(0x2000)
    s = ctypes.c_void_p(0)
    assert L.feint_integrate(None, 2, 0, A, A, None, None, s) == -1
    assert L.feint_integrate(ctypes.byref(el), 0, 0, A, A, None, None, s) == -2
    assert L.feint_integrate(ctypes.byref(el), 8, 0, A, A, None, None, s) == -2
    assert L.feint_integrate(ctypes.byref(el), 2, 7, A, A, None, None, s) == -3
    assert L.feint_integrate(ctypes.byref(_el(-1)), 2, 0, A, A, None, None, s) == -1
    assert L.feint_integrate(ctypes.byref(_el(4, null=True)), 2, 0, A, A, None, None, s) == -1
    assert L.feint_integrate(ctypes.byref(el), 2, 0, None, A, None, None, s) == -1
    assert L.feint_integrate(ctypes.byref(_el(0, null=True)), 2, 0, None, None, None, None, s) == 0
    G = ctypes.c_void_p(0x3000)
    assert L.feint_integrate_adjoint(ctypes.byref(el), 2, 2, G, G, G, G, G, G, G, s) == -3
    assert L.feint_integrate_adjoint(ctypes.byref(el), 9, 0, G, G, G, G, G, G, G, s) == -2


def test_tiles():
    L = native.lib()
    for p in range(1, 8):
        for form in range(4):
            n = L.feint_tile_count(p, form)
            assert n >= 1
            buf = ctypes.create_string_buffer(16)
            assert L.feint_tile_describe(p, form, n - 1, buf, 16) == 0
            assert re.fullmatch(rb"(\d+x\d+(s|sa|p|c|f|fw|fwg|fz)?|v\d+)(o\d)?", buf.value)
            assert L.feint_tile_set(p, form, n) == -1
    assert L.feint_tile_count(0, 0) == 0


def test_adjoint_tiles():
    L = native.lib()
    buf = ctypes.create_string_buffer(16)
    for p in range(1, 8):
        for form in (0, 1):
            n = L.feint_adjoint_tile_count(p, form)
            assert n >= 1
            assert L.feint_adjoint_tile_get(p, form) == 0
            for t in range(n):
                assert L.feint_adjoint_tile_describe(p, form, t, buf, 16) == 0
                assert re.fullmatch(rb"\d+x\d+(f|fo2|fw|fwo2)?", buf.value)
            assert L.feint_adjoint_tile_set(p, form, n) == -1
            assert L.feint_adjoint_tile_describe(p, form, n, buf, 16) == -1
        for form in (2, 3):          # split forms have no adjoint
            assert L.feint_adjoint_tile_count(p, form) == 0
            assert L.feint_adjoint_tile_get(p, form) == -1
            assert L.feint_adjoint_tile_set(p, form, 0) == -3
    assert L.feint_adjoint_tile_count(0, 0) == 0
    assert L.feint_adjoint_tile_set(8, 0, 0) == -2
    # autotune validates before touching the device
    assert L.feint_adjoint_autotune(None, 3, 0, None, None, None, None, None, None, None, 1, None, None) == -1


def test_status_strings():
    L = native.lib()
    for code in native.STATUS:
        assert L.feint_status_string(code).decode() == native.STATUS[code]


def test_assembly_plan_validation():
    """Host-detectable errors of the assembly plan come back before any device work."""
    L = native.lib()
    import numpy as np
    h = ctypes.c_void_p()
    d = np.zeros((2, 6), dtype=np.int32)
    d[0] = np.arange(6); d[1] = np.arange(3, 9)
    ptr = d.ctypes.data_as(ctypes.c_void_p)
    assert L.feint_asm_plan_create(None, 2, 6, 9, ctypes.byref(h)) == -1
    assert L.feint_asm_plan_create(ptr, 0, 6, 9, ctypes.byref(h)) == -1
    assert L.feint_asm_plan_create(ptr, 2, 7, 9, ctypes.byref(h)) == -1        # no prism has 7 shape functions
    assert L.feint_asm_plan_create(ptr, 2, 6, 8, ctypes.byref(h)) == -1        # dof 8 out of range
    d[1, 0] = d[1, 1]
    assert L.feint_asm_plan_create(ptr, 2, 6, 9, ctypes.byref(h)) == -1        # dof repeated in an element
    assert L.feint_asm_plan_create(ptr, 2, 6, 9, None) == -1
    assert L.feint_asm_plan_info(None, None, None) == -1
    assert L.feint_assemble(None, 0, None, None, None, None, 0, None) == -1


def test_fields_validation():
    L = native.lib()
    fl = native.Fields(0, 0, 0, 0, 0, 4)
    assert L.feint_integrate_fields(ctypes.byref(fl), 3, 0, None, None, None, None, None) == -1   # null inputs
    assert L.feint_integrate_fields(ctypes.byref(fl), 9, 0, None, None, None, None, None) == -2   # degree
    assert L.feint_integrate_fields(ctypes.byref(fl), 3, 7, None, None, None, None, None) == -3   # form
    assert L.feint_integrate_fields(None, 3, 0, None, None, None, None, None) == -1
    empty = native.Fields(0, 0, 0, 0, 0, 0)
    assert L.feint_integrate_fields(ctypes.byref(empty), 3, 0, None, None, None, None, None) == 0


def test_rule_counts_and_points():
    """The library's symmetric rule (host copy, no device work): the paper's
    point counts (Table 3 / 4 scalars per point), exact monomial integrals up
    to degree 2p on the triangle and 2p+1 in zeta, and agreement with the
    oracle's independently solved rule."""
    from fractions import Fraction
    from math import factorial

    import numpy as np

    import oracle
    import paper_1310_1194_amd as F
    L = native.lib()
    assert [L.feint_nq_rule(p, 1) for p in range(1, 8)] == [6, 18, 48, 80, 150, 231, 336]
    assert [L.feint_nq_rule(p, 0) for p in range(1, 8)] == [(p + 1) ** 3 for p in range(1, 8)]
    assert L.feint_nq_rule(0, 1) == -1 and L.feint_nq_rule(3, 2) == -1
    for p in range(1, 8):
        q = F.rule_points(p, "symmetric")
        assert (q[:, 3] > 0).all() and (q[:, :2] > 0).all() and (q[:, 0] + q[:, 1] < 1).all()
        for i in range(2 * p + 1):
            for j in range(2 * p + 1 - i):
                for g in (0, 2 * p, 2 * p + 1):
                    ex = Fraction(factorial(i) * factorial(j), factorial(i + j + 2)) * \
                        (Fraction(0) if g % 2 else Fraction(2, g + 1))
                    got = np.sum(q[:, 3] * q[:, 0] ** i * q[:, 1] ** j * q[:, 2] ** g)
                    assert abs(got - float(ex)) < 1e-15, (p, i, j, g)
        pts, w = oracle.prism_rule(p, "symmetric")
        assert np.abs(q[:, :3] - pts).max() < 1e-15 and np.abs(q[:, 3] - w).max() < 1e-16
    buf = np.zeros((5, 4))
    assert L.feint_rule_points(1, 1, buf.ctypes.data_as(ctypes.c_void_p), 5) == -1    # too small
    assert L.feint_rule_points(1, 3, buf.ctypes.data_as(ctypes.c_void_p), 5) == -1    # unknown rule
    assert L.feint_rule_points(8, 1, buf.ctypes.data_as(ctypes.c_void_p), 5) == -2


def test_rule_tiles_and_validation():
    L = native.lib()
    buf = ctypes.create_string_buffer(32)
    pat = re.compile(r"(\d+x\d+(s|sa|p|c|f|fw|fwg|fz)?|v\d+)(o\d)?")
    for form in range(4):
        for p in range(1, 8):
            n = L.feint_rule_tile_count(p, form, 1)
            assert n >= 1
            assert L.feint_rule_tile_count(p, form, 0) == L.feint_tile_count(p, form)
            for t in range(n):
                assert L.feint_rule_tile_describe(p, form, 1, t, buf, 32) == 0
                assert pat.fullmatch(buf.value.decode()), buf.value
            assert L.feint_rule_tile_describe(p, form, 1, n, buf, 32) == -1
            assert L.feint_rule_tile_set(p, form, 1, n) == -1
    assert L.feint_rule_tile_count(3, 0, 5) == 0 and L.feint_rule_tile_get(3, 0, 5) == -1
    el = _el(4)
    fl = native.Fields(0x1000, 0x1000, 0x1000, 0x1000, 0x1000, 4)
    A = ctypes.c_void_p(0x2000)
    s = ctypes.c_void_p(0)
    # exactly one of el and fl
    assert L.feint_integrate_rule(None, None, 3, 0, 1, A, A, None, None, s) == -1
    assert L.feint_integrate_rule(ctypes.byref(el), ctypes.byref(fl), 3, 0, 1, A, A, None, None, s) == -1
    assert L.feint_integrate_rule(ctypes.byref(el), None, 3, 0, 4, A, A, None, None, s) == -1     # rule
    assert L.feint_integrate_rule(ctypes.byref(el), None, 9, 0, 1, A, A, None, None, s) == -2
    assert L.feint_integrate_rule(ctypes.byref(el), None, 3, 6, 1, A, A, None, None, s) == -3
    assert L.feint_integrate_rule(ctypes.byref(_el(4, null=True)), None, 3, 0, 1, A, A, None, None, s) == -1
    assert L.feint_integrate_rule(ctypes.byref(_el(0, null=True)), None, 3, 0, 1, None, None, None, None, s) == 0
    assert L.feint_autotune_rule(None, None, 3, 0, 1, A, A, 1, None, s) == -1
    assert L.feint_autotune_rule(ctypes.byref(_el(0, null=True)), None, 3, 0, 1, A, A, 1, None, s) == -1


def test_hex_host_api():
    L = native.lib()
    assert [L.feint_hex_nshp(p) for p in range(0, 9)] == [-1, 8, 27, 64, 125, 216, 343, 512, -1]
    assert [L.feint_hex_nq(p) for p in range(1, 8)] == [(p + 1) ** 3 for p in range(1, 8)]
    buf = ctypes.create_string_buffer(32)
    for p in range(1, 8):
        for form in (0, 1):
            n = L.feint_hex_tile_count(p, form)
            assert n >= 1
            for t in range(n):
                assert L.feint_hex_tile_describe(p, form, t, buf, 32) == 0
                assert re.fullmatch(rb"(\d+x\d+f?|v\d+)(o\d)?|sf\d+w(x\d+)?[rl]?(o\d)?", buf.value), buf.value
            # FP64 and FP32 start with the sum factorisation in all three directions
            assert L.feint_hex_tile_describe(p, form, 0, buf, 32) == 0 and buf.value.startswith(b"sf")
        for form in (2, 3):                          # split forms
            assert L.feint_hex_tile_count(p, form) >= 1
    el = _el(4)
    A = ctypes.c_void_p(0x2000)
    s = ctypes.c_void_p(0)
    assert L.feint_integrate_hex(ctypes.byref(el), 3, 7, A, A, None, None, s) == -3
    assert L.feint_integrate_hex(ctypes.byref(el), 8, 0, A, A, None, None, s) == -2
    assert L.feint_integrate_hex(None, 3, 0, A, A, None, None, s) == -1
    assert L.feint_integrate_hex(ctypes.byref(_el(4, null=True)), 3, 0, A, A, None, None, s) == -1
    assert L.feint_integrate_hex(ctypes.byref(el), 3, 0, None, A, None, None, s) == -1
    assert L.feint_integrate_hex(ctypes.byref(_el(0, null=True)), 3, 0, None, None, None, None, s) == 0
    assert L.feint_hex_tile_set(3, 0, 99) == -1 and L.feint_hex_tile_set(3, 5, 0) == -3
    assert L.feint_hex_autotune(ctypes.byref(_el(0, null=True)), 3, 0, A, A, 1, None, s) == -1


def test_tet_host_api():
    L = native.lib()
    assert [L.feint_tet_nshp(p) for p in range(0, 9)] == [-1, 4, 10, 20, 35, 56, 84, 120, -1]
    assert [L.feint_tet_nq(p) for p in range(1, 8)] == [(p + 2) ** 3 for p in range(1, 8)]
    buf = ctypes.create_string_buffer(32)
    for p in range(1, 8):
        for form in (0, 1):
            n = L.feint_tet_tile_count(p, form)
            assert n >= 1
            for t in range(n):
                assert L.feint_tet_tile_describe(p, form, t, buf, 32) == 0
                assert re.fullmatch(rb"(\d+x\d+f?|v\d+|ref[124]s?(e\d+)?)(o\d)?", buf.value), buf.value
            # FP64 and FP32 start with the reference-matrix kernel (affine elements)
            assert L.feint_tet_tile_describe(p, form, 0, buf, 32) == 0 and buf.value.startswith(b"ref")
        for form in (2, 3):
            assert L.feint_tet_tile_count(p, form) >= 1
    el = _el(4)
    A = ctypes.c_void_p(0x2000)
    s = ctypes.c_void_p(0)
    assert L.feint_integrate_tet(ctypes.byref(el), 3, 4, A, A, None, None, s) == -3
    assert L.feint_integrate_tet(ctypes.byref(el), 0, 0, A, A, None, None, s) == -2
    assert L.feint_integrate_tet(None, 3, 0, A, A, None, None, s) == -1
    assert L.feint_integrate_tet(ctypes.byref(_el(0, null=True)), 3, 0, None, None, None, None, s) == 0
    assert L.feint_tet_tile_set(3, 1, 99) == -1


def test_laplace_host_api():
    """The Laplace-only entry points: FP64 and FP32 variants at every degree, the
    split forms refused, and every host-side error before any launch."""
    L = native.lib()
    buf = ctypes.create_string_buffer(32)
    for p in range(1, 8):
        for form in (0, 1):
            n = L.feint_laplace_tile_count(p, form)
            assert n >= 1 and L.feint_laplace_tile_get(p, form) == 0
            for t in range(n):
                assert L.feint_laplace_tile_describe(p, form, t, buf, 32) == 0
                assert re.fullmatch(rb"(\d+x\d+f[wz]?|v\d+)(o\d)?", buf.value), buf.value
        for form in (2, 3):
            assert L.feint_laplace_tile_count(p, form) == 0 and L.feint_laplace_tile_get(p, form) == -1
    X = ctypes.c_void_p(0x1000)
    A = ctypes.c_void_p(0x2000)
    s = ctypes.c_void_p(0)
    assert L.feint_integrate_laplace(X, 4, 3, 2, A, None, None, s) == -3
    assert L.feint_integrate_laplace(X, 4, 8, 0, A, None, None, s) == -2
    assert L.feint_integrate_laplace(X, -1, 3, 0, A, None, None, s) == -1
    assert L.feint_integrate_laplace(None, 4, 3, 0, A, None, None, s) == -1
    assert L.feint_integrate_laplace(X, 4, 3, 1, None, None, None, s) == -1
    assert L.feint_integrate_laplace(None, 0, 3, 0, None, None, None, s) == 0
    assert L.feint_laplace_tile_set(3, 0, 99) == -1 and L.feint_laplace_tile_set(3, 2, 0) == -3
    assert L.feint_laplace_tile_set(0, 0, 0) == -2
    assert L.feint_laplace_autotune(X, 0, 3, 0, A, 1, None, s) == -1
    assert L.feint_laplace_autotune(X, 4, 3, 0, A, 0, None, s) == -1
