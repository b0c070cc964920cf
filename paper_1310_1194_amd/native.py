"""ctypes declarations of libfeint's C interface (include/feint.h).

Loading fails loudly when the library has not been built: there is no
fallback implementation anywhere in the product path.
"""
from __future__ import annotations

import ctypes
from pathlib import Path

LIB_PATH = Path(__file__).resolve().parent / "libfeint.so"

FORMS = {"fp64": 0, "fp32": 1, "bf16x3": 2, "fp16x3": 3}
# quadrature rules: (p+1)^3 collapsed Gauss; symmetric triangle rule of degree 2p x (p+1) Gauss in zeta
RULES = {"collapsed": 0, "symmetric": 1}
STATUS = {0: "ok", -1: "invalid argument", -2: "unsupported degree", -3: "unsupported form",
          -4: "tables not prepared (stream is capturing)", -5: "HIP runtime error",
          -6: "batch too large for one launch"}

# every symbol include/feint.h declares
EXPORTS = (
    "feint_nshp", "feint_nq", "feint_elem_size", "feint_prepare", "feint_integrate", "feint_integrate_fields",
    "feint_integrate_adjoint", "feint_adjoint_tile_count", "feint_adjoint_tile_get", "feint_adjoint_tile_set",
    "feint_adjoint_tile_describe", "feint_adjoint_autotune", "feint_mixed_plan_create", "feint_mixed_bucket",
    "feint_integrate_mixed", "feint_mixed_graph_capture", "feint_mixed_graph_launch",
    "feint_mixed_plan_destroy", "feint_mixed_autotune", "feint_mixed_tile_count", "feint_mixed_tile_get",
    "feint_mixed_tile_set", "feint_mixed_tile_describe", "feint_tile_count", "feint_tile_get", "feint_tile_set",
    "feint_tile_describe", "feint_autotune", "feint_status_string", "feint_last_error",
    "feint_shutdown", "feint_asm_plan_create", "feint_asm_plan_info", "feint_asm_plan_pattern",
    "feint_asm_plan_colors", "feint_assemble", "feint_asm_plan_destroy", "feint_nq_rule", "feint_rule_points",
    "feint_prepare_rule", "feint_integrate_rule", "feint_rule_tile_count", "feint_rule_tile_get",
    "feint_rule_tile_set", "feint_rule_tile_describe", "feint_autotune_rule", "feint_hex_nshp", "feint_hex_nq",
    "feint_prepare_hex", "feint_integrate_hex", "feint_hex_tile_count", "feint_hex_tile_get", "feint_hex_tile_set",
    "feint_hex_tile_describe", "feint_hex_autotune", "feint_tet_nshp", "feint_tet_nq", "feint_prepare_tet",
    "feint_integrate_tet", "feint_tet_tile_count", "feint_tet_tile_get", "feint_tet_tile_set",
    "feint_tet_tile_describe", "feint_tet_autotune", "feint_integrate_adjoint_rule",
    "feint_integrate_mixed_noalloc", "feint_integrate_laplace", "feint_laplace_tile_count",
    "feint_laplace_tile_get", "feint_laplace_tile_set", "feint_laplace_tile_describe", "feint_laplace_autotune",
)


class FeintError(RuntimeError):
    def __init__(self, fn: str, code: int, detail: str = ""):
        msg = f"{fn} failed: {STATUS.get(code, code)}"
        if detail:
            msg += f" ({detail})"
        super().__init__(msg)
        self.code = code


class Elements(ctypes.Structure):
    _fields_ = [("coords", ctypes.c_void_p), ("D", ctypes.c_void_p), ("beta", ctypes.c_void_p),
                ("c", ctypes.c_void_p), ("f", ctypes.c_void_p), ("ne", ctypes.c_int64)]


class Fields(ctypes.Structure):
    """feint_fields: the same layout, coefficients per vertex."""
    _fields_ = [("coords", ctypes.c_void_p), ("D", ctypes.c_void_p), ("beta", ctypes.c_void_p),
                ("c", ctypes.c_void_p), ("f", ctypes.c_void_p), ("ne", ctypes.c_int64)]


_vp = ctypes.c_void_p
_i = ctypes.c_int
_i64 = ctypes.c_int64

_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1310_1194_amd.build` (or __graft_entry__.build())")
        L = ctypes.CDLL(str(LIB_PATH))
        P = ctypes.POINTER(Elements)
        sig = {
            "feint_nshp": (_i, [_i]),
            "feint_nq": (_i, [_i]),
            "feint_elem_size": (ctypes.c_size_t, [_i]),
            "feint_prepare": (_i, [_i]),
            "feint_integrate": (_i, [P, _i, _i, _vp, _vp, _vp, _vp, _vp]),
            "feint_integrate_fields": (_i, [ctypes.POINTER(Fields), _i, _i, _vp, _vp, _vp, _vp, _vp]),
            "feint_integrate_adjoint": (_i, [P, _i, _i, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
            "feint_adjoint_tile_count": (_i, [_i, _i]),
            "feint_adjoint_tile_get": (_i, [_i, _i]),
            "feint_adjoint_tile_set": (_i, [_i, _i, _i]),
            "feint_adjoint_tile_describe": (_i, [_i, _i, _i, ctypes.c_char_p, ctypes.c_size_t]),
            "feint_adjoint_autotune": (_i, [P, _i, _i, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i,
                                            ctypes.POINTER(ctypes.c_double), _vp]),
            "feint_mixed_plan_create": (_i, [_i64, _i, ctypes.POINTER(_vp)]),
            "feint_mixed_bucket": (_i, [_vp, _vp, _i64, _vp, _vp, _vp, _vp]),
            "feint_integrate_mixed": (_i, [_vp, P, _vp, _vp, _vp, _vp, _vp, _vp]),
            "feint_mixed_graph_capture": (_i, [_vp, P, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
            "feint_mixed_graph_launch": (_i, [_vp, _vp]),
            "feint_integrate_mixed_noalloc": (_i, [P, _vp, _i, _vp, _vp, _vp, _vp, _vp, _vp]),
            "feint_mixed_plan_destroy": (None, [_vp]),
            "feint_mixed_autotune": (_i, [_vp, P, _vp, _vp, _vp, _vp, _i, ctypes.POINTER(ctypes.c_double), _vp]),
            "feint_mixed_tile_count": (_i, [_vp]),
            "feint_mixed_tile_get": (_i, [_vp]),
            "feint_mixed_tile_set": (_i, [_vp, _i]),
            "feint_mixed_tile_describe": (_i, [_vp, _i, ctypes.c_char_p, ctypes.c_size_t]),
            "feint_tile_count": (_i, [_i, _i]),
            "feint_tile_get": (_i, [_i, _i]),
            "feint_tile_set": (_i, [_i, _i, _i]),
            "feint_tile_describe": (_i, [_i, _i, _i, ctypes.c_char_p, ctypes.c_size_t]),
            "feint_autotune": (_i, [P, _i, _i, _vp, _vp, _i, ctypes.POINTER(ctypes.c_double), _vp]),
            "feint_status_string": (ctypes.c_char_p, [_i]),
            "feint_last_error": (ctypes.c_char_p, []),
            "feint_shutdown": (None, []),
            "feint_asm_plan_create": (_i, [_vp, _i64, _i, _i64, ctypes.POINTER(_vp)]),
            "feint_asm_plan_info": (_i, [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i)]),
            "feint_asm_plan_pattern": (_i, [_vp, _vp, _vp, _vp]),
            "feint_asm_plan_colors": (_i, [_vp, _vp]),
            "feint_assemble": (_i, [_vp, _i, _vp, _vp, _vp, _vp, _i, _vp]),
            "feint_asm_plan_destroy": (None, [_vp]),
            "feint_nq_rule": (_i, [_i, _i]),
            "feint_rule_points": (_i, [_i, _i, _vp, _i64]),
            "feint_prepare_rule": (_i, [_i, _i]),
            "feint_integrate_rule": (_i, [P, ctypes.POINTER(Fields), _i, _i, _i, _vp, _vp, _vp, _vp, _vp]),
            "feint_rule_tile_count": (_i, [_i, _i, _i]),
            "feint_rule_tile_get": (_i, [_i, _i, _i]),
            "feint_rule_tile_set": (_i, [_i, _i, _i, _i]),
            "feint_rule_tile_describe": (_i, [_i, _i, _i, _i, ctypes.c_char_p, ctypes.c_size_t]),
            "feint_autotune_rule": (_i, [P, ctypes.POINTER(Fields), _i, _i, _i, _vp, _vp, _i,
                                         ctypes.POINTER(ctypes.c_double), _vp]),
            "feint_hex_nshp": (_i, [_i]),
            "feint_hex_nq": (_i, [_i]),
            "feint_prepare_hex": (_i, [_i]),
            "feint_integrate_hex": (_i, [P, _i, _i, _vp, _vp, _vp, _vp, _vp]),
            "feint_hex_tile_count": (_i, [_i, _i]),
            "feint_hex_tile_get": (_i, [_i, _i]),
            "feint_hex_tile_set": (_i, [_i, _i, _i]),
            "feint_hex_tile_describe": (_i, [_i, _i, _i, ctypes.c_char_p, ctypes.c_size_t]),
            "feint_hex_autotune": (_i, [P, _i, _i, _vp, _vp, _i, ctypes.POINTER(ctypes.c_double), _vp]),
            "feint_integrate_adjoint_rule": (_i, [P, _i, _i, _i, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
            "feint_tet_nshp": (_i, [_i]),
            "feint_tet_nq": (_i, [_i]),
            "feint_prepare_tet": (_i, [_i]),
            "feint_integrate_tet": (_i, [P, _i, _i, _vp, _vp, _vp, _vp, _vp]),
            "feint_tet_tile_count": (_i, [_i, _i]),
            "feint_tet_tile_get": (_i, [_i, _i]),
            "feint_tet_tile_set": (_i, [_i, _i, _i]),
            "feint_tet_tile_describe": (_i, [_i, _i, _i, ctypes.c_char_p, ctypes.c_size_t]),
            "feint_tet_autotune": (_i, [P, _i, _i, _vp, _vp, _i, ctypes.POINTER(ctypes.c_double), _vp]),
            "feint_integrate_laplace": (_i, [_vp, _i64, _i, _i, _vp, _vp, _vp, _vp]),
            "feint_laplace_tile_count": (_i, [_i, _i]),
            "feint_laplace_tile_get": (_i, [_i, _i]),
            "feint_laplace_tile_set": (_i, [_i, _i, _i]),
            "feint_laplace_tile_describe": (_i, [_i, _i, _i, ctypes.c_char_p, ctypes.c_size_t]),
            "feint_laplace_autotune": (_i, [_vp, _i64, _i, _i, _vp, _i, ctypes.POINTER(ctypes.c_double), _vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(fn: str, code: int) -> None:
    if code != 0:
        detail = lib().feint_last_error().decode() if code == -5 else ""
        raise FeintError(fn, code, detail)
