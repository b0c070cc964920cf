"""MI355X-native element-by-element numerical integration for higher-order
prismatic finite elements (Krużel & Banaś, arXiv 1310.1194), generalised to
convection-diffusion-reaction with a load vector, an adjoint, mixed-degree
batches, spatially varying coefficients, the paper's symmetric quadrature
rule, shape functions computed per point, hexahedral and tetrahedral
elements and global assembly.  Kernels:
hand-written HIP for gfx950 in libfeint.so."""
from .api import (ELEMENTS, AsmPlan, IntegrateFn, MixedPlan, adjoint_autotune, adjoint_raw, adjoint_tile_count,
                  adjoint_tile_describe, adjoint_tile_get, adjoint_tile_set, autotune, autotune_fields, elem_autotune,
                  elem_tile_count, elem_tile_describe, elem_tile_get, elem_tile_set, hex_autotune, hex_nshp,
                  hex_tile_count, hex_tile_describe, hex_tile_get, hex_tile_set, integrate, integrate_elem_raw,
                  integrate_fields_raw, integrate_hex_raw, integrate_laplace_raw, integrate_mixed_noalloc,
                  integrate_raw, laplace_autotune, laplace_tile_count, laplace_tile_describe, laplace_tile_get,
                  laplace_tile_set, integrate_tet_raw, nq, nshp, prepare,
                  rule_points, tet_nshp, tile_count, tile_describe, tile_get, tile_set)
from .native import FORMS, RULES, FeintError

__all__ = ["integrate", "MixedPlan", "AsmPlan", "integrate_raw", "integrate_fields_raw", "adjoint_raw",
           "IntegrateFn", "prepare", "nshp", "nq", "autotune", "tile_count", "tile_get", "tile_set",
           "tile_describe", "adjoint_autotune", "adjoint_tile_count", "adjoint_tile_get", "adjoint_tile_set",
           "adjoint_tile_describe", "FORMS", "RULES", "FeintError", "rule_points", "autotune_fields",
           "integrate_hex_raw", "hex_nshp", "hex_tile_count", "hex_tile_get", "hex_tile_set", "hex_tile_describe",
           "hex_autotune", "integrate_tet_raw", "tet_nshp", "integrate_elem_raw", "elem_tile_count",
           "elem_tile_get", "elem_tile_set", "elem_tile_describe", "elem_autotune", "ELEMENTS",
           "integrate_mixed_noalloc", "integrate_laplace_raw", "laplace_autotune", "laplace_tile_count",
           "laplace_tile_describe", "laplace_tile_get", "laplace_tile_set"]
