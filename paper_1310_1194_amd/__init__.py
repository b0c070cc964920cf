"""MI355X-native element-by-element numerical integration for higher-order
prismatic finite elements (Krużel & Banaś, arXiv 1310.1194), generalised to
convection-diffusion-reaction with a load vector, an adjoint, mixed-degree
batches, spatially varying coefficients and global assembly.  Kernels:
hand-written HIP for gfx950 in libfeint.so."""
from .api import (AsmPlan, IntegrateFn, MixedPlan, adjoint_autotune, adjoint_raw, adjoint_tile_count,
                  adjoint_tile_describe, adjoint_tile_get, adjoint_tile_set, autotune, integrate,
                  integrate_fields_raw, integrate_raw, nq, nshp, prepare, tile_count, tile_describe, tile_get,
                  tile_set)
from .native import FORMS, FeintError

__all__ = ["integrate", "MixedPlan", "AsmPlan", "integrate_raw", "integrate_fields_raw", "adjoint_raw",
           "IntegrateFn", "prepare", "nshp", "nq", "autotune", "tile_count", "tile_get", "tile_set",
           "tile_describe", "adjoint_autotune", "adjoint_tile_count", "adjoint_tile_get", "adjoint_tile_set",
           "adjoint_tile_describe", "FORMS", "FeintError"]
