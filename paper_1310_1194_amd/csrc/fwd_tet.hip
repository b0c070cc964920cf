// Forward kernels for tetrahedral elements (Table 1's complete-basis 3D
// element).  FP64 and FP32 start with the reference-matrix GEMM: "refR" = R
// row tiles of 16 elements per pass over the column tiles, "s" = results
// staged through LDS so that a store writes 64 consecutive entries of one
// element, "eE" = E elements per wave (64 without it).  The point-by-point
// kernels follow: the 16x16x4 MFMA kernel, below p = 3 the vector-ALU kernel
// ("vL" = L lanes per element, at p = 1 "v1" = one element per lane), and the
// 16x16x32 split kernel (bf16x3, fp16x3), all with the affine geometry; tile
// shapes per degree (n = 4, 10, 20, 35, 56, 84, 120 shape functions: 1, 1, 2,
// 3, 4, 6, 8 tiles of 16).  The first of each list is the default (the
// fastest measured at 393216 elements where measured).
#include "fwd_registry.h"

namespace feint {
namespace {
const FwdVariant d1[] = {FEINT_KT(1, double, 4, 2), FEINT_KE_G(1, double, 2, TetGeo), FEINT_KV_G(1, double, 8, 2, TetGeo), FEINT_K4U_TET(1, double, 1, 1, 2)};
const FwdVariant d2[] = {FEINT_KTS(2, double, 2), FEINT_KTE(2, double, 16, true, 2), FEINT_KT(2, double, 1, 2), FEINT_KTE(2, double, 16, false, 2), FEINT_KT(2, double, 4, 2), FEINT_KV_G(2, double, 16, 2, TetGeo), FEINT_K4U_TET(2, double, 1, 1, 2)};
const FwdVariant d3[] = {FEINT_KTE(3, double, 16, true, 2), FEINT_KTS(3, double, 2), FEINT_KT(3, double, 1, 2), FEINT_KTE(3, double, 16, false, 2), FEINT_KT(3, double, 4, 2), FEINT_K4U_TET(3, double, 2, 2, 2), FEINT_K4U_TET(3, double, 2, 1, 2),
                         FEINT_KV_G(3, double, 32, 2, TetGeo)};
const FwdVariant d4[] = {FEINT_KTE(4, double, 16, true, 2), FEINT_KTS(4, double, 2), FEINT_KT(4, double, 1, 2), FEINT_KTE(4, double, 16, false, 2), FEINT_KT(4, double, 4, 2), FEINT_K4U_TET(4, double, 3, 3, 2), FEINT_K4U_TET(4, double, 3, 1, 2)};
const FwdVariant d5[] = {FEINT_KTE(5, double, 16, true, 2), FEINT_KTS(5, double, 2), FEINT_KT(5, double, 1, 2), FEINT_KTE(5, double, 16, false, 2), FEINT_KT(5, double, 4, 2), FEINT_K4U_TET(5, double, 4, 2, 2), FEINT_K4U_TET(5, double, 4, 1, 2)};
const FwdVariant d6[] = {FEINT_KTE(6, double, 16, true, 2), FEINT_KTS(6, double, 2), FEINT_KT(6, double, 1, 2), FEINT_KTE(6, double, 16, false, 2), FEINT_KT(6, double, 4, 2), FEINT_K4U_TET(6, double, 6, 2, 1), FEINT_K4U_TET(6, double, 6, 1, 2)};
const FwdVariant d7[] = {FEINT_KTE(7, double, 16, true, 2), FEINT_KTS(7, double, 2), FEINT_KT(7, double, 1, 2), FEINT_KTE(7, double, 16, false, 2), FEINT_KT(7, double, 4, 2), FEINT_K4U_TET(7, double, 8, 2, 1), FEINT_K4U_TET(7, double, 8, 1, 2)};
const FwdVariant f1[] = {FEINT_KT(1, float, 4, 2), FEINT_KE_G(1, float, 3, TetGeo), FEINT_KE_G(1, float, 2, TetGeo), FEINT_KV_G(1, float, 8, 2, TetGeo), FEINT_K4U_TET(1, float, 1, 1, 2)};
const FwdVariant f2[] = {FEINT_KTE(2, float, 16, false, 2), FEINT_KTE(2, float, 16, true, 2), FEINT_KTS(2, float, 2), FEINT_KT(2, float, 1, 2), FEINT_KT(2, float, 4, 2), FEINT_KV_G(2, float, 16, 2, TetGeo), FEINT_K4U_TET(2, float, 1, 1, 2)};
const FwdVariant f3[] = {FEINT_KT(3, float, 1, 2), FEINT_KTE(3, float, 16, true, 2), FEINT_KTS(3, float, 2), FEINT_KTE(3, float, 16, false, 2), FEINT_KT(3, float, 4, 2), FEINT_K4U_TET(3, float, 2, 2, 2), FEINT_KV_G(3, float, 32, 2, TetGeo)};
const FwdVariant f4[] = {FEINT_KT(4, float, 1, 2), FEINT_KTE(4, float, 16, true, 2), FEINT_KTS(4, float, 2), FEINT_KTE(4, float, 16, false, 2), FEINT_KT(4, float, 4, 2), FEINT_K4U_TET(4, float, 3, 3, 2), FEINT_K4U_TET(4, float, 3, 3, 1)};
const FwdVariant f5[] = {FEINT_KT(5, float, 1, 2), FEINT_KTE(5, float, 16, true, 2), FEINT_KTS(5, float, 2), FEINT_KTE(5, float, 16, false, 2), FEINT_KT(5, float, 4, 2), FEINT_K4U_TET(5, float, 4, 4, 1), FEINT_K4U_TET(5, float, 4, 2, 2)};
const FwdVariant f6[] = {FEINT_KT(6, float, 1, 2), FEINT_KTE(6, float, 16, true, 2), FEINT_KTS(6, float, 2), FEINT_KTE(6, float, 16, false, 2), FEINT_KT(6, float, 4, 2), FEINT_K4U_TET(6, float, 6, 3, 1), FEINT_K4U_TET(6, float, 6, 2, 1)};
const FwdVariant f7[] = {FEINT_KT(7, float, 1, 2), FEINT_KTE(7, float, 16, true, 2), FEINT_KTS(7, float, 2), FEINT_KTE(7, float, 16, false, 2), FEINT_KT(7, float, 4, 2), FEINT_K4U_TET(7, float, 8, 4, 1), FEINT_K4U_TET(7, float, 8, 2, 1)};
const FwdVariant b1[] = {FEINT_K32U_G(1, BF16X3, 1, 1, 1, TetGeo)};
const FwdVariant b2[] = {FEINT_K32U_G(2, BF16X3, 1, 1, 1, TetGeo)};
const FwdVariant b3[] = {FEINT_K32U_G(3, BF16X3, 2, 2, 1, TetGeo)};
const FwdVariant b4[] = {FEINT_K32U_G(4, BF16X3, 3, 3, 1, TetGeo)};
const FwdVariant b5[] = {FEINT_K32U_G(5, BF16X3, 4, 4, 1, TetGeo), FEINT_K32U_G(5, BF16X3, 4, 2, 1, TetGeo)};
const FwdVariant b6[] = {FEINT_K32U_G(6, BF16X3, 6, 3, 1, TetGeo), FEINT_K32U_G(6, BF16X3, 6, 2, 1, TetGeo)};
const FwdVariant b7[] = {FEINT_K32U_G(7, BF16X3, 8, 4, 1, TetGeo), FEINT_K32U_G(7, BF16X3, 8, 2, 1, TetGeo)};
const FwdVariant h1[] = {FEINT_K32U_G(1, FP16X3, 1, 1, 1, TetGeo)};
const FwdVariant h2[] = {FEINT_K32U_G(2, FP16X3, 1, 1, 1, TetGeo)};
const FwdVariant h3[] = {FEINT_K32U_G(3, FP16X3, 2, 2, 1, TetGeo)};
const FwdVariant h4[] = {FEINT_K32U_G(4, FP16X3, 3, 3, 1, TetGeo)};
const FwdVariant h5[] = {FEINT_K32U_G(5, FP16X3, 4, 4, 1, TetGeo), FEINT_K32U_G(5, FP16X3, 4, 2, 1, TetGeo)};
const FwdVariant h6[] = {FEINT_K32U_G(6, FP16X3, 6, 3, 1, TetGeo), FEINT_K32U_G(6, FP16X3, 6, 2, 1, TetGeo)};
const FwdVariant h7[] = {FEINT_K32U_G(7, FP16X3, 8, 4, 1, TetGeo), FEINT_K32U_G(7, FP16X3, 8, 2, 1, TetGeo)};

#define FEINT_PICK(a1, a2, a3, a4, a5, a6, a7)                    \
    switch (p) {                                                   \
    case 1: *count = (int)(sizeof(a1) / sizeof(a1[0])); return a1; \
    case 2: *count = (int)(sizeof(a2) / sizeof(a2[0])); return a2; \
    case 3: *count = (int)(sizeof(a3) / sizeof(a3[0])); return a3; \
    case 4: *count = (int)(sizeof(a4) / sizeof(a4[0])); return a4; \
    case 5: *count = (int)(sizeof(a5) / sizeof(a5[0])); return a5; \
    case 6: *count = (int)(sizeof(a6) / sizeof(a6[0])); return a6; \
    case 7: *count = (int)(sizeof(a7) / sizeof(a7[0])); return a7; \
    }
}  // namespace

const FwdVariant *fwd_variants_tet(int form, int p, int *count) {
    switch (form) {
    case F64: FEINT_PICK(d1, d2, d3, d4, d5, d6, d7); break;
    case F32: FEINT_PICK(f1, f2, f3, f4, f5, f6, f7); break;
    case BF16X3: FEINT_PICK(b1, b2, b3, b4, b5, b6, b7); break;
    case FP16X3: FEINT_PICK(h1, h2, h3, h4, h5, h6, h7); break;
    }
    *count = 0;
    return nullptr;
}
}  // namespace feint
