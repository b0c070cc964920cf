// Forward kernels for hexahedral elements (Table 1's tensor-product element):
// the 16x16x4 MFMA kernel (FP64, FP32) point by point and the contraction per
// plane point ("f", the fastest from p = 2 in FP64 and p = 3 in FP32; at p = 3
// and 7, where (p+1)^2 leaves no spare padded column, with its load vector
// summed in FP64); the 16x16x32 split kernel (bf16x3, fp16x3); all with the trilinear
// geometry (at p = 1 first the vector-ALU kernel, "vL" = L lanes per element);
// in FP64 and FP32 first the sum factorisation in all three directions
// ("sfWw" = W waves per workgroup, "xE" = E elements per workgroup, "r" = W_q formed
// again in each pass of the slots, "l" = that and the last pass reading T2 from LDS where
// it is used, "oK" = K waves per SIMD asked of the register allocator).
// Compiled tile shapes per degree (n = 8, 27, 64, 125, 216, 343, 512 shape
// functions: 1, 2, 4, 8, 14, 22, 32 tiles of 16), the first the default.
#include "fwd_registry.h"

namespace feint {
namespace {
const FwdVariant d1[] = {FEINT_KH(1, double, 64, 8, 1), FEINT_KV_G(1, double, 8, 2, HexGeo), FEINT_K4U_HEX(1, double, 1, 1, 2),
    FEINT_KF_HEX(1, double, 2, 2, 2)};
const FwdVariant d2[] = {FEINT_KH(2, double, 64, 2, 1), FEINT_KH(2, double, 128, 4, 1), FEINT_KF_HEX(2, double, 3, 3, 2),
    FEINT_KV_G(2, double, 32, 2, HexGeo),
    FEINT_K4U_HEX(2, double, 2, 2, 2),
    FEINT_K4U_HEX(2, double, 2, 1, 2)};
const FwdVariant d3[] = {FEINT_KH(3, double, 64, 1, 1), FEINT_KH(3, double, 128, 2, 1),
    FEINT_KF_HEX(3, double, 4, 2, 2),
    FEINT_KF_HEX(3, double, 4, 1, 2),
    FEINT_KF_HEX(3, double, 4, 2, 1),
    FEINT_KF_HEX(3, double, 4, 4, 1),
    FEINT_K4U_HEX(3, double, 4, 1, 2),
    FEINT_K4U_HEX(3, double, 4, 2, 1),
    FEINT_K4U_HEX(3, double, 2, 2, 2)};
const FwdVariant d4[] = {FEINT_KH(4, double, 128, 1, 1), FEINT_KH(4, double, 256, 2, 1), FEINT_KHL(4, double, 128, 1, 3),
    FEINT_KF_HEX(4, double, 5, 3, 1),
    FEINT_KF_HEX(4, double, 5, 2, 1),
    FEINT_KF_HEX(4, double, 5, 1, 1),
    FEINT_K4U_HEX(4, double, 8, 1, 2),
    FEINT_K4U_HEX(4, double, 8, 2, 1)};
const FwdVariant d5[] = {FEINT_KH(5, double, 256, 1, 1), FEINT_KH(5, double, 256, 1, 2), FEINT_KHL(5, double, 128, 1, 2),
    FEINT_KF_HEX(5, double, 3, 2, 1),
    FEINT_KF_HEX(5, double, 2, 2, 1),
    FEINT_K4U_HEX(5, double, 7, 2, 1),
    FEINT_K4U_HEX(5, double, 14, 1, 1)};
const FwdVariant d6[] = {FEINT_KHL(6, double, 256, 1, 2), FEINT_KH(6, double, 256, 2, 1), FEINT_KH(6, double, 256, 1, 1),
    FEINT_KF_HEX(6, double, 4, 1, 1),
    FEINT_KF_HEX(6, double, 3, 2, 1),
    FEINT_KF_HEX(6, double, 2, 2, 1),
    FEINT_K4U_HEX(6, double, 8, 2, 1),
    FEINT_K4U_HEX(6, double, 11, 1, 1),
    FEINT_K4U_HEX(6, double, 6, 2, 1)};
const FwdVariant d7[] = {FEINT_KHL(7, double, 256, 1, 2), FEINT_KH(7, double, 256, 1, 1),
    FEINT_KF_HEX(7, double, 4, 1, 1),
    FEINT_KF_HEX(7, double, 2, 1, 1),
    FEINT_KF_HEX(7, double, 1, 2, 1),
    FEINT_K4U_HEX(7, double, 8, 1, 1),
    FEINT_K4U_HEX(7, double, 4, 2, 1)};
const FwdVariant f1[] = {FEINT_KH(1, float, 64, 8, 1), FEINT_KV_G(1, float, 8, 2, HexGeo), FEINT_K4U_HEX(1, float, 1, 1, 2),
    FEINT_KF_HEX(1, float, 2, 2, 2)};
const FwdVariant f2[] = {FEINT_KH(2, float, 64, 2, 1), FEINT_KH(2, float, 128, 4, 1), FEINT_K4U_HEX(2, float, 2, 2, 2),
    FEINT_KF_HEX(2, float, 3, 3, 2),
    FEINT_KV_G(2, float, 32, 2, HexGeo)};
const FwdVariant f3[] = {FEINT_KH(3, float, 64, 1, 1), FEINT_KH(3, float, 128, 2, 1),
    FEINT_KF_HEX(3, float, 4, 4, 2),
    FEINT_KF_HEX(3, float, 4, 4, 1),
    FEINT_K4U_HEX(3, float, 2, 4, 1),
    FEINT_K4U_HEX(3, float, 4, 4, 1),
    FEINT_K4U_HEX(3, float, 4, 2, 1)};
const FwdVariant f4[] = {FEINT_KH(4, float, 128, 1, 1), FEINT_KH(4, float, 256, 2, 1),
    FEINT_KF_HEX(4, float, 5, 5, 1),
    FEINT_KF_HEX(4, float, 5, 3, 1),
    FEINT_KF_HEX(4, float, 5, 2, 1),
    FEINT_K4U_HEX(4, float, 8, 4, 1),
    FEINT_K4U_HEX(4, float, 8, 2, 1)};
const FwdVariant f5[] = {FEINT_KH(5, float, 256, 1, 1),
    FEINT_KF_HEX(5, float, 6, 3, 1),
    FEINT_KF_HEX(5, float, 6, 2, 1),
    FEINT_K4U_HEX(5, float, 14, 2, 1),
    FEINT_K4U_HEX(5, float, 7, 4, 1)};
const FwdVariant f6[] = {FEINT_KH(6, float, 256, 2, 1), FEINT_KHL(6, float, 256, 1, 3), FEINT_KH(6, float, 256, 1, 1), FEINT_KHR(6, float, 256, 1, 2),
    FEINT_KF_HEX(6, float, 7, 2, 1),
    FEINT_KF_HEX(6, float, 4, 2, 1),
    FEINT_K4U_HEX(6, float, 8, 4, 1),
    FEINT_K4U_HEX(6, float, 6, 4, 1)};
const FwdVariant f7[] = {FEINT_KHR(7, float, 256, 1, 2), FEINT_KHL(7, float, 256, 1, 3), FEINT_KH(7, float, 256, 1, 1),
    FEINT_KF_HEX(7, float, 8, 1, 1),
    FEINT_KF_HEX(7, float, 4, 1, 1),
    FEINT_KF_HEX(7, float, 2, 2, 1),
    FEINT_K4U_HEX(7, float, 8, 2, 1),
    FEINT_K4U_HEX(7, float, 4, 4, 1)};
const FwdVariant b1[] = {FEINT_K32U_G(1, BF16X3, 1, 1, 1, HexGeo)};
const FwdVariant b2[] = {FEINT_K32U_G(2, BF16X3, 2, 2, 1, HexGeo)};
const FwdVariant b3[] = {FEINT_K32U_G(3, BF16X3, 4, 4, 1, HexGeo), FEINT_K32U_G(3, BF16X3, 4, 2, 1, HexGeo)};
const FwdVariant b4[] = {FEINT_K32U_G(4, BF16X3, 8, 4, 1, HexGeo), FEINT_K32U_G(4, BF16X3, 8, 2, 1, HexGeo), FEINT_K32U_G(4, BF16X3, 4, 4, 1, HexGeo)};
const FwdVariant b5[] = {FEINT_K32U_G(5, BF16X3, 7, 4, 1, HexGeo), FEINT_K32U_G(5, BF16X3, 7, 2, 1, HexGeo)};
const FwdVariant b6[] = {FEINT_K32U_G(6, BF16X3, 11, 2, 1, HexGeo), FEINT_K32U_G(6, BF16X3, 8, 2, 1, HexGeo)};
const FwdVariant b7[] = {FEINT_K32U_G(7, BF16X3, 8, 2, 1, HexGeo), FEINT_K32U_G(7, BF16X3, 8, 4, 1, HexGeo)};
const FwdVariant h1[] = {FEINT_K32U_G(1, FP16X3, 1, 1, 1, HexGeo)};
const FwdVariant h2[] = {FEINT_K32U_G(2, FP16X3, 2, 2, 1, HexGeo)};
const FwdVariant h3[] = {FEINT_K32U_G(3, FP16X3, 4, 4, 1, HexGeo), FEINT_K32U_G(3, FP16X3, 4, 2, 1, HexGeo)};
const FwdVariant h4[] = {FEINT_K32U_G(4, FP16X3, 8, 4, 1, HexGeo), FEINT_K32U_G(4, FP16X3, 8, 2, 1, HexGeo), FEINT_K32U_G(4, FP16X3, 4, 4, 1, HexGeo)};
const FwdVariant h5[] = {FEINT_K32U_G(5, FP16X3, 7, 4, 1, HexGeo), FEINT_K32U_G(5, FP16X3, 7, 2, 1, HexGeo)};
const FwdVariant h6[] = {FEINT_K32U_G(6, FP16X3, 11, 2, 1, HexGeo), FEINT_K32U_G(6, FP16X3, 8, 2, 1, HexGeo)};
const FwdVariant h7[] = {FEINT_K32U_G(7, FP16X3, 8, 2, 1, HexGeo), FEINT_K32U_G(7, FP16X3, 8, 4, 1, HexGeo)};

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

const FwdVariant *fwd_variants_hex(int form, int p, int *count) {
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
