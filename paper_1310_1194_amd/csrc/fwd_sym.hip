// Forward kernels on the symmetric prism rule (fully symmetric triangle rule
// of degree 2p x (p+1) Gauss points in zeta, the point counts of the paper's
// Table 3): the same kernels as the collapsed rule, instantiated with the
// rule's point count; a short list of shapes per (form, degree), the first
// being the default until the autotuner picks another.
#include "fwd_registry.h"

namespace feint {
namespace {
constexpr int S = 1;
// FP64
const FwdVariant d1[] = {FEINT_KE_R(1, double, 2, S), FEINT_KV_R(1, double, 8, 2, S), FEINT_K4S_R(1, double, 1, 1, 8, 1, S), FEINT_KSC_R(1, double, 1, 1, 1, S), FEINT_KF_R(1, double, 2, 2, 2, S)};
const FwdVariant d2[] = {FEINT_KV_R(2, double, 18, 2, S), FEINT_K4S_R(2, double, 2, 2, 8, 1, S), FEINT_KSC_R(2, double, 2, 2, 1, S), FEINT_KF_R(2, double, 3, 3, 2, S)};
const FwdVariant d3[] = {FEINT_KF2_R(3, double, 4, 2, 2, S), FEINT_KF_R(3, double, 4, 2, 2, S), FEINT_KF_R(3, double, 4, 2, 1, S), FEINT_K4S_R(3, double, 3, 3, 8, 1, S), FEINT_KV_R(3, double, 40, 2, S), FEINT_KSC_R(3, double, 3, 3, 1, S)};
const FwdVariant d4[] = {FEINT_KF2_R(4, double, 5, 3, 2, S), FEINT_KF_R(4, double, 5, 5, 1, S), FEINT_KF_R(4, double, 5, 3, 1, S), FEINT_K4S_R(4, double, 5, 3, 8, 2, S), FEINT_K4U_R(4, double, 5, 1, 2, S), FEINT_KSC_R(4, double, 5, 3, 1, S)};
const FwdVariant d5[] = {FEINT_KF2_R(5, double, 3, 2, 2, S), FEINT_KF2Z_R(5, double, 3, 2, 4, 2, S), FEINT_KF_R(5, double, 6, 2, 1, S), FEINT_KF_R(5, double, 3, 2, 1, S), FEINT_KF_R(5, double, 6, 1, 1, S), FEINT_K4S_R(5, double, 8, 1, 4, 2, S), FEINT_K4U_R(5, double, 8, 1, 2, S), FEINT_KSC_R(5, double, 8, 2, 1, S)};
const FwdVariant d6[] = {FEINT_KF2Z_R(6, double, 2, 2, 2, 2, S), FEINT_KF2_R(6, double, 2, 2, 2, S), FEINT_KF_R(6, double, 7, 1, 1, S), FEINT_KF_R(6, double, 4, 2, 1, S), FEINT_K4U_R(6, double, 13, 1, 2, S), FEINT_K4S_R(6, double, 13, 1, 4, 1, S), FEINT_KSC_R(6, double, 13, 1, 1, S)};
const FwdVariant d7[] = {FEINT_KF2Z_R(7, double, 2, 2, 2, 2, S), FEINT_KF2_R(7, double, 2, 2, 2, S), FEINT_KF_R(7, double, 4, 2, 1, S), FEINT_KF_R(7, double, 2, 2, 1, S), FEINT_KF_R(7, double, 4, 1, 1, S), FEINT_K4U_R(7, double, 9, 2, 1, S), FEINT_K4U_R(7, double, 6, 2, 1, S), FEINT_KSC_R(7, double, 6, 2, 1, S)};
// FP32
const FwdVariant f1[] = {FEINT_KE_R(1, float, 3, S), FEINT_KV_R(1, float, 8, 2, S), FEINT_K4S_R(1, float, 1, 1, 8, 1, S), FEINT_KSC_R(1, float, 1, 1, 1, S), FEINT_KF_R(1, float, 2, 2, 2, S)};
const FwdVariant f2[] = {FEINT_KV_R(2, float, 18, 2, S), FEINT_K4S_R(2, float, 2, 2, 8, 1, S), FEINT_KSC_R(2, float, 2, 2, 1, S), FEINT_KF_R(2, float, 3, 3, 2, S)};
const FwdVariant f3[] = {FEINT_KF_R(3, float, 4, 4, 2, S), FEINT_KF2_R(3, float, 4, 2, 2, S), FEINT_K4S_R(3, float, 3, 3, 8, 1, S), FEINT_KV_R(3, float, 40, 2, S), FEINT_KSC_R(3, float, 3, 3, 1, S)};
const FwdVariant f4[] = {FEINT_KF2_R(4, float, 5, 3, 2, S), FEINT_KF_R(4, float, 5, 3, 1, S), FEINT_KF_R(4, float, 5, 5, 1, S), FEINT_K4U_R(4, float, 5, 5, 1, S), FEINT_K4S_R(4, float, 5, 5, 8, 1, S), FEINT_KSC_R(4, float, 5, 5, 1, S)};
const FwdVariant f5[] = {FEINT_KF2_R(5, float, 6, 3, 2, S), FEINT_KF_R(5, float, 6, 6, 1, S), FEINT_KF_R(5, float, 6, 3, 1, S), FEINT_K4S_R(5, float, 8, 4, 8, 1, S), FEINT_K4U_R(5, float, 8, 8, 1, S), FEINT_KSC_R(5, float, 8, 4, 1, S)};
const FwdVariant f6[] = {FEINT_KF2_R(6, float, 2, 2, 2, S), FEINT_KF_R(6, float, 7, 4, 1, S), FEINT_KF_R(6, float, 7, 3, 1, S), FEINT_K4S_R(6, float, 13, 2, 8, 1, S), FEINT_K4U_R(6, float, 13, 4, 1, S), FEINT_KSC_R(6, float, 13, 2, 1, S)};
const FwdVariant f7[] = {FEINT_KF2Z_R(7, float, 4, 2, 4, 2, S), FEINT_KF2_R(7, float, 4, 2, 2, S), FEINT_KF_R(7, float, 8, 2, 1, S), FEINT_K4U_R(7, float, 9, 6, 1, S), FEINT_K4U_R(7, float, 9, 3, 1, S), FEINT_KSC_R(7, float, 9, 3, 1, S)};
// bf16x3
const FwdVariant b1[] = {FEINT_K32S_R(1, BF16X3, 1, 1, true, 1, S)};
const FwdVariant b2[] = {FEINT_K32S_R(2, BF16X3, 2, 2, true, 1, S)};
const FwdVariant b3[] = {FEINT_K32S_R(3, BF16X3, 3, 3, true, 1, S)};
const FwdVariant b4[] = {FEINT_K32P_R(4, BF16X3, 5, 5, 1, S), FEINT_K32U_R(4, BF16X3, 5, 3, 2, S)};
const FwdVariant b5[] = {FEINT_KF2G_R(5, 3, 2, 2, S), FEINT_K32S_R(5, BF16X3, 8, 4, false, 1, S), FEINT_K32U_R(5, BF16X3, 8, 4, 1, S)};
const FwdVariant b6[] = {FEINT_KF2G_R(6, 7, 1, 2, S), FEINT_K32S_R(6, BF16X3, 13, 2, false, 2, S), FEINT_K32U_R(6, BF16X3, 13, 2, 1, S)};
const FwdVariant b7[] = {FEINT_KF2G_R(7, 4, 2, 2, S), FEINT_KF2G_R(7, 4, 1, 2, S), FEINT_K32P_R(7, BF16X3, 6, 6, 1, S), FEINT_K32P_R(7, BF16X3, 6, 3, 1, S)};
// fp16x3
const FwdVariant h1[] = {FEINT_K32S_R(1, FP16X3, 1, 1, true, 1, S)};
const FwdVariant h2[] = {FEINT_K32S_R(2, FP16X3, 2, 2, true, 1, S)};
const FwdVariant h3[] = {FEINT_K32S_R(3, FP16X3, 3, 3, true, 1, S)};
const FwdVariant h4[] = {FEINT_K32P_R(4, FP16X3, 5, 5, 1, S), FEINT_K32U_R(4, FP16X3, 5, 3, 2, S)};
const FwdVariant h5[] = {FEINT_K32S_R(5, FP16X3, 8, 4, false, 1, S), FEINT_KF2GH_R(5, 3, 2, 2, S), FEINT_K32U_R(5, FP16X3, 8, 4, 1, S)};
const FwdVariant h6[] = {FEINT_KF2GH_R(6, 7, 1, 2, S), FEINT_K32S_R(6, FP16X3, 13, 2, false, 2, S), FEINT_K32U_R(6, FP16X3, 13, 2, 1, S)};
const FwdVariant h7[] = {FEINT_KF2GH_R(7, 4, 2, 2, S), FEINT_KF2GH_R(7, 4, 1, 2, S), FEINT_K32P_R(7, FP16X3, 6, 6, 1, S), FEINT_K32P_R(7, FP16X3, 3, 6, 1, S)};

#define FEINT_PICK(a1, a2, a3, a4, a5, a6, a7)                  \
    switch (p) {                                                 \
    case 1: *count = (int)(sizeof(a1) / sizeof(a1[0])); return a1; \
    case 2: *count = (int)(sizeof(a2) / sizeof(a2[0])); return a2; \
    case 3: *count = (int)(sizeof(a3) / sizeof(a3[0])); return a3; \
    case 4: *count = (int)(sizeof(a4) / sizeof(a4[0])); return a4; \
    case 5: *count = (int)(sizeof(a5) / sizeof(a5[0])); return a5; \
    case 6: *count = (int)(sizeof(a6) / sizeof(a6[0])); return a6; \
    case 7: *count = (int)(sizeof(a7) / sizeof(a7[0])); return a7; \
    }
}  // namespace

const FwdVariant *fwd_variants_sym(int form, int p, int *count) {
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
