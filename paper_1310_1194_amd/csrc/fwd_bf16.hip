// Forward kernels, split bf16x3 form (v_mfma_f32_16x16x32_bf16): compiled tile shapes per degree (the first is
// the default until the autotuner picks another).
#include "fwd_registry.h"

namespace feint {
namespace {
const FwdVariant v1[] = {
    FEINT_K32S(1, BF16X3, 1, 1, true, 1)};
const FwdVariant v2[] = {
    FEINT_K32S(2, BF16X3, 2, 2, true, 1)};
const FwdVariant v3[] = {
    FEINT_K32S(3, BF16X3, 3, 3, true, 1),
    FEINT_K32S(3, BF16X3, 3, 1, true, 2)};
const FwdVariant v4[] = {
    FEINT_K32Y(4, BF16X3, 5, 5, 2, 0),
    FEINT_K32Y(4, BF16X3, 5, 3, 3, 0),
    FEINT_K32P(4, BF16X3, 5, 5, 1),
    FEINT_K32U(4, BF16X3, 5, 3, 2),
    FEINT_K32U(4, BF16X3, 5, 5, 1),
    FEINT_K32S(4, BF16X3, 5, 5, true, 1),
    FEINT_K32U(4, BF16X3, 5, 3, 1),
    FEINT_K32P(4, BF16X3, 5, 3, 1),
    FEINT_KF2G(4, 3, 3, 3),
    FEINT_KF2G(4, 5, 3, 2),
    FEINT_KF2G(4, 5, 1, 3)};
const FwdVariant v5[] = {
    FEINT_KF2G(5, 3, 2, 2),
    FEINT_K32S(5, BF16X3, 8, 4, false, 1),
    FEINT_K32S(5, BF16X3, 8, 4, true, 1),
    FEINT_K32S(5, BF16X3, 4, 4, false, 2),
    FEINT_K32U(5, BF16X3, 8, 4, 1),
    FEINT_KF2G(5, 3, 3, 2)};
const FwdVariant v6[] = {
    FEINT_KF2G(6, 7, 1, 2),
    FEINT_K32S(6, BF16X3, 13, 2, false, 2),
    FEINT_K32S(6, BF16X3, 13, 2, false, 1),
    FEINT_K32S(6, BF16X3, 7, 4, false, 1),
    FEINT_K32U(6, BF16X3, 13, 2, 1)};

const FwdVariant v7[] = {
    FEINT_KF2G(7, 4, 2, 2),
    FEINT_KF2G(7, 4, 1, 2),
    FEINT_K32Y(7, BF16X3, 3, 3, 2, 1),
    FEINT_K32Y(7, BF16X3, 6, 3, 1, 1),
    FEINT_K32Y(7, BF16X3, 6, 6, 1, 1),
    FEINT_K32Y(7, BF16X3, 9, 3, 1, 1),
    FEINT_K32P(7, BF16X3, 6, 6, 1),
    FEINT_K32S(7, BF16X3, 6, 6, false, 1),
    FEINT_K32U(7, BF16X3, 6, 6, 1),
    FEINT_K32P(7, BF16X3, 6, 3, 1),
    FEINT_K32P(7, BF16X3, 3, 6, 1)};
}  // namespace

#define FEINT_N(a) (int)(sizeof(a) / sizeof(a[0]))
const FwdVariant *fwd_variants_bf16(int p, int *count) {
    switch (p) {
    case 1: *count = FEINT_N(v1); return v1;
    case 2: *count = FEINT_N(v2); return v2;
    case 3: *count = FEINT_N(v3); return v3;
    case 4: *count = FEINT_N(v4); return v4;
    case 5: *count = FEINT_N(v5); return v5;
    case 6: *count = FEINT_N(v6); return v6;
    case 7: *count = FEINT_N(v7); return v7;
    }
    *count = 0;
    return nullptr;
}
}  // namespace feint
