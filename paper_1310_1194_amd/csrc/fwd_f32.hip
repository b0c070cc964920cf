// Forward kernels, FP32 form: compiled variants per degree (the first is the default until the
// autotuner picks another): vector-ALU kernels at low degree, v_mfma_f32_16x16x4_f32 tiles point by point,
// and from p = 3 the contraction per triangle point (KF); "KxTNfw" is that contraction with the waves
// of an element sharing its point blocks through LDS (KF2), the default from p = 3 where it was
// measured faster (all but p = 3 in FP32).
#include "fwd_registry.h"

namespace feint {
namespace {
const FwdVariant v1[] = {
    FEINT_KE(1, float, 3),
    FEINT_KE(1, float, 2),
    FEINT_KV(1, float, 8, 2),
    FEINT_KV(1, float, 6, 2),
    FEINT_K4S(1, float, 1, 1, 8, 1),
    FEINT_KSC(1, float, 1, 1, 1), FEINT_KF_R(1, float, 2, 2, 2, 0)};
const FwdVariant v2[] = {
    FEINT_KV(2, float, 18, 2),
    FEINT_KV(2, float, 32, 2),
    FEINT_K4S(2, float, 2, 2, 8, 1),
    FEINT_KSC(2, float, 2, 2, 1), FEINT_KF_R(2, float, 3, 3, 2, 0)};
const FwdVariant v3[] = {
    FEINT_KF_R(3, float, 4, 4, 2, 0),
    FEINT_KF2(3, float, 4, 2, 2),
    FEINT_K4S(3, float, 3, 3, 8, 1),
    FEINT_K4S(3, float, 3, 1, 8, 2),
    FEINT_KV(3, float, 40, 2),
    FEINT_KSC(3, float, 3, 3, 1)};
const FwdVariant v4[] = {
    FEINT_KF2(4, float, 3, 5, 2),
    FEINT_KF2(4, float, 5, 3, 2),
    FEINT_KF_R(4, float, 5, 3, 1, 0),
    FEINT_KF_R(4, float, 5, 5, 1, 0),
    FEINT_K4S(4, float, 5, 5, 8, 1),
    FEINT_K4S(4, float, 5, 3, 8, 2),
    FEINT_K4U(4, float, 5, 5, 1),
    FEINT_KSC(4, float, 5, 5, 1)};
const FwdVariant v5[] = {
    FEINT_KF2Z(5, float, 3, 2, 4, 2),
    FEINT_KF2(5, float, 6, 3, 2),
    FEINT_KF_R(5, float, 6, 6, 1, 0),
    FEINT_KF_R(5, float, 6, 3, 1, 0),
    FEINT_K4U(5, float, 8, 8, 1),
    FEINT_K4S(5, float, 8, 2, 8, 2),
    FEINT_K4U(5, float, 8, 4, 1),
    FEINT_KSC(5, float, 8, 4, 1)};
const FwdVariant v6[] = {
    FEINT_KF2Z(6, float, 4, 2, 2, 2),
    FEINT_KF2(6, float, 4, 2, 2),
    FEINT_KF_R(6, float, 7, 4, 1, 0),
    FEINT_KF_R(6, float, 7, 3, 1, 0),
    FEINT_K4S(6, float, 13, 2, 8, 1),
    FEINT_K4U(6, float, 13, 4, 1),
    FEINT_KSC(6, float, 13, 2, 1)};
const FwdVariant v7[] = {
    FEINT_KF2Z(7, float, 4, 2, 4, 2),
    FEINT_KF2(7, float, 4, 2, 2),
    FEINT_KF_R(7, float, 8, 2, 1, 0),
    FEINT_K4U(7, float, 9, 6, 1),
    FEINT_K4U(7, float, 6, 3, 1),
    FEINT_KSC(7, float, 9, 3, 1)};
}  // namespace

#define FEINT_N(a) (int)(sizeof(a) / sizeof(a[0]))
const FwdVariant *fwd_variants_f32(int p, int *count) {
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
