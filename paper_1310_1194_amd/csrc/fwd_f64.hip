// Forward kernels, FP64 form: compiled variants per degree (the first is the default until the
// autotuner picks another): vector-ALU kernels at low degree, v_mfma_f64_16x16x4_f64 tiles point by point,
// and from p = 3 the contraction per triangle point (KF); "KxTNfw" is that contraction with the waves
// of an element sharing its point blocks through LDS (KF2), the default from p = 3 where it was
// measured faster (all but p = 3 in FP32).
#include "fwd_registry.h"

namespace feint {
namespace {
const FwdVariant v1[] = {
    FEINT_KE(1, double, 2),
    FEINT_KV(1, double, 8, 2),
    FEINT_KV(1, double, 6, 2),
    FEINT_K4S(1, double, 1, 1, 8, 1),
    FEINT_KSC(1, double, 1, 1, 1), FEINT_KF_R(1, double, 2, 2, 2, 0)};
const FwdVariant v2[] = {
    FEINT_KV(2, double, 18, 2),
    FEINT_KV(2, double, 32, 2),
    FEINT_K4S(2, double, 2, 2, 8, 1),
    FEINT_K4S(2, double, 2, 1, 8, 2),
    FEINT_KSC(2, double, 2, 2, 1), FEINT_KF_R(2, double, 3, 3, 2, 0)};
const FwdVariant v3[] = {
    FEINT_KF2(3, double, 4, 2, 2),
    FEINT_KF_R(3, double, 4, 2, 2, 0),
    FEINT_KF_R(3, double, 4, 1, 2, 0),
    FEINT_KF_R(3, double, 4, 2, 1, 0),
    FEINT_K4S(3, double, 3, 3, 8, 1),
    FEINT_K4S(3, double, 3, 1, 8, 2),
    FEINT_KV(3, double, 40, 2),
    FEINT_KF_R(3, double, 4, 4, 1, 0),
    FEINT_KSC(3, double, 3, 3, 1)};
const FwdVariant v4[] = {
    FEINT_KF2(4, double, 5, 3, 2),
    FEINT_KF_R(4, double, 5, 5, 1, 0),
    FEINT_KF_R(4, double, 5, 3, 1, 0),
    FEINT_KF_R(4, double, 5, 1, 1, 0),
    FEINT_K4S(4, double, 5, 3, 8, 2),
    FEINT_K4U(4, double, 5, 1, 2),
    FEINT_KSC(4, double, 5, 3, 1)};
const FwdVariant v5[] = {
    FEINT_KF2Z(5, double, 3, 2, 4, 2),
    FEINT_KF2(5, double, 3, 2, 2),
    FEINT_KF_R(5, double, 6, 2, 1, 0),
    FEINT_KF_R(5, double, 3, 2, 1, 0),
    FEINT_KF_R(5, double, 6, 1, 1, 0),
    FEINT_K4U(5, double, 8, 1, 2),
    FEINT_K4S(5, double, 8, 1, 4, 2),
    FEINT_KSC(5, double, 8, 2, 1)};
const FwdVariant v6[] = {
    FEINT_KF2Z(6, double, 4, 1, 2, 2),
    FEINT_KF2Z(6, double, 2, 2, 2, 2),
    FEINT_KF2(6, double, 2, 2, 2),
    FEINT_KF_R(6, double, 7, 1, 1, 0),
    FEINT_KF_R(6, double, 4, 2, 1, 0),
    FEINT_K4U(6, double, 13, 1, 2),
    FEINT_K4S(6, double, 13, 1, 4, 1),
    FEINT_KSC(6, double, 13, 1, 1)};
const FwdVariant v7[] = {
    FEINT_KF2Z(7, double, 2, 2, 2, 2),
    FEINT_KF2(7, double, 2, 2, 2),
    FEINT_KF_R(7, double, 4, 2, 1, 0),
    FEINT_KF_R(7, double, 2, 2, 1, 0),
    FEINT_KF_R(7, double, 4, 1, 1, 0),
    FEINT_K4U(7, double, 9, 2, 1),
    FEINT_K4U(7, double, 6, 2, 1),
    FEINT_KSC(7, double, 6, 2, 1)};
}  // namespace

#define FEINT_N(a) (int)(sizeof(a) / sizeof(a[0]))
const FwdVariant *fwd_variants_f64(int p, int *count) {
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
