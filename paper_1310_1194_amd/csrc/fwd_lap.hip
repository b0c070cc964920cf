// Forward kernels of the paper's own term (Laplace, eq. (1)) on its quadrature
// (the symmetric triangle rule of degree 2p x (p+1) Gauss points in zeta, the
// N_I of Table 3), FP64 and FP32: the vector-ALU kernels at p <= 2 (at p = 1
// also one element per lane) and the contraction per triangle point above,
// with the Laplace geometry policy (coordinates only,
// W_q = w det J [[0, 0], [0, K K^T]], no load vector), one wave per block
// ("KxTNf") or the waves of a workgroup sharing the point blocks ("KxTNfw").
// The first shape per degree is the default until the autotuner picks another.
#include "fwd_registry.h"

namespace feint {
namespace {
constexpr int S = 1;
typedef PrismLaplaceGeo L;
#define LKV(P, T, LPE, W) \
    FwdVariant{0, LPE, 3, W, &launch_direct<KV<P, T, LPE, S, L>, W>, &items_of<KV<P, T, LPE, S, L>>}
#define LKE(P, T, W) \
    FwdVariant{0, 1, 3, W, &launch_direct<KE<P, T, S, L>, W>, &items_of<KE<P, T, S, L>>}
#define LKF(P, T, TMK, TN, W) \
    FwdVariant{TMK, TN, 6, W, &launch_direct<KF<P, T, TMK, TN, S, L>, W>, &items_of<KF<P, T, TMK, TN, S, L>>}
#define LKF2(P, T, TMK, TN, W) \
    FwdVariant{TMK, TN, 13, W, &launch_coop<KF2<P, T, TMK, TN, S, L>, W>, &items_of<KF2<P, T, TMK, TN, S, L>>}
#define LKF2Z(P, T, TMK, TN, IJB, W)                                           \
    FwdVariant{TMK, TN, 16, W, &launch_coop<KF2Z<P, T, TMK, TN, IJB, S, L>, W>, \
               &items_of<KF2Z<P, T, TMK, TN, IJB, S, L>>}
// FP64
const FwdVariant d1[] = {LKE(1, double, 2), LKV(1, double, 8, 2), LKF(1, double, 2, 2, 2)};
const FwdVariant d2[] = {LKV(2, double, 18, 2), LKF(2, double, 3, 3, 2)};
const FwdVariant d3[] = {LKF2(3, double, 4, 2, 2), LKF(3, double, 4, 2, 2), LKF(3, double, 4, 2, 1), LKV(3, double, 40, 2)};
const FwdVariant d4[] = {LKF2(4, double, 5, 3, 2), LKF(4, double, 5, 5, 1), LKF(4, double, 5, 3, 1)};
const FwdVariant d5[] = {LKF2(5, double, 3, 2, 2), LKF(5, double, 6, 2, 1), LKF(5, double, 3, 2, 1)};
const FwdVariant d6[] = {LKF2Z(6, double, 2, 2, 2, 2), LKF2(6, double, 2, 2, 2), LKF(6, double, 7, 1, 1), LKF(6, double, 4, 2, 1)};
const FwdVariant d7[] = {LKF2Z(7, double, 2, 2, 2, 2), LKF2(7, double, 2, 2, 2), LKF(7, double, 4, 2, 1), LKF(7, double, 4, 1, 1)};
// FP32
const FwdVariant f1[] = {LKE(1, float, 3), LKE(1, float, 2), LKV(1, float, 8, 2), LKF(1, float, 2, 2, 2)};
const FwdVariant f2[] = {LKV(2, float, 18, 2), LKF(2, float, 3, 3, 2)};
const FwdVariant f3[] = {LKF(3, float, 4, 4, 2), LKF2(3, float, 4, 2, 2), LKV(3, float, 40, 2)};
const FwdVariant f4[] = {LKF2(4, float, 5, 3, 2), LKF(4, float, 5, 3, 1), LKF(4, float, 5, 5, 1)};
const FwdVariant f5[] = {LKF2(5, float, 6, 3, 2), LKF(5, float, 6, 6, 1), LKF(5, float, 6, 3, 1)};
const FwdVariant f6[] = {LKF2Z(6, float, 4, 2, 2, 2), LKF2(6, float, 4, 2, 2), LKF(6, float, 7, 4, 1), LKF(6, float, 7, 3, 1)};
const FwdVariant f7[] = {LKF2Z(7, float, 4, 2, 4, 2), LKF2(7, float, 4, 2, 2), LKF(7, float, 8, 2, 1), LKF(7, float, 4, 2, 1)};

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

const FwdVariant *fwd_variants_lap(int form, int p, int *count) {
    switch (form) {
    case F64: FEINT_PICK(d1, d2, d3, d4, d5, d6, d7); break;
    case F32: FEINT_PICK(f1, f2, f3, f4, f5, f6, f7); break;
    }
    *count = 0;
    return nullptr;
}
}  // namespace feint
