// Launch helpers that instantiate the forward kernels for a list of tile
// shapes of one form.
#pragma once
#include "fwd_kernels.h"
#include "fwd_staged.h"
#include "fwd_valu.h"
#include "fwd_pipe.h"
#include "fwd_sc.h"
#include "fwd_fact.h"
#include "fwd_ymfma.h"
#include "fwd_hsf.h"
#include "fwd_tref.h"

namespace feint {

template <class KER, int MINW>
void launch_direct(const FwdParams &prm, hipStream_t s) {
    const int64_t items = items_for<KER>(prm.ne);
    const int64_t blocks = (items + 3) / 4;
    hipLaunchKernelGGL((fwd_direct<KER, MINW>), dim3((unsigned)blocks), dim3(256), 0, s, prm);
}

template <class KER, int MINW>
void launch_coop(const FwdParams &prm, hipStream_t s) {
    const int64_t items = items_for<KER>(prm.ne);
    const int64_t blocks = (items + 3) / 4;
    hipLaunchKernelGGL((fwd_coop<KER, MINW>), dim3((unsigned)blocks), dim3(256), 0, s, prm);
}

template <class KER, int MINW>
void launch_staged(const FwdParams &prm, hipStream_t s) {
    const int64_t items = items_for<KER>(prm.ne);
    const int64_t blocks = (items + 3) / 4;
    hipLaunchKernelGGL((fwd_staged<KER, MINW>), dim3((unsigned)blocks), dim3(256), 0, s, prm);
}

template <class KER>
int64_t items_of(int64_t ne) { return items_for<KER>(ne); }

// U: unstaged (each wave reads the table through L2); S: LDS-staged.
// W: minimum waves per SIMD asked of the register allocator.  R: quadrature
// rule (0 = collapsed Gauss, 1 = symmetric triangle rule x Gauss in zeta);
// the forms without _R compile the collapsed rule.
#define FEINT_K4U_R(P, T, TM, TN, W, R) \
    FwdVariant{TM, TN, 0, W, &launch_direct<K4<P, T, TM, TN, R>, W>, &items_of<K4<P, T, TM, TN, R>>}
#define FEINT_K4S_R(P, T, TM, TN, SP, W, R) \
    FwdVariant{TM, TN, 1, W, &launch_staged<K4S<P, T, TM, TN, SP, R>, W>, &items_of<K4S<P, T, TM, TN, SP, R>>}
#define FEINT_K32U_R(P, F, TM, TN, W, R) \
    FwdVariant{TM, TN, 0, W, &launch_direct<K32<P, F, TM, TN, R>, W>, &items_of<K32<P, F, TM, TN, R>>}
// V: vector-ALU kernel, LPE lanes per element (tm = 0, tn = LPE, staged = 3).
#define FEINT_KV_R(P, T, LPE, W, R) \
    FwdVariant{0, LPE, 3, W, &launch_direct<KV<P, T, LPE, R>, W>, &items_of<KV<P, T, LPE, R>>}
// E: one element per lane, vector ALU (p = 1; tm = 0, tn = 1 lane per element, staged = 3).
#define FEINT_KE_R(P, T, W, R) \
    FwdVariant{0, 1, 3, W, &launch_direct<KE<P, T, R>, W>, &items_of<KE<P, T, R>>}
#define FEINT_KE(P, T, W) FEINT_KE_R(P, T, W, 0)
// R: tetrahedra from reference matrices (staged = 11): one element per lane.
#define FEINT_KT(P, T, R, W) FwdVariant{R, 1, 11, W, &launch_direct<KT<P, T, R>, W>, &items_of<KT<P, T, R>>}
#define FEINT_KTS(P, T, W) FwdVariant{1, 2, 11, W, &launch_direct<KT<P, T, 1, true>, W>, &items_of<KT<P, T, 1, true>>}
#define FEINT_KTE(P, T, E, S, W) \
    FwdVariant{1, (S ? 2 : 1) + 4 * E, 11, W, &launch_direct<KT<P, T, 1, S, E>, W>, &items_of<KT<P, T, 1, S, E>>}
#define FEINT_KE_G(P, T, W, GEO) \
    FwdVariant{0, 1, 3, W, &launch_direct<KE<P, T, 0, GEO>, W>, &items_of<KE<P, T, 0, GEO>>}
// P: software-pipelined split kernel (staged = 4).
#define FEINT_K32P_R(P, F, TM, TN, W, R) \
    FwdVariant{TM, TN, 4, W, &launch_direct<K32P<P, F, TM, TN, R>, W>, &items_of<K32P<P, F, TM, TN, R>>}
#define FEINT_K32S_R(P, F, TM, TN, SY, W, R) \
    FwdVariant{TM, TN, 1 + !(SY), W, &launch_staged<K32S<P, F, TM, TN, SY, R>, W>, \
               &items_of<K32S<P, F, TM, TN, SY, R>>}

// Y: split kernel whose Y = W_q B_q is formed on the matrix cores (staged = 7).
// CH: 1 points in chunks of 64, 0 the element's points at once.
#define FEINT_K32Y_R(P, F, TM, TN, W, R, CH)                                                  \
    FwdVariant{TM, TN, 7, W, &launch_direct<K32Y<P, F, TM, TN, R, CH>, W>, \
               &items_of<K32Y<P, F, TM, TN, R, CH>>}
#define FEINT_K32Y(P, F, TM, TN, W, CH) FEINT_K32Y_R(P, F, TM, TN, W, 0, CH)

// C: shape functions computed at each point, no B table (staged = 5).
#define FEINT_KSC_R(P, T, TM, TN, W, R) \
    FwdVariant{TM, TN, 5, W, &launch_direct<KSC<P, T, TM, TN, R>, W>, &items_of<KSC<P, T, TM, TN, R>>}

// Hexahedra: the 16x16x4 kernel with the hexahedral geometry.
#define FEINT_K4U_HEX(P, T, TM, TN, W) \
    FwdVariant{TM, TN, 0, W, &launch_direct<K4<P, T, TM, TN, 0, HexGeo>, W>, &items_of<K4<P, T, TM, TN, 0, HexGeo>>}

// Tetrahedra: the 16x16x4 kernel with the affine tetrahedral geometry.
#define FEINT_K4U_TET(P, T, TM, TN, W) \
    FwdVariant{TM, TN, 0, W, &launch_direct<K4<P, T, TM, TN, 0, TetGeo>, W>, &items_of<K4<P, T, TM, TN, 0, TetGeo>>}

// Split forms on hexahedra and tetrahedra: the 16x16x32 kernel with their geometry.
#define FEINT_K32U_G(P, F, TM, TN, W, GEO) \
    FwdVariant{TM, TN, 0, W, &launch_direct<K32<P, F, TM, TN, 0, GEO>, W>, &items_of<K32<P, F, TM, TN, 0, GEO>>}

// Vector-ALU kernel on hexahedra and tetrahedra (low degree).
#define FEINT_KV_G(P, T, LPE, W, GEO) \
    FwdVariant{0, LPE, 3, W, &launch_direct<KV<P, T, LPE, 0, GEO>, W>, &items_of<KV<P, T, LPE, 0, GEO>>}

// F: contraction per triangle point (tensor factors of B, staged = 6):
// TMK row blocks k and TN column tiles per wave.
#define FEINT_KF_R(P, T, TMK, TN, W, R) \
    FwdVariant{TMK, TN, 6, W, &launch_direct<KF<P, T, TMK, TN, R>, W>, &items_of<KF<P, T, TMK, TN, R>>}
// the same, two waves per element sharing its point blocks through LDS (staged = 13)
#define FEINT_KF2_R(P, T, TMK, TN, W, R) \
    FwdVariant{TMK, TN, 13, W, &launch_coop<KF2<P, T, TMK, TN, R>, W>, &items_of<KF2<P, T, TMK, TN, R>>}
#define FEINT_KF2(P, T, TMK, TN, W) FEINT_KF2_R(P, T, TMK, TN, W, 0)
// the split forms of it with the zeta sums taken first and shared through LDS (staged = 15)
#define FEINT_KF2G_R(P, TMK, TN, W, R) \
    FwdVariant{TMK, TN, 15, W, &launch_coop<KF2G<P, TMK, TN, R>, W>, &items_of<KF2G<P, TMK, TN, R>>}
#define FEINT_KF2G(P, TMK, TN, W) FEINT_KF2G_R(P, TMK, TN, W, 0)
#define FEINT_KF2GH_R(P, TMK, TN, W, R)                                                            \
    FwdVariant{TMK, TN, 15, W, &launch_coop<KF2G<P, TMK, TN, R, PrismGeo, FP16X3>, W>,          \
               &items_of<KF2G<P, TMK, TN, R, PrismGeo, FP16X3>>}
#define FEINT_KF2GH(P, TMK, TN, W) FEINT_KF2GH_R(P, TMK, TN, W, 0)
// FP64 / FP32 with the zeta sums taken first (staged = 16)
#define FEINT_KF2Z_R(P, T, TMK, TN, IJB, W, R)                                                     \
    FwdVariant{TMK, TN, 16, W, &launch_coop<KF2Z<P, T, TMK, TN, IJB, R>, W>,                    \
               &items_of<KF2Z<P, T, TMK, TN, IJB, R>>}
#define FEINT_KF2Z(P, T, TMK, TN, IJB, W) FEINT_KF2Z_R(P, T, TMK, TN, IJB, W, 0)
#define FEINT_KF_HEX(P, T, TMK, TN, W)                                        \
    FwdVariant{TMK, TN, 6, W, &launch_direct<KF<P, T, TMK, TN, 0, HexGeo>, W>, \
               &items_of<KF<P, T, TMK, TN, 0, HexGeo>>}

// H: hexahedra by sum factorisation in all three directions (staged = 8): EPW
// elements per workgroup of NTH threads (tm = EPW, tn = NTH / 64 waves), W waves
// per SIMD asked of the register allocator; KHR forms W_q again in every pass of
// the slots (staged = 9).
#define FEINT_KH(P, T, NTH, EPW, W) \
    FwdVariant{EPW, (NTH) / 64, 8, W, &launch_hsf<P, T, NTH, EPW, false, W>, &items_hsf<EPW>}
#define FEINT_KHR(P, T, NTH, EPW, W) \
    FwdVariant{EPW, (NTH) / 64, 9, W, &launch_hsf<P, T, NTH, EPW, true, W>, &items_hsf<EPW>}
// KHL: W_q formed again per pass, and the last pass reading T2 from LDS where it
// is used (fewer registers: two waves per SIMD in FP64 at p >= 5; staged = 10)
#define FEINT_KHL(P, T, NTH, EPW, W) \
    FwdVariant{EPW, (NTH) / 64, 10, W, &launch_hsf<P, T, NTH, EPW, true, W, true>, &items_hsf<EPW>}

#define FEINT_K4U(P, T, TM, TN, W) FEINT_K4U_R(P, T, TM, TN, W, 0)
#define FEINT_KSC(P, T, TM, TN, W) FEINT_KSC_R(P, T, TM, TN, W, 0)
#define FEINT_K4S(P, T, TM, TN, SP, W) FEINT_K4S_R(P, T, TM, TN, SP, W, 0)
#define FEINT_K32U(P, F, TM, TN, W) FEINT_K32U_R(P, F, TM, TN, W, 0)
#define FEINT_KV(P, T, LPE, W) FEINT_KV_R(P, T, LPE, W, 0)
#define FEINT_K32P(P, F, TM, TN, W) FEINT_K32P_R(P, F, TM, TN, W, 0)
#define FEINT_K32S(P, F, TM, TN, SY, W) FEINT_K32S_R(P, F, TM, TN, SY, W, 0)

}  // namespace feint
