// Launch helpers that instantiate the forward kernels for a list of tile
// shapes of one form.
#pragma once
#include "fwd_kernels.h"
#include "fwd_staged.h"
#include "fwd_valu.h"
#include "fwd_pipe.h"

namespace feint {

template <class KER, int MINW>
void launch_direct(const FwdParams &prm, hipStream_t s) {
    const int64_t items = items_for<KER>(prm.ne);
    const int64_t blocks = (items + 3) / 4;
    hipLaunchKernelGGL((fwd_direct<KER, MINW>), dim3((unsigned)blocks), dim3(256), 0, s, prm);
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
// W: minimum waves per SIMD asked of the register allocator.
#define FEINT_K4U(P, T, TM, TN, W) \
    FwdVariant{TM, TN, 0, W, &launch_direct<K4<P, T, TM, TN>, W>, &items_of<K4<P, T, TM, TN>>}
#define FEINT_K4S(P, T, TM, TN, SP, W) \
    FwdVariant{TM, TN, 1, W, &launch_staged<K4S<P, T, TM, TN, SP>, W>, &items_of<K4S<P, T, TM, TN, SP>>}
#define FEINT_K32U(P, F, TM, TN, W) \
    FwdVariant{TM, TN, 0, W, &launch_direct<K32<P, F, TM, TN>, W>, &items_of<K32<P, F, TM, TN>>}
// V: vector-ALU kernel, LPE lanes per element (tm = 0, tn = LPE, staged = 3).
#define FEINT_KV(P, T, LPE, W) \
    FwdVariant{0, LPE, 3, W, &launch_direct<KV<P, T, LPE>, W>, &items_of<KV<P, T, LPE>>}
// P: software-pipelined split kernel (staged = 4).
#define FEINT_K32P(P, F, TM, TN, W) \
    FwdVariant{TM, TN, 4, W, &launch_direct<K32P<P, F, TM, TN>, W>, &items_of<K32P<P, F, TM, TN>>}
#define FEINT_K32S(P, F, TM, TN, SY, W) \
    FwdVariant{TM, TN, 1 + !(SY), W, &launch_staged<K32S<P, F, TM, TN, SY>, W>, &items_of<K32S<P, F, TM, TN, SY>>}

}  // namespace feint
