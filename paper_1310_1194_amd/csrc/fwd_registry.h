// Launch helpers that instantiate the forward kernels for a list of tile
// shapes of one form.
#pragma once
#include "fwd_kernels.h"

namespace feint {

template <class KER>
void launch_direct(const FwdParams &prm, hipStream_t s) {
    const int64_t items = prm.ne * KER::NBLK;
    const int64_t blocks = (items + 3) / 4;
    hipLaunchKernelGGL(fwd_direct<KER>, dim3((unsigned)blocks), dim3(256), 0, s, prm);
}

template <class KER>
int64_t items_of() { return KER::NBLK; }

#define FEINT_K4(P, T, TM, TN) FwdVariant{TM, TN, &launch_direct<K4<P, T, TM, TN>>, &items_of<K4<P, T, TM, TN>>}
#define FEINT_K32(P, F, TM, TN) FwdVariant{TM, TN, &launch_direct<K32<P, F, TM, TN>>, &items_of<K32<P, F, TM, TN>>}

}  // namespace feint
