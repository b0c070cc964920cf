// Internal helpers shared by the C-ABI translation units.
#pragma once
#include <string>
#include <hip/hip_runtime.h>

#include "feint.h"
#include "launch.h"

namespace feint {

// Device copy of the tables of one degree (one allocation, sub-buffers
// 256-byte aligned).
struct DevTables {
    int p, rule, n, npad, nq, nqp, nkb, f16_shift;
    float bmax;
    const double *qw, *gll, *B64, *BT64, *tau64, *lam;
    const float *tau32;
    const float *lam32;
    const float *B32, *BT32, *Bc32;
    const uint16_t *bf_hi, *bf_lo, *hf_hi, *hf_lo;
    const float *Ycf;
    const double *Mref64;
    const float *Mref32;
    const uint16_t *taubh, *taubl, *tauhh, *tauhl;
    int tau_f16_shift;
    float f16_zc, f16_zb;
    void *base;
};

void set_error(const char *what, hipError_t e);
// Set the thread's last-error text to a message of the library's own.
void set_error_msg(const std::string &msg);
feint_status prepare_tables(int p, int rule = 0, int type = 0);
const DevTables *find_tables(int p, int rule = 0, int type = 0);
feint_status tables_for_launch(int p, hipStream_t stream, const DevTables **out, int rule = 0, int type = 0);
feint_status check_elements(const feint_elements *el);
void fill_fwd_params(FwdParams &prm, const feint_elements *el, int form, const DevTables *T);
const FwdVariant *chosen_variant(int p, int form, int rule = 0);
feint_status launch_forward(const FwdParams &prm, const FwdVariant *v, hipStream_t stream);

}  // namespace feint
