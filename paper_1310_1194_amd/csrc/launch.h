// Host-visible kernel parameter blocks and launcher registry.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace feint {

struct FwdParams {
    const double *coords, *D, *beta, *c, *f;
    int64_t ne;
    void *A, *b;
    double *xq;
    uint32_t *status;
    const double *qw;        // [nqp][4]
    const double *gll;       // [2][p+1] Gauss-Lobatto nodes and Lagrange denominators
    const double *tau64;     // prisms: [nij][4][tpad] triangle factors of B (T, dT/dxi1, dT/dxi2, T)
    const float *tau32;
    const float *lam32;
    const double *lam;       // prisms: [4][p+1][p+1] line factors (L, L, L, dL/dzeta) at the zeta points
    const double *B64;       // [nqp][4][npad]
    const float *B32;        // [nqp][4][npad]
    const float *Bc32;       // [nqp][npad][4]
    const uint16_t *Bhi;     // [nkb][npad/16][64][8] split table of the form (bf16 or fp16),
    const uint16_t *Blo;     //   in A-fragment order
    const float *Ycf;        // [nkb][npad/16][64][8] FP32 columns in B-fragment order
    const double *Mref64;    // tetrahedra: reference matrices [16][n*n padded to 16] and load vector [n]
    const float *Mref32;
    const uint16_t *taubh;   // prisms: triangle factors split into hi / lo, A-fragment order (bf16;
    const uint16_t *taubl;   //   fp16 of tau * 2^tau_f16_shift for the fp16 form)
    int tau_f16_shift;
    float f16_zc, f16_zb;    // fp16 form: |Z| <= f16_zc max|W|, load-vector zeta sums <= f16_zb max|w det J f|
    float bmax;              // max |B| (fp16 form: used for the per-element scale)
    int f16_shift;           // fp16 tables hold B * 2^f16_shift
    // mixed-degree launches: element ids in bucket order and packed offsets
    const int32_t *perm;     // nullable: element of work slot i is perm[i]
    const int64_t *offA, *offb;
    // nullable: coefficients given at the six vertices ([ne][6][9], [ne][6][3],
    // [ne][6], [ne][6]) instead of one value per element
    const double *fD, *fbeta, *fc, *ff;
};

// One compiled tile shape of a (degree, form): TM x TN 16x16 output tiles
// per wave (MFMA kernels), or tn lanes per element (vector-ALU kernels,
// tm = 0); `launch` enqueues the direct (one work item per wave) kernel.
struct FwdVariant {
    int tm, tn;
    int staged;          // 1: the table is staged through LDS per workgroup (2: A operands only),
                         // 3: vector-ALU kernel, 4: software-pipelined split kernel,
                         // 5: shape functions computed at each point (no B table),
                         // 6: contraction per triangle point (tensor factors of B),
                         // 7: split kernel with Y formed on the matrix cores,
                         // 8: hexahedra by sum factorisation (9: W_q formed in each pass,
                         // 10: and the last pass reading from LDS), 11: tetrahedra from
                         // reference matrices
    int minw;            // waves per SIMD the register allocation allows
    void (*launch)(const FwdParams &, hipStream_t);
    int64_t (*items)(int64_t ne);   // work items (waves) of a launch over ne elements
};

// Registry per form (0 FP64, 1 FP32, 2 BF16X3, 3 FP16X3); p in 1..7; rule 0
// (collapsed Gauss) or 1 (symmetric triangle rule x Gauss in zeta).
const FwdVariant *fwd_variants(int form, int p, int *count, int rule = 0);
const FwdVariant *fwd_variants_sym(int form, int p, int *count);
// Hexahedral elements (FP64 and FP32 forms; count 0 for the split forms).
const FwdVariant *fwd_variants_hex(int form, int p, int *count);
// Tetrahedral elements (FP64 and FP32 forms).
const FwdVariant *fwd_variants_tet(int form, int p, int *count);
// The Laplace term alone on the symmetric rule (FP64 and FP32 forms).
const FwdVariant *fwd_variants_lap(int form, int p, int *count);
const FwdVariant *fwd_variants_f64(int p, int *count);
const FwdVariant *fwd_variants_f32(int p, int *count);
const FwdVariant *fwd_variants_bf16(int p, int *count);
const FwdVariant *fwd_variants_f16(int p, int *count);

}  // namespace feint
