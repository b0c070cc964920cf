// Adjoint of the forward integration: gradients of
//     L = sum_e <G_e, A_e> + <g_e, b_e>
// with respect to every element's vertices, D, beta, c and f.
//
// Since A_e = sum_q B_q^T W_q B_q, <G_e, A_e> = sum_q <W_q, S_q> with the 4x4
// block S_q = B_q G_e B_q^T.  The kernel forms U = B G_e on MFMA (rows: the
// 4 nq (point, row) pairs, K = shape functions), reduces S_q = U_q B_q^T
// across lanes into LDS, and then, one point per lane, recomputes the
// Jacobian in FP64 and pushes dL/dW_q = S_q through
//   W_q = w det J [[c, (K beta)^T], [0, K D K^T]],  K = J^{-1}:
//   dL/dc = sum wd S00,  dL/dbeta = sum wd K^T s,  dL/dD = sum wd K^T S' K,
//   dL/dK = wd (S' K D^T + S'^T K D + s beta^T),  dL/d det = L_q / det,
//   dL/dJ = L_q K^T - K^T (dL/dK) K^T,  then the bilinear map to the vertices
// (s = S[0,1:3], S' = S[1:3,1:3]).  Per-point Jacobians are never stored.
// All of it is linear in S_q, so for large degrees G_e is split into blocks
// handled by different waves whose partial gradients are summed atomically.
#include <hip/hip_runtime.h>

#include <cstring>

#include "capi_internal.h"
#include "device_common.h"
#include "fwd_kernels.h"
#include "tables.h"

namespace feint {

struct AdjParams {
    const double *coords, *D, *beta, *c, *f;
    int64_t ne;
    const void *G, *g;
    double *dX, *dD, *dbeta, *dc, *df;
    const double *qw, *B64;
    const void *Brow;   // [nqp][4][npad] in the form's precision
    const void *BT;     // [npad][nqp*4]  in the form's precision
};

template <int P, typename T, int TA, int TB>
struct Adj {
    static constexpr int N = c_nshp(P), NP = c_pad16(N), NT = NP / 16, NQ = c_nq(P);
    static constexpr int NQP = c_pad8(NQ);            // table rows
    static constexpr int NQ4 = (NQ + 3) / 4 * 4;       // points covered by 16-row tiles
    static constexpr int BA = c_cdiv(NT, TA), BB = c_cdiv(NT, TB), NBLK = BA * BB;
    static constexpr bool ATOMIC = NBLK > 1;
    typedef typename AccT<T>::type V4;

    struct Smem { double S[4][64][WROW<double>::value]; };

    __device__ static void chain_rule(const AdjParams &prm, const ElemIn &E, int q, const double S[16],
                                      bool with_load, int64_t e, double gr[32]) {
        const double *qp = prm.qw + 4 * q;
        const double xi1 = qp[0], xi2 = qp[1], ze = qp[2], w = qp[3];
        double K[9];
        const double det = prism_jacobian(E.X, xi1, xi2, ze, K);
        const double wd = w * det;
        double tau = 0.0;
        if (with_load) {
            const T *gv = (const T *)prm.g + e * N;
            const double *phi = prm.B64 + (size_t)q * 4 * NP;
            for (int a = 0; a < N; ++a) tau += (double)gv[a] * phi[a];
        }
        double v[3], KD[9], M[9];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            v[i] = K[3 * i] * E.be[0] + K[3 * i + 1] * E.be[1] + K[3 * i + 2] * E.be[2];
#pragma unroll
            for (int j = 0; j < 3; ++j)
                KD[3 * i + j] = K[3 * i] * E.D[j] + K[3 * i + 1] * E.D[3 + j] + K[3 * i + 2] * E.D[6 + j];
        }
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                M[3 * i + j] = KD[3 * i] * K[3 * j] + KD[3 * i + 1] * K[3 * j + 1] + KD[3 * i + 2] * K[3 * j + 2];
        const double s[3] = {S[1], S[2], S[3]};
        double Sp[9];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) Sp[3 * i + j] = S[4 * (i + 1) + 1 + j];
        double contr = E.c * S[0];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            contr += v[i] * s[i];
#pragma unroll
            for (int j = 0; j < 3; ++j) contr += M[3 * i + j] * Sp[3 * i + j];
        }
        const double Lq = wd * (contr + E.f * tau);
        // gradient slots: vertices 0..17, D 18..26, beta 27..29, c 30, f 31
        gr[30] += wd * S[0];
        gr[31] += wd * tau;
#pragma unroll
        for (int m = 0; m < 3; ++m)
            gr[27 + m] += wd * (K[m] * s[0] + K[3 + m] * s[1] + K[6 + m] * s[2]);
        double SK[9];   // S' K
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                SK[3 * i + j] = Sp[3 * i] * K[j] + Sp[3 * i + 1] * K[3 + j] + Sp[3 * i + 2] * K[6 + j];
#pragma unroll
        for (int m = 0; m < 3; ++m)
#pragma unroll
            for (int n = 0; n < 3; ++n)   // dD_mn = wd sum_k K_km (S'K)_kn
                gr[18 + 3 * m + n] += wd * (K[m] * SK[n] + K[3 + m] * SK[3 + n] + K[6 + m] * SK[6 + n]);
        // dL/dK = wd (S' K D^T + S'^T K D + s beta^T)
        double StK[9], dK[9];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                StK[3 * i + j] = Sp[i] * K[j] + Sp[3 + i] * K[3 + j] + Sp[6 + i] * K[6 + j];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                dK[3 * i + j] = wd * (SK[3 * i] * E.D[3 * j] + SK[3 * i + 1] * E.D[3 * j + 1] + SK[3 * i + 2] * E.D[3 * j + 2]
                                      + StK[3 * i] * E.D[j] + StK[3 * i + 1] * E.D[3 + j] + StK[3 * i + 2] * E.D[6 + j]
                                      + s[i] * E.be[j]);
        // dL/dJ = Lq K^T - K^T dK K^T
        double KtdK[9], dJ[9];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                KtdK[3 * i + j] = K[i] * dK[j] + K[3 + i] * dK[3 + j] + K[6 + i] * dK[6 + j];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                dJ[3 * i + j] = Lq * K[3 * j + i] - (KtdK[3 * i] * K[3 * j] + KtdK[3 * i + 1] * K[3 * j + 1] + KtdK[3 * i + 2] * K[3 * j + 2]);
        // J columns: c0 = s(v1-v0)+t(v4-v3), c1 = s(v2-v0)+t(v5-v3), c2 = (l0(v3-v0)+l1(v4-v1)+l2(v5-v2))/2
        const double t = 0.5 * (1.0 + ze), sb = 0.5 * (1.0 - ze), l0 = 1.0 - xi1 - xi2;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double g0 = dJ[3 * d], g1 = dJ[3 * d + 1], g2 = 0.5 * dJ[3 * d + 2];
            gr[0 + d] += -sb * g0 - sb * g1 - l0 * g2;
            gr[3 + d] += sb * g0 - xi1 * g2;
            gr[6 + d] += sb * g1 - xi2 * g2;
            gr[9 + d] += -t * g0 - t * g1 + l0 * g2;
            gr[12 + d] += t * g0 + xi1 * g2;
            gr[15 + d] += t * g1 + xi2 * g2;
        }
    }

    __device__ static void run(const AdjParams &prm, int64_t e, int blk, int wave, Smem &sm) {
        const int lane = threadIdx.x & 63;
        const int i16 = lane & 15, kg = lane >> 4;
        const int ba = blk / BB, bb = blk % BB;
        const int a0 = ba * TA * 16, b0 = bb * TB * 16;
        const bool with_load = blk == 0;
        ElemIn E;
        load_elem(prm.coords, prm.D, prm.beta, prm.c, prm.f, e, E);
        const T *Ge = (const T *)prm.G + e * (int64_t)N * N;
        const T *Br = (const T *)prm.Brow;
        const T *BTt = (const T *)prm.BT;
        // this wave's block of G as B-operand fragments: G[a0 + 4ks + kg][b0 + 16 tb + i16]
        T gf[4 * TA][TB];
#pragma unroll
        for (int ks = 0; ks < 4 * TA; ++ks)
#pragma unroll
            for (int tb = 0; tb < TB; ++tb) {
                const int a = a0 + 4 * ks + kg, b = b0 + 16 * tb + i16;
                gf[ks][tb] = (a < N && b < N) ? Ge[(size_t)a * N + b] : (T)0;
            }
        double gr[32];
#pragma unroll
        for (int k = 0; k < 32; ++k) gr[k] = 0.0;

        for (int qc = 0; qc < NQ4; qc += 64) {
            const int cnt = NQ4 - qc < 64 ? NQ4 - qc : 64;     // multiple of 4
            for (int t4 = 0; t4 < cnt; t4 += 4) {
                const int q0 = qc + t4;
                double Sp[16];
#pragma unroll
                for (int k = 0; k < 16; ++k) Sp[k] = 0.0;
#pragma unroll
                for (int tb = 0; tb < TB; ++tb) {
                    const int b = b0 + 16 * tb + i16;
                    if (b0 + 16 * tb >= NP) continue;
                    V4 acc = V4{0, 0, 0, 0};
#pragma unroll
                    for (int ks = 0; ks < 4 * TA; ++ks) {
                        const int a = a0 + 4 * ks + kg;
                        if (a0 + 4 * ks < NP) {
                            const T af = BTt[(size_t)a * NQP * 4 + 4 * q0 + i16];
                            acc = mfma4(af, gf[ks][tb], acc);
                        }
                    }
#pragma unroll
                    for (int rr = 0; rr < 4; ++rr) {
                        const int row = acc_row<T>(lane, rr);   // (point q0 + row/4, r = row%4)
                        const int q = q0 + (row >> 2);
                        const T *bq = Br + (size_t)q * 4 * NP + b;
                        const double u = (double)acc[rr];
#pragma unroll
                        for (int s = 0; s < 4; ++s) Sp[4 * rr + s] += u * (double)bq[s * NP];
                    }
                }
                // reduce over the 16 columns held by lanes with the same kg
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    double v = Sp[k];
                    v += __shfl_xor(v, 1, 64);
                    v += __shfl_xor(v, 2, 64);
                    v += __shfl_xor(v, 4, 64);
                    v += __shfl_xor(v, 8, 64);
                    Sp[k] = v;
                }
                if (i16 == 0) {
#pragma unroll
                    for (int rr = 0; rr < 4; ++rr) {
                        const int row = acc_row<T>(lane, rr);
                        const int ql = t4 + (row >> 2), r = row & 3;
#pragma unroll
                        for (int s = 0; s < 4; ++s) sm.S[wave][ql][4 * r + s] = Sp[4 * rr + s];
                    }
                }
            }
            wave_sync();
            const int q = qc + lane;
            if (lane < cnt && q < NQ) {
                double S[16];
#pragma unroll
                for (int k = 0; k < 16; ++k) S[k] = sm.S[wave][lane][k];
                chain_rule(prm, E, q, S, with_load, e, gr);
            }
            wave_sync();
        }
        // reduce the 32 partial gradients over the wave
#pragma unroll
        for (int k = 0; k < 32; ++k) {
            double v = gr[k];
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
            gr[k] = v;
        }
        if (lane == 0) {
            double *outs[5] = {prm.dX + 18 * e, prm.dD + 9 * e, prm.dbeta + 3 * e, prm.dc + e, prm.df + e};
            const int base[5] = {0, 18, 27, 30, 31}, len[5] = {18, 9, 3, 1, 1};
#pragma unroll
            for (int o = 0; o < 5; ++o)
                for (int k = 0; k < len[o]; ++k) {
                    if (ATOMIC) atomicAdd(outs[o] + k, gr[base[o] + k]);
                    else outs[o][k] = gr[base[o] + k];
                }
        }
    }
};

template <class KER>
__global__ __launch_bounds__(256) void adj_direct(AdjParams prm) {
    __shared__ typename KER::Smem sm;
    const int wave = wave_uniform(threadIdx.x >> 6);
    const int64_t item = (int64_t)blockIdx.x * 4 + wave;
    if (item >= prm.ne * KER::NBLK) return;
    KER::run(prm, item / KER::NBLK, (int)(item % KER::NBLK), wave, sm);
}

__global__ void zero_f64(double *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

namespace {

template <class KER>
feint_status launch_adj(const AdjParams &prm, hipStream_t s) {
    if (KER::ATOMIC) {
        double *outs[5] = {prm.dX, prm.dD, prm.dbeta, prm.dc, prm.df};
        const int64_t len[5] = {18, 9, 3, 1, 1};
        for (int o = 0; o < 5; ++o) {
            const int64_t n = prm.ne * len[o];
            hipLaunchKernelGGL(zero_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, outs[o], n);
        }
    }
    const int64_t blocks = (prm.ne * KER::NBLK + 3) / 4;
    if (blocks > 0x7fffffffLL) return FEINT_ERR_TOO_LARGE;
    hipLaunchKernelGGL(adj_direct<KER>, dim3((unsigned)blocks), dim3(256), 0, s, prm);
    return FEINT_OK;
}

template <typename T>
feint_status dispatch_adj(int p, const AdjParams &prm, hipStream_t s) {
    switch (p) {
    case 1: return launch_adj<Adj<1, T, 1, 1>>(prm, s);
    case 2: return launch_adj<Adj<2, T, 2, 2>>(prm, s);
    case 3: return launch_adj<Adj<3, T, 3, 3>>(prm, s);
    case 4: return launch_adj<Adj<4, T, 5, 2>>(prm, s);
    case 5: return launch_adj<Adj<5, T, 4, 2>>(prm, s);
    case 6: return launch_adj<Adj<6, T, 4, 2>>(prm, s);
    case 7: return launch_adj<Adj<7, T, 3, 3>>(prm, s);
    }
    return FEINT_ERR_UNSUPPORTED_DEGREE;
}

}  // namespace
}  // namespace feint

using namespace feint;

extern "C" feint_status feint_integrate_adjoint(const feint_elements *el, int p, feint_form form, const void *G,
                                                const void *g, double *dcoords, double *dD, double *dbeta,
                                                double *dc, double *df, void *stream) {
    if (p < 1 || p > kMaxP) return FEINT_ERR_UNSUPPORTED_DEGREE;
    if (form != FEINT_FP64 && form != FEINT_FP32) return FEINT_ERR_UNSUPPORTED_FORM;
    feint_status s = check_elements(el);
    if (s != FEINT_OK) return s;
    if (el->ne == 0) return FEINT_OK;
    if (!G || !g || !dcoords || !dD || !dbeta || !dc || !df) return FEINT_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    const DevTables *T = nullptr;
    s = tables_for_launch(p, st, &T);
    if (s != FEINT_OK) return s;
    AdjParams prm;
    std::memset(&prm, 0, sizeof prm);
    prm.coords = el->coords; prm.D = el->D; prm.beta = el->beta; prm.c = el->c; prm.f = el->f;
    prm.ne = el->ne;
    prm.G = G; prm.g = g;
    prm.dX = dcoords; prm.dD = dD; prm.dbeta = dbeta; prm.dc = dc; prm.df = df;
    prm.qw = T->qw; prm.B64 = T->B64;
    prm.Brow = form == FEINT_FP64 ? (const void *)T->B64 : (const void *)T->B32;
    prm.BT = form == FEINT_FP64 ? (const void *)T->BT64 : (const void *)T->BT32;
    (void)hipGetLastError();
    s = form == FEINT_FP64 ? dispatch_adj<double>(p, prm, st) : dispatch_adj<float>(p, prm, st);
    if (s != FEINT_OK) return s;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error("adjoint launch", e); return FEINT_ERR_HIP; }
    return FEINT_OK;
}
