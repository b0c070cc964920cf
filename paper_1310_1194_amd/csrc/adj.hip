// Adjoint of the forward integration: gradients of
//     L = sum_e <G_e, A_e> + <g_e, b_e>
// with respect to every element's vertices, D, beta, c and f.
//
// Since A_e = sum_q B_q^T W_q B_q, <G_e, A_e> = sum_q <W_q, S_q> with the 4x4
// block S_q = B_q G_e B_q^T.  Per group of four points the kernel forms, on
// MFMA, the 16 rows (point, row) of U^T = G_e^T B^T (K = shape functions a)
// and then T = U B^T over the same four points (K = shape functions b): the
// accumulator registers of a U^T tile are, lane for lane, the A operand of
// the second product, so U never leaves registers.  The diagonal 4x4 blocks
// of T are the S_q of the four points (a quarter of T is used; the second
// product costs 4 MFMAs per 16x16 tile of U^T).  Then, one point per lane,
// the Jacobian is recomputed in FP64 and dL/dW_q = S_q is pushed through
//   W_q = w det J [[c, (K beta)^T], [0, K D K^T]],  K = J^{-1}:
//   dL/dc = sum wd S00,  dL/dbeta = sum wd K^T s,  dL/dD = sum wd K^T S' K,
//   dL/dK = wd (S' K D^T + S'^T K D + s beta^T),  dL/d det = L_q / det,
//   dL/dJ = L_q K^T - K^T (dL/dK) K^T,  then the bilinear map to the vertices
// (s = S[0,1:3], S' = S[1:3,1:3]).  Per-point Jacobians are never stored.
// All of it is linear in S_q, so for large degrees G_e is split into blocks
// handled by different waves whose partial gradients are summed atomically.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <mutex>

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
    const void *BT;     // [npad][nqp*4]  in the form's precision
    const void *tau;    // triangle factors [nij][4][tpad] and line factors [4][p+1][p+1],
    const void *lamT;   // both in the form's precision
};

template <int P, typename T, int TA, int TB, int R = 0>
struct Adj {
    static constexpr int N = c_nshp(P), NP = c_pad16(N), NT = NP / 16, NQ = c_nq_rule(P, R);
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

    // Sum the lanes' 32 partial gradients over the wave by recursive halving:
    // at each step a lane keeps half of its values and adds the partner's copy
    // of that half.  Lanes 2c and 2c+1 end with component c.
    __device__ static double reduce_scatter32(double v[32], int lane) {
        double w16[16], w8[8], w4[4], w2[2];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const bool up = lane & 32;
            const double keep = up ? v[j + 16] : v[j], send = up ? v[j] : v[j + 16];
            w16[j] = keep + __shfl_xor(send, 32, 64);
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const bool up = lane & 16;
            const double keep = up ? w16[j + 8] : w16[j], send = up ? w16[j] : w16[j + 8];
            w8[j] = keep + __shfl_xor(send, 16, 64);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const bool up = lane & 8;
            const double keep = up ? w8[j + 4] : w8[j], send = up ? w8[j] : w8[j + 4];
            w4[j] = keep + __shfl_xor(send, 8, 64);
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const bool up = lane & 4;
            const double keep = up ? w4[j + 2] : w4[j], send = up ? w4[j] : w4[j + 2];
            w2[j] = keep + __shfl_xor(send, 4, 64);
        }
        const bool up = lane & 2;
        double r = (up ? w2[1] : w2[0]) + __shfl_xor(up ? w2[0] : w2[1], 2, 64);
        return r + __shfl_xor(r, 1, 64);
    }

    __device__ static void run(const AdjParams &prm, int64_t e, int blk, int wave, Smem &sm) {
        const int lane = threadIdx.x & 63;
        const int i16 = lane & 15, kg = lane >> 4;
        const int ba = blk / BB, bb = blk % BB;
        const int a0 = ba * TA * 16, b0 = bb * TB * 16;
        const bool with_load = blk == 0;
        const T *Ge = (const T *)prm.G + e * (int64_t)N * N;
        const T *BTt = (const T *)prm.BT;
        // A-operand fragments of G^T over this wave's block:
        // lane (i16, kg) holds G[a0 + 4 ks + kg][b0 + 16 tb + i16]
        T gf[4 * TA][TB];
#pragma unroll
        for (int ks = 0; ks < 4 * TA; ++ks)
#pragma unroll
            for (int tb = 0; tb < TB; ++tb) {
                const int a = a0 + 4 * ks + kg, b = b0 + 16 * tb + i16;
                gf[ks][tb] = (a < N && b < N) ? Ge[(size_t)a * N + b] : (T)0;
            }
        const int nks = wave_uniform(N - a0 >= 16 * TA ? 4 * TA : (N - a0 + 3) / 4);   // k-steps with a < N
        const T *afp = BTt + (size_t)(a0 + kg) * NQP * 4 + i16;      // + 4 ks NQP*4 + 4 q0
        double gacc = 0.0;          // lanes 2c, 2c+1: component c of this wave's gradient

        // table operands of one group of four points: B^T rows a (MFMA 1) and b (MFMA 2)
        T af[4 * TA], bt[TB][4];
        auto fetch = [&](int q0, T (&fa)[4 * TA], T (&fb)[TB][4]) {
#pragma unroll
            for (int ks = 0; ks < 4 * TA; ++ks)
                fa[ks] = ks < nks ? afp[(size_t)4 * ks * NQP * 4 + 4 * q0] : (T)0;
#pragma unroll
            for (int tb = 0; tb < TB; ++tb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int b = b0 + 16 * tb + acc_row<T>(lane, r);
                    fb[tb][r] = b0 + 16 * tb < N ? BTt[(size_t)b * NQP * 4 + 4 * q0 + i16] : (T)0;
                }
        };
        fetch(0, af, bt);
        for (int qc = 0; qc < NQ4; qc += 64) {
            const int cnt = NQ4 - qc < 64 ? NQ4 - qc : 64;     // multiple of 4
            for (int t4 = 0; t4 < cnt; t4 += 4) {
                // operands of the next group are loaded while this one runs
                T afn[4 * TA], btn[TB][4];
                const int qn = qc + t4 + 4;
                if (qn < NQ4) fetch(qn, afn, btn);
                V4 tacc = V4{0, 0, 0, 0};
#pragma unroll
                for (int tb = 0; tb < TB; ++tb) {
                    if (b0 + 16 * tb >= N) continue;
                    V4 u = V4{0, 0, 0, 0};                 // U^T tile: rows b, columns (point, row)
#pragma unroll
                    for (int ks = 0; ks < 4 * TA; ++ks)
                        if (ks < nks) u = mfma4(gf[ks][tb], af[ks], u);
                    // T += U B^T: k-step r covers the rows b held in register r
#pragma unroll
                    for (int r = 0; r < 4; ++r) tacc = mfma4((T)u[r], bt[tb][r], tacc);
                }
                // diagonal blocks of T: row (point, r), column (point', s) with point = point'
                if (sizeof(T) == 8) {
                    // lane holds rows 4 rr + kg: point rr, r = kg; column i16: point i16/4, s = i16%4
                    const int pt = i16 >> 2;
                    const double v = pt == 0 ? tacc[0] : pt == 1 ? tacc[1] : pt == 2 ? tacc[2] : tacc[3];
                    sm.S[wave][t4 + pt][4 * kg + (i16 & 3)] = v;
                } else if (kg == (i16 >> 2)) {
                    // lane holds rows 4 kg + rr: point kg, r = rr
#pragma unroll
                    for (int rr = 0; rr < 4; ++rr) sm.S[wave][t4 + kg][4 * rr + (i16 & 3)] = (double)tacc[rr];
                }
                if (qn < NQ4) {
#pragma unroll
                    for (int ks = 0; ks < 4 * TA; ++ks) af[ks] = afn[ks];
#pragma unroll
                    for (int tb = 0; tb < TB; ++tb)
#pragma unroll
                        for (int r = 0; r < 4; ++r) bt[tb][r] = btn[tb][r];
                }
            }
            wave_sync();
            {
                // chain rule, one point per lane (element inputs re-read: they are
                // not kept in registers across the MFMA loop)
                ElemIn E;
                load_elem(prm.coords, prm.D, prm.beta, prm.c, prm.f, e, E);
                double gr[32];
#pragma unroll
                for (int k = 0; k < 32; ++k) gr[k] = 0.0;
                const int q = qc + lane;
                if (lane < cnt && q < NQ) {
                    double S[16];
#pragma unroll
                    for (int k = 0; k < 16; ++k) S[k] = sm.S[wave][lane][k];
                    chain_rule(prm, E, q, S, with_load, e, gr);
                }
                gacc += reduce_scatter32(gr, lane);
            }
            wave_sync();
        }
        if ((lane & 1) == 0) {
            // component c: vertices 0..17, D 18..26, beta 27..29, c 30, f 31
            const int c = lane >> 1;
            double *dst = c < 18 ? prm.dX + 18 * e + c
                        : c < 27 ? prm.dD + 9 * e + (c - 18)
                        : c < 30 ? prm.dbeta + 3 * e + (c - 27)
                        : c == 30 ? prm.dc + e : prm.df + e;
            if (ATOMIC) atomicAdd(dst, gacc);
            else *dst = gacc;
        }
    }
};

// The adjoint factorised along zeta.  Both prism rules are products of nij
// triangle points and p+1 points in zeta and B_q[r][(k,t)] = tau_r(t, ij)
// lam_r(k, m) (tau = (T, dT/dxi1, dT/dxi2, T), lam = (L, L, L, dL/dzeta)), so
//   S_q[r][s] = sum_b Hh_q[r][b] B_q[s][b],
//   Hh_(ij,m)[r][b] = sum_k lam_r(k, m) H_k[b][(ij, r)],
//   H_k[b][(ij, r)] = sum_t G[(k,t)][b] tau_r(t, ij).
// Per group of four triangle points a wave forms H_k on MFMA (rows b of its
// column tiles, columns (triangle point, r), K = t) for its row indices k,
// combines them into Hh for each zeta point m on the vector ALUs (p+1 FMAs
// per value), and feeds Hh register by register as the A operand of
// T = Hh B^T over its columns b (K = b, 4 MFMAs per column tile); the
// diagonal 4x4 blocks of T are the (partial) S_q of the group's points at m.
// Column tiles are (k', t'-tile) pairs, so the line factor of a column tile is
// the same for the whole wave.  The chain rule is the point-by-point kernel's.
template <int P, typename T, int TK, int TB, int R = 0>
struct KFA {
    typedef Adj<P, T, 1, 1, R> Base;
    static constexpr int N = c_nshp(P), NQ = c_nq_rule(P, R);
    static constexpr int NK = P + 1, NTRI = (P + 1) * (P + 2) / 2, TT = c_cdiv(NTRI, 16), TP = TT * 16;
    static constexpr int KS = c_cdiv(NTRI, 4);              // K-steps over t
    static constexpr int NIJ = NQ / NK, NCT = NK * TT;        // column tiles (k', t'-tile)
    static constexpr int CIJ = 64 / NK / 4 * 4;               // triangle points per chunk (groups of 4)
    static constexpr int BK = c_cdiv(NK, TK), BB = c_cdiv(NCT, TB), NBLK = BK * BB;
    static constexpr bool ATOMIC = NBLK > 1;
    static_assert(NIJ * NK == NQ, "the rule must be a product in zeta");
    static_assert(CIJ >= 4, "a chunk holds at least one group of four triangle points");
    typedef typename AccT<T>::type V4;
    typedef const __attribute__((address_space(4))) T CT;

    struct Smem { double S[4][64][WROW<double>::value]; };

    __device__ static void run(const AdjParams &prm, int64_t e, int blk, int wave, Smem &sm) {
        const int lane = threadIdx.x & 63;
        const int i16 = lane & 15, kg = lane >> 4;
        const int bk = blk / BB, bc = blk % BB;
        const int k0 = bk * TK, c0 = bc * TB;
        const bool with_load = blk == 0;
        const T *Ge = (const T *)prm.G + e * (int64_t)N * N;
        const T *tau = (const T *)prm.tau;
        const CT *lam = (const CT *)prm.lamT;                 // [s][k][m], wave-uniform reads
        // A operands of H_k: lane (i16, kg) holds G[(k, t = 4 s + kg)][(k'_c, t' = 16 tt_c + i16)]
        T gf[TK][KS][TB];
#pragma unroll
        for (int k = 0; k < TK; ++k)
#pragma unroll
            for (int s = 0; s < KS; ++s)
#pragma unroll
                for (int tb = 0; tb < TB; ++tb) {
                    const int c = c0 + tb, kp = c / TT, tp = (c % TT) * 16 + i16, t = 4 * s + kg;
                    gf[k][s][tb] = (k0 + k < NK && c < NCT && t < NTRI && tp < NTRI)
                                       ? Ge[(size_t)((k0 + k) * NTRI + t) * N + kp * NTRI + tp] : (T)0;
                }
        const bool rl = (i16 & 3) == 3;     // this lane's column (point, r) has r = 3: the zeta derivative
        double gacc = 0.0;
        for (int ij0 = 0; ij0 < NIJ; ij0 += CIJ) {
            const int cij = NIJ - ij0 < CIJ ? NIJ - ij0 : CIJ;
            for (int g4 = 0; g4 < cij; g4 += 4) {
                const int ijc = ij0 + g4 + (i16 >> 2);          // the triangle point of this lane's column
                const bool ijok = ijc < NIJ;
                // H_k over K = t: B operands tau_r(t = 4 s + kg, ij) at column (point, r) = i16
                V4 h[TK][TB];
#pragma unroll
                for (int k = 0; k < TK; ++k)
#pragma unroll
                    for (int tb = 0; tb < TB; ++tb) h[k][tb] = V4{0, 0, 0, 0};
#pragma unroll
                for (int s = 0; s < KS; ++s) {
                    const T tv = ijok ? tau[((size_t)ijc * 4 + (i16 & 3)) * TP + 4 * s + kg] : (T)0;
#pragma unroll
                    for (int k = 0; k < TK; ++k)
#pragma unroll
                        for (int tb = 0; tb < TB; ++tb) h[k][tb] = mfma4(gf[k][s][tb], tv, h[k][tb]);
                }
                // B operands of T at K-step j: tau_s(t' of row j of the column tile, ij), s = i16 % 4
                T tb4[TB][4];
#pragma unroll
                for (int tb = 0; tb < TB; ++tb)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int tp = ((c0 + tb) % TT) * 16 + acc_row<T>(lane, j);
                        tb4[tb][j] = ijok ? tau[((size_t)ijc * 4 + (i16 & 3)) * TP + tp] : (T)0;
                    }
                for (int m = 0; m < NK; ++m) {
                    V4 tacc = V4{0, 0, 0, 0};
#pragma unroll
                    for (int tb = 0; tb < TB; ++tb) {
                        if (c0 + tb >= NCT) continue;
                        const int kp = (c0 + tb) / TT;
                        const T lb = rl ? lam[(size_t)(3 * NK + kp) * NK + m] : lam[(size_t)kp * NK + m];
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            T hh = (T)0;
#pragma unroll
                            for (int k = 0; k < TK; ++k) {
                                if (k0 + k >= NK) continue;
                                const T lr = rl ? lam[(size_t)(3 * NK + k0 + k) * NK + m] : lam[(size_t)(k0 + k) * NK + m];
                                hh += lr * h[k][tb][j];
                            }
                            tacc = mfma4(hh, tb4[tb][j] * lb, tacc);
                        }
                    }
                    // diagonal blocks: row (point, r), column (point', s), point = point'
                    const int pl = g4 + (i16 >> 2);             // chunk-local triangle point of this lane's column
                    if (sizeof(T) == 8) {
                        // lane holds rows 4 jj + kg: point jj, r = kg
                        const int pt = i16 >> 2;
                        const double v = pt == 0 ? tacc[0] : pt == 1 ? tacc[1] : pt == 2 ? tacc[2] : tacc[3];
                        if (pl < cij) sm.S[wave][pl * NK + m][4 * kg + (i16 & 3)] = v;
                    } else if (kg == (i16 >> 2)) {
                        // lane holds rows 4 kg + jj: point kg, r = jj
                        if (pl < cij) {
#pragma unroll
                            for (int jj = 0; jj < 4; ++jj) sm.S[wave][pl * NK + m][4 * jj + (i16 & 3)] = (double)tacc[jj];
                        }
                    }
                }
            }
            wave_sync();
            {
                ElemIn E;
                load_elem(prm.coords, prm.D, prm.beta, prm.c, prm.f, e, E);
                double gr[32];
#pragma unroll
                for (int k = 0; k < 32; ++k) gr[k] = 0.0;
                if (lane < cij * NK) {
                    const int il = lane / NK, m = lane - il * NK;
                    const int q = m * NIJ + ij0 + il;
                    double S[16];
#pragma unroll
                    for (int k = 0; k < 16; ++k) S[k] = sm.S[wave][lane][k];
                    Base::chain_rule(prm, E, q, S, with_load, e, gr);
                }
                gacc += Base::reduce_scatter32(gr, lane);
            }
            wave_sync();
        }
        if ((lane & 1) == 0) {
            const int c = lane >> 1;
            double *dst = c < 18 ? prm.dX + 18 * e + c
                        : c < 27 ? prm.dD + 9 * e + (c - 18)
                        : c < 30 ? prm.dbeta + 3 * e + (c - 27)
                        : c == 30 ? prm.dc + e : prm.df + e;
            if (ATOMIC) atomicAdd(dst, gacc);
            else *dst = gacc;
        }
    }
};

// The same adjoint with the chain rule taken once per point: where the
// element has two blocks a workgroup of four waves takes two elements, two
// waves each, otherwise one element and its four waves take the blocks in
// turn.  Each block's share of S_q is added into one LDS array of the
// element's points (LDS atomics: the blocks' shares of a point come from
// different waves), the workgroup synchronises, and the chain rule then runs
// once per point on the element's waves, where the blocks of the one-wave
// kernel each run it on their share.  The 32 gradient components are summed
// across the element's waves through LDS and written by one wave: no atomics
// in global memory.
template <int P, typename T, int TK, int TB, int R = 0>
struct KFA2 {
    typedef KFA<P, T, TK, TB, R> F;
    typedef typename F::Base Base;
    static constexpr int N = F::N, NQ = F::NQ, NK = F::NK, NTRI = F::NTRI, TT = F::TT, TP = F::TP, KS = F::KS;
    static constexpr int NIJ = F::NIJ, NCT = F::NCT, BB = F::BB, NB = F::NBLK;
    static constexpr int WPE = NB == 2 ? 2 : 4;    // waves per element
    static constexpr int EPW = 4 / WPE;            // elements per workgroup
    static constexpr int NBLK = WPE;               // work items per element: its waves
    static constexpr int SR = 17;                  // row stride of S (doubles)
    typedef typename AccT<T>::type V4;
    typedef const __attribute__((address_space(4))) T CT;

    struct Smem {
        double S[EPW][NQ][SR];                     // per element: S_q[r][s] at 4 r + s
        double red[4][32];
    };

    __device__ static void run_coop(const AdjParams &prm, int64_t e, int wv, int wave, bool live, Smem &sm) {
        const int lane = threadIdx.x & 63;
        const int i16 = lane & 15, kg = lane >> 4;
        const int el = wave / WPE;                 // the element's area in this workgroup
        for (int i = threadIdx.x; i < EPW * NQ * SR; i += 256) (&sm.S[0][0][0])[i] = 0.0;
        __syncthreads();
        if (live) {
            const T *Ge = (const T *)prm.G + e * (int64_t)N * N;
            const T *tau = (const T *)prm.tau;
            const CT *lam = (const CT *)prm.lamT;
            const bool rl = (i16 & 3) == 3;
            for (int blk = wv; blk < NB; blk += WPE) {
                const int bk = blk / BB, bc = blk % BB;
                const int k0 = bk * TK, c0 = bc * TB;
                T gf[TK][KS][TB];
#pragma unroll
                for (int k = 0; k < TK; ++k)
#pragma unroll
                    for (int st = 0; st < KS; ++st)
#pragma unroll
                        for (int tb = 0; tb < TB; ++tb) {
                            const int c = c0 + tb, kp = c / TT, tp = (c % TT) * 16 + i16, t = 4 * st + kg;
                            gf[k][st][tb] = (k0 + k < NK && c < NCT && t < NTRI && tp < NTRI)
                                                ? Ge[(size_t)((k0 + k) * NTRI + t) * N + kp * NTRI + tp] : (T)0;
                        }
                for (int g4 = 0; g4 < NIJ; g4 += 4) {
                    const int ijc = g4 + (i16 >> 2);
                    const bool ijok = ijc < NIJ;
                    V4 h[TK][TB];
#pragma unroll
                    for (int k = 0; k < TK; ++k)
#pragma unroll
                        for (int tb = 0; tb < TB; ++tb) h[k][tb] = V4{0, 0, 0, 0};
#pragma unroll
                    for (int st = 0; st < KS; ++st) {
                        const T tv = ijok ? tau[((size_t)ijc * 4 + (i16 & 3)) * TP + 4 * st + kg] : (T)0;
#pragma unroll
                        for (int k = 0; k < TK; ++k)
#pragma unroll
                            for (int tb = 0; tb < TB; ++tb) h[k][tb] = mfma4(gf[k][st][tb], tv, h[k][tb]);
                    }
                    T tb4[TB][4];
#pragma unroll
                    for (int tb = 0; tb < TB; ++tb)
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const int tp = ((c0 + tb) % TT) * 16 + acc_row<T>(lane, j);
                            tb4[tb][j] = ijok ? tau[((size_t)ijc * 4 + (i16 & 3)) * TP + tp] : (T)0;
                        }
                    for (int m = 0; m < NK; ++m) {
                        V4 tacc = V4{0, 0, 0, 0};
#pragma unroll
                        for (int tb = 0; tb < TB; ++tb) {
                            if (c0 + tb >= NCT) continue;
                            const int kp = (c0 + tb) / TT;
                            const T lb = rl ? lam[(size_t)(3 * NK + kp) * NK + m] : lam[(size_t)kp * NK + m];
#pragma unroll
                            for (int j = 0; j < 4; ++j) {
                                T hh = (T)0;
#pragma unroll
                                for (int k = 0; k < TK; ++k) {
                                    if (k0 + k >= NK) continue;
                                    const T lr = rl ? lam[(size_t)(3 * NK + k0 + k) * NK + m] : lam[(size_t)(k0 + k) * NK + m];
                                    hh += lr * h[k][tb][j];
                                }
                                tacc = mfma4(hh, tb4[tb][j] * lb, tacc);
                            }
                        }
                        // the diagonal 4x4 blocks (point = point') are this block's share of S_q
                        if (ijok) {
                            const int q = m * NIJ + ijc;
                            if (sizeof(T) == 8) {
                                const int pt = i16 >> 2;        // lane holds rows 4 jj + kg: point jj, r = kg
                                const double v = pt == 0 ? tacc[0] : pt == 1 ? tacc[1] : pt == 2 ? tacc[2] : tacc[3];
                                atomicAdd(&sm.S[el][q][4 * kg + (i16 & 3)], v);
                            } else if (kg == (i16 >> 2)) {     // lane holds rows 4 kg + jj: point kg, r = jj
#pragma unroll
                                for (int jj = 0; jj < 4; ++jj) atomicAdd(&sm.S[el][q][4 * jj + (i16 & 3)], (double)tacc[jj]);
                            }
                        }
                    }
                }
            }
        }
        __syncthreads();
        if (live) {
            ElemIn E;
            load_elem(prm.coords, prm.D, prm.beta, prm.c, prm.f, e, E);
            double gacc = 0.0;
            for (int q0 = wv * 64; q0 < NQ; q0 += WPE * 64) {
                double gr[32];
#pragma unroll
                for (int k = 0; k < 32; ++k) gr[k] = 0.0;
                const int q = q0 + lane;
                if (q < NQ) {
                    double S[16];
#pragma unroll
                    for (int k = 0; k < 16; ++k) S[k] = sm.S[el][q][k];
                    Base::chain_rule(prm, E, q, S, true, e, gr);
                }
                gacc += Base::reduce_scatter32(gr, lane);
            }
            if ((lane & 1) == 0) sm.red[wave][lane >> 1] = gacc;
        }
        __syncthreads();
        if (live && wv == 0 && lane < 32) {
            // component c: vertices 0..17, D 18..26, beta 27..29, c 30, f 31
            const int c = lane;
            double g = 0.0;
#pragma unroll
            for (int w = 0; w < WPE; ++w) g += sm.red[el * WPE + w][c];
            double *dst = c < 18 ? prm.dX + 18 * e + c
                        : c < 27 ? prm.dD + 9 * e + (c - 18)
                        : c < 30 ? prm.dbeta + 3 * e + (c - 27)
                        : c == 30 ? prm.dc + e : prm.df + e;
            *dst = g;
        }
    }
};

template <class KER, int MINW = 1>
__global__ __launch_bounds__(256, MINW) void adj_direct(AdjParams prm) {
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

template <class KER, int MINW = 1>
__global__ __launch_bounds__(256, MINW) void adj_coop(AdjParams prm) {
    __shared__ typename KER::Smem sm;
    const int wave = wave_uniform(threadIdx.x >> 6);
    const int64_t item = (int64_t)blockIdx.x * 4 + wave;
    const bool live = item < prm.ne * KER::NBLK;     // the same for the four waves of an element
    KER::run_coop(prm, item / KER::NBLK, (int)(item % KER::NBLK), wave, live, sm);
}

template <class KER, int MINW = 1>
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
    hipLaunchKernelGGL((adj_direct<KER, MINW>), dim3((unsigned)blocks), dim3(256), 0, s, prm);
    return FEINT_OK;
}

// one workgroup per element, every wave of it reaching the barriers
template <class KER, int MINW = 1>
feint_status launch_adj_coop(const AdjParams &prm, hipStream_t s) {
    const int64_t blocks = (prm.ne * KER::NBLK + 3) / 4;
    if (blocks > 0x7fffffffLL) return FEINT_ERR_TOO_LARGE;
    hipLaunchKernelGGL((adj_coop<KER, MINW>), dim3((unsigned)blocks), dim3(256), 0, s, prm);
    return FEINT_OK;
}

// Compiled block shapes (TA x TB 16x16 tiles of G per wave, or for the
// factorised kernel TK row indices k by TB column tiles) per degree and
// quadrature rule (the same shapes for both rules, so one choice per (degree,
// form) serves both); the first is the default until feint_adjoint_autotune
// picks another.
struct AdjVariant {
    int ta, tb;
    feint_status (*launch)(const AdjParams &, hipStream_t);
    int fact;           // 1: factorised along zeta (KFA, TA = row indices k, TB = column tiles),
                        // 2: the same with a two-waves-per-SIMD register budget, 3 (4): the same with
                        // the chain rule shared by the waves of an element (KFA2; 4 at two waves per SIMD)
};
#define FEINT_ADJ(P, T, TA, TB) AdjVariant{TA, TB, &launch_adj<Adj<P, T, TA, TB, R>>, 0}
#define FEINT_ADJF(P, T, TK, TB) AdjVariant{TK, TB, &launch_adj<KFA<P, T, TK, TB, R>>, 1}
#define FEINT_ADJF2(P, T, TK, TB) AdjVariant{TK, TB, &launch_adj<KFA<P, T, TK, TB, R>, 2>, 2}
#define FEINT_ADJW(P, T, TK, TB) AdjVariant{TK, TB, &launch_adj_coop<KFA2<P, T, TK, TB, R>>, 3}
#define FEINT_ADJW2(P, T, TK, TB) AdjVariant{TK, TB, &launch_adj_coop<KFA2<P, T, TK, TB, R>, 2>, 4}

template <typename T, int R>
const AdjVariant *adj_variants_of(int p, int *count) {
    static const AdjVariant v1[] = {FEINT_ADJ(1, T, 1, 1), FEINT_ADJF(1, T, 2, 2)};
    static const AdjVariant v2[] = {FEINT_ADJ(2, T, 2, 2), FEINT_ADJ(2, T, 2, 1), FEINT_ADJF(2, T, 3, 3)};
    // from p = 3 the factorised kernel ("f", "fo2" with two waves per SIMD) first, in the
    // order measured per form (131072 elements at p = 3 and 4, 16384 at p = 5 and 7); the
    // same shapes for both forms; from p = 5 the one with the chain rule shared by the waves
    // of an element ("fw") first (p = 7: 1.4x FP64, 2.0x FP32), and in FP32 at p = 3 (two
    // waves per element, 1.1x); FP64 at p = 3 level, at p = 4 slower
    static const AdjVariant v3d[] = {FEINT_ADJF2(3, T, 4, 2), FEINT_ADJ(3, T, 3, 3), FEINT_ADJF(3, T, 4, 2),
                                     FEINT_ADJF(3, T, 4, 4), FEINT_ADJ(3, T, 3, 1), FEINT_ADJ(3, T, 3, 2),
                                     FEINT_ADJF2(3, T, 4, 1), FEINT_ADJW2(3, T, 4, 2)};
    static const AdjVariant v3f[] = {FEINT_ADJW2(3, T, 4, 2), FEINT_ADJF2(3, T, 4, 2), FEINT_ADJF(3, T, 4, 4),
                                     FEINT_ADJF(3, T, 4, 2), FEINT_ADJ(3, T, 3, 3), FEINT_ADJ(3, T, 3, 1),
                                     FEINT_ADJ(3, T, 3, 2), FEINT_ADJF2(3, T, 4, 1)};
    static const AdjVariant v4[] = {FEINT_ADJF2(4, T, 5, 1), FEINT_ADJF(4, T, 5, 1), FEINT_ADJF(4, T, 5, 2),
                                    FEINT_ADJ(4, T, 5, 2), FEINT_ADJ(4, T, 5, 1), FEINT_ADJ(4, T, 3, 3),
                                    FEINT_ADJW(4, T, 5, 1)};
    static const AdjVariant v5d[] = {FEINT_ADJW(5, T, 6, 1), FEINT_ADJF(5, T, 6, 2), FEINT_ADJF(5, T, 6, 1), FEINT_ADJ(5, T, 8, 2),
                                     FEINT_ADJ(5, T, 4, 2), FEINT_ADJ(5, T, 8, 1)};
    static const AdjVariant v5f[] = {FEINT_ADJW(5, T, 6, 1), FEINT_ADJF(5, T, 6, 1), FEINT_ADJF(5, T, 6, 2), FEINT_ADJ(5, T, 8, 2),
                                     FEINT_ADJ(5, T, 4, 2), FEINT_ADJ(5, T, 8, 1)};
    static const AdjVariant v6[] = {FEINT_ADJW(6, T, 7, 1), FEINT_ADJF(6, T, 7, 1), FEINT_ADJF(6, T, 4, 2), FEINT_ADJ(6, T, 7, 2),
                                    FEINT_ADJ(6, T, 7, 1), FEINT_ADJ(6, T, 13, 1)};
    static const AdjVariant v7d[] = {FEINT_ADJW(7, T, 8, 1), FEINT_ADJF(7, T, 8, 1), FEINT_ADJF(7, T, 4, 2), FEINT_ADJ(7, T, 6, 3),
                                     FEINT_ADJ(7, T, 9, 2), FEINT_ADJ(7, T, 6, 2), FEINT_ADJ(7, T, 9, 1)};
    static const AdjVariant v7f[] = {FEINT_ADJW(7, T, 8, 1), FEINT_ADJF(7, T, 8, 1), FEINT_ADJF(7, T, 4, 2), FEINT_ADJ(7, T, 6, 2),
                                     FEINT_ADJ(7, T, 9, 2), FEINT_ADJ(7, T, 6, 3), FEINT_ADJ(7, T, 9, 1)};
    static_assert(sizeof v3d == sizeof v3f && sizeof v5d == sizeof v5f && sizeof v7d == sizeof v7f,
                  "one count per degree for both forms");
    const bool f64 = sizeof(T) == 8;
#define FEINT_AN(a) *count = (int)(sizeof(a) / sizeof(a[0])); return a
    switch (p) {
    case 1: FEINT_AN(v1);
    case 2: FEINT_AN(v2);
    case 3: *count = (int)(sizeof(v3d) / sizeof(v3d[0])); return f64 ? v3d : v3f;
    case 4: FEINT_AN(v4);
    case 5: *count = (int)(sizeof(v5d) / sizeof(v5d[0])); return f64 ? v5d : v5f;
    case 6: FEINT_AN(v6);
    case 7: *count = (int)(sizeof(v7d) / sizeof(v7d[0])); return f64 ? v7d : v7f;
    }
#undef FEINT_AN
    *count = 0;
    return nullptr;
}

const AdjVariant *adj_variants(int form, int p, int *count, int rule = 0) {
    if (form == FEINT_FP64) return rule ? adj_variants_of<double, 1>(p, count) : adj_variants_of<double, 0>(p, count);
    if (form == FEINT_FP32) return rule ? adj_variants_of<float, 1>(p, count) : adj_variants_of<float, 0>(p, count);
    *count = 0;
    return nullptr;
}

std::mutex g_adj_mu;
int g_adj_tile[8][2];                       // chosen variant per (p, form)

const AdjVariant *adj_chosen(int p, int form, int rule) {
    int cnt = 0;
    const AdjVariant *v = adj_variants(form, p, &cnt, rule);
    if (!v || cnt == 0) return nullptr;
    std::lock_guard<std::mutex> lk(g_adj_mu);
    const int t = g_adj_tile[p][form];
    return &v[(t >= 0 && t < cnt) ? t : 0];
}

feint_status adj_setup(const feint_elements *el, int p, feint_form form, const void *G, const void *g,
                       double *dcoords, double *dD, double *dbeta, double *dc, double *df, hipStream_t st,
                       AdjParams &prm, int rule = 0) {
    if (p < 1 || p > kMaxP) return FEINT_ERR_UNSUPPORTED_DEGREE;
    if (form != FEINT_FP64 && form != FEINT_FP32) return FEINT_ERR_UNSUPPORTED_FORM;
    feint_status s = check_elements(el);
    if (s != FEINT_OK) return s;
    if (el->ne == 0) return FEINT_OK;
    if (!G || !g || !dcoords || !dD || !dbeta || !dc || !df) return FEINT_ERR_INVALID_ARG;
    const DevTables *T = nullptr;
    s = tables_for_launch(p, st, &T, rule);
    if (s != FEINT_OK) return s;
    std::memset(&prm, 0, sizeof prm);
    prm.coords = el->coords; prm.D = el->D; prm.beta = el->beta; prm.c = el->c; prm.f = el->f;
    prm.ne = el->ne;
    prm.G = G; prm.g = g;
    prm.dX = dcoords; prm.dD = dD; prm.dbeta = dbeta; prm.dc = dc; prm.df = df;
    prm.qw = T->qw; prm.B64 = T->B64;
    prm.BT = form == FEINT_FP64 ? (const void *)T->BT64 : (const void *)T->BT32;
    prm.tau = form == FEINT_FP64 ? (const void *)T->tau64 : (const void *)T->tau32;
    prm.lamT = form == FEINT_FP64 ? (const void *)T->lam : (const void *)T->lam32;
    return FEINT_OK;
}

feint_status adj_launch(const AdjVariant *v, const AdjParams &prm, hipStream_t st) {
    (void)hipGetLastError();
    feint_status s = v->launch(prm, st);
    if (s != FEINT_OK) return s;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error("adjoint launch", e); return FEINT_ERR_HIP; }
    return FEINT_OK;
}

}  // namespace
}  // namespace feint

using namespace feint;

extern "C" {

feint_status feint_integrate_adjoint(const feint_elements *el, int p, feint_form form, const void *G,
                                     const void *g, double *dcoords, double *dD, double *dbeta,
                                     double *dc, double *df, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    AdjParams prm;
    feint_status s = adj_setup(el, p, form, G, g, dcoords, dD, dbeta, dc, df, st, prm);
    if (s != FEINT_OK || el->ne == 0) return s;
    return adj_launch(adj_chosen(p, form, 0), prm, st);
}

feint_status feint_integrate_adjoint_rule(const feint_elements *el, int p, feint_form form, feint_rule rule,
                                          const void *G, const void *g, double *dcoords, double *dD,
                                          double *dbeta, double *dc, double *df, void *stream) {
    if (rule != FEINT_RULE_COLLAPSED && rule != FEINT_RULE_SYMMETRIC) return FEINT_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    AdjParams prm;
    feint_status s = adj_setup(el, p, form, G, g, dcoords, dD, dbeta, dc, df, st, prm, rule);
    if (s != FEINT_OK || el->ne == 0) return s;
    return adj_launch(adj_chosen(p, form, rule), prm, st);
}

int feint_adjoint_tile_count(int p, feint_form form) {
    int cnt = 0;
    if (p < 1 || p > kMaxP) return 0;
    adj_variants(form, p, &cnt);
    return cnt;
}

int feint_adjoint_tile_get(int p, feint_form form) {
    if (p < 1 || p > kMaxP || (form != FEINT_FP64 && form != FEINT_FP32)) return -1;
    std::lock_guard<std::mutex> lk(g_adj_mu);
    return g_adj_tile[p][form];
}

feint_status feint_adjoint_tile_set(int p, feint_form form, int tile) {
    if (p < 1 || p > kMaxP) return FEINT_ERR_UNSUPPORTED_DEGREE;
    if (form != FEINT_FP64 && form != FEINT_FP32) return FEINT_ERR_UNSUPPORTED_FORM;
    if (tile < 0 || tile >= feint_adjoint_tile_count(p, form)) return FEINT_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_adj_mu);
    g_adj_tile[p][form] = tile;
    return FEINT_OK;
}

feint_status feint_adjoint_tile_describe(int p, feint_form form, int tile, char *buf, size_t len) {
    if (p < 1 || p > kMaxP) return FEINT_ERR_UNSUPPORTED_DEGREE;
    if (form != FEINT_FP64 && form != FEINT_FP32) return FEINT_ERR_UNSUPPORTED_FORM;
    int cnt = 0;
    const AdjVariant *v = adj_variants(form, p, &cnt);
    if (!buf || len == 0 || tile < 0 || tile >= cnt) return FEINT_ERR_INVALID_ARG;
    std::snprintf(buf, len, "%dx%d%s%s", v[tile].ta, v[tile].tb,
                  v[tile].fact >= 3 ? "fw" : v[tile].fact ? "f" : "", v[tile].fact == 2 || v[tile].fact == 4 ? "o2" : "");
    return FEINT_OK;
}

feint_status feint_adjoint_autotune(const feint_elements *el, int p, feint_form form, const void *G,
                                    const void *g, double *dcoords, double *dD, double *dbeta, double *dc,
                                    double *df, int reps, double *best_ms, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    if (reps < 1 || (el && el->ne == 0)) return FEINT_ERR_INVALID_ARG;
    AdjParams prm;
    feint_status s = adj_setup(el, p, form, G, g, dcoords, dD, dbeta, dc, df, st, prm);
    if (s != FEINT_OK) return s;
    int cnt = 0;
    const AdjVariant *v = adj_variants(form, p, &cnt);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return FEINT_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return FEINT_ERR_HIP; }
    int best = 0;
    float best_t = 1e30f;
    // one launch of every variant first, so that the first ones timed do not
    // pay for the device settling (clocks, first launches) after other work
    for (int t = 0; t < cnt && s == FEINT_OK; ++t) s = adj_launch(&v[t], prm, st);
    for (int t = 0; t < cnt && s == FEINT_OK; ++t) {
        s = adj_launch(&v[t], prm, st);                     // warm-up
        if (s != FEINT_OK) break;
        (void)hipEventRecord(e0, st);
        for (int r = 0; r < reps && s == FEINT_OK; ++r) s = adj_launch(&v[t], prm, st);
        (void)hipEventRecord(e1, st);
        if (hipEventSynchronize(e1) != hipSuccess) { s = FEINT_ERR_HIP; break; }
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        ms /= reps;
        if (ms < best_t) { best_t = ms; best = t; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s != FEINT_OK) return s;
    {
        std::lock_guard<std::mutex> lk(g_adj_mu);
        g_adj_tile[p][form] = best;
    }
    if (best_ms) *best_ms = best_t;
    return FEINT_OK;
}

}  // extern "C"
