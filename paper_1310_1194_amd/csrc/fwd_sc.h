// Forward kernel that computes the shape functions at each point instead of
// reading them from precomputed tables: the paper's SC strategy (Sec. 4: the
// DD_SC and WF_SC variants compute shape functions and their derivatives in
// the point loop; the SR variants read them).  The paper builds
// them from monomials in the vertical and, separately, the horizontal
// direction combined by tensor-product rules; here the same tensor structure
// of the prism basis phi_a = T_t(xi1, xi2) L_k(zeta), a = k ntri + t, gives
// per point a short list of factors:
//   T_t and its two reference derivatives, t < ntri, by Silvester's product
//   of one-dimensional factors in the barycentric coordinates (the Lagrange
//   basis on the lattice (i/p, j/p), j outer, i inner), and
//   L_k and dL_k/dzeta, k <= p, the Lagrange basis on the Gauss-Lobatto nodes,
// and each entry of B_q is a product of two of them.
//
// Work decomposition as in the 16x16x4 kernel (K4): one wave owns a TM x TN
// block of 16x16 tiles of one element.  Per chunk of CH points each lane
// computes one point's W_q and factor list into the wave's LDS slice; then,
// point by point, the lane forms its MFMA A fragments (B rows of its TM
// shape functions, row kg) and its Y = W_q B_q column values (TN columns)
// from the factors.  No B table is read; the L2 traffic of the table is
// replaced by LDS reads and a few vector multiplies.
#pragma once
#include "fwd_kernels.h"

namespace feint {

template <int P>
struct ScLayout {
    static constexpr int NTRI = (P + 1) * (P + 2) / 2;
    static constexpr int OT = 0, OT1 = NTRI, OT2 = 2 * NTRI;      // T, dT/dxi1, dT/dxi2
    static constexpr int OL = 3 * NTRI, OLP = 3 * NTRI + P + 1;   // L, dL/dzeta
    static constexpr int NF = 3 * NTRI + 2 * (P + 1);
    static constexpr int FS = NF | 1;                             // odd row stride
};

// Factor list of one reference point into F (layout ScLayout<P>).  gll holds
// the Gauss-Lobatto nodes z_k and the reciprocals of prod_{m != k} (z_k - z_m).
template <int P, typename T>
__device__ inline void sc_factors(const double *gll, double xi1, double xi2, double ze, T *F) {
    typedef ScLayout<P> L;
    const double lam[3] = {1.0 - xi1 - xi2, xi1, xi2};
    double R[3][P + 1], dR[3][P + 1];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        // R_m(l) = prod_{s<m} (P l - s) / (s + 1)
        R[d][0] = 1.0;
        dR[d][0] = 0.0;
#pragma unroll
        for (int m = 1; m <= P; ++m) {
            const double g = (P * lam[d] - (m - 1)) / m, dg = (double)P / m;
            R[d][m] = R[d][m - 1] * g;
            dR[d][m] = dR[d][m - 1] * g + R[d][m - 1] * dg;
        }
    }
    int t = 0;
#pragma unroll
    for (int j = 0; j <= P; ++j)
#pragma unroll
        for (int i = 0; i <= P - j; ++i) {
            const int k = P - i - j;
            const double a = R[0][k], b = R[1][i], c = R[2][j];
            // lambda0 = 1 - xi1 - xi2, lambda1 = xi1, lambda2 = xi2
            F[L::OT + t] = (T)(a * b * c);
            F[L::OT1 + t] = (T)((-dR[0][k] * b + a * dR[1][i]) * c);
            F[L::OT2 + t] = (T)((-dR[0][k] * c + a * dR[2][j]) * b);
            ++t;
        }
#pragma unroll
    for (int k = 0; k <= P; ++k) {
        double v = gll[P + 1 + k], dv = 0.0;
#pragma unroll
        for (int m = 0; m <= P; ++m)
            if (m != k) {
                const double f = ze - gll[m];
                dv = dv * f + v;
                v *= f;
            }
        F[L::OL + k] = (T)v;
        F[L::OLP + k] = (T)dv;
    }
}

template <int P, typename T, int TM, int TN, int R = 0>
struct KSC {
    static constexpr int N = c_nshp(P), NP = c_pad16(N), NT = NP / 16, NQ = c_nq_rule(P, R);
    static constexpr int BM = c_cdiv(NT, TM), BN = c_cdiv(NT, TN), NBLK = BM * BN;
    static constexpr int EPI = 1;
    static constexpr int CH = 32;                      // points per chunk
    typedef typename AccT<T>::type V4;
    typedef LoadCol<P> LC;
    typedef ScLayout<P> SL;

    struct Slice {
        T W[CH][WROW<T>::value];
        double sf[CH];
        T F[CH][SL::FS];
    };
    struct Smem { Slice w[4]; };

    template <int TMV, int TNV>
    __device__ static void body(const FwdParams &prm, int64_t slot, int blk, int bi, int bj, Slice &sl) {
        constexpr int NBRV = c_cdiv(TMV * 16, 64);
        const int lane = threadIdx.x & 63;
        const int i16 = lane & 15, kg = lane >> 4;
        const int a0 = bi * TM * 16, b0 = bj * TN * 16;
        const int64_t e = elem_of(prm, slot);
        ElemIn E;
        load_elem_fwd(prm, e, E);
        // factor offsets of the lane's A-fragment entries (row kg of B for
        // shape function a) and of its Y columns; padded functions get a
        // zero multiplier
        int oa[TMV], ol[TMV], tyo[TNV], kyo[TNV];
        T ma[TMV], my[TNV];
#pragma unroll
        for (int ti = 0; ti < TMV; ++ti) {
            const int a = a0 + ti * 16 + i16;
            const int ac = a < N ? a : 0;
            const int t = ac % SL::NTRI, k = ac / SL::NTRI;
            oa[ti] = (kg == 1 ? SL::OT1 : kg == 2 ? SL::OT2 : SL::OT) + t;
            ol[ti] = (kg == 3 ? SL::OLP : SL::OL) + k;
            ma[ti] = a < N ? (T)1 : (T)0;
        }
#pragma unroll
        for (int tj = 0; tj < TNV; ++tj) {
            const int b = b0 + tj * 16 + i16;
            const int bc = b < N ? b : 0;
            tyo[tj] = bc % SL::NTRI;
            kyo[tj] = bc / SL::NTRI;
            my[tj] = b < N ? (T)1 : (T)0;
        }
        V4 acc[TMV][TNV];
#pragma unroll
        for (int ti = 0; ti < TMV; ++ti)
#pragma unroll
            for (int tj = 0; tj < TNV; ++tj) acc[ti][tj] = V4{0, 0, 0, 0};
        double bacc[NBRV];
#pragma unroll
        for (int m = 0; m < NBRV; ++m) bacc[m] = 0.0;

        for (int qc = 0; qc < NQ; qc += CH) {
            const int cnt = NQ - qc < CH ? NQ - qc : CH;
            if (lane < cnt) {
                const int q = qc + lane;
                const double *qp = prm.qw + 4 * q;
                double W[16], sf;
                field_at(prm, e, qp[0], qp[1], qp[2], E);
                const double det = point_block(E, qp[0], qp[1], qp[2], qp[3], W, sf);
                if (!(det > 0.0) && prm.status) atomicOr(prm.status, 1u);
#pragma unroll
                for (int k = 0; k < 16; ++k) sl.W[lane][k] = (T)W[k];
                sl.sf[lane] = sf;
                sc_factors<P, T>(prm.gll, qp[0], qp[1], qp[2], sl.F[lane]);
                if (prm.xq && blk == 0) {
                    double x[3];
                    prism_map(E.X, qp[0], qp[1], qp[2], x);
#pragma unroll
                    for (int d = 0; d < 3; ++d) prm.xq[(e * NQ + q) * 3 + d] = x[d];
                }
            }
            wave_sync();
            if (!LC::on && bj == 0) {
#pragma unroll
                for (int m = 0; m < NBRV; ++m) {
                    const int row = a0 + lane + 64 * m;
                    if (lane + 64 * m < TMV * 16 && row < N) {
                        const int t = row % SL::NTRI, k = row / SL::NTRI;
                        double s = 0.0;
                        for (int qq = 0; qq < cnt; ++qq)
                            s += sl.sf[qq] * ((double)sl.F[qq][SL::OT + t] * (double)sl.F[qq][SL::OL + k]);
                        bacc[m] += s;
                    }
                }
            }
            for (int qq = 0; qq < cnt; ++qq) {
                const T *Fq = sl.F[qq];
                const T w0 = sl.W[qq][4 * kg + 0], w1 = sl.W[qq][4 * kg + 1];
                const T w2 = sl.W[qq][4 * kg + 2], w3 = sl.W[qq][4 * kg + 3];
                T af[TMV], yf[TNV];
#pragma unroll
                for (int ti = 0; ti < TMV; ++ti) af[ti] = Fq[oa[ti]] * Fq[ol[ti]] * ma[ti];
#pragma unroll
                for (int tj = 0; tj < TNV; ++tj) {
                    const int t = tyo[tj], k = kyo[tj];
                    const T tv = Fq[SL::OT + t], lv = Fq[SL::OL + k];
                    yf[tj] = (lv * (w0 * tv + w1 * Fq[SL::OT1 + t] + w2 * Fq[SL::OT2 + t]) +
                              w3 * tv * Fq[SL::OLP + k]) * my[tj];
                    if (LC::on && b0 + tj * 16 == LC::tile0 && i16 == LC::lane)   // load-vector column
                        yf[tj] = kg == 0 ? (T)sl.sf[qq] : (T)0;
                }
#pragma unroll
                for (int ti = 0; ti < TMV; ++ti)
#pragma unroll
                    for (int tj = 0; tj < TNV; ++tj)
                        acc[ti][tj] = mfma4(af[ti], yf[tj], acc[ti][tj]);
            }
            wave_sync();
        }
        T *Aout = (T *)prm.A + offA_of(prm, e, N);
        T *bout = (T *)prm.b + offb_of(prm, e, N);
#pragma unroll
        for (int ti = 0; ti < TMV; ++ti)
#pragma unroll
            for (int tj = 0; tj < TNV; ++tj) {
                const int col = b0 + tj * 16 + i16;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = a0 + ti * 16 + acc_row<T>(lane, r);
                    if (row < N && col < N)
                        Aout[(size_t)row * N + col] = acc[ti][tj][r];
                    else if (LC::on && row < N && col == N)
                        bout[row] = acc[ti][tj][r];
                }
            }
        if (!LC::on && bj == 0) {
#pragma unroll
            for (int m = 0; m < NBRV; ++m) {
                const int row = a0 + lane + 64 * m;
                if (lane + 64 * m < TMV * 16 && row < N) bout[row] = (T)bacc[m];
            }
        }
    }

    __device__ static void run_slice(const FwdParams &prm, int64_t slot, int blk, Slice &sl) {
        const int bi = blk / BN, bj = blk % BN;
        constexpr int TML = NT - (BM - 1) * TM, TNL = NT - (BN - 1) * TN;
        if (bi == BM - 1) {
            if (bj == BN - 1) body<TML, TNL>(prm, slot, blk, bi, bj, sl);
            else body<TML, TN>(prm, slot, blk, bi, bj, sl);
        } else {
            if (bj == BN - 1) body<TM, TNL>(prm, slot, blk, bi, bj, sl);
            else body<TM, TN>(prm, slot, blk, bi, bj, sl);
        }
    }
    __device__ static void run(const FwdParams &prm, int64_t slot, int blk, int wave, Smem &sm) {
        run_slice(prm, slot, blk, sm.w[wave]);
    }
};

}  // namespace feint
