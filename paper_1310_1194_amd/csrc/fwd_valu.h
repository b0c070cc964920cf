// Forward kernels on the vector ALUs for low degree.  At p = 1, 2, 3 the
// element matrix (n = 6, 18, 40) fills 16x16 MFMA tiles poorly (padded to 16,
// 32, 48), while MI355X runs FP64 FMAs on the vector ALUs at the same rate as
// on the matrix cores, so these kernels group the lanes of a wave per element
// instead of per output tile.
//
// A work item is EPW = 64 / LPE consecutive element slots, LPE lanes each.
//  * Geometry (steps a3-a5): the EPW * nq (element, point) pairs are spread
//    over the 64 lanes; each lane computes W_q in FP64 and stores its 13
//    nonzero entries (W_r0 = 0 for r >= 1) and the load weight w det J f in
//    the wave's LDS slice.
//  * Contraction (step a6): lane (el, j), j < n, owns column j of A_e:
//      y_0 = W_00 B0j + W_01 B1j + W_02 B2j + W_03 B3j,
//      y_r = W_r1 B1j + W_r2 B2j + W_r3 B3j                  (r = 1..3),
//      A_ij += B_q[0][i] y_0 + ... + B_q[3][i] y_3           (i = 0..n-1).
//    B_q[r][i] is the same for every lane of the wave, so it is read with
//    scalar loads and enters the FMAs as a scalar operand; only the four
//    B_q[s][j] of the lane's own column are vector loads.
//  * Load vector (step a7): b_j += sf_q phi_j(q) in FP64.
// The FP32 form rounds W_q to FP32 and accumulates A in FP32, as the 16x16x4
// FP32 MFMA kernels do.
#pragma once
#include "device_common.h"
#include "fwd_kernels.h"

namespace feint {

template <int P, typename T, int LPE, int R = 0, class G = PrismGeo>
struct KV {
    static constexpr int N = G::nshp(P), NP = c_pad16(N), NQ = G::nq(P, R);
    static constexpr int EPW = 64 / LPE;        // element slots per work item
    static constexpr int EPI = EPW, NBLK = 1;
    static constexpr int NPT = EPW * NQ;        // (element, point) pairs per item
    static constexpr int WS = sizeof(T) == 8 ? 14 : 16;   // 13 entries, rows 16-byte aligned
    static_assert(LPE >= N && LPE <= 64, "one lane per column of an element");
    typedef const __attribute__((address_space(4))) T CT;   // read through the scalar cache

    struct Slice {                    // one wave's LDS
        T W[NPT][WS];
        double sf[NPT];
    };
    struct Smem { Slice w[4]; };

    __device__ static void run(const FwdParams &prm, int64_t group, int blk, int wave, Smem &sm) {
        run_slice(prm, group, blk, sm.w[wave]);
    }

    __device__ static void run_slice(const FwdParams &prm, int64_t group, int blk, Slice &sl) {
        (void)blk;
        const int lane = threadIdx.x & 63;
        const int64_t s0 = group * EPW;
        const int64_t nslot = prm.ne;
        const T *Bt = uniform_ptr(sizeof(T) == 8 ? (const T *)(const void *)prm.B64
                                                 : (const T *)(const void *)prm.B32);
        const double *B64 = uniform_ptr(prm.B64);
        const double *qw = uniform_ptr(prm.qw);

        // geometry: lane t handles pair (t / NQ, t % NQ), then t + 64, ...
#pragma unroll 1
        for (int t = lane; t < NPT; t += 64) {
            const int el = t / NQ, q = t - el * NQ;
            const int64_t slot = s0 + el;
            if (slot < nslot) {
                const int64_t e = elem_of(prm, slot);
                typename G::Elem E;
                G::load(prm, e, E);
                const double *qp = qw + 4 * q;
                double W[16], sf;
                G::coeffs(prm, e, qp, E);
                const double det = G::block(E, qp, W, sf);
                if (!(det > 0.0) && prm.status) atomicOr(prm.status, 1u);
                T *w = sl.W[t];
                w[0] = (T)W[0]; w[1] = (T)W[1]; w[2] = (T)W[2]; w[3] = (T)W[3];
#pragma unroll
                for (int r = 1; r < 4; ++r)
#pragma unroll
                    for (int s = 1; s < 4; ++s) w[3 * r + s] = (T)W[4 * r + s];
                sl.sf[t] = sf;
                if (prm.xq) {
                    double x[3];
                    G::map(E, qp, x);
#pragma unroll
                    for (int d = 0; d < 3; ++d) prm.xq[(e * NQ + q) * 3 + d] = x[d];
                }
            }
        }
        wave_sync();

        const int el = lane / LPE, j = lane - el * LPE;
        const int elc = el < EPW ? el : EPW - 1;
        const int jc = j < N ? j : N - 1;
        T acc[N];
#pragma unroll
        for (int i = 0; i < N; ++i) acc[i] = (T)0;
        double bj = 0.0;
        CT *Bs = (CT *)Bt;
        const T *wrow = sl.W[elc * NQ];
        const double *sfrow = &sl.sf[elc * NQ];
        const T *Bcol = Bt + jc;
        const double *Bcol64 = B64 + jc;
        // the lane's own operands of point q + 1 are loaded while point q is
        // contracted
        T wv[13], cv[4];
        double sfv, phiv;
        auto fetch = [&](int q) {
#pragma unroll
            for (int k = 0; k < 13; ++k) wv[k] = wrow[q * WS + k];
#pragma unroll
            for (int s = 0; s < 4; ++s) cv[s] = Bcol[(size_t)(4 * q + s) * NP];
            sfv = sfrow[q];
            phiv = sizeof(T) == 8 ? 0.0 : Bcol64[(size_t)4 * q * NP];
        };
        fetch(0);
#pragma unroll 1
        for (int q = 0; q < NQ; ++q) {
            const T c0 = cv[0], c1 = cv[1], c2 = cv[2], c3 = cv[3];
            T y0 = wv[0] * c0;
            y0 = fma_t(wv[1], c1, y0); y0 = fma_t(wv[2], c2, y0); y0 = fma_t(wv[3], c3, y0);
            T y1 = wv[4] * c1;
            y1 = fma_t(wv[5], c2, y1); y1 = fma_t(wv[6], c3, y1);
            T y2 = wv[7] * c1;
            y2 = fma_t(wv[8], c2, y2); y2 = fma_t(wv[9], c3, y2);
            T y3 = wv[10] * c1;
            y3 = fma_t(wv[11], c2, y3); y3 = fma_t(wv[12], c3, y3);
            bj = __builtin_fma(sfv, sizeof(T) == 8 ? (double)c0 : phiv, bj);
            if (q + 1 < NQ) fetch(q + 1);
            CT *Bsq = Bs + (size_t)q * 4 * NP;
#pragma unroll
            for (int i = 0; i < N; ++i) {
                T a = fma_t(Bsq[i], y0, acc[i]);
                a = fma_t(Bsq[NP + i], y1, a);
                a = fma_t(Bsq[2 * NP + i], y2, a);
                acc[i] = fma_t(Bsq[3 * NP + i], y3, a);
            }
        }

        const int64_t slot = s0 + el;
        if (el < EPW && j < N && slot < nslot) {
            const int64_t e = elem_of(prm, slot);
            T *Aout = (T *)prm.A + offA_of(prm, e, N);
#pragma unroll
            for (int i = 0; i < N; ++i) Aout[(size_t)i * N + j] = acc[i];
            if constexpr (G::LOAD) ((T *)prm.b)[offb_of(prm, e, N) + j] = (T)bj;
        }
    }
};

// One element per lane (p = 1, n = 6): each lane runs its own element's point
// loop -- W_q in FP64, then y_r = (W_q B_q)[r][j] (13 FMAs per column) and
// A_ij += sum_r B_q[r][i] y_r (4 per entry) -- while the whole wave is at the
// same point, so every table entry is wave-uniform and enters the FMAs as a
// scalar operand.  Against the kernel above (LPE lanes per element), no lane
// sits on a padding column and W_q needs no LDS: about half the vector
// instructions per element.  64 elements per wave; each lane loads and stores
// its own element (staging those through LDS for wave-contiguous accesses
// measured slower: the index arithmetic and the waits cost more than the
// scattered lines).  Lanes past the batch compute on element 0 and store
// nothing.
template <int P, typename T, int R = 0, class G = PrismGeo>
struct KE {
    static constexpr int N = G::nshp(P), NP = c_pad16(N), NQ = G::nq(P, R);
    static constexpr int EPI = 64, NBLK = 1;
    static_assert(N <= 8, "one element per lane holds its n^2 accumulators");
    typedef const __attribute__((address_space(4))) T CT;
    typedef const __attribute__((address_space(4))) double CD;
    struct Smem { int unused; };

    __device__ static void run(const FwdParams &prm, int64_t group, int blk, int wave, Smem &) {
        (void)blk;
        (void)wave;
        const int lane = threadIdx.x & 63;
        const int64_t slot = group * 64 + lane;
        const bool act = slot < prm.ne;
        const int64_t e = act ? elem_of(prm, slot) : 0;
        typename G::Elem E;
        G::load(prm, e, E);
        const T *Bt = uniform_ptr(sizeof(T) == 8 ? (const T *)(const void *)prm.B64
                                                 : (const T *)(const void *)prm.B32);
        const double *B64 = uniform_ptr(prm.B64);
        const double *qw = uniform_ptr(prm.qw);
        T acc[N][N];
#pragma unroll
        for (int i = 0; i < N; ++i)
#pragma unroll
            for (int j = 0; j < N; ++j) acc[i][j] = (T)0;
        double bj[N];
#pragma unroll
        for (int j = 0; j < N; ++j) bj[j] = 0.0;
#pragma unroll 1
        for (int q = 0; q < NQ; ++q) {
            const double *qp = qw + 4 * q;
            double W[16], sf;
            G::coeffs(prm, e, qp, E);
            const double det = G::block(E, qp, W, sf);
            if (act && !(det > 0.0) && prm.status) atomicOr(prm.status, 1u);
            if (act && prm.xq) {
                double x[3];
                G::map(E, qp, x);
#pragma unroll
                for (int d = 0; d < 3; ++d) prm.xq[(e * NQ + q) * 3 + d] = x[d];
            }
            const CT *Bq = (const CT *)(Bt + (size_t)q * 4 * NP);
            T w[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) w[k] = (T)W[k];
            T y[4][N];
#pragma unroll
            for (int j = 0; j < N; ++j) {
                const T c0 = Bq[j], c1 = Bq[NP + j], c2 = Bq[2 * NP + j], c3 = Bq[3 * NP + j];
                y[0][j] = fma_t(w[3], c3, fma_t(w[2], c2, fma_t(w[1], c1, w[0] * c0)));
#pragma unroll
                for (int r = 1; r < 4; ++r) y[r][j] = fma_t(w[4 * r + 3], c3, fma_t(w[4 * r + 2], c2, w[4 * r + 1] * c1));
            }
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const T b0 = Bq[i], b1 = Bq[NP + i], b2 = Bq[2 * NP + i], b3 = Bq[3 * NP + i];
#pragma unroll
                for (int j = 0; j < N; ++j)
                    acc[i][j] = fma_t(b3, y[3][j], fma_t(b2, y[2][j], fma_t(b1, y[1][j], fma_t(b0, y[0][j], acc[i][j]))));
            }
            if constexpr (G::LOAD) {
                const CD *B0 = (const CD *)(B64 + (size_t)q * 4 * NP);
#pragma unroll
                for (int j = 0; j < N; ++j) bj[j] = __builtin_fma(sf, B0[j], bj[j]);
            }
        }
        if (act) {
            T *Aout = (T *)prm.A + offA_of(prm, e, N);
#pragma unroll
            for (int i = 0; i < N; ++i)
#pragma unroll
                for (int j = 0; j < N; ++j) Aout[i * N + j] = acc[i][j];
            if constexpr (G::LOAD) {
                T *bout = (T *)prm.b + offb_of(prm, e, N);
#pragma unroll
                for (int j = 0; j < N; ++j) bout[j] = (T)bj[j];
            }
        }
    }
};

}  // namespace feint
