// Forward kernel for tetrahedra from reference matrices (FP64, FP32).  The
// tetrahedral map is affine, so J, det J and K = J^-1 are the same at every
// point and W_q = w_q W with one element block W = det J [[c, (K beta)^T],
// [0, K D K^T]] (its column 0 is zero below the diagonal).  The quadrature
// sum then separates:
//   A[a][b] = sum_q sum_(r,s) B_q[r][a] w_q W[r][s] B_q[s][b] = sum_(r,s) W[r][s] M_rs[a][b],
//   M_rs = sum_q w_q B_q[r]^T B_q[s],   b[a] = det J f sum_q w_q phi_a(q),
// with the 13 reference matrices M_rs and the reference load vector built once
// per degree on the host (extended precision).  Per element: W in FP64, then
// 13 multiply-adds per entry of A, against 8 n^2 nq flops for the
// point-by-point product -- the same sum in another order (the oracle still
// integrates point by point).
//
// A wave owns EPW (64, 32 or 16) elements.  Over a batch of elements the
// separated sum is a GEMM, A[(e)][(a,b)] = sum_k W_e[k] M_k[(a,b)] with K = 13
// slots padded to 16: each lane forms one element's W and stages it in the
// wave's LDS slice, the lanes pick up their 16x16x4 MFMA A fragments (16
// elements x 4 K-steps per row tile of 16 elements) once, and for every
// 16-entry column tile the wave loads the B fragments (M, slot-major, 16
// consecutive entries per K row, the next tile's in flight during the current
// MFMAs) and issues 4 MFMAs per row tile.  RTP row tiles take one pass over the
// column tiles before the next RTP (one: the wave's writes stay within 16
// element rows at a time); accumulator rows are elements, so 16 lanes store 16
// consecutive entries of one element, or with STG four column tiles go
// through LDS first and each store writes 64 consecutive entries of one
// element.  Stores and fragment loads go through buffer resources: a
// wave-uniform base, one fixed 32-bit offset per lane and row, the tile's
// offset in a scalar register, so the loop carries no per-lane address
// arithmetic.  The load vector b[e][a] = sf_e m0[a] follows.
#pragma once
#include "fwd_kernels.h"

namespace feint {

template <int P, typename T, int RTP = 4, bool STG = false, int EPW = 64>
struct KT {
    static constexpr int RT = EPW / 16;                // row tiles of 16 elements per wave
    static_assert(EPW == 16 || EPW == 32 || EPW == 64, "elements per wave");
    static_assert(RTP >= 1 && RT % RTP == 0, "row tiles per pass");
    static_assert(!STG || RTP == 1, "staged stores take one row tile per pass");
    typedef TetGeo G;
    static constexpr int N = G::nshp(P), NQ = G::nq(P, 0), N2 = N * N, N2P = (N2 + 15) / 16 * 16;
    static constexpr int NCT = N2P / 16;               // column tiles of 16 entries
    static constexpr int EPI = EPW, NBLK = 1;
    static constexpr int WS = 17;                      // slice row: 16 slots, odd stride
    typedef typename AccT<T>::type V4;
    static constexpr int SP = 64 + 2;                  // staging row: 64 entries + pad
    static constexpr int NB = (N2 + 63) / 64;          // 64-entry column blocks
    // W of the wave's elements; staged stores reuse it for 16 x SP values
    static constexpr int WD = STG && 16 * SP * (int)sizeof(T) > EPW * WS * 8 ? (16 * SP * (int)sizeof(T) + 7) / 8 : EPW * WS;
    struct Slice {
        double W[WD];
        double sf[EPW];
        int64_t oA[EPW], ob[EPW];                      // output offsets of the wave's elements
    };
    struct Smem { Slice w[4]; };

    __device__ static void run(const FwdParams &prm, int64_t group, int blk, int wave, Smem &sm) {
        (void)blk;
        Slice &sl = sm.w[wave];
        const int lane = threadIdx.x & 63;
        const int64_t e0 = group * EPW;
        const int64_t slot = e0 + lane;
        const bool act = lane < EPW && slot < prm.ne;
        const int nact = (int)(prm.ne - e0 < EPW ? prm.ne - e0 : EPW);
        const int64_t e = act ? elem_of(prm, slot) : 0;
        ElemTet E;
        G::load(prm, e, E);
        double K[9], W[16], sf;
        const double det = tet_jacobian(E.X, K);
        fused_block(E, K, det, W, sf);
        if (act && !(det > 0.0) && prm.status) atomicOr(prm.status, 1u);
        if (act && prm.xq) {
#pragma unroll 1
            for (int q = 0; q < NQ; ++q) {
                const double *qp = prm.qw + 4 * q;
                double x[3];
                G::map(E, qp, x);
#pragma unroll
                for (int d = 0; d < 3; ++d) prm.xq[(e * NQ + q) * 3 + d] = x[d];
            }
        }
        // W's 13 nonzero entries in the reference matrices' slot order, slots 13..15 zero;
        // lanes past the batch stage zeros
        if (lane < EPW) {
            double *row = &sl.W[lane * WS];
            const double z = act ? 1.0 : 0.0;
            row[0] = z * W[0]; row[1] = z * W[1]; row[2] = z * W[2]; row[3] = z * W[3];
#pragma unroll
            for (int r = 1; r < 4; ++r)
#pragma unroll
                for (int s = 1; s < 4; ++s) row[3 * r + s] = z * W[4 * r + s];
            row[13] = row[14] = row[15] = 0.0;
            sl.sf[lane] = z * sf;
            sl.oA[lane] = act ? offA_of(prm, e, N) : 0;
            sl.ob[lane] = act ? offb_of(prm, e, N) : 0;
        }
        wave_sync();
        // A fragments: lane l supplies A[row l % 16][k l / 16] of each row tile and K-step
        const int i16 = lane & 15, kg = lane >> 4;
        T afr[RT][4];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) afr[rt][kb] = (T)sl.W[(rt * 16 + i16) * WS + kb * 4 + kg];

        const T *Mt = sizeof(T) == 8 ? (const T *)(const void *)prm.Mref64 : (const T *)(const void *)prm.Mref32;
        const auto rM = buffer_rsrc(uniform_ptr(Mt), (uint32_t)(16 * N2P * sizeof(T)));
        const uint32_t vM = (uint32_t)((kg * N2P + i16) * sizeof(T));
        // B fragment of column tile ct, K-step kb: lane l supplies M[slot 4 kb + l / 16][entry 16 ct + l % 16]
        auto load_b = [&](int ct, T (&bf)[4]) {
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) bf[kb] = buffer_load<T>(rM, vM, (uint32_t)((kb * 4 * N2P + ct * 16) * sizeof(T)));
        };
        // the MFMAs of one column tile for row tiles G .. G + RTP - 1
        auto mma = [&](const T (&bc)[4], V4 (&acc)[RTP], auto G) {
#pragma unroll
            for (int j = 0; j < RTP; ++j) acc[j] = V4{0, 0, 0, 0};
#pragma unroll
            for (int kb = 0; kb < 4; ++kb)
#pragma unroll
                for (int j = 0; j < RTP; ++j) acc[j] = mfma4(afr[decltype(G)::value + j][kb], bc[kb], acc[j]);
        };
        // Rows as 32-bit byte offsets from the wave's first row when the whole wave
        // is in the batch and its rows lie within 4 GiB after that one: a store is
        // then a wave-uniform base plus a fixed per-lane offset, with no address
        // arithmetic inside the loop.
        const int64_t base = wave_uniform64(sl.oA[0]);
        uint32_t ro[RT][4];
        bool near = true;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t d = sl.oA[rt * 16 + acc_row<T>(lane, r)] - base;
                near = near && d >= 0 && (d + N2P) * (int64_t)sizeof(T) <= (int64_t)0xffffffffll;
                ro[rt][r] = (uint32_t)((d + i16) * (int64_t)sizeof(T));
            }
        constexpr int NFULL = N2 / 16;                 // tiles with 16 valid entries
        const auto rA = buffer_rsrc(uniform_ptr((const T *)prm.A + base), 0xffffffffu);
        const bool fastw = nact == EPW && __all(near);
        if constexpr (STG) if (fastw) {
            // 16 elements at a time; per block of four column tiles the results
            // go through the slice (free once the A fragments are in registers) so
            // that each store writes 64 consecutive entries of one element
            static_assert(16 * SP * sizeof(T) <= sizeof(Slice::W), "staging fits the slice");
            T *stg = (T *)(void *)sl.W;
            wave_sync();
            static_for<0, RT>([&](auto GI) {
                constexpr int G = decltype(GI)::value;
                const ic<G> g;
                uint32_t rowo[16];
#pragma unroll
                for (int el = 0; el < 16; ++el)
                    rowo[el] = (uint32_t)wave_uniform((int)(uint32_t)((sl.oA[G * 16 + el] - base) * (int64_t)sizeof(T)));
#pragma unroll 1
                for (int blk = 0; blk < NB; ++blk) {
                    T bf[4][4];
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        if (blk * 4 + t < NCT) load_b(blk * 4 + t, bf[t]);
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        if (blk * 4 + t < NCT) {
                            V4 acc[1];
                            mma(bf[t], acc, g);
#pragma unroll
                            for (int r = 0; r < 4; ++r) stg[acc_row<T>(lane, r) * SP + t * 16 + i16] = acc[0][r];
                        }
                    wave_sync();
                    const int col = blk * 64 + lane;
                    if (col < N2) {
#pragma unroll
                        for (int el = 0; el < 16; ++el)
                            buffer_store(stg[el * SP + lane], rA, (uint32_t)(lane * sizeof(T)), rowo[el] + (uint32_t)(blk * 64 * sizeof(T)));
                    }
                    wave_sync();
                }
            });
        }
        if constexpr (!STG) if (fastw) {
            // RTP row tiles (16 RTP elements) at a time, each group through all
            // column tiles before the next
            static_for<0, RT / RTP>([&](auto GI) {
                constexpr int G = decltype(GI)::value * RTP;
                const std::integral_constant<int, G> g;
                auto put = [&](const V4 (&acc)[RTP], uint32_t so) {
#pragma unroll
                    for (int j = 0; j < RTP; ++j)
#pragma unroll
                        for (int r = 0; r < 4; ++r) buffer_store(acc[j][r], rA, ro[G + j][r], so);
                };
                T b0[4], b1[4];
                load_b(0, b0);
                int ct = 0;
#pragma unroll 1
                for (; ct + 2 <= NFULL; ct += 2) {
                    V4 acc[RTP];
                    const uint32_t so = (uint32_t)(ct * 16 * sizeof(T));
                    load_b(ct + 1, b1);
                    mma(b0, acc, g);
                    put(acc, so);
                    load_b(ct + 2 < NCT ? ct + 2 : ct + 1, b0);
                    mma(b1, acc, g);
                    put(acc, so + 16 * sizeof(T));
                }
                // at most one full tile and the partial one left
#pragma unroll 1
                for (; ct < NCT; ++ct) {
                    V4 acc[RTP];
                    mma(b0, acc, g);
                    if (ct * 16 + i16 < N2) put(acc, (uint32_t)(ct * 16 * sizeof(T)));
                    if (ct + 1 < NCT) load_b(ct + 1, b0);
                }
            });
        }
        if (!fastw) {
            // a partial or far-apart wave: rows past the batch and entries past
            // n^2 masked, row offsets read from LDS
            T b0[4];
            load_b(0, b0);
#pragma unroll 1
            for (int ct = 0; ct < NCT; ++ct) {
                static_for<0, RT / RTP>([&](auto GI) {
                    constexpr int G = decltype(GI)::value * RTP;
                    V4 acc[RTP];
                    mma(b0, acc, std::integral_constant<int, G>());
                    if (ct * 16 + i16 < N2) {
#pragma unroll
                        for (int j = 0; j < RTP; ++j)
#pragma unroll
                            for (int r = 0; r < 4; ++r) {
                                const int el = (G + j) * 16 + acc_row<T>(lane, r);
                                if (el < nact) ((T *)prm.A)[sl.oA[el] + ct * 16 + i16] = acc[j][r];
                            }
                    }
                });
                if (ct + 1 < NCT) load_b(ct + 1, b0);
            }
        }
        // b[e][a] = sf_e m0[a] over the wave's nact x n values, lanes on consecutive
        // (element, a) pairs
        const double *m0 = prm.Mref64 + (size_t)N2P * 16;
        T *bout = (T *)prm.b;
#pragma unroll 1
        for (int i = lane; i < nact * N; i += 64) {
            const int el = i / N, a = i - el * N;
            bout[sl.ob[el] + a] = (T)(sl.sf[el] * m0[a]);
        }
    }
};

}  // namespace feint
