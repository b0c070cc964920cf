// Software-pipelined split-form kernels (bf16x3, fp16x3), gfx950.
//
// The plain split kernel forms the B fragments Y = W_q B_q of a K-block (8
// points) on the vector ALUs and then issues that block's MFMAs; the two
// depend on each other, so within a wave they run one after the other.  Here
// the FP64 geometry of all of the element's points is computed first (one
// pass, W_q and the load weights into the wave's LDS slice), and the K loop
// is pipelined by one block: while the MFMAs of block k run, the same basic
// block forms and splits Y of block k+1 and loads the A fragments of block
// k+1 and the FP32 columns of block k+2.  Two register sets alternate between
// the roles "current" and "next", so nothing is copied between iterations.
// The load vector rides in the contraction where the padded width leaves a
// spare column (n < n_pad); at p = 7 it is summed in FP64 after the K loop
// from the load weights kept in LDS.
#pragma once
#include "fwd_kernels.h"

namespace feint {

template <int P, int FORM, int TM, int TN, int R = 0>
struct K32P {
    static constexpr int N = c_nshp(P), NP = c_pad16(N), NT = NP / 16, NQ = c_nq_rule(P, R);
    static constexpr int NQP = c_pad8(NQ), NKB = NQP / 8;
    static constexpr int BM = c_cdiv(NT, TM), BN = c_cdiv(NT, TN), NBLK = BM * BN;
    static constexpr int EPI = 1;
    // LDS row of W: padded (conflict-free per-lane writes) unless four waves'
    // slices of the whole element would not fit the 160 KB of a CU
    static constexpr int RW = NQP * (20 * 4 + 8) * 4 <= 160 * 1024 ? 20 : 16;
    static constexpr int VPM = 3;                 // vector instructions scheduled after each MFMA
    typedef typename SplitT<FORM>::vec HV;
    typedef typename SplitT<FORM>::scal HS;
    typedef LoadCol<P> LC;

    struct Slice {                                // one wave's LDS: the whole element's points
        float W[NQP][RW];
        double sf[NQP];
    };
    struct Smem { Slice w[4]; };

    // W_q (FP32, times the fp16 scale of A's columns) and w det J f of every
    // point into the slice; returns the element's fp16 scales (ys for A's
    // columns, yb for the load-vector column; both 1 for bf16), as
    // K32::elem_scale derives them.
    __device__ static SplitScale geometry(const FwdParams &prm, ElemIn &E, int64_t e, int blk, Slice &sl) {
        const int lane = threadIdx.x & 63;
        double m = 0.0, mb = 0.0;
        for (int qc = 0; qc < NQP; qc += 64) {
            const int q = qc + lane;
            if (q < NQP) {
                double W[16], sf = 0.0;
                if (q < NQ) {
                    const double *qp = prm.qw + 4 * q;
                    field_at(prm, e, qp[0], qp[1], qp[2], E);
                    const double det = point_block(E, qp[0], qp[1], qp[2], qp[3], W, sf);
                    if (!(det > 0.0) && prm.status) atomicOr(prm.status, 1u);
                    if (prm.xq && blk == 0) {
                        double x[3];
                        prism_map(E.X, qp[0], qp[1], qp[2], x);
#pragma unroll
                        for (int d = 0; d < 3; ++d) prm.xq[(e * NQ + q) * 3 + d] = x[d];
                    }
                    if (FORM == FP16X3) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const double s = (fabs(W[4 * r]) + fabs(W[4 * r + 1]) + fabs(W[4 * r + 2]) +
                                              fabs(W[4 * r + 3])) * (double)prm.bmax;
                            m = s > m ? s : m;
                        }
                        mb = fabs(sf) > mb ? fabs(sf) : mb;
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < 16; ++k) W[k] = 0.0;
                }
#pragma unroll
                for (int k = 0; k < 16; ++k) sl.W[q][k] = (float)W[k];
                sl.sf[q] = sf;
            }
        }
        float ys = 1.0f, yb = 1.0f;
        if (FORM == FP16X3) {
            // bounds on |Y| over the element (A's columns, load-vector column);
            // each scaled into [2^13, 2^14)
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                const double o = __shfl_xor(m, off, 64), ob = __shfl_xor(mb, off, 64);
                m = o > m ? o : m;
                mb = ob > mb ? ob : mb;
            }
            ys = pow2_scale(m);
            yb = pow2_scale(mb);
            for (int q = lane; q < NQP; q += 64)     // each lane rescales the rows it wrote
#pragma unroll
                for (int k = 0; k < 16; ++k) sl.W[q][k] *= ys;
        }
        wave_sync();
        return SplitScale{ys, yb};
    }

    template <int TMV, int TNV>
    struct Stage {
        HV ah[TMV], al[TMV], yh[TNV], yl[TNV];
    };

    template <int TMV>
    __device__ static void load_a(const FwdParams &prm, int kb, int a0, int lane, HV (&ah)[TMV], HV (&al)[TMV]) {
#pragma unroll
        for (int ti = 0; ti < TMV; ++ti) {
            const size_t o = (((size_t)kb * NT + a0 / 16 + ti) * 64 + lane) * 8;
            ah[ti] = *(const HV *)(prm.Bhi + o);
            al[ti] = *(const HV *)(prm.Blo + o);
        }
    }

    template <int TNV>
    __device__ static void load_yc(const FwdParams &prm, int kb, int b0, int lane, float4 (&yc)[TNV][2]) {
#pragma unroll
        for (int tj = 0; tj < TNV; ++tj) {
            const float *yp = prm.Ycf + (((size_t)kb * NT + b0 / 16 + tj) * 64 + lane) * 8;
            yc[tj][0] = *(const float4 *)yp;
            yc[tj][1] = *(const float4 *)(yp + 4);
        }
    }

    // The lane's weights of block kb: W rows of its two points and their
    // load weights (times the fp16 scale).
    struct PointW {
        float wa[16], wb[16], za, zb;
    };
    __device__ static void read_w(const Slice &sl, int kb, int lane, float yb, PointW &pw) {
        const int qa = kb * 8 + 2 * (lane >> 4);
#pragma unroll
        for (int k = 0; k < 16; ++k) { pw.wa[k] = sl.W[qa][k]; pw.wb[k] = sl.W[qa + 1][k]; }
        pw.za = (float)sl.sf[qa] * yb;
        pw.zb = (float)sl.sf[qa + 1] * yb;
    }

    // Y = W_q B_q for the lane's column of tile tj and its two points,
    // split into hi and lo.
    __device__ static void form_y_tile(const PointW &pw, int tj, int b0, int lane, const float4 (&yc)[2],
                                       HV &yh, HV &yl) {
        const float s0[4] = {yc[0].x, yc[0].y, yc[0].z, yc[0].w};
        const float s1[4] = {yc[1].x, yc[1].y, yc[1].z, yc[1].w};
        float y[8];
        y[0] = pw.wa[0] * s0[0] + pw.wa[1] * s0[1] + pw.wa[2] * s0[2] + pw.wa[3] * s0[3];
        y[4] = pw.wb[0] * s1[0] + pw.wb[1] * s1[1] + pw.wb[2] * s1[2] + pw.wb[3] * s1[3];
#pragma unroll
        for (int r = 1; r < 4; ++r) {
            y[r] = pw.wa[4 * r + 1] * s0[1] + pw.wa[4 * r + 2] * s0[2] + pw.wa[4 * r + 3] * s0[3];
            y[4 + r] = pw.wb[4 * r + 1] * s1[1] + pw.wb[4 * r + 2] * s1[2] + pw.wb[4 * r + 3] * s1[3];
        }
        if (b0 + tj * 16 == LC::tile0 && (lane & 15) == LC::lane) {   // load-vector column
#pragma unroll
            for (int r = 0; r < 8; ++r) y[r] = 0.0f;
            y[0] = pw.za;
            y[4] = pw.zb;
        }
        K32<P, FORM, TM, TN, R>::split8(y, yh, yl);
    }

    // The three products of a tile go to the same accumulator; they are issued
    // product by product over the tiles, so that consecutive MFMAs are
    // independent and a dependent one comes TMV issues later.
    template <int TMV, int TNV>
    __device__ static void mfma_col(f32x4 (&acc)[TMV][TNV], const Stage<TMV, TNV> &s, int tj) {
#pragma unroll
        for (int ti = 0; ti < TMV; ++ti) acc[ti][tj] = mfma32(s.al[ti], s.yh[tj], acc[ti][tj]);
#pragma unroll
        for (int ti = 0; ti < TMV; ++ti) acc[ti][tj] = mfma32(s.ah[ti], s.yl[tj], acc[ti][tj]);
#pragma unroll
        for (int ti = 0; ti < TMV; ++ti) acc[ti][tj] = mfma32(s.ah[ti], s.yh[tj], acc[ti][tj]);
    }

    template <int TMV, int TNV>
    __device__ static void mfma_block(f32x4 (&acc)[TMV][TNV], const Stage<TMV, TNV> &s) {
#pragma unroll
        for (int tj = 0; tj < TNV; ++tj) mfma_col<TMV, TNV>(acc, s, tj);
    }

    template <int TMV, int TNV>
    __device__ static void body(const FwdParams &prm, int64_t slot, int blk, int bi, int bj, Slice &sl) {
        const int lane = threadIdx.x & 63;
        const int i16 = lane & 15, kg = lane >> 4;
        const int a0 = bi * TM * 16, b0 = bj * TN * 16;
        const int64_t e = elem_of(prm, slot);
        SplitScale sc;
        {
            ElemIn E;
            load_elem_fwd(prm, e, E);
            sc = geometry(prm, E, e, blk, sl);
        }
        const float ys = sc.ys, yb = sc.yb;
        f32x4 acc[TMV][TNV];
#pragma unroll
        for (int ti = 0; ti < TMV; ++ti)
#pragma unroll
            for (int tj = 0; tj < TNV; ++tj) acc[ti][tj] = f32x4{0, 0, 0, 0};

        Stage<TMV, TNV> s0, s1;
        float4 ycA[TNV][2], ycB[TNV][2];          // FP32 columns, alternating like the stages
        {
            float4 y0[TNV][2];
            load_a<TMV>(prm, 0, a0, lane, s0.ah, s0.al);
            load_yc<TNV>(prm, 0, b0, lane, y0);
            load_yc<TNV>(prm, NKB > 1 ? 1 : 0, b0, lane, ycA);
            PointW pw;
            read_w(sl, 0, lane, yb, pw);
#pragma unroll
            for (int tj = 0; tj < TNV; ++tj) form_y_tile(pw, tj, b0, lane, y0[tj], s0.yh[tj], s0.yl[tj]);
        }
        // one pipelined step: MFMAs of block kb from `cur` while `nxt` receives
        // block kb+1 from the columns `ycu` (loaded one step earlier) and the
        // columns of block kb+2 are loaded into `ycl` (indices clamped: the
        // last step recomputes a block it does not use, which keeps the loop
        // free of branches).  The step is issued column tile by column tile:
        // the MFMAs of column tj of block kb interleaved with forming Y of
        // column tj of block kb+1; scheduling fences keep the groups in that
        // order.
        auto step = [&](const Stage<TMV, TNV> &cur, Stage<TMV, TNV> &nxt, const float4 (&ycu)[TNV][2],
                        float4 (&ycl)[TNV][2], int kb) {
            const int k1 = kb + 1 < NKB ? kb + 1 : NKB - 1;
            const int k2 = kb + 2 < NKB ? kb + 2 : NKB - 1;
            load_a<TMV>(prm, k1, a0, lane, nxt.ah, nxt.al);
            load_yc<TNV>(prm, k2, b0, lane, ycl);
            PointW pw;
            read_w(sl, k1, lane, yb, pw);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int tj = 0; tj < TNV; ++tj) {
                mfma_col<TMV, TNV>(acc, cur, tj);
                form_y_tile(pw, tj, b0, lane, ycu[tj], nxt.yh[tj], nxt.yl[tj]);
#pragma unroll
                for (int i = 0; i < 3 * TMV; ++i) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);       // one MFMA
                    __builtin_amdgcn_sched_group_barrier(0x002, VPM, 0);     // VPM VALU
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        };
        int kb = 0;
        for (; kb + 1 < NKB; kb += 2) {
            step(s0, s1, ycA, ycB, kb);
            step(s1, s0, ycB, ycA, kb + 1);
        }
        if (kb < NKB) mfma_block<TMV, TNV>(acc, s0);

        const float unscale = FORM == FP16X3 ? ldexpf(1.0f, -prm.f16_shift) / ys : 1.0f;
        const float unscale_b = FORM == FP16X3 ? ldexpf(1.0f, -prm.f16_shift) / yb : 1.0f;
        float *Aout = (float *)prm.A + offA_of(prm, e, N);
        float *bout = (float *)prm.b + offb_of(prm, e, N);
        if (!LC::on && bj == 0) {
            // no spare column: b_row = sum_q w_q det J_q f phi_row(q) in FP64, four
            // independent partial sums per row
            constexpr int NBRV = c_cdiv(TMV * 16, 64);
#pragma unroll
            for (int m = 0; m < NBRV; ++m) {
                const int row = a0 + lane + 64 * m;
                if (lane + 64 * m < TMV * 16 && row < N) {
                    const double *phi = prm.B64 + row;
                    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
                    int q = 0;
                    for (; q + 4 <= NQ; q += 4) {
                        s0 += sl.sf[q] * phi[(size_t)q * 4 * NP];
                        s1 += sl.sf[q + 1] * phi[(size_t)(q + 1) * 4 * NP];
                        s2 += sl.sf[q + 2] * phi[(size_t)(q + 2) * 4 * NP];
                        s3 += sl.sf[q + 3] * phi[(size_t)(q + 3) * 4 * NP];
                    }
                    for (; q < NQ; ++q) s0 += sl.sf[q] * phi[(size_t)q * 4 * NP];
                    bout[row] = (float)((s0 + s1) + (s2 + s3));
                }
            }
        }
#pragma unroll
        for (int ti = 0; ti < TMV; ++ti)
#pragma unroll
            for (int tj = 0; tj < TNV; ++tj) {
                const int col = b0 + tj * 16 + i16;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = a0 + ti * 16 + 4 * kg + r;
                    if (row < N && col < N)
                        Aout[(size_t)row * N + col] = acc[ti][tj][r] * unscale;
                    else if (LC::on && row < N && col == N)
                        bout[row] = acc[ti][tj][r] * unscale_b;
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
