// Split-form forward kernels (bf16x3, fp16x3) whose right operand
// Y = W_q B_q is itself formed on the matrix cores, gfx950.
//
// The split kernels of fwd_kernels.h and fwd_pipe.h form their fragment of
// Y on the vector ALUs (13 FMAs per point and column, then the hi/lo split),
// about four vector instructions per MFMA, and the vector work and the MFMAs
// of a wave barely overlap.  Here Y is a product on the matrix cores.
//
// The eight points of a K-block are taken as two halves h of four points,
// 2 kg + h for kg = 0..3.  For a column tile and half h, the batched 4x4x4
// MFMA (16 independent 4x4 blocks, block b = lane / 4) computes in block
// (kg, column group cg), b = 4 kg + cg,
//   Y_point[r][4 cg + j] = sum_s W_point[r][s] B[(point, s)][4 cg + j],
// point = 2 kg + h: lane l = 16 kg + 4 cg + i supplies row i of W_point (its
// four values s) and column 4 cg + i of B for the point's rows s, which is half
// h (v = 4h..4h+3) of the split table fragment lane l holds anyway; the
// result lane l = 16 kg + j holds Y_point[r = 0..3][j].  So lane (kg, j) ends
// with Y of points 2 kg and 2 kg + 1, rows 0..3, column j: the B-fragment
// order of the main 16x16x32 product A += B^T Y, whose left operand is the
// same table fragment, of a row tile.  W and B are split into hi + lo with
// three products, Y (FP32) is split again for the main product.  A wave that
// holds a whole element (TM = TN = the number of tiles) loads each table
// fragment once per K-block and uses it in both roles.  The vector work left
// per K-block is splitting W (two rows of four values per lane) and Y (eight
// values per lane and column tile).
//
// W_q of the element's points is computed in FP64 (one point per lane, 64 at
// a time) into the wave's LDS slice, all at once before the K loop or chunk
// by chunk at every eighth K-block (CH); the element's inputs are re-read
// from L2 for each chunk rather than held in registers.
// The load vector rides in the spare padded column n of B^T Y, as in the
// other split kernels: B is zero there, so the Y product leaves zero in that
// column and the lane of row r = 0 adds w det J f.  Without a spare column
// (p = 7) it is summed in FP64, chunk by chunk, by the waves of the first
// column block.
#pragma once
#include "fwd_kernels.h"

namespace feint {

template <int FORM> struct SplitT4;
template <> struct SplitT4<BF16X3> { typedef bf16x4 vec; };
template <> struct SplitT4<FP16X3> { typedef f16x4 vec; };

// CH = 1: the wave's LDS slice holds a chunk of 64 points, refilled every
// eighth K-block; CH = 0: it holds all of the element's points, computed
// before the K loop (fewer registers live across the geometry; the LDS of a
// workgroup grows with the point count).
template <int P, int FORM, int TM, int TN, int R = 0, int CH = 1>
struct K32Y {
    static constexpr int N = c_nshp(P), NP = c_pad16(N), NT = NP / 16, NQ = c_nq_rule(P, R);
    static constexpr int NQP = c_pad8(NQ), NKB = NQP / 8;
    static constexpr int SQ = CH ? 64 : (NQP + 63) / 64 * 64;   // points the slice holds
    static constexpr int KPC = SQ / 8;                 // K-blocks per slice fill
    static constexpr int BM = c_cdiv(NT, TM), BN = c_cdiv(NT, TN), NBLK = BM * BN;
    static constexpr int EPI = 1;
    // one block per element: the row and column fragments are the same registers
    static constexpr bool WHOLE = TM == NT && TN == NT;
    typedef typename SplitT<FORM>::vec HV;
    typedef typename SplitT<FORM>::scal HS;
    typedef typename SplitT4<FORM>::vec HV4;
    typedef LoadCol<P> LC;
    typedef K32<P, FORM, TM, TN, R> Plain;             // per-element fp16 scales, the split of eight values

    struct Slice {                                     // one wave's LDS
        float W[SQ][WROW<float>::value];
        double sf[SQ];
    };
    struct Smem { Slice w[4]; };

    struct Frag {
        HV h, l;
    };

    __device__ static void load_frag(const FwdParams &prm, int kb, int tile, int lane, Frag &f) {
        const size_t o = (((size_t)kb * NT + tile) * 64 + lane) * 8;
        f.h = *(const HV *)(prm.Bhi + o);
        f.l = *(const HV *)(prm.Blo + o);
    }

    // hi = rn(x), lo = rn(x - hi) of four values (the residual is exact in FP32)
    __device__ static void split4(const float *x, HV4 &hi, HV4 &lo) {
        typedef float f2 __attribute__((ext_vector_type(2)));
        typedef HS h2 __attribute__((ext_vector_type(2)));
#pragma unroll
        for (int v = 0; v < 4; v += 2) {
            const f2 xx = {x[v], x[v + 1]};
            const h2 h = __builtin_convertvector(xx, h2);
            const f2 hf = __builtin_convertvector(h, f2);
            const f2 r = xx - hf;
            const h2 l = __builtin_convertvector(r, h2);
            hi[v] = h.x; hi[v + 1] = h.y;
            lo[v] = l.x; lo[v + 1] = l.y;
        }
    }

    __device__ static HV4 half_of(const HV &v, int h) {
        return h == 0 ? __builtin_shufflevector(v, v, 0, 1, 2, 3) : __builtin_shufflevector(v, v, 4, 5, 6, 7);
    }

    // W_q (FP32, times the fp16 scale of A's columns) and w det J f of the 64
    // points from qc into rows qc - base.. of the slice; the element's inputs
    // are read again here.
    __device__ static void chunk_geometry(const FwdParams &prm, int64_t e, int blk, int qc, int base, float ys,
                                          Slice &sl) {
        const int lane = threadIdx.x & 63;
        const int q = qc + lane;
        const int row = q - base;
        if (q >= NQP) return;
        double W[16], sf = 0.0;
        if (q < NQ) {
            ElemIn E;
            load_elem_fwd(prm, e, E);
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
        } else {
#pragma unroll
            for (int k = 0; k < 16; ++k) W[k] = 0.0;
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) sl.W[row][k] = (float)W[k] * ys;
        sl.sf[row] = sf;
    }

    template <int TMV, int TNV>
    __device__ static void body(const FwdParams &prm, int64_t slot, int blk, int bi, int bj, Slice &sl) {
        constexpr int NC = WHOLE ? 1 : TNV;            // column fragments held apart from the row ones
        constexpr int NBRV = c_cdiv(TMV * 16, 64);     // FP64 load-vector rows per lane (no spare column)
        const int lane = threadIdx.x & 63;
        const int i16 = lane & 15, kg = lane >> 4;
        const int ra = bi * TM, cb = bj * TN;          // first row / column tile of the block
        const int64_t e = elem_of(prm, slot);
        SplitScale sc{1.0f, 1.0f};
        if constexpr (FORM == FP16X3) {
            ElemIn E;
            load_elem_fwd(prm, e, E);
            sc = Plain::elem_scale(prm, E, e);
        }
        // W in LDS carries the fp16 scale ys of A's columns; the fp16 table carries
        // 2^f16_shift, which the Y product must not: scale W down by it
        const float wsc = FORM == FP16X3 ? ldexpf(1.0f, -prm.f16_shift) : 1.0f;
        const int wr = i16 & 3;                        // the row of W this lane supplies
        // the lane of row r = 0 in the load-vector column adds w det J f (times yb)
        const float lsel = (LC::on && i16 == LC::lane) ? sc.yb : 0.0f;
        const bool bblk = !LC::on && bj == 0;

        f32x4 acc[TMV][TNV];
#pragma unroll
        for (int ti = 0; ti < TMV; ++ti)
#pragma unroll
            for (int tj = 0; tj < TNV; ++tj) acc[ti][tj] = f32x4{0, 0, 0, 0};
        double bacc[NBRV];
#pragma unroll
        for (int m = 0; m < NBRV; ++m) bacc[m] = 0.0;

        // two fragment sets alternate: the current K-block's, and the next one's in flight
        struct Set {
            Frag a[TMV], c[NC];
        };
        auto load_set = [&](int kb, Set &st) {
#pragma unroll
            for (int ti = 0; ti < TMV; ++ti) load_frag(prm, kb, ra + ti, lane, st.a[ti]);
            if constexpr (!WHOLE) {
#pragma unroll
                for (int tj = 0; tj < TNV; ++tj) load_frag(prm, kb, cb + tj, lane, st.c[tj]);
            }
        };
        auto colf = [&](const Set &st, int tj) -> const Frag & {
            if constexpr (WHOLE) return st.a[tj];
            else return st.c[tj];
        };
        // W_q of the points from base into the slice, and their share of the FP64 load vector
        auto fill = [&](int base) {
            wave_sync();
            for (int qc = base; qc < base + SQ && qc < NQP; qc += 64) chunk_geometry(prm, e, blk, qc, base, sc.ys, sl);
            wave_sync();
            if (bblk) {
#pragma unroll
                for (int m = 0; m < NBRV; ++m) {
                    const int row = ra * 16 + lane + 64 * m;
                    if (lane + 64 * m < TMV * 16 && row < N) {
                        const int cnt = NQ - base < SQ ? NQ - base : SQ;
                        double s = 0.0;
                        for (int qq = 0; qq < cnt; ++qq) s += sl.sf[qq] * prm.B64[(size_t)(base + qq) * 4 * NP + row];
                        bacc[m] += s;
                    }
                }
            }
        };
        auto step = [&](const Set &cur, Set &nxt, int kb) {
            if constexpr (CH == 1) {
                if (kb % KPC == 0) fill(kb * 8);       // a new chunk of points
            }
            // next K-block's fragments in flight during this one (the last re-reads itself)
            load_set(kb + 1 < NKB ? kb + 1 : kb, nxt);
            // left operands of the Y product: row wr of W of point 2 kg + h, split
            HV4 wh[2], wl[2];
            float sf[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int ql = (CH ? kb % KPC : kb) * 8 + 2 * kg + h;
                const float4 w4 = *(const float4 *)&sl.W[ql][4 * wr];
                const float wv[4] = {w4.x * wsc, w4.y * wsc, w4.z * wsc, w4.w * wsc};
                split4(wv, wh[h], wl[h]);
                sf[h] = (float)sl.sf[ql];
            }
            // Y of the block's column tiles (product by product over the tiles and halves,
            // so that consecutive MFMAs are independent), then split for the main product
            f32x4 t[TNV][2];
#pragma unroll
            for (int tj = 0; tj < TNV; ++tj)
#pragma unroll
                for (int h = 0; h < 2; ++h) t[tj][h] = mfma4b(wl[h], half_of(colf(cur, tj).h, h), f32x4{0, 0, 0, 0});
#pragma unroll
            for (int tj = 0; tj < TNV; ++tj)
#pragma unroll
                for (int h = 0; h < 2; ++h) t[tj][h] = mfma4b(wh[h], half_of(colf(cur, tj).l, h), t[tj][h]);
#pragma unroll
            for (int tj = 0; tj < TNV; ++tj)
#pragma unroll
                for (int h = 0; h < 2; ++h) t[tj][h] = mfma4b(wh[h], half_of(colf(cur, tj).h, h), t[tj][h]);
            HV yh[TNV], yl[TNV];
#pragma unroll
            for (int tj = 0; tj < TNV; ++tj) {
                float y[8];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    if (LC::on && (cb + tj) * 16 == LC::tile0) t[tj][h][0] += lsel * sf[h];
#pragma unroll
                    for (int r = 0; r < 4; ++r) y[4 * h + r] = t[tj][h][r];
                }
                Plain::split8(y, yh[tj], yl[tj]);
            }
            // main product, one product at a time over the tiles
#pragma unroll
            for (int ti = 0; ti < TMV; ++ti)
#pragma unroll
                for (int tj = 0; tj < TNV; ++tj) acc[ti][tj] = mfma32(cur.a[ti].l, yh[tj], acc[ti][tj]);
#pragma unroll
            for (int ti = 0; ti < TMV; ++ti)
#pragma unroll
                for (int tj = 0; tj < TNV; ++tj) acc[ti][tj] = mfma32(cur.a[ti].h, yl[tj], acc[ti][tj]);
#pragma unroll
            for (int ti = 0; ti < TMV; ++ti)
#pragma unroll
                for (int tj = 0; tj < TNV; ++tj) acc[ti][tj] = mfma32(cur.a[ti].h, yh[tj], acc[ti][tj]);
        };
        Set s0, s1;
        if constexpr (CH == 0) fill(0);                // all of the element's points
        load_set(0, s0);
        int kb = 0;
        for (; kb + 1 < NKB; kb += 2) {
            step(s0, s1, kb);
            step(s1, s0, kb + 1);
        }
        if (kb < NKB) step(s0, s1, kb);

        const float unscale = FORM == FP16X3 ? ldexpf(1.0f, -prm.f16_shift) / sc.ys : 1.0f;
        const float unscale_b = FORM == FP16X3 ? ldexpf(1.0f, -prm.f16_shift) / sc.yb : 1.0f;
        float *Aout = (float *)prm.A + offA_of(prm, e, N);
        float *bout = (float *)prm.b + offb_of(prm, e, N);
#pragma unroll
        for (int ti = 0; ti < TMV; ++ti)
#pragma unroll
            for (int tj = 0; tj < TNV; ++tj) {
                const int col = (cb + tj) * 16 + i16;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = (ra + ti) * 16 + 4 * kg + r;
                    if (row < N && col < N)
                        Aout[(size_t)row * N + col] = acc[ti][tj][r] * unscale;
                    else if (LC::on && row < N && col == N)
                        bout[row] = acc[ti][tj][r] * unscale_b;
                }
            }
        if (bblk) {
#pragma unroll
            for (int m = 0; m < NBRV; ++m) {
                const int row = ra * 16 + lane + 64 * m;
                if (lane + 64 * m < TMV * 16 && row < N) bout[row] = (float)bacc[m];
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
