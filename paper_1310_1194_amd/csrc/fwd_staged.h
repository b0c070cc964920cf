// LDS-staged forward kernels (the direct launches of every form).
//
// The reference table B (shape-function values and reference gradients at
// the quadrature points) is identical for every element of a degree, so the
// four waves of a workgroup share it: each stage of SP points (16x16x4 forms)
// or of one 8-point K-block (split forms) is copied from global memory into
// LDS once per workgroup with coalesced 16-byte loads, double-buffered, and
// the copy of stage s+1 is in flight while the waves run the MFMAs of stage
// s.  This is the MI355X counterpart of the paper's keeping of precomputed
// shape functions in fast local memory (Sec. 2.2 and Sec. 4, SR variants),
// without its size limit: the stage size is fixed, whatever the degree.
//
// Every wave still owns one work item (element, TM x TN tile block) and its
// own slice of LDS for the per-point coefficient blocks W_q.  Waves without
// an item (the tail of the grid) take part in the copies and barriers only.
#pragma once
#include "fwd_kernels.h"

namespace feint {

// Cooperative copy of NV 16-byte vectors from `src` (global) into `dst`
// (LDS) by the 256 threads of a workgroup, split into fetch (to registers)
// and put (to LDS) so that the global latency overlaps other work.
template <int NV>
struct StageCopy {
    static constexpr int VPT = c_cdiv(NV, 256);
    uint4 r[VPT];
    __device__ void fetch(const uint4 *__restrict__ src) {
#pragma unroll
        for (int v = 0; v < VPT; ++v) {
            const int i = threadIdx.x + 256 * v;
            if (i < NV) r[v] = src[i];
        }
    }
    __device__ void put(uint4 *dst) const {
#pragma unroll
        for (int v = 0; v < VPT; ++v) {
            const int i = threadIdx.x + 256 * v;
            if (i < NV) dst[i] = r[v];
        }
    }
};

// ---------------------------------------------------------------------------
// 16x16x4 forms (FP64, FP32), stages of SP points (SP divides 64).
// ---------------------------------------------------------------------------
template <int P, typename T, int TM, int TN, int SP, int R = 0>
struct K4S {
    static constexpr int N = c_nshp(P), NP = c_pad16(N), NT = NP / 16, NQ = c_nq_rule(P, R);
    static constexpr int BM = c_cdiv(NT, TM), BN = c_cdiv(NT, TN), NBLK = BM * BN;
    static constexpr int EPI = 1;
    static constexpr int NBR = c_cdiv(TM * 16, 64);
    static constexpr int NSTAGE = c_cdiv(NQ, SP);
    static constexpr int STAGE_T = SP * 4 * NP;                  // T values per stage
    static constexpr int STAGE_V = STAGE_T * (int)sizeof(T) / 16;
    static_assert(64 % SP == 0, "stages must tile the 64-point chunks");
    typedef typename AccT<T>::type V4;
    typedef LoadCol<P> LC;

    struct Smem {
        T B[2][STAGE_T];
        T W[4][64][WROW<T>::value];   // padded rows: conflict-free per-lane writes
        double sf[4][64];
    };

    template <int TMV, int TNV>
    __device__ static void body(const FwdParams &prm, int64_t slot, int blk, int bi, int bj, int wave, bool active, Smem &sm) {
        constexpr int NBRV = c_cdiv(TMV * 16, 64);
        const int lane = threadIdx.x & 63;
        const int i16 = lane & 15, kg = lane >> 4;
        const int a0 = bi * TM * 16, b0 = bj * TN * 16;
        const int64_t e = active ? elem_of(prm, slot) : 0;
        ElemIn E;
        if (active) load_elem_fwd(prm, e, E);
        const T *tab = sizeof(T) == 8 ? (const T *)(const void *)prm.B64 : (const T *)(const void *)prm.B32;
        V4 acc[TMV][TNV];
#pragma unroll
        for (int ti = 0; ti < TMV; ++ti)
#pragma unroll
            for (int tj = 0; tj < TNV; ++tj) acc[ti][tj] = V4{0, 0, 0, 0};
        double bacc[NBRV];
#pragma unroll
        for (int m = 0; m < NBRV; ++m) bacc[m] = 0.0;

        StageCopy<STAGE_V> cp;
        cp.fetch((const uint4 *)tab);
        cp.put((uint4 *)sm.B[0]);
        __syncthreads();
        for (int s = 0; s < NSTAGE; ++s) {
            const int q0 = s * SP, buf = s & 1;
            if (s + 1 < NSTAGE) cp.fetch((const uint4 *)(tab + (size_t)(s + 1) * STAGE_T));
            if (active) {
                const int qc = q0 & ~63;
                if (q0 == qc) {                          // new 64-point chunk of W_q
                    const int cnt = NQ - qc < 64 ? NQ - qc : 64;
                    wave_sync();
                    if (lane < cnt) {
                        const int q = qc + lane;
                        const double *qp = prm.qw + 4 * q;
                        double W[16], sf;
                        field_at(prm, e, qp[0], qp[1], qp[2], E);
                        const double det = point_block(E, qp[0], qp[1], qp[2], qp[3], W, sf);
                        if (!(det > 0.0) && prm.status) atomicOr(prm.status, 1u);
#pragma unroll
                        for (int k = 0; k < 16; ++k) sm.W[wave][lane][k] = (T)W[k];
                        sm.sf[wave][lane] = sf;
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
                                double acc_b = 0.0;
                                for (int qq = 0; qq < cnt; ++qq)
                                    acc_b += sm.sf[wave][qq] * prm.B64[(size_t)(qc + qq) * 4 * NP + row];
                                bacc[m] += acc_b;
                            }
                        }
                    }
                }
                const int cnt = NQ - q0 < SP ? NQ - q0 : SP;
                for (int qq = 0; qq < cnt; ++qq) {
                    const int ql = q0 + qq - qc;
                    const T w0 = sm.W[wave][ql][4 * kg + 0], w1 = sm.W[wave][ql][4 * kg + 1];
                    const T w2 = sm.W[wave][ql][4 * kg + 2], w3 = sm.W[wave][ql][4 * kg + 3];
                    const T *Bq = sm.B[buf] + qq * 4 * NP;
                    T yf[TNV], af[TMV];
#pragma unroll
                    for (int tj = 0; tj < TNV; ++tj) {
                        {
                            const T *bp = Bq + b0 + tj * 16 + i16;
                            yf[tj] = w0 * bp[0] + w1 * bp[NP] + w2 * bp[2 * NP] + w3 * bp[3 * NP];
                        }
                        if (LC::on && b0 + tj * 16 == LC::tile0 && i16 == LC::lane)   // load-vector column
                            yf[tj] = kg == 0 ? (T)sm.sf[wave][ql] : (T)0;
                    }
#pragma unroll
                    for (int ti = 0; ti < TMV; ++ti) {
                        af[ti] = Bq[kg * NP + a0 + ti * 16 + i16];
                    }
#pragma unroll
                    for (int ti = 0; ti < TMV; ++ti)
#pragma unroll
                        for (int tj = 0; tj < TNV; ++tj)
                            acc[ti][tj] = mfma4(af[ti], yf[tj], acc[ti][tj]);
                }
            }
            if (s + 1 < NSTAGE) cp.put((uint4 *)sm.B[buf ^ 1]);
            __syncthreads();
        }
        if (!active) return;
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

    // Tile counts of the last row/column block are compile-time constants,
    // so the inner loops carry no bounds tests and stay one basic block.
    __device__ static void run(const FwdParams &prm, int64_t slot, int blk, int wave, bool active, Smem &sm) {
        const int bi = blk / BN, bj = blk % BN;
        constexpr int TML = NT - (BM - 1) * TM, TNL = NT - (BN - 1) * TN;
        if (bi == BM - 1) {
            if (bj == BN - 1) body<TML, TNL>(prm, slot, blk, bi, bj, wave, active, sm);
            else body<TML, TN>(prm, slot, blk, bi, bj, wave, active, sm);
        } else {
            if (bj == BN - 1) body<TM, TNL>(prm, slot, blk, bi, bj, wave, active, sm);
            else body<TM, TN>(prm, slot, blk, bi, bj, wave, active, sm);
        }
    }
};

// ---------------------------------------------------------------------------
// Split forms (bf16x3, fp16x3), one 8-point K-block per stage.  A stage holds
// the hi and lo A fragments [NP][32] and, when SY, the FP32 columns
// [8][NP][4] the B fragments are formed from (otherwise those are read from
// global memory, for degrees whose double-buffered stage would not fit).
// ---------------------------------------------------------------------------
template <int P, int FORM, int TM, int TN, bool SY, int R = 0>
struct K32S {
    static constexpr int N = c_nshp(P), NP = c_pad16(N), NT = NP / 16, NQ = c_nq_rule(P, R);
    static constexpr int NQP = c_pad8(NQ), NKB = NQP / 8;
    static constexpr int BM = c_cdiv(NT, TM), BN = c_cdiv(NT, TN), NBLK = BM * BN;
    static constexpr int EPI = 1;
    static constexpr int NBR = c_cdiv(TM * 16, 64);
    static constexpr int VA = NP * 32 * 2 / 16;        // 16-byte vectors of one split half
    static constexpr int VY = SY ? 8 * NP * 4 * 4 / 16 : 0;
    static constexpr int NV = 2 * VA + VY;
    typedef typename SplitT<FORM>::vec HV;
    typedef typename SplitT<FORM>::scal HS;
    typedef LoadCol<P> LC;

    struct Smem {
        uint4 S[2][NV];      // [hi A | lo A | FP32 columns]
        float W[4][64][WROW<float>::value];   // padded rows: conflict-free per-lane writes
        double sf[4][64];
    };

    __device__ static void fetch(const FwdParams &prm, int kb, uint4 (&r)[c_cdiv(NV, 256)]) {
        const uint4 *hi = (const uint4 *)(prm.Bhi + (size_t)kb * NP * 32);
        const uint4 *lo = (const uint4 *)(prm.Blo + (size_t)kb * NP * 32);
        const uint4 *yc = (const uint4 *)(prm.Ycf + (size_t)kb * NP * 32);
#pragma unroll
        for (int v = 0; v < c_cdiv(NV, 256); ++v) {
            const int i = threadIdx.x + 256 * v;
            if (i < VA) r[v] = hi[i];
            else if (i < 2 * VA) r[v] = lo[i - VA];
            else if (i < NV) r[v] = yc[i - 2 * VA];
        }
    }
    __device__ static void put(uint4 *dst, const uint4 (&r)[c_cdiv(NV, 256)]) {
#pragma unroll
        for (int v = 0; v < c_cdiv(NV, 256); ++v) {
            const int i = threadIdx.x + 256 * v;
            if (i < NV) dst[i] = r[v];
        }
    }

    template <int TMV, int TNV>
    __device__ static void body(const FwdParams &prm, int64_t slot, int blk, int bi, int bj, int wave, bool active, Smem &sm) {
        constexpr int NBRV = c_cdiv(TMV * 16, 64);
        typedef K32<P, FORM, TMV, TNV, R> Plain;
        const int lane = threadIdx.x & 63;
        const int i16 = lane & 15, kg = lane >> 4;
        const int a0 = bi * TM * 16, b0 = bj * TN * 16;
        const int64_t e = active ? elem_of(prm, slot) : 0;
        ElemIn E;
        float ys = 1.0f, yb = 1.0f;
        if (active) {
            load_elem_fwd(prm, e, E);
            if (FORM == FP16X3) {
                const SplitScale sc = Plain::elem_scale(prm, E, e);
                ys = sc.ys;
                yb = sc.yb;
            }
        }
        f32x4 acc[TMV][TNV];
#pragma unroll
        for (int ti = 0; ti < TMV; ++ti)
#pragma unroll
            for (int tj = 0; tj < TNV; ++tj) acc[ti][tj] = f32x4{0, 0, 0, 0};
        double bacc[NBRV];
#pragma unroll
        for (int m = 0; m < NBRV; ++m) bacc[m] = 0.0;

        uint4 pre[c_cdiv(NV, 256)];
        fetch(prm, 0, pre);
        put(sm.S[0], pre);
        __syncthreads();
        for (int kb = 0; kb < NKB; ++kb) {
            const int q0 = kb * 8, buf = kb & 1;
            if (kb + 1 < NKB) fetch(prm, kb + 1, pre);
            if (active) {
                const int qc = q0 & ~63;
                if (q0 == qc) {
                    const int cnt = NQP - qc < 64 ? NQP - qc : 64;
                    wave_sync();
                    if (lane < cnt) {
                        const int q = qc + lane;
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
                        } else {
#pragma unroll
                            for (int k = 0; k < 16; ++k) W[k] = 0.0;
                        }
#pragma unroll
                        for (int k = 0; k < 16; ++k) sm.W[wave][lane][k] = (float)W[k] * ys;
                        sm.sf[wave][lane] = sf;
                    }
                    wave_sync();
                    if (!LC::on && bj == 0) {
#pragma unroll
                        for (int m = 0; m < NBRV; ++m) {
                            const int row = a0 + lane + 64 * m;
                            if (lane + 64 * m < TMV * 16 && row < N) {
                                double acc_b = 0.0;
                                for (int qq = 0; qq < cnt && qc + qq < NQ; ++qq)
                                    acc_b += sm.sf[wave][qq] * prm.B64[(size_t)(qc + qq) * 4 * NP + row];
                                bacc[m] += acc_b;
                            }
                        }
                    }
                }
                const int qa = 2 * kg;                       // this lane's two points in the block
                const float *Wa = sm.W[wave][q0 + qa - qc];
                const float *Wb = sm.W[wave][q0 + qa + 1 - qc];
                float wa[16], wb[16];
#pragma unroll
                for (int k = 0; k < 16; ++k) { wa[k] = Wa[k]; wb[k] = Wb[k]; }
                const HS *Ah = (const HS *)(const void *)sm.S[buf];
                const HS *Al = (const HS *)(const void *)(sm.S[buf] + VA);
                const float *Yc = SY ? (const float *)(const void *)(sm.S[buf] + 2 * VA)
                                     : prm.Ycf + (size_t)kb * NP * 32;
                HV yh[TNV], yl[TNV], ah[TMV], al[TMV];
#pragma unroll
                for (int tj = 0; tj < TNV; ++tj) {
                    {
                        const float *yp = Yc + ((size_t)(b0 / 16 + tj) * 64 + lane) * 8;
                        const float4 s0 = *(const float4 *)yp;
                        const float4 s1 = *(const float4 *)(yp + 4);
                        float y[8];
                        y[0] = wa[0] * s0.x + wa[1] * s0.y + wa[2] * s0.z + wa[3] * s0.w;
                        y[4] = wb[0] * s1.x + wb[1] * s1.y + wb[2] * s1.z + wb[3] * s1.w;
#pragma unroll
                        for (int r = 1; r < 4; ++r) {
                            y[r] = wa[4 * r + 1] * s0.y + wa[4 * r + 2] * s0.z + wa[4 * r + 3] * s0.w;
                            y[4 + r] = wb[4 * r + 1] * s1.y + wb[4 * r + 2] * s1.z + wb[4 * r + 3] * s1.w;
                        }
                        if (LC::on && b0 + tj * 16 == LC::tile0 && i16 == LC::lane) {   // load-vector column
#pragma unroll
                            for (int r = 0; r < 8; ++r) y[r] = 0.0f;
                            y[0] = (float)sm.sf[wave][q0 + qa - qc] * yb;
                            y[4] = (float)sm.sf[wave][q0 + qa + 1 - qc] * yb;
                        }
                        Plain::split8(y, yh[tj], yl[tj]);
                    }
                }
#pragma unroll
                for (int ti = 0; ti < TMV; ++ti) {
                    {
                        const int o = ((a0 / 16 + ti) * 64 + lane) * 8;
                        ah[ti] = *(const HV *)(Ah + o);
                        al[ti] = *(const HV *)(Al + o);
                    }
                }
                // product by product over the tiles: consecutive MFMAs are independent
#pragma unroll
                for (int ti = 0; ti < TMV; ++ti)
#pragma unroll
                    for (int tj = 0; tj < TNV; ++tj) acc[ti][tj] = mfma32(al[ti], yh[tj], acc[ti][tj]);
#pragma unroll
                for (int ti = 0; ti < TMV; ++ti)
#pragma unroll
                    for (int tj = 0; tj < TNV; ++tj) acc[ti][tj] = mfma32(ah[ti], yl[tj], acc[ti][tj]);
#pragma unroll
                for (int ti = 0; ti < TMV; ++ti)
#pragma unroll
                    for (int tj = 0; tj < TNV; ++tj) acc[ti][tj] = mfma32(ah[ti], yh[tj], acc[ti][tj]);
            }
            if (kb + 1 < NKB) put(sm.S[buf ^ 1], pre);
            __syncthreads();
        }
        if (!active) return;
        const float unscale = FORM == FP16X3 ? ldexpf(1.0f, -prm.f16_shift) / ys : 1.0f;
        const float unscale_b = FORM == FP16X3 ? ldexpf(1.0f, -prm.f16_shift) / yb : 1.0f;
        float *Aout = (float *)prm.A + offA_of(prm, e, N);
        float *bout = (float *)prm.b + offb_of(prm, e, N);
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
        if (!LC::on && bj == 0) {
#pragma unroll
            for (int m = 0; m < NBRV; ++m) {
                const int row = a0 + lane + 64 * m;
                if (lane + 64 * m < TMV * 16 && row < N) bout[row] = (float)bacc[m];
            }
        }
    }

    // Tile counts of the last row/column block are compile-time constants,
    // so the inner loops carry no bounds tests and stay one basic block.
    __device__ static void run(const FwdParams &prm, int64_t slot, int blk, int wave, bool active, Smem &sm) {
        const int bi = blk / BN, bj = blk % BN;
        constexpr int TML = NT - (BM - 1) * TM, TNL = NT - (BN - 1) * TN;
        if (bi == BM - 1) {
            if (bj == BN - 1) body<TML, TNL>(prm, slot, blk, bi, bj, wave, active, sm);
            else body<TML, TN>(prm, slot, blk, bi, bj, wave, active, sm);
        } else {
            if (bj == BN - 1) body<TM, TNL>(prm, slot, blk, bi, bj, wave, active, sm);
            else body<TM, TN>(prm, slot, blk, bi, bj, wave, active, sm);
        }
    }
};

// MINW: waves per SIMD the register allocation must allow (1 = no limit).
template <class KER, int MINW>
__global__ __launch_bounds__(256, MINW) void fwd_staged(FwdParams prm) {
    __shared__ typename KER::Smem sm;
    const int wave = wave_uniform(threadIdx.x >> 6);
    const int64_t item = (int64_t)blockIdx.x * 4 + wave;
    const bool active = item < items_for<KER>(prm.ne);
    const int64_t it = active ? item : 0;
    KER::run(prm, it / KER::NBLK, (int)(it % KER::NBLK), wave, active, sm);
}

}  // namespace feint

