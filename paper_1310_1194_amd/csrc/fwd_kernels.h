// Forward element-integration kernels (hot path of Algorithm 1 generalised
// to convection-diffusion-reaction + load vector), gfx950.
//
// Work decomposition.  The element matrix A_e = sum_q B_q^T W_q B_q is a GEMM
// with M = N = n (padded to 16) and K = 4 nq: B (4nq x n) is the same for every
// element of a degree (kept in L2 and reused by every wave), W_q (4x4) is the
// per-point coefficient block computed in FP64 from the Jacobian.  One wave
// owns a TM x TN block of 16x16 output tiles of one element; a workgroup holds
// four such waves.  Per chunk of 64 points each lane computes one point's W_q
// (FP64 geometry) into the wave's LDS slice; then, point by point (16x16x4
// forms) or eight points at a time (16x16x32 split forms), the wave forms the
// B-operand fragments Y = W_q B_q in registers and issues TM x TN MFMAs whose
// A operands are rows of B read straight from the table.  The load vector
// b_e = sum_q w_q det J_q f phi(q) rides along in the contraction where the
// padded width leaves a spare column (n < NP: every degree but p = 7): column
// n of Y carries Z[(q, r)] = (r == 0 ? w_q det J_q f : 0), so column n of the
// accumulator is b_e, in the form's precision.  At p = 7 it is accumulated
// in FP64 by the waves of the first column block.
#pragma once
#include "device_common.h"
#include "launch.h"

namespace feint {

enum FormId { F64 = 0, F32 = 1, BF16X3 = 2, FP16X3 = 3 };

// Row of the 16x16 output tile held in accumulator register r of lane l.
template <typename T> __device__ inline int acc_row(int lane, int r);
template <> __device__ inline int acc_row<double>(int lane, int r) { return 4 * r + (lane >> 4); }
template <> __device__ inline int acc_row<float>(int lane, int r) { return 4 * (lane >> 4) + r; }

template <typename T> struct AccT;
template <> struct AccT<double> { typedef f64x4 type; };
template <> struct AccT<float> { typedef f32x4 type; };

template <int FORM> struct SplitT;
template <> struct SplitT<BF16X3> { typedef bf16x8 vec; typedef __bf16 scal; };
template <> struct SplitT<FP16X3> { typedef f16x8 vec; typedef _Float16 scal; };

// Element handled by a work item (identity unless a permutation is given).
__device__ inline int64_t elem_of(const FwdParams &prm, int64_t slot) {
    return prm.perm ? (int64_t)prm.perm[slot] : slot;
}
__device__ inline int64_t offA_of(const FwdParams &prm, int64_t e, int n) {
    return prm.offA ? prm.offA[e] : e * (int64_t)n * n;
}
__device__ inline int64_t offb_of(const FwdParams &prm, int64_t e, int n) {
    return prm.offb ? prm.offb[e] : e * (int64_t)n;
}

// Element inputs of a forward work item: the vertices, and the constant
// coefficients unless the launch carries vertex fields.
__device__ inline void load_elem_fwd(const FwdParams &prm, int64_t e, ElemIn &E) {
    if (prm.fD) {
        // every member defined on both paths: a member left unset on one of
        // them keeps the whole struct out of registers (private memory)
#pragma unroll
        for (int i = 0; i < 18; ++i) E.X[i] = prm.coords[18 * e + i];
#pragma unroll
        for (int m = 0; m < 9; ++m) E.D[m] = 0.0;
#pragma unroll
        for (int m = 0; m < 3; ++m) E.be[m] = 0.0;
        E.c = 0.0;
        E.f = 0.0;
    } else {
        load_elem(prm.coords, prm.D, prm.beta, prm.c, prm.f, e, E);
    }
}

// Coefficients at reference point (xi1, xi2, zeta) when the launch carries
// vertex fields: the six vertex values combined with the geometry shape
// functions N_a = lambda_a (1-zeta)/2, N_{a+3} = lambda_a (1+zeta)/2, i.e. the
// fields live in the same bilinear space as the geometry.  No-op otherwise.
__device__ inline void field_at(const FwdParams &prm, int64_t e, double xi1, double xi2, double ze, ElemIn &E) {
    if (!prm.fD) return;
    const double t = 0.5 * (1.0 + ze), s = 0.5 * (1.0 - ze), l0 = 1.0 - xi1 - xi2;
#pragma unroll
    for (int m = 0; m < 9; ++m) E.D[m] = 0.0;
#pragma unroll
    for (int m = 0; m < 3; ++m) E.be[m] = 0.0;
    E.c = 0.0;
    E.f = 0.0;
#pragma unroll 1
    for (int a = 0; a < 6; ++a) {                // one vertex at a time: 14 loads in flight
        const double *Da = prm.fD + (6 * e + a) * 9, *ba = prm.fbeta + (6 * e + a) * 3;
        const double Na = (a % 3 == 0 ? l0 : (a % 3 == 1 ? xi1 : xi2)) * (a < 3 ? s : t);
#pragma unroll
        for (int m = 0; m < 9; ++m) E.D[m] += Na * Da[m];
#pragma unroll
        for (int m = 0; m < 3; ++m) E.be[m] += Na * ba[m];
        E.c += Na * prm.fc[6 * e + a];
        E.f += Na * prm.ff[6 * e + a];
    }
}

// The load-vector column of an element with NS shape functions: whether it
// exists (a spare padded column), the first column of its 16-wide tile and
// its lane in that tile.
template <int NS> struct LoadColN {
    static constexpr int N = NS;
    static constexpr bool on = N < c_pad16(N);
    static constexpr int tile0 = N / 16 * 16, lane = N % 16;
};
template <int P> using LoadCol = LoadColN<c_nshp(P)>;

// Element geometry of a forward kernel: the element record, the shape-function
// and point counts, the element load, the coefficients at a point, W_q and the
// mapped point.  qp = (reference coordinates, weight) of the point.
struct PrismGeo {
    typedef ElemIn Elem;
    static constexpr bool LOAD = true;          // the element has a load vector
    __host__ __device__ static constexpr int nshp(int p) { return c_nshp(p); }
    __host__ __device__ static constexpr int nq(int p, int r) { return c_nq_rule(p, r); }
    __device__ static void load(const FwdParams &prm, int64_t e, Elem &E) { load_elem_fwd(prm, e, E); }
    __device__ static void coeffs(const FwdParams &prm, int64_t e, const double *qp, Elem &E) {
        field_at(prm, e, qp[0], qp[1], qp[2], E);
    }
    __device__ static double block(const Elem &E, const double *qp, double W[16], double &sf) {
        return point_block(E, qp[0], qp[1], qp[2], qp[3], W, sf);
    }
    __device__ static void map(const Elem &E, const double *qp, double x[3]) { prism_map(E.X, qp[0], qp[1], qp[2], x); }
};

// The paper's own term on prisms (its eq. (1), Laplace): A_ab = sum_q w_q det J_q
// grad phi_a . grad phi_b with no load vector, so W_q = w det J [[0, 0], [0, K K^T]];
// only the vertex coordinates are read.
struct ElemX {
    double X[18];   // vertices v0..v5
};
struct PrismLaplaceGeo {
    typedef ElemX Elem;
    static constexpr bool LOAD = false;
    __host__ __device__ static constexpr int nshp(int p) { return c_nshp(p); }
    __host__ __device__ static constexpr int nq(int p, int r) { return c_nq_rule(p, r); }
    __device__ static void load(const FwdParams &prm, int64_t e, Elem &E) {
#pragma unroll
        for (int i = 0; i < 18; ++i) E.X[i] = prm.coords[18 * e + i];
    }
    __device__ static void coeffs(const FwdParams &, int64_t, const double *, Elem &) {}
    __device__ static double block(const Elem &E, const double *qp, double W[16], double &sf) {
        double K[9];
        const double det = prism_jacobian(E.X, qp[0], qp[1], qp[2], K);
        laplace_block(K, qp[3] * det, W);
        sf = 0.0;
        return det;
    }
    __device__ static void map(const Elem &E, const double *qp, double x[3]) { prism_map(E.X, qp[0], qp[1], qp[2], x); }
};

// Hexahedra (Table 1's tensor-product element): (p+1)^3 shape functions and
// (p+1)^3 Gauss points; coordinates [ne][8][3], coefficients per element.
struct HexGeo {
    typedef ElemHex Elem;
    static constexpr bool LOAD = true;
    __host__ __device__ static constexpr int nshp(int p) { return (p + 1) * (p + 1) * (p + 1); }
    __host__ __device__ static constexpr int nq(int p, int) { return (p + 1) * (p + 1) * (p + 1); }
    __device__ static void load(const FwdParams &prm, int64_t e, Elem &E) {
#pragma unroll
        for (int i = 0; i < 24; ++i) E.X[i] = prm.coords[24 * e + i];
#pragma unroll
        for (int i = 0; i < 9; ++i) E.D[i] = prm.D[9 * e + i];
#pragma unroll
        for (int i = 0; i < 3; ++i) E.be[i] = prm.beta[3 * e + i];
        E.c = prm.c[e];
        E.f = prm.f[e];
    }
    __device__ static void coeffs(const FwdParams &, int64_t, const double *, Elem &) {}
    __device__ static double block(const Elem &E, const double *qp, double W[16], double &sf) {
        return point_block_hex(E, qp[0], qp[1], qp[2], qp[3], W, sf);
    }
    __device__ static void map(const Elem &E, const double *qp, double x[3]) { hex_map(E.X, qp[0], qp[1], qp[2], x); }
};

// Tetrahedra (Table 1's complete-basis 3D element): (p+1)(p+2)(p+3)/6 shape
// functions, (p+2)^3 collapsed Gauss points; coordinates [ne][4][3].
struct TetGeo {
    typedef ElemTet Elem;
    static constexpr bool LOAD = true;
    __host__ __device__ static constexpr int nshp(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }
    __host__ __device__ static constexpr int nq(int p, int) { return (p + 2) * (p + 2) * (p + 2); }
    __device__ static void load(const FwdParams &prm, int64_t e, Elem &E) {
#pragma unroll
        for (int i = 0; i < 12; ++i) E.X[i] = prm.coords[12 * e + i];
#pragma unroll
        for (int i = 0; i < 9; ++i) E.D[i] = prm.D[9 * e + i];
#pragma unroll
        for (int i = 0; i < 3; ++i) E.be[i] = prm.beta[3 * e + i];
        E.c = prm.c[e];
        E.f = prm.f[e];
    }
    __device__ static void coeffs(const FwdParams &, int64_t, const double *, Elem &) {}
    __device__ static double block(const Elem &E, const double *qp, double W[16], double &sf) {
        return point_block_tet(E, qp[3], W, sf);
    }
    __device__ static void map(const Elem &E, const double *qp, double x[3]) { tet_map(E.X, qp[0], qp[1], qp[2], x); }
};

// ---------------------------------------------------------------------------
// 16x16x4 forms (FP64, FP32): one point (4 K-rows) per MFMA.
// ---------------------------------------------------------------------------
template <int P, typename T, int TM, int TN, int R = 0, class G = PrismGeo>
struct K4 {
    static constexpr int N = G::nshp(P), NP = c_pad16(N), NT = NP / 16, NQ = G::nq(P, R);
    static constexpr int BM = c_cdiv(NT, TM), BN = c_cdiv(NT, TN), NBLK = BM * BN;
    static constexpr int EPI = 1;                      // element slots per work item
    static constexpr int NBR = c_cdiv(TM * 16, 64);   // load-vector rows per lane
    typedef typename AccT<T>::type V4;
    typedef LoadColN<N> LC;

    struct Slice {                    // one wave's LDS
        T W[64][WROW<T>::value];      // padded rows: conflict-free per-lane writes
        double sf[64];
    };
    struct Smem { Slice w[4]; };

    // One work item: block `blk` of element slot `slot`, with the wave's LDS
    // slice `sl`.
    template <int TMV, int TNV>
    __device__ static void body(const FwdParams &prm, int64_t slot, int blk, int bi, int bj, Slice &sl) {
        constexpr int NBRV = c_cdiv(TMV * 16, 64);
        const int lane = threadIdx.x & 63;
        const int i16 = lane & 15, kg = lane >> 4;
        const int a0 = bi * TM * 16, b0 = bj * TN * 16;
        const int64_t e = elem_of(prm, slot);
        typename G::Elem E;
        G::load(prm, e, E);
        const T *Bt = sizeof(T) == 8 ? (const T *)(const void *)prm.B64 : (const T *)(const void *)prm.B32;
        V4 acc[TMV][TNV];
#pragma unroll
        for (int ti = 0; ti < TMV; ++ti)
#pragma unroll
            for (int tj = 0; tj < TNV; ++tj) acc[ti][tj] = V4{0, 0, 0, 0};
        double bacc[NBRV];
#pragma unroll
        for (int m = 0; m < NBRV; ++m) bacc[m] = 0.0;

        for (int qc = 0; qc < NQ; qc += 64) {
            const int cnt = NQ - qc < 64 ? NQ - qc : 64;
            if (lane < cnt) {
                const int q = qc + lane;
                const double *qp = prm.qw + 4 * q;
                double W[16], sf;
                G::coeffs(prm, e, qp, E);
                const double det = G::block(E, qp, W, sf);
                if (!(det > 0.0) && prm.status) atomicOr(prm.status, 1u);
#pragma unroll
                for (int k = 0; k < 16; ++k) sl.W[lane][k] = (T)W[k];
                sl.sf[lane] = sf;
                if (prm.xq && blk == 0) {
                    double x[3];
                    G::map(E, qp, x);
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
                        double s = 0.0;
                        for (int qq = 0; qq < cnt; ++qq)
                            s += sl.sf[qq] * prm.B64[(size_t)(qc + qq) * 4 * NP + row];
                        bacc[m] += s;
                    }
                }
            }
            // The table operands of point qq + 1 (the four B rows of the
            // lane's columns and the A fragments) are loaded while point qq is
            // contracted.
            auto fetch = [&](int qq, T (&bpv)[TNV][4], T (&afv)[TMV]) {
                const T *Bq = Bt + (size_t)(qc + qq) * 4 * NP;
#pragma unroll
                for (int tj = 0; tj < TNV; ++tj)
#pragma unroll
                    for (int r = 0; r < 4; ++r) bpv[tj][r] = Bq[r * NP + b0 + tj * 16 + i16];
#pragma unroll
                for (int ti = 0; ti < TMV; ++ti) afv[ti] = Bq[kg * NP + a0 + ti * 16 + i16];
            };
            T bpc[TNV][4], afc[TMV];
            fetch(0, bpc, afc);
            for (int qq = 0; qq < cnt; ++qq) {
                T bpn[TNV][4], afn[TMV];
                fetch(qq + 1 < cnt ? qq + 1 : qq, bpn, afn);
                const T w0 = sl.W[qq][4 * kg + 0], w1 = sl.W[qq][4 * kg + 1];
                const T w2 = sl.W[qq][4 * kg + 2], w3 = sl.W[qq][4 * kg + 3];
                T yf[TNV];
#pragma unroll
                for (int tj = 0; tj < TNV; ++tj) {
                    yf[tj] = w0 * bpc[tj][0] + w1 * bpc[tj][1] + w2 * bpc[tj][2] + w3 * bpc[tj][3];
                    if (LC::on && b0 + tj * 16 == LC::tile0 && i16 == LC::lane)   // load-vector column
                        yf[tj] = kg == 0 ? (T)sl.sf[qq] : (T)0;
                }
#pragma unroll
                for (int ti = 0; ti < TMV; ++ti)
#pragma unroll
                    for (int tj = 0; tj < TNV; ++tj)
                        acc[ti][tj] = mfma4(afc[ti], yf[tj], acc[ti][tj]);
#pragma unroll
                for (int tj = 0; tj < TNV; ++tj)
#pragma unroll
                    for (int r = 0; r < 4; ++r) bpc[tj][r] = bpn[tj][r];
#pragma unroll
                for (int ti = 0; ti < TMV; ++ti) afc[ti] = afn[ti];
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

    // Tile counts of the last row/column block are compile-time constants,
    // so the inner loops carry no bounds tests and stay one basic block.
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

// Scales of the fp16 split form (1 for bf16): ys multiplies the columns of A,
// yb the load-vector column.
struct SplitScale {
    float ys, yb;
};

// The power of two that places a positive bound m in [2^13, 2^14) (1 for a
// zero or non-finite bound), clamped to 2^+-60.
__device__ inline float pow2_scale(double m) {
    if (!(m > 0.0) || !(m < 1e300)) return 1.0f;
    const int ex = 13 - (int)floor(log2(m));
    return ldexpf(1.0f, ex < -60 ? -60 : (ex > 60 ? 60 : ex));
}

// ---------------------------------------------------------------------------
// 16x16x32 split forms (bf16x3, fp16x3): eight points (32 K-rows) per MFMA.
// x = hi + lo with hi = rn(x), lo = rn(x - hi); products hi*hi + hi*lo + lo*hi
// accumulate in FP32.  B is split once on the host; Y = W_q B_q is formed in
// FP32 from the FP32 table and split in registers.  The fp16 form scales B by
// 2^f16_shift and Y by a per-element power of two so that both use the
// normal range, and unscales exactly at the store.
// ---------------------------------------------------------------------------
template <int P, int FORM, int TM, int TN, int R = 0, class G = PrismGeo>
struct K32 {
    static constexpr int N = G::nshp(P), NP = c_pad16(N), NT = NP / 16, NQ = G::nq(P, R);
    static constexpr int NQP = c_pad8(NQ);
    static constexpr int BM = c_cdiv(NT, TM), BN = c_cdiv(NT, TN), NBLK = BM * BN;
    static constexpr int EPI = 1;
    static constexpr int NBR = c_cdiv(TM * 16, 64);
    typedef typename SplitT<FORM>::vec HV;
    typedef typename SplitT<FORM>::scal HS;
    typedef LoadColN<N> LC;

    struct Slice {                            // one wave's LDS
        float W[64][WROW<float>::value];      // padded rows: conflict-free per-lane writes
        double sf[64];
    };
    struct Smem { Slice w[4]; };

    // Per-element power-of-two scales of the fp16 form: ys for the columns of
    // A (a bound on |Y| = |W_q B_q|, the largest row sum of |W_q| over the
    // element's points times max |B|) and yb for the load-vector column (the
    // largest |w det J f|), each placing its bound in [2^13, 2^14).  The two
    // are separate because f can be orders of magnitude below the other
    // coefficients: under the scale of A the load-vector column would sink
    // into the subnormal range of fp16 and lose its relative precision.
    __device__ static SplitScale elem_scale(const FwdParams &prm, const typename G::Elem &E0, int64_t e) {
        typename G::Elem E = E0;
        const int lane = threadIdx.x & 63;
        double m = 0.0, mb = 0.0;
        for (int qc = 0; qc < NQ; qc += 64) {
            const int q = qc + lane;
            if (q < NQ) {
                const double *qp = prm.qw + 4 * q;
                double W[16], sf;
                G::coeffs(prm, e, qp, E);
                G::block(E, qp, W, sf);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const double s = fabs(W[4 * r]) + fabs(W[4 * r + 1]) + fabs(W[4 * r + 2]) + fabs(W[4 * r + 3]);
                    m = s > m ? s : m;
                }
                mb = fabs(sf) > mb ? fabs(sf) : mb;
            }
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const double o = __shfl_xor(m, off, 64), ob = __shfl_xor(mb, off, 64);
            m = o > m ? o : m;
            mb = ob > mb ? ob : mb;
        }
        return SplitScale{pow2_scale(m * (double)prm.bmax), pow2_scale(mb)};
    }

    // hi = rn(y), lo = rn(y - hi), two values per conversion instruction.
    // The residual y - hi is exact in FP32; it is taken with one two-term
    // dot product of the packed hi with (-1, -0) or (-0, -1) plus y, which
    // saves converting hi back to FP32.  The zero halves are -0.0 on purpose:
    // (-1, 0) in bf16 is emitted as the inline constant -1.0, which the
    // hardware reads as the FP32 pattern, i.e. the pair (0, -1) (measured on
    // gfx950); with -0.0 the pair can only be encoded as a literal, and
    // adding -0.0 never changes the residual.
    __device__ static void split8(const float *y, HV &hi, HV &lo) {
        typedef float f2 __attribute__((ext_vector_type(2)));
        typedef HS h2 __attribute__((ext_vector_type(2)));
        const h2 m0 = {(HS)-1.0f, (HS)-0.0f}, m1 = {(HS)-0.0f, (HS)-1.0f};
#pragma unroll
        for (int v = 0; v < 8; v += 2) {
            const f2 yy = {y[v], y[v + 1]};
            const h2 h = __builtin_convertvector(yy, h2);
            const f2 r = {dot2(h, m0, yy.x), dot2(h, m1, yy.y)};
            const h2 l = __builtin_convertvector(r, h2);
            hi[v] = h.x; hi[v + 1] = h.y;
            lo[v] = l.x; lo[v + 1] = l.y;
        }
    }
    template <typename H2>
    __device__ static float dot2(H2 a, H2 b, float c) {
        if constexpr (FORM == BF16X3) return __builtin_amdgcn_fdot2_f32_bf16(a, b, c, false);
        else return __builtin_amdgcn_fdot2(a, b, c, false);
    }

    template <int TMV, int TNV>
    __device__ static void body(const FwdParams &prm, int64_t slot, int blk, int bi, int bj, Slice &sl) {
        constexpr int NBRV = c_cdiv(TMV * 16, 64);
        const int lane = threadIdx.x & 63;
        const int i16 = lane & 15, kg = lane >> 4;
        const int a0 = bi * TM * 16, b0 = bj * TN * 16;
        const int64_t e = elem_of(prm, slot);
        typename G::Elem E;
        G::load(prm, e, E);
        const SplitScale sc = FORM == FP16X3 ? elem_scale(prm, E, e) : SplitScale{1.0f, 1.0f};
        const float ys = sc.ys, yb = sc.yb;
        f32x4 acc[TMV][TNV];
#pragma unroll
        for (int ti = 0; ti < TMV; ++ti)
#pragma unroll
            for (int tj = 0; tj < TNV; ++tj) acc[ti][tj] = f32x4{0, 0, 0, 0};
        double bacc[NBRV];
#pragma unroll
        for (int m = 0; m < NBRV; ++m) bacc[m] = 0.0;

        for (int qc = 0; qc < NQP; qc += 64) {
            const int cnt = NQP - qc < 64 ? NQP - qc : 64;   // multiple of 8
            if (lane < cnt) {
                const int q = qc + lane;
                double W[16], sf = 0.0;
                if (q < NQ) {
                    const double *qp = prm.qw + 4 * q;
                    G::coeffs(prm, e, qp, E);
                    const double det = G::block(E, qp, W, sf);
                    if (!(det > 0.0) && prm.status) atomicOr(prm.status, 1u);
                    if (prm.xq && blk == 0) {
                        double x[3];
                        G::map(E, qp, x);
#pragma unroll
                        for (int d = 0; d < 3; ++d) prm.xq[(e * NQ + q) * 3 + d] = x[d];
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < 16; ++k) W[k] = 0.0;
                }
#pragma unroll
                for (int k = 0; k < 16; ++k) sl.W[lane][k] = (float)W[k] * ys;
                sl.sf[lane] = sf;
            }
            wave_sync();
            if (!LC::on && bj == 0) {
#pragma unroll
                for (int m = 0; m < NBRV; ++m) {
                    const int row = a0 + lane + 64 * m;
                    if (lane + 64 * m < TMV * 16 && row < N) {
                        double s = 0.0;
                        for (int qq = 0; qq < cnt && qc + qq < NQ; ++qq)
                            s += sl.sf[qq] * prm.B64[(size_t)(qc + qq) * 4 * NP + row];
                        bacc[m] += s;
                    }
                }
            }
            // The FP32 columns of the next K-block are fetched one iteration
            // ahead (they feed the first work of an iteration); the A
            // fragments of the current block are issued first and consumed
            // only after the fragments Y have been formed.
            const int nkbc = cnt / 8;
            const float *Yc0 = prm.Ycf + (size_t)(qc / 8) * NT * 64 * 8 + ((size_t)(b0 / 16) * 64 + lane) * 8;
            float4 ycn[TNV][2];
#pragma unroll
            for (int tj = 0; tj < TNV; ++tj) {
                ycn[tj][0] = *(const float4 *)(Yc0 + (size_t)tj * 64 * 8);
                ycn[tj][1] = *(const float4 *)(Yc0 + (size_t)tj * 64 * 8 + 4);
            }
            for (int kb = 0; kb < nkbc; ++kb) {
                const size_t kbg = (size_t)(qc / 8 + kb);
                float4 yc[TNV][2];
#pragma unroll
                for (int tj = 0; tj < TNV; ++tj) { yc[tj][0] = ycn[tj][0]; yc[tj][1] = ycn[tj][1]; }
                HV yh[TNV], yl[TNV], ah[TMV], al[TMV];
#pragma unroll
                for (int ti = 0; ti < TMV; ++ti) {
                    const size_t o = ((kbg * NT + a0 / 16 + ti) * 64 + lane) * 8;
                    ah[ti] = *(const HV *)(prm.Bhi + o);
                    al[ti] = *(const HV *)(prm.Blo + o);
                }
                const int kn = kb + 1 < nkbc ? kb + 1 : kb;      // the last block re-reads itself
#pragma unroll
                for (int tj = 0; tj < TNV; ++tj) {
                    const float *yp = Yc0 + (size_t)kn * NT * 64 * 8 + (size_t)tj * 64 * 8;
                    ycn[tj][0] = *(const float4 *)yp;
                    ycn[tj][1] = *(const float4 *)(yp + 4);
                }
                const int qa = kb * 8 + 2 * kg;        // this lane's two points (chunk-local)
                const float *Wa = sl.W[qa];
                const float *Wb = sl.W[qa + 1];
                float wa[16], wb[16];
#pragma unroll
                for (int k = 0; k < 16; ++k) { wa[k] = Wa[k]; wb[k] = Wb[k]; }
#pragma unroll
                for (int tj = 0; tj < TNV; ++tj) {
                    const float s0[4] = {yc[tj][0].x, yc[tj][0].y, yc[tj][0].z, yc[tj][0].w};
                    const float s1[4] = {yc[tj][1].x, yc[tj][1].y, yc[tj][1].z, yc[tj][1].w};
                    float y[8];
                    y[0] = wa[0] * s0[0] + wa[1] * s0[1] + wa[2] * s0[2] + wa[3] * s0[3];
                    y[4] = wb[0] * s1[0] + wb[1] * s1[1] + wb[2] * s1[2] + wb[3] * s1[3];
#pragma unroll
                    for (int r = 1; r < 4; ++r) {
                        y[r] = wa[4 * r + 1] * s0[1] + wa[4 * r + 2] * s0[2] + wa[4 * r + 3] * s0[3];
                        y[4 + r] = wb[4 * r + 1] * s1[1] + wb[4 * r + 2] * s1[2] + wb[4 * r + 3] * s1[3];
                    }
                    if (LC::on && b0 + tj * 16 == LC::tile0 && i16 == LC::lane) {   // load-vector column
#pragma unroll
                        for (int r = 0; r < 8; ++r) y[r] = 0.0f;
                        y[0] = (float)sl.sf[qa] * yb;
                        y[4] = (float)sl.sf[qa + 1] * yb;
                    }
                    split8(y, yh[tj], yl[tj]);
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
            wave_sync();
        }
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

// Work items of a launch over ne element slots (a work item covers EPI slots
// and one of NBLK tile blocks).
template <class KER>
__host__ __device__ inline int64_t items_for(int64_t ne) {
    return (ne + KER::EPI - 1) / KER::EPI * KER::NBLK;
}

// Cooperative launch: workgroup of 4 waves, one work item each, where the
// waves of a workgroup share LDS across a barrier; every wave runs the kernel
// (those past the batch with live = false) so that every wave reaches it.
template <class KER, int MINW>
__global__ __launch_bounds__(256, MINW) void fwd_coop(FwdParams prm) {
    __shared__ typename KER::Smem sm;
    const int wave = wave_uniform(threadIdx.x >> 6);
    const int64_t item = (int64_t)blockIdx.x * 4 + wave;
    const bool live = item < items_for<KER>(prm.ne);
    KER::run_coop(prm, item / KER::NBLK, (int)(item % KER::NBLK), wave, live, sm);
}

// Grid-stride-free direct launch: workgroup of 4 waves, one work item each.
template <class KER, int MINW>
__global__ __launch_bounds__(256, MINW) void fwd_direct(FwdParams prm) {
    __shared__ typename KER::Smem sm;
    const int wave = wave_uniform(threadIdx.x >> 6);
    const int64_t item = (int64_t)blockIdx.x * 4 + wave;
    if (item >= items_for<KER>(prm.ne)) return;
    KER::run(prm, item / KER::NBLK, (int)(item % KER::NBLK), wave, sm);
}

}  // namespace feint
