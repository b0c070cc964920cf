// Forward kernel that contracts per triangle point (FP64, FP32 on 16x16x4
// MFMA).  Both prism rules are products of nij triangle points and p+1 points
// in zeta (q = m nij + ij), and the basis is a product phi_(k,t) =
// T_t(xi1, xi2) L_k(zeta), so B_q[r][(k,t)] = tau_r(t, ij) lam_r(k, m) with
// tau = (T, dT/dxi1, dT/dxi2, T) and lam = (L, L, L, dL/dzeta).  Then
//   A[(k,t)][(k',t')] = sum_ij sum_r tau_r(t, ij) Z_k[(ij, r)][(k',t')],
//   Z_k[(ij, r)][b]   = sum_m lam_r(k, m) Y_(ij,m)[r][b],
//   Y_q[r][b]         = sum_s W_q[r][s] B_q[s][b]          (as in K4),
// i.e. for each row block k the element matrix is a GEMM over K = (ij, r)
// whose left operand is the triangle factor table and whose right operand Z_k
// combines the p+1 zeta points of one triangle point.  Per triangle point and
// column tile this issues (p+1) * ceil(ntri/16) MFMAs where the point-by-point
// kernel issues (p+1)^2 * ceil(ntri/16), for O((p+1)^2) extra FMAs per lane
// (forming Z), which the FP64 and FP32 matrix rates leave room for.
//
// Hexahedra (geometry policy HexGeo) have the same structure: tensor Gauss
// points with q = m (p+1)^2 + ij and the tensor basis phi_(k,t) = T_t L_k with
// the plane factor T_(i',j') = l_i'(xi1) l_j'(xi2), (p+1)^2 of them in place
// of the triangle's.
//
// Rows of A come in blocks (k, t-tile), columns in tiles (k', t'-tile) of 16
// (ntri padded to a multiple of 16, padding multiplied by zero).  A wave owns
// TMK row blocks k (all their t-tiles) and TN column tiles k' of one t'-tile
// of one element.  Since lam_0 = lam_1 = lam_2 = L, the lane's column needs
// only u = sum_{s<3} W[r][s] tau_s(t') and v = W[r][3] tau_3(t') per point,
// shared by its TN column tiles: Y[r][(k',t')] = L_k'(zeta_m) u + L'_k'(zeta_m) v.
// The load vector rides in the spare padded column of the last t'-tile of
// k' = 0: its Z_k carries sum_m lam_0(k,m) w det J f in row r = 0 (where ntri
// is a multiple of 16 it is summed separately in FP64).
#pragma once
#include "fwd_kernels.h"

namespace feint {

template <int P, typename T, int TMK, int TN, int R = 0, class G = PrismGeo>
struct KF {
    static constexpr int N = G::nshp(P), NP = c_pad16(N);
    static constexpr int NK = P + 1, NTRI = N / NK, TT = c_cdiv(NTRI, 16), TP = TT * 16;
    static constexpr int NQ = G::nq(P, R), NIJ = NQ / NK;
    static constexpr int BM = c_cdiv(NK, TMK), BK = c_cdiv(NK, TN), BN = TT * BK, NBLK = BM * BN;
    static constexpr int EPI = 1;
    static constexpr int CIJ = 64 / NK;                       // triangle points per chunk
    // The load vector rides in a spare padded column (tile (0, LCT), lane LCL) when ntri
    // leaves one; otherwise (hexahedra at p = 3 and 7) the blocks of the first column tile
    // accumulate it in FP64 beside the contraction.
    static constexpr bool SPARE = NTRI % 16 != 0;
    static constexpr int LCT = TT - 1, LCL = NTRI - LCT * 16;
    static_assert(NIJ * NK == NQ && NTRI * NK == N, "the rule and the basis must be products in zeta");
    static_assert(TN <= NK && TMK <= NK, "tile counts beyond the zeta factor");
    typedef typename AccT<T>::type V4;

    struct Slice {
        T W[64][WROW<T>::value];      // chunk point (ij - ij0) * NK + m
        double sf[64];
    };
    struct Smem { Slice w[4]; };

    // LB: this block holds the load-vector column (a compile-time flag, so the blocks
    // without it run a loop with no load-vector work at all)
    template <int TMV, int TNV, bool LB>
    __device__ static void body(const FwdParams &prm, int64_t slot, int blk, int bi, int bj, Slice &sl) {
        const int lane = threadIdx.x & 63;
        const int i16 = lane & 15, kg = lane >> 4;
        const int k0 = bi * TMK, tt = bj / BK, kp0 = (bj - tt * BK) * TN;
        const int64_t e = elem_of(prm, slot);
        typename G::Elem E;
        G::load(prm, e, E);
        const T *tau = sizeof(T) == 8 ? (const T *)(const void *)prm.tau64 : (const T *)(const void *)prm.tau32;
        const T *lam = sizeof(T) == 8 ? (const T *)(const void *)prm.lam : (const T *)(const void *)prm.lam32;
        // row factors of the lane (r = kg) for its row blocks, in registers
        T lr[TMV][NK];
#pragma unroll
        for (int k = 0; k < TMV; ++k)
#pragma unroll
            for (int m = 0; m < NK; ++m) lr[k][m] = lam[(kg * NK + k0 + k) * NK + m];
        // the lane's column t' (tau is zero beyond ntri, so padding columns contribute
        // nothing without a mask) and the column factors L_k', L'_k' of its tiles
        const int tcol = tt * 16 + i16;
        // lsel is 1 on the load-vector lane of row r = 0, else 0: that lane's column is
        // padding, where tau is zero and so is its Y, so Y + lsel w det J f places w det J f
        // there exactly and leaves every other lane unchanged, without a lane-dependent
        // branch around the Y arithmetic.
        const bool lcol = LB && i16 == LCL;
        const T lsel = (lcol && kg == 0) ? (T)1 : (T)0;
        // without a spare column: b[(k,t)] = sum_ij tau_0(t, ij) sum_m L_k(zeta_m) (w det J f)_(ij,m),
        // in FP64 from the FP64 tables, by the blocks of the first column tile
        const bool bblk = G::LOAD && !SPARE && kp0 == 0 && tt == 0;
        typedef const __attribute__((address_space(4))) double CD;
        const CD *l64 = (const CD *)prm.lam;
        double bacc[SPARE ? 1 : TMV][TT];
#pragma unroll
        for (int k = 0; k < (SPARE ? 1 : TMV); ++k)
#pragma unroll
            for (int ti = 0; ti < TT; ++ti) bacc[k][ti] = 0.0;
        // The column factors are the same for the whole wave and the table is never written
        // while kernels run: reading them through the constant address space lets them be
        // scalar loads into SGPRs instead of per-lane loads in the inner loop.
        typedef const __attribute__((address_space(4))) T CT;
        const CT *lv = (const CT *)(lam + (size_t)kp0 * NK), *ld = (const CT *)(lam + (size_t)(3 * NK + kp0) * NK);
        V4 acc[TMV][TT][TNV];
#pragma unroll
        for (int k = 0; k < TMV; ++k)
#pragma unroll
            for (int ti = 0; ti < TT; ++ti)
#pragma unroll
                for (int tj = 0; tj < TNV; ++tj) acc[k][ti][tj] = V4{0, 0, 0, 0};
        // triangle factors of point ij: A fragments (rows t) and the column's four factors
        auto fetch = [&](int ij, T (&ta)[TT], T (&tb)[4]) {
#pragma unroll
            for (int ti = 0; ti < TT; ++ti) ta[ti] = tau[((size_t)ij * 4 + kg) * TP + ti * 16 + i16];
#pragma unroll
            for (int s = 0; s < 4; ++s) tb[s] = tau[((size_t)ij * 4 + s) * TP + tcol];
        };

        for (int ij0 = 0; ij0 < NIJ; ij0 += CIJ) {
            const int cij = NIJ - ij0 < CIJ ? NIJ - ij0 : CIJ;
            if (lane < cij * NK) {
                const int il = lane / NK, m = lane - il * NK;
                const int q = m * NIJ + ij0 + il;
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
            T ta[TT], tb[4];
            fetch(ij0, ta, tb);
            for (int il = 0; il < cij; ++il) {
                T tan[TT], tbn[4];
                fetch(ij0 + (il + 1 < cij ? il + 1 : il), tan, tbn);
                // keep the next point's loads at the top of the iteration, in flight under
                // its arithmetic (the scheduler would otherwise sink them to the end)
                __builtin_amdgcn_sched_barrier(0);
                if constexpr (!SPARE) {
                    if (bblk) {
#pragma unroll
                        for (int k = 0; k < TMV; ++k) {
                            double sk = 0.0;
#pragma unroll
                            for (int m = 0; m < NK; ++m) sk += l64[(k0 + k) * NK + m] * sl.sf[il * NK + m];
#pragma unroll
                            for (int ti = 0; ti < TT; ++ti)
                                bacc[k][ti] += prm.tau64[((size_t)(ij0 + il) * 4) * TP + ti * 16 + i16] * sk;
                        }
                    }
                }
                // the lane's row r = kg of W at the p+1 points of this triangle point, folded with
                // the column's factors
                T u[NK], v[NK], sfm[NK];
#pragma unroll
                for (int m = 0; m < NK; ++m) {
                    const T *wr = &sl.W[il * NK + m][4 * kg];
                    u[m] = wr[0] * tb[0] + wr[1] * tb[1] + wr[2] * tb[2];
                    v[m] = wr[3] * tb[3];
                    sfm[m] = LB ? lsel * (T)sl.sf[il * NK + m] : (T)0;
                }
#pragma unroll
                for (int tj = 0; tj < TNV; ++tj) {
                    T y[NK];
#pragma unroll
                    for (int m = 0; m < NK; ++m) {
                        const T yv = lv[tj * NK + m] * u[m] + ld[tj * NK + m] * v[m];
                        y[m] = (LB && tj == 0) ? yv + sfm[m] : yv;     // the load-vector column carries w det J f
                    }
#pragma unroll
                    for (int k = 0; k < TMV; ++k) {
                        T z = (T)0;
#pragma unroll
                        for (int m = 0; m < NK; ++m) z += lr[k][m] * y[m];
#pragma unroll
                        for (int ti = 0; ti < TT; ++ti) acc[k][ti][tj] = mfma4(ta[ti], z, acc[k][ti][tj]);
                    }
                }
#pragma unroll
                for (int ti = 0; ti < TT; ++ti) ta[ti] = tan[ti];
#pragma unroll
                for (int s = 0; s < 4; ++s) tb[s] = tbn[s];
            }
            wave_sync();
        }
        T *Aout = (T *)prm.A + offA_of(prm, e, N);
        T *bout = (T *)prm.b + offb_of(prm, e, N);
#pragma unroll
        for (int k = 0; k < TMV; ++k)
#pragma unroll
            for (int ti = 0; ti < TT; ++ti)
#pragma unroll
                for (int tj = 0; tj < TNV; ++tj)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int tr = ti * 16 + acc_row<T>(lane, r);
                        if (tr >= NTRI) continue;
                        const int row = (k0 + k) * NTRI + tr;
                        if (tj == 0 && lcol)
                            bout[row] = acc[k][ti][tj][r];
                        else if (tcol < NTRI)
                            Aout[(size_t)row * N + (kp0 + tj) * NTRI + tcol] = acc[k][ti][tj][r];
                    }
        if constexpr (!SPARE) {
            if (bblk && kg == 0) {
#pragma unroll
                for (int k = 0; k < TMV; ++k)
#pragma unroll
                    for (int ti = 0; ti < TT; ++ti)
                        if (ti * 16 + i16 < NTRI) bout[(k0 + k) * NTRI + ti * 16 + i16] = (T)bacc[k][ti];
            }
        }
    }

    template <int TMV, int TNV>
    __device__ static void with_lb(bool lb, const FwdParams &prm, int64_t slot, int blk, int bi, int bj, Slice &sl) {
        if (lb) body<TMV, TNV, true>(prm, slot, blk, bi, bj, sl);
        else body<TMV, TNV, false>(prm, slot, blk, bi, bj, sl);
    }

    // Row blocks (TMK values of k) and column tiles (TN values of k') of the
    // last blocks are compile-time counts, so the loops carry no bounds tests.
    __device__ static void run_slice(const FwdParams &prm, int64_t slot, int blk, Slice &sl) {
        const int bi = blk / BN, bj = blk % BN;
        constexpr int TML = NK - (BM - 1) * TMK, TNL = NK - (BK - 1) * TN;
        // one call site per distinct (row count, column count): where the last blocks have
        // the regular counts the body is inlined once, not twice
        const bool lastm = TML != TMK && bi == BM - 1, lastn = TNL != TN && bj % BK == BK - 1;
        // the load-vector column: first column tile (k' = 0) of the last triangle tile
        const bool lb = G::LOAD && SPARE && bj % BK == 0 && bj / BK == LCT;
        if (lastm) {
            if (lastn) with_lb<TML, TNL>(lb, prm, slot, blk, bi, bj, sl);
            else with_lb<TML, TN>(lb, prm, slot, blk, bi, bj, sl);
        } else {
            if (lastn) with_lb<TMK, TNL>(lb, prm, slot, blk, bi, bj, sl);
            else with_lb<TMK, TN>(lb, prm, slot, blk, bi, bj, sl);
        }
    }
    __device__ static void run(const FwdParams &prm, int64_t slot, int blk, int wave, Smem &sm) {
        run_slice(prm, slot, blk, sm.w[wave]);
    }
};

// The same contraction with the element's point blocks shared by the waves
// that work on it (FP64, FP32).  Where the element has two blocks, a
// workgroup of four waves takes two elements, two waves each; otherwise it
// takes one element and its four waves take the blocks in turn.  The waves of
// an element form W_q and w det J f of its points (one point per lane, the
// points split between them) into the element's LDS area, the workgroup
// synchronises once, and each wave then contracts its blocks over all
// triangle points, reading W from that area.  The point blocks are formed
// once per element, however many blocks it has, and before any accumulator
// is live, so a block shape can be chosen for two waves per SIMD without
// repeating the FP64 geometry.
template <int P, typename T, int TMK, int TN, int R = 0, class G = PrismGeo>
struct KF2 {
    typedef KF<P, T, TMK, TN, R, G> F;
    static constexpr int N = F::N, NK = F::NK, NTRI = F::NTRI, TT = F::TT, TP = F::TP, NQ = F::NQ, NIJ = F::NIJ;
    static constexpr int BM = F::BM, BK = F::BK, BN = F::BN, NB = F::NBLK;   // blocks of an element
    static constexpr int WPE = NB == 2 ? 2 : 4;        // waves per element
    static constexpr int EPW = 4 / WPE;                // elements per workgroup
    static constexpr int EPI = 1, NBLK = WPE;          // work items: one per wave
    static constexpr bool SPARE = F::SPARE;
    static constexpr int LCT = F::LCT, LCL = F::LCL;
    typedef typename AccT<T>::type V4;

    struct ElemArea {
        T W[NQ][WROW<T>::value];      // point q in the rule's order (q = m nij + ij)
        double sf[NQ];
    };
    struct Smem { ElemArea el[EPW]; };

    template <int TMV, int TNV, bool LB>
    __device__ static void body(const FwdParams &prm, int64_t slot, int bi, int bj, const ElemArea &ea) {
        const int lane = threadIdx.x & 63;
        const int i16 = lane & 15, kg = lane >> 4;
        const int k0 = bi * TMK, tt = bj / BK, kp0 = (bj - tt * BK) * TN;
        const int64_t e = elem_of(prm, slot);
        const T *tau = sizeof(T) == 8 ? (const T *)(const void *)prm.tau64 : (const T *)(const void *)prm.tau32;
        const T *lam = sizeof(T) == 8 ? (const T *)(const void *)prm.lam : (const T *)(const void *)prm.lam32;
        T lr[TMV][NK];
#pragma unroll
        for (int k = 0; k < TMV; ++k)
#pragma unroll
            for (int m = 0; m < NK; ++m) lr[k][m] = lam[(kg * NK + k0 + k) * NK + m];
        const int tcol = tt * 16 + i16;
        const bool lcol = LB && i16 == LCL;
        const T lsel = (lcol && kg == 0) ? (T)1 : (T)0;
        const bool bblk = G::LOAD && !SPARE && kp0 == 0 && tt == 0;
        const double *l64 = prm.lam;
        double bacc[SPARE ? 1 : TMV][TT];
#pragma unroll
        for (int k = 0; k < (SPARE ? 1 : TMV); ++k)
#pragma unroll
            for (int ti = 0; ti < TT; ++ti) bacc[k][ti] = 0.0;
        typedef const __attribute__((address_space(4))) T CT;
        const CT *lv = (const CT *)(lam + (size_t)kp0 * NK), *ld = (const CT *)(lam + (size_t)(3 * NK + kp0) * NK);
        V4 acc[TMV][TT][TNV];
#pragma unroll
        for (int k = 0; k < TMV; ++k)
#pragma unroll
            for (int ti = 0; ti < TT; ++ti)
#pragma unroll
                for (int tj = 0; tj < TNV; ++tj) acc[k][ti][tj] = V4{0, 0, 0, 0};
        auto fetch = [&](int ij, T (&ta)[TT], T (&tb)[4]) {
#pragma unroll
            for (int ti = 0; ti < TT; ++ti) ta[ti] = tau[((size_t)ij * 4 + kg) * TP + ti * 16 + i16];
#pragma unroll
            for (int s = 0; s < 4; ++s) tb[s] = tau[((size_t)ij * 4 + s) * TP + tcol];
        };
        T ta[TT], tb[4];
        fetch(0, ta, tb);
        for (int ij = 0; ij < NIJ; ++ij) {
            T tan[TT], tbn[4];
            fetch(ij + 1 < NIJ ? ij + 1 : ij, tan, tbn);
            __builtin_amdgcn_sched_barrier(0);
            if constexpr (!SPARE) {
                if (bblk) {
#pragma unroll
                    for (int k = 0; k < TMV; ++k) {
                        double sk = 0.0;
#pragma unroll
                        for (int m = 0; m < NK; ++m) sk += l64[(k0 + k) * NK + m] * ea.sf[m * NIJ + ij];
#pragma unroll
                        for (int ti = 0; ti < TT; ++ti)
                            bacc[k][ti] += prm.tau64[((size_t)ij * 4) * TP + ti * 16 + i16] * sk;
                    }
                }
            }
            T u[NK], v[NK], sfm[NK];
#pragma unroll
            for (int m = 0; m < NK; ++m) {
                const T *wr = &ea.W[m * NIJ + ij][4 * kg];
                u[m] = wr[0] * tb[0] + wr[1] * tb[1] + wr[2] * tb[2];
                v[m] = wr[3] * tb[3];
                sfm[m] = LB ? lsel * (T)ea.sf[m * NIJ + ij] : (T)0;
            }
#pragma unroll
            for (int tj = 0; tj < TNV; ++tj) {
                T y[NK];
#pragma unroll
                for (int m = 0; m < NK; ++m) {
                    const T yv = lv[tj * NK + m] * u[m] + ld[tj * NK + m] * v[m];
                    y[m] = (LB && tj == 0) ? yv + sfm[m] : yv;
                }
#pragma unroll
                for (int k = 0; k < TMV; ++k) {
                    T z = (T)0;
#pragma unroll
                    for (int m = 0; m < NK; ++m) z += lr[k][m] * y[m];
#pragma unroll
                    for (int ti = 0; ti < TT; ++ti) acc[k][ti][tj] = mfma4(ta[ti], z, acc[k][ti][tj]);
                }
            }
#pragma unroll
            for (int ti = 0; ti < TT; ++ti) ta[ti] = tan[ti];
#pragma unroll
            for (int s = 0; s < 4; ++s) tb[s] = tbn[s];
        }
        T *Aout = (T *)prm.A + offA_of(prm, e, N);
        T *bout = (T *)prm.b + offb_of(prm, e, N);
#pragma unroll
        for (int k = 0; k < TMV; ++k)
#pragma unroll
            for (int ti = 0; ti < TT; ++ti)
#pragma unroll
                for (int tj = 0; tj < TNV; ++tj)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int tr = ti * 16 + acc_row<T>(lane, r);
                        if (tr >= NTRI) continue;
                        const int row = (k0 + k) * NTRI + tr;
                        if (tj == 0 && lcol)
                            bout[row] = acc[k][ti][tj][r];
                        else if (tcol < NTRI)
                            Aout[(size_t)row * N + (kp0 + tj) * NTRI + tcol] = acc[k][ti][tj][r];
                    }
        if constexpr (!SPARE) {
            if (bblk && kg == 0) {
#pragma unroll
                for (int k = 0; k < TMV; ++k)
#pragma unroll
                    for (int ti = 0; ti < TT; ++ti)
                        if (ti * 16 + i16 < NTRI) bout[(k0 + k) * NTRI + ti * 16 + i16] = (T)bacc[k][ti];
            }
        }
    }

    template <int TMV, int TNV>
    __device__ static void with_lb(bool lb, const FwdParams &prm, int64_t slot, int bi, int bj, const ElemArea &ea) {
        if (lb) body<TMV, TNV, true>(prm, slot, bi, bj, ea);
        else body<TMV, TNV, false>(prm, slot, bi, bj, ea);
    }

    // W_q and w det J f of the element's points into its LDS area, one point
    // per lane, the points split between the element's waves (WV: the wave's
    // index among them); the caller synchronises the workgroup afterwards.
    __device__ static void geometry(const FwdParams &prm, int64_t slot, int wv, bool live, ElemArea &ea) {
        const int lane = threadIdx.x & 63;
        if (!live) return;
        const int64_t e = elem_of(prm, slot);
        typename G::Elem E;
        G::load(prm, e, E);
        for (int qc = wv * 64; qc < NQ; qc += WPE * 64) {
            const int q = qc + lane;
            if (q < NQ) {
                const double *qp = prm.qw + 4 * q;
                double W[16], sf;
                G::coeffs(prm, e, qp, E);
                const double det = G::block(E, qp, W, sf);
                if (!(det > 0.0) && prm.status) atomicOr(prm.status, 1u);
#pragma unroll
                for (int k = 0; k < 16; ++k) ea.W[q][k] = (T)W[k];
                ea.sf[q] = sf;
                if (prm.xq) {
                    double x[3];
                    G::map(E, qp, x);
#pragma unroll
                    for (int d = 0; d < 3; ++d) prm.xq[(e * NQ + q) * 3 + d] = x[d];
                }
            }
        }
    }

    // Every wave of the workgroup reaches the barrier; LIVE is false for the
    // waves past the batch (the second element of the last workgroup).  WV is
    // the wave's index among its element's waves.
    __device__ static void run_coop(const FwdParams &prm, int64_t slot, int wv, int wave, bool live, Smem &sm) {
        ElemArea &ea = sm.el[wave / WPE];
        geometry(prm, slot, wv, live, ea);
        __syncthreads();
        if (!live) return;
        if constexpr (NB == WPE) {
            one_block(prm, slot, wv, ea);              // one block per wave: no loop
        } else {
            for (int blk = wv; blk < NB; blk += WPE) one_block(prm, slot, blk, ea);
        }
    }
    __device__ static void one_block(const FwdParams &prm, int64_t slot, int blk, const ElemArea &ea) {
        constexpr int TML = NK - (BM - 1) * TMK, TNL = NK - (BK - 1) * TN;
        const int bi = blk / BN, bj = blk % BN;
        const bool lastm = TML != TMK && bi == BM - 1, lastn = TNL != TN && bj % BK == BK - 1;
        const bool lb = G::LOAD && SPARE && bj % BK == 0 && bj / BK == LCT;
        if (lastm) {
            if (lastn) with_lb<TML, TNL>(lb, prm, slot, bi, bj, ea);
            else with_lb<TML, TN>(lb, prm, slot, bi, bj, ea);
        } else {
            if (lastn) with_lb<TMK, TNL>(lb, prm, slot, bi, bj, ea);
            else with_lb<TMK, TN>(lb, prm, slot, bi, bj, ea);
        }
    }
};

// The split forms (bf16x3, fp16x3) of the shared-point-block contraction,
// with the zeta sum taken first.  The main product takes eight triangle
// points per 16x16x32 MFMA: K = (triangle point 2 g + v/4 of the chunk, row
// r = v%4) for lane group g and value v, so the A operand is the
// triangle-factor table split on the host (hi + lo, in fragment order) and
// each lane forms Z_k[(ij, r)][col] for its eight K slots, splits it and
// issues hi*hi + hi*lo + lo*hi per tile.  Z_k[(ij, r)][(k', t')] =
// sum_s tau_s(t', ij) G[r][s] with G[r][s] = sum_m lam_r(k, m) lam_s(k', m)
// W_m(ij)[r][s]: G does not depend on the output column t', so each
// (triangle point, k, k') combination of a lane group's pair of triangle
// points is summed once, by one lane of the group, into the wave's LDS, and
// every lane then forms its eight Z values from the 13 nonzero G entries
// (W_m[r][0] = 0 for r >= 1) and its four tau values: 13 FMAs per eight Z
// values in place of about 70.  The load vector's zeta sum
// sum_m lam_0(k, m) w det J f rides in the G block of column k' = 0 and is
// added on the spare column, whose tau values are zero.  The point blocks
// are formed once per element into LDS as in KF2.
template <int P, int TMK, int TN, int R = 0, class G = PrismGeo, int FORM = BF16X3>
struct KF2G {
    typedef KF<P, float, TMK, TN, R, G> F;
    typedef KF2<P, float, TMK, TN, R, G> K2;
    static constexpr int N = F::N, NK = F::NK, NTRI = F::NTRI, TT = F::TT, TP = F::TP, NQ = F::NQ, NIJ = F::NIJ;
    static constexpr int BM = F::BM, BK = F::BK, BN = F::BN, NB = F::NBLK;
    static constexpr int NCH = (NIJ + 7) / 8;          // chunks of eight triangle points
    static constexpr int WPE = K2::WPE, EPW = K2::EPW;
    static constexpr int EPI = 1, NBLK = WPE;
    static constexpr int LCT = F::LCT, LCL = F::LCL;
    static constexpr int NCB = 2 * TMK * TN;            // combinations of a full block
    static constexpr int GST = NCB * 16 + 4;            // one lane group's G blocks (padded: the groups start on different banks)
    static_assert(F::SPARE, "the load vector rides in a spare padded column");
    static_assert(NCB <= 32, "at most two combinations per lane of a group");
    typedef typename K2::ElemArea ElemArea;
    struct alignas(16) Area { ElemArea a; };           // 16-byte reads of every element's point blocks
    struct Smem {
        Area el[EPW];
        float gs[4][4 * GST];                          // per wave, per lane group
    };
    typedef typename SplitT<FORM>::vec HV;
    typedef K32<P, FORM, 1, 1, R, G> Split;            // split8: hi = rn(y), lo = rn(y - hi)
    // fp16 form: the triangle table holds tau * 2^tau_f16_shift, and a block's
    // Z values are scaled by powers of two that place bounds on them in
    // [2^13, 2^14): ys from the element's largest |W| entry, yb (the
    // load-vector column) from its largest |w det J f|; undone at the store
    struct Scales { float ys, yb; };
    __device__ static Scales scales(const FwdParams &prm, const ElemArea &ea) {
        if constexpr (FORM != FP16X3) {
            return Scales{1.0f, 1.0f};
        } else {
            const int lane = threadIdx.x & 63;
            float wm = 0.0f;
            double sm = 0.0;
            for (int q = lane; q < NQ; q += 64) {
#pragma unroll
                for (int x = 0; x < 16; ++x) wm = fmaxf(wm, fabsf(ea.W[q][x]));
                sm = fmax(sm, fabs(ea.sf[q]));
            }
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                wm = fmaxf(wm, __shfl_xor(wm, off, 64));
                sm = fmax(sm, __shfl_xor(sm, off, 64));
            }
            return Scales{pow2_scale((double)wm * prm.f16_zc), pow2_scale(sm * prm.f16_zb)};
        }
    }

    template <int TMV, int TNV, bool LB>
    __device__ static void body(const FwdParams &prm, int64_t slot, int bi, int bj, const ElemArea &ea, float *gs,
                                Scales sc) {
        constexpr int NC = 2 * TMV * TNV, NCL = (NC + 15) / 16;
        const int lane = threadIdx.x & 63;
        const int i16 = lane & 15, g = lane >> 4;
        const int k0 = bi * TMK, tt = bj / BK, kp0 = (bj - tt * BK) * TN;
        const int64_t e = elem_of(prm, slot);
        const float *tau = prm.tau32;
        const float *lam = prm.lam32;                  // [r][k][m]; rows 0..2 hold L, row 3 dL
        const int tcol = tt * 16 + i16;
        const bool lcol = LB && i16 == LCL;
        const float zs = (LB && lcol) ? sc.yb : sc.ys;    // this lane's column: the load vector or A
        // this lane's combinations for the zeta sums, c = i16 + 16 cl: triangle
        // point ch of its group's pair, row k0 + ck, column kp0 + cj (lanes
        // past NC repeat combination 0 and store nothing)
        int cc[NCL], chh[NCL];
        float vv[NCL][NK], vd[NCL][NK], dv[NCL][NK], dd[NCL][NK], lk[NCL][NK];
#pragma unroll
        for (int cl = 0; cl < NCL; ++cl) {
            const int c = i16 + 16 * cl < NC ? i16 + 16 * cl : 0;
            const int ck = (c / TNV) % TMV, cj = c % TNV;
            cc[cl] = i16 + 16 * cl;
            chh[cl] = c / (TMV * TNV);
#pragma unroll
            for (int m = 0; m < NK; ++m) {
                const float a = lam[(size_t)(k0 + ck) * NK + m], da = lam[(size_t)(3 * NK + k0 + ck) * NK + m];
                const float b = lam[(size_t)(kp0 + cj) * NK + m], db = lam[(size_t)(3 * NK + kp0 + cj) * NK + m];
                vv[cl][m] = a * b; vd[cl][m] = a * db; dv[cl][m] = da * b; dd[cl][m] = da * db;
                lk[cl][m] = a;
            }
        }
        float *gw = gs + g * GST;                      // this lane group's blocks
        f32x4 acc[TMV][TT][TNV];
#pragma unroll
        for (int k = 0; k < TMV; ++k)
#pragma unroll
            for (int ti = 0; ti < TT; ++ti)
#pragma unroll
                for (int tj = 0; tj < TNV; ++tj) acc[k][ti][tj] = f32x4{0, 0, 0, 0};
        for (int c8 = 0; c8 < NCH; ++c8) {
            HV ah[TT], al[TT];
#pragma unroll
            for (int ti = 0; ti < TT; ++ti) {
                const size_t o = (((size_t)c8 * TT + ti) * 64 + lane) * 8;
                ah[ti] = *(const HV *)(prm.taubh + o);
                al[ti] = *(const HV *)(prm.taubl + o);
            }
            float tb[2][4];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int ij = c8 * 8 + 2 * g + h;
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4) tb[h][s4] = ij < NIJ ? tau[((size_t)ij * 4 + s4) * TP + tcol] * zs : 0.0f;
            }
            // G of this lane's combinations; the previous chunk's reads come
            // first.  A wave's LDS operations execute in order, so the fences only
            // keep the compiler from moving LDS accesses across them (wavefront
            // scope: no wait for the table loads in flight)
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
            for (int cl = 0; cl < NCL; ++cl) {
                const int ij = c8 * 8 + 2 * g + chh[cl];
                f32x4 g0 = {0, 0, 0, 0}, g1 = {0, 0, 0, 0}, g2 = {0, 0, 0, 0}, g3 = {0, 0, 0, 0};
                if (ij < NIJ) {
#pragma unroll
                    for (int m = 0; m < NK; ++m) {
                        const f32x4 *wr = (const f32x4 *)&ea.W[m * NIJ + ij][0];
                        const f32x4 w0 = wr[0], w1 = wr[1], w2 = wr[2], w3 = wr[3];
                        const float xvv = vv[cl][m], xvd = vd[cl][m], xdv = dv[cl][m], xdd = dd[cl][m];
                        g0[0] += xvv * w0[0]; g0[1] += xvv * w0[1]; g0[2] += xvv * w0[2]; g0[3] += xvd * w0[3];
                        g1[0] += xvv * w1[1]; g1[1] += xvv * w1[2]; g1[2] += xvd * w1[3];
                        if (LB) g1[3] += lk[cl][m] * (float)ea.sf[m * NIJ + ij];
                        g2[0] += xvv * w2[1]; g2[1] += xvv * w2[2]; g2[2] += xvd * w2[3];
                        g2[3] += xdv * w3[1]; g3[0] += xdv * w3[2]; g3[1] += xdd * w3[3];
                    }
                }
                if (cc[cl] < NC) {
                    f32x4 *gp = (f32x4 *)(gw + cc[cl] * 16);
                    gp[0] = g0; gp[1] = g1; gp[2] = g2; gp[3] = g3;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
            for (int k = 0; k < TMV; ++k)
#pragma unroll
                for (int tj = 0; tj < TNV; ++tj) {
                    float z[8];
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const f32x4 *gp = (const f32x4 *)(gw + ((h * TMV + k) * TNV + tj) * 16);
                        const f32x4 a = gp[0], b = gp[1], cc = gp[2], d = gp[3];
                        const float *t = tb[h];
                        float z0 = a[0] * t[0] + a[1] * t[1] + a[2] * t[2] + a[3] * t[3];
                        if (LB && tj == 0) z0 += lcol ? b[3] * zs : 0.0f;   // the load-vector column
                        z[4 * h + 0] = z0;
                        z[4 * h + 1] = b[0] * t[1] + b[1] * t[2] + b[2] * t[3];
                        z[4 * h + 2] = cc[0] * t[1] + cc[1] * t[2] + cc[2] * t[3];
                        z[4 * h + 3] = cc[3] * t[1] + d[0] * t[2] + d[1] * t[3];
                    }
                    HV zh, zl;
                    Split::split8(z, zh, zl);
#pragma unroll
                    for (int ti = 0; ti < TT; ++ti) {
                        acc[k][ti][tj] = mfma32(ah[ti], zl, acc[k][ti][tj]);
                        acc[k][ti][tj] = mfma32(al[ti], zh, acc[k][ti][tj]);
                        acc[k][ti][tj] = mfma32(ah[ti], zh, acc[k][ti][tj]);
                    }
                }
        }
        float *Aout = (float *)prm.A + offA_of(prm, e, N);
        float *bout = (float *)prm.b + offb_of(prm, e, N);
        const float tu = FORM == FP16X3 ? ldexpf(1.0f, -prm.tau_f16_shift) : 1.0f;
        const float ua = tu / sc.ys, ub = tu / sc.yb;
#pragma unroll
        for (int k = 0; k < TMV; ++k)
#pragma unroll
            for (int ti = 0; ti < TT; ++ti)
#pragma unroll
                for (int tj = 0; tj < TNV; ++tj)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int tr = ti * 16 + acc_row<float>(lane, r);
                        if (tr >= NTRI) continue;
                        const int row = (k0 + k) * NTRI + tr;
                        if (tj == 0 && lcol)
                            bout[row] = acc[k][ti][tj][r] * ub;
                        else if (tcol < NTRI)
                            Aout[(size_t)row * N + (kp0 + tj) * NTRI + tcol] = acc[k][ti][tj][r] * ua;
                    }
    }

    template <int TMV, int TNV>
    __device__ static void with_lb(bool lb, const FwdParams &prm, int64_t slot, int bi, int bj, const ElemArea &ea, float *gs,
                                   Scales sc) {
        if (lb) body<TMV, TNV, true>(prm, slot, bi, bj, ea, gs, sc);
        else body<TMV, TNV, false>(prm, slot, bi, bj, ea, gs, sc);
    }
    __device__ static void one_block(const FwdParams &prm, int64_t slot, int blk, const ElemArea &ea, float *gs, Scales sc) {
        constexpr int TML = NK - (BM - 1) * TMK, TNL = NK - (BK - 1) * TN;
        const int bi = blk / BN, bj = blk % BN;
        const bool lastm = TML != TMK && bi == BM - 1, lastn = TNL != TN && bj % BK == BK - 1;
        const bool lb = G::LOAD && bj % BK == 0 && bj / BK == LCT;
        if (lastm) {
            if (lastn) with_lb<TML, TNL>(lb, prm, slot, bi, bj, ea, gs, sc);
            else with_lb<TML, TN>(lb, prm, slot, bi, bj, ea, gs, sc);
        } else {
            if (lastn) with_lb<TMK, TNL>(lb, prm, slot, bi, bj, ea, gs, sc);
            else with_lb<TMK, TN>(lb, prm, slot, bi, bj, ea, gs, sc);
        }
    }
    __device__ static void run_coop(const FwdParams &prm, int64_t slot, int wv, int wave, bool live, Smem &sm) {
        ElemArea &ea = sm.el[wave / WPE].a;
        K2::geometry(prm, slot, wv, live, ea);
        __syncthreads();
        if (!live) return;
        const Scales sc = scales(prm, ea);
        for (int blk = wv; blk < NB; blk += WPE) one_block(prm, slot, blk, ea, sm.gs[wave], sc);
    }
};

// The FP64 / FP32 contraction with the zeta sums taken first, as KF2G does
// for the split form: Z_k[(ij, r)][(k', t')] = sum_s tau_s(t', ij) G[r][s]
// with G[r][s] = sum_m lam_r(k, m) lam_s(k', m) W_m(ij)[r][s].  Per batch of
// IJB triangle points, the wave's lanes form the 16 entries G[r][s] of every
// (k, k') block of the wave's tile block, one or more entries per lane, into
// the wave's LDS.  G[r][0] = 0 for r >= 1 (W_m[r][0] = 0); the slot of r = 1
// carries the load vector's zeta sum sum_m lam_0(k, m) w det J f in the block
// of column k' = 0, read from the same slot of the point blocks, where w det J
// f is stored.  Lane (r, t') then reads row r of each block and forms its Z
// value with four FMAs, against about nine vector instructions per Z value
// in KF2.  On gfx950 FP64 vector work and FP64 MFMAs never overlap, so what
// this removes comes off the FP64 time directly.
template <int P, typename T, int TMK, int TN, int IJB = 4, int R = 0, class G = PrismGeo>
struct KF2Z {
    typedef KF<P, T, TMK, TN, R, G> F;
    typedef KF2<P, T, TMK, TN, R, G> K2;
    static constexpr int N = F::N, NK = F::NK, NTRI = F::NTRI, TT = F::TT, TP = F::TP, NQ = F::NQ, NIJ = F::NIJ;
    static constexpr int BM = F::BM, BK = F::BK, BN = F::BN, NB = F::NBLK;
    static constexpr int WPE = K2::WPE, EPW = K2::EPW;
    static constexpr int EPI = 1, NBLK = WPE;
    static constexpr int LCT = F::LCT, LCL = F::LCL;
    static constexpr int NVB = 16 * TMK * TN;          // G entries of a full block per triangle point
    static constexpr int NJ = (NVB + 63) / 64;         // entries per lane
    static_assert(F::SPARE, "the load vector rides in a spare padded column");
    typedef typename K2::ElemArea ElemArea;
    typedef typename AccT<T>::type V4;
    struct alignas(16) Area { ElemArea a; };
    struct Smem {
        Area el[EPW];
        T gs[4][IJB][NJ * 64];                         // per wave
    };

    template <int TMV, int TNV, bool LB>
    __device__ static void body(const FwdParams &prm, int64_t slot, int bi, int bj, const ElemArea &ea, T (*gs)[NJ * 64]) {
        constexpr int NV = 16 * TMV * TNV;
        const int lane = threadIdx.x & 63;
        const int i16 = lane & 15, kg = lane >> 4;
        const int k0 = bi * TMK, tt = bj / BK, kp0 = (bj - tt * BK) * TN;
        const int64_t e = elem_of(prm, slot);
        const T *tau = sizeof(T) == 8 ? (const T *)(const void *)prm.tau64 : (const T *)(const void *)prm.tau32;
        const T *lam = sizeof(T) == 8 ? (const T *)(const void *)prm.lam : (const T *)(const void *)prm.lam32;
        const int tcol = tt * 16 + i16;
        const bool lcol = LB && i16 == LCL;
        const T lsel = (lcol && kg == 0) ? (T)1 : (T)0;
        // this lane's G entries v = lane + 64 j: block (k, tj) = v / 16, entry (r, s)
        int col[NJ];
        T pf[NJ][NK];
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const int v = lane + 64 * j;
            const int vv = v < NV ? v : 0;
            const int cb = vv / 16, rs = vv % 16, r = rs / 4, s = rs % 4;
            const int k = k0 + cb / TNV, kp = kp0 + cb % TNV;
            const bool ls = LB && r == 1 && s == 0 && cb % TNV == 0;   // the load-vector slot
            const bool zero = v >= NV || (r >= 1 && s == 0 && !ls);
            col[j] = rs;
#pragma unroll
            for (int m = 0; m < NK; ++m) {
                const T a = lam[(size_t)(r * NK + k) * NK + m];
                const T b = ls ? (T)1 : lam[(size_t)(s * NK + kp) * NK + m];
                pf[j][m] = zero ? (T)0 : (ls ? lam[(size_t)k * NK + m] : a * b);
            }
        }
        V4 acc[TMV][TT][TNV];
#pragma unroll
        for (int k = 0; k < TMV; ++k)
#pragma unroll
            for (int ti = 0; ti < TT; ++ti)
#pragma unroll
                for (int tj = 0; tj < TNV; ++tj) acc[k][ti][tj] = V4{0, 0, 0, 0};
        for (int ij0 = 0; ij0 < NIJ; ij0 += IJB) {
            T ta[IJB][TT], tb[IJB][4];
#pragma unroll
            for (int b = 0; b < IJB; ++b) {
                const int ij = ij0 + b < NIJ ? ij0 + b : NIJ - 1;
#pragma unroll
                for (int ti = 0; ti < TT; ++ti) ta[b][ti] = tau[((size_t)ij * 4 + kg) * TP + ti * 16 + i16];
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4) tb[b][s4] = tau[((size_t)ij * 4 + s4) * TP + tcol];
                if (kg != 0) tb[b][0] = (T)0;                 // G[r][0] of r >= 1 is not a Z term
            }
            // the batch's G entries; the previous batch's reads come first.  A
            // wave's LDS operations execute in order: the fences only keep the
            // compiler from moving LDS accesses across them
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
            for (int b = 0; b < IJB; ++b) {
                const int ij = ij0 + b;
                if (ij < NIJ) {
#pragma unroll
                    for (int j = 0; j < NJ; ++j) {
                        T gv = (T)0;
#pragma unroll
                        for (int m = 0; m < NK; ++m) gv += pf[j][m] * ea.W[m * NIJ + ij][col[j]];
                        if (lane + 64 * j < NV) gs[b][lane + 64 * j] = gv;
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
            for (int b = 0; b < IJB; ++b) {
                if (ij0 + b < NIJ) {
#pragma unroll
                    for (int tj = 0; tj < TNV; ++tj)
#pragma unroll
                        for (int k = 0; k < TMV; ++k) {
                            const T *gp = &gs[b][(k * TNV + tj) * 16];
                            T z = gp[4 * kg] * tb[b][0] + gp[4 * kg + 1] * tb[b][1] + gp[4 * kg + 2] * tb[b][2] +
                                  gp[4 * kg + 3] * tb[b][3];
                            if (LB && tj == 0) z += lsel * gp[4];   // the load-vector column
#pragma unroll
                            for (int ti = 0; ti < TT; ++ti) acc[k][ti][tj] = mfma4(ta[b][ti], z, acc[k][ti][tj]);
                        }
                }
            }
        }
        T *Aout = (T *)prm.A + offA_of(prm, e, N);
        T *bout = (T *)prm.b + offb_of(prm, e, N);
#pragma unroll
        for (int k = 0; k < TMV; ++k)
#pragma unroll
            for (int ti = 0; ti < TT; ++ti)
#pragma unroll
                for (int tj = 0; tj < TNV; ++tj)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int tr = ti * 16 + acc_row<T>(lane, r);
                        if (tr >= NTRI) continue;
                        const int row = (k0 + k) * NTRI + tr;
                        if (tj == 0 && lcol)
                            bout[row] = acc[k][ti][tj][r];
                        else if (tcol < NTRI)
                            Aout[(size_t)row * N + (kp0 + tj) * NTRI + tcol] = acc[k][ti][tj][r];
                    }
    }

    template <int TMV, int TNV>
    __device__ static void with_lb(bool lb, const FwdParams &prm, int64_t slot, int bi, int bj, const ElemArea &ea,
                                   T (*gs)[NJ * 64]) {
        if (lb) body<TMV, TNV, true>(prm, slot, bi, bj, ea, gs);
        else body<TMV, TNV, false>(prm, slot, bi, bj, ea, gs);
    }
    __device__ static void one_block(const FwdParams &prm, int64_t slot, int blk, const ElemArea &ea, T (*gs)[NJ * 64]) {
        constexpr int TML = NK - (BM - 1) * TMK, TNL = NK - (BK - 1) * TN;
        const int bi = blk / BN, bj = blk % BN;
        const bool lastm = TML != TMK && bi == BM - 1, lastn = TNL != TN && bj % BK == BK - 1;
        const bool lb = G::LOAD && bj % BK == 0 && bj / BK == LCT;
        if (lastm) {
            if (lastn) with_lb<TML, TNL>(lb, prm, slot, bi, bj, ea, gs);
            else with_lb<TML, TN>(lb, prm, slot, bi, bj, ea, gs);
        } else {
            if (lastn) with_lb<TMK, TNL>(lb, prm, slot, bi, bj, ea, gs);
            else with_lb<TMK, TN>(lb, prm, slot, bi, bj, ea, gs);
        }
    }
    __device__ static void run_coop(const FwdParams &prm, int64_t slot, int wv, int wave, bool live, Smem &sm) {
        ElemArea &ea = sm.el[wave / WPE].a;
        K2::geometry(prm, slot, wv, live, ea);
        if (live) {
            // w det J f into the W[1][0] slot (zero in every point block), by the
            // lane that formed the point
            const int lane = threadIdx.x & 63;
            for (int qc = wv * 64; qc < NQ; qc += WPE * 64)
                if (qc + lane < NQ) ea.W[qc + lane][4] = (T)ea.sf[qc + lane];
        }
        __syncthreads();
        if (!live) return;
        for (int blk = wv; blk < NB; blk += WPE) one_block(prm, slot, blk, ea, sm.gs[wave]);
    }
};

}  // namespace feint
