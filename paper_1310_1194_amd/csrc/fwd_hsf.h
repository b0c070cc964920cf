// Forward kernel for hexahedra by sum factorisation in all three directions
// (FP64, FP32 on the vector ALU): O((p+1)^7) work per element in place of the
// (p+1)^9 of the point-by-point contraction (the tensor-product reduction the
// paper's introduction notes for hexahedra).
//
// Points q = (q1, q2, q3) are tensor Gauss points, shape functions
// a = (a1, a2, a3) tensor Gauss-Lobatto Lagrange functions with the 1D factors
// l_k and their derivatives d_k.  Row s of B_q is phi (s = 0) or d/dxi_s
// (s = 1..3), a product of one 1D factor per direction, the derivative in
// direction s only.  With W_q as in the other kernels (whose column t = 0 is
// zero below the diagonal: the value phi_b only meets the value phi_a),
//   A[a][b] = sum_q sum_(s,t) B_q[s][a] W_q[s][t] B_q[t][b]
// is contracted one direction at a time, each pass keeping only the
// derivative flags the later directions still need:
//   T1[cs][ct](q2, q3; a1, b1) = sum_q1 (factors of a1, b1 in xi1) W   (cs, ct: flags in xi2, xi3)
//   T2[s3][t3](q3; a1 a2, b1 b2) = sum_q2 (factors of a2, b2 in xi2) T1
//   A[(a3 a2 a1)][(b3 b2 b1)]   = sum_q3 (factors of a3, b3 in xi3) T2
// with the classes cs in {A = {phi, d/dxi1}, B = {d/dxi2}, C = {d/dxi3}}
// (A contracts xi1 with l or d, B and C with l) and s3 = 1 only for C.
// Per element: 13 n^5 + (9 + 6n) n^5 + (4n^2 + 2n^3) n^4 fused multiply-adds
// with n = p+1, i.e. 2 n^7 at leading order, against 8 n^9 / 2 for the dense
// contraction.  The load vector is the same contraction of w det J f with the
// values alone, in FP64.
//
// Work layout: a workgroup owns EPW elements; a lane owns one (element, a1)
// slot and one pair (q3, b1) in the first two passes -- T1 for all q2 in
// registers, T2 for one a2 and all b2 -- then, after an exchange through
// LDS, one pair (b2, b1) in the last pass, which writes for its (element,
// a1, a2) the n^2 entries (a3, b3) of A: the n^2 lanes of a slot write n^2
// consecutive entries of one row per store.  Slots that do not fit the
// workgroup's lanes at once run in further passes over the same W_q.
#pragma once
#include "fwd_kernels.h"
#include "hex_factors.h"
#include <type_traits>

namespace feint {

// A table value as an FP32 instruction literal.
template <uint64_t BITS>
__device__ __forceinline__ float kval() {
    return (float)__builtin_bit_cast(double, BITS);
}
#define FEINT_HL(K, M) kval<__builtin_bit_cast(uint64_t, hexc::Fac<P>::v.L[K][M])>()
#define FEINT_HD(K, M) kval<__builtin_bit_cast(uint64_t, hexc::Fac<P>::v.D[K][M])>()

template <int P, typename T, int NTH, int EPW, bool RECOMP = false, bool LEAN = false>
struct KH {
    static constexpr int n = P + 1, N2 = n * n, N3 = N2 * n;
    // LDS strides of the exchange, in elements of T, against one row of the banks
    // (M elements = 256 bytes).  A slot writes N2 consecutive elements (lane (q3, b1))
    // and reads rows b2 = 0..n-1 at stride BS (lane (b2, b1)): BS >= N2 is the first
    // stride whose n row segments of n elements share a bank least often, and a slot
    // starts N2 banks after the previous one, so the writes of a wave fill consecutive
    // banks.
    static constexpr int M = 256 / (int)sizeof(T);
    __host__ __device__ static constexpr int bank_mult(int bs) {
        int cnt[256] = {}, mx = 0;
        for (int rh = 0; rh < n; ++rh)
            for (int rl = 0; rl < n; ++rl) {
                const int c = ++cnt[(rh * bs + rl) % M];
                mx = c > mx ? c : mx;
            }
        return mx;
    }
    __host__ __device__ static constexpr int row_stride() {
        int best = N2, bm = bank_mult(N2);
        for (int bs = N2 + 1; bs < N2 + M; ++bs)
            if (bank_mult(bs) < bm) { bm = bank_mult(bs); best = bs; }
        return best;
    }
    static constexpr int BS = row_stride();
    static constexpr int SS = 4 * n * BS + (((N2 - 4 * n * BS) % M) + M) % M;
    static constexpr int SPP = NTH / N2;                       // (element, a1) slots per pass
    static constexpr int SLOTS = EPW * n;
    static constexpr int PASSES = (SLOTS + SPP - 1) / SPP;
    static constexpr int NWC = 13;                             // nonzero entries of W_q
    static_assert(SPP >= 1, "a slot needs (p+1)^2 lanes");
    // RECOMP: with several passes, W_q is formed again at the start of each pass, so
    // that the exchange can share its space (half the LDS: two workgroups per CU)
    static constexpr bool ALIAS = PASSES == 1 || RECOMP;
    static constexpr size_t W_BYTES = (size_t)EPW * NWC * N3 * sizeof(T);
    static constexpr size_t S_BYTES = (size_t)EPW * 2 * N3 * sizeof(double);
    static constexpr size_t X_BYTES = (size_t)SPP * SS * sizeof(T);
    static constexpr size_t LDS_BYTES =
        ALIAS ? (W_BYTES + S_BYTES > X_BYTES ? W_BYTES + S_BYTES : X_BYTES) : W_BYTES + S_BYTES + X_BYTES;
    static_assert(LDS_BYTES <= 160 * 1024, "LDS budget of one workgroup");

    // W_q entries kept (row-major index into W[16]): the first column below the
    // diagonal is zero
    __device__ static constexpr int widx(int k) {
        return k < 4 ? k : k < 7 ? k + 1 : k < 10 ? k + 2 : k + 3;
    }

    __device__ static void run(const FwdParams &prm, unsigned char *smem) {
        T *Wl = (T *)smem;                                        // [EPW][13][q1][q2][q3]
        double *S0 = (double *)(smem + W_BYTES);                  // [EPW][N3]
        double *S1 = S0 + EPW * N3;
        T *Xl = (T *)(ALIAS ? smem : smem + W_BYTES + S_BYTES);    // [SPP][SS]: [4][n][BS] per slot
        const int tid = threadIdx.x;
        const int64_t e0 = (int64_t)blockIdx.x * EPW;
        const T *lam = sizeof(T) == 8 ? (const T *)(const void *)prm.lam : (const T *)(const void *)prm.lam32;
        const T *Lt = lam, *Dt = lam + 3 * N2;                    // l_k(g_m), d_k(g_m) at [k][m]
        // the factors the later passes index with wave-uniform values: FP32 literals,
        // FP64 scalar loads
        typedef const __attribute__((address_space(4))) T CT;
        const CT *Lu = (const CT *)Lt, *Du = (const CT *)Dt;
        constexpr bool LIT = sizeof(T) == 4;

        // ---- W_q, w det J f, mapped points and the det J flag, one point per lane
        // (`first`: the first time, which also writes the per-point outputs)
        auto form_w = [&](bool first) {
            for (int pi = tid; pi < EPW * N3; pi += NTH) {
                const int el = pi / N3, q = pi - el * N3;
                const int q1 = q % n, q2 = (q / n) % n, q3 = q / N2;
                const int wq = (q1 * n + q2) * n + q3;
                const int64_t e = e0 + el;
                double W[16], sf = 0.0;
                if (e < prm.ne) {
                    ElemHex E;
                    HexGeo::load(prm, e, E);
                    const double *qp = prm.qw + 4 * q;
                    const double det = HexGeo::block(E, qp, W, sf);
                    if (first && !(det > 0.0) && prm.status) atomicOr(prm.status, 1u);
                    if (first && prm.xq) {
                        double x[3];
                        HexGeo::map(E, qp, x);
#pragma unroll
                        for (int d = 0; d < 3; ++d) prm.xq[(e * N3 + q) * 3 + d] = x[d];
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < 16; ++k) W[k] = 0.0;
                }
#pragma unroll
                for (int k = 0; k < NWC; ++k) Wl[(el * NWC + k) * N3 + wq] = (T)W[widx(k)];
                if (first) S0[el * N3 + q] = sf;
            }
        };
        form_w(true);
        __syncthreads();

        // ---- load vector b[(a3 a2 a1)] = sum_q l_a1 l_a2 l_a3 (w det J f)_q, in FP64
        const double *L64 = prm.lam;
        for (int i = tid; i < EPW * N3; i += NTH) {               // S1[(q3 q2) a1] = sum_q1
            const int el = i / N3, r = i - el * N3, a1 = r % n, qq = r - a1;
            double s = 0.0;
#pragma unroll
            for (int q1 = 0; q1 < n; ++q1) s += L64[a1 * n + q1] * S0[el * N3 + qq + q1];
            S1[i] = s;
        }
        __syncthreads();
        for (int i = tid; i < EPW * N3; i += NTH) {               // S0[(q3 a2) a1] = sum_q2
            const int el = i / N3, r = i - el * N3, a1 = r % n, a2 = (r / n) % n, q3 = r / N2;
            double s = 0.0;
#pragma unroll
            for (int q2 = 0; q2 < n; ++q2) s += L64[a2 * n + q2] * S1[el * N3 + (q3 * n + q2) * n + a1];
            S0[i] = s;
        }
        __syncthreads();
        for (int i = tid; i < EPW * N3; i += NTH) {               // b[(a3 a2) a1] = sum_q3
            const int el = i / N3, r = i - el * N3, a12 = r % N2, a3 = r / N2;
            const int64_t e = e0 + el;
            double s = 0.0;
#pragma unroll
            for (int q3 = 0; q3 < n; ++q3) s += L64[a3 * n + q3] * S0[el * N3 + q3 * N2 + a12];
            if (e < prm.ne) ((T *)prm.b + offb_of(prm, e, N3))[r] = (T)s;
        }

        const int g = tid / N2, r = tid - g * N2;
        const int rh = r / n, rl = r - rh * n;                    // (q3, b1), then (b2, b1)
        for (int ps = 0; ps < PASSES; ++ps) {
            if (RECOMP && ps > 0) {                               // the exchange held W_q's space
                form_w(false);
                __syncthreads();
            }
            const int slot = ps * SPP + g;
            const bool active = g < SPP && slot < SLOTS;
            const int el = active ? slot / n : 0, a1 = active ? slot - el * n : 0;
            const int64_t e = e0 + el;
            const bool store = active && e < prm.ne;
            const int q3 = rh, b1 = rl;

            // ---- pass 1 (xi1): T1[cs][ct][q2] for this lane's (a1, q3, b1)
            T t1[9][n];
#pragma unroll
            for (int c = 0; c < 9; ++c)
#pragma unroll
                for (int m = 0; m < n; ++m) t1[c][m] = (T)0;
            if (active) {
                const T *wel = Wl + el * NWC * N3;
                for (int q1 = 0; q1 < n; ++q1) {
                    const T xa = Lt[a1 * n + q1], dxa = Dt[a1 * n + q1];
                    const T xb = Lt[b1 * n + q1], dxb = Dt[b1 * n + q1];
                    const T xab = xa * xb, xadb = xa * dxb, daxb = dxa * xb, dadb = dxa * dxb;
#pragma unroll
                    for (int q2 = 0; q2 < n; ++q2) {
                        const T *w = wel + (q1 * n + q2) * n + q3;
                        T wv[NWC];
#pragma unroll
                        for (int k = 0; k < NWC; ++k) wv[k] = w[k * N3];
                        // wv: 00 01 02 03 11 12 13 21 22 23 31 32 33
                        t1[0][q2] = fma_t(xab, wv[0], fma_t(xadb, wv[1], fma_t(dadb, wv[4], t1[0][q2])));
                        t1[1][q2] = fma_t(xab, wv[2], fma_t(daxb, wv[5], t1[1][q2]));
                        t1[2][q2] = fma_t(xab, wv[3], fma_t(daxb, wv[6], t1[2][q2]));
                        t1[3][q2] = fma_t(xadb, wv[7], t1[3][q2]);
                        t1[4][q2] = fma_t(xab, wv[8], t1[4][q2]);
                        t1[5][q2] = fma_t(xab, wv[9], t1[5][q2]);
                        t1[6][q2] = fma_t(xadb, wv[10], t1[6][q2]);
                        t1[7][q2] = fma_t(xab, wv[11], t1[7][q2]);
                        t1[8][q2] = fma_t(xab, wv[12], t1[8][q2]);
                    }
                }
            }
            if (ALIAS) __syncthreads();                           // W_q and b's space become the exchange

            T *xs = Xl + (active ? g : 0) * SS;
            for (int a2 = 0; a2 < n; ++a2) {
                // ---- pass 2 (xi2): T2[s3][t3][b2] for this lane's (a1, a2, q3, b1); LEAN: one s3
                // half at a time (2n accumulators live instead of 4n)
                auto pass2 = [&](auto s0c, auto s1c) {
                    constexpr int S0 = decltype(s0c)::value, S1 = decltype(s1c)::value;
                    T t2[4][n];
#pragma unroll
                    for (int c = 2 * S0; c < 2 * S1; ++c)
#pragma unroll
                        for (int m = 0; m < n; ++m) t2[c][m] = (T)0;
                    static_for<0, n>([&](auto q2c) {
                        constexpr int q2 = decltype(q2c)::value;
                        const CT *Lq = fresh(Lu), *Dq = fresh(Du);
                        const T ya = Lq[a2 * n + q2], dya = Dq[a2 * n + q2];
                        T v[2][3];
#pragma unroll
                        for (int ct = 0; ct < 3; ++ct) {
                            if (S0 == 0) v[0][ct] = fma_t(ya, t1[ct][q2], dya * t1[3 + ct][q2]);
                            if (S1 == 2) v[1][ct] = ya * t1[6 + ct][q2];
                        }
                        static_for<0, n>([&](auto b2c) {
                            constexpr int b2 = decltype(b2c)::value;
                            T yb, dyb;
                            if constexpr (LIT) {
                                yb = FEINT_HL(b2, q2);
                                dyb = FEINT_HD(b2, q2);
                            } else {
                                yb = Lq[b2 * n + q2];
                                dyb = Dq[b2 * n + q2];
                            }
#pragma unroll
                            for (int s = S0; s < S1; ++s) {
                                t2[2 * s][b2] = fma_t(yb, v[s][0], fma_t(dyb, v[s][1], t2[2 * s][b2]));
                                t2[2 * s + 1][b2] = fma_t(yb, v[s][2], t2[2 * s + 1][b2]);
                            }
                        });
                    });
                    if (active) {
#pragma unroll
                        for (int c = 2 * S0; c < 2 * S1; ++c)
#pragma unroll
                            for (int b2 = 0; b2 < n; ++b2) xs[(c * n + b2) * BS + q3 * n + b1] = t2[c][b2];
                    }
                };
                if constexpr (LEAN) {
                    pass2(ic<0>{}, ic<1>{});
                    pass2(ic<1>{}, ic<2>{});
                } else {
                    pass2(ic<0>{}, ic<2>{});
                }
                __syncthreads();
                // ---- pass 3 (xi3): this lane now owns (b2, b1) = (rh, rl)
                T t3[4][n];
                if (!LEAN && active) {
#pragma unroll
                    for (int c = 0; c < 4; ++c)
#pragma unroll
                        for (int m = 0; m < n; ++m) t3[c][m] = xs[(c * n + rh) * BS + m * n + rl];
                }
                if (!LEAN) __syncthreads();
                if (LEAN) {
                    // T2 read from the exchange where it is used, the q3 sum taken point by point
                    // into n accumulators (instead of 4n T2 values and 2n folded ones in registers)
                    if (store) {
                        T *row0 = (T *)prm.A + offA_of(prm, e, N3) + (size_t)(a2 * n + a1) * N3 + rh * n + rl;
                        const T *xr = xs + rh * BS + rl;
                        static_for<0, n>([&](auto a3c) {
                            constexpr int a3 = decltype(a3c)::value;
                            T acc[n];
#pragma unroll
                            for (int k = 0; k < n; ++k) acc[k] = (T)0;
                            const CT *La = fresh(Lu), *Da = fresh(Du);
                            static_for<0, n>([&](auto mc) {
                                constexpr int m = decltype(mc)::value;
                                T za, dza;
                                if constexpr (LIT) {
                                    za = FEINT_HL(a3, m);
                                    dza = FEINT_HD(a3, m);
                                } else {
                                    za = La[a3 * n + m];
                                    dza = Da[a3 * n + m];
                                }
                                const T x0 = xr[(0 * n) * BS + m * n], x1 = xr[(1 * n) * BS + m * n];
                                const T x2 = xr[(2 * n) * BS + m * n], x3 = xr[(3 * n) * BS + m * n];
                                const T u0 = fma_t(za, x0, dza * x2), u1 = fma_t(za, x1, dza * x3);
                                const CT *Lm = fresh((const CT *)&hexc::FacT<P>::v.L[m][0]);
                                const CT *Dm = fresh((const CT *)&hexc::FacT<P>::v.D[m][0]);
                                static_for<0, n>([&](auto bc) {
                                    constexpr int b3 = decltype(bc)::value;
                                    if constexpr (LIT)
                                        acc[b3] = fma_t(FEINT_HL(b3, m), u0, fma_t(FEINT_HD(b3, m), u1, acc[b3]));
                                    else
                                        acc[b3] = fma_t((T)Lm[b3], u0, fma_t((T)Dm[b3], u1, acc[b3]));
                                });
                            });
                            T *row = row0 + (size_t)a3 * N2 * N3;
#pragma unroll
                            for (int b3 = 0; b3 < n; ++b3) row[b3 * N2] = acc[b3];
                        });
                    }
                    __syncthreads();                              // the exchange is written again next
                } else if (store) {
                    T *row0 = (T *)prm.A + offA_of(prm, e, N3) + (size_t)(a2 * n + a1) * N3 + rh * n + rl;
                    static_for<0, n>([&](auto a3c) {
                        constexpr int a3 = decltype(a3c)::value;
                        T u0[n], u1[n];
                        const CT *La = fresh(Lu), *Da = fresh(Du);
                        static_for<0, n>([&](auto mc) {
                            constexpr int m = decltype(mc)::value;
                            T za, dza;
                            if constexpr (LIT) {
                                za = FEINT_HL(a3, m);
                                dza = FEINT_HD(a3, m);
                            } else {
                                za = La[a3 * n + m];
                                dza = Da[a3 * n + m];
                            }
                            u0[m] = fma_t(za, t3[0][m], dza * t3[2][m]);
                            u1[m] = fma_t(za, t3[1][m], dza * t3[3][m]);
                        });
                        T *row = row0 + (size_t)a3 * N2 * N3;
                        static_for<0, n>([&](auto b3c) {
                            constexpr int b3 = decltype(b3c)::value;
                            const CT *Lb = fresh(Lu), *Db = fresh(Du);
                            T s = (T)0;
                            static_for<0, n>([&](auto mc) {
                                constexpr int m = decltype(mc)::value;
                                if constexpr (LIT)
                                    s = fma_t(FEINT_HL(b3, m), u0[m], fma_t(FEINT_HD(b3, m), u1[m], s));
                                else
                                    s = fma_t(Lb[b3 * n + m], u0[m], fma_t(Db[b3 * n + m], u1[m], s));
                            });
                            row[b3 * N2] = s;
                        });
                    });
                }
            }
        }
    }
};

template <class KER, int NTH, int MINW>
__global__ void __launch_bounds__(NTH, MINW) fwd_hsf(FwdParams prm) {
    __shared__ __attribute__((aligned(16))) unsigned char smem[KER::LDS_BYTES];
    KER::run(prm, smem);
}

template <int P, typename T, int NTH, int EPW, bool RECOMP, int MINW, bool LEAN = false>
void launch_hsf(const FwdParams &prm, hipStream_t s) {
    const int64_t blocks = (prm.ne + EPW - 1) / EPW;
    if (blocks > 0)
        hipLaunchKernelGGL((fwd_hsf<KH<P, T, NTH, EPW, RECOMP, LEAN>, NTH, MINW>), dim3((unsigned)blocks), dim3(NTH),
                           0, s, prm);
}

// four work items per workgroup in the launcher's count (its grid-size check)
template <int EPW>
int64_t items_hsf(int64_t ne) { return 4 * ((ne + EPW - 1) / EPW); }

}  // namespace feint
