// Device-side building blocks shared by the forward, adjoint and mixed
// kernels: per-point geometry of the bilinear prism in FP64, the fused
// coefficient block W_q, MFMA wrappers and wave-level helpers (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

namespace feint {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef short i16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));

constexpr int WAVE = 64;

__host__ __device__ constexpr int c_nshp(int p) { return (p + 1) * (p + 1) * (p + 2) / 2; }
__host__ __device__ constexpr int c_nq(int p) { return (p + 1) * (p + 1) * (p + 1); }
// Points of the fully symmetric triangle rule of degree 2p (3, 6, 12, 16, 25,
// 33, 42 for p = 1..7) and of the prism rule R: 0 = collapsed Gauss
// (p+1)^3, 1 = symmetric triangle rule x (p+1) Gauss points in zeta (the
// point counts of the paper's Table 3).
__host__ __device__ constexpr int c_ntri_sym(int p) {
    return p == 1 ? 3 : p == 2 ? 6 : p == 3 ? 12 : p == 4 ? 16 : p == 5 ? 25 : p == 6 ? 33 : 42;
}
__host__ __device__ constexpr int c_nq_rule(int p, int r) { return r == 0 ? c_nq(p) : c_ntri_sym(p) * (p + 1); }
__host__ __device__ constexpr int c_pad16(int n) { return (n + 15) / 16 * 16; }
__host__ __device__ constexpr int c_pad8(int n) { return (n + 7) / 8 * 8; }
__host__ __device__ constexpr int c_cdiv(int a, int b) { return (a + b - 1) / b; }

// Per-element inputs, FP64 (gathered into registers by each wave).
struct ElemIn {
    double X[18];   // vertices v0..v5
    double D[9];
    double be[3];
    double c, f;
};

__device__ inline void load_elem(const double *__restrict__ coords, const double *__restrict__ D,
                                 const double *__restrict__ be, const double *__restrict__ c,
                                 const double *__restrict__ f, int64_t e, ElemIn &E) {
#pragma unroll
    for (int i = 0; i < 18; ++i) E.X[i] = coords[18 * e + i];
#pragma unroll
    for (int i = 0; i < 9; ++i) E.D[i] = D[9 * e + i];
#pragma unroll
    for (int i = 0; i < 3; ++i) E.be[i] = be[3 * e + i];
    E.c = c[e];
    E.f = f[e];
}

// Geometry at one reference point (xi1, xi2, zeta) of the bilinear prism
// (the Jacobian of Algorithm 1).  With t = (1+zeta)/2 the map is
// x = (1-t) T_bot(xi) + t T_top(xi), so the Jacobian columns are
//   dx/dxi1 = (1-t)(v1-v0) + t(v4-v3),  dx/dxi2 = (1-t)(v2-v0) + t(v5-v3),
//   dx/dzeta = ((v3-v0) l0 + (v4-v1) l1 + (v5-v2) l2) / 2,
// l = barycentrics of (xi1, xi2).  Returns det J; K = J^{-1} via cofactors.
__device__ inline double prism_jacobian(const double *X, double xi1, double xi2, double ze,
                                        double K[9]) {
    const double t = 0.5 * (1.0 + ze), s = 0.5 * (1.0 - ze);
    const double l0 = 1.0 - xi1 - xi2;
    double c0[3], c1[3], c2[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        c0[d] = s * (X[3 + d] - X[d]) + t * (X[12 + d] - X[9 + d]);
        c1[d] = s * (X[6 + d] - X[d]) + t * (X[15 + d] - X[9 + d]);
        c2[d] = 0.5 * (l0 * (X[9 + d] - X[d]) + xi1 * (X[12 + d] - X[3 + d]) + xi2 * (X[15 + d] - X[6 + d]));
    }
    // rows of J^{-1} are the cross products of pairs of columns / det
    const double r0[3] = {c1[1] * c2[2] - c1[2] * c2[1], c1[2] * c2[0] - c1[0] * c2[2], c1[0] * c2[1] - c1[1] * c2[0]};
    const double r1[3] = {c2[1] * c0[2] - c2[2] * c0[1], c2[2] * c0[0] - c2[0] * c0[2], c2[0] * c0[1] - c2[1] * c0[0]};
    const double r2[3] = {c0[1] * c1[2] - c0[2] * c1[1], c0[2] * c1[0] - c0[0] * c1[2], c0[0] * c1[1] - c0[1] * c1[0]};
    const double det = c0[0] * r0[0] + c0[1] * r0[1] + c0[2] * r0[2];
    const double inv = 1.0 / det;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        K[d] = r0[d] * inv;
        K[3 + d] = r1[d] * inv;
        K[6 + d] = r2[d] * inv;
    }
    return det;
}

__device__ inline void prism_map(const double *X, double xi1, double xi2, double ze, double x[3]) {
    const double t = 0.5 * (1.0 + ze), s = 0.5 * (1.0 - ze), l0 = 1.0 - xi1 - xi2;
#pragma unroll
    for (int d = 0; d < 3; ++d)
        x[d] = s * (l0 * X[d] + xi1 * X[3 + d] + xi2 * X[6 + d]) + t * (l0 * X[9 + d] + xi1 * X[12 + d] + xi2 * X[15 + d]);
}

// Fused coefficient block of one point (step a5 of the hot path):
// grad phi_a . D grad phi_b = ref_a . (K D K^T) ref_b and
// beta . grad phi_b = (K beta) . ref_b, so with wd = w det J
//   W = wd [[ c, (K beta)^T ], [ 0, K D K^T ]]     (4x4, row-major into W[16])
// and sf = wd f is the load-vector weight.  El holds D, be, c, f.
template <class El>
__device__ inline void fused_block(const El &E, const double K[9], double wd, double W[16], double &sf) {
    double KD[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            KD[3 * i + j] = K[3 * i] * E.D[j] + K[3 * i + 1] * E.D[3 + j] + K[3 * i + 2] * E.D[6 + j];
    W[0] = wd * E.c;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        W[1 + i] = wd * (K[3 * i] * E.be[0] + K[3 * i + 1] * E.be[1] + K[3 * i + 2] * E.be[2]);
        W[4 * (i + 1)] = 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j)
            W[4 * (i + 1) + 1 + j] = wd * (KD[3 * i] * K[3 * j] + KD[3 * i + 1] * K[3 * j + 1] + KD[3 * i + 2] * K[3 * j + 2]);
    }
    sf = wd * E.f;
}

// The Laplace term alone (the paper's eq. (1)): grad phi_a . grad phi_b =
// ref_a . (K K^T) ref_b, so W = wd [[0, 0], [0, K K^T]] (row-major into W[16]).
__device__ inline void laplace_block(const double K[9], double wd, double W[16]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) W[i] = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        W[4 * (i + 1)] = 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j)
            W[4 * (i + 1) + 1 + j] = wd * (K[3 * i] * K[3 * j] + K[3 * i + 1] * K[3 * j + 1] + K[3 * i + 2] * K[3 * j + 2]);
    }
}

// Prism: W_q and sf at reference point (xi1, xi2, zeta) with weight w; returns det J.
__device__ inline double point_block(const ElemIn &E, double xi1, double xi2, double ze, double w,
                                     double W[16], double &sf) {
    double K[9];
    const double det = prism_jacobian(E.X, xi1, xi2, ze, K);
    fused_block(E, K, w * det, W, sf);
    return det;
}

// ---------------------------------------------------------------------------
// Hexahedra (trilinear geometry on the reference cube [-1,1]^3; vertex
// v = i + 2j + 4k sits at (2i-1, 2j-1, 2k-1)).
struct ElemHex {
    double X[24];   // vertices v0..v7
    double D[9];
    double be[3];
    double c, f;
};

// Jacobian columns of the trilinear map as averages of the four parallel
// edge vectors, weighted by the bilinear factors of the other two
// coordinates: dx/dxi = sum over the edges along xi of
// (v_hi - v_lo) (1 +- eta)(1 +- zeta) / 8, and likewise for eta and zeta.
// Returns det J; K = J^{-1} via cofactors.
__device__ inline double hex_jacobian(const double *X, double xi, double eta, double ze, double K[9]) {
    const double a0 = 1.0 - xi, a1 = 1.0 + xi, b0 = 1.0 - eta, b1 = 1.0 + eta, g0 = 1.0 - ze, g1 = 1.0 + ze;
    double c0[3], c1[3], c2[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double x0 = X[d], x1 = X[3 + d], x2 = X[6 + d], x3 = X[9 + d];
        const double x4 = X[12 + d], x5 = X[15 + d], x6 = X[18 + d], x7 = X[21 + d];
        c0[d] = 0.125 * (b0 * g0 * (x1 - x0) + b1 * g0 * (x3 - x2) + b0 * g1 * (x5 - x4) + b1 * g1 * (x7 - x6));
        c1[d] = 0.125 * (a0 * g0 * (x2 - x0) + a1 * g0 * (x3 - x1) + a0 * g1 * (x6 - x4) + a1 * g1 * (x7 - x5));
        c2[d] = 0.125 * (a0 * b0 * (x4 - x0) + a1 * b0 * (x5 - x1) + a0 * b1 * (x6 - x2) + a1 * b1 * (x7 - x3));
    }
    const double r0[3] = {c1[1] * c2[2] - c1[2] * c2[1], c1[2] * c2[0] - c1[0] * c2[2], c1[0] * c2[1] - c1[1] * c2[0]};
    const double r1[3] = {c2[1] * c0[2] - c2[2] * c0[1], c2[2] * c0[0] - c2[0] * c0[2], c2[0] * c0[1] - c2[1] * c0[0]};
    const double r2[3] = {c0[1] * c1[2] - c0[2] * c1[1], c0[2] * c1[0] - c0[0] * c1[2], c0[0] * c1[1] - c0[1] * c1[0]};
    const double det = c0[0] * r0[0] + c0[1] * r0[1] + c0[2] * r0[2];
    const double inv = 1.0 / det;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        K[d] = r0[d] * inv;
        K[3 + d] = r1[d] * inv;
        K[6 + d] = r2[d] * inv;
    }
    return det;
}

__device__ inline void hex_map(const double *X, double xi, double eta, double ze, double x[3]) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        // trilinear interpolation, one coordinate direction at a time
        const double e00 = X[d] + 0.5 * (1.0 + xi) * (X[3 + d] - X[d]);
        const double e10 = X[6 + d] + 0.5 * (1.0 + xi) * (X[9 + d] - X[6 + d]);
        const double e01 = X[12 + d] + 0.5 * (1.0 + xi) * (X[15 + d] - X[12 + d]);
        const double e11 = X[18 + d] + 0.5 * (1.0 + xi) * (X[21 + d] - X[18 + d]);
        const double f0 = e00 + 0.5 * (1.0 + eta) * (e10 - e00), f1 = e01 + 0.5 * (1.0 + eta) * (e11 - e01);
        x[d] = f0 + 0.5 * (1.0 + ze) * (f1 - f0);
    }
}

__device__ inline double point_block_hex(const ElemHex &E, double xi, double eta, double ze, double w,
                                         double W[16], double &sf) {
    double K[9];
    const double det = hex_jacobian(E.X, xi, eta, ze, K);
    fused_block(E, K, w * det, W, sf);
    return det;
}

// ---------------------------------------------------------------------------
// Tetrahedra (affine map of the reference tetrahedron {xi >= 0, sum xi <= 1}:
// x = v0 + J xi with the edge vectors v_i - v0 as the columns of J).
struct ElemTet {
    double X[12];   // vertices v0..v3
    double D[9];
    double be[3];
    double c, f;
};

// det J and K = J^{-1} (rows = cross products of pairs of edge vectors / det);
// the same at every point of the element.
__device__ inline double tet_jacobian(const double *X, double K[9]) {
    double c0[3], c1[3], c2[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        c0[d] = X[3 + d] - X[d];
        c1[d] = X[6 + d] - X[d];
        c2[d] = X[9 + d] - X[d];
    }
    const double r0[3] = {c1[1] * c2[2] - c1[2] * c2[1], c1[2] * c2[0] - c1[0] * c2[2], c1[0] * c2[1] - c1[1] * c2[0]};
    const double r1[3] = {c2[1] * c0[2] - c2[2] * c0[1], c2[2] * c0[0] - c2[0] * c0[2], c2[0] * c0[1] - c2[1] * c0[0]};
    const double r2[3] = {c0[1] * c1[2] - c0[2] * c1[1], c0[2] * c1[0] - c0[0] * c1[2], c0[0] * c1[1] - c0[1] * c1[0]};
    const double det = c0[0] * r0[0] + c0[1] * r0[1] + c0[2] * r0[2];
    const double inv = 1.0 / det;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        K[d] = r0[d] * inv;
        K[3 + d] = r1[d] * inv;
        K[6 + d] = r2[d] * inv;
    }
    return det;
}

__device__ inline void tet_map(const double *X, double a, double b, double c, double x[3]) {
#pragma unroll
    for (int d = 0; d < 3; ++d)
        x[d] = X[d] + a * (X[3 + d] - X[d]) + b * (X[6 + d] - X[d]) + c * (X[9 + d] - X[d]);
}

__device__ inline double point_block_tet(const ElemTet &E, double w, double W[16], double &sf) {
    double K[9];
    const double det = tet_jacobian(E.X, K);
    fused_block(E, K, w * det, W, sf);
    return det;
}

// Compiler-level fence for data exchanged through LDS between lanes of one
// wave (a wave's LDS operations complete in issue order).
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int I>
using ic = std::integral_constant<int, I>;

// for (i = B; i < E; ++i) f(i) with i a compile-time constant
template <int B, int E, class Fn>
__device__ __forceinline__ void static_for(Fn &&f) {
    if constexpr (B < E) {
        f(ic<B>{});
        static_for<B + 1, E>(f);
    }
}

__device__ inline int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline int64_t wave_uniform64(int64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// A copy of a wave-uniform pointer that the compiler can see is uniform
// (values passed to non-inlined functions are otherwise taken as divergent).
template <typename T>
__device__ inline const T *uniform_ptr(const T *p) {
    const uint64_t v = (uint64_t)(uintptr_t)p;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return (const T *)(uintptr_t)(((uint64_t)hi << 32) | lo);
}

// Raw buffer access: a resource over BYTES bytes from a wave-uniform base (stride
// 0, the CDNA data-format word), addressed by a per-lane 32-bit byte offset plus
// a wave-uniform byte offset.  Accesses past BYTES are dropped (stores) or read
// zero (loads) by the hardware's range check.
__device__ inline __amdgpu_buffer_rsrc_t buffer_rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
__device__ inline void buffer_store(double v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)voff, (int)soff, 0);
}
__device__ inline void buffer_store(float v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)voff, (int)soff, 0);
}
template <typename T> __device__ inline T buffer_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff);
template <> __device__ inline double buffer_load<double>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}
template <> __device__ inline float buffer_load<float>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}

// The same wave-uniform pointer, opaque to the optimiser: table values read
// through it are loaded where they are used instead of being hoisted out of
// the loops (where, held in scalar registers across them, they can outnumber
// the scalar register file and spill).
template <class PT>
__device__ __forceinline__ PT fresh(PT p) {
    asm volatile("" : "+s"(p));
    return p;
}

// Fused multiply-add in the operands' own precision.
__device__ inline float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ inline double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Row length of per-lane LDS rows holding 16 values: padded so that the
// 16-byte accesses of 16 consecutive lanes fall in distinct banks (20 floats
// = 80 B, 18 doubles = 144 B) while every row stays 16-byte aligned.
template <typename T> struct WROW;
template <> struct WROW<float> { static constexpr int value = 20; };
template <> struct WROW<double> { static constexpr int value = 18; };

// ---- MFMA wrappers --------------------------------------------------------
// 16x16x4 (FP64, FP32): lane l supplies A[l%16][l/16] and B[l/16][l%16].
// 16x16x32 (bf16, fp16): lane l supplies A[l%16][8(l/16)+v], B[8(l/16)+v][l%16].
// FP32 accumulators: lane l holds D[4(l/16)+r][l%16], r = 0..3.
__device__ inline f64x4 mfma4(double a, double b, f64x4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline f32x4 mfma4(float a, float b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline f32x4 mfma32(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ inline f32x4 mfma32(f16x8 a, f16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}
// 16x16x16 (bf16, fp16): lane l supplies A[l%16][4(l/16)+v], B[4(l/16)+v][l%16], v = 0..3.
__device__ inline f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ inline f32x4 mfma16(f16x4 a, f16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
}
// 4x4x4, 16 independent blocks (bf16, fp16): block b = l/4; lane l supplies
// A_b[l%4][v] and B_b[v][l%4], v = 0..3, and holds D_b[r][l%4], r = 0..3.
__device__ inline f32x4 mfma4b(bf16x4 a, bf16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(a, b, c, 0, 0, 0);
}
__device__ inline f32x4 mfma4b(f16x4 a, f16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_4x4x4f16(a, b, c, 0, 0, 0);
}

}  // namespace feint
