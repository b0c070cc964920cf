// Reference tables of one polynomial degree: quadrature points and weights
// and the shape-function values and reference gradients at every point,
// laid out for the kernels.  These are the quadrature data and shape
// functions the paper's Algorithm 1 reads (and, in Sec. 2.2, recommends keeping in fast memory
// because they are identical for every element of a degree).
#pragma once
#include <cstdint>
#include <vector>

namespace feint {

constexpr int kMaxP = 7;

inline int nshp_of(int p) { return (p + 1) * (p + 1) * (p + 2) / 2; }
inline int ntri_of(int p) { return (p + 1) * (p + 2) / 2; }
inline int nq_of(int p) { return (p + 1) * (p + 1) * (p + 1); }
// Points of the symmetric triangle rule of degree 2p and of the prism rule
// `rule` (0: collapsed Gauss (p+1)^3; 1: symmetric triangle rule x (p+1)
// Gauss points in zeta).
inline int ntri_sym_of(int p) {
    static const int k[8] = {0, 3, 6, 12, 16, 25, 33, 42};
    return (p >= 1 && p <= 7) ? k[p] : 0;
}
inline int nq_rule_of(int p, int rule) { return rule == 0 ? nq_of(p) : ntri_sym_of(p) * (p + 1); }
inline int pad16(int n) { return (n + 15) / 16 * 16; }
inline int pad8(int n) { return (n + 7) / 8 * 8; }

struct HostTables {
    int p = 0, rule = 0, n = 0, npad = 0, nq = 0, nqp = 0, nkb = 0;
    int f16_shift = 0;               // fp16 tables hold B * 2^f16_shift
    std::vector<double> qw;          // [nqp][4]  xi1, xi2, zeta, w  (padded points: w = 0)
    std::vector<double> gll;         // [2][p+1]  Gauss-Lobatto nodes z_k and 1 / prod_{m != k} (z_k - z_m)
    // prisms and hexahedra: tensor factors of B (q = m nij + ij, a = k ntri + t; for
    // hexahedra ntri = nij = (p+1)^2 plane functions and points):
    int nk = 0, nij = 0, tpad = 0;
    std::vector<double> tau64;       // [nij][4][tpad]  T, dT/dxi1, dT/dxi2, T at triangle point ij
    std::vector<float> tau32;
    std::vector<double> lam;         // [4][nk][nk]     L_k, L_k, L_k, dL_k/dzeta at zeta point m
    std::vector<float> lam32;        // lam rounded to FP32
    // tau split into bf16 hi + lo in 16x16x32 A-fragment order, [nij/8 chunks][tpad/16]
    // [64 lanes][8]: lane l, value v holds tau_r(t, ij) with t = 16 tile + l%16,
    // ij = 8 chunk + 2 (l/16) + v/4, r = v%4 (zero past the last triangle point)
    std::vector<uint16_t> taub_hi, taub_lo;
    // the same in fp16, of tau * 2^tau_f16_shift (max |tau| * 2^shift in [2^13, 2^14))
    std::vector<uint16_t> tauh_hi, tauh_lo;
    int tau_f16_shift = 0;
    // fp16 form's bounds: |Z| <= f16_zc * max |W entry| of the element, and the
    // load vector's zeta sums <= f16_zb * max |w det J f|
    double f16_zc = 0.0, f16_zb = 0.0;
    std::vector<double> B64;         // [nqp][4][npad]  rows: phi, d/dxi1, d/dxi2, d/dzeta
    std::vector<float> B32;          // same, rounded to FP32
    std::vector<double> BT64;        // [npad][nqp*4]  transpose of B64 (shape-function major)
    std::vector<float> BT32;         // same, FP32
    std::vector<float> Bc32;         // [nqp][npad][4]  the four rows of a column side by side, FP32
    // Split tables in 16x16x32 MFMA A-fragment order: [nkb][npad/16][64 lanes][8],
    // lane l holds rows 16 t + l%16, k = 8 (l/16) .. +7 of K-block kb, where
    // k = 4*(point in block) + row (phi, d/dxi1, d/dxi2, d/dzeta).
    std::vector<uint16_t> bf_hi, bf_lo;   // bf16
    std::vector<uint16_t> hf_hi, hf_lo;   // fp16 of B * 2^f16_shift
    // FP32 columns in B-fragment order: [nkb][npad/16][64 lanes][2][4], lane
    // l holds column 16 t + l%16 at points 2 (l/16) and 2 (l/16) + 1 of the
    // K-block, four rows each.
    std::vector<float> Ycf;
    // Tetrahedra (affine, so W_q = w_q W with one W per element): the reference
    // matrices M_rs = sum_q w_q B_q[r]^T B_q[s] of the 13 nonzero entries (r, s) of
    // W, slot-major [16][n*n padded to a multiple of 16] (slots 0..12 in the order
    // 00 01 02 03 11 12 13 21 22 23 31 32 33, entry a*n + b; slots 13..15 and the
    // padding zero), then the reference load vector
    // m0[a] = sum_q w_q phi_a(q); summed in extended precision.
    std::vector<double> Mref;
    std::vector<float> Mref32;
};

// Points of the prism rule `rule` for degree p: qw [nq][4] = (xi1, xi2, zeta,
// w); collapsed Gauss q = (k n1 + j) n1 + i, symmetric q = k ntri + t.
void rule_points(int p, int rule, std::vector<double> &qw);

// Build every table of degree p (1..7) on quadrature rule `rule` (0, 1) in
// FP64 on the host.
HostTables build_tables(int p, int rule = 0);
// Tables of the hexahedral element of degree p: tensor Gauss rule (q = (k n1 +
// j) n1 + i, points on [-1,1]^3) and the tensor-product Gauss-Lobatto
// Lagrange basis (a = (k (p+1) + j) (p+1) + i).
HostTables build_hex_tables(int p);
// Tables of the tetrahedral element of degree p: (p+2)^3 collapsed Gauss
// points (q = (k n1 + j) n1 + i) and the Lagrange basis on the tetrahedral
// lattice (k outer, j, i inner).
HostTables build_tet_tables(int p);

// Pieces exposed for the CPU tests of the library's host logic.
void gauss_legendre_gw(int n, double *x, double *w);     // Golub-Welsch
void gauss_lobatto_nodes(int p, double *x);               // p+1 nodes, ascending
// phi[n], dphi[n][3] at one reference point, through the Vandermonde construction.
void lagrange_prism_eval(int p, const double *xi, double *phi, double *dphi);
// Points (xi1, xi2) and weights of the symmetric triangle rule of degree 2p,
// in orbit order (centroid, 3-orbits, 6-orbits).
void symmetric_triangle_rule(int p, std::vector<double> &xi1, std::vector<double> &xi2, std::vector<double> &w);

}  // namespace feint
