/*
 * feint_oracle.c -- plain, slow, FP64 CPU oracle for element-by-element
 * numerical integration on geometrically bilinear prisms.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  The GPU library shares no
 * code, header, table or constant with it; the two meet only in the seeded
 * input generator (which holds none of this arithmetic).
 *
 * What it computes (Krużel & Banaś, Sec. 2, eqs. (1)-(2), Algorithm 1),
 * generalised from the Laplace term to convection-diffusion-reaction plus a
 * load vector.  For every element e, with constant D (3x3), beta (3), c, f:
 *
 *     A_ab = sum_I  w_I det J(xi_I) [ grad phi_a . D grad phi_b
 *                                     + phi_a (beta . grad phi_b)
 *                                     + c phi_a phi_b ]
 *     b_a  = sum_I  w_I det J(xi_I) f phi_a
 *
 * with row a = test function, grad phi = J^{-T} (reference gradient)
 * (Sec. 2, change of variables) and the signed determinant (eq. (2)).
 *
 * Readings where the paper is silent (all shared with the GPU library as a
 * specification, not as code):
 *   - reference prism = triangle {xi1,xi2 >= 0, xi1+xi2 <= 1} x [-1,1];
 *   - quadrature: Duffy-collapsed Gauss-Legendre, n1 points per direction,
 *     xi1 = (1+a)(1-b)/4, xi2 = (1+b)/2, zeta = z,  w = wa wb wz (1-b)/8,
 *     point index q = (k*n1 + j)*n1 + i  (a_i, b_j, z_k);  n1 = p+1 by default;
 *   - basis (Sec. 2, Table 1 prism row: triangle complete basis x 1D basis):
 *     Lagrange on the equispaced triangle lattice (i/p, j/p), i+j <= p,
 *     ordered j outer / i inner, times 1D Lagrange on the p+1 Gauss-Lobatto
 *     nodes, ascending; shape function a = k*ntri + t;
 *   - geometry (Sec. 4, bilinear prism): x = sum_a N_a x_a with
 *     N_a = lambda_a (1-zeta)/2, N_{a+3} = lambda_a (1+zeta)/2,
 *     lambda = (1-xi1-xi2, xi1, xi2).
 *
 * Parity status of every function is listed in the test-suite; none is
 * "parity unpinned".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_MAXP 7
#define ORACLE_MAXN1 24

/* ---------------------------------------------------------------------- */
/* 1D Gauss-Legendre and Gauss-Lobatto-Legendre nodes                      */
/* ---------------------------------------------------------------------- */

/* Legendre P_n(x) and P_n'(x) by the three-term recurrence
   k P_k = (2k-1) x P_{k-1} - (k-1) P_{k-2}; derivative from
   (1-x^2) P_n' = n (P_{n-1} - x P_n).  Valid for |x| < 1. */
static void legendre(int n, double x, double *P, double *dP)
{
    double pm1 = 1.0, pk = x;
    if (n == 0) { *P = 1.0; *dP = 0.0; return; }
    for (int k = 2; k <= n; ++k) {
        double pn = ((2.0 * k - 1.0) * x * pk - (k - 1.0) * pm1) / k;
        pm1 = pk;
        pk = pn;
    }
    *P = pk;
    *dP = n * (pm1 - x * pk) / (1.0 - x * x);
}

/* n Gauss-Legendre nodes (ascending) and weights on [-1,1]:
   Newton's method on P_n, w = 2 / ((1-x^2) P_n'(x)^2). */
int oracle_gauss_legendre(int n, double *x, double *w)
{
    if (n < 1 || n > 64) return -1;
    for (int i = 0; i < n; ++i) {
        double xi = cos(M_PI * (i + 0.75) / (n + 0.5));
        double P, dP;
        for (int it = 0; it < 100; ++it) {
            legendre(n, xi, &P, &dP);
            double dx = P / dP;
            xi -= dx;
            if (fabs(dx) < 1e-17) break;
        }
        legendre(n, xi, &P, &dP);
        x[n - 1 - i] = xi;
        w[n - 1 - i] = 2.0 / ((1.0 - xi * xi) * dP * dP);
    }
    return 0;
}

/* p+1 Gauss-Lobatto-Legendre nodes (ascending): -1, the p-1 roots of P_p',
   +1.  Newton on P_p' with P_p'' from Legendre's equation
   (1-x^2) P'' = 2x P' - p(p+1) P. */
int oracle_gll_nodes(int p, double *x)
{
    if (p < 1 || p > 32) return -1;
    x[0] = -1.0;
    x[p] = 1.0;
    for (int k = 1; k < p; ++k) {
        double xi = -cos(M_PI * k / p);
        double P, dP;
        for (int it = 0; it < 100; ++it) {
            legendre(p, xi, &P, &dP);
            double d2P = (2.0 * xi * dP - p * (p + 1.0) * P) / (1.0 - xi * xi);
            double dx = dP / d2P;
            xi -= dx;
            if (fabs(dx) < 1e-17) break;
        }
        x[k] = xi;
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Quadrature on the reference prism                                      */
/* ---------------------------------------------------------------------- */

/* Collapsed Gauss rule with n1 points per direction: pts[q] = (xi1, xi2,
   zeta), w[q].  Returns the number of points n1^3. */
int oracle_rule(int n1, double *pts, double *w)
{
    double g[ORACLE_MAXN1], gw[ORACLE_MAXN1];
    if (n1 < 1 || n1 > ORACLE_MAXN1) return -1;
    oracle_gauss_legendre(n1, g, gw);
    int q = 0;
    for (int k = 0; k < n1; ++k)
        for (int j = 0; j < n1; ++j)
            for (int i = 0; i < n1; ++i) {
                double a = g[i], b = g[j], z = g[k];
                pts[3 * q + 0] = (1.0 + a) * (1.0 - b) / 4.0;
                pts[3 * q + 1] = (1.0 + b) / 2.0;
                pts[3 * q + 2] = z;
                w[q] = gw[i] * gw[j] * gw[k] * (1.0 - b) / 8.0;
                ++q;
            }
    return q;
}

/* ---------------------------------------------------------------------- */
/* Shape functions: equispaced triangle Lagrange (Silvester) x GLL Lagrange */
/* ---------------------------------------------------------------------- */

int oracle_nshp(int p) { return (p < 1 || p > ORACLE_MAXP) ? -1 : (p + 1) * (p + 1) * (p + 2) / 2; }

/* Silvester's factor R_m(lambda) = prod_{s<m} (p*lambda - s)/(s+1) and its
   derivative with respect to lambda (product rule). */
static void silvester(int p, int m, double lam, double *R, double *dR)
{
    double val = 1.0, der = 0.0;
    for (int s = 0; s < m; ++s) {
        double fac = (p * lam - s) / (s + 1.0);
        double dfac = p / (s + 1.0);
        der = der * fac + val * dfac;
        val = val * fac;
    }
    *R = val;
    *dR = der;
}

/* Nodes of the element's shape functions: nodes[a] = (xi1, xi2, zeta). */
int oracle_nodes(int p, double *nodes)
{
    double z[ORACLE_MAXP + 1];
    if (p < 1 || p > ORACLE_MAXP) return -1;
    oracle_gll_nodes(p, z);
    int a = 0;
    for (int k = 0; k <= p; ++k)
        for (int j = 0; j <= p; ++j)
            for (int i = 0; i <= p - j; ++i) {
                nodes[3 * a + 0] = (double)i / p;
                nodes[3 * a + 1] = (double)j / p;
                nodes[3 * a + 2] = z[k];
                ++a;
            }
    return a;
}

/* Values phi[a] and reference gradients dphi[a][3] (d/dxi1, d/dxi2,
   d/dzeta) of all shape functions at one point of the reference prism. */
int oracle_basis(int p, const double *xi, double *phi, double *dphi)
{
    double z[ORACLE_MAXP + 1];
    if (p < 1 || p > ORACLE_MAXP) return -1;
    oracle_gll_nodes(p, z);
    const double x1 = xi[0], x2 = xi[1], ze = xi[2];
    const double lam[3] = {1.0 - x1 - x2, x1, x2};
    const int ntri = (p + 1) * (p + 2) / 2;
    double psi[64], dpsi1[64], dpsi2[64];
    int t = 0;
    for (int j = 0; j <= p; ++j)
        for (int i = 0; i <= p - j; ++i) {
            int al[3] = {p - i - j, i, j};
            double R[3], dR[3];
            for (int m = 0; m < 3; ++m) silvester(p, al[m], lam[m], &R[m], &dR[m]);
            double dl0 = dR[0] * R[1] * R[2];   /* d psi / d lambda_0 */
            double dl1 = R[0] * dR[1] * R[2];
            double dl2 = R[0] * R[1] * dR[2];
            psi[t] = R[0] * R[1] * R[2];
            dpsi1[t] = dl1 - dl0;               /* lambda_0 = 1 - xi1 - xi2 */
            dpsi2[t] = dl2 - dl0;
            ++t;
        }
    for (int k = 0; k <= p; ++k) {
        double l = 1.0, dl = 0.0;
        for (int m = 0; m <= p; ++m) {
            if (m == k) continue;
            double fac = (ze - z[m]) / (z[k] - z[m]);
            double dfac = 1.0 / (z[k] - z[m]);
            dl = dl * fac + l * dfac;
            l = l * fac;
        }
        for (int tt = 0; tt < ntri; ++tt) {
            int a = k * ntri + tt;
            phi[a] = psi[tt] * l;
            dphi[3 * a + 0] = dpsi1[tt] * l;
            dphi[3 * a + 1] = dpsi2[tt] * l;
            dphi[3 * a + 2] = psi[tt] * dl;
        }
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Geometry of the bilinear prism                                          */
/* ---------------------------------------------------------------------- */

/* Geometry shape functions N[6] and their reference gradients dN[6][3]. */
static void geom_shape(const double *xi, double *N, double *dN)
{
    const double x1 = xi[0], x2 = xi[1], ze = xi[2];
    const double lam[3] = {1.0 - x1 - x2, x1, x2};
    const double dlam[3][2] = {{-1.0, -1.0}, {1.0, 0.0}, {0.0, 1.0}};
    for (int a = 0; a < 3; ++a) {
        double lo = (1.0 - ze) / 2.0, hi = (1.0 + ze) / 2.0;
        N[a] = lam[a] * lo;
        N[a + 3] = lam[a] * hi;
        dN[3 * a + 0] = dlam[a][0] * lo;
        dN[3 * a + 1] = dlam[a][1] * lo;
        dN[3 * a + 2] = -lam[a] / 2.0;
        dN[3 * (a + 3) + 0] = dlam[a][0] * hi;
        dN[3 * (a + 3) + 1] = dlam[a][1] * hi;
        dN[3 * (a + 3) + 2] = lam[a] / 2.0;
    }
}

static int invert3(const double *J, double *det, double *K);

/* J[d][l] = d x_d / d xi_l, det J (cofactor expansion along row 0),
   K = J^{-1} = adj(J) / det, and the mapped point x. */
int oracle_geometry(const double *X, const double *xi, double *J, double *det,
                    double *K, double *x)
{
    double N[6], dN[18];
    geom_shape(xi, N, dN);
    for (int d = 0; d < 3; ++d) {
        if (x) {
            x[d] = 0.0;
            for (int a = 0; a < 6; ++a) x[d] += N[a] * X[3 * a + d];
        }
        for (int l = 0; l < 3; ++l) {
            double s = 0.0;
            for (int a = 0; a < 6; ++a) s += X[3 * a + d] * dN[3 * a + l];
            J[3 * d + l] = s;
        }
    }
    return invert3(J, det, K);
}

/* det J (cofactor expansion along row 0) and K = J^{-1} = adj(J) / det;
   returns 1 when det J <= 0. */
static int invert3(const double *J, double *det, double *K)
{
    double c00 = J[4] * J[8] - J[5] * J[7];
    double c01 = J[5] * J[6] - J[3] * J[8];
    double c02 = J[3] * J[7] - J[4] * J[6];
    double dt = J[0] * c00 + J[1] * c01 + J[2] * c02;
    *det = dt;
    if (K) {
        /* K = adj(J)/det, adj(J)[l][d] = cofactor C[d][l] */
        K[0] = c00 / dt;
        K[3] = c01 / dt;
        K[6] = c02 / dt;
        K[1] = (J[2] * J[7] - J[1] * J[8]) / dt;
        K[4] = (J[0] * J[8] - J[2] * J[6]) / dt;
        K[7] = (J[1] * J[6] - J[0] * J[7]) / dt;
        K[2] = (J[1] * J[5] - J[2] * J[4]) / dt;
        K[5] = (J[2] * J[3] - J[0] * J[5]) / dt;
        K[8] = (J[0] * J[4] - J[1] * J[3]) / dt;
    }
    return dt > 0.0 ? 0 : 1;
}

/* ---------------------------------------------------------------------- */
/* Hexahedra (Table 1, tensor-product basis)                               */
/* ---------------------------------------------------------------------- */
/* Reference cube [-1,1]^3 (volume 8).  Vertices v = i + 2j + 4k at
   (2i-1, 2j-1, 2k-1), trilinear geometry N_v = (1 + s_v xi)(1 + t_v eta)
   (1 + u_v zeta) / 8; shape functions phi_a = L_i(xi) L_j(eta) L_k(zeta),
   a = (k (p+1) + j) (p+1) + i, with L the Lagrange basis on the p+1
   Gauss-Lobatto nodes; rule: n1^3 Gauss-Legendre points, q = (k n1 + j) n1 + i. */

int oracle_hex_nshp(int p) { return (p < 1 || p > ORACLE_MAXP) ? -1 : (p + 1) * (p + 1) * (p + 1); }

int oracle_hex_rule(int n1, double *pts, double *w)
{
    double g[ORACLE_MAXN1], gw[ORACLE_MAXN1];
    if (n1 < 1 || n1 > ORACLE_MAXN1) return -1;
    oracle_gauss_legendre(n1, g, gw);
    int q = 0;
    for (int k = 0; k < n1; ++k)
        for (int j = 0; j < n1; ++j)
            for (int i = 0; i < n1; ++i) {
                pts[3 * q + 0] = g[i];
                pts[3 * q + 1] = g[j];
                pts[3 * q + 2] = g[k];
                w[q] = gw[i] * gw[j] * gw[k];
                ++q;
            }
    return q;
}

/* Lagrange basis on the nodes z[0..p] at x: l[k], dl[k] (product formula). */
static void line_lagrange(int p, const double *z, double x, double *l, double *dl)
{
    for (int k = 0; k <= p; ++k) {
        double v = 1.0, d = 0.0;
        for (int m = 0; m <= p; ++m) {
            if (m == k) continue;
            double fac = (x - z[m]) / (z[k] - z[m]);
            double dfac = 1.0 / (z[k] - z[m]);
            d = d * fac + v * dfac;
            v = v * fac;
        }
        l[k] = v;
        dl[k] = d;
    }
}

int oracle_hex_nodes(int p, double *nodes)
{
    double z[ORACLE_MAXP + 1];
    if (p < 1 || p > ORACLE_MAXP) return -1;
    oracle_gll_nodes(p, z);
    int a = 0;
    for (int k = 0; k <= p; ++k)
        for (int j = 0; j <= p; ++j)
            for (int i = 0; i <= p; ++i) {
                nodes[3 * a + 0] = z[i];
                nodes[3 * a + 1] = z[j];
                nodes[3 * a + 2] = z[k];
                ++a;
            }
    return a;
}

int oracle_hex_basis(int p, const double *xi, double *phi, double *dphi)
{
    double z[ORACLE_MAXP + 1], l[3][ORACLE_MAXP + 1], dl[3][ORACLE_MAXP + 1];
    if (p < 1 || p > ORACLE_MAXP) return -1;
    oracle_gll_nodes(p, z);
    for (int d = 0; d < 3; ++d) line_lagrange(p, z, xi[d], l[d], dl[d]);
    int a = 0;
    for (int k = 0; k <= p; ++k)
        for (int j = 0; j <= p; ++j)
            for (int i = 0; i <= p; ++i) {
                phi[a] = l[0][i] * l[1][j] * l[2][k];
                dphi[3 * a + 0] = dl[0][i] * l[1][j] * l[2][k];
                dphi[3 * a + 1] = l[0][i] * dl[1][j] * l[2][k];
                dphi[3 * a + 2] = l[0][i] * l[1][j] * dl[2][k];
                ++a;
            }
    return 0;
}

/* Trilinear geometry shape functions N[8] and reference gradients dN[8][3]. */
static void hex_shape(const double *xi, double *N, double *dN)
{
    for (int v = 0; v < 8; ++v) {
        const double s = (v & 1) ? 1.0 : -1.0, t = (v & 2) ? 1.0 : -1.0, u = (v & 4) ? 1.0 : -1.0;
        const double a = 1.0 + s * xi[0], b = 1.0 + t * xi[1], c = 1.0 + u * xi[2];
        N[v] = a * b * c / 8.0;
        dN[3 * v + 0] = s * b * c / 8.0;
        dN[3 * v + 1] = a * t * c / 8.0;
        dN[3 * v + 2] = a * b * u / 8.0;
    }
}

/* J = sum_v x_v (grad N_v)^T, det J, K = J^{-1}, mapped point x; X [8][3]. */
int oracle_hex_geometry(const double *X, const double *xi, double *J, double *det, double *K, double *x)
{
    double N[8], dN[24];
    hex_shape(xi, N, dN);
    for (int d = 0; d < 3; ++d) {
        if (x) {
            x[d] = 0.0;
            for (int v = 0; v < 8; ++v) x[d] += N[v] * X[3 * v + d];
        }
        for (int l = 0; l < 3; ++l) {
            double s = 0.0;
            for (int v = 0; v < 8; ++v) s += X[3 * v + d] * dN[3 * v + l];
            J[3 * d + l] = s;
        }
    }
    return invert3(J, det, K);
}

/* ---------------------------------------------------------------------- */
/* Tetrahedra (Table 1, complete basis)                                    */
/* ---------------------------------------------------------------------- */
/* Reference tetrahedron {xi >= 0, xi1 + xi2 + xi3 <= 1} (volume 1/6),
   vertices v0 = 0, v1 = e1, v2 = e2, v3 = e3, affine geometry x = v0 +
   sum_i xi_i (v_i - v0).  Shape functions: Lagrange on the lattice
   (i/p, j/p, k/p), i + j + k <= p, k outer, j middle, i inner, by
   Silvester's product in the four barycentric coordinates.  Rule: n1^3
   collapsed Gauss-Legendre points (n1 = p+2 by default, exact for products of
   shape functions), z = (1+c)/2, y = (1+b)(1-z)/2, x = (1+a)(1-y-z)/2,
   w = w_a w_b w_c (1-b)(1-c)^2 / 64, q = (k n1 + j) n1 + i (a_i, b_j, c_k). */

int oracle_tet_nshp(int p) { return (p < 1 || p > ORACLE_MAXP) ? -1 : (p + 1) * (p + 2) * (p + 3) / 6; }

int oracle_tet_rule(int n1, double *pts, double *w)
{
    double g[ORACLE_MAXN1], gw[ORACLE_MAXN1];
    if (n1 < 1 || n1 > ORACLE_MAXN1) return -1;
    oracle_gauss_legendre(n1, g, gw);
    int q = 0;
    for (int k = 0; k < n1; ++k)
        for (int j = 0; j < n1; ++j)
            for (int i = 0; i < n1; ++i) {
                double a = g[i], b = g[j], c = g[k];
                double z = (1.0 + c) / 2.0;
                double y = (1.0 + b) * (1.0 - z) / 2.0;
                double x = (1.0 + a) * (1.0 - y - z) / 2.0;
                pts[3 * q + 0] = x;
                pts[3 * q + 1] = y;
                pts[3 * q + 2] = z;
                w[q] = gw[i] * gw[j] * gw[k] * (1.0 - b) * (1.0 - c) * (1.0 - c) / 64.0;
                ++q;
            }
    return q;
}

int oracle_tet_nodes(int p, double *nodes)
{
    if (p < 1 || p > ORACLE_MAXP) return -1;
    int a = 0;
    for (int k = 0; k <= p; ++k)
        for (int j = 0; j <= p - k; ++j)
            for (int i = 0; i <= p - j - k; ++i) {
                nodes[3 * a + 0] = (double)i / p;
                nodes[3 * a + 1] = (double)j / p;
                nodes[3 * a + 2] = (double)k / p;
                ++a;
            }
    return a;
}

int oracle_tet_basis(int p, const double *xi, double *phi, double *dphi)
{
    if (p < 1 || p > ORACLE_MAXP) return -1;
    const double lam[4] = {1.0 - xi[0] - xi[1] - xi[2], xi[0], xi[1], xi[2]};
    int a = 0;
    for (int k = 0; k <= p; ++k)
        for (int j = 0; j <= p - k; ++j)
            for (int i = 0; i <= p - j - k; ++i) {
                int al[4] = {p - i - j - k, i, j, k};
                double R[4], dR[4];
                for (int m = 0; m < 4; ++m) silvester(p, al[m], lam[m], &R[m], &dR[m]);
                double d0 = dR[0] * R[1] * R[2] * R[3];     /* d phi / d lambda_0 */
                phi[a] = R[0] * R[1] * R[2] * R[3];
                dphi[3 * a + 0] = R[0] * dR[1] * R[2] * R[3] - d0;
                dphi[3 * a + 1] = R[0] * R[1] * dR[2] * R[3] - d0;
                dphi[3 * a + 2] = R[0] * R[1] * R[2] * dR[3] - d0;
                ++a;
            }
    return 0;
}

/* Affine tetrahedron X [4][3]: J[d][l] = (v_{l+1} - v_0)_d, det, K, x. */
int oracle_tet_geometry(const double *X, const double *xi, double *J, double *det, double *K, double *x)
{
    for (int d = 0; d < 3; ++d) {
        for (int l = 0; l < 3; ++l) J[3 * d + l] = X[3 * (l + 1) + d] - X[d];
        if (x) x[d] = X[d] + J[3 * d] * xi[0] + J[3 * d + 1] * xi[1] + J[3 * d + 2] * xi[2];
    }
    return invert3(J, det, K);
}

/* ---------------------------------------------------------------------- */
/* Algorithm 1: element loop -> quadrature loop -> i -> j                  */
/* ---------------------------------------------------------------------- */

typedef struct {
    int type, p, n, nq;                     /* type 0: prism, 1: hexahedron, 2: tetrahedron */
    double *pts, *w, *phi, *dphi; /* [nq][3], [nq], [nq][n], [nq][n][3] */
} rule_tables;

/* Tables of degree p on a rule: the caller's points (qpts [nq][3], qw [nq])
   when qpts is given, else the collapsed Gauss rule with n1 points per
   direction (n1 <= 0: p+1). */
static int make_tables(int type, int p, int n1, int nq, const double *qpts, const double *qw, rule_tables *T)
{
    if (p < 1 || p > ORACLE_MAXP) return -1;
    if (n1 <= 0) n1 = type == 2 ? p + 2 : p + 1;
    if (n1 > ORACLE_MAXN1) return -1;
    if (qpts && (nq < 1 || !qw)) return -1;
    T->type = type;
    T->p = p;
    T->n = type == 2 ? oracle_tet_nshp(p) : type ? oracle_hex_nshp(p) : oracle_nshp(p);
    T->nq = qpts ? nq : n1 * n1 * n1;
    T->pts = (double *)malloc(sizeof(double) * 3 * T->nq);
    T->w = (double *)malloc(sizeof(double) * T->nq);
    T->phi = (double *)malloc(sizeof(double) * T->nq * T->n);
    T->dphi = (double *)malloc(sizeof(double) * 3 * T->nq * T->n);
    if (qpts) {
        memcpy(T->pts, qpts, sizeof(double) * 3 * T->nq);
        memcpy(T->w, qw, sizeof(double) * T->nq);
    } else if (type == 2) {
        oracle_tet_rule(n1, T->pts, T->w);
    } else if (type) {
        oracle_hex_rule(n1, T->pts, T->w);
    } else {
        oracle_rule(n1, T->pts, T->w);
    }
    /* Algorithm 1's shape functions at every point (the same for every
       element of degree p, so they are evaluated once) */
    for (int q = 0; q < T->nq; ++q)
        (type == 2 ? oracle_tet_basis : type ? oracle_hex_basis : oracle_basis)(
            p, T->pts + 3 * q, T->phi + (size_t)q * T->n, T->dphi + (size_t)3 * q * T->n);
    return 0;
}

static void free_tables(rule_tables *T)
{
    free(T->pts); free(T->w); free(T->phi); free(T->dphi);
}

void oracle_set_threads(int nt)
{
#ifdef _OPENMP
    if (nt > 0) omp_set_num_threads(nt);
#else
    (void)nt;
#endif
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Forward integration.  coords [ne][6][3], D [ne][3][3], beta [ne][3],
   c [ne], f [ne]  ->  A [ne][n][n] (row a = test function), b [ne][n],
   optional xq [ne][nq][3], optional flags [ne] (1 = some det J <= 0).
   n1 = points per direction of the collapsed rule (0 -> p+1). */
/* Element loop of Algorithm 1 with the CDR integrand.  Coefficients are
   constant per element (Dv etc. hold one value per element, nv = 1) or
   given at the six vertices (nv = 6) and evaluated at each point with the
   geometry shape functions, D(x_q) = sum_a N_a(xi_q) D_a (the coefficient
   fields live in the same bilinear space as the geometry). */
static int integrate_core(int type, int p, int n1, int nq, const double *qpts, const double *qw, int64_t ne,
                          int nv, const double *coords, const double *Dv, const double *betav, const double *cv,
                          const double *fv, double *A, double *b, double *xq, int32_t *flags)
{
    rule_tables T;
    if (ne < 0 || (type && nv != 1)) return -1;
    if (make_tables(type, p, n1, nq, qpts, qw, &T)) return -1;
    const int nx = type == 2 ? 12 : type ? 24 : 18;   /* coordinates per element */
    const int n = T.n, nqp = T.nq;
    int64_t e;
#pragma omp parallel for schedule(static)
    for (e = 0; e < ne; ++e) {
        const double *X = coords + (size_t)nx * e;  /* geometry data of the element */
        double *Ae = A + (size_t)e * n * n, *bv = b + (size_t)e * n;
        double *gphys = (double *)malloc(sizeof(double) * 3 * n);
        double *Dg = (double *)malloc(sizeof(double) * 3 * n);
        double *bg = (double *)malloc(sizeof(double) * n);
        int bad = 0;
        memset(Ae, 0, sizeof(double) * n * n);    /* clear the element matrix */
        memset(bv, 0, sizeof(double) * n);
        for (int q = 0; q < nqp; ++q) {           /* loop over quadrature points */
            const double *phi = T.phi + (size_t)q * n, *dphi = T.dphi + (size_t)3 * q * n;
            double J[9], K[9], det, x[3];
            bad |= (type == 2 ? oracle_tet_geometry : type ? oracle_hex_geometry : oracle_geometry)(
                X, T.pts + 3 * q, J, &det, K, x);                                      /* Jacobian, det, inverse */
            if (xq) for (int d = 0; d < 3; ++d) xq[((size_t)e * nqp + q) * 3 + d] = x[d];
            /* coefficients at the point */
            double De[9], be[3], ce, fe;
            if (nv == 1) {
                for (int m = 0; m < 9; ++m) De[m] = Dv[9 * e + m];
                for (int m = 0; m < 3; ++m) be[m] = betav[3 * e + m];
                ce = cv[e];
                fe = fv[e];
            } else {
                double N[6], dN[18];
                geom_shape(T.pts + 3 * q, N, dN);
                for (int m = 0; m < 9; ++m) De[m] = 0.0;
                for (int m = 0; m < 3; ++m) be[m] = 0.0;
                ce = fe = 0.0;
                for (int a = 0; a < 6; ++a) {
                    for (int m = 0; m < 9; ++m) De[m] += N[a] * Dv[(6 * e + a) * 9 + m];
                    for (int m = 0; m < 3; ++m) be[m] += N[a] * betav[(6 * e + a) * 3 + m];
                    ce += N[a] * cv[6 * e + a];
                    fe += N[a] * fv[6 * e + a];
                }
            }
            double wd = T.w[q] * det;
            for (int a = 0; a < n; ++a) {         /* physical derivatives: grad phi = J^{-T} ref grad */
                for (int d = 0; d < 3; ++d) {
                    double s = 0.0;
                    for (int l = 0; l < 3; ++l) s += K[3 * l + d] * dphi[3 * a + l];
                    gphys[3 * a + d] = s;
                }
                for (int d = 0; d < 3; ++d) {
                    double s = 0.0;
                    for (int m = 0; m < 3; ++m) s += De[3 * d + m] * gphys[3 * a + m];
                    Dg[3 * a + d] = s;
                }
                bg[a] = be[0] * gphys[3 * a] + be[1] * gphys[3 * a + 1] + be[2] * gphys[3 * a + 2];
            }
            for (int a = 0; a < n; ++a) {         /* double loop over shape functions, CDR integrand */
                const double *ga = gphys + 3 * a;
                for (int bb = 0; bb < n; ++bb) {
                    const double *Dgb = Dg + 3 * bb;
                    double diff = ga[0] * Dgb[0] + ga[1] * Dgb[1] + ga[2] * Dgb[2];
                    double conv = phi[a] * bg[bb];
                    double mass = ce * phi[a] * phi[bb];
                    Ae[(size_t)a * n + bb] += wd * (diff + conv + mass);
                }
                bv[a] += wd * fe * phi[a];
            }
        }
        if (flags) flags[e] = bad;
        free(gphys); free(Dg); free(bg);
    }
    free_tables(&T);
    return 0;
}

int oracle_integrate(int p, int n1, int64_t ne, const double *coords, const double *D,
                     const double *beta, const double *c, const double *f,
                     double *A, double *b, double *xq, int32_t *flags)
{
    return integrate_core(0, p, n1, 0, NULL, NULL, ne, 1, coords, D, beta, c, f, A, b, xq, flags);
}

/* Tetrahedra: coords [ne][4][3], coefficients per element; n1 collapsed
   Gauss points per direction (0 -> p+2). */
int oracle_integrate_tet(int p, int n1, int64_t ne, const double *coords, const double *D,
                         const double *beta, const double *c, const double *f,
                         double *A, double *b, double *xq, int32_t *flags)
{
    return integrate_core(2, p, n1, 0, NULL, NULL, ne, 1, coords, D, beta, c, f, A, b, xq, flags);
}

/* Hexahedra: coords [ne][8][3], coefficients per element as above; n1
   Gauss points per direction (0 -> p+1). */
int oracle_integrate_hex(int p, int n1, int64_t ne, const double *coords, const double *D,
                         const double *beta, const double *c, const double *f,
                         double *A, double *b, double *xq, int32_t *flags)
{
    return integrate_core(1, p, n1, 0, NULL, NULL, ne, 1, coords, D, beta, c, f, A, b, xq, flags);
}

/* Coefficients given at the six vertices: Dv [ne][6][9], betav [ne][6][3],
   cv [ne][6], fv [ne][6]. */
int oracle_integrate_fields(int p, int n1, int64_t ne, const double *coords, const double *Dv,
                            const double *betav, const double *cv, const double *fv,
                            double *A, double *b, double *xq, int32_t *flags)
{
    return integrate_core(0, p, n1, 0, NULL, NULL, ne, 6, coords, Dv, betav, cv, fv, A, b, xq, flags);
}

/* The same element loop on a rule given by the caller: qpts [nq][3] =
   (xi1, xi2, zeta), qw [nq]; xq (optional) is [ne][nq][3].  nv = 1:
   coefficients constant per element; nv = 6: given at the six vertices. */
int oracle_integrate_rule(int p, int nq, const double *qpts, const double *qw, int64_t ne, int nv,
                          const double *coords, const double *Dv, const double *betav, const double *cv,
                          const double *fv, double *A, double *b, double *xq, int32_t *flags)
{
    if (!qpts || (nv != 1 && nv != 6)) return -1;
    return integrate_core(0, p, 0, nq, qpts, qw, ne, nv, coords, Dv, betav, cv, fv, A, b, xq, flags);
}

/* ---------------------------------------------------------------------- */
/* Adjoint of the literal loop                                             */
/* ---------------------------------------------------------------------- */

/* Gradients of L = sum_e <G_e, A_e> + <g_e, b_e> with respect to every
   element's coordinates [ne][6][3], D [ne][3][3] (all nine entries treated
   as independent), beta [ne][3], c [ne], f [ne].  Reverse mode through the
   same steps as oracle_integrate:
     per point L_q = wd (Ldiff + Lconv + c Lmass + f Lload),  wd = w det J,
     dL/d(grad phi_a) = wd (D h_a + D^T h'_a + m_a beta),
       h_a = sum_b G_ab grad phi_b, h'_a = sum_b G_ba grad phi_b,
       m_a = sum_b G_ba phi_b;
     grad phi_a = K^T ref_a  =>  dL/dK_ld = sum_a ref_al (dL/dgrad phi_a)_d;
     dL/d det = L_q / det;  d det = det tr(K dJ);  dK = -K dJ K
       =>  dL/dJ = L_q K^T - K^T (dL/dK) K^T;
     J_dl = sum_a x_ad dN_a/dxi_l  =>  dL/dx_ad = sum_l dL/dJ_dl dN_a/dxi_l.
   Also returns the per-element loss in Le (nullable). */
static int adjoint_core(int p, int n1, int nq, const double *qpts, const double *qw, int64_t ne,
                        const double *coords, const double *D, const double *beta, const double *c,
                        const double *f, const double *G, const double *g, double *dcoords, double *dD,
                        double *dbeta, double *dc, double *df, double *Le);

int oracle_adjoint(int p, int n1, int64_t ne, const double *coords, const double *D,
                   const double *beta, const double *c, const double *f,
                   const double *G, const double *g,
                   double *dcoords, double *dD, double *dbeta, double *dc, double *df,
                   double *Le)
{
    return adjoint_core(p, n1, 0, NULL, NULL, ne, coords, D, beta, c, f, G, g, dcoords, dD, dbeta, dc, df, Le);
}

/* The adjoint on a rule given by the caller (qpts [nq][3], qw [nq]). */
int oracle_adjoint_rule(int p, int nq, const double *qpts, const double *qw, int64_t ne, const double *coords,
                        const double *D, const double *beta, const double *c, const double *f,
                        const double *G, const double *g, double *dcoords, double *dD, double *dbeta,
                        double *dc, double *df, double *Le)
{
    if (!qpts) return -1;
    return adjoint_core(p, 0, nq, qpts, qw, ne, coords, D, beta, c, f, G, g, dcoords, dD, dbeta, dc, df, Le);
}

static int adjoint_core(int p, int n1, int nq, const double *qpts, const double *qw, int64_t ne,
                        const double *coords, const double *D, const double *beta, const double *c,
                        const double *f, const double *G, const double *g, double *dcoords, double *dD,
                        double *dbeta, double *dc, double *df, double *Le)
{
    rule_tables T;
    if (ne < 0) return -1;
    if (make_tables(0, p, n1, nq, qpts, qw, &T)) return -1;
    const int n = T.n, nqp = T.nq;
    int64_t e;
#pragma omp parallel for schedule(static)
    for (e = 0; e < ne; ++e) {
        const double *X = coords + 18 * e;
        const double *De = D + 9 * e, *be = beta + 3 * e;
        const double *Ge = G + (size_t)e * n * n, *ge = g + (size_t)e * n;
        double *gphys = (double *)malloc(sizeof(double) * 3 * n);
        double *h = (double *)malloc(sizeof(double) * 3 * n);
        double *ht = (double *)malloc(sizeof(double) * 3 * n);
        double *m = (double *)malloc(sizeof(double) * n);
        double dX[18] = {0}, gD[9] = {0}, gb[3] = {0}, gc = 0.0, gf = 0.0, Ltot = 0.0;
        for (int q = 0; q < nqp; ++q) {
            const double *phi = T.phi + (size_t)q * n, *dphi = T.dphi + (size_t)3 * q * n;
            double J[9], K[9], det, N[6], dN[18];
            oracle_geometry(X, T.pts + 3 * q, J, &det, K, NULL);
            geom_shape(T.pts + 3 * q, N, dN);
            double wd = T.w[q] * det;
            for (int a = 0; a < n; ++a)
                for (int d = 0; d < 3; ++d) {
                    double s = 0.0;
                    for (int l = 0; l < 3; ++l) s += K[3 * l + d] * dphi[3 * a + l];
                    gphys[3 * a + d] = s;
                }
            for (int a = 0; a < n; ++a) {
                double h0 = 0, h1 = 0, h2 = 0, t0 = 0, t1 = 0, t2 = 0, mm = 0;
                for (int bb = 0; bb < n; ++bb) {
                    double gab = Ge[(size_t)a * n + bb], gba = Ge[(size_t)bb * n + a];
                    h0 += gab * gphys[3 * bb]; h1 += gab * gphys[3 * bb + 1]; h2 += gab * gphys[3 * bb + 2];
                    t0 += gba * gphys[3 * bb]; t1 += gba * gphys[3 * bb + 1]; t2 += gba * gphys[3 * bb + 2];
                    mm += gba * phi[bb];
                }
                h[3 * a] = h0; h[3 * a + 1] = h1; h[3 * a + 2] = h2;
                ht[3 * a] = t0; ht[3 * a + 1] = t1; ht[3 * a + 2] = t2;
                m[a] = mm;
            }
            /* point loss pieces */
            double Ldiff = 0, Lconv = 0, Lmass = 0, Lload = 0;
            double gDq[9] = {0}, gbq[3] = {0};
            for (int a = 0; a < n; ++a) {
                const double *ga = gphys + 3 * a, *ha = h + 3 * a;
                for (int d = 0; d < 3; ++d)
                    for (int mm = 0; mm < 3; ++mm) {
                        Ldiff += ga[d] * De[3 * d + mm] * ha[mm];
                        gDq[3 * d + mm] += ga[d] * ha[mm];
                    }
                for (int d = 0; d < 3; ++d) {
                    Lconv += phi[a] * be[d] * ha[d];
                    gbq[d] += phi[a] * ha[d];
                }
                Lmass += phi[a] * m[a] ;
                Lload += ge[a] * phi[a];
            }
            /* Lmass above = sum_a phi_a sum_b G_ba phi_b = sum_ab G_ab phi_a phi_b */
            double Lq = wd * (Ldiff + Lconv + c[e] * Lmass + f[e] * Lload);
            Ltot += Lq;
            for (int k = 0; k < 9; ++k) gD[k] += wd * gDq[k];
            for (int d = 0; d < 3; ++d) gb[d] += wd * gbq[d];
            gc += wd * Lmass;
            gf += wd * Lload;
            /* dL/dK */
            double dK[9] = {0};
            for (int a = 0; a < n; ++a) {
                double dga[3];
                for (int d = 0; d < 3; ++d) {
                    double s = 0.0;
                    for (int mm = 0; mm < 3; ++mm)
                        s += De[3 * d + mm] * h[3 * a + mm] + De[3 * mm + d] * ht[3 * a + mm];
                    dga[d] = wd * (s + m[a] * be[d]);
                }
                for (int l = 0; l < 3; ++l)
                    for (int d = 0; d < 3; ++d) dK[3 * l + d] += dphi[3 * a + l] * dga[d];
            }
            /* dL/dJ = Lq K^T - K^T dK K^T */
            double dJ[9];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    double s = 0.0;
                    for (int l = 0; l < 3; ++l)
                        for (int mm = 0; mm < 3; ++mm) s += K[3 * l + i] * dK[3 * l + mm] * K[3 * j + mm];
                    dJ[3 * i + j] = Lq * K[3 * j + i] - s;
                }
            for (int a = 0; a < 6; ++a)
                for (int d = 0; d < 3; ++d) {
                    double s = 0.0;
                    for (int l = 0; l < 3; ++l) s += dJ[3 * d + l] * dN[3 * a + l];
                    dX[3 * a + d] += s;
                }
        }
        memcpy(dcoords + 18 * e, dX, sizeof dX);
        memcpy(dD + 9 * e, gD, sizeof gD);
        memcpy(dbeta + 3 * e, gb, sizeof gb);
        dc[e] = gc;
        df[e] = gf;
        if (Le) Le[e] = Ltot;
        free(gphys); free(h); free(ht); free(m);
    }
    free_tables(&T);
    return 0;
}
