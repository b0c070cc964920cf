// Host construction of the reference tables (FP64, then rounded or split for
// the reduced-precision forms).
//
// Constructions used here:
//   * Gauss-Legendre nodes/weights and the interior Gauss-Lobatto nodes are
//     eigenvalues of the symmetric Jacobi matrices of the Legendre and the
//     Jacobi(1,1) recurrences (Golub-Welsch), found with cyclic Jacobi
//     rotations; a weight is 2 * (first eigenvector component)^2.
//   * Lagrange bases are obtained by inverting the generalised Vandermonde
//     matrix of a Legendre-product modal basis at the nodes (LU with partial
//     pivoting in extended precision), then evaluating the modal basis and
//     its derivatives at each quadrature point.
#include "tables.h"

#include <cmath>
#include <cstring>
#include <stdexcept>

namespace feint {
namespace {

// Eigen-decomposition of a small symmetric matrix a (n x n, row-major,
// destroyed) by cyclic Jacobi rotations.  vals[j] with eigenvector column
// vecs[:, j].
void jacobi_eigen(int n, std::vector<long double> &a, std::vector<long double> &vals,
                  std::vector<long double> &vecs) {
    vecs.assign(n * n, 0.0L);
    for (int i = 0; i < n; ++i) vecs[i * n + i] = 1.0L;
    for (int sweep = 0; sweep < 64; ++sweep) {
        long double off = 0, diag = 0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j)
                (i == j ? diag : off) += a[i * n + j] * a[i * n + j];
        if (off <= 1e-40L * diag) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                long double apq = a[p * n + q];
                if (std::fabs(apq) < 1e-300L) continue;
                long double theta = (a[q * n + q] - a[p * n + p]) / (2.0L * apq);
                long double t = (theta >= 0 ? 1.0L : -1.0L) /
                                (std::fabs(theta) + std::sqrt(theta * theta + 1.0L));
                long double c = 1.0L / std::sqrt(t * t + 1.0L), s = t * c;
                // A <- R^T A R with R the rotation in the (p, q) plane
                for (int k = 0; k < n; ++k) {
                    long double akp = a[k * n + p], akq = a[k * n + q];
                    a[k * n + p] = c * akp - s * akq;
                    a[k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {
                    long double apk = a[p * n + k], aqk = a[q * n + k];
                    a[p * n + k] = c * apk - s * aqk;
                    a[q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    long double vkp = vecs[k * n + p], vkq = vecs[k * n + q];
                    vecs[k * n + p] = c * vkp - s * vkq;
                    vecs[k * n + q] = s * vkp + c * vkq;
                }
            }
    }
    vals.resize(n);
    for (int i = 0; i < n; ++i) vals[i] = a[i * n + i];
}

// Symmetric tridiagonal matrix with zero diagonal and off-diagonal
// entries off[k] at (k, k+1); eigenvalues ascending with first components.
void tridiag_eigen(int n, const std::vector<long double> &off, std::vector<long double> &x,
                   std::vector<long double> &v0) {
    std::vector<long double> a(n * n, 0.0L), vals, vecs;
    for (int k = 0; k + 1 < n; ++k) a[k * n + k + 1] = a[(k + 1) * n + k] = off[k];
    jacobi_eigen(n, a, vals, vecs);
    std::vector<int> idx(n);
    for (int i = 0; i < n; ++i) idx[i] = i;
    for (int i = 0; i < n; ++i)       // selection sort, n <= 24
        for (int j = i + 1; j < n; ++j)
            if (vals[idx[j]] < vals[idx[i]]) std::swap(idx[i], idx[j]);
    x.resize(n);
    v0.resize(n);
    for (int i = 0; i < n; ++i) {
        x[i] = vals[idx[i]];
        long double nrm = 0;
        for (int k = 0; k < n; ++k) nrm += vecs[k * n + idx[i]] * vecs[k * n + idx[i]];
        v0[i] = vecs[idx[i]] / std::sqrt(nrm);
    }
}

// Legendre P_k(x) and P_k'(x) for k = 0..m (values into P[], derivatives into dP[]).
void legendre_all(int m, long double x, long double *P, long double *dP) {
    P[0] = 1.0L;
    dP[0] = 0.0L;
    if (m >= 1) { P[1] = x; dP[1] = 1.0L; }
    for (int k = 1; k < m; ++k) {
        P[k + 1] = ((2 * k + 1) * x * P[k] - k * P[k - 1]) / (k + 1);
        dP[k + 1] = dP[k - 1] + (2 * k + 1) * P[k];
    }
}

// Inverse of a small dense matrix by LU with partial pivoting.
std::vector<long double> invert(int n, std::vector<long double> m) {
    std::vector<int> piv(n);
    for (int i = 0; i < n; ++i) piv[i] = i;
    for (int c = 0; c < n; ++c) {
        int best = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(m[r * n + c]) > std::fabs(m[best * n + c])) best = r;
        if (m[best * n + c] == 0.0L) throw std::runtime_error("singular Vandermonde matrix");
        if (best != c) {
            for (int k = 0; k < n; ++k) std::swap(m[c * n + k], m[best * n + k]);
            std::swap(piv[c], piv[best]);
        }
        for (int r = c + 1; r < n; ++r) {
            long double l = m[r * n + c] / m[c * n + c];
            m[r * n + c] = l;
            for (int k = c + 1; k < n; ++k) m[r * n + k] -= l * m[c * n + k];
        }
    }
    std::vector<long double> inv(n * n, 0.0L);
    for (int col = 0; col < n; ++col) {
        std::vector<long double> y(n);
        for (int i = 0; i < n; ++i) {          // forward: L y = P e_col
            long double s = (piv[i] == col) ? 1.0L : 0.0L;
            for (int k = 0; k < i; ++k) s -= m[i * n + k] * y[k];
            y[i] = s;
        }
        for (int i = n - 1; i >= 0; --i) {     // backward: U x = y
            long double s = y[i];
            for (int k = i + 1; k < n; ++k) s -= m[i * n + k] * inv[k * n + col];
            inv[i * n + col] = s / m[i * n + i];
        }
    }
    return inv;
}

struct ModalBasis {
    int p = 0, ntri = 0;
    std::vector<long double> Ctri;   // [mode][t] inverse Vandermonde of the triangle
    std::vector<long double> Cline;  // [mode][k] inverse Vandermonde of the GLL line
    std::vector<int> mi, mj;         // triangle mode m = P_mi(2 xi1 - 1) P_mj(2 xi2 - 1)
};

ModalBasis make_modal(int p) {
    ModalBasis mb;
    mb.p = p;
    mb.ntri = ntri_of(p);
    for (int j = 0; j <= p; ++j)
        for (int i = 0; i + j <= p; ++i) { mb.mi.push_back(i); mb.mj.push_back(j); }
    const int nt = mb.ntri;
    std::vector<long double> V(nt * nt), Pa(p + 1), dPa(p + 1), Pb(p + 1), dPb(p + 1);
    int t = 0;
    for (int j = 0; j <= p; ++j)
        for (int i = 0; i + j <= p; ++i, ++t) {
            long double x1 = (long double)i / p, x2 = (long double)j / p;
            legendre_all(p, 2 * x1 - 1, Pa.data(), dPa.data());
            legendre_all(p, 2 * x2 - 1, Pb.data(), dPb.data());
            for (int m = 0; m < nt; ++m) V[t * nt + m] = Pa[mb.mi[m]] * Pb[mb.mj[m]];
        }
    mb.Ctri = invert(nt, V);
    double z[kMaxP + 1];
    gauss_lobatto_nodes(p, z);
    std::vector<long double> V1((p + 1) * (p + 1));
    for (int k = 0; k <= p; ++k) {
        legendre_all(p, z[k], Pa.data(), dPa.data());
        for (int m = 0; m <= p; ++m) V1[k * (p + 1) + m] = Pa[m];
    }
    mb.Cline = invert(p + 1, V1);
    return mb;
}

// The tensor factors of the prism basis phi_(k,t) = T_t(xi1, xi2) L_k(zeta):
// T, dT/dxi1, dT/dxi2 (ntri each) and L, dL/dzeta (p+1 each).
void eval_factors(const ModalBasis &mb, double x1, double x2, double ze, long double *psi, long double *d1,
                  long double *d2, long double *l, long double *dl) {
    const int p = mb.p, nt = mb.ntri;
    long double Pa[kMaxP + 1], dPa[kMaxP + 1], Pb[kMaxP + 1], dPb[kMaxP + 1], Pz[kMaxP + 1], dPz[kMaxP + 1];
    legendre_all(p, 2.0L * x1 - 1, Pa, dPa);
    legendre_all(p, 2.0L * x2 - 1, Pb, dPb);
    legendre_all(p, (long double)ze, Pz, dPz);
    for (int t = 0; t < nt; ++t) {
        long double v = 0, g1 = 0, g2 = 0;
        for (int m = 0; m < nt; ++m) {
            long double c = mb.Ctri[m * nt + t];
            v += c * Pa[mb.mi[m]] * Pb[mb.mj[m]];
            g1 += c * 2.0L * dPa[mb.mi[m]] * Pb[mb.mj[m]];
            g2 += c * 2.0L * Pa[mb.mi[m]] * dPb[mb.mj[m]];
        }
        psi[t] = v; d1[t] = g1; d2[t] = g2;
    }
    for (int k = 0; k <= p; ++k) {
        long double v = 0, g = 0;
        for (int m = 0; m <= p; ++m) {
            v += mb.Cline[m * (p + 1) + k] * Pz[m];
            g += mb.Cline[m * (p + 1) + k] * dPz[m];
        }
        l[k] = v; dl[k] = g;
    }
}

void eval_modal(const ModalBasis &mb, const double *xi, double *phi, double *dphi) {
    const int p = mb.p, nt = mb.ntri;
    long double psi[64], d1[64], d2[64], l[kMaxP + 1], dl[kMaxP + 1];
    eval_factors(mb, xi[0], xi[1], xi[2], psi, d1, d2, l, dl);
    for (int k = 0; k <= p; ++k)
        for (int t = 0; t < nt; ++t) {
            int a = k * nt + t;
            phi[a] = (double)(psi[t] * l[k]);
            dphi[3 * a + 0] = (double)(d1[t] * l[k]);
            dphi[3 * a + 1] = (double)(d2[t] * l[k]);
            dphi[3 * a + 2] = (double)(psi[t] * dl[k]);
        }
}

uint16_t to_bf16(float x) {              // round to nearest even
    uint32_t u;
    std::memcpy(&u, &x, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
float from_bf16(uint16_t h) {
    uint32_t u = (uint32_t)h << 16;
    float x;
    std::memcpy(&x, &u, 4);
    return x;
}
uint16_t to_f16(double x) {
    _Float16 h = (_Float16)(float)x;
    uint16_t u;
    std::memcpy(&u, &h, 2);
    return u;
}
double from_f16(uint16_t u) {
    _Float16 h;
    std::memcpy(&h, &u, 2);
    return (double)(float)h;
}

}  // namespace

void gauss_legendre_gw(int n, double *x, double *w) {
    if (n == 1) { x[0] = 0.0; w[0] = 2.0; return; }
    std::vector<long double> off(n - 1), xs, v0;
    for (int k = 1; k < n; ++k) off[k - 1] = k / std::sqrt(4.0L * k * k - 1.0L);
    tridiag_eigen(n, off, xs, v0);
    for (int i = 0; i < n; ++i) {
        x[i] = (double)xs[i];
        w[i] = (double)(2.0L * v0[i] * v0[i]);
    }
}

namespace {
// Fully symmetric triangle rules of degree 2p (p = 1..7; 3, 6, 12, 16, 25,
// 33, 42 points): orbit weights (summing to the triangle area 1/2) and
// barycentric parameters -- centroid weights; (w, a) of each 3-orbit
// (a, a, 1-2a); (w, a, b) of each 6-orbit (a, b, 1-a-b), a < b < 1-a-b.  They
// solve the moment equations sum_q w_q xi1^i xi2^j = i! j! / (i+j+2)!
// (i + j <= 2p), polished in 50-digit arithmetic; every weight is positive and
// every point interior.  For p <= 4 these are the classical rules; above, the
// equations have several such solutions and these are the ones taken.
// p = 1: 0 centroid, 1 3-orbits, 0 6-orbits
const long double sym1_s3[] = {
    0.166666666666666666667L, 0.166666666666666666667L};
// p = 2: 0 centroid, 2 3-orbits, 0 6-orbits
const long double sym2_s3[] = {
    0.0549758718276609338192L, 0.0915762135097707434596L,
    0.111690794839005732848L, 0.445948490915964886318L};
// p = 3: 0 centroid, 2 3-orbits, 1 6-orbits
const long double sym3_s3[] = {
    0.0254224531851034084605L, 0.0630890144915022283403L,
    0.0583931378631896830126L, 0.249286745170910421292L};
const long double sym3_s6[] = {
    0.0414255378091867875968L, 0.0531450498448169473532L, 0.310352451033784405417L};
// p = 4: 1 centroid, 3 3-orbits, 1 6-orbits
const long double sym4_c[] = {0.0721578038388935841255L};
const long double sym4_s3[] = {
    0.0162292488115990401555L, 0.0505472283170309754584L,
    0.0516086852673591251409L, 0.170569307751760206622L,
    0.0475458171336423123969L, 0.459292588292723156029L};
const long double sym4_s6[] = {
    0.0136151570872174971324L, 0.00839477740995760533721L, 0.263112829634638113422L};
// p = 5: 1 centroid, 2 3-orbits, 3 6-orbits
const long double sym5_c[] = {0.0399472523706198539156L};
const long double sym5_s3[] = {
    0.00411190934523209775932L, 0.0233088675100001907145L,
    0.0355619011161886673196L, 0.42508621060209057297L};
const long double sym5_s6[] = {
    0.0186799281171526384131L, 0.0299460319541708865031L, 0.358740141864431464578L,
    0.0154433284422819943913L, 0.0356325595875034813206L, 0.143295370426867145306L,
    0.0227152961480850090035L, 0.147925626209534437353L, 0.223766973576973006226L};
// p = 6: 0 centroid, 5 3-orbits, 3 6-orbits
const long double sym6_s3[] = {
    0.00396582125498681922966L, 0.0246463634363355947667L,
    0.0142430260344387724998L, 0.109257827659354290584L,
    0.0312706065979513802347L, 0.271462507014926084878L,
    0.0249591674640304710595L, 0.440111648658593111013L,
    0.0121334190407260165754L, 0.488203750945541551778L};
const long double sym6_s6[] = {
    0.00754183878825571929293L, 0.0213824902561705895942L, 0.127279717233589368788L,
    0.0108917925193037789663L, 0.0230341563552671394816L, 0.291655679738340960534L,
    0.0216136818297071052746L, 0.116296019677926586631L, 0.255454228638517346531L};
// p = 7: 0 centroid, 6 3-orbits, 4 6-orbits
const long double sym7_s3[] = {
    0.00246170180120004084091L, 0.0193909612487010481783L,
    0.00721684983488833380085L, 0.0617998830908726012675L,
    0.0210812943684965087691L, 0.177205532412543436957L,
    0.0258870522536457931574L, 0.273477528308838659755L,
    0.0163941767720626753207L, 0.417644719340453922509L,
    0.0109417906847144453204L, 0.488963910362178638677L};
const long double sym7_s6[] = {
    0.00250511441925033588493L, 0.00126833093287202508725L, 0.118974497696956845398L,
    0.00721815405676692024804L, 0.0146469500556544096705L, 0.298372882136257752971L,
    0.0123328766062818369814L, 0.0571247574036479390357L, 0.172266687821355578375L,
    0.0192857553935303416142L, 0.0929162493569718247582L, 0.336861459796345001744L};

struct SymOrbits {
    int n0, n1, n2;
    const long double *c, *s3, *s6;
};

SymOrbits sym_orbits(int p) {
    switch (p) {
    case 1: return {0, 1, 0, nullptr, sym1_s3, nullptr};
    case 2: return {0, 2, 0, nullptr, sym2_s3, nullptr};
    case 3: return {0, 2, 1, nullptr, sym3_s3, sym3_s6};
    case 4: return {1, 3, 1, sym4_c, sym4_s3, sym4_s6};
    case 5: return {1, 2, 3, sym5_c, sym5_s3, sym5_s6};
    case 6: return {0, 5, 3, nullptr, sym6_s3, sym6_s6};
    case 7: return {0, 6, 4, nullptr, sym7_s3, sym7_s6};
    }
    throw std::runtime_error("degree out of range");
}
}  // namespace

void symmetric_triangle_rule(int p, std::vector<double> &xi1, std::vector<double> &xi2, std::vector<double> &w) {
    const SymOrbits o = sym_orbits(p);
    xi1.clear(); xi2.clear(); w.clear();
    // barycentric (l0, l1, l2) -> (xi1, xi2) = (l1, l2)
    auto put = [&](long double wt, long double l1, long double l2) {
        xi1.push_back((double)l1); xi2.push_back((double)l2); w.push_back((double)wt);
    };
    for (int i = 0; i < o.n0; ++i) put(o.c[i], 1.0L / 3, 1.0L / 3);
    for (int i = 0; i < o.n1; ++i) {
        const long double wt = o.s3[2 * i], a = o.s3[2 * i + 1], c = 1.0L - 2 * a;
        put(wt, a, c);        // (a, a, c)
        put(wt, c, a);        // (a, c, a)
        put(wt, a, a);        // (c, a, a)
    }
    for (int i = 0; i < o.n2; ++i) {
        const long double wt = o.s6[3 * i], a = o.s6[3 * i + 1], b = o.s6[3 * i + 2], c = 1.0L - a - b;
        put(wt, b, c);        // (a, b, c)
        put(wt, c, b);        // (a, c, b)
        put(wt, a, c);        // (b, a, c)
        put(wt, c, a);        // (b, c, a)
        put(wt, a, b);        // (c, a, b)
        put(wt, b, a);        // (c, b, a)
    }
}

void gauss_lobatto_nodes(int p, double *x) {
    x[0] = -1.0;
    x[p] = 1.0;
    if (p < 2) return;
    int m = p - 1;   // roots of P_p' = roots of the Jacobi(1,1) polynomial of degree p-1
    if (m == 1) { x[1] = 0.0; return; }
    std::vector<long double> off(m - 1), xs, v0;
    for (int k = 1; k < m; ++k) off[k - 1] = std::sqrt((long double)k * (k + 2) / ((2.0L * k + 1) * (2.0L * k + 3)));
    tridiag_eigen(m, off, xs, v0);
    for (int i = 0; i < m; ++i) x[i + 1] = (double)xs[i];
}

void lagrange_prism_eval(int p, const double *xi, double *phi, double *dphi) {
    ModalBasis mb = make_modal(p);
    eval_modal(mb, xi, phi, dphi);
}

// Every layout the kernels read, derived from B64 (and nq, nqp, npad).
static void derive_layouts(HostTables &T) {
    const int np = T.npad;
    T.BT64.assign(T.B64.size(), 0.0);
    T.BT32.assign(T.B64.size(), 0.0f);
    for (int q = 0; q < T.nqp; ++q)
        for (int r = 0; r < 4; ++r)
            for (int a = 0; a < np; ++a) {
                const double v = T.B64[((size_t)q * 4 + r) * np + a];
                T.BT64[(size_t)a * T.nqp * 4 + q * 4 + r] = v;
                T.BT32[(size_t)a * T.nqp * 4 + q * 4 + r] = (float)v;
            }
    T.Bc32.assign(T.B64.size(), 0.0f);
    for (int q = 0; q < T.nqp; ++q)
        for (int a = 0; a < np; ++a)
            for (int r = 0; r < 4; ++r)
                T.Bc32[((size_t)q * np + a) * 4 + r] = (float)T.B64[((size_t)q * 4 + r) * np + a];
    T.B32.resize(T.B64.size());
    double bmax = 0.0;
    for (size_t i = 0; i < T.B64.size(); ++i) {
        T.B32[i] = (float)T.B64[i];
        bmax = std::fmax(bmax, std::fabs(T.B64[i]));
    }
    // fp16 tables are scaled so that max |B| lies in [2^13, 2^14)
    T.f16_shift = 13 - (int)std::floor(std::log2(bmax));
    const double fs = std::ldexp(1.0, T.f16_shift);
    const size_t nsplit = (size_t)T.nkb * np * 32;
    const int ntile = np / 16;
    T.bf_hi.assign(nsplit, 0); T.bf_lo.assign(nsplit, 0);
    T.hf_hi.assign(nsplit, 0); T.hf_lo.assign(nsplit, 0);
    T.Ycf.assign(nsplit, 0.0f);
    for (int kb = 0; kb < T.nkb; ++kb)
        for (int a = 0; a < np; ++a)
            for (int k = 0; k < 32; ++k) {
                const int q = kb * 8 + k / 4, r = k % 4;
                const double x = T.B64[((size_t)q * 4 + r) * np + a];
                const int lane = a % 16 + 16 * (k / 8);
                const size_t o = (((size_t)kb * ntile + a / 16) * 64 + lane) * 8 + k % 8;
                const uint16_t h = to_bf16((float)x);
                T.bf_hi[o] = h;
                T.bf_lo[o] = to_bf16((float)(x - (double)from_bf16(h)));
                const double xs = x * fs;
                const uint16_t hh = to_f16(xs);
                T.hf_hi[o] = hh;
                T.hf_lo[o] = to_f16(xs - from_f16(hh));
                // the same (point, row, column) as a B-fragment column value
                T.Ycf[o] = (float)x;
            }
}

void rule_points(int p, int rule, std::vector<double> &qw) {
    if (p < 1 || p > kMaxP) throw std::runtime_error("degree out of range");
    if (rule != 0 && rule != 1) throw std::runtime_error("unknown quadrature rule");
    const int n1 = p + 1;
    double g[kMaxP + 1], gw[kMaxP + 1];
    gauss_legendre_gw(n1, g, gw);
    qw.assign((size_t)nq_rule_of(p, rule) * 4, 0.0);
    if (rule == 0) {
        for (int k = 0; k < n1; ++k)
            for (int j = 0; j < n1; ++j)
                for (int i = 0; i < n1; ++i) {
                    int q = (k * n1 + j) * n1 + i;
                    qw[4 * q + 0] = (1.0 + g[i]) * (1.0 - g[j]) / 4.0;
                    qw[4 * q + 1] = (1.0 + g[j]) / 2.0;
                    qw[4 * q + 2] = g[k];
                    qw[4 * q + 3] = gw[i] * gw[j] * gw[k] * (1.0 - g[j]) / 8.0;
                }
    } else {              // symmetric triangle rule x Gauss in zeta, q = k * ntri + t
        std::vector<double> x1, x2, wt;
        symmetric_triangle_rule(p, x1, x2, wt);
        const int nt = (int)wt.size();
        for (int k = 0; k < n1; ++k)
            for (int t = 0; t < nt; ++t) {
                const int q = k * nt + t;
                qw[4 * q + 0] = x1[t];
                qw[4 * q + 1] = x2[t];
                qw[4 * q + 2] = g[k];
                qw[4 * q + 3] = wt[t] * gw[k];
            }
    }
}

HostTables build_tables(int p, int rule) {
    if (p < 1 || p > kMaxP) throw std::runtime_error("degree out of range");
    if (rule != 0 && rule != 1) throw std::runtime_error("unknown quadrature rule");
    HostTables T;
    T.p = p;
    T.rule = rule;
    T.n = nshp_of(p);
    T.npad = pad16(T.n);
    T.nq = nq_rule_of(p, rule);
    T.nqp = pad8(T.nq);
    T.nkb = T.nqp / 8;
    const int n = T.n, np = T.npad;
    rule_points(p, rule, T.qw);
    T.qw.resize((size_t)T.nqp * 4, 0.0);
    for (int q = T.nq; q < T.nqp; ++q) {      // padding points: centroid, zero weight
        T.qw[4 * q + 0] = 1.0 / 3.0;
        T.qw[4 * q + 1] = 1.0 / 3.0;
    }
    // line factors of the kernels that compute shape functions at each point
    T.gll.assign(2 * (p + 1), 0.0);
    gauss_lobatto_nodes(p, T.gll.data());
    for (int k = 0; k <= p; ++k) {
        long double d = 1.0L;
        for (int m = 0; m <= p; ++m)
            if (m != k) d *= (long double)T.gll[k] - (long double)T.gll[m];
        T.gll[p + 1 + k] = (double)(1.0L / d);
    }
    ModalBasis mb = make_modal(p);
    T.B64.assign((size_t)T.nqp * 4 * np, 0.0);
    std::vector<double> phi(n), dphi(3 * n);
    for (int q = 0; q < T.nq; ++q) {
        eval_modal(mb, &T.qw[4 * q], phi.data(), dphi.data());
        for (int a = 0; a < n; ++a) {
            T.B64[((size_t)q * 4 + 0) * np + a] = phi[a];
            for (int r = 0; r < 3; ++r) T.B64[((size_t)q * 4 + 1 + r) * np + a] = dphi[3 * a + r];
        }
    }
    derive_layouts(T);
    // tensor factors for the kernels that contract per triangle point: both
    // prism rules are products of nij triangle points and p+1 points in zeta
    // with q = m nij + ij, so B_q[r][(k,t)] = tau_r(t, ij) lam_r(k, m) with
    // tau = (T, dT/dxi1, dT/dxi2, T) and lam = (L, L, L, dL/dzeta)
    const int nk = p + 1, nt = ntri_of(p);
    T.nk = nk;
    T.nij = T.nq / nk;
    T.tpad = pad16(nt);
    T.tau64.assign((size_t)T.nij * 4 * T.tpad, 0.0);
    T.lam.assign((size_t)4 * nk * nk, 0.0);
    {
        long double psi[64], d1[64], d2[64], l[kMaxP + 1], dl[kMaxP + 1];
        for (int ij = 0; ij < T.nij; ++ij) {
            eval_factors(mb, T.qw[4 * ij + 0], T.qw[4 * ij + 1], 0.0, psi, d1, d2, l, dl);
            for (int t = 0; t < nt; ++t) {
                T.tau64[((size_t)ij * 4 + 0) * T.tpad + t] = (double)psi[t];
                T.tau64[((size_t)ij * 4 + 1) * T.tpad + t] = (double)d1[t];
                T.tau64[((size_t)ij * 4 + 2) * T.tpad + t] = (double)d2[t];
                T.tau64[((size_t)ij * 4 + 3) * T.tpad + t] = (double)psi[t];
            }
        }
        for (int m = 0; m < nk; ++m) {
            eval_factors(mb, 1.0 / 3.0, 1.0 / 3.0, T.qw[4 * ((size_t)m * T.nij) + 2], psi, d1, d2, l, dl);
            for (int k = 0; k < nk; ++k) {
                for (int r = 0; r < 3; ++r) T.lam[((size_t)r * nk + k) * nk + m] = (double)l[k];
                T.lam[((size_t)3 * nk + k) * nk + m] = (double)dl[k];
            }
        }
    }
    T.tau32.assign(T.tau64.begin(), T.tau64.end());
    T.lam32.assign(T.lam.begin(), T.lam.end());
    {
        const int nch = (T.nij + 7) / 8, tt = T.tpad / 16;
        T.taub_hi.assign((size_t)nch * tt * 64 * 8, 0);
        T.taub_lo.assign((size_t)nch * tt * 64 * 8, 0);
        T.tauh_hi.assign((size_t)nch * tt * 64 * 8, 0);
        T.tauh_lo.assign((size_t)nch * tt * 64 * 8, 0);
        double tmax = 0.0;
        for (double v : T.tau64) tmax = std::fmax(tmax, std::fabs(v));
        T.tau_f16_shift = tmax > 0.0 ? 13 - (int)std::floor(std::log2(tmax)) : 0;
        const double ts = std::ldexp(1.0, T.tau_f16_shift);
        // |Z| = |sum_s tau_s G[r][s]| <= max|tau| sum_s sum_m |lam_r(k,m) lam_s(k',m)| |W_m[r][s]|
        //     <= 4 max|tau| max_{r,s,k,k'} sum_m |lam_r(k,m) lam_s(k',m)| max|W|
        double lr = 0.0, l0 = 0.0;
        for (int r = 0; r < 4; ++r)
            for (int q = 0; q < 4; ++q)
                for (int k = 0; k < nk; ++k)
                    for (int kp = 0; kp < nk; ++kp) {
                        double a = 0.0;
                        for (int m = 0; m < nk; ++m)
                            a += std::fabs(T.lam[((size_t)r * nk + k) * nk + m] * T.lam[((size_t)q * nk + kp) * nk + m]);
                        lr = std::fmax(lr, a);
                    }
        for (int k = 0; k < nk; ++k) {
            double a = 0.0;
            for (int m = 0; m < nk; ++m) a += std::fabs(T.lam[(size_t)k * nk + m]);
            l0 = std::fmax(l0, a);
        }
        T.f16_zc = 4.0 * tmax * lr;
        T.f16_zb = l0;
        for (int c = 0; c < nch; ++c)
            for (int ti = 0; ti < tt; ++ti)
                for (int l = 0; l < 64; ++l)
                    for (int v = 0; v < 8; ++v) {
                        const int ij = 8 * c + 2 * (l / 16) + v / 4, r = v % 4, t = 16 * ti + l % 16;
                        if (ij >= T.nij) continue;
                        const double x = T.tau64[((size_t)ij * 4 + r) * T.tpad + t];
                        const size_t o = (((size_t)c * tt + ti) * 64 + l) * 8 + v;
                        const uint16_t h = to_bf16((float)x);
                        T.taub_hi[o] = h;
                        T.taub_lo[o] = to_bf16((float)(x - (double)from_bf16(h)));
                        const double xs = x * ts;
                        const uint16_t hh = to_f16(xs);
                        T.tauh_hi[o] = hh;
                        T.tauh_lo[o] = to_f16(xs - from_f16(hh));
                    }
    }
    return T;
}

HostTables build_hex_tables(int p) {
    if (p < 1 || p > kMaxP) throw std::runtime_error("degree out of range");
    HostTables T;
    T.p = p;
    T.rule = 0;
    const int n1 = p + 1;
    T.n = n1 * n1 * n1;
    T.npad = pad16(T.n);
    T.nq = n1 * n1 * n1;
    T.nqp = pad8(T.nq);
    T.nkb = T.nqp / 8;
    double g[kMaxP + 1], gw[kMaxP + 1];
    gauss_legendre_gw(n1, g, gw);
    T.qw.assign((size_t)T.nqp * 4, 0.0);
    for (int k = 0; k < n1; ++k)
        for (int j = 0; j < n1; ++j)
            for (int i = 0; i < n1; ++i) {
                const int q = (k * n1 + j) * n1 + i;
                T.qw[4 * q + 0] = g[i];
                T.qw[4 * q + 1] = g[j];
                T.qw[4 * q + 2] = g[k];
                T.qw[4 * q + 3] = gw[i] * gw[j] * gw[k];
            }
    // (padding points: reference centre, zero weight -- already zero)
    T.gll.assign(2 * n1, 0.0);
    gauss_lobatto_nodes(p, T.gll.data());
    // 1D Lagrange basis on the Gauss-Lobatto nodes as Legendre combinations:
    // C = V^{-1}, V[i][m] = P_m(z_i); L_k = sum_m C[m][k] P_m
    std::vector<long double> V((size_t)n1 * n1);
    long double P[kMaxP + 1], dP[kMaxP + 1];
    for (int i = 0; i < n1; ++i) {
        legendre_all(p, (long double)T.gll[i], P, dP);
        for (int m = 0; m < n1; ++m) V[i * n1 + m] = P[m];
    }
    const std::vector<long double> C = invert(n1, V);
    auto line = [&](double x, double *l, double *dl) {
        legendre_all(p, (long double)x, P, dP);
        for (int k = 0; k < n1; ++k) {
            long double v = 0, d = 0;
            for (int m = 0; m < n1; ++m) {
                v += C[m * n1 + k] * P[m];
                d += C[m * n1 + k] * dP[m];
            }
            l[k] = (double)v;
            dl[k] = (double)d;
        }
    };
    const int np = T.npad;
    T.B64.assign((size_t)T.nqp * 4 * np, 0.0);
    double lx[kMaxP + 1], dlx[kMaxP + 1], ly[kMaxP + 1], dly[kMaxP + 1], lz[kMaxP + 1], dlz[kMaxP + 1];
    for (int q = 0; q < T.nq; ++q) {
        line(T.qw[4 * q + 0], lx, dlx);
        line(T.qw[4 * q + 1], ly, dly);
        line(T.qw[4 * q + 2], lz, dlz);
        for (int k = 0; k < n1; ++k)
            for (int j = 0; j < n1; ++j)
                for (int i = 0; i < n1; ++i) {
                    const int a = (k * n1 + j) * n1 + i;
                    T.B64[((size_t)q * 4 + 0) * np + a] = lx[i] * ly[j] * lz[k];
                    T.B64[((size_t)q * 4 + 1) * np + a] = dlx[i] * ly[j] * lz[k];
                    T.B64[((size_t)q * 4 + 2) * np + a] = lx[i] * dly[j] * lz[k];
                    T.B64[((size_t)q * 4 + 3) * np + a] = lx[i] * ly[j] * dlz[k];
                }
    }
    derive_layouts(T);
    // tensor factors for the kernels that contract per plane point: q = m nij + ij with
    // ij = j n1 + i, a = k nt + t with t = j' n1 + i', so B_q[r][(k,t)] = tau_r(t, ij)
    // lam_r(k, m) with tau = (l_i' l_j', l_i'' l_j', l_i' l_j'', l_i' l_j') at (x_i, y_j) and
    // lam = (l_k, l_k, l_k, l_k') at z_m
    const int nt = n1 * n1;
    T.nk = n1;
    T.nij = nt;
    T.tpad = pad16(nt);
    T.tau64.assign((size_t)T.nij * 4 * T.tpad, 0.0);
    T.lam.assign((size_t)4 * n1 * n1, 0.0);
    for (int j = 0; j < n1; ++j)
        for (int i = 0; i < n1; ++i) {
            line(g[i], lx, dlx);
            line(g[j], ly, dly);
            const size_t ij = (size_t)j * n1 + i;
            for (int jj = 0; jj < n1; ++jj)
                for (int ii = 0; ii < n1; ++ii) {
                    const int t = jj * n1 + ii;
                    T.tau64[(ij * 4 + 0) * T.tpad + t] = lx[ii] * ly[jj];
                    T.tau64[(ij * 4 + 1) * T.tpad + t] = dlx[ii] * ly[jj];
                    T.tau64[(ij * 4 + 2) * T.tpad + t] = lx[ii] * dly[jj];
                    T.tau64[(ij * 4 + 3) * T.tpad + t] = lx[ii] * ly[jj];
                }
        }
    for (int m = 0; m < n1; ++m) {
        line(g[m], lz, dlz);
        for (int k = 0; k < n1; ++k) {
            for (int r = 0; r < 3; ++r) T.lam[((size_t)r * n1 + k) * n1 + m] = lz[k];
            T.lam[((size_t)3 * n1 + k) * n1 + m] = dlz[k];
        }
    }
    T.tau32.assign(T.tau64.begin(), T.tau64.end());
    T.lam32.assign(T.lam.begin(), T.lam.end());
    return T;
}

HostTables build_tet_tables(int p) {
    if (p < 1 || p > kMaxP) throw std::runtime_error("degree out of range");
    HostTables T;
    T.p = p;
    T.rule = 0;
    const int n1 = p + 2;
    T.n = (p + 1) * (p + 2) * (p + 3) / 6;
    T.npad = pad16(T.n);
    T.nq = n1 * n1 * n1;
    T.nqp = pad8(T.nq);
    T.nkb = T.nqp / 8;
    double g[kMaxP + 2], gw[kMaxP + 2];
    gauss_legendre_gw(n1, g, gw);
    T.qw.assign((size_t)T.nqp * 4, 0.0);
    for (int q = T.nq; q < T.nqp; ++q)        // padding points: inside, zero weight
        T.qw[4 * q + 0] = T.qw[4 * q + 1] = T.qw[4 * q + 2] = 0.25;
    // Duffy collapse of the cube onto the tetrahedron: zeta = (1+c)/2,
    // eta = (1+b)(1-zeta)/2, xi = (1+a)(1-eta-zeta)/2; |dx/d(a,b,c)| =
    // (1-b)(1-c)^2/64
    for (int k = 0; k < n1; ++k)
        for (int j = 0; j < n1; ++j)
            for (int i = 0; i < n1; ++i) {
                const int q = (k * n1 + j) * n1 + i;
                const double ze = 0.5 * (1.0 + g[k]);
                const double et = 0.5 * (1.0 + g[j]) * (1.0 - ze);
                const double xi = 0.5 * (1.0 + g[i]) * (1.0 - et - ze);
                T.qw[4 * q + 0] = xi;
                T.qw[4 * q + 1] = et;
                T.qw[4 * q + 2] = ze;
                T.qw[4 * q + 3] = gw[i] * gw[j] * gw[k] * (1.0 - g[j]) * (1.0 - g[k]) * (1.0 - g[k]) / 64.0;
            }
    T.gll.assign(2 * (p + 1), 0.0);
    // Lagrange basis on the lattice (i/p, j/p, k/p), k outer, j, i inner, as
    // combinations of the modes P_a(2 xi - 1) P_b(2 eta - 1) P_c(2 zeta - 1),
    // a + b + c <= p: C = V^{-1}, V[node][mode]
    const int n = T.n;
    std::vector<int> ma, mb, mc;
    for (int c = 0; c <= p; ++c)
        for (int b = 0; b + c <= p; ++b)
            for (int a = 0; a + b + c <= p; ++a) { ma.push_back(a); mb.push_back(b); mc.push_back(c); }
    long double P0[kMaxP + 1], dP0[kMaxP + 1], P1[kMaxP + 1], dP1[kMaxP + 1], P2[kMaxP + 1], dP2[kMaxP + 1];
    std::vector<long double> V((size_t)n * n);
    int node = 0;
    for (int k = 0; k <= p; ++k)
        for (int j = 0; j + k <= p; ++j)
            for (int i = 0; i + j + k <= p; ++i, ++node) {
                legendre_all(p, 2.0L * i / p - 1, P0, dP0);
                legendre_all(p, 2.0L * j / p - 1, P1, dP1);
                legendre_all(p, 2.0L * k / p - 1, P2, dP2);
                for (int m = 0; m < n; ++m) V[(size_t)node * n + m] = P0[ma[m]] * P1[mb[m]] * P2[mc[m]];
            }
    const std::vector<long double> C = invert(n, V);
    const int np = T.npad;
    T.B64.assign((size_t)T.nqp * 4 * np, 0.0);
    std::vector<long double> Bx((size_t)T.nq * 4 * n);    // the basis rows in extended precision
    std::vector<long double> md(n), m0(n), m1(n), m2(n);
    for (int q = 0; q < T.nq; ++q) {
        legendre_all(p, 2.0L * T.qw[4 * q + 0] - 1, P0, dP0);
        legendre_all(p, 2.0L * T.qw[4 * q + 1] - 1, P1, dP1);
        legendre_all(p, 2.0L * T.qw[4 * q + 2] - 1, P2, dP2);
        for (int m = 0; m < n; ++m) {
            md[m] = P0[ma[m]] * P1[mb[m]] * P2[mc[m]];
            m0[m] = 2 * dP0[ma[m]] * P1[mb[m]] * P2[mc[m]];
            m1[m] = 2 * P0[ma[m]] * dP1[mb[m]] * P2[mc[m]];
            m2[m] = 2 * P0[ma[m]] * P1[mb[m]] * dP2[mc[m]];
        }
        for (int a = 0; a < n; ++a) {
            long double v = 0, d0 = 0, d1 = 0, d2 = 0;
            for (int m = 0; m < n; ++m) {
                const long double cm = C[(size_t)m * n + a];
                v += cm * md[m];
                d0 += cm * m0[m];
                d1 += cm * m1[m];
                d2 += cm * m2[m];
            }
            T.B64[((size_t)q * 4 + 0) * np + a] = (double)v;
            T.B64[((size_t)q * 4 + 1) * np + a] = (double)d0;
            T.B64[((size_t)q * 4 + 2) * np + a] = (double)d1;
            T.B64[((size_t)q * 4 + 3) * np + a] = (double)d2;
            Bx[((size_t)q * 4 + 0) * n + a] = v;
            Bx[((size_t)q * 4 + 1) * n + a] = d0;
            Bx[((size_t)q * 4 + 2) * n + a] = d1;
            Bx[((size_t)q * 4 + 3) * n + a] = d2;
        }
    }
    derive_layouts(T);
    // reference matrices of the 13 nonzero entries of W (row r of B for the test
    // function a, row s for b), and the reference load vector
    static const int rs[13][2] = {{0, 0}, {0, 1}, {0, 2}, {0, 3}, {1, 1}, {1, 2}, {1, 3},
                                  {2, 1}, {2, 2}, {2, 3}, {3, 1}, {3, 2}, {3, 3}};
    const size_t n2p = ((size_t)n * n + 15) / 16 * 16;    // entries padded to whole blocks of 16 (zero)
    T.Mref.assign(n2p * 16 + n, 0.0);
    std::vector<long double> acc((size_t)13 * n * n, 0.0L), b0(n, 0.0L);
    for (int q = 0; q < T.nq; ++q) {
        const long double w = T.qw[4 * q + 3];
        const long double *Bq = &Bx[(size_t)q * 4 * n];
        for (int a = 0; a < n; ++a) {
            b0[a] += w * Bq[a];
            for (int k = 0; k < 13; ++k) {
                const long double wa = w * Bq[rs[k][0] * n + a];
                long double *row = &acc[((size_t)k * n + a) * n];
                const long double *bs = Bq + rs[k][1] * n;
                for (int b = 0; b < n; ++b) row[b] += wa * bs[b];
            }
        }
    }
    for (int a = 0; a < n; ++a) {
        for (int b = 0; b < n; ++b)
            for (int k = 0; k < 13; ++k) T.Mref[(size_t)k * n2p + (size_t)a * n + b] = (double)acc[((size_t)k * n + a) * n + b];
        T.Mref[n2p * 16 + a] = (double)b0[a];
    }
    T.Mref32.assign(T.Mref.begin(), T.Mref.end());
    return T;
}

}  // namespace feint
