// The 1D factors of the tensor-product hexahedral basis, evaluated at compile
// time for one degree: l_k and l_k' of the Lagrange polynomials on the p+1
// Gauss-Lobatto nodes, at the p+1 Gauss-Legendre points, both in ascending
// order as in the library's tables.  Kernels that index them with
// compile-time constants get them as instruction literals (no memory reads).
// Nodes by Newton's method on the Legendre recurrence: the Gauss points are
// the roots of P_n, the interior Gauss-Lobatto nodes those of P_p'.
#pragma once

namespace feint {
namespace hexc {

constexpr double kPi = 3.14159265358979323846;

constexpr double cabs(double x) { return x < 0 ? -x : x; }

// cos on [0, pi] by its Taylor series (only the starting guesses need it)
constexpr double ccos(double x) {
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 40; ++k) {
        term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
        sum += term;
    }
    return sum;
}

// P_n(x) and P_n'(x) for |x| < 1
constexpr void legendre(int n, double x, double &P, double &dP) {
    double p0 = 1.0, p1 = x;
    if (n == 0) { P = 1.0; dP = 0.0; return; }
    for (int k = 1; k < n; ++k) {
        const double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
        p0 = p1;
        p1 = p2;
    }
    P = p1;
    dP = n * (x * p1 - p0) / (x * x - 1.0);
}

// i-th Gauss-Legendre point of n, ascending
constexpr double gauss_point(int n, int i) {
    double x = -ccos(kPi * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
        double P = 0.0, dP = 0.0;
        legendre(n, x, P, dP);
        const double dx = P / dP;
        x -= dx;
        if (cabs(dx) < 1e-17) break;
    }
    return x;
}

// i-th Gauss-Lobatto node of degree p (p+1 nodes), ascending
constexpr double lobatto_node(int p, int i) {
    if (i == 0) return -1.0;
    if (i == p) return 1.0;
    double x = -ccos(kPi * i / p);
    for (int it = 0; it < 100; ++it) {
        double P = 0.0, dP = 0.0;
        legendre(p, x, P, dP);
        const double d2P = (2.0 * x * dP - p * (p + 1.0) * P) / (1.0 - x * x);   // Legendre's equation
        const double dx = dP / d2P;
        x -= dx;
        if (cabs(dx) < 1e-17) break;
    }
    return x;
}

template <int P>
struct Factors {
    static constexpr int n = P + 1;
    double L[n][n];   // [k][m] = l_k(g_m)
    double D[n][n];   // [k][m] = l_k'(g_m)
};

template <int P>
constexpr Factors<P> make_factors() {
    constexpr int n = P + 1;
    Factors<P> F{};
    double z[n] = {}, g[n] = {};
    for (int i = 0; i < n; ++i) {
        z[i] = lobatto_node(P, i);
        g[i] = gauss_point(n, i);
    }
    for (int k = 0; k < n; ++k)
        for (int m = 0; m < n; ++m) {
            const double x = g[m];
            double l = 1.0, d = 0.0;
            for (int j = 0; j < n; ++j) {
                if (j == k) continue;
                l *= (x - z[j]) / (z[k] - z[j]);
                double t = 1.0 / (z[k] - z[j]);
                for (int r = 0; r < n; ++r)
                    if (r != k && r != j) t *= (x - z[r]) / (z[k] - z[r]);
                d += t;
            }
            F.L[k][m] = l;
            F.D[k][m] = d;
        }
    return F;
}

template <int P>
struct Fac {
    static constexpr Factors<P> v = make_factors<P>();
};

// The same values point-major ([m][k]), so that the factors of every k at one
// point are contiguous.
template <int P>
constexpr Factors<P> make_factors_t() {
    constexpr int n = P + 1;
    const Factors<P> F = make_factors<P>();
    Factors<P> T{};
    for (int k = 0; k < n; ++k)
        for (int m = 0; m < n; ++m) {
            T.L[m][k] = F.L[k][m];
            T.D[m][k] = F.D[k][m];
        }
    return T;
}

template <int P>
struct FacT {
    static constexpr Factors<P> v = make_factors_t<P>();
};

}  // namespace hexc
}  // namespace feint
