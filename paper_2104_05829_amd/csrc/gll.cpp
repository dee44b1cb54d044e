// Reference element of the library (NekRS paper Sec. 2.3): Gauss--Lobatto--
// Legendre nodes and weights and the differentiation matrix Dh, on the host.
//
// Interior GLL nodes are the zeros of (1 - x^2) P_N'(x), which is a multiple
// of x P_N(x) - P_{N-1}(x); they are found by Newton's method on
// q(x) = x P_N(x) - P_{N-1}(x), started from the Chebyshev--Gauss--Lobatto
// points.  Weights 2 / (N (N+1) P_N(x_j)^2).  Dh from barycentric weights
// lambda_j = 1 / prod_{m != j} (x_j - x_m):  Dh[i][j] = (lambda_j / lambda_i) /
// (x_i - x_j) for i != j, and the diagonal such that every row sums to zero
// (Dh applied to a constant vanishes).
#include <cmath>

#include "sem_internal.h"

namespace semx {

namespace {
// P_n and P_{n-1} and their derivatives at x (n >= 1)
void legendre_pair(int n, double x, double &pn, double &pn1, double &dpn, double &dpn1)
{
    double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
    for (int m = 2; m <= n; ++m) {
        const double p2 = ((2 * m - 1) * x * p1 - (m - 1) * p0) / m;
        // derivative of the recurrence: m P_m' = (2m-1)(P_{m-1} + x P_{m-1}') - (m-1) P_{m-2}'
        const double d2 = ((2 * m - 1) * (p1 + x * d1) - (m - 1) * d0) / m;
        p0 = p1; p1 = p2;
        d0 = d1; d1 = d2;
    }
    pn = p1; pn1 = p0; dpn = d1; dpn1 = d0;
}
}  // namespace

int host_gll(int N, double *xi, double *rho, double *D)
{
    if (N < 1 || N > kMaxN) return SEM_EINVAL;
    const int nq = N + 1;
    double x[kMaxN + 1];
    x[0] = -1.0;
    x[N] = 1.0;
    for (int j = 1; j < N; ++j) {
        double t = std::cos(M_PI * (double)(N - j) / (double)N);  // ascending start points
        for (int it = 0; it < 60; ++it) {
            double pn, pn1, dpn, dpn1;
            legendre_pair(N, t, pn, pn1, dpn, dpn1);
            const double q = t * pn - pn1;
            const double dq = pn + t * dpn - dpn1;
            const double step = q / dq;
            t -= step;
            if (std::fabs(step) <= 1e-16 * (1.0 + std::fabs(t))) break;
        }
        x[j] = t;
    }
    // the rule is symmetric: average each node with its mirror image
    for (int j = 0; j < nq / 2; ++j) {
        const double a = 0.5 * (x[N - j] - x[j]);
        x[j] = -a;
        x[N - j] = a;
    }
    if (N % 2 == 0) x[N / 2] = 0.0;
    if (xi)
        for (int j = 0; j < nq; ++j) xi[j] = x[j];
    if (rho)
        for (int j = 0; j < nq; ++j) {
            double pn, pn1, dpn, dpn1;
            legendre_pair(N, x[j], pn, pn1, dpn, dpn1);
            rho[j] = 2.0 / ((double)N * (N + 1) * pn * pn);
        }
    if (D) {
        double lam[kMaxN + 1];
        for (int j = 0; j < nq; ++j) {
            double prod = 1.0;
            for (int m = 0; m < nq; ++m)
                if (m != j) prod *= (x[j] - x[m]);
            lam[j] = 1.0 / prod;
        }
        for (int i = 0; i < nq; ++i) {
            double rowsum = 0.0;
            for (int j = 0; j < nq; ++j) {
                if (j == i) continue;
                const double v = (lam[j] / lam[i]) / (x[i] - x[j]);
                D[i * nq + j] = v;
                rowsum += v;
            }
            D[i * nq + i] = -rowsum;
        }
    }
    return SEM_OK;
}

// Lagrange interpolation matrix J[i][a] = h_a(xt_i) for the cardinal basis on
// the source nodes xs (barycentric form; exact unit rows at coincident points).
void host_interp(int ns, const double *xs, int nt, const double *xt, double *J)
{
    double lam[kMaxN + 1];
    for (int a = 0; a < ns; ++a) {
        double prod = 1.0;
        for (int m = 0; m < ns; ++m)
            if (m != a) prod *= (xs[a] - xs[m]);
        lam[a] = 1.0 / prod;
    }
    for (int i = 0; i < nt; ++i) {
        int hit = -1;
        for (int a = 0; a < ns; ++a)
            if (xt[i] == xs[a]) hit = a;
        if (hit >= 0) {
            for (int a = 0; a < ns; ++a) J[i * ns + a] = (a == hit) ? 1.0 : 0.0;
            continue;
        }
        double den = 0.0;
        for (int a = 0; a < ns; ++a) den += lam[a] / (xt[i] - xs[a]);
        for (int a = 0; a < ns; ++a) J[i * ns + a] = (lam[a] / (xt[i] - xs[a])) / den;
    }
}

// Gauss--Legendre rule with M points on [-1, 1], ascending: the zeros of P_M
// by Newton's method from the start points cos(pi (j + 3/4) / (M + 1/2)),
// weights 2 / ((1 - x^2) P_M'(x)^2).
int host_gauss(int M, double *x, double *w)
{
    if (M < 1 || M > kMaxGauss) return SEM_EINVAL;
    for (int j = 0; j < M; ++j) {
        double t = -std::cos(M_PI * (j + 0.75) / (M + 0.5));
        double pn = 0.0, pn1 = 0.0, dpn = 0.0, dpn1 = 0.0;
        for (int it = 0; it < 100; ++it) {
            if (M == 1) {
                t = 0.0;
                break;
            }
            legendre_pair(M, t, pn, pn1, dpn, dpn1);
            const double step = pn / dpn;
            t -= step;
            if (std::fabs(step) <= 1e-16 * (1.0 + std::fabs(t))) break;
        }
        x[j] = t;
    }
    for (int j = 0; j < M / 2; ++j) {  // symmetric rule
        const double a = 0.5 * (x[M - 1 - j] - x[j]);
        x[j] = -a;
        x[M - 1 - j] = a;
    }
    if (M % 2 == 1) x[M / 2] = 0.0;
    for (int j = 0; j < M; ++j) {
        double dp = 1.0;
        if (M > 1) {
            double pn, pn1, dpn, dpn1;
            legendre_pair(M, x[j], pn, pn1, dpn, dpn1);
            dp = dpn;
        }
        w[j] = 2.0 / ((1.0 - x[j] * x[j]) * dp * dp);
    }
    return SEM_OK;
}

}  // namespace semx
