/*
 * Driver for sanitizer builds of the CPU oracle (sem_oracle.c): every entry
 * point on a small deformed box, with checks that need no other code:
 * sum of B equals the box volume to quadrature accuracy, the assembled
 * Neumann operator annihilates constants, QQ^T of ones is the
 * multiplicity, the maps cover every shared copy once, and interpolation to
 * the same order is the identity.  Exit status 0 when every check holds.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_gll(int N, double *xi, double *rho);
int oracle_dhat(int N, const double *xi, double *D);
int oracle_interp(int ns, const double *xs, int nt, const double *xt, double *J);
int oracle_geometry(int N, int64_t E, const double *D, const double *rho, const double *x,
                    const double *y, const double *z, double *G, double *B, double *Jac);
int oracle_ax(int N, int64_t E, const double *D, const double *G, const double *B,
              const double *kcoef, double h1, double h2, const double *u, double *w);
int oracle_diag(int N, int64_t E, const double *D, const double *G, const double *B,
                const double *kcoef, double h1, double h2, double *d);
int oracle_qqt(int64_t nL, const int64_t *gid, double *v);
int oracle_multiplicity(int64_t nL, const int64_t *gid, int32_t *mult);
int oracle_gs_maps(int64_t nL, const int64_t *gid, int64_t *ncopies, int64_t *nseg, int32_t *perm,
                   int32_t *offs);
int oracle_grad_k(int N, int64_t E, const double *D, const double *G, double h1, const double *u,
                  const double *lam, double *gk);
int oracle_interp_lvec(int ns, int nt, int64_t E, const double *J, const double *in, double *out);

#define CHECK(c)                                                   \
    do {                                                           \
        if (!(c)) {                                                \
            fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            return 1;                                              \
        }                                                          \
    } while (0)

static int run(int N, int ex, int ey, int ez)
{
    const double PI = 3.14159265358979323846, a = 0.05;
    const int nq = N + 1;
    const int64_t E = (int64_t)ex * ey * ez, np = (int64_t)nq * nq * nq, nL = E * np;
    double *xi = malloc(sizeof(double) * nq), *rho = malloc(sizeof(double) * nq);
    double *D = malloc(sizeof(double) * nq * nq), *J = malloc(sizeof(double) * nq * nq);
    double *x = malloc(sizeof(double) * nL), *y = malloc(sizeof(double) * nL), *z = malloc(sizeof(double) * nL);
    int64_t *gid = malloc(sizeof(int64_t) * nL);
    double *G = malloc(sizeof(double) * 6 * nL), *B = malloc(sizeof(double) * nL), *Jac = malloc(sizeof(double) * nL);
    double *u = malloc(sizeof(double) * nL), *w = malloc(sizeof(double) * nL), *d = malloc(sizeof(double) * nL);
    double *gk = malloc(sizeof(double) * nL), *o = malloc(sizeof(double) * nL);
    int32_t *mult = malloc(sizeof(int32_t) * nL);
    CHECK(oracle_gll(N, xi, rho) == 0);
    CHECK(oracle_dhat(N, xi, D) == 0);
    CHECK(oracle_interp(nq, xi, nq, xi, J) == 0);
    const int64_t nx = (int64_t)ex * N + 1, ny = (int64_t)ey * N + 1;
    for (int64_t e = 0; e < E; ++e) {
        const int64_t ea = e % ex, eb = (e / ex) % ey, ec = e / ((int64_t)ex * ey);
        for (int k = 0; k < nq; ++k)
            for (int j = 0; j < nq; ++j)
                for (int i = 0; i < nq; ++i) {
                    const int64_t l = e * np + (int64_t)(k * nq + j) * nq + i;
                    const double X = (ea + 0.5 * (xi[i] + 1.0)) / ex, Y = (eb + 0.5 * (xi[j] + 1.0)) / ey,
                                 Z = (ec + 0.5 * (xi[k] + 1.0)) / ez;
                    x[l] = X + a * sin(2 * PI * Y) * sin(2 * PI * Z);
                    y[l] = Y + a * sin(2 * PI * Z) * sin(2 * PI * X);
                    z[l] = Z + a * sin(2 * PI * X) * sin(2 * PI * Y);
                    gid[l] = 1 + (ea * N + i) + nx * ((eb * N + j) + ny * (ec * N + k));
                    u[l] = 1.0;
                }
    }
    CHECK(oracle_geometry(N, E, D, rho, x, y, z, G, B, Jac) == 0);
    double vol = 0.0;
    for (int64_t l = 0; l < nL; ++l) vol += B[l];
    CHECK(fabs(vol - 1.0) < 1e-3);
    CHECK(oracle_ax(N, E, D, G, B, NULL, 1.0, 0.0, u, w) == 0);
    CHECK(oracle_qqt(nL, gid, w) == 0);
    double mx = 0.0;
    for (int64_t l = 0; l < nL; ++l) mx = fmax(mx, fabs(w[l]));
    CHECK(mx < 1e-10);
    for (int64_t l = 0; l < nL; ++l) u[l] = sin(3.0 * l) + 0.5;
    CHECK(oracle_ax(N, E, D, G, B, u, 1.0, 2.0, u, w) == 0);
    CHECK(oracle_diag(N, E, D, G, B, u, 1.0, 2.0, d) == 0);
    CHECK(oracle_grad_k(N, E, D, G, 1.0, u, w, gk) == 0);
    CHECK(oracle_multiplicity(nL, gid, mult) == 0);
    for (int64_t l = 0; l < nL; ++l) o[l] = 1.0;
    CHECK(oracle_qqt(nL, gid, o) == 0);
    for (int64_t l = 0; l < nL; ++l) CHECK(o[l] == (double)mult[l]);
    int64_t nc = 0, ns = 0;
    CHECK(oracle_gs_maps(nL, gid, &nc, &ns, NULL, NULL) == 0);
    int32_t *perm = malloc(sizeof(int32_t) * (nc ? nc : 1)), *offs = malloc(sizeof(int32_t) * (ns + 1));
    CHECK(oracle_gs_maps(nL, gid, &nc, &ns, perm, offs) == 0);
    int64_t shared = 0;
    for (int64_t l = 0; l < nL; ++l) shared += mult[l] >= 2;
    CHECK(shared == nc && offs[ns] == nc);
    CHECK(oracle_interp_lvec(nq, nq, E, J, u, o) == 0);
    for (int64_t l = 0; l < nL; ++l) CHECK(fabs(o[l] - u[l]) < 1e-12);
    printf("oracle N=%d %dx%dx%d: volume %.12f, %lld shared copies in %lld segments\n", N, ex, ey, ez, vol,
           (long long)nc, (long long)ns);
    free(xi); free(rho); free(D); free(J); free(x); free(y); free(z); free(gid); free(G); free(B);
    free(Jac); free(u); free(w); free(d); free(gk); free(o); free(mult); free(perm); free(offs);
    return 0;
}

int main(void)
{
    const int cases[][4] = {{1, 2, 2, 2}, {3, 3, 2, 2}, {7, 2, 2, 3}, {5, 1, 1, 1}};
    for (int c = 0; c < 4; ++c)
        if (run(cases[c][0], cases[c][1], cases[c][2], cases[c][3])) return 1;
    return 0;
}
