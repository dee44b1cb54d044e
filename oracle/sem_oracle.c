/*
 * sem_oracle.c -- plain FP64 CPU reference for the spectral-element (SEM)
 * Poisson/Helmholtz operator, its direct-stiffness summation and the data
 * the solvers need.
 *
 * TEST INFRASTRUCTURE.  This file is the oracle that the HIP path is checked
 * against.  Only tests, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code with the HIP library.
 *
 * Everything is written as the plain definition with explicit loops, in the
 * order the paper states it (NekRS paper, Sec. 2.3 "Spectral Element
 * Discretization").  No blocking, no fusion, no reordering.
 *
 * Storage: an element-local array u^e_{ijk} is stored with i fastest,
 * idx = i + (N+1) j + (N+1)^2 k, elements contiguous (Sec. 2.3, eq. (uijk) and
 * the Kronecker form D_1 = I (x) I (x) D-hat of eq. (gradr)).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_EMESH -6

/* ------------------------------------------------------------------------ */
/* Legendre polynomial P_n and its first derivative at x, by the three-term   */
/* recurrence  k P_k = (2k-1) x P_{k-1} - (k-1) P_{k-2}  and                  */
/* P_k' = P_{k-2}' + (2k-1) P_{k-1}.                                         */
/* ------------------------------------------------------------------------ */
static void legendre(int n, double x, double *p, double *dp)
{
    double pm2 = 1.0, pm1 = x, dm2 = 0.0, dm1 = 1.0;
    if (n == 0) { *p = 1.0; *dp = 0.0; return; }
    if (n == 1) { *p = x; *dp = 1.0; return; }
    for (int k = 2; k <= n; ++k) {
        double pk = ((2.0 * k - 1.0) * x * pm1 - (k - 1.0) * pm2) / k;
        double dk = dm2 + (2.0 * k - 1.0) * pm1;
        pm2 = pm1; pm1 = pk;
        dm2 = dm1; dm1 = dk;
    }
    *p = pm1; *dp = dm1;
}

/*
 * Gauss--Lobatto--Legendre nodes xi_0..xi_N and weights rho_0..rho_N
 * (Sec. 2.3: the cardinal Lagrange basis h_i is built on the GLL points and
 * GLL quadrature gives the diagonal mass matrix).
 * Nodes: xi_0 = -1, xi_N = 1, interior nodes the roots of P_N'.  Each interior
 * root is found by Newton's method on P_N' started at -cos(pi j / N); P_N'' is
 * taken from Legendre's equation (1-x^2) P'' = 2x P' - N(N+1) P.
 * Weights: rho_j = 2 / (N (N+1) P_N(xi_j)^2).
 */
int oracle_gll(int N, double *xi, double *rho)
{
    if (N < 1 || N > 32 || !xi || !rho) return ORC_EINVAL;
    xi[0] = -1.0;
    xi[N] = 1.0;
    for (int j = 1; j < N; ++j) {
        double x = -cos(M_PI * j / N);
        for (int it = 0; it < 100; ++it) {
            double p, dp;
            legendre(N, x, &p, &dp);
            double d2p = (2.0 * x * dp - N * (N + 1.0) * p) / (1.0 - x * x);
            double dx = dp / d2p;
            x -= dx;
            if (fabs(dx) < 1e-17) break;
        }
        xi[j] = x;
    }
    /* the node set is symmetric about 0 */
    for (int j = 0; j < (N + 1) / 2; ++j) {
        double s = 0.5 * (xi[N - j] - xi[j]);
        xi[j] = -s;
        xi[N - j] = s;
    }
    if (N % 2 == 0) xi[N / 2] = 0.0;
    for (int j = 0; j <= N; ++j) {
        double p, dp;
        legendre(N, xi[j], &p, &dp);
        rho[j] = 2.0 / (N * (N + 1.0) * p * p);
    }
    return ORC_OK;
}

/*
 * One-dimensional differentiation matrix, eq. (dh):
 *   Dh[i][l] = h_l'(xi_i), row i = quadrature point, column l = node.
 * Off-diagonal entries from the GLL closed form
 *   h_l'(xi_i) = P_N(xi_i) / (P_N(xi_l) (xi_i - xi_l)),  i != l;
 * the diagonal from the fact that the derivative of the constant 1 = sum_l h_l
 * vanishes: Dh[i][i] = -sum_{l != i} Dh[i][l].
 * D is (N+1)x(N+1), row-major, D[i*(N+1)+l].
 */
int oracle_dhat(int N, const double *xi, double *D)
{
    if (N < 1 || !xi || !D) return ORC_EINVAL;
    int nq = N + 1;
    double pn[64];
    for (int j = 0; j < nq; ++j) {
        double dp;
        legendre(N, xi[j], &pn[j], &dp);
    }
    for (int i = 0; i < nq; ++i) {
        double s = 0.0;
        for (int l = 0; l < nq; ++l) {
            if (l == i) continue;
            D[i * nq + l] = pn[i] / (pn[l] * (xi[i] - xi[l]));
            s += D[i * nq + l];
        }
        D[i * nq + i] = -s;
    }
    return ORC_OK;
}

/*
 * Lagrange interpolation matrix from a node set xs (ns points) to target
 * points xt (nt points):  J[i][j] = h_j(xt_i), the cardinal polynomial of the
 * source set (h_j(xs_m) = delta_jm) evaluated at the target point, product
 * form.  Used for p-multigrid transfers and for moving coordinates between
 * orders (Sec. 3.4, p-multigrid schedule N, N/2, 1).
 */
int oracle_interp(int ns, const double *xs, int nt, const double *xt, double *J)
{
    if (ns < 1 || nt < 1 || !xs || !xt || !J) return ORC_EINVAL;
    for (int i = 0; i < nt; ++i)
        for (int j = 0; j < ns; ++j) {
            double h = 1.0;
            for (int m = 0; m < ns; ++m)
                if (m != j) h *= (xt[i] - xs[m]) / (xs[j] - xs[m]);
            J[i * ns + j] = h;
        }
    return ORC_OK;
}

#define IDX(i, j, k, e) ((i) + nq * ((j) + nq * ((k) + (int64_t)nq * (e))))

/*
 * Geometric factors, Sec. 2.3 eqs. (grad), (vBu) and (gij).
 *   dx_p/dr_q = D_q x_p (the three contractions of eqs. (gradr)-(gradt)),
 *   Jacobian J = det(dx/dr), metric dr_q/dx_p from the inverse at each point,
 *   B   = rho_i rho_j rho_k J                         (diagonal mass),
 *   G_mm' = (sum_l dr_m/dx_l dr_m'/dx_l) B           (eq. (gij)).
 * Output G is [6][E*(N+1)^3] in the order G11, G12, G13, G22, G23, G33;
 * B is [E*(N+1)^3]; Jac (optional) receives J.
 * Returns ORC_EMESH if any J <= 0.
 */
int oracle_geometry(int N, int64_t E, const double *D, const double *rho,
                    const double *x, const double *y, const double *z,
                    double *G, double *B, double *Jac)
{
    if (N < 1 || E < 1 || !D || !rho || !x || !y || !z || !G || !B) return ORC_EINVAL;
    int nq = N + 1;
    int64_t nL = E * nq * nq * nq;
    const double *X[3] = {x, y, z};
    int bad = 0;
    /* elements independent: split over threads in the timing build only */
#ifdef _OPENMP
#pragma omp parallel for schedule(static) reduction(| : bad)
#endif
    for (int64_t e = 0; e < E; ++e)
        for (int k = 0; k < nq; ++k)
            for (int j = 0; j < nq; ++j)
                for (int i = 0; i < nq; ++i) {
                    double M[3][3]; /* M[p][q] = d x_p / d r_q */
                    for (int p = 0; p < 3; ++p) {
                        double dr = 0, ds = 0, dt = 0;
                        for (int l = 0; l < nq; ++l) {
                            dr += D[i * nq + l] * X[p][IDX(l, j, k, e)];
                            ds += D[j * nq + l] * X[p][IDX(i, l, k, e)];
                            dt += D[k * nq + l] * X[p][IDX(i, j, l, e)];
                        }
                        M[p][0] = dr; M[p][1] = ds; M[p][2] = dt;
                    }
                    double det = M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1])
                               - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0])
                               + M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
                    if (!(det > 0.0)) bad = 1;
                    /* R[q][p] = d r_q / d x_p = (M^{-1})[q][p] = cofactor(M)[p][q] / det */
                    double R[3][3];
                    R[0][0] = (M[1][1] * M[2][2] - M[1][2] * M[2][1]) / det;
                    R[0][1] = (M[0][2] * M[2][1] - M[0][1] * M[2][2]) / det;
                    R[0][2] = (M[0][1] * M[1][2] - M[0][2] * M[1][1]) / det;
                    R[1][0] = (M[1][2] * M[2][0] - M[1][0] * M[2][2]) / det;
                    R[1][1] = (M[0][0] * M[2][2] - M[0][2] * M[2][0]) / det;
                    R[1][2] = (M[0][2] * M[1][0] - M[0][0] * M[1][2]) / det;
                    R[2][0] = (M[1][0] * M[2][1] - M[1][1] * M[2][0]) / det;
                    R[2][1] = (M[0][1] * M[2][0] - M[0][0] * M[2][1]) / det;
                    R[2][2] = (M[0][0] * M[1][1] - M[0][1] * M[1][0]) / det;
                    int64_t q = IDX(i, j, k, e);
                    double b = rho[i] * rho[j] * rho[k] * det;
                    B[q] = b;
                    if (Jac) Jac[q] = det;
                    int slot = 0;
                    for (int m = 0; m < 3; ++m)
                        for (int mp = m; mp < 3; ++mp) {
                            double s = 0;
                            for (int l = 0; l < 3; ++l) s += R[m][l] * R[mp][l];
                            G[slot * nL + q] = s * b;
                            ++slot;
                        }
                }
    return bad ? ORC_EMESH : ORC_OK;
}

/*
 * Unassembled operator w_L = h1 A_L(k) u_L + h2 B_L u_L, Sec. 2.3 eq. (Ae):
 *   A^e = [D1;D2;D3]^T (k o G^e) [D1;D2;D3],
 * with D1 = I(x)I(x)Dh, D2 = I(x)Dh(x)I, D3 = Dh(x)I(x)I (eqs. (gradr)-(gradt)).
 * Step 1: (ur, us, ut) = (D1 u, D2 u, D3 u).
 * Step 2: (wr, ws, wt) = k * G (ur, us, ut), G the symmetric 3x3 per point.
 * Step 3: w = D1^T wr + D2^T ws + D3^T wt.
 * Step 4: w = h1 w + h2 B u.
 * kcoef may be NULL (k = 1); B may be NULL when h2 == 0.
 */
int oracle_ax(int N, int64_t E, const double *D, const double *G, const double *B,
              const double *kcoef, double h1, double h2, const double *u, double *w)
{
    if (N < 1 || E < 1 || !D || !G || !u || !w) return ORC_EINVAL;
    if (h2 != 0.0 && !B) return ORC_EINVAL;
    int nq = N + 1;
    int np = nq * nq * nq;
    int64_t nL = E * np;
    int failed = 0;
    /* Elements are independent.  The separate timing build (-fopenmp) splits
     * the element loop over threads, each with its own scratch; the checked
     * build compiles without OpenMP and runs it as one plain loop.  The
     * arithmetic of an element is the same either way. */
#ifdef _OPENMP
#pragma omp parallel reduction(| : failed)
#endif
    {
    double *wr = malloc(sizeof(double) * np);
    double *ws = malloc(sizeof(double) * np);
    double *wt = malloc(sizeof(double) * np);
    if (!wr || !ws || !wt) failed = 1;
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
    for (int64_t e = 0; e < E; ++e) {
        if (failed) continue;
        for (int k = 0; k < nq; ++k)
            for (int j = 0; j < nq; ++j)
                for (int i = 0; i < nq; ++i) {
                    double ur = 0, us = 0, ut = 0;
                    for (int l = 0; l < nq; ++l) {
                        ur += D[i * nq + l] * u[IDX(l, j, k, e)];
                        us += D[j * nq + l] * u[IDX(i, l, k, e)];
                        ut += D[k * nq + l] * u[IDX(i, j, l, e)];
                    }
                    int64_t q = IDX(i, j, k, e);
                    double c = kcoef ? kcoef[q] : 1.0;
                    double g11 = G[0 * nL + q], g12 = G[1 * nL + q], g13 = G[2 * nL + q];
                    double g22 = G[3 * nL + q], g23 = G[4 * nL + q], g33 = G[5 * nL + q];
                    int lq = i + nq * (j + nq * k);
                    wr[lq] = c * (g11 * ur + g12 * us + g13 * ut);
                    ws[lq] = c * (g12 * ur + g22 * us + g23 * ut);
                    wt[lq] = c * (g13 * ur + g23 * us + g33 * ut);
                }
        for (int k = 0; k < nq; ++k)
            for (int j = 0; j < nq; ++j)
                for (int i = 0; i < nq; ++i) {
                    double s = 0;
                    for (int l = 0; l < nq; ++l) {
                        s += D[l * nq + i] * wr[l + nq * (j + nq * k)];
                        s += D[l * nq + j] * ws[i + nq * (l + nq * k)];
                        s += D[l * nq + k] * wt[i + nq * (j + nq * l)];
                    }
                    int64_t q = IDX(i, j, k, e);
                    double v = h1 * s;
                    if (h2 != 0.0) v += h2 * B[q] * u[q];
                    w[q] = v;
                }
    }
    free(wr); free(ws); free(wt);
    }
    return failed ? ORC_EINVAL : ORC_OK;
}

/* Threads the element loop of oracle_ax uses (1 in the checked build). */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Diagonal of the unassembled operator h1 A^e(k) + h2 B^e (for Jacobi).
 * Entry at point p = (i,j,k) of sum_{m,m'} D_m^T diag(k G_mm') D_m':
 *   sum_l Dh[l][i]^2 (kG11)[l,j,k] + sum_l Dh[l][j]^2 (kG22)[i,l,k]
 * + sum_l Dh[l][k]^2 (kG33)[i,j,l]
 * + 2 Dh[i][i] Dh[j][j] (kG12)[p] + 2 Dh[i][i] Dh[k][k] (kG13)[p]
 * + 2 Dh[j][j] Dh[k][k] (kG23)[p],
 * since D_m and D_m' (m != m') share a nonzero only on the diagonal.
 */
int oracle_diag(int N, int64_t E, const double *D, const double *G, const double *B,
                const double *kcoef, double h1, double h2, double *d)
{
    if (N < 1 || E < 1 || !D || !G || !d) return ORC_EINVAL;
    if (h2 != 0.0 && !B) return ORC_EINVAL;
    int nq = N + 1;
    int64_t nL = E * nq * nq * nq;
#define KG(s, q) ((kcoef ? kcoef[q] : 1.0) * G[(s) * nL + (q)])
    for (int64_t e = 0; e < E; ++e)
        for (int k = 0; k < nq; ++k)
            for (int j = 0; j < nq; ++j)
                for (int i = 0; i < nq; ++i) {
                    double s = 0;
                    for (int l = 0; l < nq; ++l) {
                        s += D[l * nq + i] * D[l * nq + i] * KG(0, IDX(l, j, k, e));
                        s += D[l * nq + j] * D[l * nq + j] * KG(3, IDX(i, l, k, e));
                        s += D[l * nq + k] * D[l * nq + k] * KG(5, IDX(i, j, l, e));
                    }
                    int64_t q = IDX(i, j, k, e);
                    double di = D[i * nq + i], dj = D[j * nq + j], dk = D[k * nq + k];
                    s += 2.0 * di * dj * KG(1, q) + 2.0 * di * dk * KG(2, q)
                       + 2.0 * dj * dk * KG(4, q);
                    double v = h1 * s;
                    if (h2 != 0.0) v += h2 * B[q];
                    d[q] = v;
                }
#undef KG
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Gather-scatter QQ^T (Sec. 2.3 eq. (dssum) and the Q / Q^T discussion;     */
/* Sec. 3.2 gs_setup / gs_op contract: equal global pointers are summed,      */
/* a unique pointer leaves its entry unchanged, pointer 0 is a singleton).   */
/* ------------------------------------------------------------------------ */
typedef struct { int64_t g; int64_t i; } gpair;

static int cmp_gpair(const void *a, const void *b)
{
    const gpair *x = a, *y = b;
    if (x->g != y->g) return x->g < y->g ? -1 : 1;
    if (x->i != y->i) return x->i < y->i ? -1 : 1;
    return 0;
}

/*
 * Compact numbering: cid[l] = index (0..ng-1) of gid[l] among the distinct
 * nonzero gids, -1 for gid 0.  Returns ng, or a negative code.
 */
static int64_t compact_ids(int64_t nL, const int64_t *gid, int64_t *cid)
{
    int64_t m = 0;
    for (int64_t l = 0; l < nL; ++l) if (gid[l] != 0) ++m;
    gpair *pr = malloc(sizeof(gpair) * (m ? m : 1));
    if (!pr) return ORC_EINVAL;
    m = 0;
    for (int64_t l = 0; l < nL; ++l) {
        cid[l] = -1;
        if (gid[l] != 0) { pr[m].g = gid[l]; pr[m].i = l; ++m; }
    }
    qsort(pr, m, sizeof(gpair), cmp_gpair);
    int64_t ng = 0;
    for (int64_t a = 0; a < m; ++a) {
        if (a > 0 && pr[a].g != pr[a - 1].g) ++ng;
        cid[pr[a].i] = ng;
    }
    if (m > 0) ++ng;
    free(pr);
    return ng;
}

/*
 * v <- QQ^T v by a global accumulator: every local copy is added to the
 * accumulator of its global pointer in ascending local-index order, then each
 * copy receives its accumulator.  Entries with pointer 0 are not touched.
 */
int oracle_qqt(int64_t nL, const int64_t *gid, double *v)
{
    if (nL < 0 || !gid || !v) return ORC_EINVAL;
    int64_t *cid = malloc(sizeof(int64_t) * (nL ? nL : 1));
    if (!cid) return ORC_EINVAL;
    int64_t ng = compact_ids(nL, gid, cid);
    if (ng < 0) { free(cid); return (int)ng; }
    double *acc = calloc(ng ? ng : 1, sizeof(double));
    if (!acc) { free(cid); return ORC_EINVAL; }
    for (int64_t l = 0; l < nL; ++l)
        if (cid[l] >= 0) acc[cid[l]] += v[l];
    for (int64_t l = 0; l < nL; ++l)
        if (cid[l] >= 0) v[l] = acc[cid[l]];
    free(acc);
    free(cid);
    return ORC_OK;
}

/* gs_op of Sec. 3.2 with the library's associative, commutative operations:
 * op 0 sum (identical to oracle_qqt: from 0, copies in ascending local index
 * order), 1 product, 2 minimum (fmin), 3 maximum (fmax), the last three started
 * from the node's first copy and combined with the others in ascending local
 * index order.  Every copy of a node receives the result; pointer 0 and
 * unique pointers are left unchanged. */
int oracle_gs_op(int64_t nL, const int64_t *gid, int op, double *v)
{
    if (nL < 0 || !gid || !v || op < 0 || op > 3) return ORC_EINVAL;
    int64_t *cid = malloc(sizeof(int64_t) * (nL ? nL : 1));
    if (!cid) return ORC_EINVAL;
    int64_t ng = compact_ids(nL, gid, cid);
    if (ng < 0) { free(cid); return (int)ng; }
    double *acc = calloc(ng ? ng : 1, sizeof(double));
    unsigned char *seen = calloc(ng ? ng : 1, 1);
    if (!acc || !seen) { free(acc); free(seen); free(cid); return ORC_EINVAL; }
    for (int64_t l = 0; l < nL; ++l) {
        const int64_t c = cid[l];
        if (c < 0) continue;
        if (op == 0) {
            acc[c] += v[l];
        } else if (!seen[c]) {
            acc[c] = v[l];
            seen[c] = 1;
        } else if (op == 1) {
            acc[c] = acc[c] * v[l];
        } else if (op == 2) {
            acc[c] = fmin(acc[c], v[l]);
        } else {
            acc[c] = fmax(acc[c], v[l]);
        }
    }
    for (int64_t l = 0; l < nL; ++l) {
        const int64_t c = cid[l];
        if (c >= 0) v[l] = acc[c];
    }
    free(seen);
    free(acc);
    free(cid);
    return ORC_OK;
}

/* Multiplicity of each local copy: number of copies with the same nonzero
 * global pointer (1 for pointer 0). */
int oracle_multiplicity(int64_t nL, const int64_t *gid, int32_t *mult)
{
    if (nL < 0 || !gid || !mult) return ORC_EINVAL;
    int64_t *cid = malloc(sizeof(int64_t) * (nL ? nL : 1));
    if (!cid) return ORC_EINVAL;
    int64_t ng = compact_ids(nL, gid, cid);
    int32_t *cnt = calloc(ng ? ng : 1, sizeof(int32_t));
    if (!cnt) { free(cid); return ORC_EINVAL; }
    for (int64_t l = 0; l < nL; ++l) if (cid[l] >= 0) cnt[cid[l]]++;
    for (int64_t l = 0; l < nL; ++l) mult[l] = cid[l] >= 0 ? cnt[cid[l]] : 1;
    free(cnt);
    free(cid);
    return ORC_OK;
}

/*
 * Sorted gather-scatter maps, by definition: the (gid, local index) pairs
 * with gid != 0 sorted lexicographically, keeping only global pointers held
 * by two or more copies.  perm[0..ncopies) lists local indices in that order;
 * offs[0..nseg] are the segment starts.  When perm/offs are NULL only the
 * counts are returned.
 */
int oracle_gs_maps(int64_t nL, const int64_t *gid, int64_t *ncopies, int64_t *nseg,
                   int32_t *perm, int32_t *offs)
{
    if (nL < 0 || !gid || !ncopies || !nseg) return ORC_EINVAL;
    int64_t m = 0;
    for (int64_t l = 0; l < nL; ++l) if (gid[l] != 0) ++m;
    gpair *pr = malloc(sizeof(gpair) * (m ? m : 1));
    if (!pr) return ORC_EINVAL;
    m = 0;
    for (int64_t l = 0; l < nL; ++l)
        if (gid[l] != 0) { pr[m].g = gid[l]; pr[m].i = l; ++m; }
    qsort(pr, m, sizeof(gpair), cmp_gpair);
    int64_t nc = 0, ns = 0;
    int64_t a = 0;
    while (a < m) {
        int64_t b = a;
        while (b < m && pr[b].g == pr[a].g) ++b;
        if (b - a >= 2) {
            if (offs) offs[ns] = (int32_t)nc;
            for (int64_t t = a; t < b; ++t) {
                if (perm) perm[nc] = (int32_t)pr[t].i;
                ++nc;
            }
            ++ns;
        }
        a = b;
    }
    if (offs) offs[ns] = (int32_t)nc;
    *ncopies = nc;
    *nseg = ns;
    free(pr);
    return ORC_OK;
}

/*
 * Gradient of L with respect to the per-copy coefficient k of the
 * variable-coefficient operator A(k) = Q^T A_L(k) Q (eq. (Ae) with k scaling
 * G pointwise).  With A(k) u = b and A lam = dL/du,
 *   dL/dk[e,q] = -h1 sum_{m,m'} (D_m lam)_q G_mm'[q] (D_m' u)_q,
 * the reference-space gradients taken as in eqs. (gradr)-(gradt).
 */
int oracle_grad_k(int N, int64_t E, const double *D, const double *G, double h1,
                  const double *u, const double *lam, double *gk)
{
    if (N < 1 || E < 1 || !D || !G || !u || !lam || !gk) return ORC_EINVAL;
    int nq = N + 1;
    int64_t nL = E * nq * nq * nq;
    for (int64_t e = 0; e < E; ++e)
        for (int k = 0; k < nq; ++k)
            for (int j = 0; j < nq; ++j)
                for (int i = 0; i < nq; ++i) {
                    double a[3] = {0, 0, 0}, c[3] = {0, 0, 0};
                    for (int l = 0; l < nq; ++l) {
                        a[0] += D[i * nq + l] * lam[IDX(l, j, k, e)];
                        a[1] += D[j * nq + l] * lam[IDX(i, l, k, e)];
                        a[2] += D[k * nq + l] * lam[IDX(i, j, l, e)];
                        c[0] += D[i * nq + l] * u[IDX(l, j, k, e)];
                        c[1] += D[j * nq + l] * u[IDX(i, l, k, e)];
                        c[2] += D[k * nq + l] * u[IDX(i, j, l, e)];
                    }
                    int64_t q = IDX(i, j, k, e);
                    double g[3][3];
                    g[0][0] = G[0 * nL + q]; g[0][1] = g[1][0] = G[1 * nL + q];
                    g[0][2] = g[2][0] = G[2 * nL + q]; g[1][1] = G[3 * nL + q];
                    g[1][2] = g[2][1] = G[4 * nL + q]; g[2][2] = G[5 * nL + q];
                    double s = 0;
                    for (int m = 0; m < 3; ++m)
                        for (int mp = 0; mp < 3; ++mp) s += a[m] * g[m][mp] * c[mp];
                    gk[q] = -h1 * s;
                }
    return ORC_OK;
}

/* Interpolate an L-vector from order Ns to order Nt element by element with
 * the tensor product of the 1D matrix J (nt x ns): out = (J (x) J (x) J) in. */
int oracle_interp_lvec(int ns, int nt, int64_t E, const double *J, const double *in, double *out)
{
    if (ns < 1 || nt < 1 || E < 1 || !J || !in || !out) return ORC_EINVAL;
    int64_t pin = (int64_t)ns * ns * ns, pout = (int64_t)nt * nt * nt;
    for (int64_t e = 0; e < E; ++e)
        for (int k = 0; k < nt; ++k)
            for (int j = 0; j < nt; ++j)
                for (int i = 0; i < nt; ++i) {
                    double s = 0;
                    for (int c = 0; c < ns; ++c)
                        for (int b = 0; b < ns; ++b)
                            for (int a = 0; a < ns; ++a)
                                s += J[k * ns + c] * J[j * ns + b] * J[i * ns + a]
                                   * in[e * pin + a + ns * (b + ns * c)];
                    out[e * pout + i + nt * (j + nt * k)] = s;
                }
    return ORC_OK;
}
