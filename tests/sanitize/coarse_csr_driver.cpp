// Host check of the coarse-system assembly (coarse_csr.h) against the
// definition A = sum_e P_e^T A_e P_e on the free nodes, formed as a dense
// matrix element by element in the same order, on small box meshes of
// trilinear elements: Dirichlet and Neumann boundaries, node ids permuted,
// a collapsed element (two local points on one node), and no free nodes.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "coarse_csr.h"

static int fail(const char *what, int c)
{
    std::printf("FAIL case %d: %s\n", c, what);
    return 1;
}

static int run_case(int c, int ex, int ey, int ez, bool dirichlet, bool permute, bool collapse, unsigned seed)
{
    const int nx = ex + 1, ny = ey + 1, nz = ez + 1, np = 8;
    const int64_t E = (int64_t)ex * ey * ez;
    std::mt19937_64 g(seed);
    std::vector<int32_t> node((size_t)nx * ny * nz, -1);
    int32_t nf = 0;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const bool bnd = i == 0 || j == 0 || k == 0 || i == ex || j == ey || k == ez;
                if (!(dirichlet && bnd)) node[((size_t)k * ny + j) * nx + i] = nf++;
            }
    std::vector<int32_t> relabel((size_t)nf);
    for (int32_t i = 0; i < nf; ++i) relabel[(size_t)i] = i;
    if (permute) std::shuffle(relabel.begin(), relabel.end(), g);
    std::vector<int32_t> uid((size_t)E * np);
    int64_t e = 0;
    for (int k = 0; k < ez; ++k)
        for (int j = 0; j < ey; ++j)
            for (int i = 0; i < ex; ++i, ++e) {
                int q = 0;
                for (int cz = 0; cz < 2; ++cz)
                    for (int cy = 0; cy < 2; ++cy)
                        for (int cx = 0; cx < 2; ++cx) {
                            const int32_t id = node[((size_t)(k + cz) * ny + (j + cy)) * nx + (i + cx)];
                            uid[(size_t)e * np + q++] = id < 0 ? -1 : relabel[(size_t)id];
                        }
            }
    if (collapse && E > 1)
        for (int q = 0; q < np; ++q)
            if (uid[(size_t)np + q] >= 0) {  // element 1: point 7 onto its first free point
                uid[(size_t)np + 7] = uid[(size_t)np + q];
                break;
            }
    std::uniform_real_distribution<double> d(-1.0, 1.0);
    std::vector<double> Ae((size_t)E * np * np);
    for (int64_t el = 0; el < E; ++el)
        for (int q = 0; q < np; ++q)
            for (int p = 0; p < np; ++p) Ae[((size_t)el * np + q) * np + p] = d(g) + (q == p ? 10.0 : 0.0);
    // the definition, dense, summed element by element
    std::vector<double> A((size_t)nf * nf, 0.0);
    std::vector<char> touched((size_t)nf * nf, 0);
    for (int64_t el = 0; el < E; ++el)
        for (int q = 0; q < np; ++q) {
            const int32_t r = uid[(size_t)el * np + q];
            if (r < 0) continue;
            for (int p = 0; p < np; ++p) {
                const int32_t cc = uid[(size_t)el * np + p];
                if (cc < 0) continue;
                A[(size_t)r * nf + cc] += Ae[((size_t)el * np + q) * np + p];
                touched[(size_t)r * nf + cc] = 1;
            }
        }
    std::vector<int32_t> row, col;
    std::vector<double> val, dinv;
    if (semx::assemble_free_csr(E, np, nf, uid.data(), Ae.data(), row, col, val, dinv) != -1)
        return fail("reported a nonpositive diagonal", c);
    if ((int64_t)row.size() != (int64_t)nf + 1 || row[0] != 0 || (size_t)row[(size_t)nf] != col.size() ||
        val.size() != col.size() || (int64_t)dinv.size() != nf)
        return fail("array sizes", c);
    for (int32_t r = 0; r < nf; ++r) {
        int32_t k = row[(size_t)r];
        for (int32_t cc = 0; cc < nf; ++cc) {
            if (!touched[(size_t)r * nf + cc]) continue;
            if (k >= row[(size_t)r + 1] || col[(size_t)k] != cc) return fail("column pattern", c);
            if (std::memcmp(&val[(size_t)k], &A[(size_t)r * nf + cc], sizeof(double)) != 0)
                return fail("value differs from the element-by-element sum", c);
            ++k;
        }
        if (k != row[(size_t)r + 1]) return fail("extra columns", c);
        if (dinv[(size_t)r] != 1.0 / A[(size_t)r * nf + r]) return fail("inverse diagonal", c);
    }
    // a nonpositive diagonal is reported at its row
    if (nf > 0 && E > 0) {
        const int32_t r0 = uid[0] >= 0 ? uid[0] : -1;
        if (r0 >= 0) {
            std::vector<double> Ab(Ae);
            Ab[0] -= A[(size_t)r0 * nf + r0] + 1.0;  // row r0's diagonal becomes -1
            if (semx::assemble_free_csr(E, np, nf, uid.data(), Ab.data(), row, col, val, dinv) != r0)
                return fail("nonpositive diagonal not reported at its row", c);
        }
    }
    std::printf("ok case %d: %dx%dx%d %s%s%s nf=%d nnz=%zu\n", c, ex, ey, ez, dirichlet ? "dirichlet" : "neumann",
                permute ? " permuted" : "", collapse ? " collapsed" : "", nf, col.size());
    return 0;
}

int main()
{
    int bad = 0;
    bad += run_case(0, 1, 1, 1, true, false, false, 1);
    bad += run_case(1, 2, 1, 1, false, false, false, 2);
    bad += run_case(2, 3, 3, 2, true, true, false, 3);
    bad += run_case(3, 3, 3, 2, false, true, true, 4);
    bad += run_case(4, 4, 3, 3, true, false, true, 5);
    bad += run_case(5, 5, 4, 3, false, true, false, 6);
    return bad;
}
