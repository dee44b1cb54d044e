// Host-side driver for sanitizer builds of libsem's host code: the Schwarz
// setup (face walk, 1D eigenproblems, weights; threaded per element range)
// and the GLL construction.  Built from the library's own sources
// (schwarz.hip, gll.cpp) with a host sanitizer; no device work is done.
//
// Mesh: a structured E = ex*ey*ez box of order N (global pointers by the
// lattice index of every node, homogeneous Dirichlet on the box faces), with
// the elements listed in a scrambled order so the face walk meets arbitrary
// element numbers.  Prints a checksum of every output; exits nonzero on a
// library error or a mismatch between two thread counts.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstdarg>
#include <cstring>
#include <vector>

#include "../../include/sem.h"

namespace semx {
// the library's error hook (defined in api.hip, which this test executable does not link)
void set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    std::vfprintf(stderr, fmt, ap);
    va_end(ap);
    std::fputc('\n', stderr);
}
int host_gll(int N, double *xi, double *rho, double *D);
}  // namespace semx

struct Out {
    std::vector<int32_t> ix, cover;
    std::vector<float> S, lam, w;
};

static int run(int N, int ex, int ey, int ez, const char *threads, Out &o)
{
    setenv("SEM_HOST_THREADS", threads, 1);
    const int nq = N + 1, ne = N + 3;
    const int64_t E = (int64_t)ex * ey * ez, np = (int64_t)nq * nq * nq, nL = E * np;
    std::vector<int64_t> gid(nL);
    std::vector<uint8_t> dir(nL);
    std::vector<double> len(3 * E);
    // scrambled element order: position p holds lattice element (p * stride) mod E
    int64_t stride = 7;
    while (E % stride == 0 || stride % 2 == 0) stride += 2;
    const int64_t nx = (int64_t)ex * N + 1, ny = (int64_t)ey * N + 1, nz = (int64_t)ez * N + 1;
    for (int64_t p = 0; p < E; ++p) {
        const int64_t le = (p * stride) % E;
        const int64_t a = le % ex, b = (le / ex) % ey, c = le / ((int64_t)ex * ey);
        for (int k = 0; k < nq; ++k)
            for (int j = 0; j < nq; ++j)
                for (int i = 0; i < nq; ++i) {
                    const int64_t gx = a * N + i, gy = b * N + j, gz = c * N + k;
                    const int64_t l = p * np + (int64_t)(k * nq + j) * nq + i;
                    gid[l] = 1 + gx + nx * (gy + ny * gz);
                    dir[l] = gx == 0 || gx == nx - 1 || gy == 0 || gy == ny - 1 || gz == 0 || gz == nz - 1;
                }
        len[3 * p + 0] = 1.0 / ex;
        len[3 * p + 1] = 1.0 / ey;
        len[3 * p + 2] = 1.0 / ez;
    }
    o.ix.assign((size_t)E * ne * ne * ne, 0);
    o.S.assign((size_t)E * 3 * ne * ne, 0.0f);
    o.lam.assign((size_t)E * 3 * ne, 0.0f);
    o.cover.assign(nL, 0);
    o.w.assign(nL, 0.0f);
    return sem_schwarz_setup_host(N, E, gid.data(), dir.data(), len.data(), o.ix.data(), o.S.data(),
                                  o.lam.data(), o.cover.data(), o.w.data());
}

template <typename T>
static bool same(const std::vector<T> &a, const std::vector<T> &b)
{
    return a.size() == b.size() && std::memcmp(a.data(), b.data(), sizeof(T) * a.size()) == 0;
}

int main(int argc, char **argv)
{
    const int N = argc > 1 ? std::atoi(argv[1]) : 3;
    const int ex = argc > 2 ? std::atoi(argv[2]) : 12, ey = argc > 3 ? std::atoi(argv[3]) : 12,
              ez = argc > 4 ? std::atoi(argv[4]) : 8;
    for (int n = 1; n <= 15; ++n) {
        std::vector<double> xi(n + 1), rho(n + 1), D((n + 1) * (n + 1));
        if (semx::host_gll(n, xi.data(), rho.data(), D.data()) != 0) return 3;
    }
    Out a, b;
    if (run(N, ex, ey, ez, "1", a) != SEM_OK) return 4;
    if (run(N, ex, ey, ez, "16", b) != SEM_OK) return 5;
    const bool eq = same(a.ix, b.ix) && same(a.S, b.S) && same(a.lam, b.lam) && same(a.cover, b.cover) &&
                    same(a.w, b.w);
    double cs = 0.0;
    for (float v : b.S) cs += v;
    for (float v : b.w) cs += v;
    int64_t ci = 0;
    for (int32_t v : b.ix) ci += v;
    std::printf("setup N=%d %dx%dx%d: 1 vs 16 threads %s, checksum %.9e %lld\n", N, ex, ey, ez,
                eq ? "bit-identical" : "DIFFER", cs, (long long)ci);
    return eq ? 0 : 6;
}
