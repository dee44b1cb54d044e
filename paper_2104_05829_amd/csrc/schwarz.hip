// Overlapping Schwarz smoothing with fast-diagonalisation local solves (the
// CHEBY-ASM / CHEBY-RAS smoothers of the NekRS paper, Sec. 3.4).
//
// Subdomain of element e: its nodes plus one node layer of every neighbour,
// ne = N + 3 points per direction.  Local operator: the separable operator of
// the extended box, h1 (Mz(x)My(x)Kx + Mz(x)Ky(x)Mx + Kz(x)My(x)Mx) + h2 Mz(x)My(x)Mx,
// from the 1D SEM stiffness K_d and GLL mass M_d of the element and its two
// neighbours along d (element extents: the mean length of the element's node
// lines), restricted to the kept points (absent outside the domain; an
// all-Dirichlet element face drops its layer).  Fast diagonalisation:
// K_d S_d = M_d S_d diag(lam_d), S_d^T M_d S_d = I, so the local inverse is
// (Sz(x)Sy(x)Sx) diag(1 / (h1 (lx + ly + lz) + h2)) (Sz(x)Sy(x)Sx)^T.
// Combination: ASM adds every subdomain's solution into the copies it covers
// and weights the assembled sum by 1 / (subdomains containing the node); RAS
// keeps each element's own points and averages the copies.
//
// Setup (host, once per level): the extended-point gather map by walking
// across element faces through the global pointers (any conforming hex mesh
// with N >= 2), the 1D operators and their eigen-decompositions (cyclic
// Jacobi on M^{-1/2} K M^{-1/2}), and the accumulation lists.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <thread>
#include <numeric>
#include <vector>

#include "sem_internal.h"

namespace semx {

// ------------------------------------------------------------------- setup
namespace {

// symmetric eigen-decomposition A = V diag(w) V^T by cyclic Jacobi rotations
void jacobi_eig(int n, std::vector<double> A, std::vector<double> &w, std::vector<double> &V)
{
    V.assign(n * n, 0.0);
    for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j)
                (i == j ? diag : off) += A[i * n + j] * A[i * n + j];
        if (off <= 1e-30 * diag) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = A[p * n + q];
                if (apq == 0.0) continue;
                const double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {  // A <- A J (columns p, q)
                    const double akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = c * akp - s * akq;
                    A[k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {  // A <- J^T A (rows p, q)
                    const double apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = c * apk - s * aqk;
                    A[q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {  // V <- V J
                    const double vkp = V[k * n + p], vkq = V[k * n + q];
                    V[k * n + p] = c * vkp - s * vkq;
                    V[k * n + q] = s * vkp + c * vkq;
                }
            }
    }
    w.resize(n);
    for (int i = 0; i < n; ++i) w[i] = A[i * n + i];
}

// FDM data of one direction: S [ne][ne] (row = point, column = mode) and lam
// [ne] for the element of length L between neighbours of lengths Lm, Lp (< 0:
// absent); drop_lo / drop_hi remove the element's end points (Dirichlet face)
void fdm_direction(int N, const double *rho, const double *D, double L, double Lm, double Lp,
                   bool drop_lo, bool drop_hi, float *S, float *lam, uint8_t *keep)
{
    const int ne = N + 3, n3 = 3 * N + 1, nq = N + 1;
    std::vector<double> K3(n3 * n3, 0.0), M3(n3, 0.0);
    const double lens[3] = {Lm, L, Lp};
    for (int el = 0; el < 3; ++el) {
        const double Le = lens[el];
        if (!(Le > 0.0)) continue;
        const int off = el * N;
        for (int i = 0; i < nq; ++i) {
            M3[off + i] += 0.5 * Le * rho[i];
            for (int j = 0; j < nq; ++j) {
                double kij = 0.0;  // (2/L) sum_q D[q][i] rho[q] D[q][j]
                for (int q = 0; q < nq; ++q) kij += D[q * nq + i] * rho[q] * D[q * nq + j];
                K3[(off + i) * n3 + off + j] += (2.0 / Le) * kij;
            }
        }
    }
    for (int a = 0; a < ne; ++a) keep[a] = 1;
    keep[0] = Lm > 0.0;
    keep[ne - 1] = Lp > 0.0;
    if (drop_lo) keep[1] = 0;
    if (drop_hi) keep[ne - 2] = 0;
    std::vector<int> idx;
    for (int a = 0; a < ne; ++a)
        if (keep[a]) idx.push_back(a);
    const int m = (int)idx.size();
    // B = M^{-1/2} K M^{-1/2} on the kept points (M diagonal)
    std::vector<double> B(m * m), w, V;
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) {
            const int gi = N - 1 + idx[i], gj = N - 1 + idx[j];
            B[i * m + j] = K3[gi * n3 + gj] / std::sqrt(M3[gi] * M3[gj]);
        }
    jacobi_eig(m, B, w, V);
    for (int t = 0; t < ne * ne; ++t) S[t] = 0.0f;
    for (int a = 0; a < ne; ++a) lam[a] = 1.0f;
    for (int i = 0; i < m; ++i) {
        const int gi = N - 1 + idx[i];
        for (int k = 0; k < m; ++k) S[idx[i] * ne + k] = (float)(V[i * m + k] / std::sqrt(M3[gi]));
    }
    for (int k = 0; k < m; ++k) lam[k] = (float)w[k];
}

struct FaceLink {
    int64_t nb = -1;   // neighbour element, -1 on the boundary
    int rax[3] = {0, 0, 0};  // axis of nb that each axis of e maps to
    int sgn[3] = {1, 1, 1};  // orientation of that map
    int64_t org[3] = {0, 0, 0};  // nb coordinates of e's face point (1, 1)
};

}  // namespace

void free_schwarz(Level &L)
{
    void *ptrs[] = {L.sz_ix, L.sz_S, L.sz_lam, L.sz_rc, L.sz_off, L.sz_src, L.sz_w};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    L.sz_ix = nullptr;
    L.sz_S = L.sz_lam = nullptr;
    L.sz_rc = L.sz_off = L.sz_src = nullptr;
    L.sz_w = nullptr;
    L.sz_ne = L.sz_next = 0;
    L.sz_nrc = 0;
}

// Host setup of one level: gather map ix [E][ne^3], FDM data S [E][3][ne][ne]
// and lam [E][3][ne], accumulation lists off [nL+1] / src, weight w [nL].
struct SchwarzHost {
    std::vector<int32_t> ix, off;
    std::vector<float> S, lam, w;
};

// host threads for the per-element setup work: SEM_HOST_THREADS when set to
// 1..64 (read at every setup), else the hardware concurrency, at most 16.
// The result does not depend on the count (disjoint per-element ranges, a
// deterministic merge of sorted runs).
static int host_threads()
{
    if (const char *env = std::getenv("SEM_HOST_THREADS")) {
        const long v = std::strtol(env, nullptr, 10);
        if (v >= 1 && v <= 64) return (int)v;
    }
    const unsigned hc = std::thread::hardware_concurrency();
    return (int)std::max(1u, std::min(16u, hc));
}

// fn(lo, hi) on [0, n) split into contiguous ranges, one per thread
template <typename Fn>
static void parallel_ranges(int64_t n, Fn fn)
{
    const int nt = (int)std::min<int64_t>(host_threads(), std::max<int64_t>(1, n / 64));
    if (nt <= 1) {
        fn((int64_t)0, n);
        return;
    }
    std::vector<std::thread> th;
    for (int i = 0; i < nt; ++i) th.emplace_back(fn, n * i / nt, n * (i + 1) / nt);
    for (auto &t : th) t.join();
}

// sort v (pairs, lexicographic) in threaded chunks, then merge them pairwise
static void parallel_sort(std::vector<std::pair<int64_t, int64_t>> &v)
{
    const int64_t n = (int64_t)v.size();
    const int nt = (int)std::min<int64_t>(host_threads(), std::max<int64_t>(1, n / 4096));
    std::vector<int64_t> cut(nt + 1);
    for (int i = 0; i <= nt; ++i) cut[i] = n * i / nt;
    {
        std::vector<std::thread> th;
        for (int i = 0; i < nt; ++i)
            th.emplace_back([&, i] { std::sort(v.begin() + cut[i], v.begin() + cut[i + 1]); });
        for (auto &t : th) t.join();
    }
    for (int width = 1; width < nt; width *= 2) {
        std::vector<std::thread> th;
        for (int i = 0; i + width < nt; i += 2 * width) {
            const int64_t a = cut[i], m = cut[i + width], b = cut[std::min(i + 2 * width, nt)];
            th.emplace_back([&v, a, m, b] { std::inplace_merge(v.begin() + a, v.begin() + m, v.begin() + b); });
        }
        for (auto &t : th) t.join();
    }
}

static int schwarz_host(int N, int64_t E, const int64_t *gid, const uint8_t *dir, const double *len,
                        SchwarzHost &out)
{
    const int nq = N + 1, ne = N + 3;
    const int64_t np = (int64_t)nq * nq * nq, nL = E * np, ne3 = (int64_t)ne * ne * ne;
    if (N < 2) {
        set_error("Schwarz smoother needs N >= 2 on its levels (got N = %d)", N);
        return SEM_EINVAL;
    }
    if (E * ne3 >= (int64_t)1 << 31) {
        set_error("Schwarz smoother: level too large for 32-bit indices");
        return SEM_EINVAL;
    }
    // copies of every nonzero pointer, sorted by (pointer, copy)
    std::vector<int64_t> ord;
    {
        std::vector<std::pair<int64_t, int64_t>> gl;
        gl.reserve(nL);
        for (int64_t l = 0; l < nL; ++l)
            if (gid[l] != 0) gl.emplace_back(gid[l], l);
        parallel_sort(gl);
        ord.resize(gl.size());
        for (size_t i = 0; i < gl.size(); ++i) ord[i] = gl[i].second;
    }
    auto first_of = [&](int64_t g) {
        return std::lower_bound(ord.begin(), ord.end(), g, [&](int64_t l, int64_t v) { return gid[l] < v; });
    };
    auto copy_in = [&](int64_t g, int64_t e) -> int64_t {  // copy of pointer g in element e
        if (g == 0) return -1;
        for (auto lo = first_of(g); lo != ord.end() && gid[*lo] == g; ++lo)
            if (*lo / np == e) return *lo;
        return -1;
    };
    auto lidx = [&](const int64_t c[3]) { return (c[2] * nq + c[1]) * nq + c[0]; };
    // face links: neighbour across face (d, side) and the affine map of e's
    // face coordinates into it, from the face-interior node (1, 1) and its
    // neighbours along the two face axes
    std::vector<FaceLink> link(E * 6);
    for (int64_t e = 0; e < E; ++e)
        for (int d = 0; d < 3; ++d)
            for (int side = 0; side < 2; ++side) {
                FaceLink &F = link[e * 6 + d * 2 + side];
                const int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
                int64_t c0[3];
                c0[d] = side ? N : 0;
                c0[d1] = 1;
                c0[d2] = 1;
                const int64_t g0 = gid[e * np + lidx(c0)];
                int64_t q0 = -1;
                if (g0 != 0)
                    for (auto lo = first_of(g0); lo != ord.end() && gid[*lo] == g0; ++lo)
                        if (*lo / np != e) {
                            q0 = *lo;
                            break;
                        }
                if (q0 < 0) continue;  // boundary face
                F.nb = q0 / np;
                const int64_t p0 = q0 % np;
                const int64_t A0[3] = {p0 % nq, (p0 / nq) % nq, p0 / ((int64_t)nq * nq)};
                bool seen[3] = {false, false, false};
                for (int k = 0; k < 2; ++k) {
                    const int dk = k == 0 ? d1 : d2;
                    int64_t c1[3] = {c0[0], c0[1], c0[2]};
                    const int step = N >= 3 ? 1 : -1;
                    c1[dk] += step;
                    const int64_t q1 = copy_in(gid[e * np + lidx(c1)], F.nb);
                    if (q1 < 0) {
                        set_error("Schwarz smoother: element %lld face %d is not conforming", (long long)e,
                                  d * 2 + side);
                        return SEM_EMESH;
                    }
                    const int64_t p1 = q1 % np;
                    const int64_t A1[3] = {p1 % nq, (p1 / nq) % nq, p1 / ((int64_t)nq * nq)};
                    int ax = -1, sg = 0, moved = 0;
                    for (int a = 0; a < 3; ++a)
                        if (A1[a] != A0[a]) {
                            ax = a;
                            sg = (int)((A1[a] - A0[a]) * step);
                            ++moved;
                        }
                    if (moved != 1 || (sg != 1 && sg != -1) || seen[ax]) {
                        set_error("Schwarz smoother: bad face map at element %lld", (long long)e);
                        return SEM_EMESH;
                    }
                    F.rax[dk] = ax;
                    F.sgn[dk] = sg;
                    seen[ax] = true;
                }
                int dn = 0;
                while (seen[dn]) ++dn;
                if (A0[dn] != 0 && A0[dn] != N) {
                    set_error("Schwarz smoother: face of element %lld does not meet a face", (long long)e);
                    return SEM_EMESH;
                }
                F.rax[d] = dn;                      // face normal axis of nb
                F.sgn[d] = (A0[dn] == 0) ? 1 : -1;  // inward step in nb
                for (int a = 0; a < 3; ++a) F.org[a] = A0[a];
            }
    // copy at extended coordinates c (each in [-1, N+1]) of element e, by
    // crossing one face per out-of-range axis; -1 outside the domain
    auto walk = [&](int64_t e, int64_t c[3]) -> int64_t {
        for (int guard = 0; guard < 4; ++guard) {
            int d = -1;
            for (int a = 0; a < 3; ++a)
                if (c[a] < 0 || c[a] > N) {
                    d = a;
                    break;
                }
            if (d < 0) return e * np + lidx(c);
            const FaceLink &F = link[e * 6 + d * 2 + (c[d] < 0 ? 0 : 1)];
            if (F.nb < 0) return -1;
            const int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
            const int64_t k1 = std::min<int64_t>(std::max<int64_t>(c[d1], 0), N);
            const int64_t k2 = std::min<int64_t>(std::max<int64_t>(c[d2], 0), N);
            int64_t cn[3] = {F.org[0], F.org[1], F.org[2]};
            // clamped face point relative to (1, 1), then the offsets that are
            // still outside along the face axes, then one step into nb
            cn[F.rax[d1]] += F.sgn[d1] * (k1 - 1 + (c[d1] - k1));
            cn[F.rax[d2]] += F.sgn[d2] * (k2 - 1 + (c[d2] - k2));
            cn[F.rax[d]] += F.sgn[d];
            e = F.nb;
            c[0] = cn[0];
            c[1] = cn[1];
            c[2] = cn[2];
        }
        return -1;
    };
    std::vector<double> D(nq * nq), rho(nq);
    SEM_TRY(host_gll(N, nullptr, rho.data(), D.data()));
    out.S.assign((size_t)E * 3 * ne * ne, 0.0f);
    out.lam.assign((size_t)E * 3 * ne, 1.0f);
    out.ix.assign((size_t)E * ne3, -1);
    auto face_dirichlet = [&](int64_t e, int d, int side) {
        const int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
        for (int v = 0; v < nq; ++v)
            for (int u = 0; u < nq; ++u) {
                int64_t c[3];
                c[d] = side ? N : 0;
                c[d1] = u;
                c[d2] = v;
                if (!dir[e * np + lidx(c)]) return false;
            }
        return true;
    };
    // every element's FDM modes and extended-point map, independently
    parallel_ranges(E, [&](int64_t e0, int64_t e1) {
        std::vector<uint8_t> keep(3 * ne);
        for (int64_t e = e0; e < e1; ++e) {
            for (int d = 0; d < 3; ++d) {
                const FaceLink &Fl = link[e * 6 + d * 2], &Fh = link[e * 6 + d * 2 + 1];
                const double Lm = Fl.nb >= 0 ? len[Fl.nb * 3 + Fl.rax[d]] : -1.0;
                const double Lp = Fh.nb >= 0 ? len[Fh.nb * 3 + Fh.rax[d]] : -1.0;
                fdm_direction(N, rho.data(), D.data(), len[e * 3 + d], Lm, Lp, face_dirichlet(e, d, 0),
                              face_dirichlet(e, d, 1), out.S.data() + ((size_t)e * 3 + d) * ne * ne,
                              out.lam.data() + ((size_t)e * 3 + d) * ne, keep.data() + d * ne);
            }
            for (int c = 0; c < ne; ++c)
                for (int b = 0; b < ne; ++b)
                    for (int a = 0; a < ne; ++a) {
                        if (!(keep[a] && keep[ne + b] && keep[2 * ne + c])) continue;
                        int64_t cc[3] = {a - 1, b - 1, c - 1};
                        out.ix[(size_t)e * ne3 + ((int64_t)c * ne + b) * ne + a] = (int32_t)walk(e, cc);
                    }
        }
    });
    // offsets of the local-solution entries landing on every copy (only the
    // counts, off[l + 1] - off[l], are used)
    out.off.assign(nL + 1, 0);
    for (int64_t t = 0; t < E * ne3; ++t)
        if (out.ix[t] >= 0) ++out.off[out.ix[t] + 1];
    std::partial_sum(out.off.begin(), out.off.end(), out.off.begin());
    // weight: mask / (subdomains containing the node), summed over its copies
    std::vector<double> node_cov(nL);
    for (int64_t l = 0; l < nL; ++l) node_cov[l] = out.off[l + 1] - out.off[l];
    for (size_t i = 0; i < ord.size();) {
        size_t j = i;
        double acc = 0.0;
        while (j < ord.size() && gid[ord[j]] == gid[ord[i]]) acc += out.off[ord[j] + 1] - out.off[ord[j]], ++j;
        for (size_t k = i; k < j; ++k) node_cov[ord[k]] = acc;
        i = j;
    }
    out.w.assign(nL, 0.0f);
    for (int64_t l = 0; l < nL; ++l)
        out.w[l] = (!dir[l] && node_cov[l] > 0.0) ? (float)(1.0 / node_cov[l]) : 0.0f;
    return SEM_OK;
}

int build_schwarz(Level &L, hipStream_t s)
{
    if (L.sz_ix) return SEM_OK;
    if ((int64_t)L.len.size() != 3 * L.E) {
        set_error("Schwarz smoother: element extents missing");
        return SEM_EINVAL;
    }
    std::vector<int64_t> gid(L.nL);
    std::vector<uint8_t> dir(L.nL);
    SEM_HIP(hipMemcpyAsync(gid.data(), L.gid, sizeof(int64_t) * L.nL, hipMemcpyDeviceToHost, s));
    SEM_HIP(hipMemcpyAsync(dir.data(), L.dir, sizeof(uint8_t) * L.nL, hipMemcpyDeviceToHost, s));
    SEM_HIP(hipStreamSynchronize(s));
    SchwarzHost H;
    SEM_TRY(schwarz_host(L.N, L.E, gid.data(), dir.data(), L.len.data(), H));
    // compact extension map and the lists of copies receiving extension values
    const int ne = L.N + 3, nq = L.nq;
    const int next = ne * ne * ne - nq * nq * nq;
    const int64_t E = L.E, ne3 = (int64_t)ne * ne * ne;
    std::vector<int32_t> hx((size_t)E * next, -1);
    parallel_ranges(E, [&](int64_t e0, int64_t e1) {
        for (int64_t e = e0; e < e1; ++e)
            for (int c = 0; c < ne; ++c)
                for (int b = 0; b < ne; ++b)
                    for (int a = 0; a < ne; ++a) {
                        const bool inner = a > 0 && a < ne - 1 && b > 0 && b < ne - 1 && c > 0 && c < ne - 1;
                        if (inner) continue;
                        hx[e * next + schwarz_ext_slot(ne, a, b, c)] =
                            H.ix[(size_t)e * ne3 + ((int64_t)c * ne + b) * ne + a];
                    }
    });
    // copies receiving extension values (ascending) and, per copy, its
    // extension entries in ascending slot order: a counting pass over slots
    std::vector<int32_t> cnt(L.nL + 1, 0);
    for (int64_t slot = 0; slot < E * next; ++slot)
        if (hx[slot] >= 0) ++cnt[hx[slot] + 1];
    std::vector<int32_t> rc, off, src;
    std::vector<int32_t> pos(L.nL, -1);  // first list position of each receiving copy
    int64_t total = 0;
    for (int64_t q = 0; q < L.nL; ++q)
        if (cnt[q + 1] > 0) {
            rc.push_back((int32_t)q);
            off.push_back((int32_t)total);
            pos[q] = (int32_t)total;
            total += cnt[q + 1];
        }
    off.push_back((int32_t)total);
    src.assign(total, 0);
    for (int64_t slot = 0; slot < E * next; ++slot)
        if (hx[slot] >= 0) src[pos[hx[slot]]++] = (int32_t)slot;
    auto up = [&](void **dst, const void *src_, size_t bytes) -> int {
        SEM_HIP(hipMalloc(dst, bytes > 0 ? bytes : 4));
        if (bytes) SEM_HIP(hipMemcpyAsync(*dst, src_, bytes, hipMemcpyHostToDevice, s));
        return SEM_OK;
    };
    SEM_TRY(up((void **)&L.sz_ix, hx.data(), sizeof(int32_t) * hx.size()));
    SEM_TRY(up((void **)&L.sz_S, H.S.data(), sizeof(float) * H.S.size()));
    SEM_TRY(up((void **)&L.sz_lam, H.lam.data(), sizeof(float) * H.lam.size()));
    SEM_TRY(up((void **)&L.sz_rc, rc.data(), sizeof(int32_t) * rc.size()));
    SEM_TRY(up((void **)&L.sz_off, off.data(), sizeof(int32_t) * off.size()));
    SEM_TRY(up((void **)&L.sz_src, src.data(), sizeof(int32_t) * src.size()));
    SEM_TRY(up((void **)&L.sz_w, H.w.data(), sizeof(float) * H.w.size()));
    SEM_HIP(hipStreamSynchronize(s));
    L.sz_ne = ne;
    L.sz_next = next;
    L.sz_nrc = (int64_t)rc.size();
    return SEM_OK;
}

// ------------------------------------------------------------------ kernels
// Local FDM solves, EPB elements per workgroup, ne^2 threads per element.
// Every 1D transform is applied by threads that each own one whole line of
// the direction transformed: the c-lines by thread (a, b) in registers
// (gathered inputs, and the final transform back), the b-lines by thread
// (a, k) and the a-lines by thread (b, k), read from and written to two LDS
// buffers, so a thread reads ne values per transform rather than ne^2, and the
// forward a transform, the division by the eigenvalue sum and the transform
// back along a run in one pass on the thread's row.  The rows of the
// element's S matrices are read from LDS (every lane of the element reads the
// same row).  Own points are read directly and written to acc; extension
// points are gathered through the compact map and (ASM) written to U.  The
// eigenbases and the extension map of an element are loaded once and serve
// every vector of the batch in turn.  FP32.
template <int NE>
struct FdmShape {
    static constexpr int NQ = NE - 2, NE2 = NE * NE, THREADS = 256;
    static constexpr int EPB = THREADS / NE2;
    static constexpr int NEXT = NE * NE * NE - NQ * NQ * NQ;
    static constexpr int LDP = NE + 1;
    static constexpr int NEP = (NE + 3) & ~3;  // S rows padded to 16 bytes
};

template <int NE, bool EXT_OUT>
__global__ void __launch_bounds__(FdmShape<NE>::THREADS)
fdm_kernel(int64_t E, const int32_t *__restrict__ ix, const float *__restrict__ Sg,
           const float *__restrict__ lamg, const float *__restrict__ r, const float *__restrict__ t,
           int64_t ld, float *__restrict__ acc, float *__restrict__ U, float h1, float h2, VSet vs)
{
    using F = FdmShape<NE>;
    constexpr int NQ = F::NQ, NE2 = F::NE2, EPB = F::EPB, NEXT = F::NEXT, LDP = F::LDP, NEP = F::NEP;
    constexpr int NP = NQ * NQ * NQ;
    __shared__ __align__(16) float sS[EPB][3][NE][NEP];  // Sx, Sy, Sz of each element, rows [m][.]
    __shared__ float sl[EPB][3][NE];                     // eigenvalues along x, y, z
    __shared__ float sa[EPB][NE][NE][LDP];               // [c][b][a]
    __shared__ float sb[EPB][NE][NE][LDP];
    const int tid = threadIdx.x;
    const int el = tid / NE2, ij = tid - el * NE2;
    const int a = ij % NE, b = ij / NE;  // also (x, k) of the line-owner stages
    const bool lane = el < EPB;
    const bool acol = a == 0 || a == NE - 1 || b == 0 || b == NE - 1;  // border column
    // extension slots of this column: ebase + c (border column), or ebase and
    // ebase + 1 for c = 0 and c = ne-1 (inner column)
    const int ebase = schwarz_ext_slot(NE, a, b, 0);
    const int64_t groups = (E + EPB - 1) / EPB;
    for (int64_t g = blockIdx.x; g < groups; g += gridDim.x) {
        const int64_t e = g * EPB + el;
        const bool act = lane && e < E;
        __syncthreads();  // LDS of the previous group consumed
        // the element's eigenbases and eigenvalues and this column's
        // extension copies, once for every vector of the batch
        int32_t q[NE];
        if (act) {
            const float *Se = Sg + e * 3 * NE2;
#pragma unroll
            for (int d = 0; d < 3; ++d) sS[el][d][b][a] = Se[d * NE2 + ij];
            if (ij < 3 * NE) (&sl[el][0][0])[ij] = lamg[e * 3 * NE + ij];
            const int32_t *ixe = ix + e * NEXT;
            if (acol) {
#pragma unroll
                for (int c = 0; c < NE; ++c) q[c] = ixe[ebase + c];
            } else {
                q[0] = ixe[ebase];
                q[NE - 1] = ixe[ebase + 1];
            }
        }
        __syncthreads();  // sS, sl ready
        for (int f = 0; f < vs.n; ++f) {
            const int64_t v = vs.at(f);
            const float *rv = r + v * ld;
            const float *tv = t ? t + v * ld : nullptr;
            float vv[NE];
            if (act) {
                auto gather = [&](int32_t qq) {
                    return qq >= 0 ? (tv ? rv[qq] - tv[qq] : rv[qq]) : 0.0f;
                };
                if (acol) {
#pragma unroll
                    for (int c = 0; c < NE; ++c) vv[c] = gather(q[c]);
                } else {
                    const float *re = rv + e * NP + (b - 1) * NQ + (a - 1);
                    const float *te = tv ? tv + e * NP + (b - 1) * NQ + (a - 1) : nullptr;
                    vv[0] = gather(q[0]);
#pragma unroll
                    for (int c = 1; c < NE - 1; ++c)
                        vv[c] = te ? re[(c - 1) * NQ * NQ] - te[(c - 1) * NQ * NQ] : re[(c - 1) * NQ * NQ];
                    vv[NE - 1] = gather(q[NE - 1]);
                }
                // modes along c: w[k] = sum_c Sz[c][k] vv[c]
                float w[NE];
#pragma unroll
                for (int k = 0; k < NE; ++k) w[k] = 0.0f;
#pragma unroll
                for (int c = 0; c < NE; ++c) {
                    const float *Sr = &sS[el][2][c][0];
#pragma unroll
                    for (int k = 0; k < NE; ++k) w[k] += Sr[k] * vv[c];
                }
#pragma unroll
                for (int k = 0; k < NE; ++k) sa[el][k][b][a] = w[k];
            }
            __syncthreads();
            if (act) {
                // modes along b on the line (a, k = b): y[j] = sum_m Sy[m][j] x[m]
                const int k = b;
                float x[NE], y[NE];
#pragma unroll
                for (int m = 0; m < NE; ++m) x[m] = sa[el][k][m][a];
#pragma unroll
                for (int j = 0; j < NE; ++j) y[j] = 0.0f;
#pragma unroll
                for (int m = 0; m < NE; ++m) {
                    const float *Sr = &sS[el][1][m][0];
#pragma unroll
                    for (int j = 0; j < NE; ++j) y[j] += Sr[j] * x[m];
                }
#pragma unroll
                for (int j = 0; j < NE; ++j) sb[el][k][j][a] = y[j];
            }
            __syncthreads();
            if (act) {
                // the row (b = a, k = b) along a: modes, division by the
                // eigenvalue sum, and back
                const int bb = a, k = b;
                float x[NE], y[NE];
#pragma unroll
                for (int m = 0; m < NE; ++m) x[m] = sb[el][k][bb][m];
#pragma unroll
                for (int i = 0; i < NE; ++i) y[i] = 0.0f;
#pragma unroll
                for (int m = 0; m < NE; ++m) {
                    const float *Sr = &sS[el][0][m][0];
#pragma unroll
                    for (int i = 0; i < NE; ++i) y[i] += Sr[i] * x[m];
                }
                const float lyz = sl[el][1][bb], lzk = sl[el][2][k];
#pragma unroll
                for (int i = 0; i < NE; ++i) y[i] *= __builtin_amdgcn_rcpf(h1 * (sl[el][0][i] + lyz + lzk) + h2);
                // the rows of Sx are read again below rather than kept in
                // registers from the forward pass (that would cost ne^2 VGPRs)
                asm volatile("" ::: "memory");
#pragma unroll
                for (int i = 0; i < NE; ++i) {
                    const float *Sr = &sS[el][0][i][0];
                    float sum = 0.0f;
#pragma unroll
                    for (int m = 0; m < NE; ++m) sum += Sr[m] * y[m];
                    sa[el][k][bb][i] = sum;
                }
            }
            __syncthreads();
            if (act) {
                // back along b on the line (a, k = b)
                const int k = b;
                float x[NE];
#pragma unroll
                for (int m = 0; m < NE; ++m) x[m] = sa[el][k][m][a];
#pragma unroll
                for (int j = 0; j < NE; ++j) {
                    const float *Sr = &sS[el][1][j][0];
                    float sum = 0.0f;
#pragma unroll
                    for (int m = 0; m < NE; ++m) sum += Sr[m] * x[m];
                    sb[el][k][j][a] = sum;
                }
            }
            __syncthreads();
            if (act) {
                // back along c on the column (a, b), in registers
                float w[NE];
#pragma unroll
                for (int k = 0; k < NE; ++k) w[k] = sb[el][k][b][a];
                float *acce = acc + v * ld + e * NP + (b - 1) * NQ + (a - 1);
                float *Ue = EXT_OUT ? U + v * E * NEXT + e * NEXT : nullptr;
                auto line = [&](int c) {
                    const float *Sr = &sS[el][2][c][0];
                    float sum = 0.0f;
#pragma unroll
                    for (int k = 0; k < NE; ++k) sum += Sr[k] * w[k];
                    return sum;
                };
                if (acol) {
                    if (EXT_OUT)
#pragma unroll
                        for (int c = 0; c < NE; ++c) Ue[ebase + c] = line(c);
                } else {
#pragma unroll
                    for (int c = 1; c < NE - 1; ++c) acce[(c - 1) * NQ * NQ] = line(c);
                    if (EXT_OUT) {
                        Ue[ebase] = line(0);
                        Ue[ebase + 1] = line(NE - 1);
                    }
                }
            }
            // the next vector's first LDS writes (sa) follow this vector's
            // last sa reads (before the barrier above); its sb writes follow
            // a barrier every thread reaches after the reads of sb here
        }
    }
}

// Extension values of the neighbours' local solutions added into the copies
// that receive them, every vector of the batch in one pass over the lists: a
// thread holds the first kAsmRegs source indices of its copy in registers
// (a copy interior to a box of hexahedra receives from at most 7 extended
// subdomains), so the lists are read once per call; the summation order per
// copy is the list order for every vector.
constexpr int kAsmRegs = 8;

__global__ void asm_ext_kernel(int64_t nrc, const int32_t *__restrict__ rc,
                               const int32_t *__restrict__ off, const int32_t *__restrict__ src,
                               const float *__restrict__ U, int64_t ldU, float *__restrict__ acc,
                               int64_t ld, VSet vs)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nrc;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t c = rc[i];
        const int32_t q0 = off[i], nq = off[i + 1] - q0;
        int32_t sq[kAsmRegs];
#pragma unroll
        for (int j = 0; j < kAsmRegs; ++j) sq[j] = j < nq ? src[q0 + j] : 0;
        for (int q = 0; q < vs.n; ++q) {
            const int64_t v = vs.at(q);
            const float *Uv = U + v * ldU;
            float s = acc[v * ld + c];
#pragma unroll
            for (int j = 0; j < kAsmRegs; ++j)
                if (j < nq) s += Uv[sq[j]];
            for (int j = kAsmRegs; j < nq; ++j) s += Uv[src[q0 + j]];
            acc[v * ld + c] = s;
        }
    }
}

int launch_schwarz(const Level &L, bool ras, const float *r, const float *t, float *U, float *acc,
                   const VSet &vs, double h1, double h2, hipStream_t s)
{
    if (vs.n <= 0) return SEM_OK;
    if (!L.sz_ix) {
        set_error("Schwarz smoother not built on this level");
        return SEM_EINVAL;
    }
    // one workgroup per EPB elements (a persistent grid capped at the
    // resident count, or at 8 per CU, was slower: the last, partial round of
    // workgroups leaves CUs idle)
#define SEM_FDM(NE)                                                                                   \
    case NE: {                                                                                        \
        const dim3 grid((unsigned)((L.E + FdmShape<NE>::EPB - 1) / FdmShape<NE>::EPB));              \
        if (ras)                                                                                      \
            hipLaunchKernelGGL((fdm_kernel<NE, false>), grid, dim3(FdmShape<NE>::THREADS), 0, s, L.E, \
                               L.sz_ix, L.sz_S, L.sz_lam, r, t, L.nL, acc, U, (float)h1, (float)h2, vs); \
        else                                                                                          \
            hipLaunchKernelGGL((fdm_kernel<NE, true>), grid, dim3(FdmShape<NE>::THREADS), 0, s, L.E,  \
                               L.sz_ix, L.sz_S, L.sz_lam, r, t, L.nL, acc, U, (float)h1, (float)h2, vs); \
        SEM_HIP(hipGetLastError());                                                                   \
        break;                                                                                        \
    }
    switch (L.sz_ne) {
        SEM_FDM(5) SEM_FDM(6) SEM_FDM(7) SEM_FDM(8) SEM_FDM(9) SEM_FDM(10) SEM_FDM(11)
    default: set_error("Schwarz smoother: unsupported order N = %d", L.N); return SEM_EINVAL;
    }
#undef SEM_FDM
    if (!ras && L.sz_nrc > 0) {
        const int64_t ldU = L.E * (int64_t)L.sz_next;
        const int64_t groups = (L.sz_nrc + 255) / 256;
        const unsigned g = (unsigned)std::min<int64_t>(groups, (int64_t)(L.n_cu > 0 ? L.n_cu : 256) * 8);
        hipLaunchKernelGGL(asm_ext_kernel, dim3(g), dim3(256), 0, s, L.sz_nrc, L.sz_rc,
                           L.sz_off, L.sz_src, (const float *)U, ldU, acc, L.nL, vs);
        SEM_HIP(hipGetLastError());
    }
    return SEM_OK;
}

}  // namespace semx

using namespace semx;

extern "C" int sem_schwarz_setup_host(int N, int64_t E, const int64_t *gid, const uint8_t *dirichlet,
                                      const double *len, int32_t *ix, float *S, float *lam,
                                      int32_t *cover, float *weight)
{
    if (!gid || !len || E < 1 || N < 1) {
        set_error("sem_schwarz_setup_host: bad argument");
        return SEM_EINVAL;
    }
    const int64_t nL = E * (int64_t)(N + 1) * (N + 1) * (N + 1);
    std::vector<uint8_t> zero;
    if (!dirichlet) {
        zero.assign(nL, 0);
        dirichlet = zero.data();
    }
    SchwarzHost H;
    const int rc = schwarz_host(N, E, gid, dirichlet, len, H);
    if (rc != SEM_OK) return rc;
    if (ix) std::copy(H.ix.begin(), H.ix.end(), ix);
    if (S) std::copy(H.S.begin(), H.S.end(), S);
    if (lam) std::copy(H.lam.begin(), H.lam.end(), lam);
    if (cover)
        for (int64_t l = 0; l < nL; ++l) cover[l] = H.off[l + 1] - H.off[l];
    if (weight) std::copy(H.w.begin(), H.w.end(), weight);
    return SEM_OK;
}
