// C ABI of libsem: handle lifecycle, setup, operator and gather-scatter entry
// points, introspection.  The solver entry lives in solve.hip.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "sem_internal.h"

namespace semx {

static thread_local char g_err[1024] = "";

void set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

static void free_level(Level &L)
{
    free_schwarz(L);
    free_coarse_csr(L);
    void *ptrs[] = {L.G, L.B, L.G32, L.B32, L.W, L.W32, L.gid, L.dir, L.perm, L.offs,
                    L.chunk_perm, L.over,
                    L.D, L.D32, L.Jc, L.Jc32, L.Dinv, L.Dinv32};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    L = Level{};
}

// mean extent of each element along r, s, t: the mean distance between the end
// nodes of the element's node lines in that direction
__global__ void elem_len_kernel(int64_t E, int nq, const double *__restrict__ x,
                                const double *__restrict__ y, const double *__restrict__ z,
                                double *__restrict__ len)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    const int N = nq - 1, np = nq * nq * nq;
    const double *X[3] = {x + e * np, y + e * np, z + e * np};
    for (int d = 0; d < 3; ++d) {
        double acc = 0.0;
        for (int v = 0; v < nq; ++v)
            for (int u = 0; u < nq; ++u) {
                int p0, p1;  // line along d through (u, v) of the other two axes
                if (d == 0) { p0 = (v * nq + u) * nq; p1 = p0 + N; }
                else if (d == 1) { p0 = v * nq * nq + u; p1 = p0 + N * nq; }
                else { p0 = v * nq + u; p1 = p0 + N * nq * nq; }
                double s2 = 0.0;
                for (int c = 0; c < 3; ++c) {
                    const double dd = X[c][p1] - X[c][p0];
                    s2 += dd * dd;
                }
                acc += sqrt(s2);
            }
        len[e * 3 + d] = acc / (nq * nq);
    }
}

__global__ void cast_f64_to_f32_kernel(int64_t n, const double *__restrict__ a, float *__restrict__ b)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) b[t] = (float)a[t];
}

static int cast_to_f32(int64_t n, const double *a, float *b, hipStream_t s)
{
    if (n == 0) return SEM_OK;
    const int bs = 256;
    hipLaunchKernelGGL(cast_f64_to_f32_kernel, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, s,
                       n, a, b);
    SEM_HIP(hipGetLastError());
    return SEM_OK;
}

// coarse copy (e, kc, jc, ic) takes the global pointer and Dirichlet flag of
// the fine copy (e, f(kc), f(jc), f(ic)), where f maps coarse line positions
// to fine ones with f(0) = 0, f(Nc) = Nf and f(Nc - a) = Nf - f(a); the map
// commutes with every reorientation of an edge or face, so copies of one
// coarse node on neighbouring elements land on copies of one fine node.
__global__ void coarse_ids_kernel(int64_t E, int nqf, int nqc, const int *__restrict__ fmap,
                                  const int64_t *__restrict__ gid_f, const uint8_t *__restrict__ dir_f,
                                  int64_t *__restrict__ gid_c, uint8_t *__restrict__ dir_c)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int npc = nqc * nqc * nqc, npf = nqf * nqf * nqf;
    if (t >= E * npc) return;
    const int64_t e = t / npc;
    const int p = (int)(t - e * npc);
    const int ic = p % nqc, jc = (p / nqc) % nqc, kc = p / (nqc * nqc);
    const int64_t q = e * npf + fmap[ic] + nqf * (fmap[jc] + nqf * fmap[kc]);
    gid_c[t] = gid_f[q];
    dir_c[t] = dir_f[q];
}

static void line_map(int Nf, int Nc, int *f)
{
    f[0] = 0;
    f[Nc] = Nf;
    for (int a = 1; a < Nc; ++a) {
        const double x = (double)a * Nf / Nc;
        const double fl = std::floor(x);
        int v;
        if (x - fl == 0.5)  // tie: round toward the middle of the line
            v = (x < 0.5 * Nf) ? (int)fl + 1 : (int)fl;
        else
            v = (int)std::lround(x);
        f[a] = v;
    }
}

static int alloc_copy(void **dst, const void *src, size_t bytes, hipStream_t s)
{
    SEM_HIP(hipMalloc(dst, bytes));
    SEM_HIP(hipMemcpyAsync(*dst, src, bytes, hipMemcpyHostToDevice, s));
    return SEM_OK;
}

// Build one level from device coordinates/pointers: D, maps, weights,
// geometry (FP64, and FP32 copies when `f32`).
static int build_level(Level &L, int N, int64_t E, const double *x, const double *y,
                       const double *z, const int64_t *gid, const uint8_t *dir, bool f32,
                       int *bad, hipStream_t s)
{
    L.gid = const_cast<int64_t *>(gid);
    L.dir = const_cast<uint8_t *>(dir);
    {
        int dev = 0, ncu = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
            L.n_cu = ncu;
    }
    L.N = N;
    L.nq = N + 1;
    L.np = L.nq * L.nq * L.nq;
    L.E = E;
    L.nL = E * L.np;
    // D followed by rho (geometry reads rho after D)
    std::vector<double> hD(L.nq * L.nq + L.nq);
    SEM_TRY(host_gll(N, nullptr, hD.data() + L.nq * L.nq, hD.data()));
    SEM_TRY(alloc_copy((void **)&L.D, hD.data(), sizeof(double) * hD.size(), s));
    std::vector<float> hD32(L.nq * L.nq);
    for (int t = 0; t < L.nq * L.nq; ++t) hD32[t] = (float)hD[t];
    SEM_TRY(alloc_copy((void **)&L.D32, hD32.data(), sizeof(float) * hD32.size(), s));
    SEM_HIP(hipStreamSynchronize(s));  // host vectors go out of scope
    SEM_TRY(build_maps(L, gid, dir, x, y, z, bad, s));
    SEM_HIP(hipMalloc(&L.G, sizeof(double) * 6 * L.nL));
    SEM_HIP(hipMalloc(&L.B, sizeof(double) * L.nL));
    SEM_TRY(launch_geometry(L, x, y, z, L.G, L.B, bad, s));
    {
        double *dlen = nullptr;
        SEM_HIP(hipMalloc(&dlen, sizeof(double) * 3 * E));
        hipLaunchKernelGGL(elem_len_kernel, dim3((unsigned)((E + 127) / 128)), dim3(128), 0, s, E, L.nq,
                           x, y, z, dlen);
        hipError_t e1 = hipGetLastError();
        L.len.assign(3 * E, 0.0);
        if (e1 == hipSuccess)
            e1 = hipMemcpyAsync(L.len.data(), dlen, sizeof(double) * 3 * E, hipMemcpyDeviceToHost, s);
        if (e1 == hipSuccess) e1 = hipStreamSynchronize(s);
        (void)hipFree(dlen);
        SEM_HIP(e1);
    }
    if (f32) {
        SEM_HIP(hipMalloc(&L.G32, sizeof(float) * 6 * L.nL));
        SEM_HIP(hipMalloc(&L.B32, sizeof(float) * L.nL));
        SEM_TRY(cast_to_f32(6 * L.nL, L.G, L.G32, s));
        SEM_TRY(cast_to_f32(L.nL, L.B, L.B32, s));
    }
    return SEM_OK;
}

static int setup_impl(const sem_mesh *m, const sem_setup_opts *o, hipStream_t s, sem_handle h)
{
    const int N = m->N;
    const int64_t E = m->E;
    const int nq = N + 1;
    const int64_t nL = E * nq * nq * nq;
    SEM_HIP(hipGetDevice(&h->device));
    SEM_TRY(noalloc_attach(h->device));
    int levels[kMaxLevels] = {N, 0, 0, 0};
    int nlev = 1;
    if (o && o->pmg) {
        nlev = o->n_levels;
        for (int l = 0; l < nlev; ++l) levels[l] = o->levels[l];
    }
    h->n_levels = nlev;

    int *bad = nullptr;
    SEM_HIP(hipMalloc(&bad, sizeof(int)));
    SEM_HIP(hipMemsetAsync(bad, 0, sizeof(int), s));

    double *x = nullptr, *y = nullptr, *z = nullptr;
    int64_t *gid = nullptr;
    uint8_t *dir = nullptr;
    int rc = SEM_OK;
    do {
        if ((rc = alloc_copy((void **)&x, m->x, sizeof(double) * nL, s))) break;
        if ((rc = alloc_copy((void **)&y, m->y, sizeof(double) * nL, s))) break;
        if ((rc = alloc_copy((void **)&z, m->z, sizeof(double) * nL, s))) break;
        if ((rc = alloc_copy((void **)&gid, m->gid, sizeof(int64_t) * nL, s))) break;
        if (m->dirichlet) {
            if ((rc = alloc_copy((void **)&dir, m->dirichlet, nL, s))) break;
        } else {
            if (hipMalloc(&dir, nL) != hipSuccess || hipMemsetAsync(dir, 0, nL, s) != hipSuccess) {
                set_error("setup: allocation of the Dirichlet mask failed");
                rc = SEM_ENOMEM;
                break;
            }
        }
        const bool f32_fine = nlev > 1;
        rc = build_level(h->lv[0], N, E, x, y, z, gid, dir, f32_fine, bad, s);
        gid = nullptr;  // owned by the level from here on, also on failure
        dir = nullptr;
        if (rc != SEM_OK) break;
        // coarse levels: coordinates interpolated from the finer level,
        // pointers by the line map.  px/py/pz hold the finer level's
        // coordinates (level 0: the uploaded ones).
        double *px = x, *py = y, *pz = z;
        for (int l = 1; l < nlev && rc == SEM_OK; ++l) {
            Level &F = h->lv[l - 1];
            const int Nc = levels[l];
            const int nqc = Nc + 1;
            const int64_t nLc = E * nqc * nqc * nqc;
            double xf[kMaxN + 1], xc[kMaxN + 1];
            host_gll(F.N, xf, nullptr, nullptr);
            host_gll(Nc, xc, nullptr, nullptr);
            std::vector<double> Jfc(nqc * F.nq), Jcf(F.nq * nqc);
            host_interp(F.nq, xf, nqc, xc, Jfc.data());   // fine nodes -> coarse points
            host_interp(nqc, xc, F.nq, xf, Jcf.data());   // coarse nodes -> fine points
            std::vector<float> Jcf32(Jcf.begin(), Jcf.end());
            int hmap[kMaxN + 1];
            line_map(F.N, Nc, hmap);
            double *dJfc = nullptr, *xcv = nullptr, *ycv = nullptr, *zcv = nullptr;
            int64_t *gidc = nullptr;
            uint8_t *dirc = nullptr;
            int *fmap = nullptr;
            rc = alloc_copy((void **)&dJfc, Jfc.data(), sizeof(double) * Jfc.size(), s);
            if (rc == SEM_OK) rc = alloc_copy((void **)&F.Jc, Jcf.data(), sizeof(double) * Jcf.size(), s);
            if (rc == SEM_OK)
                rc = alloc_copy((void **)&F.Jc32, Jcf32.data(), sizeof(float) * Jcf32.size(), s);
            if (rc == SEM_OK) rc = alloc_copy((void **)&fmap, hmap, sizeof(int) * nqc, s);
            if (rc == SEM_OK &&
                (hipMalloc(&xcv, sizeof(double) * nLc) != hipSuccess ||
                 hipMalloc(&ycv, sizeof(double) * nLc) != hipSuccess ||
                 hipMalloc(&zcv, sizeof(double) * nLc) != hipSuccess ||
                 hipMalloc(&gidc, sizeof(int64_t) * nLc) != hipSuccess ||
                 hipMalloc(&dirc, nLc) != hipSuccess)) {
                set_error("setup: coarse level allocation failed");
                rc = SEM_ENOMEM;
            }
            if (rc == SEM_OK) rc = launch_interp<double>(E, F.nq, nqc, dJfc, px, xcv, false, s);
            if (rc == SEM_OK) rc = launch_interp<double>(E, F.nq, nqc, dJfc, py, ycv, false, s);
            if (rc == SEM_OK) rc = launch_interp<double>(E, F.nq, nqc, dJfc, pz, zcv, false, s);
            if (rc == SEM_OK) {
                const int bs = 256;
                hipLaunchKernelGGL(coarse_ids_kernel, dim3((unsigned)((nLc + bs - 1) / bs)),
                                   dim3(bs), 0, s, E, F.nq, nqc, fmap, F.gid, F.dir, gidc, dirc);
                if (hipGetLastError() != hipSuccess) {
                    set_error("setup: coarse pointer kernel failed to launch");
                    rc = SEM_EHIP;
                }
            }
            const bool f32 = (l < nlev - 1);
            if (rc == SEM_OK) {
                rc = build_level(h->lv[l], Nc, E, xcv, ycv, zcv, gidc, dirc, f32, bad, s);
                gidc = nullptr;  // owned by the level from here on, also on failure
                dirc = nullptr;
            }
            (void)hipStreamSynchronize(s);
            if (px != x) {
                (void)hipFree(px);
                (void)hipFree(py);
                (void)hipFree(pz);
            }
            px = xcv;
            py = ycv;
            pz = zcv;
            if (gidc) (void)hipFree(gidc);
            if (dirc) (void)hipFree(dirc);
            if (fmap) (void)hipFree(fmap);
            if (dJfc) (void)hipFree(dJfc);
        }
        if (px != x) {
            if (px) (void)hipFree(px);
            if (py) (void)hipFree(py);
            if (pz) (void)hipFree(pz);
        }
        if (rc != SEM_OK) break;
        int hbad = 0;
        if (hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            set_error("setup: %s", hipGetErrorString(hipGetLastError()));
            rc = SEM_EHIP;
            break;
        }
        if (hbad) {
            set_error("setup: mesh rejected (%s%s%s)", (hbad & 1) ? "nonpositive Jacobian " : "",
                      (hbad & 2) ? "copies of a global node disagree in coordinates " : "",
                      (hbad & 4) ? "copies of a global node disagree in the Dirichlet flag" : "");
            rc = SEM_EMESH;
        }
    } while (0);
    if (rc == SEM_OK) {  // the handle keeps the level-0 coordinates
        h->cx = x;
        h->cy = y;
        h->cz = z;
        x = y = z = nullptr;
    }
    if (x) (void)hipFree(x);
    if (y) (void)hipFree(y);
    if (z) (void)hipFree(z);
    if (gid) (void)hipFree(gid);
    if (dir) (void)hipFree(dir);
    (void)hipFree(bad);
    return rc;
}

}  // namespace semx

using namespace semx;

extern "C" {

int sem_gll(int N, double *xi, double *rho, double *D)
{
    if (N < 1 || N > kMaxN) {
        set_error("sem_gll: N=%d outside [1, %d]", N, kMaxN);
        return SEM_EINVAL;
    }
    return host_gll(N, xi, rho, D);
}

int sem_setup(const sem_mesh *m, const sem_setup_opts *o, void *stream, sem_handle *out)
{
    if (!out) {
        set_error("sem_setup: null output handle");
        return SEM_EINVAL;
    }
    *out = nullptr;
    if (!m || !m->x || !m->y || !m->z || !m->gid) {
        set_error("sem_setup: null mesh or mesh array");
        return SEM_EINVAL;
    }
    if (m->N < 1 || m->N > kMaxN) {
        set_error("sem_setup: N=%d outside [1, %d]", m->N, kMaxN);
        return SEM_EINVAL;
    }
    const int64_t np = (int64_t)(m->N + 1) * (m->N + 1) * (m->N + 1);
    if (m->E < 1 || m->E > (int64_t)(INT32_MAX - 1) / np) {
        set_error("sem_setup: E=%lld out of range (E*(N+1)^3 must be < 2^31)", (long long)m->E);
        return SEM_EINVAL;
    }
    if (o && o->pmg) {
        if (o->n_levels < 2 || o->n_levels > kMaxLevels || o->levels[0] != m->N) {
            set_error("sem_setup: multigrid needs 2..%d levels starting at N", kMaxLevels);
            return SEM_EINVAL;
        }
        for (int l = 1; l < o->n_levels; ++l)
            if (o->levels[l] < 1 || o->levels[l] >= o->levels[l - 1]) {
                set_error("sem_setup: multigrid orders must decrease to >= 1");
                return SEM_EINVAL;
            }
    }
    const int64_t nL = m->E * np;
    for (int64_t l = 0; l < nL; ++l)
        if (m->gid[l] < 0) {
            set_error("sem_setup: negative global pointer at copy %lld", (long long)l);
            return SEM_EINVAL;
        }
    if (m->dirichlet)
        for (int64_t l = 0; l < nL; ++l)
            if (m->dirichlet[l] > 1) {
                set_error("sem_setup: Dirichlet flag must be 0 or 1");
                return SEM_EINVAL;
            }
    sem_handle h = new (std::nothrow) sem_handle_s();
    if (!h) {
        set_error("sem_setup: out of host memory");
        return SEM_ENOMEM;
    }
    const int rc = setup_impl(m, o, (hipStream_t)stream, h);
    if (rc != SEM_OK) {
        sem_free(h);
        return rc;
    }
    *out = h;
    return SEM_OK;
}

int sem_free(sem_handle h)
{
    if (!h) return SEM_OK;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(h->device);
    free_workspace(h);
    for (int l = 0; l < kMaxLevels; ++l) free_level(h->lv[l]);
    free_advect(h);
    void *coords[] = {h->cx, h->cy, h->cz};
    for (void *p : coords)
        if (p) (void)hipFree(p);
    (void)hipSetDevice(cur);
    delete h;
    return SEM_OK;
}

static int check_level(sem_handle h, int level, const char *who)
{
    if (!h) {
        set_error("%s: null handle", who);
        return SEM_EINVAL;
    }
    if (level < 0 || level >= h->n_levels) {
        set_error("%s: level %d not in handle (%d levels)", who, level, h->n_levels);
        return SEM_EINVAL;
    }
    return SEM_OK;
}

int sem_ax(sem_handle h, const double *u, double *w, double h1, double h2, const double *k,
           void *stream)
{
    SEM_TRY(check_level(h, 0, "sem_ax"));
    if (!u || !w) {
        set_error("sem_ax: null vector");
        return SEM_EINVAL;
    }
    const Level &L = h->lv[0];
    return launch_ax<double>(L, L.G, L.B, L.D, u, w, h1, h2, k, nullptr, nullptr,
                             (hipStream_t)stream);
}

int sem_gs(sem_handle h, double *v, int op, void *stream)
{
    SEM_TRY(check_level(h, 0, "sem_gs"));
    if (!v) {
        set_error("sem_gs: null vector");
        return SEM_EINVAL;
    }
    if (op != SEM_GS_ADD && op != SEM_GS_MUL && op != SEM_GS_MIN && op != SEM_GS_MAX) {
        set_error("sem_gs: unknown operation %d", op);
        return SEM_EINVAL;
    }
    return launch_gs_op<double>(h->lv[0], v, op, (hipStream_t)stream);
}

int sem_ax_level(sem_handle h, int level, int dtype, const void *u, void *w, double h1, double h2,
                 void *stream)
{
    SEM_TRY(check_level(h, level, "sem_ax_level"));
    if (!u || !w) {
        set_error("sem_ax_level: null vector");
        return SEM_EINVAL;
    }
    const Level &L = h->lv[level];
    if (dtype == SEM_F64)
        return launch_ax<double>(L, L.G, L.B, L.D, (const double *)u, (double *)w, h1, h2, nullptr,
                                 nullptr, nullptr, (hipStream_t)stream);
    if (dtype == SEM_F32) {
        if (!L.G32) {
            set_error("sem_ax_level: level %d has no FP32 operator", level);
            return SEM_EINVAL;
        }
        return launch_ax<float>(L, L.G32, L.B32, L.D32, (const float *)u, (float *)w, h1, h2,
                                nullptr, nullptr, nullptr, (hipStream_t)stream);
    }
    set_error("sem_ax_level: bad dtype %d", dtype);
    return SEM_EINVAL;
}

int sem_gs_level(sem_handle h, int level, int dtype, void *v, void *stream)
{
    SEM_TRY(check_level(h, level, "sem_gs_level"));
    if (!v) {
        set_error("sem_gs_level: null vector");
        return SEM_EINVAL;
    }
    if (dtype == SEM_F64) return launch_gs<double>(h->lv[level], (double *)v, (hipStream_t)stream);
    if (dtype == SEM_F32) return launch_gs<float>(h->lv[level], (float *)v, (hipStream_t)stream);
    set_error("sem_gs_level: bad dtype %d", dtype);
    return SEM_EINVAL;
}

// batched operator / gather-scatter: nrhs fields at base + r*ld, in groups of kMaxRhs
static int check_batch(sem_handle h, int level, int nrhs, int64_t ld, const void *a, const void *b,
                       const char *who)
{
    SEM_TRY(check_level(h, level, who));
    if (!a || !b) {
        set_error("%s: null vector", who);
        return SEM_EINVAL;
    }
    if (nrhs < 1) {
        set_error("%s: nrhs = %d", who, nrhs);
        return SEM_EINVAL;
    }
    if (nrhs > 1 && ld < h->lv[level].nL) {
        set_error("%s: ld = %lld below n_local = %lld", who, (long long)ld, (long long)h->lv[level].nL);
        return SEM_EINVAL;
    }
    return SEM_OK;
}

int sem_ax_level_multi(sem_handle h, int level, int dtype, int nrhs, const void *u, void *w, int64_t ld,
                       double h1, double h2, void *stream)
{
    SEM_TRY(check_batch(h, level, nrhs, ld, u, w, "sem_ax_level_multi"));
    const Level &L = h->lv[level];
    if (dtype == SEM_F32 && !L.G32) {
        set_error("sem_ax_level_multi: level %d has no FP32 operator", level);
        return SEM_EINVAL;
    }
    if (dtype != SEM_F64 && dtype != SEM_F32) {
        set_error("sem_ax_level_multi: bad dtype %d", dtype);
        return SEM_EINVAL;
    }
    const hipStream_t s = (hipStream_t)stream;
    for (int r0 = 0; r0 < nrhs; r0 += kMaxRhs) {
        const VSet vs = VSet::first(std::min(kMaxRhs, nrhs - r0));
        if (dtype == SEM_F64)
            SEM_TRY(launch_ax_multi<double>(L, L.G, L.B, L.D, (const double *)u + r0 * ld, ld,
                                            (double *)w + r0 * ld, ld, vs, h1, h2, nullptr, nullptr, 0,
                                            nullptr, s, nullptr, 0));
        else
            SEM_TRY(launch_ax_multi<float>(L, L.G32, L.B32, L.D32, (const float *)u + r0 * ld, ld,
                                           (float *)w + r0 * ld, ld, vs, h1, h2, nullptr, nullptr, 0,
                                           nullptr, s, nullptr, 0));
    }
    return SEM_OK;
}

int sem_gs_level_multi(sem_handle h, int level, int dtype, int nrhs, void *v, int64_t ld, void *stream)
{
    SEM_TRY(check_batch(h, level, nrhs, ld, v, v, "sem_gs_level_multi"));
    if (dtype != SEM_F64 && dtype != SEM_F32) {
        set_error("sem_gs_level_multi: bad dtype %d", dtype);
        return SEM_EINVAL;
    }
    const Level &L = h->lv[level];
    const hipStream_t s = (hipStream_t)stream;
    for (int r0 = 0; r0 < nrhs; r0 += kMaxRhs) {
        const VSet vs = VSet::first(std::min(kMaxRhs, nrhs - r0));
        if (dtype == SEM_F64)
            SEM_TRY(launch_gs_multi<double>(L, (double *)v + r0 * ld, ld, vs, s, nullptr, 0));
        else
            SEM_TRY(launch_gs_multi<float>(L, (float *)v + r0 * ld, ld, vs, s, nullptr, 0));
    }
    return SEM_OK;
}

int sem_ax_multi(sem_handle h, int nrhs, const double *u, double *w, int64_t ld, double h1, double h2,
                 void *stream)
{
    return sem_ax_level_multi(h, 0, SEM_F64, nrhs, u, w, ld, h1, h2, stream);
}

int sem_gs_multi(sem_handle h, int nrhs, double *v, int64_t ld, void *stream)
{
    return sem_gs_level_multi(h, 0, SEM_F64, nrhs, v, ld, stream);
}

int sem_grad_k(sem_handle h, const double *u, const double *lam, double h1, double *gk, void *stream)
{
    SEM_TRY(check_level(h, 0, "sem_grad_k"));
    if (!u || !lam || !gk) {
        set_error("sem_grad_k: null vector");
        return SEM_EINVAL;
    }
    return launch_grad_k(h->lv[0], u, lam, h1, gk, (hipStream_t)stream);
}

int sem_info(sem_handle h, int level, sem_info_t *info)
{
    SEM_TRY(check_level(h, level, "sem_info"));
    if (!info) {
        set_error("sem_info: null output");
        return SEM_EINVAL;
    }
    const Level &L = h->lv[level];
    info->N = L.N;
    info->E = L.E;
    info->n_local = L.nL;
    info->n_unique = L.n_unique;
    info->n_shared_copies = L.ncopies;
    info->n_segments = L.nseg;
    info->n_levels = h->n_levels;
    return SEM_OK;
}

int sem_get_maps(sem_handle h, int level, int32_t *perm, int32_t *offs, void *stream)
{
    SEM_TRY(check_level(h, level, "sem_get_maps"));
    const Level &L = h->lv[level];
    hipStream_t s = (hipStream_t)stream;
    if (perm && L.ncopies)
        SEM_HIP(hipMemcpyAsync(perm, L.perm, sizeof(int32_t) * L.ncopies, hipMemcpyDeviceToDevice, s));
    if (offs)
        SEM_HIP(hipMemcpyAsync(offs, L.offs, sizeof(int32_t) * (L.nseg + 1), hipMemcpyDeviceToDevice, s));
    return SEM_OK;
}

// handle layout [E][np][6] -> caller layout [6][n_local]
__global__ void unblock_G_kernel(int64_t nL, int np, const double *__restrict__ Gb, double *__restrict__ G)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 6 * nL) return;
    const int slot = (int)(t / nL);
    const int64_t q = t - slot * nL;
    G[t] = Gb[q * 6 + slot];
}

int sem_get_geometry(sem_handle h, int level, double *G, double *B, void *stream)
{
    SEM_TRY(check_level(h, level, "sem_get_geometry"));
    const Level &L = h->lv[level];
    hipStream_t s = (hipStream_t)stream;
    if (G) {
        const int bs = 256;
        hipLaunchKernelGGL(unblock_G_kernel, dim3((unsigned)((6 * L.nL + bs - 1) / bs)), dim3(bs),
                           0, s, L.nL, L.np, L.G, G);
        SEM_HIP(hipGetLastError());
    }
    if (B) SEM_HIP(hipMemcpyAsync(B, L.B, sizeof(double) * L.nL, hipMemcpyDeviceToDevice, s));
    return SEM_OK;
}

int sem_get_weights(sem_handle h, int level, double *W, int64_t *gid, void *stream)
{
    SEM_TRY(check_level(h, level, "sem_get_weights"));
    const Level &L = h->lv[level];
    hipStream_t s = (hipStream_t)stream;
    if (W) SEM_HIP(hipMemcpyAsync(W, L.W, sizeof(double) * L.nL, hipMemcpyDeviceToDevice, s));
    if (gid) SEM_HIP(hipMemcpyAsync(gid, L.gid, sizeof(int64_t) * L.nL, hipMemcpyDeviceToDevice, s));
    return SEM_OK;
}

const char *sem_strerror(int code)
{
    switch (code) {
    case SEM_OK: return "success";
    case SEM_EINVAL: return "invalid argument";
    case SEM_ENOMEM: return "out of memory";
    case SEM_EHIP: return "HIP runtime error";
    case SEM_ENOCONV: return "solver did not converge within maxit";
    case SEM_EBREAKDOWN: return "solver breakdown (nonpositive curvature or NaN)";
    case SEM_EMESH: return "invalid mesh (nonpositive Jacobian or inconsistent copies)";
    default: return "unknown status";
    }
}

const char *sem_last_error(void) { return g_err; }

}  // extern "C"
