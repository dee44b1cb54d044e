// Krylov solvers of libsem (NekRS paper, Sec. 2.3 cost discussion and
// Sec. 3.4 preconditioning):
//   * Jacobi-PCG in FP64 (the viscous Helmholtz solver of the paper);
//   * flexible CG (Polak-Ribiere beta) preconditioned by one p-multigrid
//     V-cycle: Chebyshev-accelerated Jacobi pre/post smoothing in FP32 on every
//     level above the coarsest, FP64 Jacobi-PCG on the coarsest level; the
//     outer iteration, its inner products and the coarse solve stay FP64.
// All vectors are replicated L-vectors; inner products over unique free nodes
// are L-space sums weighted by the counting weight W (0 on Dirichlet copies).
// The iteration scalars live on the device (KrylovScalars); kernels after
// convergence see `done` and return, so batches of iterations are enqueued
// without a host round trip per iteration.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "sem_internal.h"

namespace semx {

constexpr int kRB = 256;          // reduction block size
constexpr int kMaxRedBlocks = 1024;

static int red_grid(int64_t n)
{
    const int64_t nb = (n + kRB - 1) / kRB;
    return (int)std::max<int64_t>(1, std::min<int64_t>(nb, kMaxRedBlocks));
}

// deterministic block sum of NV values per thread; thread v < NV writes
// out[blockIdx.x * NV + v]
template <int NV>
__device__ inline void block_sum_store(const double (&v)[NV], double *out)
{
    __shared__ double sh[NV][kRB];
    const int t = threadIdx.x;
#pragma unroll
    for (int q = 0; q < NV; ++q) sh[q][t] = v[q];
    __syncthreads();
    for (int st = kRB / 2; st > 0; st >>= 1) {
        if (t < st)
#pragma unroll
            for (int q = 0; q < NV; ++q) sh[q][t] += sh[q][t + st];
        __syncthreads();
    }
    if (t < NV) out[(int64_t)blockIdx.x * NV + t] = sh[t][0];
}

// deterministic sum of nb partial records of NV values (one block of kRB)
template <int NV>
__device__ inline void sum_partials(const double *partial, int64_t nb, double (&res)[NV])
{
    __shared__ double sh[NV][kRB];
    const int t = threadIdx.x;
    double acc[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) acc[q] = 0.0;
    for (int64_t b = t; b < nb; b += kRB)
#pragma unroll
        for (int q = 0; q < NV; ++q) acc[q] += partial[b * NV + q];
#pragma unroll
    for (int q = 0; q < NV; ++q) sh[q][t] = acc[q];
    __syncthreads();
    for (int st = kRB / 2; st > 0; st >>= 1) {
        if (t < st)
#pragma unroll
            for (int q = 0; q < NV; ++q) sh[q][t] += sh[q][t + st];
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < NV; ++q) res[q] = sh[q][0];
}

// ------------------------------------------------------------------ vectors
template <typename T>
__global__ void fill_kernel(int64_t n, T *v, T val)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        v[i] = val;
}

template <typename T, typename TW>
__global__ void mask_kernel(int64_t n, const TW *__restrict__ W, T *__restrict__ v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        if (!(W[i] > TW(0))) v[i] = T(0);
}

template <typename TA, typename TB>
__global__ void convert_kernel(int64_t n, const TA *__restrict__ a, TB *__restrict__ b)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        b[i] = (TB)a[i];
}

__global__ void invert_diag_kernel(int64_t n, const double *__restrict__ W,
                                   const double *__restrict__ d, double *__restrict__ Dinv,
                                   float *__restrict__ Dinv32)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double v = (W[i] > 0.0 && d[i] != 0.0) ? 1.0 / d[i] : 0.0;
        Dinv[i] = v;
        if (Dinv32) Dinv32[i] = (float)v;
    }
}

// partial (W a b) sums, FP64
__global__ void dot_kernel(int64_t n, const double *__restrict__ W, const double *__restrict__ a,
                           const double *__restrict__ b, double *__restrict__ partial)
{
    double s[1] = {0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        s[0] += W[i] * a[i] * b[i];
    block_sum_store<1>(s, partial);
}

// ---------------------------------------------------------------- Jacobi-PCG
// r = b - Ax (Ax may be null: x = 0), p = Dinv r; partials (W r p, W r r, W b b)
__global__ void pcg_init_kernel(int64_t n, const double *__restrict__ b, const double *__restrict__ Ax,
                                const double *__restrict__ Dinv, const double *__restrict__ W,
                                double *__restrict__ r, double *__restrict__ p,
                                double *__restrict__ partial, int precondition)
{
    double s[3] = {0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double ri = b[i] - (Ax ? Ax[i] : 0.0);
        r[i] = ri;
        const double zi = precondition ? Dinv[i] * ri : ri;
        if (p) p[i] = zi;
        const double wi = W[i];
        s[0] += wi * ri * zi;
        s[1] += wi * ri * ri;
        s[2] += wi * b[i] * b[i];
    }
    block_sum_store<3>(s, partial);
}

__global__ void fin_init_kernel(const double *partial, int64_t nb, KrylovScalars *sc, double tol,
                                int maxit)
{
    double res[3];
    sum_partials<3>(partial, nb, res);
    if (threadIdx.x == 0) {
        sc->rz = res[0];
        sc->rz_old = res[0];
        sc->rz2[0] = res[0];
        sc->rz2[1] = res[0];
        sc->rr = res[1];
        sc->bb = res[2];
        sc->tol2 = tol * tol * res[2];
        sc->iters = 0;
        sc->maxit = maxit;
        sc->status = SEM_OK;
        sc->alpha = sc->beta = sc->pw = sc->zw = 0.0;
        const bool bad = !isfinite(res[0]) || !isfinite(res[1]) || !isfinite(res[2]);
        if (bad) sc->status = SEM_EBREAKDOWN;
        sc->done = (bad || res[2] == 0.0 || res[1] <= sc->tol2 || maxit <= 0) ? 1 : 0;
    }
}

// ------------------------------------------------- fused Krylov iterations
// QQ^T value of copy l.  With segid == nullptr, w is already assembled (a
// gs_kernel pass ran before); otherwise the sum over the copies of its node is
// taken on the fly in the canonical order, starting from 0 (bit-identical to
// gs_kernel's).  The on-the-fly form trades the gs pass for dependent
// scattered loads and is only worth it for tiny levels.
template <typename T>
__device__ inline T assembled_value(const T *__restrict__ w, int64_t l,
                                    const int32_t *__restrict__ segid,
                                    const int32_t *__restrict__ perm,
                                    const int32_t *__restrict__ offs)
{
    if (segid == nullptr) return w[l];
    const int sg = segid[l];
    if (sg < 0) return w[l];
    const int a = offs[sg], b = offs[sg + 1];
    T acc = T(0);
    for (int o = a; o < b; ++o) acc += w[perm[o]];
    return acc;
}

// Jacobi-PCG update.  Every block sums the operator kernel's partials of
// (p, A_L p) in the same fixed order, so all blocks hold the same alpha;
// x += alpha p; r -= alpha QQ^T(A_L p); partials (W r Dinv r, W r r).
// rz2[parity] is the current (r, z).
__global__ void pcg_update_fused_kernel(int64_t n, KrylovScalars *sc, int parity,
                                        const double *__restrict__ pax, int64_t nbax,
                                        const double *__restrict__ p, const double *__restrict__ w,
                                        const int32_t *__restrict__ segid,
                                        const int32_t *__restrict__ perm,
                                        const int32_t *__restrict__ offs,
                                        const double *__restrict__ Dinv,
                                        const double *__restrict__ W, double *__restrict__ x,
                                        double *__restrict__ r, double *__restrict__ partial)
{
    if (sc->done) return;
    double res[1];
    sum_partials<1>(pax, nbax, res);
    const double pw = res[0];
    if (!(pw > 0.0) || !isfinite(pw)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            sc->pw = pw;
            sc->status = SEM_EBREAKDOWN;
            sc->done = 1;
        }
        return;
    }
    const double a = sc->rz2[parity] / pw;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->pw = pw;
        sc->alpha = a;
    }
    double s[2] = {0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        x[i] += a * p[i];
        const double ri = r[i] - a * assembled_value(w, i, segid, perm, offs);
        r[i] = ri;
        const double wr = W[i] * ri;
        s[0] += wr * Dinv[i] * ri;
        s[1] += wr * ri;
    }
    block_sum_store<2>(s, partial);
}

// Jacobi-PCG direction update with beta and the convergence decision taken
// by every block from the update's partials (identical in all blocks);
// block 0 records them.  `iter` is the 1-based number of this iteration.
__global__ void pcg_p_fused_kernel(int64_t n, KrylovScalars *sc, int parity, int iter,
                                   const double *__restrict__ pu, int64_t nbu,
                                   const double *__restrict__ Dinv, const double *__restrict__ r,
                                   double *__restrict__ p)
{
    if (sc->done) return;
    double res[2];
    sum_partials<2>(pu, nbu, res);
    const double rz = res[0], rr = res[1];
    const bool bad = !isfinite(rz) || !isfinite(rr);
    const bool stop = bad || rr <= sc->tol2 || iter >= sc->maxit;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->iters = iter;
        sc->rr = rr;
        sc->rz = rz;
        sc->rz2[parity ^ 1] = rz;
        if (bad) sc->status = SEM_EBREAKDOWN;
        if (stop) sc->done = 1;
    }
    if (stop) return;
    const double be = rz / sc->rz2[parity];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = Dinv[i] * r[i] + be * p[i];
}

// flexible-CG update: alpha from the operator partials, x += alpha p,
// r -= alpha QQ^T(A_L p); partial (W r r)
__global__ void fcg_update_fused_kernel(int64_t n, KrylovScalars *sc, int parity,
                                        const double *__restrict__ pax, int64_t nbax,
                                        const double *__restrict__ p, const double *__restrict__ w,
                                        const int32_t *__restrict__ segid,
                                        const int32_t *__restrict__ perm,
                                        const int32_t *__restrict__ offs,
                                        const double *__restrict__ W, double *__restrict__ x,
                                        double *__restrict__ r, double *__restrict__ partial)
{
    if (sc->done) return;
    double res[1];
    sum_partials<1>(pax, nbax, res);
    const double pw = res[0];
    if (!(pw > 0.0) || !isfinite(pw)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            sc->pw = pw;
            sc->status = SEM_EBREAKDOWN;
            sc->done = 1;
        }
        return;
    }
    const double a = sc->rz2[parity] / pw;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->pw = pw;
        sc->alpha = a;
    }
    double s[1] = {0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        x[i] += a * p[i];
        const double ri = r[i] - a * assembled_value(w, i, segid, perm, offs);
        r[i] = ri;
        s[0] += W[i] * ri * ri;
    }
    block_sum_store<1>(s, partial);
}

// (z, w)_W and (z, r)_W for assembled w
__global__ void dot_zw_kernel(int64_t n, const KrylovScalars *sc, const double *__restrict__ W,
                              const double *__restrict__ z, const double *__restrict__ wa,
                              const double *__restrict__ r, double *__restrict__ partial)
{
    if (sc->done) return;
    double s[2] = {0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double wz = W[i] * z[i];
        s[0] += wz * wa[i];
        s[1] += wz * r[i];
    }
    block_sum_store<2>(s, partial);
}

// Polak-Ribiere direction update, beta = (z_new, r_new - r_old) / (z_old, r_old)
// = -alpha (z_new, A p) / rz_old (r_new - r_old = -alpha A p), taken by every
// block from the partials of dot_zw_kernel; first = 1 gives p = z.
__global__ void fcg_p_fused_kernel(int64_t n, KrylovScalars *sc, int parity,
                                   const double *__restrict__ pz, int64_t nbz,
                                   const double *__restrict__ z, double *__restrict__ p, int first)
{
    if (sc->done) return;
    double res[2];
    sum_partials<2>(pz, nbz, res);
    const double zw = res[0], zr = res[1];
    const double be = first ? 0.0 : -sc->alpha * zw / sc->rz2[parity];
    const bool bad = !isfinite(be) || !isfinite(zr);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->zw = zw;
        sc->beta = be;
        sc->rz = zr;
        sc->rz2[parity ^ 1] = zr;
        if (bad) {
            sc->status = SEM_EBREAKDOWN;
            sc->done = 1;
        }
    }
    if (bad) return;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = z[i] + be * p[i];
}

// Chebyshev step with QQ^T of the operator output taken on the fly:
// res = r - QQ^T t (t = A_L x, or absent when x = 0),
// d = c1 d + c2 Dinv res, x += d (x = d when `init`)
__global__ void cheb_fused_kernel(int64_t n, const float *__restrict__ r, const float *__restrict__ t,
                                  const int32_t *__restrict__ segid, const int32_t *__restrict__ perm,
                                  const int32_t *__restrict__ offs, const float *__restrict__ Dinv,
                                  float *__restrict__ d, float *__restrict__ x, float c1, float c2,
                                  int init)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float res = t ? r[i] - assembled_value(t, i, segid, perm, offs) : r[i];
        const float di = (init ? 0.0f : c1 * d[i]) + c2 * Dinv[i] * res;
        d[i] = di;
        x[i] = init ? di : x[i] + di;
    }
}

// s = W (r - QQ^T t)
__global__ void wresid_fused_kernel(int64_t n, const float *__restrict__ W,
                                    const float *__restrict__ r, const float *__restrict__ t,
                                    const int32_t *__restrict__ segid,
                                    const int32_t *__restrict__ perm,
                                    const int32_t *__restrict__ offs, float *__restrict__ s)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        s[i] = W[i] * (r[i] - assembled_value(t, i, segid, perm, offs));
}

// flexible CG convergence decision after the update (one block): iteration
// count, (r, r)_W, done
__global__ void fin_conv_kernel(const double *partial, int64_t nb, KrylovScalars *sc)
{
    if (sc->done) return;
    double res[1];
    sum_partials<1>(partial, nb, res);
    if (threadIdx.x == 0) {
        sc->iters += 1;
        sc->rr = res[0];
        if (!isfinite(res[0])) {
            sc->status = SEM_EBREAKDOWN;
            sc->done = 1;
        } else if (res[0] <= sc->tol2 || sc->iters >= sc->maxit) {
            sc->done = 1;
        }
    }
}

// y += a (prolongation added to the smoothed iterate)
template <typename T>
__global__ void add_kernel(int64_t n, const T *__restrict__ a, T *__restrict__ y)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] += a[i];
}

// ---------------------------------------------------------- load / adjoint
// y = B o x (mass-weighted copy)
__global__ void mass_kernel(int64_t n, const double *__restrict__ B, const double *__restrict__ x,
                            double *__restrict__ y)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = B[i] * x[i];
}

// ----------------------------------------------------------------- Lanczos
// start vector: SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) of each copy's
// global pointer, top 53 bits to [-1, 1); zero on Dirichlet copies
__global__ void splitmix_kernel(int64_t n, const int64_t *__restrict__ gid,
                                const double *__restrict__ W, uint64_t seed, double *__restrict__ v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t zz = seed + ((uint64_t)gid[i] + 1ULL) * 0x9E3779B97F4A7C15ULL;
        zz = (zz ^ (zz >> 30)) * 0xBF58476D1CE4E5B9ULL;
        zz = (zz ^ (zz >> 27)) * 0x94D049BB133111EBULL;
        zz ^= zz >> 31;
        const double u = (double)(zz >> 11) * (1.0 / 9007199254740992.0);
        v[i] = (W[i] > 0.0) ? 2.0 * u - 1.0 : 0.0;
    }
}

// y = a * sqrt(Dinv) x + b * y
__global__ void sqrtd_axpby_kernel(int64_t n, const double *__restrict__ Dinv,
                                   const double *__restrict__ x, double a, double b,
                                   double *__restrict__ y)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = a * sqrt(Dinv[i]) * x[i] + (b == 0.0 ? 0.0 : b * y[i]);
}

// y = a x + b y
__global__ void axpby_kernel(int64_t n, const double *__restrict__ x, double a, double b,
                             double *__restrict__ y)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = a * x[i] + b * y[i];
}

// ============================================================== host side
#define LAUNCH_V(kern, n, s, ...)                                                           \
    do {                                                                                    \
        hipLaunchKernelGGL(kern, dim3(red_grid(n)), dim3(kRB), 0, s, __VA_ARGS__);          \
        SEM_HIP(hipGetLastError());                                                         \
    } while (0)
#define LAUNCH_1(kern, s, ...)                                                              \
    do {                                                                                    \
        hipLaunchKernelGGL(kern, dim3(1), dim3(kRB), 0, s, __VA_ARGS__);                    \
        SEM_HIP(hipGetLastError());                                                         \
    } while (0)

void free_workspace(sem_handle h)
{
    Workspace &w = h->ws;
    void *ptrs[] = {w.r, w.p, w.w, w.z, w.aux, w.partial, w.partial_ax, w.sc, w.sc_c, w.c_r,
                    w.c_p, w.c_w};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    for (int l = 0; l < kMaxLevels; ++l) {
        void *q[] = {w.mg_r[l], w.mg_x[l], w.mg_t[l], w.mg_d[l], w.mg_s[l]};
        for (void *p : q)
            if (p) (void)hipFree(p);
    }
    if (w.host_sc) (void)hipHostFree(w.host_sc);
    h->ws = Workspace{};
    for (int l = 0; l < kMaxLevels; ++l) {
        if (h->lv[l].Dinv) (void)hipFree(h->lv[l].Dinv);
        if (h->lv[l].Dinv32) (void)hipFree(h->lv[l].Dinv32);
        h->lv[l].Dinv = nullptr;
        h->lv[l].Dinv32 = nullptr;
    }
    h->key = PrecondKey{};
}

static int ensure_workspace(sem_handle h, bool pmg)
{
    Workspace &w = h->ws;
    const Level &F = h->lv[0];
    if (!w.r) {
        w.nL = F.nL;
        SEM_HIP(hipMalloc(&w.r, sizeof(double) * F.nL));
        SEM_HIP(hipMalloc(&w.p, sizeof(double) * F.nL));
        SEM_HIP(hipMalloc(&w.w, sizeof(double) * F.nL));
        SEM_HIP(hipMalloc(&w.z, sizeof(double) * F.nL));
        // vector-kernel partials: at most kMaxRedBlocks records of 3; operator
        // partials: one per workgroup of the persistent operator grid
        w.n_partial = 3 * kMaxRedBlocks;
        SEM_HIP(hipMalloc(&w.partial, sizeof(double) * w.n_partial));
        w.n_partial_ax = (int64_t)(F.n_cu > 0 ? F.n_cu : 256) * kAxMaxBlocksPerCU + 64;
        SEM_HIP(hipMalloc(&w.partial_ax, sizeof(double) * w.n_partial_ax));
        SEM_HIP(hipMalloc(&w.sc, sizeof(KrylovScalars)));
        SEM_HIP(hipMalloc(&w.sc_c, sizeof(KrylovScalars)));
        SEM_HIP(hipHostMalloc((void **)&w.host_sc, 2 * sizeof(KrylovScalars), hipHostMallocDefault));
    }
    for (int l = 0; l < h->n_levels; ++l) {
        Level &L = h->lv[l];
        if (!L.Dinv) SEM_HIP(hipMalloc(&L.Dinv, sizeof(double) * L.nL));
        if (pmg && l < h->n_levels - 1 && !L.Dinv32) SEM_HIP(hipMalloc(&L.Dinv32, sizeof(float) * L.nL));
    }
    if (pmg && !w.c_r) {
        for (int l = 0; l + 1 < h->n_levels; ++l) {
            const int64_t n = h->lv[l].nL;
            SEM_HIP(hipMalloc(&w.mg_r[l], sizeof(float) * n));
            SEM_HIP(hipMalloc(&w.mg_x[l], sizeof(float) * n));
            SEM_HIP(hipMalloc(&w.mg_t[l], sizeof(float) * n));
            SEM_HIP(hipMalloc(&w.mg_d[l], sizeof(float) * n));
            SEM_HIP(hipMalloc(&w.mg_s[l], sizeof(float) * n));
        }
        const int lc = h->n_levels - 1;
        const int64_t n = h->lv[lc].nL;
        SEM_HIP(hipMalloc(&w.mg_r[lc], sizeof(double) * n));  // coarse rhs
        SEM_HIP(hipMalloc(&w.mg_x[lc], sizeof(double) * n));  // coarse solution
        SEM_HIP(hipMalloc(&w.c_r, sizeof(double) * n));
        SEM_HIP(hipMalloc(&w.c_p, sizeof(double) * n));
        SEM_HIP(hipMalloc(&w.c_w, sizeof(double) * n));
    }
    return SEM_OK;
}

// FP64 Dinv (and FP32 copy) of level l for h1 A(k) + h2 B: diag, QQ^T, invert
static int compute_dinv(sem_handle h, int l, const double *k, double h1, double h2, bool f32,
                        hipStream_t s)
{
    Level &L = h->lv[l];
    double *d = h->ws.z;  // scratch, fine-level sized >= level size
    SEM_TRY(launch_diag<double>(L, k, h1, h2, d, s));
    SEM_TRY(launch_gs<double>(L, d, s));
    LAUNCH_V(invert_diag_kernel, L.nL, s, L.nL, L.W, d, L.Dinv, f32 ? L.Dinv32 : nullptr);
    return SEM_OK;
}

static double host_sum_partials(const std::vector<double> &p) {
    double s = 0.0;
    for (double v : p) s += v;
    return s;
}

static int host_dot(const Level &L, const double *a, const double *b, double *partial, double *out,
                    hipStream_t s)
{
    const int nb = red_grid(L.nL);
    LAUNCH_V(dot_kernel, L.nL, s, L.nL, L.W, a, b, partial);
    std::vector<double> hp(nb);
    SEM_HIP(hipMemcpyAsync(hp.data(), partial, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
    SEM_HIP(hipStreamSynchronize(s));
    *out = host_sum_partials(hp);
    return SEM_OK;
}

// largest eigenvalue of the symmetric tridiagonal (a, b) by Sturm bisection
static double tridiag_max_eig(const std::vector<double> &a, const std::vector<double> &b)
{
    const int m = (int)a.size();
    double lo = 1e300, hi = -1e300;
    for (int i = 0; i < m; ++i) {
        const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(b[i]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
    }
    auto count_below = [&](double x) {  // eigenvalues < x
        int c = 0;
        double q = a[0] - x;
        if (q < 0) ++c;
        for (int i = 1; i < m; ++i) {
            const double qq = (q == 0.0) ? 1e-300 : q;
            q = a[i] - x - b[i - 1] * b[i - 1] / qq;
            if (q < 0) ++c;
        }
        return c;
    };
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (count_below(mid) >= m) hi = mid; else lo = mid;
    }
    return hi;
}

// Lanczos estimate of lambda_max(Dinv A) on level l (FP64 operator), in the
// W inner product on the symmetric form Dinv^{1/2} A Dinv^{1/2}
static int lanczos_lmax(sem_handle h, int l, double h1, double h2, int steps, double *lmax,
                        hipStream_t s)
{
    Level &L = h->lv[l];
    Workspace &w = h->ws;
    const int64_t n = L.nL;
    double *v = w.r, *vp = w.p, *t = w.w, *u = w.z;
    LAUNCH_V(splitmix_kernel, n, s, n, L.gid, L.W, h->lanczos_seed, v);
    double nrm2 = 0.0;
    SEM_TRY(host_dot(L, v, v, w.partial, &nrm2, s));
    if (!(nrm2 > 0.0)) {
        *lmax = 1.0;
        return SEM_OK;
    }
    LAUNCH_V(axpby_kernel, n, s, n, v, 1.0 / std::sqrt(nrm2), 0.0, v);
    LAUNCH_V(fill_kernel<double>, n, s, n, vp, 0.0);
    std::vector<double> al, be;
    double beta = 0.0;
    for (int it = 0; it < steps; ++it) {
        // t = S v ; u = A t (restricted) ; u = S u - beta vp
        LAUNCH_V(sqrtd_axpby_kernel, n, s, n, L.Dinv, v, 1.0, 0.0, t);
        SEM_TRY(launch_ax<double>(L, L.G, L.B, L.D, t, u, h1, h2, nullptr, nullptr, nullptr, s));
        SEM_TRY(launch_gs<double>(L, u, s));
        LAUNCH_V((mask_kernel<double, double>), n, s, n, L.W, u);
        LAUNCH_V(sqrtd_axpby_kernel, n, s, n, L.Dinv, u, 1.0, 0.0, t);  // t = S A S v
        LAUNCH_V(axpby_kernel, n, s, n, vp, -beta, 1.0, t);              // t -= beta vp
        double alpha = 0.0;
        SEM_TRY(host_dot(L, t, v, w.partial, &alpha, s));
        LAUNCH_V(axpby_kernel, n, s, n, v, -alpha, 1.0, t);              // t -= alpha v
        al.push_back(alpha);
        double b2 = 0.0;
        SEM_TRY(host_dot(L, t, t, w.partial, &b2, s));
        beta = std::sqrt(std::max(b2, 0.0));
        if (!(beta > 1e-300) || it + 1 == steps) break;
        be.push_back(beta);
        // vp = v ; v = t / beta
        SEM_HIP(hipMemcpyAsync(vp, v, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        LAUNCH_V(axpby_kernel, n, s, n, t, 1.0 / beta, 0.0, v);
    }
    be.resize(al.size() > 0 ? al.size() - 1 : 0);
    *lmax = tridiag_max_eig(al, be);
    return SEM_OK;
}

struct ChebCoef {
    double theta, delta;
};

// FP32 operator on a smoother level: t = QQ^T A_L x (Dirichlet copies of t are
// ignored by the consumers, whose Dinv and W vanish there)
static int apply_f32(const Level &L, const float *x, float *t, double h1, double h2, hipStream_t s)
{
    SEM_TRY(launch_ax<float>(L, L.G32, L.B32, L.D32, x, t, h1, h2, nullptr, nullptr, nullptr, s));
    return launch_gs<float>(L, t, s);
}

// Chebyshev-accelerated Jacobi (Saad, Iterative Methods, Alg. 12.1, applied to
// Dinv A x = Dinv r) with `deg` updates; x == 0 on entry when `zero`.
static int chebyshev(const Level &L, int l, sem_handle h, const float *r, float *x, bool zero,
                     double lmin, double lmax, int deg, double h1, double h2, hipStream_t s)
{
    Workspace &w = h->ws;
    float *t = (float *)w.mg_t[l], *d = (float *)w.mg_d[l];
    const int64_t n = L.nL;
    const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
    const double sigma = theta / delta;
    double rho_prev = 1.0 / sigma;
    if (zero) {
        LAUNCH_V(cheb_fused_kernel, n, s, n, r, (const float *)nullptr, (const int32_t *)nullptr, L.perm, L.offs,
                 L.Dinv32, d, x, 0.0f, (float)(1.0 / theta), 1);
    } else {
        SEM_TRY(apply_f32(L, x, t, h1, h2, s));
        LAUNCH_V(cheb_fused_kernel, n, s, n, r, (const float *)t, (const int32_t *)nullptr, L.perm, L.offs,
                 L.Dinv32, d, x, 0.0f, (float)(1.0 / theta), 0);
    }
    for (int k = 1; k < deg; ++k) {
        const double rho = 1.0 / (2.0 * sigma - rho_prev);
        SEM_TRY(apply_f32(L, x, t, h1, h2, s));
        LAUNCH_V(cheb_fused_kernel, n, s, n, r, (const float *)t, (const int32_t *)nullptr, L.perm, L.offs,
                 L.Dinv32, d, x, (float)(rho * rho_prev), (float)(2.0 * rho / delta), 0);
        rho_prev = rho;
    }
    return SEM_OK;
}

struct SolveCfg {
    double h1, h2, tol, coarse_tol;
    int maxit, check_every, deg, coarse_maxit;
};

// enqueue Jacobi-PCG iterations first_iter .. first_iter+iters-1 (1-based)
// on level L: operator with fused (p, A_L p), QQ^T, update with alpha, and
// direction update with beta and the convergence decision -- four kernels per
// iteration, no single-block reduction kernels
static int pcg_iterations(const Level &L, const double *k, double h1, double h2, double *x,
                          double *r, double *p, double *w, double *pax, double *partial,
                          KrylovScalars *sc, int first_iter, int iters, hipStream_t s)
{
    const int64_t n = L.nL;
    const int nbv = red_grid(n);
    for (int c = 0; c < iters; ++c) {
        const int it = first_iter + c;
        const int parity = (it - 1) & 1;
        int64_t nbax = 0;
        SEM_TRY(launch_ax<double>(L, L.G, L.B, L.D, p, w, h1, h2, k, pax, &nbax, s, &sc->done));
        SEM_TRY(launch_gs<double>(L, w, s, &sc->done));
        LAUNCH_V(pcg_update_fused_kernel, n, s, n, sc, parity, (const double *)pax, nbax,
                 (const double *)p, (const double *)w, (const int32_t *)nullptr, L.perm, L.offs,
                 L.Dinv, L.W, x, r, partial);
        LAUNCH_V(pcg_p_fused_kernel, n, s, n, sc, parity, it, (const double *)partial,
                 (int64_t)nbv, L.Dinv, (const double *)r, p);
    }
    return SEM_OK;
}

// start a Jacobi-PCG on level L: x given (Ax computed) or zero
static int pcg_start(const Level &L, const double *k, double h1, double h2, const double *b,
                     double *x, bool zero, double *r, double *p, double *w, double *partial,
                     KrylovScalars *sc, double tol, int maxit, hipStream_t s)
{
    const int64_t n = L.nL;
    const double *Ax = nullptr;
    if (zero) {
        LAUNCH_V(fill_kernel<double>, n, s, n, x, 0.0);
    } else {
        LAUNCH_V((mask_kernel<double, double>), n, s, n, L.W, x);
        SEM_TRY(launch_ax<double>(L, L.G, L.B, L.D, x, w, h1, h2, k, nullptr, nullptr, s));
        SEM_TRY(launch_gs<double>(L, w, s));
        Ax = w;
    }
    LAUNCH_V(pcg_init_kernel, n, s, n, b, Ax, L.Dinv, L.W, r, p, partial, 1);
    LAUNCH_1(fin_init_kernel, s, partial, (int64_t)red_grid(n), sc, tol, maxit);
    return SEM_OK;
}

// one V-cycle from level l: input rhs in mg_r[l] (FP32; FP64 on the coarsest),
// output in mg_x[l]
static int vcycle(sem_handle h, int l, const SolveCfg &cfg, hipStream_t s)
{
    Workspace &w = h->ws;
    const int lc = h->n_levels - 1;
    const Level &L = h->lv[l];
    if (l == lc) {
        double *b = (double *)w.mg_r[l], *x = (double *)w.mg_x[l];
        SEM_TRY(pcg_start(L, nullptr, cfg.h1, cfg.h2, b, x, true, w.c_r, w.c_p, w.c_w, w.partial,
                          w.sc_c, cfg.coarse_tol, cfg.coarse_maxit, s));
        SEM_TRY(pcg_iterations(L, nullptr, cfg.h1, cfg.h2, x, w.c_r, w.c_p, w.c_w, w.partial_ax,
                               w.partial, w.sc_c, 1, cfg.coarse_maxit, s));
        return SEM_OK;
    }
    const int64_t n = L.nL;
    float *r = (float *)w.mg_r[l], *x = (float *)w.mg_x[l], *t = (float *)w.mg_t[l],
          *sres = (float *)w.mg_s[l];
    const double lmax = L.lmax;
    const double lmin_f = h->key.lo, lmax_f = h->key.hi;
    // pre-smoothing from x = 0
    SEM_TRY(chebyshev(L, l, h, r, x, true, lmin_f * lmax, lmax_f * lmax, cfg.deg, cfg.h1, cfg.h2, s));
    // restricted residual s = W (r - A x)
    SEM_TRY(apply_f32(L, x, t, cfg.h1, cfg.h2, s));
    LAUNCH_V(wresid_fused_kernel, n, s, n, L.W32, (const float *)r, (const float *)t,
             (const int32_t *)nullptr, L.perm, L.offs, sres);
    const Level &C = h->lv[l + 1];
    const int64_t nc = C.nL;
    if (l + 1 == lc) {
        // restrict in FP32 into t's coarse-sized head, then FP64 for the coarse solve
        float *tc = t;  // n >= nc
        SEM_TRY(launch_interp<float>(L.E, L.nq, C.nq, L.Jc32, sres, tc, true, s));
        LAUNCH_V((convert_kernel<float, double>), nc, s, nc, tc, (double *)w.mg_r[l + 1]);
        SEM_TRY(launch_gs<double>(C, (double *)w.mg_r[l + 1], s));
        LAUNCH_V((mask_kernel<double, double>), nc, s, nc, C.W, (double *)w.mg_r[l + 1]);
        SEM_TRY(vcycle(h, l + 1, cfg, s));
        LAUNCH_V((convert_kernel<double, float>), nc, s, nc, (const double *)w.mg_x[l + 1], tc);
        // prolong: x += J e_c  (sres reused for the fine-sized interpolant)
        SEM_TRY(launch_interp<float>(L.E, C.nq, L.nq, L.Jc32, tc, sres, false, s));
    } else {
        float *rc = (float *)w.mg_r[l + 1];
        SEM_TRY(launch_interp<float>(L.E, L.nq, C.nq, L.Jc32, sres, rc, true, s));
        SEM_TRY(launch_gs<float>(C, rc, s));
        LAUNCH_V((mask_kernel<float, float>), nc, s, nc, C.W32, rc);
        SEM_TRY(vcycle(h, l + 1, cfg, s));
        SEM_TRY(launch_interp<float>(L.E, C.nq, L.nq, L.Jc32, (const float *)w.mg_x[l + 1], sres,
                                     false, s));
    }
    LAUNCH_V(add_kernel<float>, n, s, n, (const float *)sres, x);
    // post-smoothing
    SEM_TRY(chebyshev(L, l, h, r, x, false, lmin_f * lmax, lmax_f * lmax, cfg.deg, cfg.h1, cfg.h2, s));
    return SEM_OK;
}

// z = M(r): V-cycle on the FP64 fine residual
static int precondition_pmg(sem_handle h, const double *r, double *z, const SolveCfg &cfg,
                            hipStream_t s)
{
    Workspace &w = h->ws;
    const Level &F = h->lv[0];
    const int64_t n = F.nL;
    LAUNCH_V((convert_kernel<double, float>), n, s, n, r, (float *)w.mg_r[0]);
    SEM_TRY(vcycle(h, 0, cfg, s));
    LAUNCH_V((convert_kernel<float, double>), n, s, n, (const float *)w.mg_x[0], z);
    LAUNCH_V((mask_kernel<double, double>), n, s, n, F.W, z);
    return SEM_OK;
}

static int read_scalars(sem_handle h, const KrylovScalars *sc, KrylovScalars *out, hipStream_t s)
{
    SEM_HIP(hipMemcpyAsync(h->ws.host_sc, sc, sizeof(KrylovScalars), hipMemcpyDeviceToHost, s));
    SEM_HIP(hipStreamSynchronize(s));
    *out = *h->ws.host_sc;
    return SEM_OK;
}

// true residual ||b - A x||_W / ||b||_W in FP64
static int true_residual(sem_handle h, const double *k, double h1, double h2, const double *b,
                         const double *x, double *rel, hipStream_t s)
{
    const Level &F = h->lv[0];
    Workspace &w = h->ws;
    SEM_TRY(launch_ax<double>(F, F.G, F.B, F.D, x, w.w, h1, h2, k, nullptr, nullptr, s));
    SEM_TRY(launch_gs<double>(F, w.w, s));
    // pcg_init computes (W r r, W b b) for r = b - Ax
    LAUNCH_V(pcg_init_kernel, F.nL, s, F.nL, b, (const double *)w.w, F.Dinv, F.W, w.z,
             (double *)nullptr, w.partial, 0);
    const int nb = red_grid(F.nL);
    std::vector<double> hp(3 * nb);
    SEM_HIP(hipMemcpyAsync(hp.data(), w.partial, sizeof(double) * 3 * nb, hipMemcpyDeviceToHost, s));
    SEM_HIP(hipStreamSynchronize(s));
    double rr = 0, bb = 0;
    for (int i = 0; i < nb; ++i) {
        rr += hp[3 * i + 1];
        bb += hp[3 * i + 2];
    }
    *rel = bb > 0 ? std::sqrt(rr / bb) : 0.0;
    return SEM_OK;
}

int pcg_solve(sem_handle h, const double *b, double *x, const sem_solve_opts *o,
              sem_solve_stats *st, hipStream_t s)
{
    using clk = std::chrono::steady_clock;
    const bool pmg = o->precond == SEM_PRECOND_PMG;
    if (pmg && h->n_levels < 2) {
        set_error("sem_pcg_solve: PMG needs a handle built with multigrid levels");
        return SEM_EINVAL;
    }
    if (pmg && o->k) {
        set_error("sem_pcg_solve: PMG supports constant coefficients only (k = NULL)");
        return SEM_EINVAL;
    }
    SolveCfg cfg{o->h1, o->h2, o->tol, o->coarse_tol, o->maxit, std::max(1, o->check_every),
                 std::max(1, o->cheb_degree), std::max(1, o->coarse_maxit)};
    const auto t0 = clk::now();
    SEM_TRY(ensure_workspace(h, pmg));
    Workspace &w = h->ws;
    const Level &F = h->lv[0];
    const int64_t n = F.nL;
    // preconditioner data, cached for constant coefficients
    PrecondKey key;
    key.valid = true;
    key.h1 = o->h1;
    key.h2 = o->h2;
    key.precond = o->precond;
    key.cheb_degree = pmg ? cfg.deg : 0;
    key.lanczos_steps = pmg ? o->lanczos_steps : 0;
    key.lo = pmg ? o->cheb_lo : 0;
    key.hi = pmg ? o->cheb_hi : 0;
    const PrecondKey &old = h->key;
    const bool same = !o->k && old.valid && old.h1 == key.h1 && old.h2 == key.h2 &&
                      (old.precond == key.precond || !pmg) && old.lanczos_steps >= key.lanczos_steps &&
                      (!pmg || (old.precond == SEM_PRECOND_PMG && old.lanczos_steps == key.lanczos_steps));
    if (!same) {
        h->key.valid = false;
        SEM_TRY(compute_dinv(h, 0, o->k, o->h1, o->h2, pmg, s));
        if (pmg) {
            for (int l = 1; l < h->n_levels; ++l)
                SEM_TRY(compute_dinv(h, l, nullptr, o->h1, o->h2, l < h->n_levels - 1, s));
            for (int l = 0; l + 1 < h->n_levels; ++l)
                SEM_TRY(lanczos_lmax(h, l, o->h1, o->h2, std::max(2, o->lanczos_steps), &h->lv[l].lmax, s));
        }
        if (!o->k) h->key = key;
    }
    h->key.lo = key.lo;
    h->key.hi = key.hi;
    h->key.cheb_degree = key.cheb_degree;
    SEM_HIP(hipStreamSynchronize(s));
    const auto t1 = clk::now();

    KrylovScalars hs{};
    int coarse_total = 0;
    if (!pmg) {
        SEM_TRY(pcg_start(F, o->k, o->h1, o->h2, b, x, o->zero_guess != 0, w.r, w.p, w.w, w.partial,
                          w.sc, o->tol, o->maxit, s));
        SEM_TRY(read_scalars(h, w.sc, &hs, s));
        int it = 0;
        while (!hs.done) {
            SEM_TRY(pcg_iterations(F, o->k, o->h1, o->h2, x, w.r, w.p, w.w, w.partial_ax, w.partial,
                                   w.sc, it + 1, cfg.check_every, s));
            it += cfg.check_every;
            SEM_TRY(read_scalars(h, w.sc, &hs, s));
        }
    } else {
        // r = b - A x ; z = M r ; p = z ; rz = (z, r)
        const double *Ax = nullptr;
        if (o->zero_guess) {
            LAUNCH_V(fill_kernel<double>, n, s, n, x, 0.0);
        } else {
            LAUNCH_V((mask_kernel<double, double>), n, s, n, F.W, x);
            SEM_TRY(launch_ax<double>(F, F.G, F.B, F.D, x, w.w, o->h1, o->h2, nullptr, nullptr, nullptr, s));
            SEM_TRY(launch_gs<double>(F, w.w, s));
            Ax = w.w;
        }
        LAUNCH_V(pcg_init_kernel, n, s, n, b, Ax, F.Dinv, F.W, w.r, (double *)nullptr, w.partial, 0);
        LAUNCH_1(fin_init_kernel, s, w.partial, (int64_t)red_grid(n), w.sc, o->tol, o->maxit);
        SEM_TRY(read_scalars(h, w.sc, &hs, s));
        const int nbv = red_grid(n);
        if (!hs.done) {
            SEM_TRY(precondition_pmg(h, w.r, w.z, cfg, s));
            LAUNCH_V(dot_zw_kernel, n, s, n, (const KrylovScalars *)w.sc, F.W, (const double *)w.z,
                     (const double *)w.r, (const double *)w.r, w.partial);
            LAUNCH_V(fcg_p_fused_kernel, n, s, n, w.sc, 1, (const double *)w.partial, (int64_t)nbv,
                     (const double *)w.z, w.p, 1);
        }
        for (int it = 0; !hs.done; ++it) {
            const int parity = it & 1;
            int64_t nbax = 0;
            SEM_TRY(launch_ax<double>(F, F.G, F.B, F.D, w.p, w.w, o->h1, o->h2, nullptr, w.partial_ax,
                                      &nbax, s, &w.sc->done));
            SEM_TRY(launch_gs<double>(F, w.w, s, &w.sc->done));
            LAUNCH_V(fcg_update_fused_kernel, n, s, n, w.sc, parity, (const double *)w.partial_ax,
                     nbax, (const double *)w.p, (const double *)w.w, (const int32_t *)nullptr, F.perm,
                     F.offs, F.W, x, w.r, w.partial);
            LAUNCH_1(fin_conv_kernel, s, w.partial, (int64_t)nbv, w.sc);
            SEM_TRY(read_scalars(h, w.sc, &hs, s));
            if (hs.done) break;
            SEM_TRY(precondition_pmg(h, w.r, w.z, cfg, s));
            LAUNCH_V(dot_zw_kernel, n, s, n, (const KrylovScalars *)w.sc, F.W, (const double *)w.z,
                     (const double *)w.w, (const double *)w.r, w.partial);
            LAUNCH_V(fcg_p_fused_kernel, n, s, n, w.sc, parity, (const double *)w.partial,
                     (int64_t)nbv, (const double *)w.z, w.p, 0);
            KrylovScalars csc{};
            SEM_HIP(hipMemcpyAsync(&w.host_sc[1], w.sc_c, sizeof(KrylovScalars), hipMemcpyDeviceToHost, s));
            SEM_TRY(read_scalars(h, w.sc, &hs, s));
            csc = w.host_sc[1];
            coarse_total += csc.iters;
        }
    }
    const auto t2 = clk::now();
    double trr = 0.0;
    SEM_TRY(true_residual(h, o->k, o->h1, o->h2, b, x, &trr, s));
    if (st) {
        st->iters = hs.iters;
        st->rel_res = hs.bb > 0 ? std::sqrt(std::max(hs.rr, 0.0) / hs.bb) : 0.0;
        st->converged = (hs.status == SEM_OK && (hs.bb == 0.0 || hs.rr <= hs.tol2)) ? 1 : 0;
        st->true_rel_res = trr;
        st->ms_setup = std::chrono::duration<double, std::milli>(t1 - t0).count();
        st->ms_solve = std::chrono::duration<double, std::milli>(t2 - t1).count();
        st->coarse_iters = coarse_total;
    }
    if (hs.status == SEM_EBREAKDOWN) {
        set_error("sem_pcg_solve: breakdown after %d iterations", hs.iters);
        return SEM_EBREAKDOWN;
    }
    if (!(hs.bb == 0.0 || hs.rr <= hs.tol2)) {
        set_error("sem_pcg_solve: not converged after %d iterations (rel res %.3e)", hs.iters,
                  hs.bb > 0 ? std::sqrt(hs.rr / hs.bb) : 0.0);
        return SEM_ENOCONV;
    }
    return SEM_OK;
}

// b = R QQ^T (B o f)
int assemble_load(sem_handle h, const double *f, double *b, hipStream_t s)
{
    const Level &F = h->lv[0];
    const int64_t n = F.nL;
    LAUNCH_V(mass_kernel, n, s, n, F.B, f, b);
    SEM_TRY(launch_gs<double>(F, b, s));
    LAUNCH_V((mask_kernel<double, double>), n, s, n, F.W, b);
    return SEM_OK;
}

int adjoint(sem_handle h, const double *u, const double *g, const sem_solve_opts *o, double *lam,
            double *grad_f, double *grad_k, sem_solve_stats *st, hipStream_t s)
{
    const Level &F = h->lv[0];
    const int64_t n = F.nL;
    SEM_TRY(ensure_workspace(h, false));
    if (!h->ws.aux) SEM_HIP(hipMalloc(&h->ws.aux, sizeof(double) * n));
    // right-hand side R QQ^T g in a workspace vector the solver does not touch
    double *rhs = h->ws.aux;
    SEM_HIP(hipMemcpyAsync(rhs, g, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    SEM_TRY(launch_gs<double>(F, rhs, s));
    LAUNCH_V((mask_kernel<double, double>), n, s, n, F.W, rhs);
    sem_solve_opts oo = *o;
    oo.zero_guess = 1;
    if (oo.k != nullptr || h->n_levels < 2) oo.precond = SEM_PRECOND_JACOBI;
    const int rc = pcg_solve(h, rhs, lam, &oo, st, s);
    if (rc != SEM_OK && rc != SEM_ENOCONV) return rc;
    if (grad_f) LAUNCH_V(mass_kernel, n, s, n, F.B, lam, grad_f);
    if (grad_k) SEM_TRY(launch_grad_k(F, u, lam, o->h1, grad_k, s));
    SEM_HIP(hipStreamSynchronize(s));
    return rc;
}

}  // namespace semx

using namespace semx;

extern "C" {

int sem_rhs(sem_handle h, const double *f, double *b, void *stream)
{
    if (!h || !f || !b) {
        set_error("sem_rhs: null argument");
        return SEM_EINVAL;
    }
    return assemble_load(h, f, b, (hipStream_t)stream);
}

int sem_adjoint(sem_handle h, const double *u, const double *g, const sem_solve_opts *o,
                double *lam, double *grad_f, double *grad_k, sem_solve_stats *st, void *stream)
{
    if (!h || !u || !g || !o || !lam) {
        set_error("sem_adjoint: null argument");
        return SEM_EINVAL;
    }
    return adjoint(h, u, g, o, lam, grad_f, grad_k, st, (hipStream_t)stream);
}

void sem_solve_opts_default(sem_solve_opts *o)
{
    if (!o) return;
    o->h1 = 1.0;
    o->h2 = 0.0;
    o->k = nullptr;
    o->tol = 1e-8;
    o->maxit = 1000;
    o->precond = SEM_PRECOND_JACOBI;
    o->check_every = 8;
    o->cheb_degree = 2;
    o->lanczos_steps = 20;
    o->cheb_lo = 0.1;
    o->cheb_hi = 1.1;
    o->coarse_tol = 1e-2;
    o->coarse_maxit = 20;
    o->zero_guess = 1;
}

int sem_pcg_solve(sem_handle h, const double *b, double *x, const sem_solve_opts *o,
                  sem_solve_stats *st, void *stream)
{
    if (!h || !b || !x || !o) {
        set_error("sem_pcg_solve: null argument");
        return SEM_EINVAL;
    }
    if (!(o->tol >= 0.0) || o->maxit < 0 || (o->precond != SEM_PRECOND_JACOBI && o->precond != SEM_PRECOND_PMG)) {
        set_error("sem_pcg_solve: bad options");
        return SEM_EINVAL;
    }
    if (o->precond == SEM_PRECOND_PMG &&
        (!(o->cheb_hi > o->cheb_lo) || !(o->cheb_lo > 0.0) || o->lanczos_steps < 2)) {
        set_error("sem_pcg_solve: bad Chebyshev options");
        return SEM_EINVAL;
    }
    return pcg_solve(h, b, x, o, st, (hipStream_t)stream);
}

}  // extern "C"
