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
#include <cstdlib>
#include <initializer_list>
#include <cmath>
#include <mutex>
#include <vector>

#include "sem_internal.h"
#include "coarse_csr.h"

namespace semx {

constexpr int kRB = 256;          // reduction block size
constexpr int kMaxRedBlocks = 1024;
constexpr int kRedMinPerThread = 4;  // entries per thread before a second block is used

// blocks of the vector kernels over n entries: at most kMaxRedBlocks, and at
// least kRedMinPerThread entries per thread, so a small level's kernels
// dispatch few blocks and leave few partial records for the next kernel
static int red_grid(int64_t n)
{
    const int64_t nb = (n + (int64_t)kRB * kRedMinPerThread - 1) / ((int64_t)kRB * kRedMinPerThread);
    return (int)std::max<int64_t>(1, std::min<int64_t>(nb, kMaxRedBlocks));
}

// the vectorised forms apply (float4 per lane for FP32 streams, a double2
// pair per lane for FP64 ones): n and ld multiples of 4, every array (null
// entries ignored) 16-byte aligned
static bool vec_ok(int64_t n, int64_t ld, std::initializer_list<const void *> ptrs)
{
    if ((n | ld) & 3) return false;
    for (const void *p : ptrs)
        if (p && (reinterpret_cast<uintptr_t>(p) & 15)) return false;
    return true;
}

// Fixed-order tree over the kRB per-thread values acc[q] of a block: pairs
// (t, t + st) for st = kRB / 2, ..., 1, the steps down to 64 through LDS and
// the last six inside wavefront 0 by lane shuffles (same pairs, no barriers).
// The block's sums end in thread 0's acc.
template <int NV>
__device__ inline void block_tree(double (&sh)[NV][kRB], double (&acc)[NV])
{
    const int t = threadIdx.x;
#pragma unroll
    for (int q = 0; q < NV; ++q) sh[q][t] = acc[q];
    __syncthreads();
#pragma unroll
    for (int st = kRB / 2; st >= 64; st >>= 1) {
        if (t < st)
#pragma unroll
            for (int q = 0; q < NV; ++q) sh[q][t] += sh[q][t + st];
        __syncthreads();
    }
    if (t < 64) {
#pragma unroll
        for (int q = 0; q < NV; ++q) acc[q] = sh[q][t];
#pragma unroll
        for (int st = 32; st >= 1; st >>= 1)
#pragma unroll
            for (int q = 0; q < NV; ++q) acc[q] += __shfl_down(acc[q], st, 64);
    }
}

// deterministic block sum of NV values per thread; thread 0 writes
// out[blockIdx.x * NV + q] for q < NV
template <int NV>
__device__ inline void block_sum_store(const double (&v)[NV], double *out)
{
    __shared__ double sh[NV][kRB];
    double acc[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) acc[q] = v[q];
    block_tree<NV>(sh, acc);
    if (threadIdx.x == 0)
#pragma unroll
        for (int q = 0; q < NV; ++q) out[(int64_t)blockIdx.x * NV + q] = acc[q];
}

// deterministic sum of nb partial records of NV values (one block of kRB),
// returned to every thread.  Thread t adds records t, t + kRB, ... in order;
// the loads of kPartUnroll consecutive records are issued before their adds,
// so a long partial list costs few memory round trips.
constexpr int kPartUnroll = 8;
template <int NV>
__device__ inline void sum_partials(const double *partial, int64_t nb, double (&res)[NV])
{
    __shared__ double sh[NV][kRB];
    __shared__ double bc[NV];
    const int t = threadIdx.x;
    double acc[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) acc[q] = 0.0;
    int64_t b = t;
    for (; b + (kPartUnroll - 1) * kRB < nb; b += kPartUnroll * kRB) {
        double v[kPartUnroll][NV];
#pragma unroll
        for (int u = 0; u < kPartUnroll; ++u)
#pragma unroll
            for (int q = 0; q < NV; ++q) v[u][q] = partial[(b + u * kRB) * NV + q];
#pragma unroll
        for (int u = 0; u < kPartUnroll; ++u)
#pragma unroll
            for (int q = 0; q < NV; ++q) acc[q] += v[u][q];
    }
    for (; b < nb; b += kRB)
#pragma unroll
        for (int q = 0; q < NV; ++q) acc[q] += partial[b * NV + q];
    block_tree<NV>(sh, acc);
    if (t == 0)
#pragma unroll
        for (int q = 0; q < NV; ++q) bc[q] = acc[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q) res[q] = bc[q];
}

// Paired forms of the FP64 vector kernels: lane work on two consecutive
// points, one double2 (16 bytes) per FP64 array and one float2 per FP32 array
// (arrays 16-byte aligned, checked by the launching code).
// two consecutive values g*2, g*2+1 as one access
__device__ inline void ld2(const double *p, int64_t g, double (&o)[2])
{
    const double2 a = reinterpret_cast<const double2 *>(p)[g];
    o[0] = a.x;
    o[1] = a.y;
}
__device__ inline void st2(double *p, int64_t g, const double (&o)[2])
{
    reinterpret_cast<double2 *>(p)[g] = make_double2(o[0], o[1]);
}
__device__ inline void ld2(const float *p, int64_t g, float (&o)[2])
{
    const float2 a = reinterpret_cast<const float2 *>(p)[g];
    o[0] = a.x;
    o[1] = a.y;
}
__device__ inline void st2(float *p, int64_t g, const float (&o)[2])
{
    reinterpret_cast<float2 *>(p)[g] = make_float2(o[0], o[1]);
}

// ------------------------------------------------------------------ vectors
// Kernels over a batch of vectors take the batch `vs` and the leading
// dimension of each array; grid.y runs over the vectors of the batch, and
// vector v's Krylov scalars and partial sums are sc[v] and partial + v * pst.
__device__ inline int64_t vsel(const VSet &vs) { return vs.at(blockIdx.y); }

#define GRID_LOOP(i, n)                                                                    \
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n);              \
         i += (int64_t)gridDim.x * blockDim.x)

template <typename T>
__global__ void fill_kernel(int64_t n, VSet vs, int64_t ld, T *v, T val)
{
    T *q = v + vsel(vs) * ld;
    GRID_LOOP(i, n) q[i] = val;
}

template <typename T, typename TW>
__global__ void mask_kernel(int64_t n, VSet vs, int64_t ld, const TW *__restrict__ W, T *__restrict__ v)
{
    T *q = v + vsel(vs) * ld;
    GRID_LOOP(i, n)
        if (!(W[i] > TW(0))) q[i] = T(0);
}

template <typename TA, typename TB>
__global__ void convert_kernel(int64_t n, VSet vs, int64_t lda, const TA *__restrict__ a, int64_t ldb,
                               TB *__restrict__ b)
{
    const int64_t v = vsel(vs);
    const TA *pa = a + v * lda;
    TB *pb = b + v * ldb;
    GRID_LOOP(i, n) pb[i] = (TB)pa[i];
}

__global__ void invert_diag_kernel(int64_t n, const double *__restrict__ W,
                                   const double *__restrict__ d, double *__restrict__ Dinv,
                                   float *__restrict__ Dinv32)
{
    GRID_LOOP(i, n) {
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
    GRID_LOOP(i, n) s[0] += W[i] * a[i] * b[i];
    block_sum_store<1>(s, partial);
}

// ---------------------------------------------------------------- Jacobi-PCG
// r = b - Ax (Ax may be null: x = 0), p = Dinv r; partials (W r p, W r r, W b b)
// r32 (nullable): FP32 copy of r, the p-multigrid input
__global__ void pcg_init_kernel(int64_t n, VSet vs, int64_t ldb, const double *__restrict__ b,
                                int64_t ld, const double *__restrict__ Ax,
                                const double *__restrict__ Dinv, const double *__restrict__ W,
                                double *__restrict__ r, double *__restrict__ p,
                                float *__restrict__ r32, double *__restrict__ partial, int64_t pst,
                                int precondition)
{
    const int64_t v = vsel(vs);
    b += v * ldb;
    if (Ax) Ax += v * ld;
    r += v * ld;
    if (p) p += v * ld;
    if (r32) r32 += v * ld;
    double s[3] = {0.0, 0.0, 0.0};
    GRID_LOOP(i, n) {
        const double ri = b[i] - (Ax ? Ax[i] : 0.0);
        r[i] = ri;
        if (r32) r32[i] = (float)ri;
        const double zi = precondition ? Dinv[i] * ri : ri;
        if (p) p[i] = zi;
        const double wi = W[i];
        s[0] += wi * ri * zi;
        s[1] += wi * ri * ri;
        s[2] += wi * b[i] * b[i];
    }
    block_sum_store<3>(s, partial + v * pst);
}

// reference (b, b)_W per vector for the stopping test (0: that of the
// right-hand side being solved); set when the system solved is the remainder
// of a projected guess and the tolerance stays relative to the original b
struct BbRef {
    double v[kMaxRhs];
};

// one block per vector
__global__ void fin_init_kernel(VSet vs, const double *partial, int64_t pst, int64_t nb,
                                KrylovScalars *sc, double tol, int maxit, BbRef ref)
{
    const int64_t v = vsel(vs);
    sc += v;
    double res[3];
    sum_partials<3>(partial + v * pst, nb, res);
    if (ref.v[v] > 0.0) res[2] = ref.v[v];
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
// Jacobi-PCG update.  Every block sums the operator kernel's partials of
// (p, A_L p) in the same fixed order, so all blocks hold the same alpha;
// x += alpha p; r -= alpha QQ^T(A_L p) (w already assembled); partials
// (W r Dinv r, W r r).  rz2[parity] is the current (r, z).
__global__ void pcg_update_fused_kernel(int64_t n, VSet vs, int64_t ld, int64_t ldx,
                                        KrylovScalars *sc, int parity,
                                        const double *__restrict__ pax, int64_t pst_ax, int64_t nbax,
                                        const double *__restrict__ p, const double *__restrict__ w,
                                        const double *__restrict__ Dinv,
                                        const double *__restrict__ W, double *__restrict__ x,
                                        double *__restrict__ r, double *__restrict__ partial,
                                        int64_t pst)
{
    const int64_t v = vsel(vs);
    sc += v;
    if (sc->done) return;
    p += v * ld;
    w += v * ld;
    r += v * ld;
    x += v * ldx;
    double res[1];
    sum_partials<1>(pax + v * pst_ax, nbax, res);
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
    GRID_LOOP(i, n) {
        x[i] += a * p[i];
        const double ri = r[i] - a * w[i];
        r[i] = ri;
        const double wr = W[i] * ri;
        s[0] += wr * Dinv[i] * ri;
        s[1] += wr * ri;
    }
    block_sum_store<2>(s, partial + v * pst);
}

// Jacobi-PCG direction update with beta and the convergence decision taken
// by every block from the update's partials (identical in all blocks);
// block 0 records them.  `iter` is the 1-based number of this iteration.
__global__ void pcg_p_fused_kernel(int64_t n, VSet vs, int64_t ld, KrylovScalars *sc, int parity,
                                   int iter, const double *__restrict__ pu, int64_t pst, int64_t nbu,
                                   const double *__restrict__ Dinv, const double *__restrict__ r,
                                   double *__restrict__ p)
{
    const int64_t v = vsel(vs);
    sc += v;
    if (sc->done) return;
    r += v * ld;
    p += v * ld;
    double res[2];
    sum_partials<2>(pu + v * pst, nbu, res);
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
    GRID_LOOP(i, n) p[i] = Dinv[i] * r[i] + be * p[i];
}

// flexible-CG update: alpha from the operator partials, x += alpha p,
// r -= alpha QQ^T(A_L p), r32 = FP32 copy of r (the V-cycle input);
// partial (W r r)
template <bool PAIR>
__global__ void fcg_update_fused_kernel(int64_t n, VSet vs, int64_t ld, int64_t ldx,
                                        KrylovScalars *sc, int parity,
                                        const double *__restrict__ pax, int64_t pst_ax, int64_t nbax,
                                        const double *__restrict__ p, const double *__restrict__ w,
                                        const double *__restrict__ W, double *__restrict__ x,
                                        double *__restrict__ r, float *__restrict__ r32,
                                        double *__restrict__ partial, int64_t pst)
{
    const int64_t v = vsel(vs);
    sc += v;
    if (sc->done) return;
    p += v * ld;
    w += v * ld;
    r += v * ld;
    r32 += v * ld;
    x += v * ldx;
    double res[1];
    sum_partials<1>(pax + v * pst_ax, nbax, res);
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
    if constexpr (PAIR) {
        GRID_LOOP(g, n >> 1) {
            double pp[2], ww[2], xx[2], rr[2], wt[2];
            float rf[2];
            ld2(p, g, pp);
            ld2(w, g, ww);
            ld2(x, g, xx);
            ld2(r, g, rr);
            ld2(W, g, wt);
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                xx[k] += a * pp[k];
                const double ri = rr[k] - a * ww[k];
                rr[k] = ri;
                rf[k] = (float)ri;
                s[0] += wt[k] * ri * ri;
            }
            st2(x, g, xx);
            st2(r, g, rr);
            st2(r32, g, rf);
        }
    } else {
        GRID_LOOP(i, n) {
            x[i] += a * p[i];
            const double ri = r[i] - a * w[i];
            r[i] = ri;
            r32[i] = (float)ri;
            s[0] += W[i] * ri * ri;
        }
    }
    block_sum_store<1>(s, partial + v * pst);
}

// (z, w)_W and (z, r)_W for assembled w, z the FP32 V-cycle output taken to
// FP64 (W = 0 on Dirichlet copies applies the restriction)
__global__ void dot_zw_kernel(int64_t n, VSet vs, int64_t ld, const KrylovScalars *sc,
                              const double *__restrict__ W, const float *__restrict__ z,
                              const double *__restrict__ wa, const double *__restrict__ r,
                              double *__restrict__ partial, int64_t pst)
{
    const int64_t v = vsel(vs);
    if (sc[v].done) return;
    z += v * ld;
    wa += v * ld;
    r += v * ld;
    double s[2] = {0.0, 0.0};
    GRID_LOOP(i, n) {
        const double wz = W[i] * (double)z[i];
        s[0] += wz * wa[i];
        s[1] += wz * r[i];
    }
    block_sum_store<2>(s, partial + v * pst);
}

// Polak-Ribiere direction update, beta = (z_new, r_new - r_old) / (z_old, r_old)
// = -alpha (z_new, A p) / rz_old (r_new - r_old = -alpha A p), taken by every
// block from the partials of dot_zw_kernel; first = 1 gives p = z without
// reading p (on the first iteration p is uninitialised memory, and a 0 * p
// term would turn any NaN bit pattern it holds into a NaN direction).  z is
// the FP32 V-cycle output, zero on Dirichlet copies (mask W32 > 0).
template <bool PAIR>
__global__ void fcg_p_fused_kernel(int64_t n, VSet vs, int64_t ld, KrylovScalars *sc, int parity,
                                   const double *__restrict__ pz, int64_t pst, int64_t nbz,
                                   const float *__restrict__ z, const float *__restrict__ W32,
                                   double *__restrict__ p, int first)
{
    const int64_t v = vsel(vs);
    sc += v;
    if (sc->done) return;
    z += v * ld;
    p += v * ld;
    double res[2];
    sum_partials<2>(pz + v * pst, nbz, res);
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
    if constexpr (PAIR) {
        GRID_LOOP(g, n >> 1) {
            float zz[2], wt[2];
            double pp[2] = {0.0, 0.0};
            ld2(z, g, zz);
            ld2(W32, g, wt);
            if (!first) ld2(p, g, pp);
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const double zk = wt[k] > 0.0f ? (double)zz[k] : 0.0;
                pp[k] = first ? zk : zk + be * pp[k];
            }
            st2(p, g, pp);
        }
    } else {
        GRID_LOOP(i, n) {
            const double zi = W32[i] > 0.0f ? (double)z[i] : 0.0;
            p[i] = first ? zi : zi + be * p[i];
        }
    }
}

// Chebyshev step on assembled t = QQ^T A_L x (t null when x = 0):
// res = r - t, d = c1 d + c2 Dinv res, x += d (x = d when `init`)
// One Chebyshev-Jacobi point update (res = r - t, or r when t is absent).
__device__ inline void cheb_pt(float r, float t, bool has_t, float dinv, float &d, float &x,
                               float c1, float c2, int init)
{
    const float res = has_t ? r - t : r;
    const float di = (init ? 0.0f : c1 * d) + c2 * dinv * res;
    d = di;
    x = init ? di : x + di;
}

// FP32 streaming kernels take 16 bytes per lane (float4) when V4: n and ld
// multiples of 4 and every array 16-byte aligned (checked by the caller); the
// arithmetic per point is the same as in the one-float form.
#define FLOAT4_AT(p, i) (reinterpret_cast<const float4 *>(p)[i])

template <bool V4>
__global__ void cheb_fused_kernel(int64_t n, VSet vs, int64_t ld, const float *__restrict__ r,
                                  const float *__restrict__ t, const float *__restrict__ Dinv,
                                  float *__restrict__ d, float *__restrict__ x, float c1, float c2,
                                  int init)
{
    const int64_t v = vsel(vs);
    r += v * ld;
    if (t) t += v * ld;
    d += v * ld;
    x += v * ld;
    const bool ht = t != nullptr;
    if constexpr (V4) {
        GRID_LOOP(i, n >> 2) {
            const float4 rv = FLOAT4_AT(r, i), gv = FLOAT4_AT(Dinv, i);
            const float4 tv = ht ? FLOAT4_AT(t, i) : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            float4 dv = make_float4(0.0f, 0.0f, 0.0f, 0.0f), xv = dv;
            if (!init) {
                dv = FLOAT4_AT(d, i);
                xv = FLOAT4_AT(x, i);
            }
            cheb_pt(rv.x, tv.x, ht, gv.x, dv.x, xv.x, c1, c2, init);
            cheb_pt(rv.y, tv.y, ht, gv.y, dv.y, xv.y, c1, c2, init);
            cheb_pt(rv.z, tv.z, ht, gv.z, dv.z, xv.z, c1, c2, init);
            cheb_pt(rv.w, tv.w, ht, gv.w, dv.w, xv.w, c1, c2, init);
            reinterpret_cast<float4 *>(d)[i] = dv;
            reinterpret_cast<float4 *>(x)[i] = xv;
        }
    } else {
        GRID_LOOP(i, n) {
            float di = init ? 0.0f : d[i], xi = init ? 0.0f : x[i];
            cheb_pt(r[i], ht ? t[i] : 0.0f, ht, Dinv[i], di, xi, c1, c2, init);
            d[i] = di;
            x[i] = xi;
        }
    }
}

// Chebyshev step with the Schwarz smoother: z = wgt o acc (acc = QQ^T of the
// combined local solutions), d = c1 d + c2 z, x += d (x = d when `init`)
template <bool V4>
__global__ void cheb_w_kernel(int64_t n, VSet vs, int64_t ld, const float *__restrict__ wgt,
                              const float *__restrict__ acc, float *__restrict__ d,
                              float *__restrict__ x, float c1, float c2, int init)
{
    const int64_t v = vsel(vs);
    acc += v * ld;
    d += v * ld;
    x += v * ld;
    auto pt = [&](float wg, float ac, float &dd, float &xx) {
        const float di = (init ? 0.0f : c1 * dd) + c2 * wg * ac;
        dd = di;
        xx = init ? di : xx + di;
    };
    if constexpr (V4) {
        GRID_LOOP(i, n >> 2) {
            const float4 wv = FLOAT4_AT(wgt, i), av = FLOAT4_AT(acc, i);
            float4 dv = make_float4(0.0f, 0.0f, 0.0f, 0.0f), xv = dv;
            if (!init) {
                dv = FLOAT4_AT(d, i);
                xv = FLOAT4_AT(x, i);
            }
            pt(wv.x, av.x, dv.x, xv.x);
            pt(wv.y, av.y, dv.y, xv.y);
            pt(wv.z, av.z, dv.z, xv.z);
            pt(wv.w, av.w, dv.w, xv.w);
            reinterpret_cast<float4 *>(d)[i] = dv;
            reinterpret_cast<float4 *>(x)[i] = xv;
        }
    } else {
        GRID_LOOP(i, n) {
            float di = init ? 0.0f : d[i], xi = init ? 0.0f : x[i];
            pt(wgt[i], acc[i], di, xi);
            d[i] = di;
            x[i] = xi;
        }
    }
}

// partial (W a b) sums of FP32 vectors in FP64
__global__ void dot32_kernel(int64_t n, const double *__restrict__ W, const float *__restrict__ a,
                             const float *__restrict__ b, double *__restrict__ partial)
{
    double s[1] = {0.0};
    GRID_LOOP(i, n) s[0] += W[i] * (double)a[i] * (double)b[i];
    block_sum_store<1>(s, partial);
}

// y = alpha (w o x)   (w nullable: y = alpha x)
__global__ void wscale32_kernel(int64_t n, const float *__restrict__ w, const float *__restrict__ x,
                                float alpha, float *__restrict__ y)
{
    GRID_LOOP(i, n) y[i] = alpha * (w ? w[i] * x[i] : x[i]);
}

// s = W (r - t) for assembled t
__global__ void wresid_fused_kernel(int64_t n, VSet vs, int64_t ld, const float *__restrict__ W,
                                    const float *__restrict__ r, const float *__restrict__ t,
                                    float *__restrict__ s)
{
    const int64_t v = vsel(vs);
    r += v * ld;
    t += v * ld;
    s += v * ld;
    GRID_LOOP(i, n) s[i] = W[i] * (r[i] - t[i]);
}

// flexible CG convergence decision after the update (one block per vector):
// iteration count, (r, r)_W, done
__global__ void fin_conv_kernel(VSet vs, const double *partial, int64_t pst, int64_t nb,
                                KrylovScalars *sc)
{
    const int64_t v = vsel(vs);
    sc += v;
    if (sc->done) return;
    double res[1];
    sum_partials<1>(partial + v * pst, nb, res);
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
__global__ void add_kernel(int64_t n, VSet vs, int64_t ld, const T *__restrict__ a, T *__restrict__ y)
{
    const int64_t v = vsel(vs);
    a += v * ld;
    y += v * ld;
    GRID_LOOP(i, n) y[i] += a[i];
}

// ------------------------------------------------------------- projection
struct Coefs {
    double c[kMaxProj];
};

// partial sums of (W a, y_q) for q < m, y_q = Y + q * ldY (kMaxProj records
// per block, the first m used)
__global__ void wdots_kernel(int64_t n, const double *__restrict__ W, const double *__restrict__ a,
                             const double *__restrict__ Y, int64_t ldY, int m,
                             double *__restrict__ partial)
{
    double s[kMaxProj];
#pragma unroll
    for (int q = 0; q < kMaxProj; ++q) s[q] = 0.0;
    GRID_LOOP(i, n) {
        const double wa = W[i] * a[i];
#pragma unroll
        for (int q = 0; q < kMaxProj; ++q)
            if (q < m) s[q] += wa * Y[q * ldY + i];
    }
    block_sum_store<kMaxProj>(s, partial);
}

// out = c0 base + sum_{q < m} c_q y_q  (base nullable; out may be base)
__global__ void lincomb_kernel(int64_t n, const double *base, double c0,
                               const double *__restrict__ Y, int64_t ldY, int m, Coefs c,
                               double *out)
{
    GRID_LOOP(i, n) {
        double acc = base ? c0 * base[i] : 0.0;
#pragma unroll
        for (int q = 0; q < kMaxProj; ++q)
            if (q < m) acc += c.c[q] * Y[q * ldY + i];
        out[i] = acc;
    }
}

// out = c0 a0 + c1 a1 + c2 a2 (a1, a2 nullable; out may alias any input)
__global__ void lincomb3_kernel(int64_t n, const double *a0, double c0, const double *a1, double c1,
                                const double *a2, double c2, double *out)
{
    GRID_LOOP(i, n) {
        double acc = c0 * a0[i];
        if (a1) acc += c1 * a1[i];
        if (a2) acc += c2 * a2[i];
        out[i] = acc;
    }
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

// y = a x + b y (y not read when b = 0; x may be y)
__global__ void axpby_kernel(int64_t n, const double *x, double a, double b, double *y)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = a * x[i] + (b == 0.0 ? 0.0 : b * y[i]);
}

// ============================================================== host side
#define LAUNCH_V(kern, n, s, ...)                                                           \
    do {                                                                                    \
        hipLaunchKernelGGL(kern, dim3(red_grid(n)), dim3(kRB), 0, s, __VA_ARGS__);          \
        SEM_HIP(hipGetLastError());                                                         \
    } while (0)
// one grid row per vector of the batch vs
#define LAUNCH_B(kern, len_, vs_, s_, ...)                                                  \
    do {                                                                                    \
        hipLaunchKernelGGL(kern, dim3(red_grid(len_), (unsigned)(vs_).n), dim3(kRB), 0, s_, \
                           __VA_ARGS__);                                                    \
        SEM_HIP(hipGetLastError());                                                         \
    } while (0)
// the vectorised form of a vector kernel (kern<true>) when ok_, else the
// one-value form; the grid (and so the number of partial records) is the same
// for both
#define LAUNCH_B_VEC(ok_, kern, len_, vs_, s_, ...)                                          \
    do {                                                                                    \
        if (ok_)                                                                            \
            LAUNCH_B(kern<true>, len_, vs_, s_, __VA_ARGS__);                               \
        else                                                                                \
            LAUNCH_B(kern<false>, len_, vs_, s_, __VA_ARGS__);                              \
    } while (0)
#define LAUNCH_1B(kern, vs_, s_, ...)                                                       \
    do {                                                                                    \
        hipLaunchKernelGGL(kern, dim3(1, (unsigned)(vs_).n), dim3(kRB), 0, s_, __VA_ARGS__); \
        SEM_HIP(hipGetLastError());                                                         \
    } while (0)

// stride, in ints, between the `done` flags of consecutive KrylovScalars
constexpr int kScStride = (int)(sizeof(KrylovScalars) / sizeof(int));
static_assert(sizeof(KrylovScalars) % sizeof(int) == 0, "KrylovScalars size");

// Solver workspace allocation.  With SEM_POISON_WORKSPACE set to a nonzero
// value in the environment, every new buffer is filled with 0xFF bytes (NaN
// as FP32 and FP64), so that a kernel reading workspace it has not written
// shows up as NaN instead of depending on what the memory held before.
static int ws_alloc(void **p, size_t bytes)
{
    SEM_HIP(hipMalloc(p, bytes));
    const char *e = std::getenv("SEM_POISON_WORKSPACE");
    if (e && std::atoi(e) != 0) SEM_HIP(hipMemset(*p, 0xFF, bytes));
    return SEM_OK;
}

static void free_vectors(Workspace &w)
{
    void *ptrs[] = {w.r, w.p, w.w, w.z, w.c_r, w.c_p, w.c_w};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    w.r = w.p = w.w = w.z = w.c_r = w.c_p = w.c_w = nullptr;
    for (int l = 0; l < kMaxLevels; ++l) {
        void **q[] = {&w.mg_r[l], &w.mg_x[l], &w.mg_t[l], &w.mg_d[l], &w.mg_s[l]};
        for (void **p : q) {
            if (*p) (void)hipFree(*p);
            *p = nullptr;
        }
    }
    w.nv = 0;
    w.pmg = false;
}

static void free_projection(Workspace &w)
{
    for (int v = 0; v < kMaxRhs; ++v) {
        if (w.proj[v].xt) (void)hipFree(w.proj[v].xt);
        if (w.proj[v].bt) (void)hipFree(w.proj[v].bt);
        w.proj[v] = Workspace::Proj{};
    }
    if (w.proj_xb) (void)hipFree(w.proj_xb);
    if (w.proj_bp) (void)hipFree(w.proj_bp);
    w.proj_xb = w.proj_bp = nullptr;
    w.proj_L = w.proj_nv = 0;
}

// ------------------------------------------------------------ phase clock
constexpr int kClockEvents = 512;

static int clock_begin(Workspace &w, bool on)
{
    PhaseClock &c = w.clk;
    c.on = on;
    c.n = 0;
    for (double &m : c.ms) m = 0.0;
    if (on && c.ev.empty()) {
        c.ev.assign(kClockEvents, nullptr);
        c.ph.assign(kClockEvents, -1);
        for (auto &e : c.ev) SEM_HIP(hipEventCreate(&e));
    }
    return SEM_OK;
}

// Charge the intervals of the current chain; the stream has reached its last
// event (after a host synchronisation), or `wait` waits for it.  The chain
// restarts empty: the idle time of the host round trip is charged to nothing.
static int clock_flush(Workspace &w, bool wait)
{
    PhaseClock &c = w.clk;
    if (!c.on || c.n == 0) return SEM_OK;
    if (wait) SEM_HIP(hipEventSynchronize(c.ev[c.n - 1]));
    for (int i = 1; i < c.n; ++i) {
        float ms = 0.0f;
        SEM_HIP(hipEventElapsedTime(&ms, c.ev[i - 1], c.ev[i]));
        if (c.ph[i] >= 0) c.ms[c.ph[i]] += ms;
    }
    c.n = 0;
    return SEM_OK;
}

// A phase boundary on `s`: the device time since the previous boundary is
// phase p's (p = -1, or an empty chain: only the chain's start is set).
static int clock_mark(Workspace &w, int p, hipStream_t s)
{
    PhaseClock &c = w.clk;
    if (!c.on) return SEM_OK;
    if (c.n == (int)c.ev.size()) {  // pool used up: charge it, continue the chain from here
        SEM_TRY(clock_flush(w, true));
        p = -1;
    }
    SEM_HIP(hipEventRecord(c.ev[c.n], s));
    c.ph[c.n] = c.n == 0 ? -1 : p;
    ++c.n;
    return SEM_OK;
}

void free_workspace(sem_handle h)
{
    Workspace &w = h->ws;
    for (auto &e : w.clk.ev)
        if (e) (void)hipEventDestroy(e);
    w.clk.ev.clear();
    for (auto &g : w.vg)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (w.cap) (void)hipStreamDestroy(w.cap);
    free_vectors(w);
    free_projection(w);
    if (w.sz_U) (void)hipFree(w.sz_U);
    for (int l = 0; l < kMaxLevels; ++l)
        if (w.sz_acc[l]) (void)hipFree(w.sz_acc[l]);
    void *ptrs[] = {w.aux, w.partial, w.partial_ax, w.sc, w.sc_c};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
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

// workspace for batches of up to nv vectors (grown, never shrunk)
static int ensure_workspace(sem_handle h, bool pmg, int nv)
{
    Workspace &w = h->ws;
    const Level &F = h->lv[0];
    if (!w.sc) {
        w.nL = F.nL;
        // vector-kernel partials: at most kMaxRedBlocks records of 3 per
        // vector; operator partials: one per workgroup of the persistent grid
        w.pst = 3 * kMaxRedBlocks;
        SEM_TRY(ws_alloc((void **)&w.partial, sizeof(double) * std::max<int64_t>(w.pst * kMaxRhs,
                                                                         (int64_t)kMaxProj * kMaxRedBlocks)));
        w.pst_ax = (int64_t)(F.n_cu > 0 ? F.n_cu : 256) * kAxMaxBlocksPerCU + 64;
        SEM_TRY(ws_alloc((void **)&w.partial_ax, sizeof(double) * w.pst_ax * kMaxRhs));
        SEM_TRY(ws_alloc((void **)&w.sc, sizeof(KrylovScalars) * kMaxRhs));
        SEM_TRY(ws_alloc((void **)&w.sc_c, sizeof(KrylovScalars) * kMaxRhs));
        SEM_HIP(hipHostMalloc((void **)&w.host_sc, 2 * kMaxRhs * sizeof(KrylovScalars),
                              hipHostMallocDefault));
    }
    if (w.nv < nv || (pmg && !w.pmg)) {
        const int nvn = std::max(nv, w.nv);
        const bool pm = pmg || w.pmg;
        free_vectors(w);
        const int64_t n = F.nL;
        SEM_TRY(ws_alloc((void **)&w.r, sizeof(double) * n * nvn));
        SEM_TRY(ws_alloc((void **)&w.p, sizeof(double) * n * nvn));
        SEM_TRY(ws_alloc((void **)&w.w, sizeof(double) * n * nvn));
        SEM_TRY(ws_alloc((void **)&w.z, sizeof(double) * n * nvn));
        if (pm) {
            for (int l = 0; l + 1 < h->n_levels; ++l) {
                const int64_t m = h->lv[l].nL * nvn;
                SEM_TRY(ws_alloc((void **)&w.mg_r[l], sizeof(float) * m));
                SEM_TRY(ws_alloc((void **)&w.mg_x[l], sizeof(float) * m));
                SEM_TRY(ws_alloc((void **)&w.mg_t[l], sizeof(float) * m));
                SEM_TRY(ws_alloc((void **)&w.mg_d[l], sizeof(float) * m));
                if (h->lv[l].nq > 8)  // unfused transfers stage the residual here
                    SEM_TRY(ws_alloc((void **)&w.mg_s[l], sizeof(float) * m));
            }
            const int lc = h->n_levels - 1;
            const int64_t m = h->lv[lc].nL * nvn;
            SEM_TRY(ws_alloc((void **)&w.mg_r[lc], sizeof(double) * m));  // coarse rhs
            SEM_TRY(ws_alloc((void **)&w.mg_x[lc], sizeof(double) * m));  // coarse solution
            SEM_TRY(ws_alloc((void **)&w.c_r, sizeof(double) * m));
            SEM_TRY(ws_alloc((void **)&w.c_p, sizeof(double) * m));
            SEM_TRY(ws_alloc((void **)&w.c_w, sizeof(double) * m));
        }
        w.nv = nvn;
        w.pmg = pm;
    }
    for (int l = 0; l < h->n_levels; ++l) {
        Level &L = h->lv[l];
        if (!L.Dinv) SEM_TRY(ws_alloc((void **)&L.Dinv, sizeof(double) * L.nL));
        if (pmg && l < h->n_levels - 1 && !L.Dinv32) SEM_TRY(ws_alloc((void **)&L.Dinv32, sizeof(float) * L.nL));
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
    const VSet one = VSet::one();
    double *v = w.r, *vp = w.p, *t = w.w, *u = w.z;
    LAUNCH_V(splitmix_kernel, n, s, n, L.gid, L.W, h->lanczos_seed, v);
    double nrm2 = 0.0;
    SEM_TRY(host_dot(L, v, v, w.partial, &nrm2, s));
    if (!(nrm2 > 0.0)) {
        *lmax = 1.0;
        return SEM_OK;
    }
    LAUNCH_V(axpby_kernel, n, s, n, v, 1.0 / std::sqrt(nrm2), 0.0, v);
    LAUNCH_B(fill_kernel<double>, n, one, s, n, one, (int64_t)0, vp, 0.0);
    std::vector<double> al, be;
    double beta = 0.0;
    for (int it = 0; it < steps; ++it) {
        // t = S v ; u = A t (restricted) ; u = S u - beta vp
        LAUNCH_V(sqrtd_axpby_kernel, n, s, n, L.Dinv, v, 1.0, 0.0, t);
        SEM_TRY(launch_ax<double>(L, L.G, L.B, L.D, t, u, h1, h2, nullptr, nullptr, nullptr, s));
        SEM_TRY(launch_gs<double>(L, u, s));
        LAUNCH_B((mask_kernel<double, double>), n, one, s, n, one, (int64_t)0, L.W, u);
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

// FP32 operator on a smoother level for the batch vs (arrays [nv][nL]):
// t = QQ^T A_L x (Dirichlet copies of t are ignored by the consumers, whose
// Dinv and W vanish there)
static int apply_f32(const Level &L, const VSet &vs, const float *x, float *t, double h1, double h2,
                     hipStream_t s)
{
    SEM_TRY(launch_ax_multi<float>(L, L.G32, L.B32, L.D32, x, L.nL, t, L.nL, vs, h1, h2, nullptr,
                                   nullptr, 0, nullptr, s, nullptr, 0));
    return launch_gs_multi<float>(L, t, L.nL, vs, s, nullptr, 0);
}

// Chebyshev-accelerated Jacobi (Saad, Iterative Methods, Alg. 12.1, applied to
// Dinv A x = Dinv r) with `deg` updates; x == 0 on entry when `zero`.
// one smoothing correction of the batch: with Jacobi, d = c1 d + c2 Dinv (r - t)
// fused; with Schwarz, the local FDM solutions of r - t combined, QQ^T and
// weighted, then d = c1 d + c2 z.  t null: x = 0 (res = r).
static int smooth_step(const Level &L, int l, sem_handle h, const VSet &vs, int smoother,
                       const float *r, const float *t, float *d, float *x, float c1, float c2,
                       int init, double h1, double h2, hipStream_t s)
{
    const int64_t n = L.nL;
    if (smoother == SEM_SMOOTH_JACOBI) {
        if (vec_ok(n, n, {r, t, L.Dinv32, d, x}))
            LAUNCH_B(cheb_fused_kernel<true>, n / 4, vs, s, n, vs, n, r, t, L.Dinv32, d, x, c1, c2,
                     init);
        else
            LAUNCH_B(cheb_fused_kernel<false>, n, vs, s, n, vs, n, r, t, L.Dinv32, d, x, c1, c2, init);
        return SEM_OK;
    }
    Workspace &w = h->ws;
    const bool ras = smoother == SEM_SMOOTH_RAS;
    float *acc = w.sz_acc[l];
    SEM_TRY(launch_schwarz(L, ras, r, t, w.sz_U, acc, vs, h1, h2, s));
    SEM_TRY(launch_gs_multi<float>(L, acc, n, vs, s, nullptr, 0));
    const float *wgt = ras ? L.W32 : L.sz_w;
    if (vec_ok(n, n, {wgt, acc, d, x}))
        LAUNCH_B(cheb_w_kernel<true>, n / 4, vs, s, n, vs, n, wgt, (const float *)acc, d, x, c1, c2,
                 init);
    else
        LAUNCH_B(cheb_w_kernel<false>, n, vs, s, n, vs, n, wgt, (const float *)acc, d, x, c1, c2,
                 init);
    return SEM_OK;
}

// Chebyshev acceleration (Saad, Iterative Methods, Alg. 12.1) of the smoother
// x <- x + M^{-1}(r - A x), M = Jacobi or Schwarz, with `deg` updates; x == 0
// on entry when `zero`.
static int chebyshev(const Level &L, int l, sem_handle h, const VSet &vs, int smoother,
                     const float *r, float *x, bool zero, double lmin, double lmax, int deg,
                     double h1, double h2, hipStream_t s)
{
    Workspace &w = h->ws;
    float *t = (float *)w.mg_t[l], *d = (float *)w.mg_d[l];
    const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
    const double sigma = theta / delta;
    double rho_prev = 1.0 / sigma;
    if (zero) {
        SEM_TRY(smooth_step(L, l, h, vs, smoother, r, nullptr, d, x, 0.0f, (float)(1.0 / theta), 1, h1,
                            h2, s));
    } else {
        SEM_TRY(apply_f32(L, vs, x, t, h1, h2, s));
        SEM_TRY(smooth_step(L, l, h, vs, smoother, r, t, d, x, 0.0f, (float)(1.0 / theta), 0, h1, h2,
                            s));
    }
    for (int k = 1; k < deg; ++k) {
        const double rho = 1.0 / (2.0 * sigma - rho_prev);
        SEM_TRY(apply_f32(L, vs, x, t, h1, h2, s));
        SEM_TRY(smooth_step(L, l, h, vs, smoother, r, t, d, x, (float)(rho * rho_prev),
                            (float)(2.0 * rho / delta), 0, h1, h2, s));
        rho_prev = rho;
    }
    return SEM_OK;
}

// Schwarz workspace for batches of nv vectors
static int ensure_schwarz_ws(sem_handle h, int nv)
{
    Workspace &w = h->ws;
    const int ns = h->n_levels - 1;  // smoothed levels
    int64_t ulen = 0;
    for (int l = 0; l < ns; ++l) {
        const int64_t ne = h->lv[l].nq + 2;
        ulen = std::max(ulen, h->lv[l].E * ne * ne * ne);
    }
    bool have = w.sz_U && w.sz_nv >= nv && w.sz_U_len >= ulen;
    for (int l = 0; l < ns; ++l) have = have && w.sz_acc[l] != nullptr;
    if (have) return SEM_OK;
    if (w.sz_U) (void)hipFree(w.sz_U);
    w.sz_U = nullptr;
    for (int l = 0; l < kMaxLevels; ++l) {
        if (w.sz_acc[l]) (void)hipFree(w.sz_acc[l]);
        w.sz_acc[l] = nullptr;
    }
    const int nvn = std::max(nv, w.sz_nv);
    ulen = std::max(ulen, w.sz_U_len);
    SEM_TRY(ws_alloc((void **)&w.sz_U, sizeof(float) * ulen * nvn));
    for (int l = 0; l < ns; ++l) SEM_TRY(ws_alloc((void **)&w.sz_acc[l], sizeof(float) * h->lv[l].nL * nvn));
    w.sz_U_len = ulen;
    w.sz_nv = nvn;
    return SEM_OK;
}

// host (W a, b) of FP32 vectors
static int host_dot32(const Level &L, const float *a, const float *b, double *partial, double *out,
                      hipStream_t s)
{
    const int nb = red_grid(L.nL);
    LAUNCH_V(dot32_kernel, L.nL, s, L.nL, L.W, a, b, partial);
    std::vector<double> hp(nb);
    SEM_HIP(hipMemcpyAsync(hp.data(), partial, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
    SEM_HIP(hipStreamSynchronize(s));
    *out = host_sum_partials(hp);
    return SEM_OK;
}

// lambda_max(M^{-1} A) of smoothed level l for the Schwarz smoother by the
// power method (W-norm ratio) in the smoother's FP32 arithmetic, started from
// the SplitMix64 values of the global pointers
static int schwarz_lmax(sem_handle h, int l, int smoother, double h1, double h2, int steps,
                        double *lmax, hipStream_t s)
{
    Level &L = h->lv[l];
    Workspace &w = h->ws;
    const int64_t n = L.nL;
    const VSet one = VSet::one();
    const bool ras = smoother == SEM_SMOOTH_RAS;
    float *v = (float *)w.mg_x[l], *t = (float *)w.mg_t[l], *z = (float *)w.mg_d[l];
    float *acc = w.sz_acc[l];
    LAUNCH_V(splitmix_kernel, n, s, n, L.gid, L.W, h->lanczos_seed, w.r);
    LAUNCH_B((convert_kernel<double, float>), n, one, s, n, one, (int64_t)0, (const double *)w.r,
             (int64_t)0, v);
    double nv2 = 0.0;
    SEM_TRY(host_dot32(L, v, v, w.partial, &nv2, s));
    if (!(nv2 > 0.0)) {
        *lmax = 1.0;
        return SEM_OK;
    }
    LAUNCH_V(wscale32_kernel, n, s, n, (const float *)nullptr, (const float *)v,
             (float)(1.0 / std::sqrt(nv2)), v);
    double lam = 1.0;
    for (int it = 0; it < steps; ++it) {
        SEM_TRY(apply_f32(L, one, v, t, h1, h2, s));
        SEM_TRY(launch_schwarz(L, ras, t, nullptr, w.sz_U, acc, one, h1, h2, s));
        SEM_TRY(launch_gs_multi<float>(L, acc, n, one, s, nullptr, 0));
        LAUNCH_V(wscale32_kernel, n, s, n, (const float *)(ras ? L.W32 : L.sz_w), (const float *)acc,
                 1.0f, z);
        double z2 = 0.0;
        SEM_TRY(host_dot32(L, z, z, w.partial, &z2, s));
        lam = std::sqrt(std::max(z2, 0.0));
        if (!(lam > 0.0)) break;
        LAUNCH_V(wscale32_kernel, n, s, n, (const float *)nullptr, (const float *)z, (float)(1.0 / lam), v);
    }
    *lmax = lam > 0.0 ? lam : 1.0;
    return SEM_OK;
}

struct SolveCfg {
    double h1, h2, tol, coarse_tol;
    int maxit, check_every, deg, coarse_maxit;
    int smoother;
};

// Vector arrays of one Krylov solve on a level: x may be the caller's array
// (leading dimension ldx); r, p, w are workspace arrays [nv][L.nL].
struct KrylovVecs {
    double *x;
    int64_t ldx;
    double *r, *p, *w;
    KrylovScalars *sc;
};

// Reduction buffers and inverse diagonal of a Jacobi-PCG: the handle's
// workspace and level data, or the allocation-free solve's static scratch.
struct PcgBufs {
    double *partial;
    int64_t pst;
    double *partial_ax;
    int64_t pst_ax;
    const double *Dinv;
};

static PcgBufs ws_bufs(sem_handle h, const Level &L)
{
    return PcgBufs{h->ws.partial, h->ws.pst, h->ws.partial_ax, h->ws.pst_ax, L.Dinv};
}

// enqueue Jacobi-PCG iterations first_iter .. first_iter+iters-1 (1-based)
// on level L for the batch vs: operator with fused (p, A_L p), QQ^T, update
// with alpha, and direction update with beta and the convergence decision --
// four kernels per iteration, no single-block reduction kernels
static int pcg_iterations(sem_handle h, const Level &L, const VSet &vs, const double *k, double h1,
                          double h2, const KrylovVecs &kv, const PcgBufs &pb, int first_iter,
                          int iters, hipStream_t s, bool timed = false)
{
    Workspace &ws = h->ws;
    const int64_t n = L.nL;
    const int nbv = red_grid(n);
    const int *skip = &kv.sc[0].done;
    for (int c = 0; c < iters; ++c) {
        const int it = first_iter + c;
        const int parity = (it - 1) & 1;
        int64_t nbax = 0;
        SEM_TRY(launch_ax_multi<double>(L, L.G, L.B, L.D, kv.p, n, kv.w, n, vs, h1, h2, k,
                                        pb.partial_ax, pb.pst_ax, &nbax, s, skip, kScStride));
        if (timed) SEM_TRY(clock_mark(ws, kPhaseAx, s));
        SEM_TRY(launch_gs_multi<double>(L, kv.w, n, vs, s, skip, kScStride));
        if (timed) SEM_TRY(clock_mark(ws, kPhaseGs, s));
        LAUNCH_B(pcg_update_fused_kernel, n, vs, s, n, vs, n, kv.ldx, kv.sc, parity,
                 (const double *)pb.partial_ax, pb.pst_ax, nbax, (const double *)kv.p,
                 (const double *)kv.w, pb.Dinv, L.W, kv.x, kv.r, pb.partial, pb.pst);
        LAUNCH_B(pcg_p_fused_kernel, n, vs, s, n, vs, n, kv.sc, parity, it,
                 (const double *)pb.partial, pb.pst, (int64_t)nbv, pb.Dinv, (const double *)kv.r,
                 kv.p);
        if (timed) SEM_TRY(clock_mark(ws, kPhaseVec, s));
    }
    return SEM_OK;
}

// start a Jacobi-PCG on level L for the batch vs: x given (Ax computed) or zero
static int pcg_start(const Level &L, const VSet &vs, const double *k, double h1, double h2,
                     const double *b, int64_t ldb, const KrylovVecs &kv, const PcgBufs &pb,
                     bool zero, double tol, int maxit, const BbRef &ref, hipStream_t s)
{
    const int64_t n = L.nL;
    const double *Ax = nullptr;
    if (zero) {
        LAUNCH_B(fill_kernel<double>, n, vs, s, n, vs, kv.ldx, kv.x, 0.0);
    } else {
        LAUNCH_B((mask_kernel<double, double>), n, vs, s, n, vs, kv.ldx, L.W, kv.x);
        SEM_TRY(launch_ax_multi<double>(L, L.G, L.B, L.D, kv.x, kv.ldx, kv.w, n, vs, h1, h2, k,
                                        nullptr, 0, nullptr, s, nullptr, 0));
        SEM_TRY(launch_gs_multi<double>(L, kv.w, n, vs, s, nullptr, 0));
        Ax = kv.w;
    }
    LAUNCH_B(pcg_init_kernel, n, vs, s, n, vs, ldb, b, n, Ax, pb.Dinv, L.W, kv.r, kv.p,
             (float *)nullptr, pb.partial, pb.pst, 1);
    LAUNCH_1B(fin_init_kernel, vs, s, vs, (const double *)pb.partial, pb.pst, (int64_t)red_grid(n),
              kv.sc, tol, maxit, ref);
    return SEM_OK;
}

// ------------------------------------------------- assembled coarse operator
// The coarsest level (N = 1 in the default schedule) is small: its operator is
// assembled once per (h1, h2) on the free unique nodes, and the coarse
// Jacobi-PCG runs on those nodes with a sparse product instead of the
// matrix-free operator and QQ^T on the element copies.  Mathematically the
// same iteration (the assembled matrix is Q^T A_L Q restricted to the free
// nodes, its diagonal the assembled diagonal); the vectors are 1/multiplicity
// the length, and one launch (the product) replaces two.

void free_coarse_csr(Level &L)
{
    void *ptrs[] = {L.cs_row, L.cs_col, L.cs_uid, L.cs_rep, L.cs_val, L.cs_dinv, L.cs_one, L.cs_bu, L.cs_xu};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    L.cs_row = L.cs_col = L.cs_uid = L.cs_rep = nullptr;
    L.cs_val = L.cs_dinv = L.cs_one = L.cs_bu = L.cs_xu = nullptr;
    L.cs_nf = L.cs_nnz = 0;
}

// u[i] = 1 at local point p of every element, 0 elsewhere
__global__ void unit_point_kernel(int64_t n, int np, int pt, double *__restrict__ u)
{
    GRID_LOOP(i, n) u[i] = (i % np == pt) ? 1.0 : 0.0;
}

// bu[i] = b[rep[i]] (b assembled: every copy of a node holds its value)
__global__ void csr_gather_kernel(int64_t nf, VSet vs, int64_t ldb, const int32_t *__restrict__ rep,
                                  const double *__restrict__ b, int64_t ldu, double *__restrict__ bu)
{
    const int64_t v = vsel(vs);
    b += v * ldb;
    bu += v * ldu;
    GRID_LOOP(i, nf) bu[i] = b[rep[i]];
}

// x[l] = xu[uid[l]] on free copies, 0 on Dirichlet copies
__global__ void csr_scatter_kernel(int64_t n, VSet vs, const int32_t *__restrict__ uid,
                                   const double *__restrict__ xu, int64_t ldu, double *__restrict__ x,
                                   int64_t ldx)
{
    const int64_t v = vsel(vs);
    xu += v * ldu;
    x += v * ldx;
    GRID_LOOP(l, n) {
        const int32_t i = uid[l];
        x[l] = i >= 0 ? xu[i] : 0.0;
    }
}

// y = A p on the free nodes and the partials of (p, y), kCsrLanes lanes per
// row (entries lane, lane + kCsrLanes, ... of the row, then a fixed butterfly
// over the lanes, whose first lane keeps the row's value), so every run adds
// in the same order.  Vectors flagged done are skipped.
constexpr int kCsrLanes = 8;

__global__ void csr_spmv_dot_kernel(int64_t nf, VSet vs, int64_t ld, const int32_t *__restrict__ row,
                                    const int32_t *__restrict__ col, const double *__restrict__ val,
                                    const double *__restrict__ p, double *__restrict__ y,
                                    double *__restrict__ partial, int64_t pst,
                                    const KrylovScalars *__restrict__ sc)
{
    const int64_t v = vsel(vs);
    if (sc[v].done) return;
    p += v * ld;
    y += v * ld;
    const int sub = threadIdx.x % kCsrLanes;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x / kCsrLanes;
    double s[1] = {0.0};
    for (int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kCsrLanes; r < nf; r += stride) {
        const int32_t a = row[r], b = row[r + 1];
        double acc = 0.0;
        for (int32_t k = a + sub; k < b; k += kCsrLanes) acc += val[k] * p[col[k]];
        acc += __shfl_xor(acc, 4, kCsrLanes);
        acc += __shfl_xor(acc, 2, kCsrLanes);
        acc += __shfl_xor(acc, 1, kCsrLanes);
        if (sub == 0) {
            y[r] = acc;
            s[0] += p[r] * acc;
        }
    }
    block_sum_store<1>(s, partial + v * pst);
}

// Assemble the coarsest level's operator h1 A + h2 B on its free unique
// nodes: the element matrices come from the level's own element operator
// applied to the unit vector of each local point (all elements at once),
// then the host adds them into rows by global pointer in element order.
static int build_coarse_csr(sem_handle h, double h1, double h2, hipStream_t s)
{
    Level &L = h->lv[h->n_levels - 1];
    free_coarse_csr(L);
    const int np = L.np;
    const int64_t E = L.E, n = L.nL;
    if ((int64_t)np * np * E > ((int64_t)1 << 31) - 1) {
        set_error("coarse operator: too many element-matrix entries (%lld)", (long long)((int64_t)np * np * E));
        return SEM_EINVAL;
    }
    std::vector<double> Ae((size_t)E * np * np), hw((size_t)n);
    double *u = nullptr, *wv = nullptr;
    int rc = SEM_OK;
    if (hipMalloc(&u, sizeof(double) * n) != hipSuccess || hipMalloc(&wv, sizeof(double) * n) != hipSuccess) {
        set_error("coarse operator: allocation failed");
        rc = SEM_ENOMEM;
    }
    for (int pt = 0; pt < np && rc == SEM_OK; ++pt) {
        hipLaunchKernelGGL(unit_point_kernel, dim3(red_grid(n)), dim3(kRB), 0, s, n, np, pt, u);
        if (hipGetLastError() != hipSuccess) rc = SEM_EHIP;
        if (rc == SEM_OK) rc = launch_ax<double>(L, L.G, L.B, L.D, u, wv, h1, h2, nullptr, nullptr, nullptr, s);
        if (rc == SEM_OK && (hipMemcpyAsync(hw.data(), wv, sizeof(double) * n, hipMemcpyDeviceToHost, s) != hipSuccess ||
                             hipStreamSynchronize(s) != hipSuccess))
            rc = SEM_EHIP;
        if (rc == SEM_OK)
            for (int64_t e = 0; e < E; ++e)
                for (int q = 0; q < np; ++q) Ae[((size_t)e * np + q) * np + pt] = hw[(size_t)e * np + q];
    }
    if (u) (void)hipFree(u);
    if (wv) (void)hipFree(wv);
    if (rc != SEM_OK) {
        if (rc == SEM_EHIP) set_error("coarse operator: %s", hipGetErrorString(hipGetLastError()));
        return rc;
    }
    // free unique nodes, numbered by first copy
    std::vector<int64_t> gid((size_t)n);
    std::vector<double> W((size_t)n);
    SEM_HIP(hipMemcpyAsync(gid.data(), L.gid, sizeof(int64_t) * n, hipMemcpyDeviceToHost, s));
    SEM_HIP(hipMemcpyAsync(W.data(), L.W, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    SEM_HIP(hipStreamSynchronize(s));
    std::vector<int64_t> order((size_t)n);
    for (int64_t l = 0; l < n; ++l) order[l] = l;
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return gid[a] < gid[b]; });
    std::vector<int32_t> uid((size_t)n, -1), rep;
    {
        // first copy of each pointer (pointer 0: every copy its own node)
        std::vector<int64_t> first((size_t)n, -1);
        for (int64_t i = 0; i < n;) {
            int64_t j = i;
            while (j < n && gid[order[j]] == gid[order[i]] && gid[order[i]] != 0) ++j;
            if (j == i) j = i + 1;
            for (int64_t k = i; k < j; ++k) first[order[k]] = order[i];
            i = j;
        }
        for (int64_t l = 0; l < n; ++l) {
            if (!(W[l] > 0.0)) continue;  // Dirichlet copy
            if (first[l] == l) {
                uid[l] = (int32_t)rep.size();
                rep.push_back((int32_t)l);
            }
        }
        for (int64_t l = 0; l < n; ++l)
            if (W[l] > 0.0) uid[l] = uid[first[l]];
    }
    const int64_t nf = (int64_t)rep.size();
    std::vector<int32_t> row, col;
    std::vector<double> val, dinv, one((size_t)nf, 1.0);
    const int64_t bad = assemble_free_csr(E, np, nf, uid.data(), Ae.data(), row, col, val, dinv);
    if (bad >= 0) {
        set_error("coarse operator: nonpositive diagonal at node %lld", (long long)bad);
        return SEM_EBREAKDOWN;
    }
    auto up = [&](void **dst, const void *src, size_t bytes) -> int {
        SEM_HIP(hipMalloc(dst, bytes > 0 ? bytes : 8));
        if (bytes && src) SEM_HIP(hipMemcpyAsync(*dst, src, bytes, hipMemcpyHostToDevice, s));
        return SEM_OK;
    };
    int r2 = SEM_OK;
    if (r2 == SEM_OK) r2 = up((void **)&L.cs_row, row.data(), sizeof(int32_t) * row.size());
    if (r2 == SEM_OK) r2 = up((void **)&L.cs_col, col.data(), sizeof(int32_t) * col.size());
    if (r2 == SEM_OK) r2 = up((void **)&L.cs_val, val.data(), sizeof(double) * val.size());
    if (r2 == SEM_OK) r2 = up((void **)&L.cs_dinv, dinv.data(), sizeof(double) * dinv.size());
    if (r2 == SEM_OK) r2 = up((void **)&L.cs_one, one.data(), sizeof(double) * one.size());
    if (r2 == SEM_OK) r2 = up((void **)&L.cs_uid, uid.data(), sizeof(int32_t) * uid.size());
    if (r2 == SEM_OK) r2 = up((void **)&L.cs_rep, rep.data(), sizeof(int32_t) * rep.size());
    if (r2 == SEM_OK) r2 = up((void **)&L.cs_bu, nullptr, sizeof(double) * nf * kMaxRhs);
    if (r2 == SEM_OK) r2 = up((void **)&L.cs_xu, nullptr, sizeof(double) * nf * kMaxRhs);
    if (r2 == SEM_OK && hipStreamSynchronize(s) != hipSuccess) r2 = SEM_EHIP;
    if (r2 != SEM_OK) {
        free_coarse_csr(L);
        return r2;
    }
    L.cs_nf = nf;
    L.cs_nnz = (int64_t)col.size();
    return SEM_OK;
}

// the coarse Jacobi-PCG on the assembled free-node system for the batch vs:
// b the assembled coarse right-hand sides (L-vectors, leading dimension n),
// the solutions scattered back into x (L-vectors, 0 on Dirichlet copies)
static int coarse_csr_solve(sem_handle h, const Level &L, const VSet &vs, const double *b, double *x,
                            const SolveCfg &cfg, hipStream_t s)
{
    Workspace &w = h->ws;
    const int64_t n = L.nL, nf = L.cs_nf;
    // the vectors are short: one entry per thread where the partial buffers
    // allow, so each kernel is a single round of memory accesses
    const int nbv = (int)std::max<int64_t>(1, std::min<int64_t>((nf + kRB - 1) / kRB, kMaxRedBlocks));
#define LAUNCH_NB(kern, ...)                                                                     \
    do {                                                                                         \
        hipLaunchKernelGGL(kern, dim3((unsigned)nbv, (unsigned)vs.n), dim3(kRB), 0, s, __VA_ARGS__); \
        SEM_HIP(hipGetLastError());                                                              \
    } while (0)
    LAUNCH_NB(csr_gather_kernel, nf, vs, n, (const int32_t *)L.cs_rep, b, nf, L.cs_bu);
    const KrylovVecs kv{L.cs_xu, nf, w.c_r, w.c_p, w.c_w, w.sc_c};
    LAUNCH_NB(fill_kernel<double>, nf, vs, nf, kv.x, 0.0);
    LAUNCH_NB(pcg_init_kernel, nf, vs, nf, (const double *)L.cs_bu, nf, (const double *)nullptr,
              (const double *)L.cs_dinv, (const double *)L.cs_one, kv.r, kv.p, (float *)nullptr, w.partial,
              w.pst, 1);
    LAUNCH_1B(fin_init_kernel, vs, s, vs, (const double *)w.partial, w.pst, (int64_t)nbv, kv.sc,
              cfg.coarse_tol, cfg.coarse_maxit, BbRef{});
    // one row per group of lanes where the partial buffers allow (a row's
    // loads are a dependent chain, so rows are not stacked on a thread)
    const int nbax = (int)std::max<int64_t>(
        1, std::min<int64_t>((nf * kCsrLanes + kRB - 1) / kRB, kMaxRedBlocks));
    for (int it = 1; it <= cfg.coarse_maxit; ++it) {
        const int parity = (it - 1) & 1;
        hipLaunchKernelGGL(csr_spmv_dot_kernel, dim3((unsigned)nbax, (unsigned)vs.n), dim3(kRB), 0, s, nf, vs,
                           nf, (const int32_t *)L.cs_row, (const int32_t *)L.cs_col, (const double *)L.cs_val,
                           (const double *)kv.p, kv.w, w.partial_ax, w.pst_ax, (const KrylovScalars *)kv.sc);
        SEM_HIP(hipGetLastError());
        LAUNCH_NB(pcg_update_fused_kernel, nf, vs, nf, kv.ldx, kv.sc, parity, (const double *)w.partial_ax,
                  w.pst_ax, (int64_t)nbax, (const double *)kv.p, (const double *)kv.w,
                  (const double *)L.cs_dinv, (const double *)L.cs_one, kv.x, kv.r, w.partial, w.pst);
        LAUNCH_NB(pcg_p_fused_kernel, nf, vs, nf, kv.sc, parity, it, (const double *)w.partial, w.pst,
                  (int64_t)nbv, (const double *)L.cs_dinv, (const double *)kv.r, kv.p);
    }
#undef LAUNCH_NB
    LAUNCH_B(csr_scatter_kernel, n, vs, s, n, vs, (const int32_t *)L.cs_uid, (const double *)L.cs_xu, nf, x, n);
    return SEM_OK;
}

// one V-cycle from level l for the batch vs: right-hand sides in mg_r[l]
// (FP32; FP64 on the coarsest), output in mg_x[l], arrays [nv][nL of level l]
static int vcycle(sem_handle h, int l, const VSet &vs, const SolveCfg &cfg, hipStream_t s)
{
    Workspace &w = h->ws;
    const int lc = h->n_levels - 1;
    const Level &L = h->lv[l];
    const int64_t n = L.nL;
    if (l == lc) {
        double *b = (double *)w.mg_r[l];
        SEM_TRY(clock_mark(w, kPhasePrec, s));
        if (L.cs_row) {
            SEM_TRY(coarse_csr_solve(h, L, vs, b, (double *)w.mg_x[l], cfg, s));
            SEM_TRY(clock_mark(w, kPhaseCoarse, s));
            return SEM_OK;
        }
        const KrylovVecs kv{(double *)w.mg_x[l], n, w.c_r, w.c_p, w.c_w, w.sc_c};
        const PcgBufs pb = ws_bufs(h, L);
        SEM_TRY(pcg_start(L, vs, nullptr, cfg.h1, cfg.h2, b, n, kv, pb, true, cfg.coarse_tol,
                          cfg.coarse_maxit, BbRef{}, s));
        SEM_TRY(pcg_iterations(h, L, vs, nullptr, cfg.h1, cfg.h2, kv, pb, 1, cfg.coarse_maxit, s));
        SEM_TRY(clock_mark(w, kPhaseCoarse, s));
        return SEM_OK;
    }
    float *r = (float *)w.mg_r[l], *x = (float *)w.mg_x[l], *t = (float *)w.mg_t[l],
          *sres = (float *)w.mg_s[l];
    const double lmax = cfg.smoother == SEM_SMOOTH_JACOBI ? L.lmax : L.sz_lmax;
    const double lmin_f = h->key.lo, lmax_f = h->key.hi;
    // pre-smoothing from x = 0
    SEM_TRY(chebyshev(L, l, h, vs, cfg.smoother, r, x, true, lmin_f * lmax, lmax_f * lmax, cfg.deg,
                      cfg.h1, cfg.h2, s));
    // restricted residual s = W (r - A x), coarse-grid correction x += J e_c
    SEM_TRY(apply_f32(L, vs, x, t, cfg.h1, cfg.h2, s));
    const Level &C = h->lv[l + 1];
    const int64_t nc = C.nL;
    const bool coarsest = l + 1 == lc;  // FP64 coarse solve below
    if (L.nq <= 8) {
        // fused transfers (residual and mask into the restriction, the
        // correction added inside the prolongation)
        if (coarsest) {
            double *bc = (double *)w.mg_r[l + 1];
            SEM_TRY(launch_restrict_resid<double>(L, C, r, t, bc, vs, s));
            SEM_TRY(launch_gs_multi<double>(C, bc, nc, vs, s, nullptr, 0));
        } else {
            float *rc = (float *)w.mg_r[l + 1];
            SEM_TRY(launch_restrict_resid<float>(L, C, r, t, rc, vs, s));
            SEM_TRY(launch_gs_multi<float>(C, rc, nc, vs, s, nullptr, 0));
        }
        SEM_TRY(vcycle(h, l + 1, vs, cfg, s));
        if (coarsest)
            SEM_TRY(launch_prolong_add<double>(L, C, (const double *)w.mg_x[l + 1], x, vs, s));
        else
            SEM_TRY(launch_prolong_add<float>(L, C, (const float *)w.mg_x[l + 1], x, vs, s));
    } else {
        LAUNCH_B(wresid_fused_kernel, n, vs, s, n, vs, n, L.W32, (const float *)r, (const float *)t,
                 sres);
        if (coarsest) {
            // restrict in FP32 into the head of t (n >= nc), then FP64 for the coarse solve
            double *bc = (double *)w.mg_r[l + 1];
            for (int q = 0; q < vs.n; ++q) {
                const int64_t v = vs.at(q);
                SEM_TRY(launch_interp<float>(L.E, L.nq, C.nq, L.Jc32, sres + v * n, t + v * n, true, s));
            }
            LAUNCH_B((convert_kernel<float, double>), nc, vs, s, nc, vs, n, (const float *)t, nc, bc);
            SEM_TRY(launch_gs_multi<double>(C, bc, nc, vs, s, nullptr, 0));
            LAUNCH_B((mask_kernel<double, double>), nc, vs, s, nc, vs, nc, C.W, bc);
            SEM_TRY(vcycle(h, l + 1, vs, cfg, s));
            LAUNCH_B((convert_kernel<double, float>), nc, vs, s, nc, vs, nc,
                     (const double *)w.mg_x[l + 1], n, t);
            // prolong: sres = J e_c (sres reused for the fine-sized interpolant)
            for (int q = 0; q < vs.n; ++q) {
                const int64_t v = vs.at(q);
                SEM_TRY(launch_interp<float>(L.E, C.nq, L.nq, L.Jc32, t + v * n, sres + v * n, false, s));
            }
        } else {
            float *rc = (float *)w.mg_r[l + 1];
            for (int q = 0; q < vs.n; ++q) {
                const int64_t v = vs.at(q);
                SEM_TRY(launch_interp<float>(L.E, L.nq, C.nq, L.Jc32, sres + v * n, rc + v * nc, true, s));
            }
            SEM_TRY(launch_gs_multi<float>(C, rc, nc, vs, s, nullptr, 0));
            LAUNCH_B((mask_kernel<float, float>), nc, vs, s, nc, vs, nc, C.W32, rc);
            SEM_TRY(vcycle(h, l + 1, vs, cfg, s));
            const float *xc = (const float *)w.mg_x[l + 1];
            for (int q = 0; q < vs.n; ++q) {
                const int64_t v = vs.at(q);
                SEM_TRY(launch_interp<float>(L.E, C.nq, L.nq, L.Jc32, xc + v * nc, sres + v * n, false, s));
            }
        }
        LAUNCH_B(add_kernel<float>, n, vs, s, n, vs, n, (const float *)sres, x);
    }
    // post-smoothing
    SEM_TRY(chebyshev(L, l, h, vs, cfg.smoother, r, x, false, lmin_f * lmax, lmax_f * lmax, cfg.deg,
                      cfg.h1, cfg.h2, s));
    return SEM_OK;
}

// FNV-1a hash of the bytes of the values added
struct Fnv {
    uint64_t h = 1469598103934665603ULL;
    template <typename T>
    void add(const T &v)
    {
        const unsigned char *p = reinterpret_cast<const unsigned char *>(&v);
        for (size_t i = 0; i < sizeof(T); ++i) {
            h ^= p[i];
            h *= 1099511628211ULL;
        }
    }
};

// every pointer and value the kernels of a V-cycle from level 0 take
static uint64_t vcycle_sig(sem_handle h, const VSet &vs, const SolveCfg &cfg)
{
    const Workspace &w = h->ws;
    Fnv f;
    f.add(vs.n);
    f.add(vs.pack);
    f.add(cfg.h1);
    f.add(cfg.h2);
    f.add(cfg.coarse_tol);
    f.add(cfg.coarse_maxit);
    f.add(cfg.deg);
    f.add(cfg.smoother);
    f.add(h->key.lo);
    f.add(h->key.hi);
    f.add(h->n_levels);
    const void *wp[] = {w.partial, w.partial_ax, w.sc, w.sc_c, w.c_r, w.c_p, w.c_w, w.sz_U};
    for (const void *p : wp) f.add(p);
    f.add(w.nv);
    f.add(w.pst);
    f.add(w.pst_ax);
    f.add(w.sz_U_len);
    for (int l = 0; l < h->n_levels; ++l) {
        const Level &L = h->lv[l];
        const void *lp[] = {w.mg_r[l], w.mg_x[l], w.mg_t[l], w.mg_d[l], w.mg_s[l], w.sz_acc[l],
                            L.G, L.B, L.G32, L.B32, L.D, L.D32, L.W, L.W32, L.Jc, L.Jc32, L.Dinv,
                            L.Dinv32, L.chunk_perm, L.over, L.perm, L.offs, L.sz_ix, L.sz_S, L.sz_lam,
                            L.sz_rc, L.sz_off, L.sz_src, L.sz_w, L.cs_row, L.cs_col, L.cs_val, L.cs_dinv,
                            L.cs_one, L.cs_uid, L.cs_rep, L.cs_bu, L.cs_xu};
        for (const void *p : lp) f.add(p);
        f.add(L.cs_nf);
        f.add(L.lmax);
        f.add(L.sz_lmax);
        f.add(L.nchunks);
        f.add(L.nover);
        f.add(L.sz_nrc);
        f.add(L.nL);
    }
    return f.h;
}

// one V-cycle from level 0 on `s`: replayed from the graph captured for this
// live set and state, captured first when there is none
static int vcycle_run(sem_handle h, const VSet &vs, const SolveCfg &cfg, bool graphs, hipStream_t s)
{
    Workspace &w = h->ws;
    if (!graphs || w.vg_broken) return vcycle(h, 0, vs, cfg, s);
    const uint64_t sig = vcycle_sig(h, vs, cfg);
    for (auto &g : w.vg)
        if (g.exec && g.sig == sig && g.n == vs.n && g.pack == vs.pack) {
            SEM_HIP(hipGraphLaunch(g.exec, s));
            return SEM_OK;
        }
    if (!w.cap) SEM_HIP(hipStreamCreateWithFlags(&w.cap, hipStreamNonBlocking));
    SEM_HIP(hipStreamBeginCapture(w.cap, hipStreamCaptureModeThreadLocal));
    const int rc = vcycle(h, 0, vs, cfg, w.cap);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(w.cap, &graph);
    hipGraphExec_t exec = nullptr;
    hipError_t ei = hipErrorUnknown;
    if (rc == SEM_OK && ec == hipSuccess && graph) ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) {
        (void)hipGetLastError();
        w.vg_broken = true;  // keep solving, kernel by kernel
        return vcycle(h, 0, vs, cfg, s);
    }
    auto &slot = w.vg[w.vg_next];
    w.vg_next = (w.vg_next + 1) % (int)(sizeof(w.vg) / sizeof(w.vg[0]));
    if (slot.exec) (void)hipGraphExecDestroy(slot.exec);
    slot.exec = exec;
    slot.sig = sig;
    slot.n = vs.n;
    slot.pack = vs.pack;
    SEM_HIP(hipGraphLaunch(exec, s));
    return SEM_OK;
}

// host copies of the outer (and coarse) scalars of every vector slot
static int read_scalars(sem_handle h, bool coarse, hipStream_t s)
{
    Workspace &w = h->ws;
    SEM_HIP(hipMemcpyAsync(w.host_sc, w.sc, kMaxRhs * sizeof(KrylovScalars), hipMemcpyDeviceToHost, s));
    if (coarse)
        SEM_HIP(hipMemcpyAsync(w.host_sc + kMaxRhs, w.sc_c, kMaxRhs * sizeof(KrylovScalars),
                               hipMemcpyDeviceToHost, s));
    SEM_HIP(hipStreamSynchronize(s));
    return SEM_OK;
}

// vectors of `all` whose solve is still running
static VSet live_set(const Workspace &w, const VSet &all)
{
    VSet act{0, 0u};
    for (int q = 0; q < all.n; ++q)
        if (!w.host_sc[all.at(q)].done) act.push(all.at(q));
    return act;
}

// true residuals ||b - A x||_W / ||b||_W in FP64 for the batch vs
static int true_residual(sem_handle h, const VSet &vs, const double *k, double h1, double h2,
                         const double *b, const double *x, int64_t ld, double *rel, hipStream_t s)
{
    const Level &F = h->lv[0];
    Workspace &w = h->ws;
    const int64_t n = F.nL;
    SEM_TRY(launch_ax_multi<double>(F, F.G, F.B, F.D, x, ld, w.w, n, vs, h1, h2, k, nullptr, 0,
                                    nullptr, s, nullptr, 0));
    SEM_TRY(launch_gs_multi<double>(F, w.w, n, vs, s, nullptr, 0));
    // pcg_init computes (W r r, W b b) for r = b - Ax
    LAUNCH_B(pcg_init_kernel, n, vs, s, n, vs, ld, b, n, (const double *)w.w, F.Dinv, F.W, w.z,
             (double *)nullptr, (float *)nullptr, w.partial, w.pst, 0);
    const int nb = red_grid(n);
    std::vector<double> hp((size_t)3 * nb * vs.n);
    for (int q = 0; q < vs.n; ++q)
        SEM_HIP(hipMemcpyAsync(hp.data() + (size_t)3 * nb * q, w.partial + vs.at(q) * w.pst,
                               sizeof(double) * 3 * nb, hipMemcpyDeviceToHost, s));
    SEM_HIP(hipStreamSynchronize(s));
    for (int q = 0; q < vs.n; ++q) {
        double rr = 0, bb = 0;
        const double *pq = hp.data() + (size_t)3 * nb * q;
        for (int i = 0; i < nb; ++i) {
            rr += pq[3 * i + 1];
            bb += pq[3 * i + 2];
        }
        rel[q] = bb > 0 ? std::sqrt(rr / bb) : 0.0;
    }
    return SEM_OK;
}

// (W a, y_q) for q < m, summed on the host in block order
static int host_wdots(const Level &L, const double *a, const double *Y, int64_t ldY, int m,
                      double *out, double *partial, hipStream_t s)
{
    const int nb = red_grid(L.nL);
    LAUNCH_V(wdots_kernel, L.nL, s, L.nL, L.W, a, Y, ldY, m, partial);
    std::vector<double> hp((size_t)nb * kMaxProj);
    SEM_HIP(hipMemcpyAsync(hp.data(), partial, sizeof(double) * hp.size(), hipMemcpyDeviceToHost, s));
    SEM_HIP(hipStreamSynchronize(s));
    for (int q = 0; q < m; ++q) {
        double acc = 0.0;
        for (int b = 0; b < nb; ++b) acc += hp[(size_t)b * kMaxProj + q];
        out[q] = acc;
    }
    return SEM_OK;
}

// projection spaces for slots 0 .. nv-1 with up to L vectors, for h1 A + h2 B
static int ensure_projection(sem_handle h, int nv, int L, double h1, double h2)
{
    Workspace &w = h->ws;
    const int64_t n = h->lv[0].nL;
    if (w.proj_L != L) {
        free_projection(w);
        w.proj_L = L;
    }
    if (w.proj_h1 != h1 || w.proj_h2 != h2) {
        for (int v = 0; v < kMaxRhs; ++v) w.proj[v].l = 0;
        w.proj_h1 = h1;
        w.proj_h2 = h2;
    }
    for (int v = 0; v < nv; ++v) {
        if (!w.proj[v].xt) SEM_TRY(ws_alloc((void **)&w.proj[v].xt, sizeof(double) * n * L));
        if (!w.proj[v].bt) SEM_TRY(ws_alloc((void **)&w.proj[v].bt, sizeof(double) * n * L));
    }
    if (w.proj_nv < nv) {
        if (w.proj_xb) (void)hipFree(w.proj_xb);
        if (w.proj_bp) (void)hipFree(w.proj_bp);
        w.proj_xb = w.proj_bp = nullptr;
        SEM_TRY(ws_alloc((void **)&w.proj_xb, sizeof(double) * n * nv));
        SEM_TRY(ws_alloc((void **)&w.proj_bp, sizeof(double) * n * nv));
        w.proj_nv = nv;
    }
    return SEM_OK;
}

// projected guess of slot v: xb = sum alpha_q xt_q, bp = b - sum alpha_q bt_q
// with alpha_q = (xt_q, b)_W; returns (b, b)_W and ||bp||_W / ||b||_W
static int proj_guess(sem_handle h, int v, const double *b, double *bb_out, double *rel_out,
                      hipStream_t s)
{
    Workspace &w = h->ws;
    const Level &F = h->lv[0];
    const int64_t n = F.nL;
    const Workspace::Proj &P = w.proj[v];
    double *xb = w.proj_xb + v * n, *bp = w.proj_bp + v * n;
    double bb = 0.0, pp = 0.0;
    SEM_TRY(host_dot(F, b, b, w.partial, &bb, s));
    if (P.l > 0) {
        double al[kMaxProj];
        SEM_TRY(host_wdots(F, b, P.xt, n, P.l, al, w.partial, s));
        Coefs ca{}, cb{};
        for (int q = 0; q < P.l; ++q) {
            ca.c[q] = al[q];
            cb.c[q] = -al[q];
        }
        LAUNCH_V(lincomb_kernel, n, s, n, (const double *)nullptr, 0.0, (const double *)P.xt, n, P.l,
                 ca, xb);
        LAUNCH_V(lincomb_kernel, n, s, n, b, 1.0, (const double *)P.bt, n, P.l, cb, bp);
    } else {
        LAUNCH_V(lincomb3_kernel, n, s, n, b, 0.0, (const double *)nullptr, 0.0,
                 (const double *)nullptr, 0.0, xb);
        LAUNCH_V(lincomb3_kernel, n, s, n, b, 1.0, (const double *)nullptr, 0.0,
                 (const double *)nullptr, 0.0, bp);
    }
    SEM_TRY(host_dot(F, bp, bp, w.partial, &pp, s));
    *bb_out = bb;
    *rel_out = bb > 0.0 ? std::sqrt(std::max(pp, 0.0) / bb) : 0.0;
    return SEM_OK;
}

// after the solve of slot v: x holds dx (solution of A dx = bp); grow the
// space by dx (A-orthogonalised, A-normalised) or restart it from the final
// x, and complete x = xb + dx
static int proj_update(sem_handle h, int v, const double *b, double *x, double h1, double h2,
                       hipStream_t s)
{
    Workspace &w = h->ws;
    const Level &F = h->lv[0];
    const int64_t n = F.nL;
    const VSet one = VSet::one();
    Workspace::Proj &P = w.proj[v];
    const double *xb = w.proj_xb + v * n, *bp = w.proj_bp + v * n;
    double *aw = w.w;  // A dx
    SEM_TRY(launch_ax<double>(F, F.G, F.B, F.D, x, aw, h1, h2, nullptr, nullptr, nullptr, s));
    SEM_TRY(launch_gs<double>(F, aw, s));
    LAUNCH_B((mask_kernel<double, double>), n, one, s, n, one, (int64_t)0, F.W, aw);
    if (P.l < w.proj_L) {
        double gam[kMaxProj] = {};
        if (P.l > 0) SEM_TRY(host_wdots(F, aw, P.xt, n, P.l, gam, w.partial, s));
        Coefs cg{};
        for (int q = 0; q < P.l; ++q) cg.c[q] = -gam[q];
        double *xn = P.xt + P.l * n, *bn = P.bt + P.l * n;
        LAUNCH_V(lincomb_kernel, n, s, n, (const double *)x, 1.0, (const double *)P.xt, n, P.l, cg, xn);
        LAUNCH_V(lincomb_kernel, n, s, n, (const double *)aw, 1.0, (const double *)P.bt, n, P.l, cg, bn);
        double nu2 = 0.0, dxw = 0.0;
        SEM_TRY(host_dot(F, xn, bn, w.partial, &nu2, s));
        SEM_TRY(host_dot(F, x, aw, w.partial, &dxw, s));
        if (nu2 > 1e-28 * std::max(dxw, 1e-300)) {
            const double inv = 1.0 / std::sqrt(nu2);
            LAUNCH_V(lincomb3_kernel, n, s, n, (const double *)xn, inv, (const double *)nullptr, 0.0,
                     (const double *)nullptr, 0.0, xn);
            LAUNCH_V(lincomb3_kernel, n, s, n, (const double *)bn, inv, (const double *)nullptr, 0.0,
                     (const double *)nullptr, 0.0, bn);
            P.l += 1;
        }
        LAUNCH_V(lincomb3_kernel, n, s, n, (const double *)x, 1.0, xb, 1.0, (const double *)nullptr,
                 0.0, x);
    } else {
        LAUNCH_V(lincomb3_kernel, n, s, n, (const double *)x, 1.0, xb, 1.0, (const double *)nullptr,
                 0.0, x);
        // A x = A xb + A dx = (b - bp) + A dx
        double *x0 = P.xt, *b0 = P.bt;
        LAUNCH_V(lincomb3_kernel, n, s, n, b, 1.0, bp, -1.0, (const double *)aw, 1.0, b0);
        double nu2 = 0.0;
        SEM_TRY(host_dot(F, x, b0, w.partial, &nu2, s));
        if (nu2 > 0.0) {
            const double inv = 1.0 / std::sqrt(nu2);
            LAUNCH_V(lincomb3_kernel, n, s, n, (const double *)x, inv, (const double *)nullptr, 0.0,
                     (const double *)nullptr, 0.0, x0);
            LAUNCH_V(lincomb3_kernel, n, s, n, (const double *)b0, inv, (const double *)nullptr, 0.0,
                     (const double *)nullptr, 0.0, b0);
            P.l = 1;
        } else {
            P.l = 0;
        }
    }
    return SEM_OK;
}

// nv solves with one operator, in lockstep: vector v's right-hand side and
// iterate are b + v*ld and x + v*ld; every kernel serves the unconverged ones
// Preconditioner data for opts on the handle's levels (inverse diagonals,
// the Chebyshev interval's lambda_max per smoothed level, the Schwarz data
// when a Schwarz smoother is asked for), cached for constant coefficients.
static int prepare_precond(sem_handle h, const sem_solve_opts *o, const SolveCfg &cfg, bool pmg, int nv,
                           hipStream_t s)
{
    PrecondKey key;
    key.valid = true;
    key.h1 = o->h1;
    key.h2 = o->h2;
    key.precond = o->precond;
    key.smoother = cfg.smoother;
    key.cheb_degree = pmg ? cfg.deg : 0;
    key.lanczos_steps = pmg ? o->lanczos_steps : 0;
    key.lo = pmg ? o->cheb_lo : 0;
    key.hi = pmg ? o->cheb_hi : 0;
    const PrecondKey &old = h->key;
    const bool same = !o->k && old.valid && old.h1 == key.h1 && old.h2 == key.h2 &&
                      (old.precond == key.precond || !pmg) && old.lanczos_steps >= key.lanczos_steps &&
                      (!pmg || (old.precond == SEM_PRECOND_PMG && old.lanczos_steps == key.lanczos_steps &&
                                old.smoother == key.smoother));
    if (cfg.smoother != SEM_SMOOTH_JACOBI) {
        for (int l = 0; l + 1 < h->n_levels; ++l) SEM_TRY(build_schwarz(h->lv[l], s));
        SEM_TRY(ensure_schwarz_ws(h, nv));
    }
    if (!same) {
        h->key.valid = false;
        SEM_TRY(compute_dinv(h, 0, o->k, o->h1, o->h2, pmg, s));
        if (pmg) {
            for (int l = 1; l < h->n_levels; ++l)
                SEM_TRY(compute_dinv(h, l, nullptr, o->h1, o->h2, l < h->n_levels - 1, s));
            SEM_TRY(build_coarse_csr(h, o->h1, o->h2, s));
            for (int l = 0; l + 1 < h->n_levels; ++l) {
                if (cfg.smoother == SEM_SMOOTH_JACOBI)
                    SEM_TRY(lanczos_lmax(h, l, o->h1, o->h2, std::max(2, o->lanczos_steps), &h->lv[l].lmax, s));
                else
                    SEM_TRY(schwarz_lmax(h, l, cfg.smoother, o->h1, o->h2, std::max(2, o->lanczos_steps),
                                         &h->lv[l].sz_lmax, s));
            }
        }
        if (!o->k) h->key = key;
    }
    h->key.lo = key.lo;
    h->key.hi = key.hi;
    h->key.cheb_degree = key.cheb_degree;
    return SEM_OK;
}

int pcg_solve(sem_handle h, int nv, const double *b, double *x, int64_t ld, const sem_solve_opts *o,
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
    const bool proj = o->proj_dim > 0;
    if (proj && o->k) {
        set_error("sem_pcg_solve: projected initial guesses need constant coefficients (k = NULL)");
        return SEM_EINVAL;
    }
    SolveCfg cfg{o->h1, o->h2, o->tol, o->coarse_tol, o->maxit, std::max(1, o->check_every),
                 std::max(1, o->cheb_degree), std::max(1, o->coarse_maxit),
                 pmg ? o->smoother : SEM_SMOOTH_JACOBI};
    const auto t0 = clk::now();
    SEM_TRY(ensure_workspace(h, pmg, nv));
    Workspace &w = h->ws;
    const Level &F = h->lv[0];
    const int64_t n = F.nL;
    SEM_TRY(prepare_precond(h, o, cfg, pmg, nv, s));
    SEM_HIP(hipStreamSynchronize(s));
    const auto t1 = clk::now();

    const VSet all = VSet::first(nv);
    const KrylovVecs kv{x, ld, w.r, w.p, w.w, w.sc};
    std::vector<int> coarse_total(nv, 0);
    // projected initial guesses: solve for the remainder dx (into x) of each
    // right-hand side, from zero, to the tolerance of the original b
    std::vector<int> proj_used(nv, 0);
    std::vector<double> proj_rel(nv, 0.0);
    BbRef ref{};
    const double *bs = b;  // right-hand sides the Krylov solve sees
    int64_t ldbs = ld;
    if (proj) {
        SEM_TRY(ensure_projection(h, nv, o->proj_dim, o->h1, o->h2));
        for (int v = 0; v < nv; ++v) {
            proj_used[v] = w.proj[v].l;
            double bb = 0.0;
            SEM_TRY(proj_guess(h, v, b + v * ld, &bb, &proj_rel[v], s));
            ref.v[v] = bb;
        }
        bs = w.proj_bp;
        ldbs = n;
    }
    const bool zero = proj || o->zero_guess != 0;
    // phase timers: a new event chain after every host synchronisation
    SEM_TRY(clock_begin(w, o->timers != 0));
    auto sync_point = [&](bool coarse) -> int {
        SEM_TRY(read_scalars(h, coarse, s));
        SEM_TRY(clock_flush(w, false));
        return clock_mark(w, -1, s);
    };
    SEM_TRY(clock_mark(w, -1, s));
    if (!pmg) {
        SEM_TRY(pcg_start(F, all, o->k, o->h1, o->h2, bs, ldbs, kv, ws_bufs(h, F), zero, o->tol,
                          o->maxit, ref, s));
        SEM_TRY(clock_mark(w, kPhaseVec, s));
        SEM_TRY(sync_point(false));
        VSet act = live_set(w, all);
        int it = 0;
        while (act.n > 0) {
            SEM_TRY(pcg_iterations(h, F, act, o->k, o->h1, o->h2, kv, ws_bufs(h, F), it + 1,
                                   cfg.check_every, s, true));
            it += cfg.check_every;
            SEM_TRY(sync_point(false));
            act = live_set(w, act);
        }
    } else {
        // r = b - A x ; z = M r ; p = z ; rz = (z, r)
        const double *Ax = nullptr;
        if (zero) {
            LAUNCH_B(fill_kernel<double>, n, all, s, n, all, ld, x, 0.0);
        } else {
            LAUNCH_B((mask_kernel<double, double>), n, all, s, n, all, ld, F.W, x);
            SEM_TRY(launch_ax_multi<double>(F, F.G, F.B, F.D, x, ld, w.w, n, all, o->h1, o->h2,
                                            nullptr, nullptr, 0, nullptr, s, nullptr, 0));
            SEM_TRY(launch_gs_multi<double>(F, w.w, n, all, s, nullptr, 0));
            Ax = w.w;
        }
        float *r32 = (float *)w.mg_r[0], *z32 = (float *)w.mg_x[0];  // V-cycle input, output
        LAUNCH_B(pcg_init_kernel, n, all, s, n, all, ldbs, bs, n, Ax, F.Dinv, F.W, w.r,
                 (double *)nullptr, r32, w.partial, w.pst, 0);
        LAUNCH_1B(fin_init_kernel, all, s, all, (const double *)w.partial, w.pst,
                  (int64_t)red_grid(n), w.sc, o->tol, o->maxit, ref);
        SEM_TRY(clock_mark(w, kPhaseVec, s));
        SEM_TRY(sync_point(false));
        VSet act = live_set(w, all);
        const int nbv = red_grid(n);
        const int *skip = &w.sc[0].done;
        const bool vec = vec_ok(n, ld, {x}) && vec_ok(n, n, {w.r, w.p, w.w, r32, z32, F.W, F.W32});
        VSet cycled{0, 0u};  // vectors whose coarse counts are still to be read
        if (act.n > 0) {
            SEM_TRY(vcycle_run(h, act, cfg, o->use_graphs != 0, s));
            SEM_TRY(clock_mark(w, kPhasePrec, s));
            LAUNCH_B(dot_zw_kernel, n, act, s, n, act, n, (const KrylovScalars *)w.sc, F.W,
                     (const float *)z32, (const double *)w.r, (const double *)w.r, w.partial,
                     w.pst);
            LAUNCH_B_VEC(vec, fcg_p_fused_kernel, n, act, s, n, act, n, w.sc, 1,
                        (const double *)w.partial, w.pst, (int64_t)nbv, (const float *)z32, F.W32,
                        w.p, 1);
            SEM_TRY(clock_mark(w, kPhaseVec, s));
            cycled = act;
        }
        for (int it = 0; act.n > 0; ++it) {
            const int parity = it & 1;
            int64_t nbax = 0;
            SEM_TRY(launch_ax_multi<double>(F, F.G, F.B, F.D, w.p, n, w.w, n, act, o->h1, o->h2,
                                            nullptr, w.partial_ax, w.pst_ax, &nbax, s, skip,
                                            kScStride));
            SEM_TRY(clock_mark(w, kPhaseAx, s));
            SEM_TRY(launch_gs_multi<double>(F, w.w, n, act, s, skip, kScStride));
            SEM_TRY(clock_mark(w, kPhaseGs, s));
            LAUNCH_B_VEC(vec, fcg_update_fused_kernel, n, act, s, n, act, n, ld, w.sc, parity,
                        (const double *)w.partial_ax, w.pst_ax, nbax, (const double *)w.p,
                        (const double *)w.w, F.W, x, w.r, r32, w.partial, w.pst);
            LAUNCH_1B(fin_conv_kernel, act, s, act, (const double *)w.partial, w.pst, (int64_t)nbv,
                      w.sc);
            SEM_TRY(clock_mark(w, kPhaseVec, s));
            // one host synchronisation per iteration: outer scalars, and the
            // coarse-solve counts of the V-cycle that preceded this update
            SEM_TRY(sync_point(cycled.n > 0));
            for (int q = 0; q < cycled.n; ++q)
                coarse_total[cycled.at(q)] += w.host_sc[kMaxRhs + cycled.at(q)].iters;
            cycled = VSet{0, 0u};
            act = live_set(w, act);
            if (act.n == 0) break;
            SEM_TRY(vcycle_run(h, act, cfg, o->use_graphs != 0, s));
            SEM_TRY(clock_mark(w, kPhasePrec, s));
            LAUNCH_B(dot_zw_kernel, n, act, s, n, act, n, (const KrylovScalars *)w.sc, F.W,
                     (const float *)z32, (const double *)w.w, (const double *)w.r, w.partial,
                     w.pst);
            LAUNCH_B_VEC(vec, fcg_p_fused_kernel, n, act, s, n, act, n, w.sc, parity,
                        (const double *)w.partial, w.pst, (int64_t)nbv, (const float *)z32, F.W32,
                        w.p, 0);
            SEM_TRY(clock_mark(w, kPhaseVec, s));
            cycled = act;
        }
    }
    SEM_TRY(clock_flush(w, true));
    const bool timed = w.clk.on;
    double phase_ms[kPhases];
    std::copy(w.clk.ms, w.clk.ms + kPhases, phase_ms);
    w.clk.on = false;
    std::vector<KrylovScalars> hs(w.host_sc, w.host_sc + nv);
    if (proj)
        for (int v = 0; v < nv; ++v) SEM_TRY(proj_update(h, v, b + v * ld, x + v * ld, o->h1, o->h2, s));
    SEM_HIP(hipStreamSynchronize(s));
    const auto t2 = clk::now();
    std::vector<double> trr(nv, 0.0);
    SEM_TRY(true_residual(h, all, o->k, o->h1, o->h2, b, x, ld, trr.data(), s));
    int rc = SEM_OK;
    for (int v = 0; v < nv; ++v) {
        const KrylovScalars &q = hs[v];
        const bool conv = q.status == SEM_OK && (q.bb == 0.0 || q.rr <= q.tol2);
        if (st) {
            st[v].iters = q.iters;
            st[v].rel_res = q.bb > 0 ? std::sqrt(std::max(q.rr, 0.0) / q.bb) : 0.0;
            st[v].converged = conv ? 1 : 0;
            st[v].true_rel_res = trr[v];
            st[v].ms_setup = std::chrono::duration<double, std::milli>(t1 - t0).count();
            st[v].ms_solve = std::chrono::duration<double, std::milli>(t2 - t1).count();
            st[v].coarse_iters = coarse_total[v];
            st[v].proj_vectors = proj_used[v];
            st[v].proj_rel_res = proj_rel[v];
            st[v].ms_ax = timed ? phase_ms[kPhaseAx] : 0.0;
            st[v].ms_gs = timed ? phase_ms[kPhaseGs] : 0.0;
            st[v].ms_vec = timed ? phase_ms[kPhaseVec] : 0.0;
            st[v].ms_prec = timed ? phase_ms[kPhasePrec] : 0.0;
            st[v].ms_coarse = timed ? phase_ms[kPhaseCoarse] : 0.0;
        }
        if (q.status == SEM_EBREAKDOWN) {
            if (rc != SEM_EBREAKDOWN)
                set_error("sem_pcg_solve: breakdown of system %d after %d iterations", v, q.iters);
            rc = SEM_EBREAKDOWN;
        } else if (!conv && rc == SEM_OK) {
            set_error("sem_pcg_solve: system %d not converged after %d iterations (rel res %.3e)", v,
                      q.iters, q.bb > 0 ? std::sqrt(q.rr / q.bb) : 0.0);
            rc = SEM_ENOCONV;
        }
    }
    return rc;
}

// One application of the p-multigrid preconditioner, z = M^{-1} r: the
// V-cycle the flexible CG applies to its residual, on an FP64 vector.
int pmg_apply(sem_handle h, const double *r, double *z, const sem_solve_opts *o, hipStream_t s)
{
    if (h->n_levels < 2) {
        set_error("sem_pmg_apply: the handle has no multigrid levels");
        return SEM_EINVAL;
    }
    if (o->k) {
        set_error("sem_pmg_apply: PMG supports constant coefficients only (k = NULL)");
        return SEM_EINVAL;
    }
    sem_solve_opts oo = *o;
    oo.precond = SEM_PRECOND_PMG;
    SolveCfg cfg{oo.h1, oo.h2, oo.tol, oo.coarse_tol, oo.maxit, std::max(1, oo.check_every),
                 std::max(1, oo.cheb_degree), std::max(1, oo.coarse_maxit), oo.smoother};
    SEM_TRY(ensure_workspace(h, true, 1));
    SEM_TRY(prepare_precond(h, &oo, cfg, true, 1, s));
    Workspace &w = h->ws;
    const Level &F = h->lv[0];
    const int64_t n = F.nL;
    const VSet one = VSet::one();
    float *r32 = (float *)w.mg_r[0], *z32 = (float *)w.mg_x[0];  // V-cycle input, output
    LAUNCH_B((convert_kernel<double, float>), n, one, s, n, one, n, r, n, r32);
    LAUNCH_B((mask_kernel<float, float>), n, one, s, n, one, n, F.W32, r32);
    SEM_TRY(vcycle_run(h, one, cfg, oo.use_graphs != 0, s));
    LAUNCH_B((convert_kernel<float, double>), n, one, s, n, one, n, (const float *)z32, n, z);
    LAUNCH_B((mask_kernel<double, float>), n, one, s, n, one, n, F.W32, z);
    return SEM_OK;
}

// b = R QQ^T (B o f)
int assemble_load(sem_handle h, const double *f, double *b, hipStream_t s)
{
    const Level &F = h->lv[0];
    const int64_t n = F.nL;
    const VSet one = VSet::one();
    LAUNCH_V(mass_kernel, n, s, n, F.B, f, b);
    SEM_TRY(launch_gs<double>(F, b, s));
    LAUNCH_B((mask_kernel<double, double>), n, one, s, n, one, (int64_t)0, F.W, b);
    return SEM_OK;
}

int adjoint(sem_handle h, const double *u, const double *g, const sem_solve_opts *o, double *lam,
            double *grad_f, double *grad_k, sem_solve_stats *st, hipStream_t s)
{
    const Level &F = h->lv[0];
    const int64_t n = F.nL;
    SEM_TRY(ensure_workspace(h, false, 1));
    if (!h->ws.aux) SEM_TRY(ws_alloc((void **)&h->ws.aux, sizeof(double) * n));
    // right-hand side R QQ^T g in a workspace vector the solver does not touch
    double *rhs = h->ws.aux;
    SEM_HIP(hipMemcpyAsync(rhs, g, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    SEM_TRY(launch_gs<double>(F, rhs, s));
    const VSet one = VSet::one();
    LAUNCH_B((mask_kernel<double, double>), n, one, s, n, one, (int64_t)0, F.W, rhs);
    sem_solve_opts oo = *o;
    oo.zero_guess = 1;
    oo.proj_dim = 0;  // the forward solves' spaces stay untouched
    if (oo.k != nullptr || h->n_levels < 2) oo.precond = SEM_PRECOND_JACOBI;
    const int rc = pcg_solve(h, 1, rhs, lam, n, &oo, st, s);
    if (rc != SEM_OK && rc != SEM_ENOCONV) return rc;
    if (grad_f) LAUNCH_V(mass_kernel, n, s, n, F.B, lam, grad_f);
    if (grad_k) SEM_TRY(launch_grad_k(F, u, lam, o->h1, grad_k, s));
    SEM_HIP(hipStreamSynchronize(s));
    return rc;
}


// ------------------------------------------------ allocation-free Jacobi-PCG
// Device scratch of sem_pcg_solve_noalloc: the Krylov scalars, the reduction
// partials, the inverse diagonal Dinv and the vectors r, p, w of one FP64
// Jacobi-PCG.  One copy per GPU, held from the library's first use on that
// GPU until the process ends; every call on a GPU shares it (and finds the
// last call's contents), so calls that overlap on one GPU race.
constexpr size_t kNoAllocBytes = (size_t)SEM_NOALLOC_SCRATCH_MIB << 20;
constexpr size_t kNoAllocHead = 256;                             // KrylovScalars
constexpr int64_t kNoAllocPst = 3 * kMaxRedBlocks;               // vector-kernel partials
constexpr int64_t kNoAllocPstAx = 8192;                          // operator partials
constexpr size_t kNoAllocVecOff =
    kNoAllocHead + sizeof(double) * (size_t)(kNoAllocPst + kNoAllocPstAx);
static_assert(sizeof(KrylovScalars) <= kNoAllocHead, "scalar record");
static_assert(kNoAllocVecOff % 256 == 0, "vector alignment");
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

// the device address of `scratch` on each GPU (the array's name in host code
// is a host-side stand-in, not a device address)
constexpr int kNoAllocMaxDevices = 64;
static std::mutex g_scratch_mu;
static unsigned char *g_scratch[kNoAllocMaxDevices] = {};

// largest level-0 L-vector the scratch holds: four vectors (Dinv, r, p, w) of
// a multiple of 32 doubles, so each starts 256-byte aligned
constexpr int64_t kNoAllocMaxLocal =
    (int64_t)((kNoAllocBytes - kNoAllocVecOff) / (4 * sizeof(double))) & ~(int64_t)31;
static_assert(kNoAllocMaxLocal == SEM_NOALLOC_MAX_LOCAL, "limit stated in sem.h");

// Look up the scratch address on device `dev` (current) once; called by
// sem_setup for the handle's device.
int noalloc_attach(int dev)
{
    if (dev < 0 || dev >= kNoAllocMaxDevices) {
        set_error("setup: device %d beyond the %d devices the allocation-free solve supports", dev,
                  kNoAllocMaxDevices);
        return SEM_EINVAL;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[dev]) return SEM_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        set_error("setup: address of the allocation-free solve's scratch: %s", hipGetErrorString(e));
        return SEM_EHIP;
    }
    g_scratch[dev] = (unsigned char *)p;
    return SEM_OK;
}

// host copy of the scalar record, the stream synchronised
static int read_one_scalar(const KrylovScalars *sc, KrylovScalars *out, hipStream_t s)
{
    SEM_HIP(hipMemcpyAsync(out, sc, sizeof(KrylovScalars), hipMemcpyDeviceToHost, s));
    SEM_HIP(hipStreamSynchronize(s));
    return SEM_OK;
}

// The Jacobi-PCG of pcg_solve for one right-hand side, every buffer beyond
// b and x in the device scratch: the same kernels in the same order, so the
// iterates equal those of sem_pcg_solve with the Jacobi preconditioner.
static int pcg_solve_noalloc(sem_handle h, const double *b, double *x, const sem_solve_opts *o,
                             sem_solve_stats *st, hipStream_t s)
{
    using clk = std::chrono::steady_clock;
    const Level &F = h->lv[0];
    const int64_t n = F.nL;
    unsigned char *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (h->device >= 0 && h->device < kNoAllocMaxDevices) base = g_scratch[h->device];
    }
    if (!base) {
        set_error("sem_pcg_solve_noalloc: no scratch address for device %d", h->device);
        return SEM_EHIP;
    }
    const int64_t pst_ax = (int64_t)(F.n_cu > 0 ? F.n_cu : 256) * kAxMaxBlocksPerCU + 64;
    if (pst_ax > kNoAllocPstAx) {
        set_error("sem_pcg_solve_noalloc: %d compute units exceed the scratch's operator partials",
                  F.n_cu);
        return SEM_EINVAL;
    }
    const size_t vb = ((size_t)n * sizeof(double) + 255) & ~(size_t)255;
    KrylovScalars *sc = (KrylovScalars *)base;
    double *partial = (double *)(base + kNoAllocHead);
    double *partial_ax = partial + kNoAllocPst;
    double *Dinv = (double *)(base + kNoAllocVecOff);
    double *r = (double *)(base + kNoAllocVecOff + vb);
    double *p = (double *)(base + kNoAllocVecOff + 2 * vb);
    double *w = (double *)(base + kNoAllocVecOff + 3 * vb);
    const VSet one = VSet::one();
    const auto t0 = clk::now();
    // Dinv of h1 A(k) + h2 B: assembled diagonal (in r), inverted on free copies
    SEM_TRY(launch_diag<double>(F, o->k, o->h1, o->h2, r, s));
    SEM_TRY(launch_gs<double>(F, r, s));
    LAUNCH_V(invert_diag_kernel, n, s, n, F.W, (const double *)r, Dinv, (float *)nullptr);
    SEM_HIP(hipStreamSynchronize(s));
    const auto t1 = clk::now();
    const KrylovVecs kv{x, n, r, p, w, sc};
    const PcgBufs pb{partial, kNoAllocPst, partial_ax, pst_ax, Dinv};
    const int check = std::max(1, o->check_every);
    SEM_TRY(pcg_start(F, one, o->k, o->h1, o->h2, b, n, kv, pb, o->zero_guess != 0, o->tol, o->maxit,
                      BbRef{}, s));
    KrylovScalars hs{};
    SEM_TRY(read_one_scalar(sc, &hs, s));
    for (int it = 0; !hs.done; it += check) {
        SEM_TRY(pcg_iterations(h, F, one, o->k, o->h1, o->h2, kv, pb, it + 1, check, s));
        SEM_TRY(read_one_scalar(sc, &hs, s));
    }
    const auto t2 = clk::now();
    // true residual b - QQ^T A_L x (into w, then r), (W r r, W b b) summed on
    // the host in block order
    SEM_TRY(launch_ax_multi<double>(F, F.G, F.B, F.D, x, n, w, n, one, o->h1, o->h2, o->k, nullptr, 0,
                                    nullptr, s, nullptr, 0));
    SEM_TRY(launch_gs_multi<double>(F, w, n, one, s, nullptr, 0));
    LAUNCH_B(pcg_init_kernel, n, one, s, n, one, n, b, n, (const double *)w, (const double *)Dinv,
             F.W, r, (double *)nullptr, (float *)nullptr, partial, kNoAllocPst, 0);
    const int nb = red_grid(n);
    double hp[3 * kMaxRedBlocks];
    SEM_HIP(hipMemcpyAsync(hp, partial, sizeof(double) * 3 * nb, hipMemcpyDeviceToHost, s));
    SEM_HIP(hipStreamSynchronize(s));
    double rr = 0.0, bb = 0.0;
    for (int i = 0; i < nb; ++i) {
        rr += hp[3 * i + 1];
        bb += hp[3 * i + 2];
    }
    const bool conv = hs.status == SEM_OK && (hs.bb == 0.0 || hs.rr <= hs.tol2);
    if (st) {
        *st = sem_solve_stats{};
        st->iters = hs.iters;
        st->rel_res = hs.bb > 0 ? std::sqrt(std::max(hs.rr, 0.0) / hs.bb) : 0.0;
        st->converged = conv ? 1 : 0;
        st->true_rel_res = bb > 0 ? std::sqrt(rr / bb) : 0.0;
        st->ms_setup = std::chrono::duration<double, std::milli>(t1 - t0).count();
        st->ms_solve = std::chrono::duration<double, std::milli>(t2 - t1).count();
    }
    if (hs.status == SEM_EBREAKDOWN) {
        set_error("sem_pcg_solve_noalloc: breakdown after %d iterations", hs.iters);
        return SEM_EBREAKDOWN;
    }
    if (!conv) {
        set_error("sem_pcg_solve_noalloc: not converged after %d iterations (rel res %.3e)", hs.iters,
                  hs.bb > 0 ? std::sqrt(hs.rr / hs.bb) : 0.0);
        return SEM_ENOCONV;
    }
    return SEM_OK;
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
    o->proj_dim = 0;
    o->smoother = SEM_SMOOTH_JACOBI;
    o->use_graphs = 0;
    o->timers = 0;
}

int sem_smoother_apply(sem_handle h, int level, int smoother, double h1, double h2, const float *r,
                       float *z, void *stream)
{
    if (!h || !r || !z) {
        set_error("sem_smoother_apply: null argument");
        return SEM_EINVAL;
    }
    if (level < 0 || level >= h->n_levels) {
        set_error("sem_smoother_apply: level %d not in handle (%d levels)", level, h->n_levels);
        return SEM_EINVAL;
    }
    if (smoother != SEM_SMOOTH_ASM && smoother != SEM_SMOOTH_RAS) {
        set_error("sem_smoother_apply: smoother must be SEM_SMOOTH_ASM or SEM_SMOOTH_RAS");
        return SEM_EINVAL;
    }
    const hipStream_t s = (hipStream_t)stream;
    Level &L = h->lv[level];
    if (!L.W32) {
        set_error("sem_smoother_apply: level %d has no FP32 data", level);
        return SEM_EINVAL;
    }
    SEM_TRY(build_schwarz(L, s));
    SEM_TRY(ensure_workspace(h, false, 1));
    // this level's buffers (the handle's smoothed levels may not include it)
    Workspace &w = h->ws;
    const int64_t ne = L.nq + 2, ulen = L.E * ne * ne * ne;
    if (!w.sz_U || w.sz_U_len < ulen) {
        // one vector's worth for this level; the solver's batch buffers are
        // sized again by ensure_schwarz_ws when a solve needs them
        if (w.sz_U) (void)hipFree(w.sz_U);
        w.sz_U = nullptr;
        const int nvn = std::max(1, w.sz_nv);
        const int64_t len = std::max<int64_t>(ulen, w.sz_U_len);
        SEM_TRY(ws_alloc((void **)&w.sz_U, sizeof(float) * len * nvn));
        w.sz_U_len = len;
        w.sz_nv = nvn;
    }
    const VSet one = VSet::one();
    const bool ras = smoother == SEM_SMOOTH_RAS;
    SEM_TRY(launch_schwarz(L, ras, r, nullptr, w.sz_U, z, one, h1, h2, s));
    SEM_TRY(launch_gs_multi<float>(L, z, L.nL, one, s, nullptr, 0));
    LAUNCH_V(wscale32_kernel, L.nL, s, L.nL, (const float *)(ras ? L.W32 : L.sz_w), (const float *)z,
             1.0f, z);
    return SEM_OK;
}

int sem_proj_reset(sem_handle h)
{
    if (!h) {
        set_error("sem_proj_reset: null handle");
        return SEM_EINVAL;
    }
    for (int v = 0; v < kMaxRhs; ++v) h->ws.proj[v].l = 0;
    return SEM_OK;
}

static int check_solve_opts(const char *who, const sem_solve_opts *o)
{
    if (!(o->tol >= 0.0) || o->maxit < 0 || (o->precond != SEM_PRECOND_JACOBI && o->precond != SEM_PRECOND_PMG)) {
        set_error("%s: bad options", who);
        return SEM_EINVAL;
    }
    if (o->smoother != SEM_SMOOTH_JACOBI && o->smoother != SEM_SMOOTH_ASM && o->smoother != SEM_SMOOTH_RAS) {
        set_error("%s: bad smoother %d", who, o->smoother);
        return SEM_EINVAL;
    }
    if (o->proj_dim < 0 || o->proj_dim > kMaxProj) {
        set_error("%s: proj_dim = %d outside 0..%d", who, o->proj_dim, kMaxProj);
        return SEM_EINVAL;
    }
    if (o->precond == SEM_PRECOND_PMG &&
        (!(o->cheb_hi > o->cheb_lo) || !(o->cheb_lo > 0.0) || o->lanczos_steps < 2)) {
        set_error("%s: bad Chebyshev options", who);
        return SEM_EINVAL;
    }
    return SEM_OK;
}

int sem_pcg_solve(sem_handle h, const double *b, double *x, const sem_solve_opts *o,
                  sem_solve_stats *st, void *stream)
{
    if (!h || !b || !x || !o) {
        set_error("sem_pcg_solve: null argument");
        return SEM_EINVAL;
    }
    SEM_TRY(check_solve_opts("sem_pcg_solve", o));
    return pcg_solve(h, 1, b, x, h->lv[0].nL, o, st, (hipStream_t)stream);
}

int sem_pmg_apply(sem_handle h, const double *r, double *z, const sem_solve_opts *o, void *stream)
{
    if (!h || !r || !z || !o) {
        set_error("sem_pmg_apply: null argument");
        return SEM_EINVAL;
    }
    SEM_TRY(check_solve_opts("sem_pmg_apply", o));
    return pmg_apply(h, r, z, o, (hipStream_t)stream);
}

int sem_pcg_solve_multi(sem_handle h, int nrhs, const double *b, double *x, int64_t ld,
                        const sem_solve_opts *o, sem_solve_stats *st, void *stream)
{
    if (!h || !b || !x || !o) {
        set_error("sem_pcg_solve_multi: null argument");
        return SEM_EINVAL;
    }
    if (nrhs < 1 || nrhs > kMaxRhs) {
        set_error("sem_pcg_solve_multi: nrhs = %d outside 1..%d", nrhs, kMaxRhs);
        return SEM_EINVAL;
    }
    if (ld < h->lv[0].nL) {
        set_error("sem_pcg_solve_multi: ld = %lld below n_local = %lld", (long long)ld,
                  (long long)h->lv[0].nL);
        return SEM_EINVAL;
    }
    SEM_TRY(check_solve_opts("sem_pcg_solve_multi", o));
    return pcg_solve(h, nrhs, b, x, ld, o, st, (hipStream_t)stream);
}

int sem_pcg_solve_noalloc(sem_handle h, const double *b, double *x, const sem_solve_opts *o,
                          sem_solve_stats *st, void *stream)
{
    if (!h || !b || !x || !o) {
        set_error("sem_pcg_solve_noalloc: null argument");
        return SEM_EINVAL;
    }
    SEM_TRY(check_solve_opts("sem_pcg_solve_noalloc", o));
    if (o->precond != SEM_PRECOND_JACOBI || o->proj_dim != 0 || o->timers != 0 || o->use_graphs != 0) {
        set_error("sem_pcg_solve_noalloc: Jacobi preconditioner only, without projection, timers or graphs");
        return SEM_EINVAL;
    }
    if (h->lv[0].nL > kNoAllocMaxLocal) {
        set_error("sem_pcg_solve_noalloc: %lld local points exceed the limit of %lld (%d MiB scratch)",
                  (long long)h->lv[0].nL, (long long)kNoAllocMaxLocal, SEM_NOALLOC_SCRATCH_MIB);
        return SEM_EINVAL;
    }
    int dev = -1;
    SEM_HIP(hipGetDevice(&dev));
    if (dev != h->device) {
        set_error("sem_pcg_solve_noalloc: current device %d is not the handle's device %d", dev, h->device);
        return SEM_EINVAL;
    }
    return pcg_solve_noalloc(h, b, x, o, st, (hipStream_t)stream);
}

}  // extern "C"
