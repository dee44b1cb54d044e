// Gather-scatter, geometry, operator diagonal, dL/dk and transfer kernels.
#include "sem_internal.h"

namespace semx {

// ---------------------------------------------------------------------------
// QQ^T (Sec. 2.3 eq. (dssum); gs_op(+) of Sec. 3.2) as a segmented reduction
// over the sorted maps.  The shared copies (perm, canonical order) are packed
// into chunks of whole segments of at most 64 copies; one 64-lane wavefront
// takes one chunk: lane l loads copy l (one coalesced load of the chunk's
// padded copy list, one gathered value), then sums the lanes of its segment in ascending order by cross-lane
// reads and writes the total back.  Each sum starts from 0 and adds the
// copies in ascending local index order, so the result is bit-identical to a
// sequential pass.  Unshared copies are never touched.  Segments with more
// than 64 copies (not in conforming hex meshes of moderate valence) go to a
// one-thread-per-segment pass.
// ---------------------------------------------------------------------------

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2;
// give XCD x the x-th contiguous range of workgroups so that neighbouring
// segments (which share cache lines of the L-vector) meet in one L2.
__device__ inline int64_t xcd_chunk_block(int64_t b, int64_t nb)
{
    const int64_t x = b % 8, q = b / 8;
    const int64_t per = nb / 8, rem = nb % 8;
    return x * per + (x < rem ? x : rem) + q;
}

constexpr int kGsWavesPerBlock = 4;

// The reduction of a segment (gs_op of Sec. 3.2): the sum (the direct-
// stiffness summation QQ^T, started from 0 as the plain definition is), or
// the product, minimum or maximum of the copies started from the first copy;
// every form combines the copies in ascending local index order.
template <int OP, typename T>
__device__ __forceinline__ T gs_combine(T a, T b)
{
    if constexpr (OP == SEM_GS_MUL) return a * b;
    else if constexpr (OP == SEM_GS_MIN) return fmin(a, b);
    else if constexpr (OP == SEM_GS_MAX) return fmax(a, b);
    else return a + b;
}

// One map load per lane ahead of the values: the chunk's copy list padded to
// 64 lanes (cperm[c][lane]: the copy, with kGsSegStart set where it starts a
// segment, or -1 past the chunk's end), so the gathers depend on a single
// coalesced load; the chunk size and the segment starts follow by ballots.
// The copy indices are applied to every vector of the batch in turn.
template <typename T, int OP = SEM_GS_ADD>
__global__ void __launch_bounds__(64 * kGsWavesPerBlock)
gs_chunk_kernel(int64_t nchunks, const int32_t *__restrict__ cperm, T *__restrict__ v, int64_t ld,
                VSet vs, const int *__restrict__ skip, int skip_stride)
{
    uint32_t pack;
    const int na = live_vectors(vs, skip, skip_stride, &pack);
    if (na == 0) return;
    const int lane = threadIdx.x & 63;
    const int64_t c = xcd_chunk_block(blockIdx.x, gridDim.x) * kGsWavesPerBlock + (threadIdx.x >> 6);
    if (c >= nchunks) return;  // uniform per wavefront
    const int ent = cperm[c * 64 + lane];
    const bool act = ent >= 0;
    const int idx = act ? (ent & (kGsSegStart - 1)) : 0;
    // the gathers of every live vector are issued before the first sum so
    // their latencies overlap; each vector's sum is the same as alone
    T val[kMaxRhs];
#pragma unroll
    for (int q = 0; q < kMaxRhs; ++q)
        val[q] = (q < na && act) ? v[(int64_t)((pack >> (8 * q)) & 255u) * ld + idx] : T(0);
    const uint64_t m = __ballot(act && (ent & kGsSegStart));  // bit l: lane l starts a segment
    const int cnt = __popcll(__ballot(act));  // the chunk's copies are lanes 0 .. cnt-1
    const uint64_t upto = (lane == 63) ? ~0ULL : ((2ULL << lane) - 1ULL);
    const int s0 = 63 - __clzll((long long)(m & upto));      // first lane of my segment
    const uint64_t above = m & ~upto;
    const int e0 = above ? (__ffsll((long long)above) - 1) : cnt;  // one past its last lane
    const int len = act ? e0 - s0 : 0;
    int maxlen = len;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) maxlen = max(maxlen, __shfl_xor(maxlen, o));
#pragma unroll
    for (int q = 0; q < kMaxRhs; ++q) {
        if (q >= na) break;
        constexpr int j0 = OP == SEM_GS_ADD ? 0 : 1;
        T acc = OP == SEM_GS_ADD ? T(0) : __shfl(val[q], s0);
        for (int j = j0; j < maxlen; ++j) {  // wave-uniform trip count
            const T other = __shfl(val[q], min(s0 + j, 63));
            if (j < len) acc = gs_combine<OP>(acc, other);
        }
        if (act) v[(int64_t)((pack >> (8 * q)) & 255u) * ld + idx] = acc;
    }
}

// segments listed in `segs`, one thread each (copies in canonical order)
template <typename T, int OP = SEM_GS_ADD>
__global__ void gs_segment_kernel(int64_t nseg, const int32_t *__restrict__ segs,
                                  const int32_t *__restrict__ perm,
                                  const int32_t *__restrict__ offs, T *__restrict__ v, int64_t ld,
                                  VSet vs, const int *__restrict__ skip, int skip_stride)
{
    uint32_t pack;
    const int na = live_vectors(vs, skip, skip_stride, &pack);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (na == 0 || t >= nseg) return;
    const int sidx = segs[t];
    const int a = offs[sidx], b = offs[sidx + 1];
    for (int q = 0; q < na; ++q) {
        T *vq = v + (int64_t)((pack >> (8 * q)) & 255u) * ld;
        T acc = OP == SEM_GS_ADD ? T(0) : vq[perm[a]];
        for (int o = OP == SEM_GS_ADD ? a : a + 1; o < b; ++o) acc = gs_combine<OP>(acc, vq[perm[o]]);
        for (int o = a; o < b; ++o) vq[perm[o]] = acc;
    }
}

template <typename T>
int launch_gs_multi(const Level &L, T *v, int64_t ld, const VSet &vs, hipStream_t s,
                    const int *skip, int skip_stride)
{
    if (vs.n <= 0) return SEM_OK;
    if (L.nchunks > 0) {
        const int64_t nb = (L.nchunks + kGsWavesPerBlock - 1) / kGsWavesPerBlock;
        hipLaunchKernelGGL(gs_chunk_kernel<T>, dim3((unsigned)nb), dim3(64 * kGsWavesPerBlock), 0, s,
                           L.nchunks, L.chunk_perm, v, ld, vs, skip, skip_stride);
        SEM_HIP(hipGetLastError());
    }
    if (L.nover > 0) {
        const int bs = 256;
        const int64_t nb = (L.nover + bs - 1) / bs;
        hipLaunchKernelGGL(gs_segment_kernel<T>, dim3((unsigned)nb), dim3(bs), 0, s, L.nover, L.over,
                           L.perm, L.offs, v, ld, vs, skip, skip_stride);
        SEM_HIP(hipGetLastError());
    }
    return SEM_OK;
}

template <typename T>
int launch_gs(const Level &L, T *v, hipStream_t s, const int *skip)
{
    return launch_gs_multi<T>(L, v, 0, VSet::one(), s, skip, 0);
}

// one field with any gs_op reduction (the solver paths use the sum only)
template <typename T, int OP>
static int launch_gs_one_op(const Level &L, T *v, hipStream_t s)
{
    const VSet vs = VSet::one();
    if (L.nchunks > 0) {
        const int64_t nb = (L.nchunks + kGsWavesPerBlock - 1) / kGsWavesPerBlock;
        hipLaunchKernelGGL((gs_chunk_kernel<T, OP>), dim3((unsigned)nb), dim3(64 * kGsWavesPerBlock), 0, s,
                           L.nchunks, L.chunk_perm, v, (int64_t)0, vs, (const int *)nullptr, 0);
        SEM_HIP(hipGetLastError());
    }
    if (L.nover > 0) {
        const int bs = 256;
        const int64_t nb = (L.nover + bs - 1) / bs;
        hipLaunchKernelGGL((gs_segment_kernel<T, OP>), dim3((unsigned)nb), dim3(bs), 0, s, L.nover, L.over,
                           L.perm, L.offs, v, (int64_t)0, vs, (const int *)nullptr, 0);
        SEM_HIP(hipGetLastError());
    }
    return SEM_OK;
}

template <typename T>
int launch_gs_op(const Level &L, T *v, int op, hipStream_t s)
{
    switch (op) {
    case SEM_GS_ADD: return launch_gs<T>(L, v, s, nullptr);
    case SEM_GS_MUL: return launch_gs_one_op<T, SEM_GS_MUL>(L, v, s);
    case SEM_GS_MIN: return launch_gs_one_op<T, SEM_GS_MIN>(L, v, s);
    case SEM_GS_MAX: return launch_gs_one_op<T, SEM_GS_MAX>(L, v, s);
    default: set_error("gather-scatter: unknown operation %d", op); return SEM_EINVAL;
    }
}
template int launch_gs_op<double>(const Level &, double *, int, hipStream_t);
template int launch_gs<double>(const Level &, double *, hipStream_t, const int *);
template int launch_gs<float>(const Level &, float *, hipStream_t, const int *);
template int launch_gs_multi<double>(const Level &, double *, int64_t, const VSet &, hipStream_t,
                                     const int *, int);
template int launch_gs_multi<float>(const Level &, float *, int64_t, const VSet &, hipStream_t,
                                    const int *, int);

// ---------------------------------------------------------------------------
// Geometric factors (Sec. 2.3 eqs. (grad), (vBu), (gij)): one block per
// element, one thread per point.  dx_p/dr_q = D_q x_p; J = det; dr/dx from the
// adjugate; B = rho_i rho_j rho_k J; G_mm' = (sum_l dr_m/dx_l dr_m'/dx_l) B.
// G is written point-interleaved [E][np][6].  bad is set when J <= 0.
// ---------------------------------------------------------------------------
__global__ void geometry_kernel(int64_t E, int nq, const double *__restrict__ x,
                                const double *__restrict__ y, const double *__restrict__ z,
                                const double *__restrict__ D, const double *__restrict__ rho,
                                double *__restrict__ G, double *__restrict__ B, int *bad)
{
    const int64_t e = blockIdx.x;
    const int np = nq * nq * nq;
    for (int p = threadIdx.x; p < np; p += blockDim.x) {
        const int i = p % nq, j = (p / nq) % nq, k = p / (nq * nq);
        const double *xs[3] = {x + e * np, y + e * np, z + e * np};
        double M[3][3];  // M[a][q] = d x_a / d r_q
        for (int a = 0; a < 3; ++a) {
            double dr = 0, ds = 0, dt = 0;
            for (int l = 0; l < nq; ++l) {
                dr += D[i * nq + l] * xs[a][l + nq * (j + nq * k)];
                ds += D[j * nq + l] * xs[a][i + nq * (l + nq * k)];
                dt += D[k * nq + l] * xs[a][i + nq * (j + nq * l)];
            }
            M[a][0] = dr;
            M[a][1] = ds;
            M[a][2] = dt;
        }
        // adjugate: C[q][a] = cofactor of M[a][q]; (dr/dx)[q][a] = C[q][a] / J
        double C[3][3];
        C[0][0] = M[1][1] * M[2][2] - M[1][2] * M[2][1];
        C[0][1] = M[0][2] * M[2][1] - M[0][1] * M[2][2];
        C[0][2] = M[0][1] * M[1][2] - M[0][2] * M[1][1];
        C[1][0] = M[1][2] * M[2][0] - M[1][0] * M[2][2];
        C[1][1] = M[0][0] * M[2][2] - M[0][2] * M[2][0];
        C[1][2] = M[0][2] * M[1][0] - M[0][0] * M[1][2];
        C[2][0] = M[1][0] * M[2][1] - M[1][1] * M[2][0];
        C[2][1] = M[0][1] * M[2][0] - M[0][0] * M[2][1];
        C[2][2] = M[0][0] * M[1][1] - M[0][1] * M[1][0];
        const double J = M[0][0] * C[0][0] + M[0][1] * C[1][0] + M[0][2] * C[2][0];
        if (!(J > 0.0)) atomicOr(bad, 1);
        const double w = rho[i] * rho[j] * rho[k] * J;
        B[e * np + p] = w;
        // G_mm' = sum_a (C[m][a]/J)(C[m'][a]/J) rho J = sum_a C[m][a] C[m'][a] rho / J
        const double sc = rho[i] * rho[j] * rho[k] / J;
        double *Ge = G + (e * np + p) * 6;
        int slot = 0;
        for (int m = 0; m < 3; ++m)
            for (int mp = m; mp < 3; ++mp) {
                const double g = C[m][0] * C[mp][0] + C[m][1] * C[mp][1] + C[m][2] * C[mp][2];
                Ge[slot] = g * sc;
                ++slot;
            }
    }
}

int launch_geometry(const Level &L, const double *x, const double *y, const double *z, double *G,
                    double *B, int *bad, hipStream_t s)
{
    // rho lives right after D in the level's D buffer (see setup)
    const double *rho = L.D + L.nq * L.nq;
    const int bs = L.np >= 256 ? 256 : ((L.np + 63) / 64) * 64;
    hipLaunchKernelGGL(geometry_kernel, dim3((unsigned)L.E), dim3(bs), 0, s, L.E, L.nq, x, y, z,
                       L.D, rho, G, B, bad);
    SEM_HIP(hipGetLastError());
    return SEM_OK;
}

// ---------------------------------------------------------------------------
// Diagonal of the unassembled h1 A^e(k) + h2 B^e: for m = m' the sum of
// Dh[l][i]^2 G_mm over the line, for m != m' only the point itself couples
// (D_m and D_m' share a nonzero only on the diagonal).
// ---------------------------------------------------------------------------
__global__ void diag_kernel(int64_t nL, int nq, const double *__restrict__ G,
                            const double *__restrict__ B, const double *__restrict__ kc,
                            const double *__restrict__ D, double h1, double h2,
                            double *__restrict__ d)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nL) return;
    const int np = nq * nq * nq;
    const int64_t e = q / np;
    const int p = (int)(q - e * np);
    const int i = p % nq, j = (p / nq) % nq, k = p / (nq * nq);
    const double *Ge = G + e * np * 6;  // [np][6]
    const double *ke = kc ? kc + e * np : nullptr;
    double s = 0.0;
    for (int l = 0; l < nq; ++l) {
        const int pi = l + nq * (j + nq * k), pj = i + nq * (l + nq * k), pk = i + nq * (j + nq * l);
        s += D[l * nq + i] * D[l * nq + i] * Ge[pi * 6 + 0] * (ke ? ke[pi] : 1.0);
        s += D[l * nq + j] * D[l * nq + j] * Ge[pj * 6 + 3] * (ke ? ke[pj] : 1.0);
        s += D[l * nq + k] * D[l * nq + k] * Ge[pk * 6 + 5] * (ke ? ke[pk] : 1.0);
    }
    const double c = ke ? ke[p] : 1.0;
    const double di = D[i * nq + i], dj = D[j * nq + j], dk = D[k * nq + k];
    s += 2.0 * c * (di * dj * Ge[p * 6 + 1] + di * dk * Ge[p * 6 + 2] + dj * dk * Ge[p * 6 + 4]);
    double v = h1 * s;
    if (h2 != 0.0) v += h2 * B[q];
    d[q] = v;
}

template <typename T>
int launch_diag(const Level &L, const double *k, double h1, double h2, double *d, hipStream_t s)
{
    const int bs = 256;
    const int64_t nb = (L.nL + bs - 1) / bs;
    hipLaunchKernelGGL(diag_kernel, dim3((unsigned)nb), dim3(bs), 0, s, L.nL, L.nq, L.G, L.B, k,
                       L.D, h1, h2, d);
    SEM_HIP(hipGetLastError());
    return SEM_OK;
}
template int launch_diag<double>(const Level &, const double *, double, double, double *,
                                 hipStream_t);

// ---------------------------------------------------------------------------
// dL/dk per copy: -h1 (D lam)^T G (D u), reference-space gradients of both
// fields at the point (eqs. (gradr)-(gradt)) contracted with G.
// ---------------------------------------------------------------------------
__global__ void grad_k_kernel(int64_t nL, int nq, const double *__restrict__ G,
                              const double *__restrict__ D, const double *__restrict__ u,
                              const double *__restrict__ lam, double h1, double *__restrict__ gk)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nL) return;
    const int np = nq * nq * nq;
    const int64_t e = q / np;
    const int p = (int)(q - e * np);
    const int i = p % nq, j = (p / nq) % nq, k = p / (nq * nq);
    const double *ue = u + e * np, *le = lam + e * np;
    double a0 = 0, a1 = 0, a2 = 0, c0 = 0, c1 = 0, c2 = 0;
    for (int l = 0; l < nq; ++l) {
        const int pi = l + nq * (j + nq * k), pj = i + nq * (l + nq * k), pk = i + nq * (j + nq * l);
        a0 += D[i * nq + l] * le[pi];
        a1 += D[j * nq + l] * le[pj];
        a2 += D[k * nq + l] * le[pk];
        c0 += D[i * nq + l] * ue[pi];
        c1 += D[j * nq + l] * ue[pj];
        c2 += D[k * nq + l] * ue[pk];
    }
    const double *Ge = G + (e * np + p) * 6;
    const double g11 = Ge[0], g12 = Ge[1], g13 = Ge[2], g22 = Ge[3], g23 = Ge[4], g33 = Ge[5];
    const double s = a0 * (g11 * c0 + g12 * c1 + g13 * c2) + a1 * (g12 * c0 + g22 * c1 + g23 * c2)
                   + a2 * (g13 * c0 + g23 * c1 + g33 * c2);
    gk[q] = -h1 * s;
}

// The same pointwise product for elements that fit one wavefront (nq <= 8),
// in the element operator's layout: thread (i, j) holds the k-lines of u and
// lam in registers (t-derivatives there, D entries wave-uniform), the r- and
// s-derivatives read LDS rows; every element's u, lam, G and gk move once
// (72 B per point), coalesced.  The sums run in the same order as above.
template <int NQ>
__global__ void __launch_bounds__(64)
grad_k_elem_kernel(int64_t E, const double *__restrict__ G, const double *__restrict__ D,
                   const double *__restrict__ u, const double *__restrict__ lam, double h1,
                   double *__restrict__ gk)
{
    constexpr int TPE = NQ * NQ, EPB = 64 / TPE, NP = NQ * NQ * NQ, LD = (NQ % 2 == 0) ? NQ + 1 : NQ;
    __shared__ double su[EPB][NQ][NQ][LD];
    __shared__ double sl[EPB][NQ][NQ][LD];
    const int tid = threadIdx.x;
    const int el = tid / TPE, ij = tid - el * TPE;
    const int i = ij % NQ, j = ij / NQ;
    const int64_t e = (int64_t)blockIdx.x * EPB + el;
    const bool act = el < EPB && e < E;
    double ru[NQ], rl[NQ], Di[NQ], Dj[NQ];
#pragma unroll
    for (int l = 0; l < NQ; ++l) {
        Di[l] = D[i * NQ + l];
        Dj[l] = D[j * NQ + l];
    }
    const int64_t base = (act ? e : 0) * NP + ij;
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
        ru[k] = act ? u[base + k * TPE] : 0.0;
        rl[k] = act ? lam[base + k * TPE] : 0.0;
        if (el < EPB) {
            su[el][k][j][i] = ru[k];
            sl[el][k][j][i] = rl[k];
        }
    }
    // one wavefront: order the LDS writes before the reads
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (!act) return;
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
        double a0 = 0, a1 = 0, a2 = 0, c0 = 0, c1 = 0, c2 = 0;
#pragma unroll
        for (int l = 0; l < NQ; ++l) {
            const double dk = D[k * NQ + l];
            a0 += Di[l] * sl[el][k][j][l];
            a1 += Dj[l] * sl[el][k][l][i];
            a2 += dk * rl[l];
            c0 += Di[l] * su[el][k][j][l];
            c1 += Dj[l] * su[el][k][l][i];
            c2 += dk * ru[l];
        }
        const double2 *g2 = reinterpret_cast<const double2 *>(G + (base + k * TPE) * 6);
        const double2 ga = g2[0], gb = g2[1], gc = g2[2];
        const double g11 = ga.x, g12 = ga.y, g13 = gb.x, g22 = gb.y, g23 = gc.x, g33 = gc.y;
        const double sum = a0 * (g11 * c0 + g12 * c1 + g13 * c2) + a1 * (g12 * c0 + g22 * c1 + g23 * c2)
                         + a2 * (g13 * c0 + g23 * c1 + g33 * c2);
        gk[base + k * TPE] = -h1 * sum;
    }
}

int launch_grad_k(const Level &L, const double *u, const double *lam, double h1, double *gk,
                  hipStream_t s)
{
#define SEM_GK(NQ)                                                                          \
    case NQ: {                                                                              \
        constexpr int EPB = 64 / (NQ * NQ);                                                 \
        const int64_t nb = (L.E + EPB - 1) / EPB;                                           \
        hipLaunchKernelGGL(grad_k_elem_kernel<NQ>, dim3((unsigned)nb), dim3(64), 0, s, L.E, L.G, \
                           L.D, u, lam, h1, gk);                                            \
        SEM_HIP(hipGetLastError());                                                         \
        return SEM_OK;                                                                      \
    }
    switch (L.nq) {
        SEM_GK(2) SEM_GK(3) SEM_GK(4) SEM_GK(5) SEM_GK(6) SEM_GK(7) SEM_GK(8)
    default: break;
    }
#undef SEM_GK
    const int bs = 256;
    const int64_t nb = (L.nL + bs - 1) / bs;
    hipLaunchKernelGGL(grad_k_kernel, dim3((unsigned)nb), dim3(bs), 0, s, L.nL, L.nq, L.G, L.D, u,
                       lam, h1, gk);
    SEM_HIP(hipGetLastError());
    return SEM_OK;
}

// ---------------------------------------------------------------------------
// Elementwise tensor-product interpolation between orders, sum-factorised in
// three LDS passes: out = (J (x) J (x) J) in with J [nt][ns] (transpose=false),
// or out = (J^T (x) J^T (x) J^T) in with J [ns][nt] stored as [nt_in][ns_out]
// (transpose=true, the restriction).  One block per element.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void interp_kernel(int64_t E, int ns, int nt, const T *__restrict__ J, bool transpose,
                              const T *__restrict__ in, T *__restrict__ out)
{
    extern __shared__ unsigned char smem_raw[];
    T *sin = reinterpret_cast<T *>(smem_raw);            // ns^3
    T *t1 = sin + ns * ns * ns;                          // ns*ns*nt  [c][b][i]
    T *t2 = t1 + ns * ns * nt;                           // ns*nt*nt  [c][j][i]
    __shared__ T sJ[16 * 16];
    const int64_t e = blockIdx.x;
    const int tid = threadIdx.x, nth = blockDim.x;
    // matrix A [nt][ns]: A[a][b] = J[a][b] or J[b][a] (J given as [ns][nt] then)
    for (int t = tid; t < nt * ns; t += nth) {
        const int a = t / ns, b = t % ns;
        sJ[t] = transpose ? J[b * nt + a] : J[a * ns + b];
    }
    const int pin = ns * ns * ns, pout = nt * nt * nt;
    for (int t = tid; t < pin; t += nth) sin[t] = in[e * pin + t];
    __syncthreads();
    for (int t = tid; t < ns * ns * nt; t += nth) {
        const int i = t % nt, b = (t / nt) % ns, c = t / (nt * ns);
        T s = 0;
        for (int a = 0; a < ns; ++a) s += sJ[i * ns + a] * sin[a + ns * (b + ns * c)];
        t1[t] = s;
    }
    __syncthreads();
    for (int t = tid; t < ns * nt * nt; t += nth) {
        const int i = t % nt, j = (t / nt) % nt, c = t / (nt * nt);
        T s = 0;
        for (int b = 0; b < ns; ++b) s += sJ[j * ns + b] * t1[i + nt * (b + ns * c)];
        t2[t] = s;
    }
    __syncthreads();
    for (int t = tid; t < pout; t += nth) {
        const int i = t % nt, j = (t / nt) % nt, k = t / (nt * nt);
        T s = 0;
        for (int c = 0; c < ns; ++c) s += sJ[k * ns + c] * t2[i + nt * (j + nt * c)];
        out[e * pout + t] = s;
    }
}

template <typename T>
int launch_interp(int64_t E, int ns, int nt, const T *J, const T *in, T *out, bool transpose,
                  hipStream_t s)
{
    if (ns > 16 || nt > 16) {
        set_error("interp: order too large");
        return SEM_EINVAL;
    }
    const size_t shm = sizeof(T) * ((size_t)ns * ns * ns + (size_t)ns * ns * nt + (size_t)ns * nt * nt);
    const int pout = nt * nt * nt;
    const int bs = pout >= 256 ? 256 : ((pout + 63) / 64) * 64;
    hipLaunchKernelGGL(interp_kernel<T>, dim3((unsigned)E), dim3(bs), shm, s, E, ns, nt, J,
                       transpose, in, out);
    SEM_HIP(hipGetLastError());
    return SEM_OK;
}
template int launch_interp<double>(int64_t, int, int, const double *, const double *, double *,
                                   bool, hipStream_t);
template int launch_interp<float>(int64_t, int, int, const float *, const float *, float *, bool,
                                  hipStream_t);


// ---------------------------------------------------------------------------
// Fused p-multigrid transfers between a smoother level F (nq_F <= 8, so an
// element's (i,j) columns fit one wavefront) and the next coarser level C, for
// a batch of vectors (grid.y).  J = F.Jc32 [nq_F][nq_C] interpolates coarse
// nodes to fine points (Sec. 3.4: the coarse spaces are nested, J the
// tensor-product Lagrange interpolation).  A lane owns fine column (i,j) and
// its k-line; contractions run k in registers, then j and i through LDS.
//   restriction: out_C = mask_C o (J^T (x) J^T (x) J^T) [W_F (r - t)]
//   prolongation: x_F += (J (x) J (x) J) in_C
// Masking the restricted residual before QQ^T equals masking after it: all
// copies of a Dirichlet node carry W = 0.
// ---------------------------------------------------------------------------
template <int NF>
struct XferShape {
    static constexpr int TPE = NF * NF;
    static constexpr int EPB = 64 / TPE;
    static constexpr int LDI = (NF % 2 == 0) ? NF + 1 : NF;
};

template <int NF, typename TO>
__global__ void __launch_bounds__(64)
restrict_resid_kernel(int64_t E, int nc, const float *__restrict__ J, const float *__restrict__ W,
                      const float *__restrict__ r, const float *__restrict__ t, int64_t ldf,
                      const float *__restrict__ Wc, TO *__restrict__ out, int64_t ldc, VSet vs)
{
    using X = XferShape<NF>;
    constexpr int TPE = X::TPE, EPB = X::EPB, LDI = X::LDI, NPF = NF * NF * NF;
    __shared__ float sJ[NF][NF];                // sJ[f][c] = J[f][c], c < nc
    __shared__ float sv[EPB][NF][NF][LDI];      // [c][j][i] after the k contraction
    __shared__ float sw[EPB][NF][NF][LDI];      // [c][b][i] after the j contraction
    const int64_t v = vs.at(blockIdx.y);
    r += v * ldf;
    t += v * ldf;
    out += v * ldc;
    const int tid = threadIdx.x;
    const int el = tid / TPE, ij = tid - el * TPE;
    const int i = ij % NF, j = ij / NF;
    const bool lane_ok = el < EPB;
    if (tid < NF * nc) sJ[tid / nc][tid % nc] = J[tid];
    const int ncc = nc * nc * nc;
    const int64_t groups = (E + EPB - 1) / EPB;
    for (int64_t g = blockIdx.x; g < groups; g += gridDim.x) {
        const int64_t e = g * EPB + el;
        const bool act = lane_ok && e < E;
        __syncthreads();  // sJ ready; LDS of the previous group consumed
        if (act) {
            float sk[NF];
#pragma unroll
            for (int k = 0; k < NF; ++k) {
                const int64_t p = e * NPF + k * TPE + ij;
                sk[k] = W[p] * (r[p] - t[p]);
            }
#pragma unroll
            for (int c = 0; c < NF; ++c) {
                if (c < nc) {
                    float a = 0.0f;
#pragma unroll
                    for (int k = 0; k < NF; ++k) a += sJ[k][c] * sk[k];
                    sv[el][c][j][i] = a;
                }
            }
        }
        __syncthreads();
        if (act) {
            for (int o = ij; o < nc * nc * NF; o += TPE) {
                const int i2 = o % NF, b = (o / NF) % nc, c = o / (NF * nc);
                float a = 0.0f;
#pragma unroll
                for (int jj = 0; jj < NF; ++jj) a += sJ[jj][b] * sv[el][c][jj][i2];
                sw[el][c][b][i2] = a;
            }
        }
        __syncthreads();
        if (act) {
            for (int o = ij; o < ncc; o += TPE) {
                const int a0 = o % nc, b = (o / nc) % nc, c = o / (nc * nc);
                float a = 0.0f;
#pragma unroll
                for (int ii = 0; ii < NF; ++ii) a += sJ[ii][a0] * sw[el][c][b][ii];
                const int64_t q = e * ncc + o;
                out[q] = Wc[q] > 0.0f ? (TO)a : TO(0);
            }
        }
    }
}

template <int NF, typename TI>
__global__ void __launch_bounds__(64)
prolong_add_kernel(int64_t E, int nc, const float *__restrict__ J, const TI *__restrict__ in,
                   int64_t ldc, float *__restrict__ x, int64_t ldf, VSet vs)
{
    using X = XferShape<NF>;
    constexpr int TPE = X::TPE, EPB = X::EPB, LDI = X::LDI, NPF = NF * NF * NF;
    __shared__ float sJ[NF][NF];             // sJ[f][c] = J[f][c], c < nc
    __shared__ float se[EPB][NF * NF * NF];  // coarse values [c][b][a]
    __shared__ float su[EPB][NF][NF][LDI];   // [c][b][i] after the a contraction
    const int64_t v = vs.at(blockIdx.y);
    in += v * ldc;
    x += v * ldf;
    const int tid = threadIdx.x;
    const int el = tid / TPE, ij = tid - el * TPE;
    const int i = ij % NF, j = ij / NF;
    const bool lane_ok = el < EPB;
    if (tid < NF * nc) sJ[tid / nc][tid % nc] = J[tid];
    const int ncc = nc * nc * nc;
    const int64_t groups = (E + EPB - 1) / EPB;
    for (int64_t g = blockIdx.x; g < groups; g += gridDim.x) {
        const int64_t e = g * EPB + el;
        const bool act = lane_ok && e < E;
        __syncthreads();
        if (act)
            for (int o = ij; o < ncc; o += TPE) se[el][o] = (float)in[e * ncc + o];
        __syncthreads();
        if (act) {
            for (int o = ij; o < nc * nc * NF; o += TPE) {
                const int i2 = o % NF, b = (o / NF) % nc, c = o / (NF * nc);
                float a = 0.0f;
                for (int aa = 0; aa < nc; ++aa) a += sJ[i2][aa] * se[el][aa + nc * (b + nc * c)];
                su[el][c][b][i2] = a;
            }
        }
        __syncthreads();
        if (act) {
            float u2[NF];
#pragma unroll
            for (int c = 0; c < NF; ++c) {
                float a = 0.0f;
                if (c < nc)
                    for (int b = 0; b < nc; ++b) a += sJ[j][b] * su[el][c][b][i];
                u2[c] = a;
            }
#pragma unroll
            for (int k = 0; k < NF; ++k) {
                float a = 0.0f;
#pragma unroll
                for (int c = 0; c < NF; ++c)
                    if (c < nc) a += sJ[k][c] * u2[c];
                const int64_t p = e * NPF + k * TPE + ij;
                x[p] += a;
            }
        }
    }
}

static int64_t xfer_grid(const Level &F)
{
    const int epb = 64 / (F.nq * F.nq);
    const int64_t groups = (F.E + epb - 1) / epb;
    const int64_t cap = (int64_t)(F.n_cu > 0 ? F.n_cu : 256) * 16;
    return groups < cap ? groups : cap;
}

template <typename TO>
int launch_restrict_resid(const Level &F, const Level &C, const float *r, const float *t, TO *out,
                          const VSet &vs, hipStream_t s)
{
    if (vs.n <= 0) return SEM_OK;
    if (F.nq > 8 || C.nq >= F.nq || C.E != F.E || !C.W32 || !F.W32 || !F.Jc32) {
        set_error("restrict: unsupported level pair nq %d -> %d", F.nq, C.nq);
        return SEM_EINVAL;
    }
    const dim3 grid((unsigned)xfer_grid(F), (unsigned)vs.n), block(64);
#define SEM_RX(NF)                                                                          \
    case NF:                                                                                \
        hipLaunchKernelGGL((restrict_resid_kernel<NF, TO>), grid, block, 0, s, F.E, C.nq,   \
                           F.Jc32, F.W32, r, t, F.nL, C.W32, out, C.nL, vs);                \
        break
    switch (F.nq) {
        SEM_RX(2); SEM_RX(3); SEM_RX(4); SEM_RX(5); SEM_RX(6); SEM_RX(7); SEM_RX(8);
    default: set_error("restrict: nq %d", F.nq); return SEM_EINVAL;
    }
#undef SEM_RX
    SEM_HIP(hipGetLastError());
    return SEM_OK;
}

template <typename TI>
int launch_prolong_add(const Level &F, const Level &C, const TI *in, float *x, const VSet &vs,
                       hipStream_t s)
{
    if (vs.n <= 0) return SEM_OK;
    if (F.nq > 8 || C.nq >= F.nq || C.E != F.E || !F.Jc32) {
        set_error("prolong: unsupported level pair nq %d -> %d", C.nq, F.nq);
        return SEM_EINVAL;
    }
    const dim3 grid((unsigned)xfer_grid(F), (unsigned)vs.n), block(64);
#define SEM_PX(NF)                                                                          \
    case NF:                                                                                \
        hipLaunchKernelGGL((prolong_add_kernel<NF, TI>), grid, block, 0, s, F.E, C.nq,      \
                           F.Jc32, in, C.nL, x, F.nL, vs);                                  \
        break
    switch (F.nq) {
        SEM_PX(2); SEM_PX(3); SEM_PX(4); SEM_PX(5); SEM_PX(6); SEM_PX(7); SEM_PX(8);
    default: set_error("prolong: nq %d", F.nq); return SEM_EINVAL;
    }
#undef SEM_PX
    SEM_HIP(hipGetLastError());
    return SEM_OK;
}
template int launch_restrict_resid<float>(const Level &, const Level &, const float *, const float *,
                                          float *, const VSet &, hipStream_t);
template int launch_restrict_resid<double>(const Level &, const Level &, const float *, const float *,
                                           double *, const VSet &, hipStream_t);
template int launch_prolong_add<float>(const Level &, const Level &, const float *, float *,
                                       const VSet &, hipStream_t);
template int launch_prolong_add<double>(const Level &, const Level &, const double *, float *,
                                        const VSet &, hipStream_t);

}  // namespace semx
