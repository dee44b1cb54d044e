// Matrix-free element operator  w = h1 A_L(k) u + h2 B u  (NekRS paper,
// Sec. 2.3, eq. (Ae)):  A^e = [D1;D2;D3]^T (k o G^e) [D1;D2;D3].
//
// Thread layout (the 2D-thread / 1D-register structure of Sec. 3.3): a thread
// owns one (i,j) column of an element and keeps the k-line of u and of the
// result in registers; u and the r/s-direction fluxes sit in LDS.  With
// (N+1)^2 <= 64 every element lives inside one 64-lane wavefront, so LDS
// traffic of an element is ordered without workgroup barriers and the
// r-flux can overwrite u plane by plane (8.6 KiB of LDS per element at N=7).
//   step 1: ur = D1 u, us = D2 u  (LDS rows), ut = D3 u (registers)
//   step 2: (wr, ws, wt) = k G (ur, us, ut), G the symmetric 3x3 per point,
//           the six factors of a point contiguous ([E][np][6], 48 B, three
//           16-byte loads per lane, each wavefront reading 3 KiB contiguous
//           per plane)
//   step 3: w = D1^T wr + D2^T ws (LDS) + D3^T wt (registers, accumulated
//           while the k-planes are swept)
// The grid is persistent (a few workgroups per CU, each sweeping elements
// with a grid stride) and the next element's u is loaded while the current
// one is computed.
// Bytes per point (FP64 Poisson): u 8 + G 48 + w 8 = 64 (+8 for B, +8 for k).
#pragma once
#include "sem_internal.h"

// FMA contraction within single expressions only: the single-vector and the
// batched kernels below then round every point identically.
#pragma clang fp contract(on)

namespace semx {

template <int NQ>
struct AxShape {
    static constexpr int TPE = NQ * NQ;                       // threads per element
    static constexpr int EPB = TPE <= 64 ? 64 / TPE : 1;      // elements per block
    static constexpr int THREADS = EPB * TPE;
    static constexpr bool ONE_WAVE = THREADS <= 64;
    static constexpr int LD = (NQ % 2 == 0) ? NQ + 1 : NQ;    // padded LDS row
};

template <bool ONE_WAVE>
__device__ inline void block_sync()
{
    if constexpr (ONE_WAVE) {
        // all threads of the block are one wavefront: order LDS accesses
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// six geometric factors of one point, stored contiguously
__device__ inline void load_g6(const double *p, double g[6])
{
    const double2 *q = reinterpret_cast<const double2 *>(p);
    const double2 a = q[0], b = q[1], c = q[2];
    g[0] = a.x; g[1] = a.y; g[2] = b.x; g[3] = b.y; g[4] = c.x; g[5] = c.y;
}
__device__ inline void load_g6(const float *p, float g[6])
{
    const float2 *q = reinterpret_cast<const float2 *>(p);
    const float2 a = q[0], b = q[1], c = q[2];
    g[0] = a.x; g[1] = a.y; g[2] = b.x; g[3] = b.y; g[4] = c.x; g[5] = c.y;
}

template <int NQ, typename T, bool HELM, bool VARK, bool DOT>
__global__ void __launch_bounds__(AxShape<NQ>::THREADS)
ax_kernel(int64_t E, const T *__restrict__ G, const T *__restrict__ B,
          const T *__restrict__ kc, const T *__restrict__ Dg, T h1, T h2,
          const T *__restrict__ u, T *__restrict__ w, double *__restrict__ partial,
          const int *__restrict__ skip)
{
    if (skip != nullptr && *skip != 0) return;
    using S = AxShape<NQ>;
    constexpr int TPE = S::TPE, EPB = S::EPB, LD = S::LD;
    constexpr int NP = NQ * NQ * NQ;
    constexpr bool INPLACE = S::ONE_WAVE;
    __shared__ T su[EPB][NQ][NQ][LD];
    __shared__ T sr_[INPLACE ? 1 : EPB][NQ][NQ][LD];
    __shared__ T ss[EPB][NQ][NQ][LD];

    const int tid = threadIdx.x;
    const int el = (EPB == 1) ? 0 : tid / TPE;  // element slot within the block
    const int ij = (EPB == 1) ? tid : tid - el * TPE;
    const int i = ij % NQ;
    const int j = ij / NQ;

    T Di[NQ], Dj[NQ], DTi[NQ], DTj[NQ];
#pragma unroll
    for (int l = 0; l < NQ; ++l) {
        Di[l] = Dg[i * NQ + l];
        Dj[l] = Dg[j * NQ + l];
        DTi[l] = Dg[l * NQ + i];
        DTj[l] = Dg[l * NQ + j];
    }

    double dot = 0.0;
    T rn[NQ];
    int64_t g = blockIdx.x;  // element group: elements g*EPB .. g*EPB+EPB-1
    {
        const int64_t e0 = g * EPB + el;
        if (e0 < E) {
#pragma unroll
            for (int k = 0; k < NQ; ++k) rn[k] = u[e0 * NP + ij + k * TPE];
        } else {
#pragma unroll
            for (int k = 0; k < NQ; ++k) rn[k] = T(0);
        }
    }
    for (; g * EPB < E; g += gridDim.x) {
        const int64_t e = g * EPB + el;
        const bool active = e < E;
        const int64_t base = (active ? e : 0) * NP + ij;
        T ru[NQ], rw[NQ];
#pragma unroll
        for (int k = 0; k < NQ; ++k) {
            ru[k] = rn[k];
            su[el][k][j][i] = ru[k];
            rw[k] = T(0);
        }
        {  // next element's u, loaded while this one is computed
            const int64_t en = (g + gridDim.x) * EPB + el;
            if (en < E) {
#pragma unroll
                for (int k = 0; k < NQ; ++k) rn[k] = u[en * NP + ij + k * TPE];
            }
        }
        block_sync<S::ONE_WAVE>();

        const T *Ge = G + base * 6;
#pragma unroll
        for (int k = 0; k < NQ; ++k) {
            T ur = 0, us = 0, ut = 0;
#pragma unroll
            for (int l = 0; l < NQ; ++l) {
                ur += Di[l] * su[el][k][j][l];
                us += Dj[l] * su[el][k][l][i];
                ut += Dg[k * NQ + l] * ru[l];
            }
            T gg[6];
            load_g6(Ge + k * TPE * 6, gg);
            if constexpr (VARK) {
                const T c = kc[base + k * TPE];
#pragma unroll
                for (int q = 0; q < 6; ++q) gg[q] *= c;
            }
            const T wr = gg[0] * ur + gg[1] * us + gg[2] * ut;
            const T ws = gg[1] * ur + gg[3] * us + gg[4] * ut;
            const T wt = gg[2] * ur + gg[4] * us + gg[5] * ut;
            if constexpr (INPLACE)
                su[el][k][j][i] = wr;  // plane k of u is no longer read
            else
                sr_[el][k][j][i] = wr;
            ss[el][k][j][i] = ws;
#pragma unroll
            for (int m = 0; m < NQ; ++m) rw[m] += Dg[k * NQ + m] * wt;
        }
        block_sync<S::ONE_WAVE>();

#pragma unroll
        for (int k = 0; k < NQ; ++k) {
            T acc = rw[k];
#pragma unroll
            for (int l = 0; l < NQ; ++l) {
                acc += DTi[l] * (INPLACE ? su[el][k][j][l] : sr_[el][k][j][l]);
                acc += DTj[l] * ss[el][k][l][i];
            }
            T out = h1 * acc;
            if constexpr (HELM) out += h2 * B[base + k * TPE] * ru[k];
            if (active) w[base + k * TPE] = out;
            if constexpr (DOT)
                if (active) dot += (double)ru[k] * (double)out;
        }
        block_sync<S::ONE_WAVE>();  // LDS is rewritten by the next element
    }

    if constexpr (DOT) {
        // deterministic block sum: LDS slots, summed by thread 0 in order
        __shared__ double sdot[S::THREADS];
        sdot[tid] = dot;
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
            for (int t = 0; t < S::THREADS; ++t) s += sdot[t];
            partial[blockIdx.x] = s;
        }
    }
}

// workgroups per CU of the persistent grid, by variant (measured on the 16^3
// and 32^3 boxes at N=7): FP64 Poisson 8, FP64 with the mass term 12, FP32 16
template <typename T>
inline int ax_blocks_per_cu(bool helm)
{
    return sizeof(T) == 4 ? 16 : (helm ? 12 : 8);
}

// Persistent grid over `groups` element groups with at most `cap`
// workgroups: the fewest workgroups that keep the per-workgroup count
// ceil(groups / cap), so every workgroup sweeps the same number of groups
// (up to one) and no tail of single-group workgroups is left behind.
inline int64_t balanced_grid(int64_t groups, int64_t cap)
{
    if (groups <= cap) return groups;
    const int64_t per = (groups + cap - 1) / cap;
    return (groups + per - 1) / per;
}

// Batched operator for nq <= 8 (an element fits one wavefront): the six
// geometric factors (and B) of a thread's k-line are loaded into registers
// once per element and applied to every live vector of the batch in turn, so
// G is read once for up to kMaxRhs fields (Sec. 3.3, reuse of the geometric
// factors across the components of a vector field).  Per point the arithmetic
// is that of ax_kernel, in the same order.  PF: the next vector's u (or the
// first vector of the next element) is loaded while the current one is
// computed.  DTL: the rows of D^T come from an LDS table instead of
// registers (fewer registers per lane, more waves per SIMD).  Without the
// mass term the launch bound asks for two waves per SIMD: the FP64 form then
// fits 248 VGPRs (some SGPRs kept in VGPR lanes) instead of 270 at one wave
// per SIMD, and three fields at 16^3 take 48.5-49.5 instead of 51 us; with the
// mass term the same bound spills 14 VGPRs and made the 32^3 lockstep p-MG
// solve 1 ms slower, so that form keeps one wave per SIMD.
template <int NQ, typename T, bool HELM, bool DOT, bool PF, bool DTL>
__global__ void __launch_bounds__(AxShape<NQ>::THREADS, HELM ? 1 : 2)
ax_multi_kernel(int64_t E, const T *__restrict__ G, const T *__restrict__ B,
                const T *__restrict__ Dg, T h1, T h2, const T *__restrict__ u, int64_t ldu,
                T *__restrict__ w, int64_t ldw, VSet vs, double *__restrict__ partial, int64_t pst,
                const int *__restrict__ skip, int skip_stride)
{
    using S = AxShape<NQ>;
    static_assert(S::ONE_WAVE, "the batched operator keeps one element group per wavefront");
    constexpr int TPE = S::TPE, EPB = S::EPB, LD = S::LD;
    constexpr int NP = NQ * NQ * NQ;
    __shared__ T su[EPB][NQ][NQ][LD];
    __shared__ T ss[EPB][NQ][NQ][LD];
    __shared__ T sdt[DTL ? NQ : 1][NQ];  // sdt[a][b] = D[b][a]
    __shared__ double sdot[DOT ? kMaxRhs : 1][S::THREADS];

    uint32_t pack;
    const int na = live_vectors(vs, skip, skip_stride, &pack);
    if (na == 0) return;  // uniform over the grid

    const int tid = threadIdx.x;
    const int el = (EPB == 1) ? 0 : tid / TPE;
    const int ij = (EPB == 1) ? tid : tid - el * TPE;
    const int i = ij % NQ;
    const int j = ij / NQ;

    T Di[NQ], Dj[NQ], DTi[DTL ? 1 : NQ], DTj[DTL ? 1 : NQ];
#pragma unroll
    for (int l = 0; l < NQ; ++l) {
        Di[l] = Dg[i * NQ + l];
        Dj[l] = Dg[j * NQ + l];
        if constexpr (!DTL) {
            DTi[l] = Dg[l * NQ + i];
            DTj[l] = Dg[l * NQ + j];
        }
    }
    if constexpr (DTL)
        if (tid < NQ * NQ) sdt[tid / NQ][tid % NQ] = Dg[(tid % NQ) * NQ + tid / NQ];
    if constexpr (DOT)
#pragma unroll
        for (int q = 0; q < kMaxRhs; ++q) sdot[q][tid] = 0.0;
    block_sync<true>();

    T rn[PF ? NQ : 1];
    int64_t g = blockIdx.x;  // element group: elements g*EPB .. g*EPB+EPB-1
    if constexpr (PF) {
        const int64_t e0 = g * EPB + el;
        const int64_t v0 = pack & 255u;
#pragma unroll
        for (int k = 0; k < NQ; ++k) rn[k] = e0 < E ? u[v0 * ldu + e0 * NP + ij + k * TPE] : T(0);
    }
    for (; g * EPB < E; g += gridDim.x) {
        const int64_t e = g * EPB + el;
        const bool active = e < E;
        const int64_t base = (active ? e : 0) * NP + ij;
        T gr[NQ][6];
        T bm[HELM ? NQ : 1];
#pragma unroll
        for (int k = 0; k < NQ; ++k) {
            load_g6(G + (base + k * TPE) * 6, gr[k]);
            if constexpr (HELM) bm[k] = B[base + k * TPE];
        }
#pragma unroll 1
        for (int q = 0; q < na; ++q) {
            const int64_t v = (pack >> (8 * q)) & 255u;
            T ru[NQ], rw[NQ];
            if constexpr (PF) {
#pragma unroll
                for (int k = 0; k < NQ; ++k) ru[k] = rn[k];
                const bool last = q + 1 == na;
                const int64_t en = (last ? g + gridDim.x : g) * EPB + el;
                if (en < E) {
                    const int64_t vn = (pack >> (8 * (last ? 0 : q + 1))) & 255u;
#pragma unroll
                    for (int k = 0; k < NQ; ++k) rn[k] = u[vn * ldu + en * NP + ij + k * TPE];
                }
            } else {
#pragma unroll
                for (int k = 0; k < NQ; ++k) ru[k] = u[v * ldu + base + k * TPE];
            }
#pragma unroll
            for (int k = 0; k < NQ; ++k) {
                su[el][k][j][i] = ru[k];
                rw[k] = T(0);
            }
            block_sync<true>();
#pragma unroll
            for (int k = 0; k < NQ; ++k) {
                T ur = 0, us = 0, ut = 0;
#pragma unroll
                for (int l = 0; l < NQ; ++l) {
                    ur += Di[l] * su[el][k][j][l];
                    us += Dj[l] * su[el][k][l][i];
                    ut += Dg[k * NQ + l] * ru[l];
                }
                const T wr = gr[k][0] * ur + gr[k][1] * us + gr[k][2] * ut;
                const T ws = gr[k][1] * ur + gr[k][3] * us + gr[k][4] * ut;
                const T wt = gr[k][2] * ur + gr[k][4] * us + gr[k][5] * ut;
                su[el][k][j][i] = wr;
                ss[el][k][j][i] = ws;
#pragma unroll
                for (int m = 0; m < NQ; ++m) rw[m] += Dg[k * NQ + m] * wt;
            }
            block_sync<true>();
            double dot = 0.0;
            if constexpr (DOT) dot = sdot[q][tid];
#pragma unroll
            for (int k = 0; k < NQ; ++k) {
                T acc = rw[k];
#pragma unroll
                for (int l = 0; l < NQ; ++l) {
                    T dti, dtj;
                    if constexpr (DTL) {
                        dti = sdt[i][l];
                        dtj = sdt[j][l];
                    } else {
                        dti = DTi[l];
                        dtj = DTj[l];
                    }
                    acc += dti * su[el][k][j][l];
                    acc += dtj * ss[el][k][l][i];
                }
                T out = h1 * acc;
                if constexpr (HELM) out += h2 * bm[k] * ru[k];
                if (active) w[v * ldw + base + k * TPE] = out;
                if constexpr (DOT)
                    if (active) dot += (double)ru[k] * (double)out;
            }
            if constexpr (DOT) sdot[q][tid] = dot;
            block_sync<true>();  // LDS is rewritten by the next vector
        }
    }

    if constexpr (DOT) {
        // deterministic block sums, one thread per live vector
        __syncthreads();
        if (tid < na) {
            double s = 0.0;
            for (int t = 0; t < S::THREADS; ++t) s += sdot[tid][t];
            partial[(int64_t)((pack >> (8 * tid)) & 255u) * pst + blockIdx.x] = s;
        }
    }
}

// batched-operator variant and workgroups per CU of its grid (measured on
// the 16^3 and 32^3 boxes at N=7 with three fields: prefetch on, D^T in
// registers, 12 workgroups per CU for FP64 and FP32)
constexpr bool kAxMultiPrefetch = true;
constexpr bool kAxMultiDtLds = false;
template <typename T>
inline int ax_multi_blocks_per_cu(bool helm)
{
    (void)helm;
    return 12;
}

template <int NQ, typename T>
static int ax_dispatch(const Level &L, const T *G, const T *B, const T *D, const T *u, T *w,
                       double h1, double h2, const T *k, double *partial, int64_t *nblocks,
                       hipStream_t s, const int *skip)
{
    using S = AxShape<NQ>;
    const int64_t groups = (L.E + S::EPB - 1) / S::EPB;
    const bool helm_ = h2 != 0.0;
    const int64_t cap = (int64_t)(L.n_cu > 0 ? L.n_cu : 256) * ax_blocks_per_cu<T>(helm_);
    const int64_t nb = balanced_grid(groups, cap);
    if (nblocks) *nblocks = nb;
    if (nb == 0) return SEM_OK;
    const bool helm = h2 != 0.0;
    const bool vark = k != nullptr;
    const bool dot = partial != nullptr;
    dim3 grid((unsigned)nb), block(S::THREADS);
#define SEM_AX_LAUNCH(H, V, P)                                                              \
    hipLaunchKernelGGL((ax_kernel<NQ, T, H, V, P>), grid, block, 0, s, L.E, G, B, k, D,    \
                       (T)h1, (T)h2, u, w, partial, skip)
    if (helm) {
        if (vark) { if (dot) SEM_AX_LAUNCH(true, true, true); else SEM_AX_LAUNCH(true, true, false); }
        else { if (dot) SEM_AX_LAUNCH(true, false, true); else SEM_AX_LAUNCH(true, false, false); }
    } else {
        if (vark) { if (dot) SEM_AX_LAUNCH(false, true, true); else SEM_AX_LAUNCH(false, true, false); }
        else { if (dot) SEM_AX_LAUNCH(false, false, true); else SEM_AX_LAUNCH(false, false, false); }
    }
#undef SEM_AX_LAUNCH
    SEM_HIP(hipGetLastError());
    return SEM_OK;
}

template <typename T>
int launch_ax(const Level &L, const T *G, const T *B, const T *D, const T *u, T *w, double h1,
              double h2, const T *k, double *partial, int64_t *nblocks, hipStream_t s,
              const int *skip)
{
    switch (L.nq) {
    case 2: return ax_dispatch<2, T>(L, G, B, D, u, w, h1, h2, k, partial, nblocks, s, skip);
    case 3: return ax_dispatch<3, T>(L, G, B, D, u, w, h1, h2, k, partial, nblocks, s, skip);
    case 4: return ax_dispatch<4, T>(L, G, B, D, u, w, h1, h2, k, partial, nblocks, s, skip);
    case 5: return ax_dispatch<5, T>(L, G, B, D, u, w, h1, h2, k, partial, nblocks, s, skip);
    case 6: return ax_dispatch<6, T>(L, G, B, D, u, w, h1, h2, k, partial, nblocks, s, skip);
    case 7: return ax_dispatch<7, T>(L, G, B, D, u, w, h1, h2, k, partial, nblocks, s, skip);
    case 8: return ax_dispatch<8, T>(L, G, B, D, u, w, h1, h2, k, partial, nblocks, s, skip);
    case 9: return ax_dispatch<9, T>(L, G, B, D, u, w, h1, h2, k, partial, nblocks, s, skip);
    case 10: return ax_dispatch<10, T>(L, G, B, D, u, w, h1, h2, k, partial, nblocks, s, skip);
    case 11: return ax_dispatch<11, T>(L, G, B, D, u, w, h1, h2, k, partial, nblocks, s, skip);
    case 12: return ax_dispatch<12, T>(L, G, B, D, u, w, h1, h2, k, partial, nblocks, s, skip);
    case 13: return ax_dispatch<13, T>(L, G, B, D, u, w, h1, h2, k, partial, nblocks, s, skip);
    case 14: return ax_dispatch<14, T>(L, G, B, D, u, w, h1, h2, k, partial, nblocks, s, skip);
    case 15: return ax_dispatch<15, T>(L, G, B, D, u, w, h1, h2, k, partial, nblocks, s, skip);
    case 16: return ax_dispatch<16, T>(L, G, B, D, u, w, h1, h2, k, partial, nblocks, s, skip);
    default: set_error("ax: unsupported order N=%d", L.N); return SEM_EINVAL;
    }
}

template <int NQ, typename T>
static int ax_multi_dispatch(const Level &L, const T *G, const T *B, const T *D, const T *u,
                             int64_t ldu, T *w, int64_t ldw, const VSet &vs, double h1, double h2,
                             double *partial, int64_t pst, int64_t *nblocks, hipStream_t s,
                             const int *skip, int skip_stride)
{
    using S = AxShape<NQ>;
    const int64_t groups = (L.E + S::EPB - 1) / S::EPB;
    const bool helm = h2 != 0.0;
    const int64_t cap = (int64_t)(L.n_cu > 0 ? L.n_cu : 256) * ax_multi_blocks_per_cu<T>(helm);
    const int64_t nb = balanced_grid(groups, cap);
    if (nblocks) *nblocks = nb;
    if (nb == 0) return SEM_OK;
    constexpr bool PF = kAxMultiPrefetch, DTL = kAxMultiDtLds;
    dim3 grid((unsigned)nb), block(S::THREADS);
#define SEM_AXM_LAUNCH(H, P)                                                                \
    hipLaunchKernelGGL((ax_multi_kernel<NQ, T, H, P, PF, DTL>), grid, block, 0, s, L.E, G, B, \
                       D, (T)h1, (T)h2, u, ldu, w, ldw, vs, partial, pst, skip, skip_stride)
    if (helm) {
        if (partial) SEM_AXM_LAUNCH(true, true); else SEM_AXM_LAUNCH(true, false);
    } else {
        if (partial) SEM_AXM_LAUNCH(false, true); else SEM_AXM_LAUNCH(false, false);
    }
#undef SEM_AXM_LAUNCH
    SEM_HIP(hipGetLastError());
    return SEM_OK;
}

template <typename T>
int launch_ax_multi(const Level &L, const T *G, const T *B, const T *D, const T *u, int64_t ldu, T *w,
                    int64_t ldw, const VSet &vs, double h1, double h2, const T *k, double *partial,
                    int64_t pst, int64_t *nblocks, hipStream_t s, const int *skip, int skip_stride)
{
    if (vs.n <= 0) return SEM_OK;
    if (vs.n == 1 || k != nullptr || L.nq > 8) {
        // one field at a time (variable coefficient, or elements wider than a wavefront)
        for (int q = 0; q < vs.n; ++q) {
            const int64_t v = vs.at(q);
            SEM_TRY(launch_ax<T>(L, G, B, D, u + v * ldu, w + v * ldw, h1, h2, k,
                                 partial ? partial + v * pst : nullptr, nblocks, s,
                                 skip ? skip + v * skip_stride : nullptr));
        }
        return SEM_OK;
    }
    switch (L.nq) {
    case 2: return ax_multi_dispatch<2, T>(L, G, B, D, u, ldu, w, ldw, vs, h1, h2, partial, pst, nblocks, s, skip, skip_stride);
    case 3: return ax_multi_dispatch<3, T>(L, G, B, D, u, ldu, w, ldw, vs, h1, h2, partial, pst, nblocks, s, skip, skip_stride);
    case 4: return ax_multi_dispatch<4, T>(L, G, B, D, u, ldu, w, ldw, vs, h1, h2, partial, pst, nblocks, s, skip, skip_stride);
    case 5: return ax_multi_dispatch<5, T>(L, G, B, D, u, ldu, w, ldw, vs, h1, h2, partial, pst, nblocks, s, skip, skip_stride);
    case 6: return ax_multi_dispatch<6, T>(L, G, B, D, u, ldu, w, ldw, vs, h1, h2, partial, pst, nblocks, s, skip, skip_stride);
    case 7: return ax_multi_dispatch<7, T>(L, G, B, D, u, ldu, w, ldw, vs, h1, h2, partial, pst, nblocks, s, skip, skip_stride);
    case 8: return ax_multi_dispatch<8, T>(L, G, B, D, u, ldu, w, ldw, vs, h1, h2, partial, pst, nblocks, s, skip, skip_stride);
    default: set_error("ax: unsupported order N=%d", L.N); return SEM_EINVAL;
    }
}

}  // namespace semx
