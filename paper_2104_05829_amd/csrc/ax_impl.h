// Matrix-free element operator  w = h1 A_L(k) u + h2 B u  (NekRS paper,
// Sec. 2.3, eq. (Ae)):  A^e = [D1;D2;D3]^T (k o G^e) [D1;D2;D3].
//
// Thread layout (the 2D-thread / 1D-register structure of Sec. 3.3): a thread
// owns one (i,j) column of an element and keeps the k-line of u and of the
// result in registers; u and the intermediate r/s-direction fluxes sit in LDS.
// With (N+1)^2 <= 64 every element lives inside one 64-lane wavefront, so the
// kernel needs no workgroup barrier: LDS traffic of one wave is ordered.
//   step 1: ur = D1 u, us = D2 u  (LDS rows), ut = D3 u (registers)
//   step 2: (wr, ws, wt) = k G (ur, us, ut), G the symmetric 3x3 per point,
//           G streamed coalesced from HBM (element-blocked [E][6][np])
//   step 3: w = D1^T wr + D2^T ws (LDS) + D3^T wt (registers, accumulated
//           while the k-planes are swept)
// Bytes per point (FP64 Poisson): u 8 + G 48 + w 8 = 64 (+8 for B, +8 for k).
#pragma once
#include "sem_internal.h"

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
    __shared__ T su[EPB][NQ][NQ][LD];
    __shared__ T sr[EPB][NQ][NQ][LD];
    __shared__ T ss[EPB][NQ][NQ][LD];

    const int tid = threadIdx.x;
    const int el = tid / TPE;
    const int ij = tid - el * TPE;
    const int i = ij % NQ;
    const int j = ij / NQ;
    const int64_t e = (int64_t)blockIdx.x * EPB + el;
    const bool active = e < E;

    T Di[NQ], Dj[NQ], DTi[NQ], DTj[NQ];
#pragma unroll
    for (int l = 0; l < NQ; ++l) {
        Di[l] = Dg[i * NQ + l];
        Dj[l] = Dg[j * NQ + l];
        DTi[l] = Dg[l * NQ + i];
        DTj[l] = Dg[l * NQ + j];
    }

    const int64_t base = (active ? e : 0) * NP + j * NQ + i;
    T ru[NQ], rw[NQ];
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
        ru[k] = active ? u[base + k * TPE] : T(0);
        su[el][k][j][i] = ru[k];
        rw[k] = T(0);
    }
    block_sync<S::ONE_WAVE>();

    const T *Ge = G + (active ? e : 0) * 6 * NP + j * NQ + i;
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
        T ur = 0, us = 0, ut = 0;
#pragma unroll
        for (int l = 0; l < NQ; ++l) {
            ur += Di[l] * su[el][k][j][l];
            us += Dj[l] * su[el][k][l][i];
            ut += Dg[k * NQ + l] * ru[l];
        }
        const int off = k * TPE;
        T g11 = Ge[0 * NP + off], g12 = Ge[1 * NP + off], g13 = Ge[2 * NP + off];
        T g22 = Ge[3 * NP + off], g23 = Ge[4 * NP + off], g33 = Ge[5 * NP + off];
        if constexpr (VARK) {
            const T c = kc[base + off];
            g11 *= c; g12 *= c; g13 *= c; g22 *= c; g23 *= c; g33 *= c;
        }
        const T wr = g11 * ur + g12 * us + g13 * ut;
        const T ws = g12 * ur + g22 * us + g23 * ut;
        const T wt = g13 * ur + g23 * us + g33 * ut;
        sr[el][k][j][i] = wr;
        ss[el][k][j][i] = ws;
#pragma unroll
        for (int m = 0; m < NQ; ++m) rw[m] += Dg[k * NQ + m] * wt;
    }
    block_sync<S::ONE_WAVE>();

    double dot = 0.0;
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
        T acc = rw[k];
#pragma unroll
        for (int l = 0; l < NQ; ++l) {
            acc += DTi[l] * sr[el][k][j][l];
            acc += DTj[l] * ss[el][k][l][i];
        }
        T out = h1 * acc;
        if constexpr (HELM) out += h2 * B[base + k * TPE] * ru[k];
        if (active) w[base + k * TPE] = out;
        if constexpr (DOT) dot += (double)ru[k] * (double)out;
    }

    if constexpr (DOT) {
        // deterministic block sum: LDS slots, summed by thread 0 in order
        __shared__ double sdot[S::THREADS];
        sdot[tid] = active ? dot : 0.0;
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
            for (int t = 0; t < S::THREADS; ++t) s += sdot[t];
            partial[blockIdx.x] = s;
        }
    }
}

template <int NQ, typename T>
static int ax_dispatch(const Level &L, const T *G, const T *B, const T *D, const T *u, T *w,
                       double h1, double h2, const T *k, double *partial, int64_t *nblocks,
                       hipStream_t s, const int *skip)
{
    using S = AxShape<NQ>;
    const int64_t nb = (L.E + S::EPB - 1) / S::EPB;
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

}  // namespace semx
