// Dealiased advection operator (NekRS paper Sec. 2.1 eqs. (stdadv) and (hyp):
// the advection term of the EXT and characteristics formulations; Sec. 2.3:
// its integrand has degree 3N and needs a quadrature finer than GLL;
// Sec. 3.3: the advection kernels, whose 2D thread structure with 1D register
// arrays along the third direction is the layout used here).
//
// Per element, with the M-point Gauss rule in each direction:
//   J [M][nq]  interpolation from the GLL nodes to the Gauss points,
//   Jd = J Dh  derivative of the interpolant at the Gauss points,
//   F [9][M^3] = rho~ |det X| dr_q/dx_d (index 3 q + d), X = dx/dr of the
//              interpolated element map (built once per mesh),
//   ct [3][M^3] = F . (J3 c)     (once per velocity field),
//   out = J3^T sum_q ct_q d_q(J3 w)   (every advected field).
//
// Thread layout (one workgroup per element, M^2 lanes rounded up to whole
// wavefronts): lane t = a + M b owns the Gauss column (b, a) and keeps values
// along the third index in registers.  The i-contraction runs on lanes
// t = j + nq k over GLL rows (coefficients J[a][i] are wave-uniform), the
// j-contraction on the columns with the lane's rows of J and Jd in registers,
// and the k-contractions forward and back run entirely in registers, the
// transposed interpolation along c being accumulated point by point so the
// Gauss-point integrand is never stored.  Two LDS buffers alternate between
// the stages.
#include <algorithm>
#include <vector>

#include "sem_internal.h"

namespace semx {

namespace {

template <int NQ, int M>
struct AdvShape {
    static constexpr int NP = NQ * NQ * NQ;
    static constexpr int MM = M * M;
    static constexpr int M3 = MM * M;
    static constexpr int SA = (2 * NQ * NQ * M > NQ * MM) ? 2 * NQ * NQ * M : NQ * MM;
    static constexpr int SB = NQ * NQ * M;  // >= NP since M >= NQ
    static constexpr int THREADS = ((MM + 63) / 64) * 64;
};

// stage 1: rows (k, j) of u in LDS (sU [k][j][i]) -> sP [k][j][a] = J u,
// sQ [k][j][a] = Jd u (contraction over i)
template <int NQ, int M>
__device__ __forceinline__ void stage_rows(const double *__restrict__ J, const double *__restrict__ Jd,
                                           const double *sU, double *sP, double *sQ)
{
    const int t = threadIdx.x;
    if (t < NQ * NQ) {
        const int j = t % NQ, k = t / NQ;
        double r[NQ];
#pragma unroll
        for (int i = 0; i < NQ; ++i) r[i] = sU[(k * NQ + j) * NQ + i];
#pragma unroll
        for (int a = 0; a < M; ++a) {
            double p = 0.0, q = 0.0;
#pragma unroll
            for (int i = 0; i < NQ; ++i) {
                p += J[a * NQ + i] * r[i];
                q += Jd[a * NQ + i] * r[i];
            }
            sP[(k * NQ + j) * M + a] = p;
            sQ[(k * NQ + j) * M + a] = q;
        }
    }
}

// stage 2 on the lane's Gauss column (b, a): Tr[k] = (J_b . sQ)[k], Ts[k] =
// (Jd_b . sP)[k], Tt[k] = (J_b . sP)[k] (contraction over j)
template <int NQ, int M>
__device__ __forceinline__ void stage_cols(const double *Jb, const double *Jdb, int a, const double *sP,
                                           const double *sQ, double *Tr, double *Ts, double *Tt)
{
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
        double xr = 0.0, xs = 0.0, xt = 0.0;
#pragma unroll
        for (int j = 0; j < NQ; ++j) {
            const double p = sP[(k * NQ + j) * M + a];
            const double q = sQ[(k * NQ + j) * M + a];
            xr += Jb[j] * q;
            xs += Jdb[j] * p;
            xt += Jb[j] * p;
        }
        Tr[k] = xr;
        Ts[k] = xs;
        Tt[k] = xt;
    }
}

template <int NQ, int M>
__global__ void __launch_bounds__((AdvShape<NQ, M>::THREADS)) __attribute__((amdgpu_waves_per_eu(1, 8)))
    advect_kernel(int64_t E, const double *__restrict__ J, const double *__restrict__ Jd,
                  const double *__restrict__ ct, int nf, const double *__restrict__ w, int64_t ldw,
                  double *__restrict__ out, int64_t ldo)
{
    using S = AdvShape<NQ, M>;
    constexpr int NP = S::NP, MM = S::MM, M3 = S::M3, TH = S::THREADS;
    __shared__ double sA[S::SA];
    __shared__ double sB[S::SB];
    double *sP = sA, *sQ = sA + NQ * NQ * M, *sG = sA;
    double *sU = sB, *sH = sB;
    const int t = threadIdx.x;
    const bool col = t < MM;
    const int a = col ? t % M : 0, b = col ? t / M : 0;
    double Jb[NQ], Jdb[NQ];
#pragma unroll
    for (int j = 0; j < NQ; ++j) {
        Jb[j] = J[b * NQ + j];
        Jdb[j] = Jd[b * NQ + j];
    }
    // the next field (or the next element's first field) is loaded into
    // registers while the current one is computed
    constexpr int PFN = (NP + TH - 1) / TH;
    double un[PFN];
    if (blockIdx.x < E) {
#pragma unroll
        for (int q = 0; q < PFN; ++q) {
            const int i = t + q * TH;
            un[q] = i < NP ? w[blockIdx.x * (int64_t)NP + i] : 0.0;
        }
    }
    for (int64_t e = blockIdx.x; e < E; e += gridDim.x) {
        double c0[M], c1[M], c2[M];
        for (int f = 0; f < nf; ++f) {
#pragma unroll
            for (int q = 0; q < PFN; ++q) {
                const int i = t + q * TH;
                if (i < NP) sU[i] = un[q];
            }
            if (f == 0 && col) {  // issued after the staged field, consumed two stages later
                const double *cte = ct + e * 3 * M3 + t;
#pragma unroll
                for (int c = 0; c < M; ++c) {
                    c0[c] = cte[c * MM];
                    c1[c] = cte[M3 + c * MM];
                    c2[c] = cte[2 * M3 + c * MM];
                }
            }
            {
                int64_t en = e;
                int fn = f + 1;
                if (fn == nf) {
                    fn = 0;
                    en = e + gridDim.x;
                }
                if (en < E) {
                    const double *src = w + fn * ldw + en * NP;
#pragma unroll
                    for (int q = 0; q < PFN; ++q) {
                        const int i = t + q * TH;
                        un[q] = i < NP ? src[i] : 0.0;
                    }
                }
            }
            __syncthreads();
            // contraction over i on GLL rows (k, j)
            if (t < NQ * NQ) {
                const int j = t % NQ, k = t / NQ;
                double r[NQ];
#pragma unroll
                for (int i = 0; i < NQ; ++i) r[i] = sU[(k * NQ + j) * NQ + i];
#pragma unroll
                for (int a2 = 0; a2 < M; ++a2) {
                    double p = 0.0, q = 0.0;
#pragma unroll
                    for (int i = 0; i < NQ; ++i) {
                        p += J[a2 * NQ + i] * r[i];
                        q += Jd[a2 * NQ + i] * r[i];
                    }
                    sP[(k * NQ + j) * M + a2] = p;
                    sQ[(k * NQ + j) * M + a2] = q;
                }
            }
            __syncthreads();
            double G[NQ];
            if (col) {
                // contraction over j on the lane's Gauss column
                double Tr[NQ], Ts[NQ], Tt[NQ];
#pragma unroll
                for (int k = 0; k < NQ; ++k) {
                    double xr = 0.0, xs = 0.0, xt = 0.0;
#pragma unroll
                    for (int j = 0; j < NQ; ++j) {
                        const double p = sP[(k * NQ + j) * M + a], q = sQ[(k * NQ + j) * M + a];
                        xr += Jb[j] * q;
                        xs += Jdb[j] * p;
                        xt += Jb[j] * p;
                    }
                    Tr[k] = xr;
                    Ts[k] = xs;
                    Tt[k] = xt;
                }
                // over k: derivatives at the Gauss points, integrand, and the
                // transposed interpolation back along k, point by point
#pragma unroll
                for (int k = 0; k < NQ; ++k) G[k] = 0.0;
#pragma unroll
                for (int c = 0; c < M; ++c) {
                    double dr = 0.0, ds = 0.0, dt = 0.0;
#pragma unroll
                    for (int k = 0; k < NQ; ++k) {
                        dr += J[c * NQ + k] * Tr[k];
                        ds += J[c * NQ + k] * Ts[k];
                        dt += Jd[c * NQ + k] * Tt[k];
                    }
                    const double fv = c0[c] * dr + c1[c] * ds + c2[c] * dt;
#pragma unroll
                    for (int k = 0; k < NQ; ++k) G[k] += J[c * NQ + k] * fv;
                }
            }
            __syncthreads();  // every lane is done reading sP / sQ
            if (col) {
#pragma unroll
                for (int k = 0; k < NQ; ++k) sG[(k * M + b) * M + a] = G[k];
            }
            __syncthreads();
            // contraction over b -> j on lanes (a, k)
            if (t < NQ * M) {
                const int a2 = t % M, k = t / M;
                double H[NQ];
#pragma unroll
                for (int j = 0; j < NQ; ++j) H[j] = 0.0;
#pragma unroll
                for (int b2 = 0; b2 < M; ++b2) {
                    const double g = sG[(k * M + b2) * M + a2];
#pragma unroll
                    for (int j = 0; j < NQ; ++j) H[j] += J[b2 * NQ + j] * g;
                }
#pragma unroll
                for (int j = 0; j < NQ; ++j) sH[(k * NQ + j) * M + a2] = H[j];
            }
            __syncthreads();
            // contraction over a -> i on GLL rows (k, j)
            if (t < NQ * NQ) {
                const int j = t % NQ, k = t / NQ;
                double h[M];
#pragma unroll
                for (int a2 = 0; a2 < M; ++a2) h[a2] = sH[(k * NQ + j) * M + a2];
                double o[NQ];
#pragma unroll
                for (int i = 0; i < NQ; ++i) o[i] = 0.0;
#pragma unroll
                for (int a2 = 0; a2 < M; ++a2)
#pragma unroll
                    for (int i = 0; i < NQ; ++i) o[i] += J[a2 * NQ + i] * h[a2];
                double *op = out + f * ldo + e * NP + (k * NQ + j) * NQ;
#pragma unroll
                for (int i = 0; i < NQ; ++i) op[i] = o[i];
            }
            __syncthreads();  // sH is read before the next field is staged into sB
        }
    }
}

// The 3D thread-block variant (Sec. 3.3: one thread per quadrature point,
// possible while the M^3 points fit one workgroup, M <= 10): thread
// t = a + M b + M^2 c owns the Gauss point (c, b, a) and keeps its three
// contravariant velocity components in registers; every contraction is a
// pass through LDS (three buffers used in rotation) with a barrier between.
template <int NQ, int M>
struct Adv3Shape {
    static constexpr int NP = NQ * NQ * NQ, MM = M * M, M3 = MM * M;
    static constexpr int THREADS = ((M3 + 63) / 64) * 64;
    static constexpr int SX = (2 * NQ * NQ * M > NQ * MM) ? 2 * NQ * NQ * M : NQ * MM;  // P, Q; then G
    static constexpr int SY = (3 * NQ * MM > NQ * NQ * M) ? 3 * NQ * MM : NQ * NQ * M;  // T; then H
    static constexpr int SZ = (NP > M3) ? NP : M3;                                     // u; then f
};

template <int NQ, int M>
__global__ void __launch_bounds__((Adv3Shape<NQ, M>::THREADS))
    advect3d_kernel(int64_t E, const double *__restrict__ J, const double *__restrict__ Jd,
                    const double *__restrict__ ct, int nf, const double *__restrict__ w, int64_t ldw,
                    double *__restrict__ out, int64_t ldo)
{
    using S = Adv3Shape<NQ, M>;
    constexpr int NP = S::NP, MM = S::MM, M3 = S::M3, TH = S::THREADS;
    static_assert(TH <= 1024, "the 3D variant needs M^3 <= 1024");
    __shared__ double sX[S::SX], sY[S::SY], sZ[S::SZ];
    __shared__ double sJ[M * NQ], sJd[M * NQ];
    const int t = threadIdx.x;
    for (int i = t; i < M * NQ; i += TH) {
        sJ[i] = J[i];
        sJd[i] = Jd[i];
    }
    const bool pt = t < M3;
    const int a = t % M, b = (t / M) % M, c = t / MM;
    for (int64_t e = blockIdx.x; e < E; e += gridDim.x) {
        double c0 = 0.0, c1 = 0.0, c2 = 0.0;
        if (pt) {
            const double *cte = ct + e * 3 * M3 + t;
            c0 = cte[0];
            c1 = cte[M3];
            c2 = cte[2 * M3];
        }
        for (int f = 0; f < nf; ++f) {
            __syncthreads();  // the previous field's last reads are done
            const double *u = w + f * ldw + e * NP;
            for (int i = t; i < NP; i += TH) sZ[i] = u[i];
            __syncthreads();
            // over i: P[k][j][a] = J u, Q[k][j][a] = Jd u
            if (t < NQ * NQ * M) {
                const int a2 = t % M, j = (t / M) % NQ, k = t / (M * NQ);
                double pp = 0.0, qq = 0.0;
#pragma unroll
                for (int i = 0; i < NQ; ++i) {
                    const double ui = sZ[(k * NQ + j) * NQ + i];
                    pp += sJ[a2 * NQ + i] * ui;
                    qq += sJd[a2 * NQ + i] * ui;
                }
                sX[(k * NQ + j) * M + a2] = pp;
                sX[NQ * NQ * M + (k * NQ + j) * M + a2] = qq;
            }
            __syncthreads();
            // over j: the three partial derivative fields T[d][k][b][a]
            if (t < NQ * MM) {
                const int a2 = t % M, b2 = (t / M) % M, k = t / MM;
                double xr = 0.0, xs = 0.0, xt = 0.0;
#pragma unroll
                for (int j = 0; j < NQ; ++j) {
                    const double pp = sX[(k * NQ + j) * M + a2];
                    const double qq = sX[NQ * NQ * M + (k * NQ + j) * M + a2];
                    xr += sJ[b2 * NQ + j] * qq;
                    xs += sJd[b2 * NQ + j] * pp;
                    xt += sJ[b2 * NQ + j] * pp;
                }
                sY[k * MM + b2 * M + a2] = xr;
                sY[(NQ + k) * MM + b2 * M + a2] = xs;
                sY[(2 * NQ + k) * MM + b2 * M + a2] = xt;
            }
            __syncthreads();
            // over k: reference derivatives at the thread's Gauss point, integrand
            if (pt) {
                double dr = 0.0, ds = 0.0, dt = 0.0;
#pragma unroll
                for (int k = 0; k < NQ; ++k) {
                    dr += sJ[c * NQ + k] * sY[k * MM + b * M + a];
                    ds += sJ[c * NQ + k] * sY[(NQ + k) * MM + b * M + a];
                    dt += sJd[c * NQ + k] * sY[(2 * NQ + k) * MM + b * M + a];
                }
                sZ[t] = c0 * dr + c1 * ds + c2 * dt;
            }
            __syncthreads();
            // back over c: G[k][b][a]
            if (t < NQ * MM) {
                const int a2 = t % M, b2 = (t / M) % M, k = t / MM;
                double g = 0.0;
#pragma unroll
                for (int c2i = 0; c2i < M; ++c2i) g += sJ[c2i * NQ + k] * sZ[c2i * MM + b2 * M + a2];
                sX[k * MM + b2 * M + a2] = g;
            }
            __syncthreads();
            // back over b: H[k][j][a]
            if (t < NQ * NQ * M) {
                const int a2 = t % M, j = (t / M) % NQ, k = t / (M * NQ);
                double hh = 0.0;
#pragma unroll
                for (int b2 = 0; b2 < M; ++b2) hh += sJ[b2 * NQ + j] * sX[k * MM + b2 * M + a2];
                sY[(k * NQ + j) * M + a2] = hh;
            }
            __syncthreads();
            // back over a: out[k][j][i]
            if (t < NP) {
                const int i = t % NQ, j = (t / NQ) % NQ, k = t / (NQ * NQ);
                double o = 0.0;
#pragma unroll
                for (int a2 = 0; a2 < M; ++a2) o += sJ[a2 * NQ + i] * sY[(k * NQ + j) * M + a2];
                out[f * ldo + e * NP + t] = o;
            }
        }
    }
}

// Reference gradients out[e * ostride + q * M^3 + p], q = r, s, t, of the
// interpolant of the L-vector u at the Gauss points p = a + M b + M^2 c.
template <int NQ, int M>
__global__ void __launch_bounds__(256)
    fine_grad_kernel(int64_t E, const double *__restrict__ J, const double *__restrict__ Jd,
                     const double *__restrict__ u, double *__restrict__ out, int64_t ostride)
{
    using S = AdvShape<NQ, M>;
    __shared__ double sA[S::SA];
    __shared__ double sB[S::SB];
    double *sP = sA, *sQ = sA + NQ * NQ * M;
    double *sU = sB;
    const int t = threadIdx.x;
    const bool col = t < S::MM;
    const int a = col ? t % M : 0, b = col ? t / M : 0;
    double Jb[NQ], Jdb[NQ];
#pragma unroll
    for (int j = 0; j < NQ; ++j) {
        Jb[j] = J[b * NQ + j];
        Jdb[j] = Jd[b * NQ + j];
    }
    for (int64_t e = blockIdx.x; e < E; e += gridDim.x) {
        const double *ue = u + e * S::NP;
        for (int i = t; i < S::NP; i += blockDim.x) sU[i] = ue[i];
        __syncthreads();
        stage_rows<NQ, M>(J, Jd, sU, sP, sQ);
        __syncthreads();
        if (col) {
            double *oe = out + e * ostride + t;
            double Tr[NQ], Ts[NQ], Tt[NQ];
            stage_cols<NQ, M>(Jb, Jdb, a, sP, sQ, Tr, Ts, Tt);
#pragma unroll
            for (int c = 0; c < M; ++c) {
                double dr = 0.0, ds = 0.0, dt = 0.0;
#pragma unroll
                for (int k = 0; k < NQ; ++k) {
                    dr += J[c * NQ + k] * Tr[k];
                    ds += J[c * NQ + k] * Ts[k];
                    dt += Jd[c * NQ + k] * Tt[k];
                }
                oe[c * S::MM] = dr;
                oe[S::M3 + c * S::MM] = ds;
                oe[2 * S::M3 + c * S::MM] = dt;
            }
        }
        __syncthreads();  // sU / sP are rewritten for the next element
    }
}

// F [E][9][M^3]: raw derivatives X[d][q] = dx_d/dr_q at index 3 d + q on
// entry; rho~ |det X| dr_q/dx_d = rho~ sign(det X) adj(X)[q][d] at index
// 3 q + d on exit.  bad |= 1 where det X <= 0.
__global__ void metric_kernel(int64_t E, int M, const double *__restrict__ wq, double *__restrict__ F,
                              int *bad)
{
    const int64_t M3 = (int64_t)M * M * M;
    const int64_t n = E * M3;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = g / M3, p = g % M3;
        double *Fe = F + e * 9 * M3 + p;
        double X[9];
#pragma unroll
        for (int m = 0; m < 9; ++m) X[m] = Fe[m * M3];
        // X[3 d + q]: rows d = x, y, z; columns q = r, s, t
        double A[9];  // adjugate, A[3 q + d]
        A[0] = X[4] * X[8] - X[5] * X[7];
        A[1] = X[2] * X[7] - X[1] * X[8];
        A[2] = X[1] * X[5] - X[2] * X[4];
        A[3] = X[5] * X[6] - X[3] * X[8];
        A[4] = X[0] * X[8] - X[2] * X[6];
        A[5] = X[2] * X[3] - X[0] * X[5];
        A[6] = X[3] * X[7] - X[4] * X[6];
        A[7] = X[1] * X[6] - X[0] * X[7];
        A[8] = X[0] * X[4] - X[1] * X[3];
        const double det = X[0] * A[0] + X[1] * A[3] + X[2] * A[6];
        if (!(det > 0.0)) atomicOr(bad, 1);
        const int ia = (int)(p % M), ib = (int)((p / M) % M), ic = (int)(p / ((int64_t)M * M));
        const double rho = wq[ia] * wq[ib] * wq[ic] * (det < 0.0 ? -1.0 : 1.0);
#pragma unroll
        for (int m = 0; m < 9; ++m) Fe[m * M3] = rho * A[m];
    }
}

// ct[e][q][p] = sum_d F[e][3 q + d][p] (J3 c_d)[p]: the three velocity
// components interpolated to the Gauss points and turned contravariant in one
// pass.  Lane t = a + M b owns the Gauss column (b, a) as in the advection
// kernel; the components go through LDS one after another (contraction over
// i on GLL rows, then over j and k on the column in registers), the lane
// keeps its 3 M interpolated values in registers, and the column's nine
// factors are read and the three products written point by point, so the
// interpolated velocity never reaches memory.
template <int NQ, int M>
__global__ void __launch_bounds__((AdvShape<NQ, M>::THREADS))
    velocity_kernel(int64_t E, const double *__restrict__ J, const double *__restrict__ F,
                    const double *__restrict__ c, int64_t ldc, double *__restrict__ ct)
{
    using S = AdvShape<NQ, M>;
    constexpr int NP = S::NP, MM = S::MM, M3 = S::M3, TH = S::THREADS;
    __shared__ double sU[NP];
    __shared__ double sP[NQ * NQ * M];
    const int t = threadIdx.x;
    const bool col = t < MM;
    const int a = col ? t % M : 0, b = col ? t / M : 0;
    double Jb[NQ];
#pragma unroll
    for (int j = 0; j < NQ; ++j) Jb[j] = J[b * NQ + j];
    for (int64_t e = blockIdx.x; e < E; e += gridDim.x) {
        double v[3][M];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double *ue = c + d * ldc + e * NP;
            for (int i = t; i < NP; i += TH) sU[i] = ue[i];
            __syncthreads();
            // over i on GLL rows (k, j): sP[k][j][a] = (J u)[k][j][a]
            for (int r = t; r < NQ * NQ; r += TH) {
                double ri[NQ];
#pragma unroll
                for (int i = 0; i < NQ; ++i) ri[i] = sU[r * NQ + i];
#pragma unroll
                for (int a2 = 0; a2 < M; ++a2) {
                    double p = 0.0;
#pragma unroll
                    for (int i = 0; i < NQ; ++i) p += J[a2 * NQ + i] * ri[i];
                    sP[r * M + a2] = p;
                }
            }
            __syncthreads();
            if (col) {
                double Tt[NQ];
#pragma unroll
                for (int k = 0; k < NQ; ++k) {
                    double x = 0.0;
#pragma unroll
                    for (int j = 0; j < NQ; ++j) x += Jb[j] * sP[(k * NQ + j) * M + a];
                    Tt[k] = x;
                }
#pragma unroll
                for (int cc = 0; cc < M; ++cc) {
                    double x = 0.0;
#pragma unroll
                    for (int k = 0; k < NQ; ++k) x += J[cc * NQ + k] * Tt[k];
                    v[d][cc] = x;
                }
            }
            __syncthreads();  // sU and sP are rewritten for the next component
        }
        if (col) {
            const double *Fe = F + e * 9 * M3 + t;
            double *ce = ct + e * 3 * M3 + t;
#pragma unroll
            for (int cc = 0; cc < M; ++cc) {
                const int p = cc * MM;
#pragma unroll
                for (int q = 0; q < 3; ++q)
                    ce[q * M3 + p] = Fe[(3 * q) * M3 + p] * v[0][cc] + Fe[(3 * q + 1) * M3 + p] * v[1][cc] +
                                     Fe[(3 * q + 2) * M3 + p] * v[2][cc];
            }
        }
    }
}

int rule_default(int N) { return (3 * N + 2) / 2; }

// automatic choice: the 3D thread block up to this M, the 2D one above.  On
// 32^3 elements, three fields, the 2D block is faster at every compiled pair
// (N, M) = (3, 5) 75 vs 126 us, (4, 7) 170 vs 488, (5, 8) 256 vs 577,
// (6, 10) 558 vs 1556, so the 3D block is never picked automatically.
constexpr int kAdv3AutoMaxM = 0;

bool rule_supported(int N, int M) { return N >= 1 && N <= 7 && (M == rule_default(N) || M == rule_default(N) + 1); }

int64_t adv_grid(const Level &L)
{
    const int64_t cap = (int64_t)(L.n_cu > 0 ? L.n_cu : 256) * 8;
    return std::max<int64_t>(1, std::min<int64_t>(L.E, cap));
}

// dispatch over the compiled (nq, M) pairs: M = ceil((3N+1)/2) and one more
#define SEM_ADV_PAIRS(X) \
    X(2, 2) X(2, 3) X(3, 4) X(3, 5) X(4, 5) X(4, 6) X(5, 7) X(5, 8) X(6, 8) X(6, 9) X(7, 10) X(7, 11) X(8, 11) X(8, 12)

int launch_fine_grad(const Level &L, int M, const double *J, const double *Jd, const double *u, double *out,
                     int64_t ostride, hipStream_t s)
{
    const dim3 grid((unsigned)adv_grid(L));
#define SEM_FG(NQ_, M_)                                                                              \
    if (L.nq == NQ_ && M == M_) {                                                                    \
        hipLaunchKernelGGL((fine_grad_kernel<NQ_, M_>), grid, dim3(AdvShape<NQ_, M_>::THREADS), 0, s, L.E, J, \
                           Jd, u, out, ostride);                                                     \
        SEM_HIP(hipGetLastError());                                                                  \
        return SEM_OK;                                                                               \
    }
    SEM_ADV_PAIRS(SEM_FG)
#undef SEM_FG
    set_error("advection: no kernel for N = %d, M = %d", L.N, M);
    return SEM_EINVAL;
}

int launch_velocity(const Level &L, int M, const double *J, const double *F, const double *c, int64_t ldc,
                    double *ct, hipStream_t s)
{
    const int64_t cap = (int64_t)(L.n_cu > 0 ? L.n_cu : 256) * 16;
    const dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>(L.E, cap)));
#define SEM_VEL(NQ_, M_)                                                                            \
    if (L.nq == NQ_ && M == M_) {                                                                   \
        hipLaunchKernelGGL((velocity_kernel<NQ_, M_>), grid, dim3(AdvShape<NQ_, M_>::THREADS), 0, s, \
                           L.E, J, F, c, ldc, ct);                                                  \
        SEM_HIP(hipGetLastError());                                                                 \
        return SEM_OK;                                                                              \
    }
    SEM_ADV_PAIRS(SEM_VEL)
#undef SEM_VEL
    set_error("advection: no kernel for N = %d, M = %d", L.N, M);
    return SEM_EINVAL;
}

#define SEM_ADV3_PAIRS(X) \
    X(2, 2) X(2, 3) X(3, 4) X(3, 5) X(4, 5) X(4, 6) X(5, 7) X(5, 8) X(6, 8) X(6, 9) X(7, 10)

bool has_3d(int nq, int M)
{
#define SEM_H3(NQ_, M_) \
    if (nq == NQ_ && M == M_) return true;
    SEM_ADV3_PAIRS(SEM_H3)
#undef SEM_H3
    return false;
}

int launch_advect(const Level &L, int M, int variant, const double *J, const double *Jd, const double *ct,
                  int nf, const double *w, int64_t ldw, double *out, int64_t ldo, hipStream_t s)
{
    if (variant == SEM_ADVECT_3D) {
        const dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>(L.E, (int64_t)(L.n_cu > 0 ? L.n_cu : 256) * 8)));
#define SEM_ADV3(NQ_, M_)                                                                           \
    if (L.nq == NQ_ && M == M_) {                                                                   \
        hipLaunchKernelGGL((advect3d_kernel<NQ_, M_>), grid, dim3(Adv3Shape<NQ_, M_>::THREADS), 0, s, \
                           L.E, J, Jd, ct, nf, w, ldw, out, ldo);                                   \
        SEM_HIP(hipGetLastError());                                                                 \
        return SEM_OK;                                                                              \
    }
        SEM_ADV3_PAIRS(SEM_ADV3)
#undef SEM_ADV3
        set_error("advection: no 3D kernel for N = %d, M = %d", L.N, M);
        return SEM_EINVAL;
    }
    // 16 workgroups per CU (measured at N = 7, M = 11: 4 per CU 712 us, 16 per
    // CU 623 us for three fields on 32^3 elements)
    const int64_t cap = (int64_t)(L.n_cu > 0 ? L.n_cu : 256) * 16;
    const dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>(L.E, cap)));
#define SEM_ADV(NQ_, M_)                                                                             \
    if (L.nq == NQ_ && M == M_) {                                                                    \
        hipLaunchKernelGGL((advect_kernel<NQ_, M_>), grid, dim3(AdvShape<NQ_, M_>::THREADS), 0, s,   \
                           L.E, J, Jd, ct, nf, w, ldw, out, ldo);                                    \
        SEM_HIP(hipGetLastError());                                                                  \
        return SEM_OK;                                                                               \
    }
    SEM_ADV_PAIRS(SEM_ADV)
#undef SEM_ADV
    set_error("advection: no kernel for N = %d, M = %d", L.N, M);
    return SEM_EINVAL;
}

int alloc_upload(double **dst, const std::vector<double> &v)
{
    SEM_HIP(hipMalloc(dst, sizeof(double) * v.size()));
    SEM_HIP(hipMemcpy(*dst, v.data(), sizeof(double) * v.size(), hipMemcpyHostToDevice));
    return SEM_OK;
}

int advect_setup(sem_handle h, int M, hipStream_t s)
{
    const Level &L = h->lv[0];
    const int N = L.N, nq = L.nq;
    std::vector<double> xi(nq), D(nq * nq), g(M), wq(M), J(M * nq), Jd(M * nq, 0.0);
    SEM_TRY(host_gll(N, xi.data(), nullptr, D.data()));
    SEM_TRY(host_gauss(M, g.data(), wq.data()));
    host_interp(nq, xi.data(), M, g.data(), J.data());
    for (int a = 0; a < M; ++a)
        for (int l = 0; l < nq; ++l) {
            double v = 0.0;
            for (int i = 0; i < nq; ++i) v += J[a * nq + i] * D[i * nq + l];
            Jd[a * nq + l] = v;
        }
    auto &A = h->adv;
    SEM_TRY(alloc_upload(&A.J, J));
    SEM_TRY(alloc_upload(&A.Jd, Jd));
    SEM_TRY(alloc_upload(&A.wq, wq));
    const int64_t M3 = (int64_t)M * M * M;
    SEM_HIP(hipMalloc(&A.F, sizeof(double) * 9 * M3 * L.E));
    const double *X[3] = {h->cx, h->cy, h->cz};
    for (int d = 0; d < 3; ++d)
        SEM_TRY(launch_fine_grad(L, M, A.J, A.Jd, X[d], A.F + 3 * d * M3, 9 * M3, s));
    int *bad = nullptr;
    SEM_HIP(hipMalloc(&bad, sizeof(int)));
    int hbad = 0;
    int rc = SEM_OK;
    if (hipMemsetAsync(bad, 0, sizeof(int), s) != hipSuccess) rc = SEM_EHIP;
    if (rc == SEM_OK) {
        const int64_t n = L.E * M3;
        const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
        hipLaunchKernelGGL(metric_kernel, dim3(blocks), dim3(256), 0, s, L.E, M, A.wq, A.F, bad);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            rc = SEM_EHIP;
    }
    (void)hipFree(bad);
    if (rc != SEM_OK) {
        set_error("advection setup: %s", hipGetErrorString(hipGetLastError()));
        return rc;
    }
    if (hbad) {
        set_error("advection setup: det(dx/dr) <= 0 at a Gauss point");
        return SEM_EMESH;
    }
    A.M = M;
    return SEM_OK;
}

}  // namespace

void free_advect(sem_handle h)
{
    auto &A = h->adv;
    void *ptrs[] = {A.J, A.Jd, A.wq, A.F};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    A = sem_handle_s::Advect{};
}

}  // namespace semx

using namespace semx;

extern "C" {

int sem_advect_setup(sem_handle h, int M, int variant, int *M_used, void *stream)
{
    if (!h || h->n_levels < 1) {
        set_error("sem_advect_setup: null handle");
        return SEM_EINVAL;
    }
    const int N = h->lv[0].N;
    if (M == 0) M = rule_default(N);
    if (M < N + 1 || M > kMaxGauss || !rule_supported(N, M)) {
        set_error("sem_advect_setup: M = %d not supported for N = %d (N <= 7, M = %d or %d)", M, N,
                  rule_default(N), rule_default(N) + 1);
        return SEM_EINVAL;
    }
    if (!h->cx) {
        set_error("sem_advect_setup: the handle holds no coordinates");
        return SEM_EINVAL;
    }
    if (variant != SEM_ADVECT_AUTO && variant != SEM_ADVECT_2D && variant != SEM_ADVECT_3D) {
        set_error("sem_advect_setup: bad variant %d", variant);
        return SEM_EINVAL;
    }
    const bool can3 = has_3d(N + 1, M);
    if (variant == SEM_ADVECT_3D && !can3) {
        set_error("sem_advect_setup: the 3D variant needs M^3 <= 1024 (M = %d, N = %d)", M, N);
        return SEM_EINVAL;
    }
    if (variant == SEM_ADVECT_AUTO) variant = (can3 && M <= kAdv3AutoMaxM) ? SEM_ADVECT_3D : SEM_ADVECT_2D;
    free_advect(h);
    const int rc = advect_setup(h, M, (hipStream_t)stream);
    if (rc != SEM_OK) {
        free_advect(h);
        return rc;
    }
    h->adv.variant = variant;
    if (M_used) *M_used = M;
    return SEM_OK;
}

int sem_advect_velocity(sem_handle h, const double *c, int64_t ldc, double *ct, void *stream)
{
    if (!h || !c || !ct) {
        set_error("sem_advect_velocity: null argument");
        return SEM_EINVAL;
    }
    const auto &A = h->adv;
    if (A.M == 0) {
        set_error("sem_advect_velocity: call sem_advect_setup first");
        return SEM_EINVAL;
    }
    const Level &L = h->lv[0];
    if (ldc < L.nL) {
        set_error("sem_advect_velocity: ldc = %lld < n_local = %lld", (long long)ldc, (long long)L.nL);
        return SEM_EINVAL;
    }
    const hipStream_t s = (hipStream_t)stream;
    return launch_velocity(L, A.M, A.J, A.F, c, ldc, ct, s);
}

int sem_advect(sem_handle h, const double *ct, int nf, const double *w, int64_t ldw, double *out, int64_t ldo,
               void *stream)
{
    if (!h) {
        set_error("sem_advect: null handle");
        return SEM_EINVAL;
    }
    const auto &A = h->adv;
    if (A.M == 0) {
        set_error("sem_advect: call sem_advect_setup first");
        return SEM_EINVAL;
    }
    if (nf < 0 || nf > kMaxRhs) {
        set_error("sem_advect: nf = %d outside [0, %d]", nf, kMaxRhs);
        return SEM_EINVAL;
    }
    if (nf == 0) return SEM_OK;
    if (!ct || !w || !out) {
        set_error("sem_advect: null argument");
        return SEM_EINVAL;
    }
    const Level &L = h->lv[0];
    if (nf > 1 && (ldw < L.nL || ldo < L.nL)) {
        set_error("sem_advect: leading dimensions must be >= n_local = %lld", (long long)L.nL);
        return SEM_EINVAL;
    }
    return launch_advect(L, A.M, A.variant, A.J, A.Jd, ct, nf, w, ldw, out, ldo, (hipStream_t)stream);
}

}  // extern "C"
