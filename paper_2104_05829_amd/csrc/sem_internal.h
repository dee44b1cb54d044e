// Internal declarations of libsem (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/sem.h"

namespace semx {

// thread-local detail text for sem_last_error()
void set_error(const char *fmt, ...);

#define SEM_HIP(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess) {                                                            \
            ::semx::set_error("%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__,    \
                              __LINE__);                                                   \
            return SEM_EHIP;                                                               \
        }                                                                                  \
    } while (0)

#define SEM_TRY(expr)                        \
    do {                                     \
        int rc_ = (expr);                    \
        if (rc_ != SEM_OK) return rc_;       \
    } while (0)

constexpr int kMaxN = 15;
// flag bit of a chunk lane's copy index: the copy starts a segment
constexpr int32_t kGsSegStart = 1 << 30;
// largest Gauss rule of the dealiased advection operator (M^2 threads per element)
constexpr int kMaxGauss = 16;
// largest number of workgroups per CU of the persistent element-operator grid
// (the operator's partial-sum buffer holds one value per workgroup)
constexpr int kAxMaxBlocksPerCU = 16;
constexpr int kMaxLevels = 4;
// largest number of vectors one batched operator / gather-scatter / solve
// call processes together
constexpr int kMaxRhs = SEM_MAX_RHS;
// largest projection space (earlier solutions kept per right-hand-side slot)
constexpr int kMaxProj = SEM_MAX_PROJ;

// A batch of vectors v = idx(0) .. idx(n-1) of an array with leading
// dimension ld (vector v starts at base + v * ld); indices packed 8 bits each.
struct VSet {
    int n;
    uint32_t pack;
    __host__ __device__ int at(int q) const { return (int)((pack >> (8 * q)) & 255u); }
    static VSet one() { return VSet{1, 0u}; }
    static VSet first(int n)
    {
        VSet v{0, 0u};
        for (int q = 0; q < n; ++q) v.push(q);
        return v;
    }
    void push(int v)
    {
        pack |= (uint32_t)v << (8 * n);
        ++n;
    }
};

// Vectors of a batch that are still to be processed: the batch's vector
// indices minus those whose flag skip[v * skip_stride] is set, packed 8 bits
// each into *pack; returns their number.
__device__ inline int live_vectors(const VSet &vs, const int *skip, int skip_stride, uint32_t *pack)
{
    int na = 0;
    uint32_t pk = 0;
#pragma unroll
    for (int q = 0; q < kMaxRhs; ++q) {
        if (q < vs.n) {
            const int v = vs.at(q);
            if (skip == nullptr || skip[(int64_t)v * skip_stride] == 0) {
                pk |= (uint32_t)v << (8 * na);
                ++na;
            }
        }
    }
    *pack = pk;
    return na;
}

// Device scalars of one Krylov solve (kept on the device between kernels).
struct KrylovScalars {
    double rz;      // (r, z)_W of the current iterate
    double rz_old;  // previous (r, z)_W (flexible CG)
    double pw;      // (p, A p)_W
    double zw;      // (z_new, A p)_W (flexible CG Polak-Ribiere term)
    double alpha;
    double beta;
    double rr;      // (r, r)_W
    double bb;      // (b, b)_W
    double tol2;    // tol^2 (b, b)_W
    double rz2[2];  // (r, z)_W by iteration parity (written by one block while
                    // the other slot is read by all blocks of the same kernel)
    int iters;
    int done;       // 1 once converged or failed; later kernels become no-ops
    int status;     // SEM_OK / SEM_EBREAKDOWN
    int maxit;
};

// One polynomial order of the discretisation on the handle's mesh.
struct Level {
    int N = 0, nq = 0, np = 0;
    int n_cu = 0;  // compute units of the device (persistent grid size)
    int64_t E = 0, nL = 0;
    int64_t n_unique = 0, ncopies = 0, nseg = 0;
    // geometry: G point-interleaved [E][np][6] (G11,G12,G13,G22,G23,G33), B [nL]
    double *G = nullptr, *B = nullptr;
    float *G32 = nullptr, *B32 = nullptr;
    double *W = nullptr;   // counting weight, 0 on Dirichlet copies
    float *W32 = nullptr;
    int64_t *gid = nullptr;
    uint8_t *dir = nullptr;
    int32_t *perm = nullptr, *offs = nullptr;
    // wavefront chunks of whole segments for the gather-scatter kernel
    int64_t nchunks = 0, nover = 0;
    // [nchunks][64] copy of each lane (perm order), | kGsSegStart where it
    // starts a segment, -1 past the chunk's end
    int32_t *chunk_perm = nullptr;
    int32_t *over = nullptr;                          // segments longer than 64 copies
    double *D = nullptr;   // Dh [nq][nq] (row = point)
    float *D32 = nullptr;
    // interpolation from the next coarser level's nodes to this level's
    // points: J [nq][nq_coarse]; null on the coarsest level
    double *Jc = nullptr;
    float *Jc32 = nullptr;
    // per-operator preconditioner data
    double *Dinv = nullptr;
    float *Dinv32 = nullptr;
    double lmax = 0.0;
    // element extents along r, s, t [E][3] (host), for the Schwarz smoother
    std::vector<double> len;
    // overlapping Schwarz smoother (built on first use): extended points
    // ne = nq + 2 per direction, of which the n_ext = ne^3 - nq^3 outside the
    // element (enumerated by schwarz_ext_slot); sz_ix [E][n_ext] copy gathered
    // at each of them (-1 absent); FDM data sz_S [E][3][ne][ne] (row = point,
    // column = mode) and sz_lam [E][3][ne]; ASM lists: the sz_nrc copies that
    // receive extension values, sz_rc, with sz_off [nrc+1] / sz_src (indices
    // into the extension results [E][n_ext], ascending); weight sz_w [nL] =
    // mask / (subdomains containing the node)
    int sz_ne = 0, sz_next = 0;
    int64_t sz_nrc = 0;
    int32_t *sz_ix = nullptr;
    float *sz_S = nullptr, *sz_lam = nullptr;
    int32_t *sz_rc = nullptr, *sz_off = nullptr, *sz_src = nullptr;
    float *sz_w = nullptr;
    double sz_lmax = 0.0;  // lambda_max(M^{-1} A) estimate for the current key
    // the coarsest level's operator assembled on its free unique nodes (built
    // per (h1, h2) with the p-multigrid preconditioner): CSR cs_row [nf+1],
    // cs_col / cs_val [nnz], inverse diagonal cs_dinv and unit weights cs_one
    // [nf]; cs_uid [nL] the free node of each copy (-1 on Dirichlet copies),
    // cs_rep [nf] one copy of each node; cs_bu / cs_xu [kMaxRhs][nf] the
    // right-hand sides and solutions of the coarse solves on these nodes
    int64_t cs_nf = 0, cs_nnz = 0;
    int32_t *cs_row = nullptr, *cs_col = nullptr, *cs_uid = nullptr, *cs_rep = nullptr;
    double *cs_val = nullptr, *cs_dinv = nullptr, *cs_one = nullptr, *cs_bu = nullptr, *cs_xu = nullptr;
};

// Phase timers of a solve (sem_solve_opts.timers): a chain of events on the
// solver's stream, restarted after every host synchronisation; the interval
// that ends at event i is charged to phase ph[i] (-1: the chain's start).
enum SolvePhase { kPhaseAx = 0, kPhaseGs, kPhaseVec, kPhasePrec, kPhaseCoarse, kPhases };
struct PhaseClock {
    bool on = false;
    std::vector<hipEvent_t> ev;  // pool, created on first use
    std::vector<int> ph;
    int n = 0;                   // events recorded in the current chain
    double ms[kPhases] = {};
};

struct Workspace {
    int64_t nL = 0;
    int nv = 0;        // vectors per array (batched solves), grown on demand
    bool pmg = false;  // multigrid vectors allocated
    // FP64 outer vectors, [nv][nL]
    double *r = nullptr, *p = nullptr, *w = nullptr, *z = nullptr;
    double *aux = nullptr;  // adjoint right-hand side
    // reduction partials (vector v at + v * pst) and scalars (one per vector)
    double *partial = nullptr;     // vector-kernel partial sums
    int64_t pst = 0;
    double *partial_ax = nullptr;  // operator-kernel partial sums of (p, A_L p)
    int64_t pst_ax = 0;
    KrylovScalars *sc = nullptr;      // outer [kMaxRhs]
    KrylovScalars *sc_c = nullptr;    // coarse [kMaxRhs]
    KrylovScalars *host_sc = nullptr; // pinned mirror: outer, then coarse
    // multigrid per-level vectors [nv][nL of the level] (FP32 on smoother
    // levels, FP64 on the coarsest)
    void *mg_r[kMaxLevels] = {}, *mg_x[kMaxLevels] = {}, *mg_t[kMaxLevels] = {},
         *mg_d[kMaxLevels] = {}, *mg_s[kMaxLevels] = {};
    double *c_r = nullptr, *c_p = nullptr, *c_w = nullptr;  // coarse CG
    // projection of initial guesses: per right-hand-side slot, l A-orthonormal
    // vectors xt [L][nL] and bt = A xt [L][nL]; projected guess and remainder
    // right-hand side of the current solve [nv_proj][nL]
    struct Proj {
        double *xt = nullptr, *bt = nullptr;
        int l = 0;
    } proj[kMaxRhs];
    int proj_L = 0, proj_nv = 0;
    double proj_h1 = 0.0, proj_h2 = 0.0;
    double *proj_xb = nullptr, *proj_bp = nullptr;
    // Schwarz smoother: local solutions [nv][E][ne^3] of the largest smoothed
    // level and the combined sums [nv][nL] per smoothed level
    float *sz_U = nullptr;
    int64_t sz_U_len = 0;
    float *sz_acc[kMaxLevels] = {};
    int sz_nv = 0;
    // captured V-cycles, one per live right-hand-side set, each with a hash
    // of every pointer and value its kernels take; captured on `cap`
    struct VGraph {
        hipGraphExec_t exec = nullptr;
        uint32_t pack = 0;
        int n = 0;
        uint64_t sig = 0;
    } vg[8];
    int vg_next = 0;
    bool vg_broken = false;  // capture failed once: launch kernel by kernel
    hipStream_t cap = nullptr;
    PhaseClock clk;
};

struct PrecondKey {
    bool valid = false;
    double h1 = 0, h2 = 0;
    int precond = -1;
    int smoother = 0;
    int cheb_degree = 0, lanczos_steps = 0;
    double lo = 0, hi = 0;
};

}  // namespace semx

struct sem_handle_s {
    int device = 0;
    int n_levels = 0;
    semx::Level lv[semx::kMaxLevels];
    // level-0 coordinates [nL] each (kept for the advection metrics)
    double *cx = nullptr, *cy = nullptr, *cz = nullptr;
    // dealiased advection on the M-point Gauss rule: interpolation J and
    // derivative Jd = J Dh [M][nq], weights wq [M], metric factors
    // F [E][9][M^3] = rho~ |det X| dr_q/dx_d at index 3 q + d
    struct Advect {
        int M = 0;
        int variant = 0;  // SEM_ADVECT_2D or SEM_ADVECT_3D
        double *J = nullptr, *Jd = nullptr, *wq = nullptr, *F = nullptr;
    } adv;
    semx::Workspace ws;
    semx::PrecondKey key;
    uint64_t lanczos_seed = 0x5eed5eedULL;
};

namespace semx {

// ---- kernels (launchers) ------------------------------------------------
// Element operator w = h1 A_L(k) u + h2 B u on a level; optional per-block
// partial sums of u.w written to `partial` (one per block, count returned via
// *nblocks).  T = double or float.
// `skip` (nullable): device flag; when nonzero at launch time the kernel does
// nothing (used to turn the tail of an enqueued iteration batch into no-ops).
template <typename T>
int launch_ax(const Level &L, const T *G, const T *B, const T *D, const T *u, T *w, double h1,
              double h2, const T *k, double *partial, int64_t *nblocks, hipStream_t s,
              const int *skip = nullptr);

template <typename T>
int launch_gs(const Level &L, T *v, hipStream_t s, const int *skip = nullptr);
// one field, any reduction SEM_GS_ADD / MUL / MIN / MAX (SEM_EINVAL otherwise)
template <typename T>
int launch_gs_op(const Level &L, T *v, int op, hipStream_t s);

// Batched forms: the vectors of `vs` (vector v at u + v * ldu, w + v * ldw),
// one launch for the whole batch; the element operator reads each element's
// geometric factors once for all vectors.  skip (nullable) + v * skip_stride
// is vector v's flag: vectors flagged at launch time are left untouched.
// Operator partial sums of u_v.w_v go to partial[v * pst + block].
template <typename T>
int launch_ax_multi(const Level &L, const T *G, const T *B, const T *D, const T *u, int64_t ldu, T *w,
                    int64_t ldw, const VSet &vs, double h1, double h2, const T *k, double *partial,
                    int64_t pst, int64_t *nblocks, hipStream_t s, const int *skip, int skip_stride);

template <typename T>
int launch_gs_multi(const Level &L, T *v, int64_t ld, const VSet &vs, hipStream_t s,
                    const int *skip, int skip_stride);

int launch_geometry(const Level &L, const double *x, const double *y, const double *z,
                    double *G, double *B, int *bad, hipStream_t s);

template <typename T>
int launch_diag(const Level &L, const double *k, double h1, double h2, double *d, hipStream_t s);

// look up the allocation-free solve's scratch address on device dev (current);
// once per device, from sem_setup
int noalloc_attach(int dev);

int launch_grad_k(const Level &L, const double *u, const double *lam, double h1, double *gk,
                  hipStream_t s);

// elementwise tensor-product interpolation out = (J (x) J (x) J) in, J [nt][ns]
template <typename T>
int launch_interp(int64_t E, int ns, int nt, const T *J, const T *in, T *out, bool transpose,
                  hipStream_t s);

// fused p-multigrid transfers between smoother level F (nq <= 8) and the next
// coarser level C for a batch of vectors (fine arrays [nv][F.nL], coarse
// [nv][C.nL]): out = mask_C (J^T)^3 [W_F (r - t)] and x += J^3 in
template <typename TO>
int launch_restrict_resid(const Level &F, const Level &C, const float *r, const float *t, TO *out,
                          const VSet &vs, hipStream_t s);
template <typename TI>
int launch_prolong_add(const Level &F, const Level &C, const TI *in, float *x, const VSet &vs,
                       hipStream_t s);

// Extended point (a, b, c) outside the element (some coordinate 0 or ne-1):
// its slot in [0, n_ext).  Columns (a, b) on the border of the ne x ne square
// hold ne slots each; inner columns hold their two end points.
__host__ __device__ inline int schwarz_ext_slot(int ne, int a, int b, int c)
{
    int col;
    if (b == 0) col = a;
    else if (b == ne - 1) col = ne + a;
    else if (a == 0) col = 2 * ne + (b - 1);
    else if (a == ne - 1) col = 2 * ne + (ne - 2) + (b - 1);
    else return (4 * ne - 4) * ne + ((b - 1) * (ne - 2) + (a - 1)) * 2 + (c == ne - 1 ? 1 : 0);
    return col * ne + c;
}

// overlapping Schwarz smoother of a level (schwarz.hip): build_schwarz fills
// the sz_* fields; launch_schwarz computes the local FDM solutions of
// res = r - t (t nullable: res = r) for the batch vs: each element's own
// points go to acc [nv][nL], and for ASM the extension points to U
// [nv][E][n_ext], then added into the receiving copies of acc; the caller
// applies QQ^T and the weight (sz_w for ASM, W32 for RAS).
int build_schwarz(Level &L, hipStream_t s);
void free_schwarz(Level &L);
void free_coarse_csr(Level &L);
void free_advect(sem_handle h);
int launch_schwarz(const Level &L, bool ras, const float *r, const float *t, float *U, float *acc,
                   const VSet &vs, double h1, double h2, hipStream_t s);

// setup helpers
int build_maps(Level &L, const int64_t *gid_dev, const uint8_t *dir_dev, const double *x,
               const double *y, const double *z, int *bad_dev, hipStream_t s);
int build_gs_chunks(Level &L, hipStream_t s);

int host_gll(int N, double *xi, double *rho, double *D);
void host_interp(int ns, const double *xs, int nt, const double *xt, double *J);
int host_gauss(int M, double *x, double *w);

// solver entry (solve.hip)
int pcg_solve(sem_handle h, int nv, const double *b, double *x, int64_t ld,
              const sem_solve_opts *o, sem_solve_stats *st, hipStream_t s);
void free_workspace(sem_handle h);

}  // namespace semx
