/*
 * sem.h -- C ABI of libsem: the matrix-free spectral-element (SEM)
 * Poisson/Helmholtz operator on hexahedral Gauss--Lobatto--Legendre (GLL)
 * elements, its direct-stiffness summation QQ^T, and preconditioned CG around
 * them, on one AMD Instinct MI355X (gfx950).
 *
 * Notation follows the NekRS paper (Fischer et al., "NekRS, a GPU-Accelerated
 * Spectral Element Navier-Stokes Solver"), Sec. 2.3 and Sec. 3.2-3.4.
 *
 * Layout.  A field is an "L-vector": one value per local copy, element-major,
 * E blocks of (N+1)^3 values, each block indexed [k][j][i] with i fastest,
 * idx = i + (N+1) j + (N+1)^2 k + (N+1)^3 e (Sec. 2.3, eq. (uijk) with
 * D_1 = I (x) I (x) Dh acting on i).  Device arrays hold FP64 unless stated.
 *
 * Ownership.  The caller owns every array it passes.  Host arrays given to
 * sem_setup are copied and may be freed afterwards.  The handle owns the
 * geometric factors, gather-scatter maps, weights and solver workspaces.
 * sem_ax and sem_gs allocate nothing; sem_pcg_solve allocates its workspace
 * on first use and keeps it in the handle.  A handle serves one call at a
 * time (it is not re-entrant); distinct handles are independent.
 *
 * Streams.  Every device call takes a hipStream_t (as void*, NULL = the null
 * stream) and enqueues its kernels on it without synchronising, except
 * sem_setup and sem_pcg_solve, which synchronise that stream before they
 * return.  Pointers passed to a call must stay valid until the stream reaches
 * it.
 *
 * Errors.  Every function returns SEM_OK (0) or a negative code below.
 * sem_strerror() names a code; sem_last_error() returns a thread-local text
 * with the detail of the last failure in the calling thread.
 */
#ifndef SEM_H_
#define SEM_H_

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define SEM_API __attribute__((visibility("default")))
#else
#define SEM_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sem_handle_s *sem_handle;

enum sem_status {
    SEM_OK = 0,
    SEM_EINVAL = -1,      /* bad argument: null pointer, size, order, option */
    SEM_ENOMEM = -2,      /* device or host allocation failed */
    SEM_EHIP = -3,        /* a HIP runtime call failed */
    SEM_ENOCONV = -4,     /* solver hit maxit; x holds the last iterate */
    SEM_EBREAKDOWN = -5,  /* p^T A p <= 0 or a NaN in the iteration */
    SEM_EMESH = -6        /* Jacobian <= 0, or copies of one global pointer
                             disagree in coordinates or Dirichlet flag */
};

enum sem_dtype { SEM_F64 = 0, SEM_F32 = 1 };

/* Largest number of right-hand sides sem_pcg_solve_multi takes in one call
 * (and the batch size in which sem_ax_multi / sem_gs_multi process theirs). */
#define SEM_MAX_RHS 4
/* Largest projection space (earlier solutions kept per right-hand-side slot). */
#define SEM_MAX_PROJ 16
enum sem_precond { SEM_PRECOND_JACOBI = 0, SEM_PRECOND_PMG = 1 };
/* p-multigrid smoother (Sec. 3.4): Chebyshev-accelerated Jacobi, or
 * Chebyshev-accelerated overlapping Schwarz with fast-diagonalisation local
 * solves, combined additively (ASM) or restricted (RAS). */
enum sem_smoother { SEM_SMOOTH_JACOBI = 0, SEM_SMOOTH_ASM = 1, SEM_SMOOTH_RAS = 2 };

/*
 * Mesh description (host arrays, E*(N+1)^3 entries each, L-vector layout).
 *   x, y, z    node coordinates x^e_ijk of the isoparametric map
 *              (Sec. 2.3, eq. (xijk)); copies of one node must agree.
 *   gid        global pointer of each copy, >= 0 (the gs_setup contract of
 *              Sec. 3.2): copies with equal nonzero pointers are one global
 *              node; 0 marks a singleton (e.g. element-interior points).
 *   dirichlet  1 on copies of nodes with homogeneous Dirichlet data, else 0;
 *              NULL means none (pure Neumann).  This is the restriction R of
 *              the footnote on A = R Abar R^T in Sec. 2.3.
 */
typedef struct {
    int N;                     /* polynomial order, 1 <= N <= 15 */
    int64_t E;                 /* number of elements, E*(N+1)^3 < 2^31 */
    const double *x, *y, *z;
    const int64_t *gid;
    const uint8_t *dirichlet;
} sem_mesh;

/*
 * Setup options.  pmg != 0 builds the p-multigrid hierarchy of Sec. 3.4
 * (orders levels[0] = N > levels[1] > ... >= 1, at most 4 levels); coarse
 * levels are rediscretised on coordinates interpolated from the fine mesh.
 * NULL opts = no multigrid.
 */
typedef struct {
    int pmg;
    int n_levels;
    int levels[4];
} sem_setup_opts;

/*
 * Build a handle: GLL nodes, weights and Dh (Sec. 2.3, eq. (dh)); geometric
 * factors G (six, eq. (gij)) and mass B = diag(rho J) (eq. (vBu)); gather-
 * scatter maps (shared copies sorted by (global pointer, local index));
 * multiplicity and counting weight W = 1/multiplicity (0 on Dirichlet copies).
 * Returns SEM_EINVAL for a bad order, size or pointer, SEM_EMESH for a
 * nonpositive Jacobian or inconsistent copies.  Synchronises `stream`.
 */
SEM_API int sem_setup(const sem_mesh *mesh, const sem_setup_opts *opts, void *stream, sem_handle *out);

/* Release every device and host resource of the handle (NULL is a no-op). */
SEM_API int sem_free(sem_handle h);

/*
 * Unassembled operator, Sec. 2.3 eq. (Ae):
 *   w_L = h1 A_L(k) u_L + h2 B_L u_L,
 *   A^e(k) = [D1;D2;D3]^T (k o G^e) [D1;D2;D3],
 * per element, no summation across elements (that is sem_gs).
 * u, w: device L-vectors (distinct, not overlapping).  k: device L-vector of
 * pointwise coefficients or NULL for k = 1.  FP64.
 */
SEM_API int sem_ax(sem_handle h, const double *u, double *w, double h1, double h2, const double *k,
           void *stream);

/* gather-scatter reductions (the associative, commutative operations of
 * gs_op, Sec. 3.2) */
enum sem_gs_op { SEM_GS_ADD = 0, SEM_GS_MUL = 1, SEM_GS_MIN = 2, SEM_GS_MAX = 3 };

/*
 * Gather-scatter in place (Sec. 3.2, gs_op(gsh, w_L, op)).  With op =
 * SEM_GS_ADD it is the direct-stiffness summation v <- QQ^T v (Sec. 2.3 eq.
 * (dssum) and the Q / Q^T discussion): every copy of a global node receives
 * the sum over all its copies, formed from 0 by adding the copies in
 * ascending local index order, so the result is deterministic.  SEM_GS_MUL,
 * SEM_GS_MIN and SEM_GS_MAX give every copy the product, minimum (fmin) or
 * maximum (fmax) over the node's copies, formed from the first copy in the
 * same order.  Copies with pointer 0 or a unique pointer are unchanged.
 * v: device L-vector, FP64.  Another op: SEM_EINVAL.
 */
SEM_API int sem_gs(sem_handle h, double *v, int op, void *stream);

/*
 * Several fields through the same operator, as the three velocity components
 * of a vector Helmholtz solve (Sec. 3.3: for velocity-oriented work the
 * geometric factors of an element serve every component):
 *   w_r = h1 A_L u_r + h2 B_L u_r for
 * r = 0 .. nrhs-1, with u_r = u + r*ld and w_r = w + r*ld (device L-vectors,
 * FP64, ld >= n_local when nrhs > 1, u and w not overlapping).  The geometric factors of an
 * element are read once per batch of up to SEM_MAX_RHS fields.  Each w_r is
 * bit-identical to sem_ax(u_r) with k = NULL.  nrhs >= 1.
 */
SEM_API int sem_ax_multi(sem_handle h, int nrhs, const double *u, double *w, int64_t ld, double h1,
                         double h2, void *stream);

/* v_r <- QQ^T v_r for v_r = v + r*ld, r = 0 .. nrhs-1 (as sem_gs, bit-identical
 * to it per field; the maps are read once per batch of SEM_MAX_RHS fields). */
SEM_API int sem_gs_multi(sem_handle h, int nrhs, double *v, int64_t ld, void *stream);

/*
 * The same two operations at multigrid level `level` (0 = fine) in FP64 or
 * FP32; u, w, v are level-sized device L-vectors of that dtype.  FP32 is the
 * smoother precision of Sec. 3.4 (FP32 data and accumulation).
 */
SEM_API int sem_ax_level(sem_handle h, int level, int dtype, const void *u, void *w, double h1, double h2,
                 void *stream);
SEM_API int sem_gs_level(sem_handle h, int level, int dtype, void *v, void *stream);

/* Batched forms at a level, as sem_ax_multi / sem_gs_multi (fields at
 * base + r*ld, ld >= the level's n_local when nrhs > 1), in FP64 or FP32. */
SEM_API int sem_ax_level_multi(sem_handle h, int level, int dtype, int nrhs, const void *u, void *w,
                               int64_t ld, double h1, double h2, void *stream);
SEM_API int sem_gs_level_multi(sem_handle h, int level, int dtype, int nrhs, void *v, int64_t ld,
                               void *stream);

typedef struct {
    double h1, h2;       /* operator h1 A(k) + h2 B (h1 = 1/Re, h2 = beta0/dt) */
    const double *k;     /* device L-vector coefficient, NULL = 1 (Jacobi only) */
    double tol;          /* stop when ||r||_W <= tol ||b||_W */
    int maxit;
    int precond;         /* SEM_PRECOND_JACOBI or SEM_PRECOND_PMG */
    int check_every;     /* iterations between host convergence checks, >= 1 */
    int cheb_degree;     /* Chebyshev-Jacobi degree per smoothing (PMG), e.g. 2 */
    int lanczos_steps;   /* steps for the lambda_max estimate (PMG), e.g. 20 */
    double cheb_lo, cheb_hi;  /* smoothing interval as fractions of lambda_max */
    double coarse_tol;   /* coarsest-level Jacobi-PCG relative tolerance */
    int coarse_maxit;
    int zero_guess;      /* 1: ignore x on entry and start from 0 */
    int proj_dim;        /* 0: off; L in 1..SEM_MAX_PROJ: initial guess projected onto
                            up to L earlier solutions (see sem_proj_reset); x on entry
                            is then ignored; constant coefficients only (k = NULL) */
    int smoother;        /* PMG smoother, enum sem_smoother.  Schwarz: subdomain = the
                            element plus one node layer of its neighbours ((N+3)^3
                            points), local operator = the separable operator of that box
                            from the element's mean extents, solved by fast
                            diagonalisation in FP32; ASM weights the overlapping sum by
                            1 / (subdomains containing the node); needs N >= 2 on every
                            smoothed level and a conforming hex mesh; the Chebyshev
                            interval uses the power-method lambda_max of M^{-1} A */
    int use_graphs;      /* PMG: 1 replays each V-cycle of the outer FCG from a HIP graph
                            captured once per set of unconverged right-hand sides and
                            state (recaptured when a pointer or value its kernels take
                            changes); the iterates equal those of 0 (kernels launched
                            one by one, the default) bit for bit.  No effect with
                            Jacobi. */
    int timers;          /* 1: time the solver's phases with HIP events on `stream` (fills
                            the ms_ax .. ms_coarse fields of the stats); adds event records
                            between kernels and no host synchronisation.  0: off (fields 0) */
} sem_solve_opts;

typedef struct {
    int iters;             /* outer iterations taken */
    int converged;         /* 1 if ||r||_W <= tol ||b||_W was reached */
    double rel_res;        /* recursive ||r||_W / ||b||_W at exit */
    double true_rel_res;   /* ||b - A x||_W / ||b||_W recomputed in FP64 */
    double ms_solve;       /* wall time of the iteration (host clock) */
    double ms_setup;       /* preconditioner setup done inside this call */
    int coarse_iters;      /* total coarsest-level iterations (PMG) */
    int proj_vectors;      /* earlier solutions the initial guess was projected onto */
    double proj_rel_res;   /* ||b - A xbar||_W / ||b||_W of the projected guess xbar */
    /* Phase times with opts->timers = 1 (else 0): device time between
     * consecutive phase boundaries on the stream, launch gaps included, summed
     * over the iteration (for sem_pcg_solve_multi the phases serve every
     * system at once and each record holds the same totals):
     *   ms_ax     element operator applications of the outer iteration
     *   ms_gs     their gather-scatter QQ^T
     *   ms_vec    vector updates, inner products and convergence decisions
     *             of the outer iteration (with Jacobi, the preconditioner too)
     *   ms_prec   p-multigrid V-cycle without its coarsest-level solve
     *             (smoothing, transfers, level operators)
     *   ms_coarse coarsest-level Jacobi-PCG inside the V-cycles */
    double ms_ax, ms_gs, ms_vec, ms_prec, ms_coarse;
} sem_solve_stats;

/* Fill opts with defaults: h1 = 1, h2 = 0, k = NULL, tol = 1e-8, maxit = 1000,
 * Jacobi, check_every = 8, cheb_degree = 2, lanczos_steps = 20,
 * interval [0.1, 1.1] lambda_max, coarse_tol = 1e-2, coarse_maxit = 20,
 * zero_guess = 1, proj_dim = 0, smoother = SEM_SMOOTH_JACOBI, use_graphs = 0, timers = 0. */
SEM_API void sem_solve_opts_default(sem_solve_opts *opts);

/*
 * Solve R (h1 A(k) + h2 B) R^T x = R b (Sec. 2.3, eq. (aip) with the
 * restriction footnote), on replicated L-vectors:
 *   b  device, assembled and replicated: b = QQ^T(B_L f_L) for a load f; its
 *      Dirichlet copies are ignored.
 *   x  device, in: initial guess (unless opts->zero_guess), out: solution,
 *      replicated, zero on Dirichlet copies.
 * Jacobi: PCG with the inverse assembled diagonal.  PMG: flexible CG
 * preconditioned by one p-multigrid V-cycle (Sec. 3.4): Chebyshev-accelerated
 * Jacobi smoothing in FP32 on every level above the coarsest, FP64 Jacobi-PCG
 * on the coarsest; outer iteration, inner products and coarse solve in FP64.
 * Returns SEM_ENOCONV (x = last iterate, stats filled) when maxit is reached,
 * SEM_EBREAKDOWN on a nonpositive curvature or NaN.  stats may be NULL.
 * Synchronises `stream`.
 */
SEM_API int sem_pcg_solve(sem_handle h, const double *b, double *x, const sem_solve_opts *opts,
                  sem_solve_stats *stats, void *stream);

/*
 * One application of the p-multigrid preconditioner of sem_pcg_solve (Sec. 3.4):
 * z = M^{-1} r, the V-cycle the flexible CG applies to its residual, with the
 * smoothing, transfers and coarse solve set by opts (h1, h2, smoother,
 * cheb_degree, lanczos_steps, cheb_lo / cheb_hi, coarse_tol, coarse_maxit,
 * use_graphs; precond is taken as SEM_PRECOND_PMG, k must be NULL).
 *   r  device L-vector, FP64, replicated; its Dirichlet copies are ignored.
 *   z  device L-vector, FP64, out: the V-cycle output (FP32 arithmetic inside
 *      the smoothed levels), zero on Dirichlet copies.
 * The preconditioner data (inverse diagonals, lambda_max estimates, Schwarz
 * subdomains) are built on the first call for given coefficients and cached
 * in the handle, as for sem_pcg_solve.  Needs a handle built with levels.
 */
SEM_API int sem_pmg_apply(sem_handle h, const double *r, double *z, const sem_solve_opts *opts,
                          void *stream);

/*
 * Allocation-free form of sem_pcg_solve, for callers that cannot allocate
 * device memory (code under HIP stream capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same FP64 Jacobi-PCG, one right-hand
 * side, with every buffer beyond b and x (Krylov scalars, reduction partials,
 * the inverse diagonal, the vectors r, p, w) in a static device array of
 * SEM_NOALLOC_SCRATCH_MIB MiB per GPU that the library holds from its first
 * use on that GPU until the process ends.  b, x, opts, stats and the stream as
 * for sem_pcg_solve; the iterates, solution and stats equal sem_pcg_solve's
 * with the Jacobi preconditioner.
 *   Limits: opts->precond = SEM_PRECOND_JACOBI, proj_dim = 0, timers = 0,
 *   use_graphs = 0, and
 *   n_local <= SEM_NOALLOC_MAX_LOCAL, else SEM_EINVAL with nothing enqueued;
 *   the current device must be the handle's.
 *   Calls no hipMalloc/hipFree (nor any allocating library routine); the
 *   inverse diagonal is recomputed each call (its cost is one operator-sized
 *   pass).  Every call on a GPU shares that GPU's scratch, so calls that
 *   overlap on one GPU (several host threads, or streams that run concurrently)
 *   race and give undefined results; serialise them.  Synchronises `stream`.
 */
#define SEM_NOALLOC_SCRATCH_MIB 96
#define SEM_NOALLOC_MAX_LOCAL 3142880
SEM_API int sem_pcg_solve_noalloc(sem_handle h, const double *b, double *x, const sem_solve_opts *opts,
                                  sem_solve_stats *stats, void *stream);

/*
 * Projection of initial guesses for successive right-hand sides (the pressure
 * initial guesses of Sec. 3.4 / Sec. 4, after Fischer, CMAME 163, 1998).  With
 * opts->proj_dim = L > 0 every solve keeps, per right-hand-side slot (slot 0
 * for sem_pcg_solve, slot r for row r of sem_pcg_solve_multi), up to L earlier
 * solution increments xt_i, orthonormal in the A inner product, and A xt_i:
 *   xbar = sum_i (xt_i, b)_W xt_i  (the A-norm best guess from the space),
 *   solve A dx = b - A xbar from zero to ||r||_W <= tol ||b||_W,  x = xbar + dx,
 * then dx, A-orthogonalised and A-normalised, joins the space, or the space
 * restarts from x / ||x||_A once it holds L vectors.  Spaces belong to the
 * handle's operator (h1, h2) and are cleared when h1, h2 or L change, or by
 * this call (all slots).  Device memory: 2 L n_local doubles per slot used.
 */
SEM_API int sem_proj_reset(sem_handle h);

/*
 * One application of the overlapping Schwarz smoother of a level (Sec. 3.4;
 * the construction is described at sem_solve_opts.smoother), for tests and
 * inspection:  z = M^{-1} r with M^{-1} = weight o QQ^T(sum over subdomains of
 * the FDM local solutions of r), FP32 device L-vectors of the level (r
 * replicated, zero on Dirichlet copies; z may not alias r).  smoother =
 * SEM_SMOOTH_ASM or SEM_SMOOTH_RAS; the level needs N >= 2 and FP32 data
 * (every level above the coarsest).  Builds the level's Schwarz data on first
 * use (host work, synchronises `stream` then).
 */
SEM_API int sem_smoother_apply(sem_handle h, int level, int smoother, double h1, double h2,
                               const float *r, float *z, void *stream);

/*
 * The host part of the Schwarz setup for one level, on host arrays (no
 * device work; for inspection and tests).  In: order N (>= 2), E elements,
 * gid and dirichlet per copy (as in sem_mesh; dirichlet may be NULL), len
 * [E][3] element extents along r, s, t.  Out (each may be NULL; ne = N+3):
 *   ix     [E][ne^3]        copy gathered at extended point (a, b, c) of each
 *                           element, a fastest; -1 when absent
 *   S, lam [E][3][ne][ne], [E][3][ne]  FDM modes (row = point) and eigenvalues
 *                           per direction r, s, t (padded modes: zero columns, 1)
 *   cover  [n_local]        extended points (all elements) gathered from each copy
 *   weight [n_local]        ASM weight: 0 on Dirichlet copies, else 1 / (number
 *                           of subdomains containing the node)
 * Returns SEM_EMESH when a face does not conform.
 */
SEM_API int sem_schwarz_setup_host(int N, int64_t E, const int64_t *gid, const uint8_t *dirichlet,
                                   const double *len, int32_t *ix, float *S, float *lam,
                                   int32_t *cover, float *weight);

/*
 * nrhs independent solves with one operator, advanced in lockstep so that
 * every operator application and gather-scatter serves all unconverged
 * systems at once (b_r = b + r*ld, x_r = x + r*ld, 1 <= nrhs <= SEM_MAX_RHS,
 * ld >= n_local): the velocity Helmholtz solves of a time step (Sec. 2.2
 * splitting; vector operator reuse of Sec. 3.3).
 * Each system keeps its own Krylov scalars and stops at its own tolerance;
 * with opts->k set the operator is applied field by field.  stats, if not
 * NULL, holds nrhs records.  Returns SEM_OK when every system converged,
 * else SEM_EBREAKDOWN if any broke down, else SEM_ENOCONV.  Synchronises
 * `stream`.
 */
SEM_API int sem_pcg_solve_multi(sem_handle h, int nrhs, const double *b, double *x, int64_t ld,
                                const sem_solve_opts *opts, sem_solve_stats *stats, void *stream);

/*
 * Gradient of a loss with respect to the per-copy coefficient k of
 * A(k) = Q^T A_L(k) Q, given the forward solution u and adjoint lam
 * (A lam = dL/du):
 *   gk[e,q] = -h1 sum_{m,m'} (D_m lam)_q G_mm'[q] (D_m' u)_q
 * (reference-space gradients as in eqs. (gradr)-(gradt)).  Device L-vectors.
 */
SEM_API int sem_grad_k(sem_handle h, const double *u, const double *lam, double h1, double *gk,
               void *stream);

/*
 * Load vector of the weak form (Sec. 2.3: b_i = (phi_i, f) by GLL quadrature,
 * eq. (vBu)), assembled and restricted:  b = R QQ^T (B_L o f_L), i.e. Dirichlet
 * copies of b are zero.  f, b: device L-vectors (may alias).
 */
SEM_API int sem_rhs(sem_handle h, const double *f, double *b, void *stream);

/*
 * Hand-written adjoint of the solve u = A(k)^{-1} R QQ^T(B f) for a loss L(u)
 * with g = dL/du_L (per copy):
 *   lam    = A(k)^{-1} R QQ^T g      (one more solve; A is symmetric)
 *   grad_f = B_L o lam              (dL/df_L per copy)
 *   grad_k = -h1 (D lam)^T G (D u)  (dL/dk_L per copy, as sem_grad_k; NULL to skip)
 * u is the forward solution (replicated L-vector).  opts gives h1, h2, k and
 * the tolerance of the adjoint solve (Jacobi-preconditioned; PMG if k is NULL
 * and the handle has levels).  lam is output storage; grad_f may be NULL.
 * Returns the adjoint solve's status.  Synchronises `stream`.
 */
SEM_API int sem_adjoint(sem_handle h, const double *u, const double *g, const sem_solve_opts *opts,
                        double *lam, double *grad_f, double *grad_k, sem_solve_stats *stats,
                        void *stream);

/* Sizes of a level (0 = fine). */
typedef struct {
    int N;
    int64_t E;
    int64_t n_local;         /* E (N+1)^3 */
    int64_t n_unique;        /* distinct global nodes (pointer-0 copies count once each) */
    int64_t n_shared_copies; /* copies whose global node has 2+ copies */
    int64_t n_segments;      /* global nodes with 2+ copies */
    int n_levels;            /* levels in the handle */
} sem_info_t;
SEM_API int sem_info(sem_handle h, int level, sem_info_t *info);

/*
 * Copies of handle data into caller device buffers (for inspection and
 * tests): perm [n_shared_copies] and offs [n_segments+1] (int32) of the sorted
 * maps; G [6][n_local] in the order G11, G12, G13, G22, G23, G33 and B
 * [n_local]; W [n_local] counting weight; gid [n_local] (int64) global
 * pointers of the level.  Any output may be NULL.
 */
SEM_API int sem_get_maps(sem_handle h, int level, int32_t *perm, int32_t *offs, void *stream);
SEM_API int sem_get_geometry(sem_handle h, int level, double *G, double *B, void *stream);
SEM_API int sem_get_weights(sem_handle h, int level, double *W, int64_t *gid, void *stream);

/* GLL nodes xi[N+1], weights rho[N+1] and Dh[(N+1)^2] (row = point) of the
 * library, on the host (any output may be NULL).  No device work. */
SEM_API int sem_gll(int N, double *xi, double *rho, double *D);

/*
 * Dealiased advection (the advection term u . grad w of the EXT formulation
 * and of the characteristics subproblem, Sec. 2.1 eqs. (stdadv), (hyp); its
 * degree-3N integrand needs a quadrature finer than GLL, Sec. 2.3; the
 * advection kernels of Sec. 3.3).  Level 0 only, FP64.  The weak form
 * (v, c . grad w) on each element is evaluated on the M-point Gauss-Legendre
 * rule per direction (M^3 points):
 *   ct_q  = rho~ |det X| (dr_q/dx . J3 c),  q = r, s, t   (contravariant
 *           weighted velocity at the Gauss points; X = dx/dr of the
 *           interpolated element map, rho~ the products of Gauss weights)
 *   out_e = J3^T ( sum_q ct_q  d_q (J3 w_e) )
 * with J3 = J (x) J (x) J the interpolation from the GLL points to the Gauss
 * points and d_q the derivative of the interpolant along r_q, so that
 * v_L . out_L = sum over elements and Gauss points of rho~ |det X| v c.grad w,
 * exact for polynomial integrands of degree <= 2M - 1 per variable.
 *
 * sem_advect_setup: builds J, Jd and the metric factors for the rule
 *   (M = 0: the smallest rule exact for degree 3N, M = ceil((3N+1)/2)); M must
 *   be N+1..16 and, for the compiled kernels, one of the two rules
 *   ceil((3N+1)/2) or ceil((3N+1)/2) + 1, with N <= 7; *M_used (nullable)
 *   receives M.  variant picks the element kernel (the 2D and 3D thread blocks
 *   of Sec. 3.3, enum sem_advect_variant); both give the same result up to
 *   rounding order.  Device memory 72 M^3 bytes per element (freed by sem_free or
 *   a new setup).  Synchronises `stream`.  SEM_EMESH if det X <= 0 at a Gauss
 *   point.
 * sem_advect_velocity: ct [E][3][M^3] (point index a + M b + M^2 c, a along r)
 *   from the velocity c (three level-0 L-vectors at c + d * ldc, d = x, y, z;
 *   ldc >= n_local).  ct is caller-owned device memory of 3 E M^3 doubles and
 *   may be reused for any number of advected fields.
 * sem_advect: out (nf L-vectors at out + f * ldo) = the local (unassembled)
 *   advection of the nf fields at w + f * ldw by ct; 0 <= nf <= SEM_MAX_RHS
 *   (nf = 0 does nothing); ldw, ldo >= n_local when nf > 1; out may not alias
 *   w or ct.  Apply sem_gs for the assembled form and the inverse assembled
 *   mass for the strong form of the hyperbolic substep.
 * All three are asynchronous on `stream` except the setup; errors:
 *   SEM_EINVAL (null handle or pointer, setup missing, unsupported M or nf).
 */
enum sem_advect_variant {
    SEM_ADVECT_AUTO = 0,  /* the faster of the two for (N, M) as measured on MI355X: the 2D
                             variant at every compiled pair */
    SEM_ADVECT_2D = 1,    /* thread per Gauss column, register arrays along the third index */
    SEM_ADVECT_3D = 2     /* thread per Gauss point (M^3 <= 1024, so M <= 10) */
};
SEM_API int sem_advect_setup(sem_handle h, int M, int variant, int *M_used, void *stream);
SEM_API int sem_advect_velocity(sem_handle h, const double *c, int64_t ldc, double *ct, void *stream);
SEM_API int sem_advect(sem_handle h, const double *ct, int nf, const double *w, int64_t ldw,
                       double *out, int64_t ldo, void *stream);

SEM_API const char *sem_strerror(int code);
SEM_API const char *sem_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SEM_H_ */
