"""Oracle iterations: Jacobi-PCG, Chebyshev-Jacobi smoothing, the p-multigrid
V-cycle, flexible CG and the adjoint of the variable-coefficient solve.

TEST INFRASTRUCTURE (see the package docstring).  Plain FP64 numpy over
L-vectors; the operator, gather-scatter and diagonal come from the C oracle.

Conventions (NekRS paper, Sec. 2.3): the assembled operator acting on a
replicated L-vector is  A u = R Qbar^T A_L Q R^T u, realised as
mask * QQ^T(A_L(mask * u)) where mask zeroes Dirichlet copies (the footnote
on the Neumann operator and the restriction R).  Inner products over unique
free degrees of freedom are L-space sums weighted by the counting weight
W = 1/multiplicity, zero on Dirichlet copies (Sec. 3.4, counting weight).
"""
from __future__ import annotations

import math

import numpy as np

from . import ax, diag, dhat, geometry, gll, grad_k, interp_lvec, interp_matrix, multiplicity, qqt


class Level:
    """Discrete operator h1 A(k) + h2 B of one polynomial order on one mesh."""

    def __init__(self, N, x, y, z, gid, dirichlet, h1=1.0, h2=0.0, k=None):
        self.N = N
        self.xi, self.rho = gll(N)
        self.D = dhat(N, self.xi)
        self.G, self.B, self.J = geometry(N, x, y, z, self.D, self.rho)
        self.gid = np.ascontiguousarray(gid, dtype=np.int64).reshape(-1)
        self.mask = 1.0 - np.asarray(dirichlet, dtype=np.float64).reshape(-1)
        self.mult = multiplicity(self.gid).astype(np.float64)
        self.W = self.mask / self.mult
        self.h1, self.h2 = h1, h2
        self.k = None if k is None else np.asarray(k, dtype=np.float64).reshape(-1)
        d = qqt(self.gid, diag(N, self.D, self.G, h1, h2, self.B, self.k))
        self.Dinv = np.where(self.mask > 0, 1.0 / np.where(d != 0, d, 1.0), 0.0)
        self.Bbar = qqt(self.gid, self.B)

    @property
    def n_local(self):
        return self.gid.size

    def ax_local(self, u):
        """Unassembled h1 A_L(k) u + h2 B_L u."""
        return ax(self.N, self.D, self.G, u, self.h1, self.h2, self.B, self.k)

    def apply(self, u):
        """Assembled, restricted operator on a replicated L-vector."""
        return self.mask * qqt(self.gid, self.ax_local(self.mask * u))

    def apply_neumann(self, u):
        """Neumann operator QQ^T A_L u (no restriction)."""
        return qqt(self.gid, self.ax_local(u))

    def dot(self, a, b):
        return float(np.sum(self.W * a * b))

    def norm(self, a):
        return math.sqrt(max(self.dot(a, a), 0.0))

    def rhs(self, f):
        """b = mask * QQ^T(B_L f_L): the discrete (phi_i, f) (Sec. 2.3, b_i)."""
        return self.mask * qqt(self.gid, self.B * np.asarray(f, dtype=np.float64).reshape(-1))


def pcg_jacobi(lv: Level, b, x0=None, tol=1e-10, maxit=10000):
    """Jacobi-preconditioned CG (Sec. 2.3 cost discussion; Saad, Iterative
    Methods for Sparse Linear Systems, Alg. 9.1) on the restricted system.
    Stops when ||r||_W <= tol ||b||_W.  Returns (x, iters, rel_res_history)."""
    b = lv.mask * np.asarray(b, dtype=np.float64).reshape(-1)
    x = np.zeros_like(b) if x0 is None else lv.mask * np.array(x0, dtype=np.float64).reshape(-1)
    r = b - lv.apply(x)
    bn = lv.norm(b)
    if bn == 0.0:
        return x, 0, [0.0]
    hist = [lv.norm(r) / bn]
    z = lv.Dinv * r
    p = z.copy()
    rz = lv.dot(r, z)
    it = 0
    while it < maxit and hist[-1] > tol:
        w = lv.apply(p)
        alpha = rz / lv.dot(p, w)
        x += alpha * p
        r -= alpha * w
        it += 1
        hist.append(lv.norm(r) / bn)
        if hist[-1] <= tol:
            break
        z = lv.Dinv * r
        rz_new = lv.dot(r, z)
        beta = rz_new / rz
        rz = rz_new
        p = z + beta * p
    return x, it, hist


def splitmix64_uniform(keys, seed: int):
    """Counter-based uniform[-1, 1) numbers: SplitMix64 (Steele, Lea & Flood,
    "Fast splittable pseudorandom number generators", OOPSLA 2014) applied to
    seed + key * golden-gamma, top 53 bits scaled to [0, 1)."""
    k = np.asarray(keys, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (k + np.uint64(1)) * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    u = (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return 2.0 * u - 1.0


def lanczos_lambda_max(lv: Level, steps=20, seed=12345):
    """Largest eigenvalue of Dinv A by `steps` Lanczos steps on the symmetric
    form Dinv^{1/2} A Dinv^{1/2} in the W inner product (no reorthogonalisation).
    The start vector is the SplitMix64 value of each copy's global pointer,
    so copies of a node agree."""
    s = np.sqrt(lv.Dinv)
    v = lv.mask * splitmix64_uniform(lv.gid, seed)
    v /= lv.norm(v)
    v_prev = np.zeros_like(v)
    beta = 0.0
    alphas, betas = [], []
    for _ in range(steps):
        w = s * lv.apply(s * v) - beta * v_prev
        alpha = lv.dot(w, v)
        w -= alpha * v
        alphas.append(alpha)
        beta = lv.norm(w)
        if beta == 0.0:
            break
        betas.append(beta)
        v_prev, v = v, w / beta
    m = len(alphas)
    T = np.diag(alphas) + np.diag(betas[: m - 1], 1) + np.diag(betas[: m - 1], -1)
    return float(np.linalg.eigvalsh(T)[-1])


def chebyshev(lv: Level, r, x, lmin, lmax, degree):
    """Chebyshev acceleration of Jacobi (Saad, Alg. 12.1 applied to
    Dinv A x = Dinv r) with `degree` updates on the interval [lmin, lmax].
    x may be None (zero initial guess, which saves the first residual)."""
    theta = 0.5 * (lmax + lmin)
    delta = 0.5 * (lmax - lmin)
    sigma = theta / delta
    rho_prev = 1.0 / sigma
    if x is None:
        x = np.zeros_like(r)
        res = r.copy()
    else:
        x = x.copy()
        res = r - lv.apply(x)
    d = lv.Dinv * res / theta
    x += d
    for _ in range(1, degree):
        rho = 1.0 / (2.0 * sigma - rho_prev)
        res = r - lv.apply(x)
        d = rho * rho_prev * d + (2.0 * rho / delta) * (lv.Dinv * res)
        x += d
        rho_prev = rho
    return x


class PMG:
    """p-multigrid V-cycle with Chebyshev-Jacobi pre- and post-smoothing on
    every level but the coarsest (Sec. 3.4: schedule N, N/2, 1 and two
    Chebyshev-accelerated Jacobi sweeps at the upper levels); coarse problem
    solved by Jacobi-PCG.  Levels are rediscretised on coordinates
    interpolated from the fine mesh; box meshes only (coarse numbering from
    the structured generator)."""

    def __init__(self, mesh_factory, fine_mesh, levels=(7, 3, 1), h1=1.0, h2=0.0, degree=2,
                 lmin_frac=0.1, lmax_frac=1.1, lanczos_steps=20, coarse_tol=1e-4,
                 coarse_maxit=200):
        self.levels = []
        self.J = []
        x, y, z = fine_mesh.x, fine_mesh.y, fine_mesh.z
        prev = None
        for li, N in enumerate(levels):
            m = mesh_factory(N)
            if prev is not None:
                Nf = levels[li - 1]
                xf, _ = gll(Nf)
                xc, _ = gll(N)
                Jfc = interp_matrix(xf, xc)  # fine nodes -> coarse points
                x = interp_lvec(Jfc, x, Nf + 1, N + 1)
                y = interp_lvec(Jfc, y, Nf + 1, N + 1)
                z = interp_lvec(Jfc, z, Nf + 1, N + 1)
                self.J.append(interp_matrix(xc, xf))  # coarse nodes -> fine points
            lv = Level(N, x, y, z, m.gid, m.dirichlet, h1, h2)
            self.levels.append(lv)
            prev = lv
        self.degree = degree
        self.bounds = []
        for lv in self.levels[:-1]:
            lam = lanczos_lambda_max(lv, lanczos_steps)
            self.bounds.append((lmin_frac * lam, lmax_frac * lam))
        self.coarse_tol = coarse_tol
        self.coarse_maxit = coarse_maxit
        self.coarse_iters = []

    def vcycle(self, r, l=0):
        lv = self.levels[l]
        if l == len(self.levels) - 1:
            x, it, _ = pcg_jacobi(lv, r, tol=self.coarse_tol, maxit=self.coarse_maxit)
            self.coarse_iters.append(it)
            return x
        lmin, lmax = self.bounds[l]
        x = chebyshev(lv, r, None, lmin, lmax, self.degree)
        s = r - lv.apply(x)
        lc = self.levels[l + 1]
        nf, nc = lv.N + 1, lc.N + 1
        rc = lc.mask * qqt(lc.gid, interp_lvec(self.J[l].T.copy(), lv.W * s, nf, nc))
        ec = self.vcycle(rc, l + 1)
        x = x + interp_lvec(self.J[l], ec, nc, nf)
        x = chebyshev(lv, r, x, lmin, lmax, self.degree)
        return x


def fcg(lv: Level, b, precond, x0=None, tol=1e-8, maxit=1000):
    """Flexible CG (Notay 2000), Polak-Ribiere form
    beta = (z_new, r_new - r_old) / (z_old, r_old), for a nonlinear
    preconditioner (Sec. 3.4: flexible PCG).  Returns (x, iters, history)."""
    b = lv.mask * np.asarray(b, dtype=np.float64).reshape(-1)
    x = np.zeros_like(b) if x0 is None else lv.mask * np.array(x0, dtype=np.float64).reshape(-1)
    r = b - lv.apply(x)
    bn = lv.norm(b)
    hist = [lv.norm(r) / bn]
    z = lv.mask * precond(r)
    p = z.copy()
    rz = lv.dot(r, z)
    it = 0
    while it < maxit and hist[-1] > tol:
        w = lv.apply(p)
        alpha = rz / lv.dot(p, w)
        x += alpha * p
        r_old = r
        r = r - alpha * w
        it += 1
        hist.append(lv.norm(r) / bn)
        if hist[-1] <= tol:
            break
        z = lv.mask * precond(r)
        beta = lv.dot(z, r - r_old) / rz
        rz = lv.dot(z, r)
        p = z + beta * p
    return x, it, hist


def true_rel_res(lv: Level, b, x):
    b = lv.mask * np.asarray(b).reshape(-1)
    return lv.norm(b - lv.apply(x)) / lv.norm(b)


# --------------------------------------------------------------------------
# adjoint of  -div(k grad u) = f  (homogeneous Dirichlet), per-copy k and f
# --------------------------------------------------------------------------

def adjoint_loss_grad(mesh, N, f, k, u_target, tol=1e-14, maxit=20000):
    """Forward A(k) u = mask QQ^T(B f); loss L = 1/2 sum_L W Bbar (u - u_t)^2
    (= 1/2 ||u - u_t||_B^2 over unique free nodes); adjoint A lam =
    mask QQ^T(dL/du_L); dL/df = B o lam; dL/dk = -(D lam)^T G (D u) per copy.
    Returns (L, u, lam, dL/df, dL/dk, iters_fwd, iters_adj)."""
    lv = Level(N, mesh.x, mesh.y, mesh.z, mesh.gid, mesh.dirichlet, 1.0, 0.0, k)
    b = lv.rhs(f)
    u, itf, _ = pcg_jacobi(lv, b, tol=tol, maxit=maxit)
    ut = np.asarray(u_target, dtype=np.float64).reshape(-1)
    diff = u - ut
    L = 0.5 * float(np.sum(lv.W * lv.Bbar * diff * diff))
    g = lv.W * lv.Bbar * diff
    rhs = lv.mask * qqt(lv.gid, g)
    lam, ita, _ = pcg_jacobi(lv, rhs, tol=tol, maxit=maxit)
    gf = lv.B * lam
    gk = grad_k(N, lv.D, lv.G, u, lam, 1.0)
    return L, u, lam, gf, gk, itf, ita


def adjoint_loss(mesh, N, f, k, u_target, tol=1e-14, maxit=20000):
    lv = Level(N, mesh.x, mesh.y, mesh.z, mesh.gid, mesh.dirichlet, 1.0, 0.0, k)
    u, _, _ = pcg_jacobi(lv, lv.rhs(f), tol=tol, maxit=maxit)
    diff = u - np.asarray(u_target).reshape(-1)
    return 0.5 * float(np.sum(lv.W * lv.Bbar * diff * diff))
