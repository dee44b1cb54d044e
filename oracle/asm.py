"""Overlapping Schwarz smoothing with fast-diagonalisation (FDM) local solves,
and its Chebyshev acceleration (CHEBY-ASM / CHEBY-RAS of Sec. 3.4).

TEST INFRASTRUCTURE (see the package docstring).  Plain FP64 numpy on box
meshes (element e = ex + Ex (ey + Ey ez) as `inputs.box_mesh` lays them out).

The paper names the smoother, its cost (about 12 E (N+3)^4 operations for the
local solves) and the two ways of combining the local solutions (ASM: exchange
and add with a counting weight; RAS: each element keeps its own data), citing
the published FDM/Schwarz method (Deville, Fischer & Mund 2002; Lottes &
Fischer 2005).  The construction below follows that method:

  subdomain       element e extended by one node layer into every neighbour,
                  (N+3)^3 points; points outside the domain are absent, and an
                  element face whose nodes are all Dirichlet drops its points;
  local operator  the separable operator of the extended box
                    A~ = h1 (Mz (x) My (x) Kx + Mz (x) Ky (x) Mx + Kz (x) My (x) Mx)
                         + h2 Mz (x) My (x) Mx,
                  K_d, M_d the 1D SEM stiffness and GLL mass of the three
                  elements (neighbour, e, neighbour) along direction d, restricted
                  to the kept points (homogeneous Dirichlet beyond them); element
                  length along d = the mean distance between the end nodes of
                  the element's node lines in that direction;
  FDM             K_d s = lambda M_d s with S_d^T M_d S_d = I, so
                  A~^{-1} = (Sz (x) Sy (x) Sx) diag(1 / (h1 (lx + ly + lz) + h2)) (Sz (x) Sy (x) Sx)^T;
  combination     ASM: z = mask o QQ^T(sum_e P_e^T u_e) / c, with c the number of
                  subdomains that contain the node (the counting weight of the
                  overlapping sum); RAS: z = mask o QQ^T(own part of u_e) / mult.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg

from . import dhat, gll, qqt
from .solvers import Level, pcg_jacobi, splitmix64_uniform


def element_lengths(N, x, y, z):
    """[E, 3] mean extent of each element along its r, s, t directions."""
    nq = N + 1
    X = np.stack([np.asarray(a, dtype=np.float64).reshape(-1, nq, nq, nq) for a in (x, y, z)], axis=-1)
    Lr = np.linalg.norm(X[:, :, :, N, :] - X[:, :, :, 0, :], axis=-1).mean(axis=(1, 2))
    Ls = np.linalg.norm(X[:, :, N, :, :] - X[:, :, 0, :, :], axis=-1).mean(axis=(1, 2))
    Lt = np.linalg.norm(X[:, N, :, :, :] - X[:, 0, :, :, :], axis=-1).mean(axis=(1, 2))
    return np.stack([Lr, Ls, Lt], axis=1)


def elem_1d(N, L, rho, D):
    """1D SEM stiffness and mass of one element of length L."""
    K = (2.0 / L) * D.T @ np.diag(rho) @ D
    M = (L / 2.0) * np.diag(rho)
    return K, M


def extended_1d(N, rho, D, L, Lm, Lp, drop_lo, drop_hi):
    """(K, M, keep) on the N+3 extended points of one direction: the element
    of length L between neighbours of lengths Lm, Lp (None = no neighbour),
    assembled over the present elements and restricted to the kept points.
    keep[a] for a = 0 .. N+2 (point a - 1 in element coordinates)."""
    n3 = 3 * N + 1
    K3, M3 = np.zeros((n3, n3)), np.zeros((n3, n3))
    for off, Le in ((0, Lm), (N, L), (2 * N, Lp)):
        if Le is None:
            continue
        Ke, Me = elem_1d(N, Le, rho, D)
        K3[off:off + N + 1, off:off + N + 1] += Ke
        M3[off:off + N + 1, off:off + N + 1] += Me
    keep = np.ones(N + 3, dtype=bool)
    keep[0] = Lm is not None
    keep[N + 2] = Lp is not None
    if drop_lo:
        keep[1] = False
    if drop_hi:
        keep[N + 1] = False
    idx = (N - 1) + np.nonzero(keep)[0]
    return K3[np.ix_(idx, idx)], M3[np.ix_(idx, idx)], keep


def fdm_1d(K, M, keep):
    """(S, lam) padded to N+3: S^T M S = I on the kept rows, K S = M S diag(lam);
    columns beyond the kept count are zero with lam = 1."""
    n = keep.size
    lam, V = scipy.linalg.eigh(K, M)
    S = np.zeros((n, n))
    S[np.nonzero(keep)[0], :lam.size] = V
    lf = np.ones(n)
    lf[:lam.size] = lam
    return S, lf


class Schwarz:
    """Overlapping Schwarz operator M^{-1} of one level of a box mesh."""

    def __init__(self, lv: Level, shape, x, y, z, dirichlet, variant="asm"):
        if variant not in ("asm", "ras"):
            raise ValueError(variant)
        self.lv, self.variant = lv, variant
        N = lv.N
        self.N = N
        ne = N + 3
        self.ne = ne
        Ex, Ey, Ez = shape
        E = Ex * Ey * Ez
        nq = N + 1
        xi, rho = gll(N)
        D = dhat(N, xi)
        Lens = element_lengths(N, x, y, z)
        dirm = np.asarray(dirichlet).reshape(E, nq, nq, nq).astype(bool)
        eidx = np.arange(E)
        ec = np.stack([eidx % Ex, (eidx // Ex) % Ey, eidx // (Ex * Ey)], axis=1)
        # lattice point -> first local copy
        nx, ny, nz = Ex * N + 1, Ey * N + 1, Ez * N + 1
        lat = -np.ones(nx * ny * nz, dtype=np.int64)
        kk, jj, ii = np.meshgrid(np.arange(nq), np.arange(nq), np.arange(nq), indexing="ij")
        for e in range(E - 1, -1, -1):  # lowest element index wins
            g = (ec[e, 0] * N + ii) + nx * ((ec[e, 1] * N + jj) + ny * (ec[e, 2] * N + kk))
            lat[g.reshape(-1)] = e * nq ** 3 + np.arange(nq ** 3)
        strides = (1, Ex, Ex * Ey)
        dims = (Ex, Ey, Ez)
        face_dir = (
            (lambda e: dirm[e, :, :, 0].all(), lambda e: dirm[e, :, :, N].all()),
            (lambda e: dirm[e, :, 0, :].all(), lambda e: dirm[e, :, N, :].all()),
            (lambda e: dirm[e, 0, :, :].all(), lambda e: dirm[e, N, :, :].all()),
        )
        cc, bb, aa = np.meshgrid(np.arange(ne), np.arange(ne), np.arange(ne), indexing="ij")
        own = (aa >= 1) & (aa <= N + 1) & (bb >= 1) & (bb <= N + 1) & (cc >= 1) & (cc <= N + 1)
        self.S, self.lam, self.ix, self.tp, self.tq = [], [], [], [], []
        for e in range(E):
            Sd, ld, keeps = [], [], []
            for d in range(3):
                lo = ec[e, d] > 0
                hi = ec[e, d] < dims[d] - 1
                Lm = Lens[e - strides[d], d] if lo else None
                Lp = Lens[e + strides[d], d] if hi else None
                K, M, keep = extended_1d(N, rho, D, Lens[e, d], Lm, Lp, face_dir[d][0](e), face_dir[d][1](e))
                S, lam = fdm_1d(K, M, keep)
                Sd.append(S)
                ld.append(lam)
                keeps.append(keep)
            kept = keeps[0][aa] & keeps[1][bb] & keeps[2][cc]
            g = (ec[e, 0] * N + aa - 1) + nx * ((ec[e, 1] * N + bb - 1) + ny * (ec[e, 2] * N + cc - 1))
            ix = np.where(kept, lat[np.where(kept, g, 0)], -1)
            self.S.append(Sd)
            self.lam.append(ld)
            self.ix.append(ix)
            # points whose local solution is added back, and the copies they go to
            if variant == "asm":
                pts = np.nonzero((ix >= 0).reshape(-1))[0]
                self.tp.append(pts)
                self.tq.append(ix.reshape(-1)[pts])
            else:
                sel = (ix >= 0) & own
                pts = np.nonzero(sel.reshape(-1))[0]
                self.tp.append(pts)
                c, b, a = np.unravel_index(pts, (ne, ne, ne))
                self.tq.append(e * nq ** 3 + ((c - 1) * nq + (b - 1)) * nq + (a - 1))
        ones = np.zeros(lv.n_local)
        for e in range(E):
            np.add.at(ones, self.tq[e], 1.0)
        self.count = qqt(lv.gid, ones)  # subdomains containing each node

    def local_solve(self, e, rt, h1, h2):
        """A~_e^{-1} rt on the extended points ([c][b][a])."""
        Sx, Sy, Sz = self.S[e]
        lx, ly, lz = self.lam[e]
        t = np.einsum("ai,cba->cbi", Sx, rt)
        t = np.einsum("bj,cbi->cji", Sy, t)
        t = np.einsum("ck,cji->kji", Sz, t)
        t = t / (h1 * (lz[:, None, None] + ly[None, :, None] + lx[None, None, :]) + h2)
        t = np.einsum("ck,kji->cji", Sz, t)
        t = np.einsum("bj,cji->cbi", Sy, t)
        t = np.einsum("ai,cbi->cba", Sx, t)
        return t

    def apply(self, r):
        lv = self.lv
        r = np.asarray(r, dtype=np.float64).reshape(-1)
        acc = np.zeros_like(r)
        for e in range(len(self.ix)):
            ix = self.ix[e]
            rt = np.where(ix >= 0, r[np.maximum(ix, 0)], 0.0)
            u = self.local_solve(e, rt, lv.h1, lv.h2)
            np.add.at(acc, self.tq[e], u.reshape(-1)[self.tp[e]])
        return lv.mask * qqt(lv.gid, acc) / np.where(self.count > 0, self.count, 1.0)


def power_lambda_max(lv: Level, Minv, steps=20, seed=12345):
    """Largest eigenvalue of M^{-1} A by the power method (W-norm ratio),
    started from the SplitMix64 values of the global pointers."""
    v = lv.mask * splitmix64_uniform(lv.gid, seed)
    v /= lv.norm(v)
    lam = 0.0
    for _ in range(steps):
        w = Minv(lv.apply(v))
        lam = lv.norm(w)
        if lam == 0.0:
            break
        v = w / lam
    return lam


def chebyshev_m(lv: Level, Minv, r, x, lmin, lmax, degree):
    """Chebyshev acceleration (Saad, Alg. 12.1) of x <- x + M^{-1}(r - A x)
    with `degree` updates on [lmin, lmax]; x None means x = 0."""
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
    d = Minv(res) / theta
    x += d
    for _ in range(1, degree):
        rho = 1.0 / (2.0 * sigma - rho_prev)
        res = r - lv.apply(x)
        d = rho * rho_prev * d + (2.0 * rho / delta) * Minv(res)
        x += d
        rho_prev = rho
    return x


class SchwarzPMG:
    """p-multigrid V-cycle (the schedule and transfers of `solvers.PMG`) with
    Chebyshev-accelerated Schwarz smoothing on every level but the coarsest
    (CHEBY-ASM / CHEBY-RAS of Sec. 3.4); the interval is [lo, hi] times the
    power-method estimate of lambda_max(M^{-1} A).  Box meshes only."""

    def __init__(self, mesh_factory, fine_mesh, levels=(7, 3, 1), h1=1.0, h2=0.0, degree=2,
                 lmin_frac=0.1, lmax_frac=1.1, power_steps=20, coarse_tol=1e-2, coarse_maxit=20,
                 variant="asm"):
        from . import interp_lvec, interp_matrix
        self.levels, self.J, self.M = [], [], []
        x, y, z = fine_mesh.x, fine_mesh.y, fine_mesh.z
        for li, N in enumerate(levels):
            m = mesh_factory(N)
            if li > 0:
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
            if li < len(levels) - 1:
                self.M.append(Schwarz(lv, fine_mesh.shape, x, y, z, m.dirichlet, variant))
        self.degree = degree
        self.bounds = []
        for lv, M in zip(self.levels[:-1], self.M):
            lam = power_lambda_max(lv, M.apply, power_steps)
            self.bounds.append((lmin_frac * lam, lmax_frac * lam))
        self.coarse_tol, self.coarse_maxit = coarse_tol, coarse_maxit
        self.coarse_iters = []

    def vcycle(self, r, l=0):
        lv = self.levels[l]
        if l == len(self.levels) - 1:
            x, it, _ = pcg_jacobi(lv, r, tol=self.coarse_tol, maxit=self.coarse_maxit)
            self.coarse_iters.append(it)
            return x
        lmin, lmax = self.bounds[l]
        Minv = self.M[l].apply
        x = chebyshev_m(lv, Minv, r, None, lmin, lmax, self.degree)
        s = r - lv.apply(x)
        lc = self.levels[l + 1]
        nf, nc = lv.N + 1, lc.N + 1
        from . import interp_lvec
        rc = lc.mask * qqt(lc.gid, interp_lvec(self.J[l].T.copy(), lv.W * s, nf, nc))
        ec = self.vcycle(rc, l + 1)
        x = x + interp_lvec(self.J[l], ec, nc, nf)
        return chebyshev_m(lv, Minv, r, x, lmin, lmax, self.degree)
