"""Dense brute-force forms of the SEM operator for tiny meshes.

TEST INFRASTRUCTURE (see the package docstring).  Every operator is formed as
an explicit matrix: D_1 = I (x) I (x) Dh, D_2 = I (x) Dh (x) I,
D_3 = Dh (x) I (x) I (Sec. 2.3, eqs. (gradr)-(gradt)), the element matrix
A^e = sum_{m,m'} D_m^T diag(k G_mm') D_m' (eq. (Ae)), the Boolean
global-to-local map Q (u_L = Q u), the assembled Neumann operator
Abar = Q^T A_L Q and the restricted A = R Abar R^T (footnote to the
Q^T A_L Q discussion).  Linear solves use a dense Cholesky factorisation.
"""
from __future__ import annotations

import numpy as np


def derivative_matrices(D):
    nq = D.shape[0]
    I = np.eye(nq)
    D1 = np.kron(I, np.kron(I, D))
    D2 = np.kron(I, np.kron(D, I))
    D3 = np.kron(D, np.kron(I, I))
    return D1, D2, D3


def element_matrices(N, D, G, B=None, k=None, h1=1.0, h2=0.0):
    """List of dense (N+1)^3 x (N+1)^3 matrices h1 A^e(k) + h2 B^e."""
    np_ = (N + 1) ** 3
    nL = G.shape[1]
    E = nL // np_
    Ds = derivative_matrices(D)
    pair = {(0, 0): 0, (0, 1): 1, (0, 2): 2, (1, 1): 3, (1, 2): 4, (2, 2): 5}
    out = []
    for e in range(E):
        sl = slice(e * np_, (e + 1) * np_)
        kk = np.ones(np_) if k is None else np.asarray(k).reshape(-1)[sl]
        Ae = np.zeros((np_, np_))
        for m in range(3):
            for mp in range(3):
                g = G[pair[(min(m, mp), max(m, mp))], sl] * kk
                Ae += Ds[m].T @ (g[:, None] * Ds[mp])
        Ae *= h1
        if h2 != 0.0:
            Ae += h2 * np.diag(np.asarray(B).reshape(-1)[sl])
        out.append(Ae)
    return out


def boolean_q(gid):
    """Dense Q (n_local x n_global) with Q[l, c] = 1 when copy l is global
    node c; pointer-0 copies each get their own column.  Returns (Q, keys)
    where keys[c] is the pointer of column c (negative for singletons)."""
    g = np.asarray(gid, dtype=np.int64).reshape(-1)
    keys = np.where(g != 0, g, -(np.arange(g.size) + 1))
    uniq, col = np.unique(keys, return_inverse=True)
    Q = np.zeros((g.size, uniq.size))
    Q[np.arange(g.size), col] = 1.0
    return Q, uniq


def block_diag(mats):
    n = sum(m.shape[0] for m in mats)
    A = np.zeros((n, n))
    o = 0
    for m in mats:
        s = m.shape[0]
        A[o:o + s, o:o + s] = m
        o += s
    return A


def assembled(N, D, G, gid, B=None, k=None, h1=1.0, h2=0.0):
    """(Abar, Q, A_L) with Abar = Q^T A_L Q."""
    AL = block_diag(element_matrices(N, D, G, B, k, h1, h2))
    Q, _ = boolean_q(gid)
    return Q.T @ AL @ Q, Q, AL


def free_columns(Q, dirichlet):
    """Global columns that are not Dirichlet (R keeps these rows)."""
    d = np.asarray(dirichlet).reshape(-1).astype(bool)
    is_dir = (Q[d].sum(axis=0) > 0)
    return np.where(~is_dir)[0]


def solve_restricted(Abar, Q, dirichlet, b_local):
    """Solve R Abar R^T u = R b for a replicated b_local (one value per copy);
    returns u as a replicated L-vector with zeros on Dirichlet copies."""
    free = free_columns(Q, dirichlet)
    A = Abar[np.ix_(free, free)]
    # one copy per global node: average of the (equal) copies
    cnt = Q.sum(axis=0)
    bg = (Q.T @ np.asarray(b_local).reshape(-1)) / cnt
    Lc = np.linalg.cholesky(A)
    y = np.linalg.solve(Lc, bg[free])
    uf = np.linalg.solve(Lc.T, y)
    ug = np.zeros(Q.shape[1])
    ug[free] = uf
    return Q @ ug
