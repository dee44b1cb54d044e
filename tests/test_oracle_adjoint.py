"""Pins for the oracle adjoint of -div(k grad u) = f with homogeneous
Dirichlet data: central finite differences in f (exact, the loss is
quadratic in f) and in k, and a dense-matrix gradient on a tiny mesh.  CPU."""
import numpy as np

import oracle
from oracle import dense, solvers
from paper_2104_05829_amd import inputs


def _case(shape=(2, 2, 2), N=3):
    xi, _ = oracle.gll(N)
    m = inputs.box_mesh(*shape, xi, deform="cyclic")
    g = inputs.fourier_field(m.x, m.y, m.z, 4, 40).reshape(-1)
    k = np.exp(0.5 * g)
    f = 1.0 + inputs.fourier_field(m.x, m.y, m.z, 4, 41).reshape(-1)
    ut = inputs.sin3(m.x, m.y, m.z).reshape(-1)
    return m, N, f, k, ut


def test_adjoint_gradients_vs_central_differences():
    m, N, f, k, ut = _case()
    L, u, lam, gf, gk, itf, ita = solvers.adjoint_loss_grad(m, N, f, k, ut)
    rng = np.random.default_rng(42)
    h = 1e-6
    for _ in range(3):
        d = rng.standard_normal(f.size)
        d /= np.linalg.norm(d)
        fd = (solvers.adjoint_loss(m, N, f + h * d, k, ut)
              - solvers.adjoint_loss(m, N, f - h * d, k, ut)) / (2 * h)
        an = float(gf @ d)
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3), (fd, an)
        dk = rng.standard_normal(k.size)
        dk /= np.linalg.norm(dk)
        fdk = (solvers.adjoint_loss(m, N, f, k + h * dk, ut)
               - solvers.adjoint_loss(m, N, f, k - h * dk, ut)) / (2 * h)
        ank = float(gk @ dk)
        assert abs(fdk - ank) <= 1e-6 * max(abs(ank), 1e-3), (fdk, ank)


def test_adjoint_matches_dense_gradient():
    """Dense: u = Q R^T A^{-1} R Q^T (B f); L = 1/2 sum W Bbar (u-ut)^2;
    dL/df = B Q R^T A^{-1} R Q^T g;  dL/dk_q = -lam^T (dA_L/dk_q) u with
    dA_L/dk_q = sum D_m^T e_q G_mm'(q) e_q^T D_m' (explicit per copy)."""
    m, N, f, k, ut = _case(shape=(2, 1, 1), N=2)
    L, u, lam, gf, gk, _, _ = solvers.adjoint_loss_grad(m, N, f, k, ut)
    lv = solvers.Level(N, m.x, m.y, m.z, m.gid, m.dirichlet, 1.0, 0.0, k)
    Abar, Q, AL = dense.assembled(N, lv.D, lv.G, m.gid, None, k)
    free = dense.free_columns(Q, m.dirichlet)
    R = np.zeros((free.size, Q.shape[1]))
    R[np.arange(free.size), free] = 1.0
    A = R @ Abar @ R.T
    Ainv = np.linalg.inv(A)
    S = Q @ R.T @ Ainv @ R @ Q.T
    ud = S @ (lv.B * f)
    np.testing.assert_allclose(u, ud, atol=1e-11 * np.abs(ud).max())
    Bbar = Q @ (Q.T @ lv.B)
    W = lv.W
    g = W * Bbar * (ud - ut)
    gf_d = lv.B * (S @ g)
    np.testing.assert_allclose(gf, gf_d, atol=1e-11 * np.abs(gf_d).max())
    lam_d = S @ g
    Ds = dense.derivative_matrices(lv.D)
    np_ = (N + 1) ** 3
    pair = {(0, 0): 0, (0, 1): 1, (0, 2): 2, (1, 1): 3, (1, 2): 4, (2, 2): 5}
    gk_d = np.zeros_like(gk)
    for q in range(u.size):
        e, ql = divmod(q, np_)
        sl = slice(e * np_, (e + 1) * np_)
        s = 0.0
        for mm in range(3):
            for mp in range(3):
                gq = lv.G[pair[(min(mm, mp), max(mm, mp))], q]
                s += (Ds[mm] @ lam_d[sl])[ql] * gq * (Ds[mp] @ ud[sl])[ql]
        gk_d[q] = -s
    np.testing.assert_allclose(gk, gk_d, atol=1e-10 * np.abs(gk_d).max())
