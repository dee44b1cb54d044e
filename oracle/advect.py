"""Dealiased advection operator of the spectral element method.

TEST INFRASTRUCTURE (see the package docstring).  Plain FP64 numpy; the
Gauss-Legendre rule is numpy's, the Lagrange interpolation matrix and the GLL
differentiation matrix come from the C oracle.

The advection term c . grad w appears in the explicit EXT part of the time
integration and in the hyperbolic subproblem of the characteristics method
(Sec. 2.1, eqs. (stdadv) and (hyp)).  Its integrand has degree 3N, so the GLL
rule of the Poisson operator is not accurate enough for it and it is
evaluated on a finer quadrature (Sec. 2.3, remark after eq. (vBu)); the
kernels are the 2D and 3D thread-block advection kernels of Sec. 3.3.

For an element with GLL coordinates x and velocity c (degree-N tensor
polynomials given at the (N+1)^3 GLL points) the weak form (v, c . grad w)
is evaluated with the M-point Gauss-Legendre rule in each direction (M^3
points; by default M = ceil((3N+1)/2), the smallest rule exact for degree
3N):

  J        [M][N+1]  Lagrange interpolation from the GLL nodes to the Gauss
                     points; Jd = J Dh the derivative of the interpolant there
  X_q      dx/dr_q at the Gauss points: (J x J x Jd) x, (J x Jd x J) x,
           (Jd x J x J) x for q = r, s, t (and the same for y, z)
  F[q][d]  = rho~ |det X| dr_q/dx_d: the product Gauss weight times the
           Jacobian times the inverse metric, nine values per Gauss point
  ct_q     = sum_d F[q][d] (J x J x J) c_d   contravariant weighted velocity
  out      = (J x J x J)^T sum_q ct_q d_q(J w),   d_r(J w) = (J x J x Jd) w

so v^T out = sum over Gauss points of rho~ |det X| v (c . grad w), the exact
integral over the element whenever the integrand is a polynomial of degree
<= 2M - 1 in each reference variable (affine elements with c, v, w of
degree N: degree 3N - 1).  Arrays are element-major with i (the r
direction) fastest: [E][k][j][i] at the GLL points, [E][c][b][a] at the
Gauss points; ct is [E][3][M][M][M] (q = r, s, t).
"""
from __future__ import annotations

import numpy as np

from . import dhat, gll, interp_matrix


def default_m(N: int) -> int:
    """Smallest Gauss rule exact for degree 3N: 2M - 1 >= 3N."""
    return (3 * N + 2) // 2


def gauss(M: int):
    """Gauss-Legendre nodes and weights on [-1, 1] (numpy)."""
    return np.polynomial.legendre.leggauss(M)


def matrices(N: int, M: int):
    """(J, Jd, weights) for GLL order N and the M-point Gauss rule."""
    xi, _ = gll(N)
    g, wg = gauss(M)
    J = interp_matrix(xi, g)
    Jd = J @ dhat(N, xi)
    return J, Jd, wg


def _t3(Ac, Ab, Aa, u):
    """out[e][c][b][a] = sum Ac[c,k] Ab[b,j] Aa[a,i] u[e][k][j][i]."""
    return np.einsum("ck,bj,ai,ekji->ecba", Ac, Ab, Aa, u, optimize=True)


def _elems(v, nq):
    return np.asarray(v, dtype=np.float64).reshape(-1, nq, nq, nq)


def fine_metrics(N: int, M: int, x, y, z):
    """F [E][3 (q)][3 (d)][M][M][M] = rho~ |det X| dr_q/dx_d at the Gauss points."""
    nq = N + 1
    J, Jd, wg = matrices(N, M)
    X = np.empty((_elems(x, nq).shape[0], 3, 3, M, M, M))  # X[e][d][q] = dx_d/dr_q
    for d, coord in enumerate((x, y, z)):
        u = _elems(coord, nq)
        X[:, d, 0] = _t3(J, J, Jd, u)
        X[:, d, 1] = _t3(J, Jd, J, u)
        X[:, d, 2] = _t3(Jd, J, J, u)
    Xp = np.moveaxis(X, (1, 2), (-2, -1))  # [E][c][b][a][d][q]
    det = np.linalg.det(Xp)
    inv = np.linalg.inv(Xp)  # inv[..., q, d] = dr_q/dx_d
    rho3 = wg[:, None, None] * wg[None, :, None] * wg[None, None, :]
    F = (rho3 * np.abs(det))[..., None, None] * inv
    return np.moveaxis(F, (-2, -1), (1, 2))


def conv_velocity(N: int, M: int, x, y, z, c):
    """ct [E][3][M][M][M]: contravariant weighted velocity at the Gauss points
    for the velocity c = (cx, cy, cz) given at the GLL points."""
    nq = N + 1
    J, _, _ = matrices(N, M)
    F = fine_metrics(N, M, x, y, z)
    cf = np.stack([_t3(J, J, J, _elems(cd, nq)) for cd in c], axis=1)  # [E][d][c][b][a]
    return np.einsum("eqdcba,edcba->eqcba", F, cf)


def advect(N: int, M: int, ct, w):
    """Local (unassembled) dealiased advection of the field w by the
    contravariant velocity ct: out = J3^T sum_q ct_q d_q(J3 w), as an
    L-vector of the shape of w."""
    nq = N + 1
    J, Jd, _ = matrices(N, M)
    u = _elems(w, nq)
    ct = np.asarray(ct, dtype=np.float64).reshape(u.shape[0], 3, M, M, M)
    f = (ct[:, 0] * _t3(J, J, Jd, u) + ct[:, 1] * _t3(J, Jd, J, u)
         + ct[:, 2] * _t3(Jd, J, J, u))
    out = np.einsum("ck,bj,ai,ecba->ekji", J, J, J, f, optimize=True)
    return out.reshape(np.shape(w))


def fine_volume(N: int, M: int, x, y, z):
    """Sum over the Gauss points of rho~ |det X| (the element volumes)."""
    nq = N + 1
    J, Jd, wg = matrices(N, M)
    X = np.empty((_elems(x, nq).shape[0], 3, 3, M, M, M))
    for d, coord in enumerate((x, y, z)):
        u = _elems(coord, nq)
        X[:, d, 0] = _t3(J, J, Jd, u)
        X[:, d, 1] = _t3(J, Jd, J, u)
        X[:, d, 2] = _t3(Jd, J, J, u)
    det = np.linalg.det(np.moveaxis(X, (1, 2), (-2, -1)))
    rho3 = wg[:, None, None] * wg[None, :, None] * wg[None, None, :]
    return np.sum(rho3 * np.abs(det), axis=(1, 2, 3))
