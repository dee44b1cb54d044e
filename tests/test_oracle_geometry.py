"""Pins for the oracle's geometric factors (Sec. 2.3, eqs. (grad), (vBu),
(gij)) and mass matrix.  CPU only."""
import numpy as np
import pytest

import oracle
from paper_2104_05829_amd import inputs


def _mesh(shape, N, **kw):
    xi, _ = oracle.gll(N)
    return inputs.box_mesh(*shape, xi, **kw)


@pytest.mark.parametrize("N", [1, 3, 7])
def test_undeformed_cube_closed_form(N):
    """Cube elements of side h: J = (h/2)^3, G_mm = rho_ijk h/2, off-diagonal
    G = 0, B = rho_ijk (h/2)^3."""
    m = _mesh((2, 2, 2), N, L=(1.0, 1.0, 1.0))
    G, B, J = oracle.geometry(N, m.x, m.y, m.z)
    xi, rho = oracle.gll(N)
    h = 0.5
    r3 = np.einsum("k,j,i->kji", rho, rho, rho).reshape(-1)
    r3 = np.tile(r3, m.E)
    np.testing.assert_allclose(J, (h / 2) ** 3, rtol=1e-13)
    np.testing.assert_allclose(B, r3 * (h / 2) ** 3, rtol=1e-13)
    for s in (0, 3, 5):
        np.testing.assert_allclose(G[s], r3 * (h / 2), rtol=1e-13)
    for s in (1, 2, 4):
        assert np.max(np.abs(G[s])) < 1e-13


def test_affine_nonsymmetric_map():
    """Single element x = c + M r with a non-normal M: dr/dx = M^{-1},
    G = M^{-1} M^{-T} rho det M.  A transposed metric would fail here."""
    N = 4
    xi, rho = oracle.gll(N)
    M = np.array([[1.3, 0.4, -0.2], [0.1, 0.9, 0.5], [-0.3, 0.2, 1.1]])
    R = np.stack(np.meshgrid(xi, xi, xi, indexing="ij"), -1)  # [k, j, i] -> (t, s, r)
    r = R[..., 2]
    s = R[..., 1]
    t = R[..., 0]
    c = np.array([0.3, -0.2, 0.7])
    X = c[0] + M[0, 0] * r + M[0, 1] * s + M[0, 2] * t
    Y = c[1] + M[1, 0] * r + M[1, 1] * s + M[1, 2] * t
    Z = c[2] + M[2, 0] * r + M[2, 1] * s + M[2, 2] * t
    G, B, J = oracle.geometry(N, X, Y, Z)
    Mi = np.linalg.inv(M)
    Gm = Mi @ Mi.T
    det = np.linalg.det(M)
    r3 = np.einsum("k,j,i->kji", rho, rho, rho).reshape(-1)
    np.testing.assert_allclose(J, det, rtol=1e-13)
    np.testing.assert_allclose(B, r3 * det, rtol=1e-13)
    for slot, (a, b) in enumerate([(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]):
        np.testing.assert_allclose(G[slot], Gm[a, b] * r3 * det, rtol=1e-12, atol=1e-15)


def _exact_perturbed_volume(origin, L, amp):
    """Volume of the image of the box under cyclic_perturbation: integral of
    det(I + grad d) by a 48-point Gauss-Legendre rule per direction (numpy)."""
    g, w = np.polynomial.legendre.leggauss(48)
    pts = [o + 0.5 * (g + 1.0) * l for o, l in zip(origin, L)]
    wts = [0.5 * l * w for l in L]
    X, Y, Z = np.meshgrid(*pts, indexing="ij")
    Wt = np.einsum("a,b,c->abc", *wts)
    A = 2 * np.pi * amp
    s = lambda v: np.sin(2 * np.pi * v)
    c = lambda v: np.cos(2 * np.pi * v)
    P = np.zeros(X.shape + (3, 3))
    P[..., 0, 1] = A * c(Y) * s(Z)
    P[..., 0, 2] = A * s(Y) * c(Z)
    P[..., 1, 0] = A * c(X) * s(Z)
    P[..., 1, 2] = A * s(X) * c(Z)
    P[..., 2, 0] = A * c(X) * s(Y)
    P[..., 2, 1] = A * s(X) * c(Y)
    return float(np.sum(Wt * np.linalg.det(np.eye(3) + P)))


def test_deformed_volume_converges_spectrally():
    """sum(B) (the discrete integral of 1, eq. (vBu)) converges exponentially
    in N to the exact volume of the perturbed, off-centre box."""
    origin, L, amp = (0.1, 0.2, 0.3), (0.7, 0.8, 0.9), 0.05
    vex = _exact_perturbed_volume(origin, L, amp)
    errs = []
    for N in (2, 4, 6, 8, 10):
        xi, _ = oracle.gll(N)
        m = inputs.box_mesh(2, 2, 2, xi, L=L, origin=origin, deform="cyclic", amp=amp)
        G, B, J = oracle.geometry(N, m.x, m.y, m.z)
        errs.append(abs(B.sum() - vex))
        Jn = J / (0.35 * 0.4 * 0.45 / 8)  # det of the perturbation map, near 1
        assert Jn.min() > 0.8 and Jn.max() < 1.2
    assert errs[-1] < 1e-12
    assert errs[0] > 1e-6
    for a, b in zip(errs, errs[1:]):
        assert b < a / 10 or b < 1e-13


def test_deformed_G_symmetric_psd():
    N = 5
    m = _mesh((2, 2, 2), N, deform="cyclic", amp=0.05)
    G, B, J = oracle.geometry(N, m.x, m.y, m.z)
    Gm = np.stack([np.stack([G[0], G[1], G[2]], -1), np.stack([G[1], G[3], G[4]], -1),
                   np.stack([G[2], G[4], G[5]], -1)], -2)
    ev = np.linalg.eigvalsh(Gm)
    assert ev.min() > 0


def test_nonpositive_jacobian_rejected():
    N = 2
    m = _mesh((1, 1, 1), N)
    with pytest.raises(ValueError):
        oracle.geometry(N, m.x[:, :, :, ::-1].copy(), m.y, m.z)
