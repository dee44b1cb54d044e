"""Pins for the oracle's element operator (Sec. 2.3, eq. (Ae)), its diagonal,
and the assembled Neumann/Dirichlet operators.  CPU only."""
import numpy as np
import pytest

import oracle
from oracle import dense
from paper_2104_05829_amd import inputs


def _setup(shape, N, deform="cyclic", bc="dirichlet", **kw):
    xi, rho = oracle.gll(N)
    m = inputs.box_mesh(*shape, xi, deform=deform, bc=bc, **kw)
    D = oracle.dhat(N, xi)
    G, B, J = oracle.geometry(N, m.x, m.y, m.z, D, rho)
    return m, D, G, B


@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 1, 1), (2, 2, 2)])
@pytest.mark.parametrize("N", [1, 2, 3, 5])
def test_ax_equals_dense_kronecker(shape, N):
    """Matrix-free loops == dense sum_mm' D_m^T G_mm' D_m' with Kronecker D_m."""
    m, D, G, B = _setup(shape, N)
    rng = np.random.default_rng(7)
    u = rng.uniform(-1, 1, m.n_local)
    k = np.exp(0.3 * rng.standard_normal(m.n_local))
    for (h1, h2, kk) in [(1.0, 0.0, None), (0.7, 10.0, None), (1.0, 0.0, k), (2.0, 3.0, k)]:
        w = oracle.ax(N, D, G, u, h1, h2, B, kk)
        AL = dense.block_diag(dense.element_matrices(N, D, G, B, kk, h1, h2))
        ref = AL @ u
        assert np.linalg.norm(w - ref) <= 1e-13 * np.linalg.norm(ref)
        d = oracle.diag(N, D, G, h1, h2, B, kk)
        np.testing.assert_allclose(d, np.diag(AL), rtol=1e-13, atol=1e-14 * np.abs(d).max())


@pytest.mark.parametrize("N", [1, 3, 6])
def test_undeformed_element_closed_form(N):
    """Cube of side h: A^e = (h/2)(Bh(x)Bh(x)Kh + Bh(x)Kh(x)Bh + Kh(x)Bh(x)Bh),
    Kh = Dh^T Bh Dh, Bh = diag(rho)."""
    m, D, G, B = _setup((1, 1, 1), N, deform=None, L=(0.6, 0.6, 0.6))
    xi, rho = oracle.gll(N)
    Bh = np.diag(rho)
    Kh = D.T @ Bh @ D
    h = 0.6
    Ae = (h / 2) * (np.kron(Bh, np.kron(Bh, Kh)) + np.kron(Bh, np.kron(Kh, Bh))
                    + np.kron(Kh, np.kron(Bh, Bh)))
    np_ = (N + 1) ** 3
    cols = np.stack([oracle.ax(N, D, G, np.eye(np_)[c]) for c in range(np_)], 1)
    np.testing.assert_allclose(cols, Ae, atol=1e-13 * np.abs(Ae).max())


@pytest.mark.parametrize("N", [3, 4, 6])
def test_energy_of_polynomial_on_box(N):
    """For u = x^2 y on an affine box, GLL quadrature of |grad u|^2 (degree
    <= 2N-1 per variable) is exact:  u^T A u = int (4 x^2 y^2 + x^4) dV."""
    a, b, c = 0.9, 1.3, 0.7
    xi, rho = oracle.gll(N)
    m = inputs.box_mesh(3, 2, 2, xi, L=(a, b, c), deform=None, bc="neumann")
    D = oracle.dhat(N, xi)
    G, B, _ = oracle.geometry(N, m.x, m.y, m.z, D, rho)
    u = (m.x ** 2 * m.y).reshape(-1)
    energy = float(u @ oracle.ax(N, D, G, u))
    exact = 4 * (a ** 3 / 3) * (b ** 3 / 3) * c + (a ** 5 / 5) * b * c
    assert abs(energy - exact) < 1e-12 * exact
    # and u^T B u = int u^2 for degree 2N-1 >= 4 in x, 2 in y
    if N >= 3:
        mass = float(np.sum(B * u * u))
        assert abs(mass - (a ** 5 / 5) * (b ** 3 / 3) * c) < 1e-12


@pytest.mark.parametrize("N", [2, 3])
def test_assembled_operator_properties(N):
    """Neumann operator Qbar = Q^T A_L Q: symmetric, annihilates constants,
    exactly one zero eigenvalue on a connected mesh; R Abar R^T is SPD; the
    matrix-free QQ^T A_L u equals Q Q^T A_L u with the dense Boolean Q."""
    m, D, G, B = _setup((2, 2, 1), N, bc="dirichlet")
    Abar, Q, AL = dense.assembled(N, D, G, m.gid)
    assert np.max(np.abs(Abar - Abar.T)) < 1e-13 * np.abs(Abar).max()
    assert np.max(np.abs(Abar @ np.ones(Abar.shape[0]))) < 1e-12 * np.abs(Abar).max()
    ev = np.linalg.eigvalsh(Abar)
    scale = ev[-1]
    assert abs(ev[0]) < 1e-12 * scale and ev[1] > 1e-6 * scale
    free = dense.free_columns(Q, m.dirichlet)
    assert np.linalg.eigvalsh(Abar[np.ix_(free, free)])[0] > 0
    u = np.random.default_rng(3).uniform(-1, 1, m.n_local)
    w = oracle.qqt(m.gid, oracle.ax(N, D, G, u))
    ref = Q @ (Q.T @ (AL @ u))
    assert np.linalg.norm(w - ref) < 1e-13 * np.linalg.norm(ref)
    ones = np.ones(m.n_local)
    assert np.max(np.abs(oracle.qqt(m.gid, oracle.ax(N, D, G, ones)))) < 1e-12 * scale


def test_operator_symmetry_matrix_free():
    """v^T (QQ^T A_L u) = u^T (QQ^T A_L v)  for continuous u, v (W-weighted)."""
    N = 4
    m, D, G, B = _setup((3, 2, 2), N, bc="neumann")
    W = 1.0 / oracle.multiplicity(m.gid)
    u = inputs.gaussian_per_node(m.gid, 1)
    v = inputs.gaussian_per_node(m.gid, 2)
    Au = oracle.qqt(m.gid, oracle.ax(N, D, G, u, 1.0, 5.0, B))
    Av = oracle.qqt(m.gid, oracle.ax(N, D, G, v, 1.0, 5.0, B))
    a, b = np.sum(W * v * Au), np.sum(W * u * Av)
    assert abs(a - b) < 1e-12 * max(abs(a), 1.0)


def test_timing_build_is_bit_identical(tmp_path):
    """The all-core timing build of the oracle (OpenMP over elements, -O3
    -march=native) computes the same geometric factors and element operator,
    bit for bit, as the checked build."""
    from paper_2104_05829_amd import inputs
    N = 5
    xi, rho = oracle.gll(N)
    D = oracle.dhat(N, xi)
    m = inputs.box_mesh(5, 4, 3, xi, deform="cyclic")
    T = oracle.timing_lib(str(tmp_path))
    G, B, J = oracle.geometry(N, m.x, m.y, m.z, D, rho)
    Gt, Bt, Jt = oracle.geometry(N, m.x, m.y, m.z, D, rho, _lib=T)
    assert np.array_equal(G, Gt) and np.array_equal(B, Bt) and np.array_equal(J, Jt)
    u = np.random.default_rng(3).uniform(-1, 1, m.n_local)
    k = np.random.default_rng(4).uniform(0.5, 2, m.n_local)
    for kw in (dict(), dict(h2=3.0, B=B), dict(h2=3.0, B=B, k=k)):
        assert np.array_equal(oracle.ax(N, D, G, u, **kw), oracle.ax(N, D, G, u, _lib=T, **kw))
    assert oracle.lib().oracle_threads() == 1
