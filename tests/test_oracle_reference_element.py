"""Pins for the oracle's reference element: GLL nodes/weights, the 1D
differentiation matrix Dh (Sec. 2.3, eq. (dh)) and Lagrange interpolation.
CPU only."""
import math
import os

import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

import oracle


def _golden(golden_dir):
    rows = {}
    with open(os.path.join(golden_dir, "gll_closed_forms.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            n, nodes, weights = (p.strip() for p in line.split("|"))
            env = {"sqrt": math.sqrt}
            rows[int(n)] = (np.array([eval(s, env) for s in nodes.split(";")]),
                            np.array([eval(s, env) for s in weights.split(";")]))
    return rows


def test_gll_closed_forms(golden_dir):
    for N, (xs, ws) in _golden(golden_dir).items():
        xi, rho = oracle.gll(N)
        np.testing.assert_allclose(xi, xs, rtol=0, atol=2e-16)
        np.testing.assert_allclose(rho, ws, rtol=0, atol=4e-16)


@pytest.mark.parametrize("N", range(1, 17))
def test_gll_against_library_roots_and_sums(N):
    xi, rho = oracle.gll(N)
    # interior nodes are the roots of P_N' (numpy's Legendre-series root finder)
    if N >= 2:
        c = np.zeros(N + 1)
        c[N] = 1.0
        roots = np.sort(npleg.legroots(npleg.legder(c)))
        np.testing.assert_allclose(xi[1:-1], roots, atol=1e-13)
    assert xi[0] == -1.0 and xi[-1] == 1.0
    np.testing.assert_array_equal(xi, -xi[::-1])
    np.testing.assert_array_equal(rho, rho[::-1])
    assert abs(rho.sum() - 2.0) < 1e-14
    assert abs(rho[0] - 2.0 / (N * (N + 1))) < 1e-15
    assert np.all(np.diff(xi) > 0) and np.all(rho > 0)


@pytest.mark.parametrize("N", range(1, 13))
def test_gll_quadrature_exactness(N):
    """Exact for degree <= 2N-1 (Sec. 2.3 accuracy statement), not for 2N."""
    xi, rho = oracle.gll(N)
    for m in range(0, 2 * N):
        exact = 0.0 if m % 2 else 2.0 / (m + 1)
        assert abs(rho @ xi ** m - exact) < 1e-14, (N, m)
    m = 2 * N
    assert abs(rho @ xi ** m - 2.0 / (m + 1)) > 1e-9


@pytest.mark.parametrize("N", range(1, 16))
def test_dhat_differentiates_polynomials_exactly(N):
    """Dh applied to nodal values of x^m gives m x^(m-1) for m <= N."""
    xi, _ = oracle.gll(N)
    D = oracle.dhat(N, xi)
    for m in range(0, N + 1):
        d = D @ xi ** m
        ref = m * xi ** (m - 1) if m > 0 else np.zeros_like(xi)
        assert np.max(np.abs(d - ref)) <= 1e-13 * N * N, (N, m)
    assert np.max(np.abs(D.sum(axis=1))) <= 1e-13 * N
    # not exact one degree higher: the interpolant of x^(N+1) differs
    m = N + 1
    assert np.max(np.abs(D @ xi ** m - m * xi ** (m - 1))) > 1e-8


@pytest.mark.parametrize("N", [1, 2, 3, 5, 7, 9])
def test_dhat_known_entries(N):
    """Row/column convention Dh[i][l] = h_l'(xi_i): endpoint diagonals are
    -N(N+1)/4 and +N(N+1)/4, interior diagonals vanish; for N=1 the rows are
    (-1/2, 1/2)."""
    xi, _ = oracle.gll(N)
    D = oracle.dhat(N, xi)
    assert abs(D[0, 0] + N * (N + 1) / 4) < 1e-12 * N * N
    assert abs(D[N, N] - N * (N + 1) / 4) < 1e-12 * N * N
    for i in range(1, N):
        assert abs(D[i, i]) < 1e-12 * N
    # derivative of h_l from numpy's polynomial fit of the cardinal function
    for l in range(N + 1):
        e = np.zeros(N + 1)
        e[l] = 1.0
        p = np.polynomial.Polynomial.fit(xi, e, N, domain=[-1, 1], window=[-1, 1])
        np.testing.assert_allclose(D[:, l], p.deriv()(xi), atol=1e-10 * N * N)
    if N == 1:
        np.testing.assert_allclose(D, [[-0.5, 0.5], [-0.5, 0.5]], atol=1e-16)


def test_interp_matrix():
    xf, _ = oracle.gll(7)
    xc, _ = oracle.gll(3)
    J = oracle.interp_matrix(xc, xf)  # coarse nodes -> fine points
    assert J.shape == (8, 4)
    for m in range(4):
        np.testing.assert_allclose(J @ xc ** m, xf ** m, atol=1e-14)
    np.testing.assert_allclose(J.sum(axis=1), 1.0, atol=1e-15)
    Jid = oracle.interp_matrix(xf, xf)
    np.testing.assert_allclose(Jid, np.eye(8), atol=1e-15)
    # endpoint rows are exact unit vectors
    assert J[0, 0] == 1.0 and np.all(J[0, 1:] == 0.0)


@pytest.mark.parametrize("Ns,Nt", [(7, 3), (3, 7), (3, 1), (1, 3), (5, 2), (2, 5), (4, 4)])
def test_interp_lvec_reproduces_polynomials(Ns, Nt):
    """Elementwise tensor-product interpolation from the order-Ns GLL nodes to
    the order-Nt GLL points reproduces every polynomial of degree <= Ns per
    variable exactly (the p-multigrid transfers of Sec. 3.4 between nested
    spaces).  Each element holds a different polynomial with unequal degrees
    per axis (x^a y^b z^c terms, a, b, c not all equal), so a transposed axis,
    a wrong element stride or a transposed J fails."""
    xs, _ = oracle.gll(Ns)
    xt, _ = oracle.gll(Nt)
    J = oracle.interp_matrix(xs, xt)
    rng = np.random.default_rng(Ns * 10 + Nt)
    E = 3
    degs = [(Ns, max(Ns - 1, 0), max(Ns - 2, 0)), (0, Ns, 1 % (Ns + 1)), (max(Ns - 1, 0), 0, Ns)]

    def poly(e, r, s, t):
        a, b, c = degs[e]
        coef = rng_coef[e]
        return coef[0] * r ** a * s ** b * t ** c + coef[1] * r ** b * t ** a + coef[2] * s ** c + coef[3]

    rng_coef = rng.standard_normal((E, 4))
    vin = np.concatenate([poly(e, xs[None, None, :], xs[None, :, None], xs[:, None, None]).reshape(-1)
                          for e in range(E)])
    out = oracle.interp_lvec(J, vin, Ns + 1, Nt + 1)
    ref = np.concatenate([poly(e, xt[None, None, :], xt[None, :, None], xt[:, None, None]).reshape(-1)
                          for e in range(E)])
    np.testing.assert_allclose(out, ref, atol=1e-13 * np.max(np.abs(ref)))
    if Nt < Ns:
        # a polynomial of degree above Nt per variable is not reproduced going
        # back up from Nt: the round trip differs (the pin is not vacuous)
        back = oracle.interp_lvec(oracle.interp_matrix(xt, xs), out, Nt + 1, Ns + 1)
        assert np.max(np.abs(back - vin)) > 1e-6 * np.max(np.abs(vin))
