"""Pins for the oracle's projection of initial guesses (Fischer 1998, the
pressure initial guesses the NekRS paper cites): exactness for a right-hand
side in the span of earlier ones, optimality against the A-norm normal
equations of the raw earlier solutions (a different algorithm), A-orthonormal
basis, restart when the space is full, and the tolerance relative to the
original right-hand side.  CPU only."""
import numpy as np
import pytest

import oracle
from oracle import dense, solvers
from oracle.projection import Projection
from paper_2104_05829_amd import inputs


def _problem(h2=5.0):
    N = 3
    xi, _ = oracle.gll(N)
    m = inputs.box_mesh(2, 2, 2, xi, deform="cyclic")
    lv = solvers.Level(N, m.x, m.y, m.z, m.gid, m.dirichlet, 1.0, h2)
    Abar, Q, _ = dense.assembled(N, lv.D, lv.G, m.gid, lv.B, None, 1.0, h2)

    def exact(bp, tol_rel):
        return dense.solve_restricted(Abar, Q, m.dirichlet, bp), 1

    def b_of(seed):
        return lv.rhs(inputs.gaussian_per_node(m.gid, seed))

    return m, lv, exact, b_of


def test_rhs_in_span_is_solved_by_projection_alone():
    m, lv, exact, b_of = _problem()
    P = Projection(lv, 8)
    b1, b2 = b_of(1), b_of(2)
    x1, _, _ = P.solve(b1, exact, 1e-12)
    x2, _, _ = P.solve(b2, exact, 1e-12)
    b3 = 2.0 * b1 - 0.5 * b2
    xbar, bp = P.project(b3)
    ref = 2.0 * x1 - 0.5 * x2
    assert np.max(np.abs(xbar - ref)) <= 1e-11 * np.max(np.abs(ref))
    assert lv.norm(bp) <= 1e-11 * lv.norm(b3)
    x3, it, _ = P.solve(b3, exact, 1e-10)
    assert it == 0 and P.size == 2  # nothing new to add


def test_projection_is_the_a_norm_best_approximation():
    """xbar equals X c with (X^T A X) c = X^T b for the raw earlier solutions
    X (normal equations of min ||X c - A^{-1} b||_A, solved densely)."""
    m, lv, exact, b_of = _problem()
    P = Projection(lv, 8)
    X = []
    for s in (1, 2, 3, 4):
        x, _, _ = P.solve(b_of(s), exact, 1e-12)
        X.append(x)
    b5 = b_of(5) + 0.3 * b_of(1)
    xbar, _ = P.project(b5)
    X = np.array(X)
    AX = np.array([lv.apply(x) for x in X])
    M = np.array([[lv.dot(xi, axj) for axj in AX] for xi in X])
    rhs = np.array([lv.dot(xi, b5) for xi in X])
    c = np.linalg.solve(M, rhs)
    ref = c @ X
    assert np.max(np.abs(xbar - ref)) <= 1e-9 * np.max(np.abs(ref))
    # error of xbar is A-orthogonal to the space
    xs, _ = exact(b5, 0)
    for xi in X:
        assert abs(lv.dot(xi, lv.apply(xs - xbar))) <= 1e-10 * lv.norm(b5) * lv.norm(xi)


def test_basis_is_a_orthonormal_and_bt_is_a_xt():
    """Also with loose inner solves (tolerance 1e-3), whose corrections are
    not A-orthogonal to the space by themselves, so Gram-Schmidt matters."""
    m, lv, exact, b_of = _problem()

    def loose(bp, tol_rel):
        x, it, _ = solvers.pcg_jacobi(lv, bp, tol=1e-3)
        return x, it

    for inner in (exact, loose):
        P = Projection(lv, 8)
        for s in range(1, 6):
            P.solve(b_of(s), inner, 1e-12)
        _check_basis(lv, P)


def _check_basis(lv, P):
    assert P.size == 5
    G = np.array([[lv.dot(xi, lv.apply(xj)) for xj in P.xt] for xi in P.xt])
    assert np.max(np.abs(G - np.eye(5))) <= 1e-10
    for xt, bt in zip(P.xt, P.bt):
        assert np.max(np.abs(bt - lv.apply(xt))) <= 1e-10 * np.max(np.abs(bt))


def test_full_space_restarts_from_the_latest_solution():
    m, lv, exact, b_of = _problem()
    P = Projection(lv, 3)
    for s in (1, 2, 3):
        P.solve(b_of(s), exact, 1e-12)
    assert P.size == 3
    x4, _, _ = P.solve(b_of(4), exact, 1e-12)
    assert P.size == 1
    nu = np.sqrt(lv.dot(x4, lv.apply(x4)))
    assert np.max(np.abs(P.xt[0] - x4 / nu)) <= 1e-12 * np.max(np.abs(x4 / nu))


@pytest.mark.parametrize("L", [2, 8])
def test_tolerance_is_relative_to_the_original_rhs(L):
    """With an iterative inner solver the final true residual meets
    tol ||b|| and a slowly varying sequence needs fewer inner iterations than
    solving from zero."""
    m, lv, exact, b_of = _problem(h2=1.0)
    f0, f1, f2 = (inputs.gaussian_per_node(m.gid, s) for s in (11, 12, 13))
    P = Projection(lv, L)
    tol = 1e-8

    def inner(bp, tol_rel):
        x, it, _ = solvers.pcg_jacobi(lv, bp, tol=tol_rel)
        return x, it

    its_p, its_0 = [], []
    for n in range(6):
        t = 0.1 * n
        b = lv.rhs(f0 + np.sin(t) * f1 + t * t * f2)
        x, it, _ = P.solve(b, inner, tol)
        assert solvers.true_rel_res(lv, b, x) <= 1.5 * tol
        its_p.append(it)
        its_0.append(solvers.pcg_jacobi(lv, b, tol=tol)[1])
    assert sum(its_p[2:]) < sum(its_0[2:])


# ---- the pins above must catch plausible mistakes in the projection ------
_Base = Projection  # the real class (the name Projection is swapped below)


class _MutProjectWrongVector(_Base):
    def project(self, b):
        b = np.asarray(b, dtype=np.float64).reshape(-1)
        xbar, bp = np.zeros_like(b), b.copy()
        for xt, bt in zip(self.xt, self.bt):
            a = self.lv.dot(xt, b)
            xbar += a * xt
            bp -= a * xt  # mistake: subtracts the solution basis, not A of it
        return xbar, bp


class _MutAlphaFromBt(_Base):
    def project(self, b):
        b = np.asarray(b, dtype=np.float64).reshape(-1)
        xbar, bp = np.zeros_like(b), b.copy()
        for xt, bt in zip(self.xt, self.bt):
            a = self.lv.dot(bt, b)  # mistake: coefficient from bt
            xbar += a * xt
            bp -= a * bt
        return xbar, bp


class _MutNoGramSchmidtOnBt(_Base):
    def update(self, x, dx):
        import math
        lv = self.lv
        if self.size >= self.L:
            return _Base.update(self, x, dx)
        w = lv.apply(dx)
        gam = [lv.dot(xt, w) for xt in self.xt]
        v = np.array(dx, dtype=np.float64)
        for g, xt in zip(gam, self.xt):
            v -= g * xt
        bv = w.copy()  # mistake: bt of the new vector not orthogonalised
        nu = math.sqrt(max(lv.dot(v, bv), 1e-300))
        self.xt.append(v / nu)
        self.bt.append(bv / nu)


class _MutRestartUnnormalised(_Base):
    def update(self, x, dx):
        if self.size >= self.L:
            self.xt, self.bt = [np.array(x)], [self.lv.apply(x)]  # mistake: no A-normalisation
            return
        return _Base.update(self, x, dx)


_PINS = ["test_rhs_in_span_is_solved_by_projection_alone",
         "test_projection_is_the_a_norm_best_approximation",
         "test_basis_is_a_orthonormal_and_bt_is_a_xt",
         "test_full_space_restarts_from_the_latest_solution"]


@pytest.mark.parametrize("mutant", [_MutProjectWrongVector, _MutAlphaFromBt, _MutNoGramSchmidtOnBt,
                                    _MutRestartUnnormalised])
def test_pins_catch_projection_mutant(mutant, monkeypatch):
    import sys
    mod = sys.modules[__name__]
    monkeypatch.setattr(mod, "Projection", mutant)
    caught = 0
    for name in _PINS:
        try:
            getattr(mod, name)()
        except AssertionError:
            caught += 1
    assert caught >= 1, mutant.__name__
