"""Pins for the oracle's Schwarz smoother (FDM local solves on overlapping
extended elements, CHEBY-ASM / CHEBY-RAS of Sec. 3.4): the FDM inverse
against a dense solve of the separable operator, the separable operator
against the dense assembled SEM operator restricted to the extended
subdomain on an undeformed box (an independent construction: 3D element
matrices from the C oracle, Boolean assembly), a single Dirichlet element
where the Schwarz operator is the exact inverse, and the smoother's effect on
p-multigrid iteration counts.  CPU only."""
import numpy as np
import pytest

import oracle
from oracle import asm, dense, solvers
from paper_2104_05829_amd import inputs


def _setup(shape, N, deform=None, h1=1.0, h2=0.0, bc="dirichlet", variant="asm"):
    xi, _ = oracle.gll(N)
    m = inputs.box_mesh(*shape, xi, deform=deform, bc=bc)
    lv = solvers.Level(N, m.x, m.y, m.z, m.gid, m.dirichlet, h1, h2)
    S = asm.Schwarz(lv, m.shape, m.x, m.y, m.z, m.dirichlet, variant)
    return m, lv, S


def _dense_separable(N, e, S, m, lv, h1, h2):
    xi, rho = oracle.gll(N)
    D = oracle.dhat(N, xi)
    Lens = asm.element_lengths(N, m.x, m.y, m.z)
    Ex, Ey, Ez = m.shape
    ec = (e % Ex, (e // Ex) % Ey, e // (Ex * Ey))
    strides, dims = (1, Ex, Ex * Ey), (Ex, Ey, Ez)
    nq = N + 1
    dirm = m.dirichlet.reshape(-1, nq, nq, nq).astype(bool)
    lo_dir = (dirm[e, :, :, 0].all(), dirm[e, :, 0, :].all(), dirm[e, 0, :, :].all())
    hi_dir = (dirm[e, :, :, N].all(), dirm[e, :, N, :].all(), dirm[e, N, :, :].all())
    KM = []
    for d in range(3):
        Lm = Lens[e - strides[d], d] if ec[d] > 0 else None
        Lp = Lens[e + strides[d], d] if ec[d] < dims[d] - 1 else None
        KM.append(asm.extended_1d(N, rho, D, Lens[e, d], Lm, Lp, lo_dir[d], hi_dir[d]))
    (Kx, Mx, kx), (Ky, My, ky), (Kz, Mz, kz) = KM
    A = h1 * (np.kron(Mz, np.kron(My, Kx)) + np.kron(Mz, np.kron(Ky, Mx)) + np.kron(Kz, np.kron(My, Mx)))
    A += h2 * np.kron(Mz, np.kron(My, Mx))
    kept = kz[:, None, None] & ky[None, :, None] & kx[None, None, :]
    return A, kept


@pytest.mark.parametrize("e,h2", [(13, 0.0), (13, 3.0), (0, 1.0), (5, 0.0)])
def test_fdm_inverse_is_the_separable_inverse(e, h2):
    N = 4
    m, lv, S = _setup((3, 3, 3), N, deform="cyclic", h2=h2)
    A, kept = _dense_separable(N, e, S, m, lv, 1.0, h2)
    rng = np.random.default_rng(3)
    rt = np.where(kept, rng.standard_normal(kept.shape), 0.0)
    u = S.local_solve(e, rt, 1.0, h2)
    ref = np.linalg.solve(A, rt[kept])
    assert np.max(np.abs(u[kept] - ref)) <= 1e-11 * np.max(np.abs(ref))
    assert np.all(u[~kept] == 0.0)


@pytest.mark.parametrize("e", [13, 0, 4, 22])
@pytest.mark.parametrize("h2", [0.0, 7.0])
def test_separable_operator_equals_assembled_operator_on_undeformed_box(e, h2):
    """On a box of equal undeformed elements the separable operator of an
    extended subdomain is exactly the assembled SEM operator restricted to the
    subdomain's nodes (homogeneous Dirichlet around it)."""
    N = 3
    m, lv, S = _setup((3, 3, 3), N, h2=h2)
    A, kept = _dense_separable(N, e, S, m, lv, 1.0, h2)
    Abar, Q, _ = dense.assembled(N, lv.D, lv.G, m.gid, lv.B, None, 1.0, h2)
    copies = S.ix[e][kept]
    cols = np.argmax(Q[copies], axis=1)
    ref = Abar[np.ix_(cols, cols)]
    assert np.max(np.abs(A - ref)) <= 1e-11 * np.max(np.abs(ref))


def _stretched_box(N, lx, ly, lz):
    """Box of affine rectangular elements with unequal lengths lx[i], ly[j],
    lz[k] per element column (a remap of the unit box's element coordinates)."""
    xi, _ = oracle.gll(N)
    m = inputs.box_mesh(len(lx), len(ly), len(lz), xi)
    Ex, Ey, Ez = m.shape
    e = np.arange(m.E)
    ec = (e % Ex, (e // Ex) % Ey, e // (Ex * Ey))
    for arr, lens, c, n in ((m.x, lx, ec[0], Ex), (m.y, ly, ec[1], Ey), (m.z, lz, ec[2], Ez)):
        edges = np.concatenate([[0.0], np.cumsum(lens)])
        h = 1.0 / n
        t = (arr - c[:, None, None, None] * h) / h  # in [0, 1] inside the element
        arr[...] = edges[c][:, None, None, None] + t * np.asarray(lens)[c][:, None, None, None]
    return m


@pytest.mark.parametrize("e", [13, 0, 14, 22])
def test_separable_operator_on_unequal_affine_elements(e):
    """Elements of unequal lengths (affine boxes): the extended subdomain must
    take each neighbour's own length."""
    N = 3
    m = _stretched_box(N, (0.7, 1.0, 1.6), (1.2, 0.5, 0.9), (0.6, 1.1, 0.8))
    lv = solvers.Level(N, m.x, m.y, m.z, m.gid, m.dirichlet, 1.0, 2.0)
    S = asm.Schwarz(lv, m.shape, m.x, m.y, m.z, m.dirichlet)
    A, kept = _dense_separable(N, e, S, m, lv, 1.0, 2.0)
    Abar, Q, _ = dense.assembled(N, lv.D, lv.G, m.gid, lv.B, None, 1.0, 2.0)
    cols = np.argmax(Q[S.ix[e][kept]], axis=1)
    ref = Abar[np.ix_(cols, cols)]
    assert np.max(np.abs(A - ref)) <= 1e-11 * np.max(np.abs(ref))


@pytest.mark.parametrize("variant", ["asm", "ras"])
def test_single_dirichlet_element_gives_the_exact_inverse(variant):
    N = 5
    m, lv, S = _setup((1, 1, 1), N, h2=2.0, variant=variant)
    b = lv.rhs(inputs.gaussian_per_node(m.gid, 4))
    z = S.apply(b)
    Abar, Q, _ = dense.assembled(N, lv.D, lv.G, m.gid, lv.B, None, 1.0, 2.0)
    ref = dense.solve_restricted(Abar, Q, m.dirichlet, b)
    assert np.max(np.abs(z - ref)) <= 1e-11 * np.max(np.abs(ref))


def test_counting_weight_and_positivity():
    N = 4
    m, lv, S = _setup((3, 3, 2), N, deform="cyclic", h2=1.0)
    # every free node lies in its owners' subdomains and in the neighbours' extensions
    free = lv.mask > 0
    assert np.all(S.count[free] >= lv.mult[free])
    assert np.all(S.count[~free] == 0)
    rng = np.random.default_rng(8)
    for _ in range(3):
        r = lv.mask * oracle.qqt(m.gid, rng.standard_normal(m.n_local) * lv.W)
        assert lv.dot(r, S.apply(r)) > 0.0


def test_schwarz_preconditioned_fcg_beats_jacobi():
    N = 5
    m, lv, S = _setup((3, 3, 3), N, deform="cyclic", h2=0.5)
    b = lv.rhs(inputs.gaussian_per_node(m.gid, 12))
    _, it_j, _ = solvers.pcg_jacobi(lv, b, tol=1e-8)
    x, it_s, _ = solvers.fcg(lv, b, S.apply, tol=1e-8)
    assert solvers.true_rel_res(lv, b, x) <= 2e-8
    assert it_s < it_j / 2, (it_s, it_j)


@pytest.mark.parametrize("variant", ["asm", "ras"])
def test_cheby_schwarz_pmg_halves_iterations(variant):
    """Sec. 3.4 reports about half the pressure iterations of CHEBY-JAC for
    CHEBY-ASM; on a deformed 4^3 box (N = 7 -> 3 -> 1) the oracle's Schwarz
    smoother, with the Chebyshev interval [0.25, 1.1] lambda_max, needs at
    most 60% of CHEBY-JAC's FCG iterations."""
    N, shape = 7, (4, 4, 4)
    xi, _ = oracle.gll(N)
    m = inputs.box_mesh(*shape, xi, deform="cyclic")
    lv = solvers.Level(N, m.x, m.y, m.z, m.gid, m.dirichlet, 1.0, 0.0)
    b = lv.rhs(inputs.gaussian_per_node(m.gid, 30))
    fac = lambda n: inputs.box_mesh(*shape, oracle.gll(n)[0])  # noqa: E731
    jac = solvers.PMG(fac, m, levels=(7, 3, 1), coarse_tol=1e-2, coarse_maxit=20)
    _, it_j, _ = solvers.fcg(lv, b, jac.vcycle, tol=1e-8)
    mg = asm.SchwarzPMG(fac, m, levels=(7, 3, 1), lmin_frac=0.25, variant=variant)
    x, it_s, _ = solvers.fcg(lv, b, mg.vcycle, tol=1e-8)
    assert solvers.true_rel_res(lv, b, x) <= 2e-8
    assert it_s <= 0.6 * it_j, (it_s, it_j)


# ---- the pins above must catch plausible mistakes in the Schwarz oracle ---
_real_ext1d, _real_fdm1d, _real_solve = asm.extended_1d, asm.fdm_1d, asm.Schwarz.local_solve


def _mut_ext_offset(N, rho, D, L, Lm, Lp, drop_lo, drop_hi):
    if Lm is not None and Lp is not None:
        Lm, Lp = Lp, Lm  # neighbour lengths swapped
    return _real_ext1d(N, rho, D, L, Lm, Lp, drop_lo, drop_hi)


def _mut_ext_lengths(N, rho, D, L, Lm, Lp, drop_lo, drop_hi):
    return _real_ext1d(N, rho, D, 0.5 * L, Lm, Lp, drop_lo, drop_hi)  # half the element length


def _mut_fdm_no_mass(K, M, keep):
    return _real_fdm1d(K, np.eye(K.shape[0]), keep)


def _mut_solve_no_h2(self, e, rt, h1, h2):
    return _real_solve(self, e, rt, h1, 0.0)


_MUTANTS = {
    "ext_neighbours_swapped": ("extended_1d", _mut_ext_offset),
    "ext_wrong_length": ("extended_1d", _mut_ext_lengths),
    "fdm_without_mass": ("fdm_1d", _mut_fdm_no_mass),
    "solve_drops_h2": ("local_solve", _mut_solve_no_h2),
}


@pytest.mark.parametrize("name", sorted(_MUTANTS))
def test_pins_catch_schwarz_mutant(name, monkeypatch):
    attr, fn = _MUTANTS[name]
    if attr == "local_solve":
        monkeypatch.setattr(asm.Schwarz, "local_solve", fn)
    else:
        monkeypatch.setattr(asm, attr, fn)
    pins = [lambda: test_fdm_inverse_is_the_separable_inverse(13, 3.0),
            lambda: test_fdm_inverse_is_the_separable_inverse(0, 1.0),
            lambda: test_separable_operator_equals_assembled_operator_on_undeformed_box(13, 7.0),
            lambda: test_separable_operator_equals_assembled_operator_on_undeformed_box(0, 0.0),
            lambda: test_single_dirichlet_element_gives_the_exact_inverse("asm"),
            lambda: test_separable_operator_on_unequal_affine_elements(13)]
    caught = 0
    for pin in pins:
        try:
            pin()
        except AssertionError:
            caught += 1
    assert caught >= 1, name
