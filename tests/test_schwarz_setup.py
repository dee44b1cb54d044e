"""The library's host-side Schwarz setup (extended-point gather map by walking
across faces through the global pointers, FDM modes per direction, weights)
against the oracle's lattice construction on box meshes, and its invariance
under renumbering of element-local axes (elements rotated and mirrored in
their own frames, so the face walk meets every orientation).  CPU only: the
library is called through its host-only entry point."""
import numpy as np
import pytest

import oracle
from oracle import asm, solvers
from paper_2104_05829_amd import inputs
from paper_2104_05829_amd import sem as S


def _keys(gid, copies):
    """Node identity of copies: the pointer, or the copy itself for pointer 0."""
    g = gid[copies]
    return np.where(g != 0, g, -(copies.astype(np.int64) + 1))


class _LibFDM:
    """Duck-typed holder so the oracle's local solve runs on library data."""

    def __init__(self, Slib, lamlib):
        self.S = [[Slib[e, d].astype(np.float64) for d in range(3)] for e in range(Slib.shape[0])]
        self.lam = [[lamlib[e, d].astype(np.float64) for d in range(3)] for e in range(Slib.shape[0])]


CASES = [((3, 3, 3), 3, "dirichlet", False), ((3, 2, 2), 7, "dirichlet", True),
         ((2, 3, 2), 2, "neumann", False), ((2, 2, 3), 5, "dirichlet", False),
         ((1, 1, 1), 4, "dirichlet", False)]


@pytest.mark.parametrize("shape,N,bc,iz", CASES)
def test_host_setup_matches_oracle(shape, N, bc, iz):
    xi, _ = oracle.gll(N)
    m = inputs.box_mesh(*shape, xi, deform="cyclic", bc=bc, interior_zero=iz)
    lv = solvers.Level(N, m.x, m.y, m.z, m.gid, m.dirichlet, 1.0, 2.0)
    O = asm.Schwarz(lv, m.shape, m.x, m.y, m.z, m.dirichlet)
    lens = asm.element_lengths(N, m.x, m.y, m.z)
    ix, Sl, laml, cover, weight = S.schwarz_setup_host(N, m.gid, m.dirichlet, lens)
    gid = m.gid.reshape(-1)
    lib_fdm = _LibFDM(Sl, laml)
    rng = np.random.default_rng(7)
    for e in range(m.E):
        oi = O.ix[e]
        li = ix[e]
        assert np.array_equal(oi >= 0, li >= 0), e
        pres = oi >= 0
        assert np.array_equal(_keys(gid, oi[pres]), _keys(gid, li[pres].astype(np.int64))), e
        rt = np.where(pres, rng.standard_normal(pres.shape), 0.0)
        u_or = O.local_solve(e, rt, 1.0, 2.0)
        u_lib = asm.Schwarz.local_solve(lib_fdm, e, rt, 1.0, 2.0)
        assert np.max(np.abs(u_lib - u_or)) <= 2e-5 * np.max(np.abs(u_or)), e
    w_or = np.where(O.count > 0, 1.0 / np.where(O.count > 0, O.count, 1.0), 0.0) * lv.mask
    assert np.max(np.abs(weight - w_or)) <= 1e-6
    # every extended point gathers from exactly one copy
    assert cover.sum() == int(np.sum(ix >= 0))


def _rotate(arr, nq, perm, flips):
    """Element-local renumbering: axes (k, j, i) permuted by perm, then flipped."""
    a = arr.reshape(-1, nq, nq, nq)
    out = np.empty_like(a)
    for e in range(a.shape[0]):
        b = np.transpose(a[e], perm[e])
        for ax in range(3):
            if flips[e][ax]:
                b = np.flip(b, axis=ax)
        out[e] = b
    return out


@pytest.mark.parametrize("N", [2, 3, 4])
def test_host_setup_is_invariant_under_local_renumbering(N):
    """Renumbering the axes of each element (random permutation and mirror)
    leaves the Schwarz operator, seen on global nodes, unchanged: the same
    nodes per subdomain, the same weights per node, and the same local inverse
    as a matrix over the subdomain's nodes."""
    nq = N + 1
    xi, _ = oracle.gll(N)
    m = inputs.box_mesh(3, 3, 2, xi, deform="cyclic", bc="dirichlet")
    rng = np.random.default_rng(11)
    perm = [tuple(rng.permutation(3)) for _ in range(m.E)]
    flips = [tuple(bool(f) for f in rng.integers(0, 2, 3)) for _ in range(m.E)]
    rot = {k: _rotate(getattr(m, k), nq, perm, flips) for k in ("x", "y", "z", "gid", "dirichlet")}
    base = S.schwarz_setup_host(N, m.gid, m.dirichlet, asm.element_lengths(N, m.x, m.y, m.z))
    turned = S.schwarz_setup_host(N, rot["gid"], rot["dirichlet"],
                                  asm.element_lengths(N, rot["x"], rot["y"], rot["z"]))
    g0, g1 = m.gid.reshape(-1), rot["gid"].reshape(-1)
    # weights per node
    w0 = dict(zip(g0.tolist(), base[4].tolist()))
    for g, w in zip(g1.tolist(), turned[4].tolist()):
        assert abs(w0[g] - w) <= 1e-7
    ne = N + 3
    fdm0, fdm1 = _LibFDM(base[1], base[2]), _LibFDM(turned[1], turned[2])
    for e in range(m.E):
        i0, i1 = base[0][e], turned[0][e]
        k0 = _keys(g0, i0[i0 >= 0].astype(np.int64))
        k1 = _keys(g1, i1[i1 >= 0].astype(np.int64))
        assert sorted(k0.tolist()) == sorted(k1.tolist()), e
        # local inverse as a matrix over the subdomain's nodes
        def mat(fdm, ix, g):
            pres = np.argwhere(ix >= 0)
            keys = _keys(g, ix[ix >= 0].astype(np.int64))
            M = np.zeros((len(pres), len(pres)))
            for col, (c, b, a) in enumerate(pres):
                rt = np.zeros((ne, ne, ne))
                rt[c, b, a] = 1.0
                u = asm.Schwarz.local_solve(fdm, e, rt, 1.0, 0.5)
                M[:, col] = u[ix >= 0]
            order = np.argsort(keys)
            return M[np.ix_(order, order)]
        A0, A1 = mat(fdm0, i0, g0), mat(fdm1, i1, g1)
        assert np.max(np.abs(A0 - A1)) <= 1e-5 * np.max(np.abs(A0)), e


def test_host_setup_rejects_nonconforming_and_low_order():
    xi, _ = oracle.gll(1)
    m = inputs.box_mesh(2, 2, 2, xi)
    with pytest.raises(S.SemError):
        S.schwarz_setup_host(1, m.gid, m.dirichlet, np.ones((m.E, 3)))
    xi, _ = oracle.gll(3)
    m = inputs.box_mesh(2, 1, 1, xi)
    g = m.gid.copy()
    g[1, 1, 2, 0] = 10 ** 6  # element 1's shared face no longer matches element 0's
    with pytest.raises(S.SemError):
        S.schwarz_setup_host(3, g, m.dirichlet, np.ones((m.E, 3)))
