"""Projected initial guesses on the GPU against the oracle's projection
(Fischer 1998; the pressure initial guesses the NekRS paper uses): per solve
the number of stored solutions used, the relative residual of the projected
guess, the iteration count and the solution; exact recovery of a right-hand
side in the span; separate spaces per lockstep slot; reset rules."""
import ctypes

import numpy as np
import pytest

import oracle
from oracle import solvers
from oracle.projection import Projection
from paper_2104_05829_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU runs, skipped there
    pytest.skip("no GPU", allow_module_level=True)

from paper_2104_05829_amd import Sem, SemError, sem as S  # noqa: E402


def _mesh(shape, N, **kw):
    xi, _ = oracle.gll(N)
    return inputs.box_mesh(*shape, xi, **kw)


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), device="cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("L", [3, 8])
def test_projection_sequence_matches_oracle(L):
    print(f"[gpu] projection sequence L={L}", flush=True)
    N, h2, tol = 5, 5.0, 1e-10
    m = _mesh((3, 3, 2), N, deform="cyclic")
    lv = solvers.Level(N, m.x, m.y, m.z, m.gid, m.dirichlet, 1.0, h2)
    P = Projection(lv, L)

    def inner(bp, tol_rel):
        x, it, _ = solvers.pcg_jacobi(lv, bp, tol=tol_rel)
        return x, it

    s = Sem(m)
    for n, f in enumerate(inputs.load_sequence(m.gid, 7, seed=60, period=8.0)):
        b = lv.rhs(f)
        size_before = P.size
        xo, ito, xbar = P.solve(b, inner, tol)
        rel_o = lv.norm(b - lv.apply(xbar)) / lv.norm(b)
        x, st, rc = s.solve(_dev(b), tol=tol, h2=h2, check_every=1, proj_dim=L)
        assert rc == 0 and st["converged"], (n, st)
        assert st["proj_vectors"] == size_before, (n, st["proj_vectors"], size_before)
        # the two projections differ by what the earlier (tol-accurate) solves differ by
        assert abs(st["proj_rel_res"] - rel_o) <= 1e-6 * rel_o + 100 * tol, (n, st["proj_rel_res"], rel_o)
        assert abs(st["iters"] - ito) <= 2, (n, st["iters"], ito)
        assert st["true_rel_res"] <= 1.5 * tol
        xh = _host(x)
        assert np.max(np.abs(xh - xo)) <= 1e-8 * np.max(np.abs(xo))
    s.free()


def test_rhs_in_span_needs_no_iterations():
    print("[gpu] projection exact span", flush=True)
    N = 5
    m = _mesh((3, 2, 2), N, deform="cyclic")
    lv = solvers.Level(N, m.x, m.y, m.z, m.gid, m.dirichlet, 1.0, 2.0)
    b1 = lv.rhs(inputs.gaussian_per_node(m.gid, 1))
    b2 = lv.rhs(inputs.gaussian_per_node(m.gid, 2))
    s = Sem(m)
    kw = dict(h2=2.0, proj_dim=4, check_every=1)
    x1, _, _ = s.solve(_dev(b1), tol=1e-13, **kw)
    x2, _, _ = s.solve(_dev(b2), tol=1e-13, **kw)
    x3, st, rc = s.solve(_dev(2.0 * b1 - 0.5 * b2), tol=1e-8, **kw)
    assert rc == 0 and st["iters"] == 0 and st["proj_vectors"] == 2, st
    assert st["proj_rel_res"] <= 1e-10 and st["true_rel_res"] <= 1e-9, st
    ref = 2.0 * _host(x1) - 0.5 * _host(x2)
    assert np.max(np.abs(_host(x3) - ref)) <= 1e-10 * np.max(np.abs(ref))
    s.free()


def test_lockstep_slots_keep_separate_spaces_pmg():
    """Three velocity-like sequences solved in lockstep with p-MG: slot r
    projects onto its own earlier solutions only, every solve meets the
    tolerance and agrees with the oracle's tight solution."""
    print("[gpu] projection lockstep pmg", flush=True)
    N = 7
    m = _mesh((4, 4, 4), N, deform="cyclic")
    lv = solvers.Level(N, m.x, m.y, m.z, m.gid, m.dirichlet, 1.0, 10.0)
    seqs = [inputs.load_sequence(m.gid, 4, seed=70 + 10 * r, period=10.0) for r in range(3)]
    s = Sem(m, levels=(7, 3, 1))
    rels = []
    for n in range(4):
        B = np.stack([lv.rhs(seqs[r][n]) for r in range(3)])
        X, sts, rc = s.solve_multi(_dev(B), tol=1e-8, h1=1.0, h2=10.0, precond="pmg", proj_dim=6)
        assert rc == 0
        Xh = _host(X)
        for r in range(3):
            assert sts[r]["proj_vectors"] == n and sts[r]["true_rel_res"] <= 1.5e-8, (n, r, sts[r])
            xo, _, _ = solvers.pcg_jacobi(lv, B[r], tol=1e-13)
            err = np.sqrt(np.sum(lv.W * (Xh[r] - xo) ** 2) / np.sum(lv.W * xo ** 2))
            assert err < 1e-6, (n, r, err)
        rels.append([st["proj_rel_res"] for st in sts])
    assert all(rel == 1.0 for rel in rels[0])
    assert all(r3 < 0.2 for r3 in rels[3]), rels
    s.free()


def test_projection_reset_rules_and_errors():
    print("[gpu] projection reset", flush=True)
    N = 3
    m = _mesh((2, 2, 2), N, deform="cyclic")
    lv = solvers.Level(N, m.x, m.y, m.z, m.gid, m.dirichlet, 1.0, 1.0)
    b = _dev(lv.rhs(inputs.gaussian_per_node(m.gid, 3)))
    s = Sem(m)
    _, st, _ = s.solve(b, h2=1.0, proj_dim=2, tol=1e-12)
    _, st, _ = s.solve(b, h2=1.0, proj_dim=2)
    assert st["proj_vectors"] == 1 and st["iters"] == 0, st
    s.proj_reset()
    _, st, _ = s.solve(b, h2=1.0, proj_dim=2)
    assert st["proj_vectors"] == 0
    _, st, _ = s.solve(b, h2=3.0, proj_dim=2)  # another operator: space cleared
    assert st["proj_vectors"] == 0
    _, st, _ = s.solve(b, h2=3.0, proj_dim=3)  # another size: cleared
    assert st["proj_vectors"] == 0
    with pytest.raises(SemError):
        s.solve(b, proj_dim=S.SEM_MAX_PROJ + 1)
    with pytest.raises(SemError):
        s.solve(b, proj_dim=2, k=torch.ones_like(b))
    s.free()


def test_full_size_projected_sequence():
    """The benchmark's projection workload at full size (32^3 deformed
    Helmholtz box, N = 7, FCG + FP32 p-MG to 1e-8, loads of
    inputs.load_sequence with period 40 and eps 1e-3), four loads: the space
    grows by one solution per solve, every solve reaches the tolerance with
    the oracle recomputing the true residual of the last one in FP64 on the
    whole mesh, later solves need fewer iterations than from zero, and each
    solution agrees with the from-zero solution to the solver tolerance."""
    import math
    print("[gpu] projection 32^3 sequence", flush=True)
    N, h2, tol = 7, 10.0, 1e-8
    m = _mesh((32, 32, 32), N, deform="cyclic", amp=0.05)
    s = Sem(m, levels=(7, 3, 1))
    W = 1.0 - m.dirichlet.reshape(-1).astype(np.float64)
    loads = inputs.load_sequence(m.gid, 4, seed=60, period=40.0, eps=1e-3)
    Wd = _dev(W / oracle.multiplicity(m.gid))
    last = None
    for n, f in enumerate(loads):
        b = s.rhs(_dev(f)) * _dev(W)
        x0, st0, rc0 = s.solve(b, tol=tol, h2=h2, precond="pmg")
        x, st, rc = s.solve(b, tol=tol, h2=h2, precond="pmg", proj_dim=8)
        assert rc == 0 and rc0 == 0 and st["converged"], (n, st)
        assert st["proj_vectors"] == n, (n, st)
        assert st["true_rel_res"] <= 1.5e-8, (n, st)
        if n >= 2:
            assert st["iters"] < st0["iters"], (n, st["iters"], st0["iters"])
        d = float(torch.sqrt(torch.sum(Wd * (x - x0) ** 2) / torch.sum(Wd * x0 ** 2)))
        assert d <= 1e-6, (n, d)
        last = (b, x, st)
    b, x, st = last
    Xh, Bh = _host(x), _host(b)
    G, Bm, _ = oracle.geometry(N, m.x, m.y, m.z)
    xi, _ = oracle.gll(N)
    Dh = oracle.dhat(N, xi)
    Wc = W / oracle.multiplicity(m.gid)
    res = W * (Bh - oracle.qqt(m.gid, oracle.ax(N, Dh, G, Xh, h1=1.0, h2=h2, B=Bm)))
    rel = math.sqrt(np.sum(Wc * res * res) / np.sum(Wc * Bh * Bh))
    assert rel <= 1.5e-8 and abs(rel - st["true_rel_res"]) <= 1e-3 * rel + 1e-12, (rel, st)
    s.free()
