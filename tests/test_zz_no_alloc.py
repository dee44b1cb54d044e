"""sem_pcg_solve_noalloc, the Jacobi-PCG whose buffers live in the library's
static device scratch, against sem_pcg_solve (Jacobi) through the C ABI: two
calls in a row on different meshes, the second smaller, then the first mesh
again; every solution, iteration count and residual bit for bit equal to the
allocating entry point's, and the solution checked against the oracle."""
import math

import numpy as np
import pytest

import oracle
from oracle import solvers
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


def _case(shape, N, seed, h2, variable_k):
    m = _mesh(shape, N, deform="cyclic", amp=0.05)
    s = Sem(m)
    lv = solvers.Level(N, m.x, m.y, m.z, m.gid, m.dirichlet, 1.0, h2)
    b = _dev(lv.rhs(inputs.gaussian_per_node(m.gid, seed)))
    k = None
    if variable_k:
        rng = np.random.default_rng(seed + 100)
        k = _dev(np.exp(0.3 * rng.standard_normal(m.n_local)))
    return m, s, lv, b, k


def _compare(s, lv, b, k, h2):
    kw = dict(tol=1e-10, h1=1.0, h2=h2, maxit=5000)
    if k is not None:
        kw["k"] = k
    xa, sta, rca = s.solve(b, **kw)
    xn = torch.full_like(b, float("nan"))  # every entry must be written
    xn, stn, rcn = s.solve_noalloc(b, xn, zero_guess=1, **kw)
    torch.cuda.synchronize()
    assert rca == rcn == 0 and stn["converged"], (sta, stn)
    assert torch.equal(xa, xn)
    for f in ("iters", "rel_res", "true_rel_res"):
        assert sta[f] == stn[f], (f, sta[f], stn[f])
    if k is None:  # the oracle's Jacobi-PCG on the same system
        xo, ito, _ = solvers.pcg_jacobi(lv, b.cpu().numpy(), tol=1e-10, maxit=5000)
        xh = xn.cpu().numpy()
        err = math.sqrt(np.sum(lv.W * (xh - xo) ** 2) / np.sum(lv.W * xo ** 2))
        assert err <= 1e-8 and abs(ito - stn["iters"]) <= 2, (err, ito, stn["iters"])
    return xn, stn


def test_noalloc_matches_allocating_solve_on_two_meshes():
    print("[gpu] noalloc: 6x6x6 N=7, then 3x3x2 N=5, then 6x6x6 again", flush=True)
    big = _case((6, 6, 6), 7, 60, 10.0, False)
    small = _case((3, 3, 2), 5, 61, 0.0, True)
    x1, st1 = _compare(big[1], big[2], big[3], big[4], 10.0)
    _compare(small[1], small[2], small[3], small[4], 0.0)
    x3, st3 = _compare(big[1], big[2], big[3], big[4], 10.0)
    assert torch.equal(x1, x3) and st1["iters"] == st3["iters"]
    # an initial guess (zero_guess = 0) is honoured like sem_pcg_solve's
    s, b = big[1], big[3]
    x0 = 0.5 * x1
    xa, sta, _ = s.solve(b, x=x0.clone(), zero_guess=0, tol=1e-10, h1=1.0, h2=10.0)
    xn, stn, _ = s.solve_noalloc(b, x0.clone(), zero_guess=0, tol=1e-10, h1=1.0, h2=10.0)
    torch.cuda.synchronize()
    assert torch.equal(xa, xn) and sta["iters"] == stn["iters"] < st1["iters"]
    big[1].free()
    small[1].free()


def test_noalloc_rejects_what_it_cannot_hold():
    print("[gpu] noalloc: limits", flush=True)
    m = _mesh((2, 2, 2), 3, deform="cyclic")
    s = Sem(m, levels=(3, 1))
    b = s.rhs(_dev(inputs.gaussian_per_node(m.gid, 5)))
    x = torch.zeros_like(b)
    for kw in (dict(precond="pmg"), dict(proj_dim=2), dict(timers=1), dict(use_graphs=1)):
        with pytest.raises(SemError):
            s.solve_noalloc(b, x, **kw)
    s.free()
    # a mesh beyond the scratch's limit is refused before any device work
    E = 20 * 20 * 16
    assert E * 512 > S.SEM_NOALLOC_MAX_LOCAL
    m = _mesh((20, 20, 16), 7)
    s = Sem(m)
    b = torch.zeros(s.n_local, dtype=torch.float64, device="cuda")
    with pytest.raises(SemError, match="exceed the limit"):
        s.solve_noalloc(b, torch.zeros_like(b))
    s.free()
