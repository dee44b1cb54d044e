"""Batched operator, gather-scatter and lockstep solves (several fields through
one operator, the velocity components of Sec. 2.2 / Sec. 3.3) on the GPU.

Bars: every field of a batched operator or gather-scatter call is bitwise
equal to the single-field call on the same input (same arithmetic per point,
same summation order), and the single-field calls are themselves held to the
oracle here again; rows of the leading-dimension padding are never written.
Lockstep solves: each system against the oracle's own solve of it
(iterations, solution) and against the single-system library solve; at the
benchmark's 32^3 size the oracle recomputes each true residual."""
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

import ctypes  # noqa: E402

from paper_2104_05829_amd import Sem, SemError, sem as S  # noqa: E402


def _mesh(shape, N, **kw):
    xi, _ = oracle.gll(N)
    return inputs.box_mesh(*shape, xi, **kw)


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), device="cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _batch(rows, pad, dtype=torch.float64, fill=float("nan")):
    """[nrhs, n] view with leading dimension n + pad; padding set to `fill`."""
    nr, n = rows.shape
    full = torch.full((nr, n + pad), fill, dtype=dtype, device="cuda")
    full[:, :n] = torch.tensor(rows, dtype=dtype, device="cuda")
    return full, full[:, :n]


AX_CASES = [((2, 2, 3), 7, 3, 0), ((2, 2, 3), 7, 5, 37), ((3, 2, 2), 7, 2, 0), ((3, 3, 3), 3, 4, 5),
            ((3, 3, 3), 1, 3, 0), ((2, 3, 2), 5, 3, 11), ((2, 1, 2), 10, 3, 3), ((2, 2, 2), 7, 1, 0)]


@pytest.mark.parametrize("shape,N,nrhs,pad", AX_CASES)
@pytest.mark.parametrize("h2", [0.0, 10.0])
def test_ax_multi_bitwise_equals_single(shape, N, nrhs, pad, h2):
    print(f"[gpu] ax_multi {shape} N={N} nrhs={nrhs} pad={pad} h2={h2}", flush=True)
    m = _mesh(shape, N, deform="cyclic")
    s = Sem(m)
    n = m.n_local
    U = np.stack([inputs.uniform_lvector(n, 10 + r) for r in range(nrhs)])
    _, Uv = _batch(U, pad, fill=0.0)
    Wfull, Wv = _batch(np.zeros_like(U), pad)
    s.ax_multi(Uv, Wv, h1=1.3, h2=h2)
    Wm = _host(Wfull)
    for r in range(nrhs):
        w1 = _host(s.ax(_dev(U[r]), h1=1.3, h2=h2))
        np.testing.assert_array_equal(Wm[r, :n], w1)
    assert np.all(np.isnan(Wm[:, n:]))  # padding untouched
    # and against the oracle (first and last field)
    lv = solvers.Level(N, m.x, m.y, m.z, m.gid, m.dirichlet, 1.3, h2)
    for r in (0, nrhs - 1):
        ref = lv.ax_local(U[r])
        assert np.max(np.abs(Wm[r, :n] - ref)) <= 1e-12 * np.max(np.abs(ref))
    s.free()


@pytest.mark.parametrize("shape,N,nrhs,pad", [((4, 4, 4), 7, 3, 0), ((3, 3, 3), 3, 5, 19),
                                              ((3, 2, 3), 2, 2, 1)])
def test_gs_multi_bitwise_equals_single(shape, N, nrhs, pad):
    print(f"[gpu] gs_multi {shape} N={N} nrhs={nrhs}", flush=True)
    m = _mesh(shape, N)
    s = Sem(m)
    n = m.n_local
    V = np.stack([inputs.uniform_lvector(n, 20 + r) for r in range(nrhs)])
    Vfull, Vv = _batch(V, pad)
    Vv.copy_(torch.tensor(V, device="cuda"))
    s.gs_multi(Vv)
    Vm = _host(Vfull)
    for r in range(nrhs):
        np.testing.assert_array_equal(Vm[r, :n], oracle.qqt(m.gid, V[r]))
        np.testing.assert_array_equal(Vm[r, :n], _host(s.gs(_dev(V[r]))))
    assert np.all(np.isnan(Vm[:, n:]))
    s.free()


@pytest.mark.parametrize("level", [0, 1, 2])
def test_fp32_level_multi_bitwise_equals_single(level):
    print(f"[gpu] fp32 level multi {level}", flush=True)
    m = _mesh((3, 3, 2), 7, deform="cyclic")
    s = Sem(m, levels=(7, 3, 1))
    n = s.info(level)["n_local"]
    dt = torch.float32 if level < 2 else torch.float64
    U = np.stack([inputs.uniform_lvector(n, 40 + r) for r in range(3)])
    Ut = torch.tensor(U, dtype=dt, device="cuda")
    W = s.ax_level_multi(level, Ut, h1=1.0, h2=10.0)
    Wh = _host(W)
    for r in range(3):
        np.testing.assert_array_equal(Wh[r], _host(s.ax_level(level, Ut[r].contiguous(), h1=1.0, h2=10.0)))
    G = Ut.clone()
    s.gs_level_multi(level, G)
    Gh = _host(G)
    for r in range(3):
        np.testing.assert_array_equal(Gh[r], _host(s.gs_level(level, Ut[r].clone())))
    s.free()


def _helmholtz_problem(shape, N, nrhs, h2=10.0, seed=30, **kw):
    m = _mesh(shape, N, deform="cyclic", **kw)
    lv = solvers.Level(N, m.x, m.y, m.z, m.gid, m.dirichlet, 1.0, h2)
    B = np.stack([lv.rhs(inputs.gaussian_per_node(m.gid, seed + r)) for r in range(nrhs)])
    return m, lv, B


def test_solve_multi_jacobi_matches_oracle_and_single():
    print("[gpu] solve_multi jacobi", flush=True)
    N = 5
    m, lv, B = _helmholtz_problem((3, 3, 2), N, 3)
    s = Sem(m)
    X, sts, rc = s.solve_multi(_dev(B), tol=1e-12, h2=10.0, check_every=1)
    assert rc == 0
    Xh = _host(X)
    for r in range(3):
        xo, ito, _ = solvers.pcg_jacobi(lv, B[r], tol=1e-12)
        assert sts[r]["converged"] and abs(sts[r]["iters"] - ito) <= 2, (r, sts[r], ito)
        assert np.max(np.abs(Xh[r] - xo)) <= 1e-9 * np.max(np.abs(xo))
        x1, st1, rc1 = s.solve(_dev(B[r]), tol=1e-12, h2=10.0, check_every=1)
        assert rc1 == 0 and abs(st1["iters"] - sts[r]["iters"]) <= 1
        assert np.max(np.abs(_host(x1) - Xh[r])) <= 1e-10 * np.max(np.abs(xo))
    s.free()


def test_solve_multi_pmg_matches_single_and_oracle():
    """FCG + FP32 p-MG on three right-hand sides in lockstep: each reaches a
    true FP64 residual of 1e-8 with the single solve's iteration count (+-1)
    and agrees with the oracle's tight solution."""
    print("[gpu] solve_multi pmg", flush=True)
    N = 7
    m, lv, B = _helmholtz_problem((4, 4, 4), N, 3)
    s = Sem(m, levels=(7, 3, 1))
    X, sts, rc = s.solve_multi(_dev(B), tol=1e-8, h1=1.0, h2=10.0, precond="pmg")
    assert rc == 0
    Xh = _host(X)
    for r in range(3):
        st = sts[r]
        assert st["converged"] and st["true_rel_res"] <= 1.5e-8, (r, st)
        assert st["coarse_iters"] > 0
        x1, st1, rc1 = s.solve(_dev(B[r]), tol=1e-8, h1=1.0, h2=10.0, precond="pmg")
        assert rc1 == 0 and abs(st1["iters"] - st["iters"]) <= 1, (st1, st)
        xo, _, _ = solvers.pcg_jacobi(lv, B[r], tol=1e-13)
        err = np.sqrt(np.sum(lv.W * (Xh[r] - xo) ** 2) / np.sum(lv.W * xo ** 2))
        assert err < 1e-6, (r, err)
    s.free()


@pytest.mark.parametrize("precond", ["jacobi", "pmg"])
def test_solve_multi_systems_stop_independently(precond):
    """A zero right-hand side (done at once), a smooth load and a rough one
    stop at their own iterations; each keeps its own count and solution,
    equal to its single solve's."""
    print(f"[gpu] solve_multi mixed {precond}", flush=True)
    N = 7
    m = _mesh((3, 3, 3), N, deform="cyclic")
    lv = solvers.Level(N, m.x, m.y, m.z, m.gid, m.dirichlet, 1.0, 5.0)
    f_smooth = inputs.sin3(m.x, m.y, m.z).reshape(-1)
    B = np.stack([np.zeros(m.n_local), lv.rhs(f_smooth), lv.rhs(inputs.gaussian_per_node(m.gid, 7))])
    s = Sem(m, levels=(7, 3, 1))
    kw = dict(tol=1e-9, h1=1.0, h2=5.0, precond=precond, check_every=1)
    X, sts, rc = s.solve_multi(_dev(B), **kw)
    assert rc == 0
    Xh = _host(X)
    assert sts[0]["iters"] == 0 and sts[0]["converged"] and np.all(Xh[0] == 0.0)
    assert sts[1]["iters"] > 0 and sts[2]["iters"] > 0, sts
    for r in (1, 2):
        x1, st1, _ = s.solve(_dev(B[r]), **kw)
        assert abs(st1["iters"] - sts[r]["iters"]) <= 1, (r, st1, sts[r])
        assert sts[r]["true_rel_res"] <= 2e-9
        assert np.max(np.abs(_host(x1) - Xh[r])) <= 1e-7 * np.max(np.abs(Xh[r]))
    s.free()


def test_solve_multi_argument_errors():
    print("[gpu] solve_multi errors", flush=True)
    m = _mesh((2, 2, 2), 3)
    s = Sem(m)
    n = m.n_local
    L = S.lib()
    o = S.SemSolveOpts()
    L.sem_solve_opts_default(ctypes.byref(o))
    b = torch.zeros(5, n, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    pb, px = ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr())
    h = s._handle()
    for nr, ld in ((0, n), (5, n), (2, n - 1)):
        rc = L.sem_pcg_solve_multi(h, nr, pb, px, ld, ctypes.byref(o), None, None)
        assert rc == S.SEM_EINVAL, (nr, ld, rc)
    assert L.sem_ax_multi(h, 0, pb, px, n, 1.0, 0.0, None) == S.SEM_EINVAL
    assert L.sem_ax_multi(h, 2, pb, px, n - 1, 1.0, 0.0, None) == S.SEM_EINVAL
    assert L.sem_gs_multi(h, 2, None, n, None) == S.SEM_EINVAL
    assert L.sem_ax_level_multi(h, 1, S.SEM_F64, 1, pb, px, n, 1.0, 0.0, None) == S.SEM_EINVAL
    with pytest.raises(SemError):
        s.solve_multi(b[:2], precond="pmg")  # handle without levels
    s.free()


def test_c3_full_size_three_rhs_pmg():
    """The benchmark's three-RHS configuration: 32^3 deformed Helmholtz box,
    N=7, p-MG in lockstep.  The oracle recomputes every true residual
    ||b - A x||_W / ||b||_W in FP64 on the whole mesh."""
    print("[gpu] c3 full size three rhs", flush=True)
    N = 7
    m = _mesh((32, 32, 32), N, deform="cyclic", amp=0.05)
    s = Sem(m, levels=(7, 3, 1))
    b1 = [inputs.gaussian_per_node(m.gid, 30 + r) for r in range(3)]
    Bd = torch.empty(3, m.n_local, dtype=torch.float64, device="cuda")
    for r in range(3):
        s.rhs(_dev(b1[r]), out=Bd[r])
    X, sts, rc = s.solve_multi(Bd, tol=1e-8, h1=1.0, h2=10.0, precond="pmg")
    assert rc == 0
    Xh, Bh = _host(X), _host(Bd)
    G, Bm, _ = oracle.geometry(N, m.x, m.y, m.z)
    xi, _ = oracle.gll(N)
    Dh = oracle.dhat(N, xi)
    mask = 1.0 - m.dirichlet.reshape(-1).astype(np.float64)
    W = mask / oracle.multiplicity(m.gid)  # counting weight, 0 on Dirichlet copies
    for r in range(3):
        assert sts[r]["converged"] and 5 <= sts[r]["iters"] <= 30, sts[r]
        Ax = oracle.qqt(m.gid, oracle.ax(N, Dh, G, Xh[r], h1=1.0, h2=10.0, B=Bm))
        res = mask * (Bh[r] - Ax)
        rel = math.sqrt(np.sum(W * res * res) / np.sum(W * Bh[r] * Bh[r]))
        assert rel <= 1.5e-8, (r, rel)
        assert abs(rel - sts[r]["true_rel_res"]) <= 1e-3 * rel + 1e-12
    s.free()


@pytest.mark.parametrize("smoother", ["jacobi", "asm", "ras"])
def test_graph_replay_matches_kernel_by_kernel(smoother):
    """The V-cycle replayed from captured graphs gives the same iterates as
    the kernels launched one by one: repeated single and lockstep solves
    (the graphs replayed many times, with eager solves, host reads and
    synchronisations between them) return bit-identical solutions and the
    same iteration counts; a change of h2 recaptures."""
    print(f"[gpu] graph replay {smoother}", flush=True)
    N = 5
    m = _mesh((3, 3, 3), N, deform="cyclic")
    s = Sem(m, levels=(5, 3, 1))
    B = torch.stack([s.rhs(_dev(inputs.gaussian_per_node(m.gid, 70 + r))) for r in range(3)])
    for h2 in (2.0, 2.0, 7.0):
        kw = dict(tol=1e-9, h1=1.0, h2=h2, precond="pmg", smoother=smoother, cheb_lo=0.25)
        xe, ste, rce = s.solve(B[0].clone(), use_graphs=0, **kw)
        for rep in range(3):
            xg, stg, rcg = s.solve(B[0].clone(), use_graphs=1, **kw)
            assert rcg == rce == 0 and stg["iters"] == ste["iters"], (rep, stg, ste)
            assert torch.equal(xg, xe), rep
            torch.cuda.synchronize()
        Xe, stse, _ = s.solve_multi(B.clone(), use_graphs=0, **kw)
        for rep in range(2):
            Xg, stsg, _ = s.solve_multi(B.clone(), use_graphs=1, **kw)
            assert [a["iters"] for a in stsg] == [a["iters"] for a in stse], rep
            assert torch.equal(Xg, Xe), rep
    s.free()
