"""The C ABI: libsem.so loads, exports every function include/sem.h declares,
and its host-only calls behave (no GPU needed: only calls that return before
any device work)."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_2104_05829_amd import sem as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sem.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"SEM_API\s+[\w\s\*]*?\b(sem_\w+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("sem_setup", "sem_ax", "sem_gs", "sem_pcg_solve", "sem_grad_k", "sem_free",
                     "sem_rhs", "sem_adjoint", "sem_strerror", "sem_last_error", "sem_ax_multi",
                     "sem_gs_multi", "sem_pcg_solve_multi"):
        assert required in names
    assert len(names) >= 16


def test_library_exports_every_declared_symbol():
    L = S.lib()
    for name in _declared():
        assert hasattr(L, name), name
        assert name in S._SIGS, f"binding lacks a signature for {name}"


def _struct_fields(txt, name):
    end = txt.index("} " + name + ";")
    start = txt.rindex("typedef struct {", 0, end)
    body = re.sub(r"/\*.*?\*/", "", txt[start + len("typedef struct {"):end], flags=re.S)
    out = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        for part in decl.split(","):
            m = re.search(r"(\w+)\s*(\[\d+\])?\s*$", part.strip())
            out.append(m.group(1))
    return out


def test_struct_layouts_match_header():
    """Field order of the ctypes mirrors follows the header."""
    txt = open(HEADER).read()
    for cname, mirror in (("sem_mesh", S.SemMesh), ("sem_setup_opts", S.SemSetupOpts),
                          ("sem_solve_opts", S.SemSolveOpts), ("sem_solve_stats", S.SemSolveStats),
                          ("sem_info_t", S.SemInfo)):
        assert _struct_fields(txt, cname) == [f for f, _ in mirror._fields_], cname


@pytest.mark.parametrize("N", [1, 2, 3, 5, 7, 10, 15])
def test_library_gll_agrees_with_oracle(N):
    """Independent implementations (library: Newton on x P_N - P_{N-1},
    barycentric Dh; oracle: Newton on P_N', Legendre-ratio Dh)."""
    xi, rho, D = S.gll(N)
    xo, ro = oracle.gll(N)
    Do = oracle.dhat(N, xo)
    np.testing.assert_allclose(xi, xo, atol=2e-16 * N)
    np.testing.assert_allclose(rho, ro, rtol=1e-14)
    np.testing.assert_allclose(D, Do, atol=1e-13 * N * N)


def test_host_error_paths():
    L = S.lib()
    assert L.sem_strerror(0) == b"success"
    assert L.sem_strerror(S.SEM_EMESH).startswith(b"invalid mesh")
    assert L.sem_gll(0, None, None, None) == S.SEM_EINVAL
    assert b"N=0" in L.sem_last_error()
    h = ctypes.c_void_p()
    # null mesh / null out / bad order / bad element count: rejected on the host
    assert L.sem_setup(None, None, None, ctypes.byref(h)) == S.SEM_EINVAL
    x = np.zeros(8)
    g = np.arange(1, 9, dtype=np.int64)
    m = S.SemMesh(0, 1, x.ctypes.data, x.ctypes.data, x.ctypes.data, g.ctypes.data, None)
    assert L.sem_setup(ctypes.byref(m), None, None, ctypes.byref(h)) == S.SEM_EINVAL
    m = S.SemMesh(1, 0, x.ctypes.data, x.ctypes.data, x.ctypes.data, g.ctypes.data, None)
    assert L.sem_setup(ctypes.byref(m), None, None, ctypes.byref(h)) == S.SEM_EINVAL
    gneg = -g
    m = S.SemMesh(1, 1, x.ctypes.data, x.ctypes.data, x.ctypes.data, gneg.ctypes.data, None)
    assert L.sem_setup(ctypes.byref(m), None, None, ctypes.byref(h)) == S.SEM_EINVAL
    assert b"negative" in L.sem_last_error()
    m = S.SemMesh(1, 1, x.ctypes.data, x.ctypes.data, x.ctypes.data, g.ctypes.data, None)
    bad = S.SemSetupOpts(1, 2, (ctypes.c_int * 4)(1, 2, 0, 0))  # coarse order not smaller
    assert L.sem_setup(ctypes.byref(m), ctypes.byref(bad), None, ctypes.byref(h)) == S.SEM_EINVAL
    assert not h.value
    # null handle everywhere
    assert L.sem_ax(None, None, None, 1.0, 0.0, None, None) == S.SEM_EINVAL
    assert L.sem_gs(None, None, S.SEM_GS_ADD, None) == S.SEM_EINVAL
    o = S.Sem.default_opts()
    assert L.sem_pcg_solve(None, None, None, ctypes.byref(o), None, None) == S.SEM_EINVAL
    assert L.sem_free(None) == 0
    assert L.sem_rhs(None, None, None, None) == S.SEM_EINVAL
    assert L.sem_adjoint(None, None, None, ctypes.byref(o), None, None, None, None, None) == S.SEM_EINVAL
    assert L.sem_grad_k(None, None, None, 1.0, None, None) == S.SEM_EINVAL
    assert L.sem_ax_level(None, 0, 0, None, None, 1.0, 0.0, None) == S.SEM_EINVAL
    assert L.sem_gs_level(None, 0, 0, None, None) == S.SEM_EINVAL
    assert L.sem_ax_multi(None, 3, None, None, 10, 1.0, 0.0, None) == S.SEM_EINVAL
    assert L.sem_gs_multi(None, 3, None, 10, None) == S.SEM_EINVAL
    assert L.sem_ax_level_multi(None, 0, 0, 3, None, None, 10, 1.0, 0.0, None) == S.SEM_EINVAL
    assert L.sem_gs_level_multi(None, 0, 0, 3, None, 10, None) == S.SEM_EINVAL
    assert L.sem_pcg_solve_multi(None, 3, None, None, 10, ctypes.byref(o), None, None) == S.SEM_EINVAL
    assert L.sem_proj_reset(None) == S.SEM_EINVAL
    assert L.sem_advect_setup(None, 0, 0, None, None) == S.SEM_EINVAL
    assert L.sem_advect_velocity(None, None, 10, None, None) == S.SEM_EINVAL
    assert L.sem_advect(None, None, 1, None, 10, None, 10, None) == S.SEM_EINVAL
    info = S.SemInfo()
    assert L.sem_info(None, 0, ctypes.byref(info)) == S.SEM_EINVAL


def test_default_solver_options():
    o = S.Sem.default_opts()
    assert (o.h1, o.h2, o.tol, o.maxit, o.precond, o.cheb_degree, o.lanczos_steps) == \
        (1.0, 0.0, 1e-8, 1000, S.SEM_PRECOND_JACOBI, 2, 20)
    assert (o.coarse_tol, o.coarse_maxit) == (1e-2, 20)
    assert (o.cheb_lo, o.cheb_hi, o.zero_guess, o.proj_dim) == (0.1, 1.1, 1, 0)
    assert (o.smoother, o.use_graphs) == (S.SEM_SMOOTH_JACOBI, 0)


def test_binding_constants_match_header():
    """The limits the binding states are the header's."""
    txt = open(HEADER).read()
    for name in ("SEM_MAX_RHS", "SEM_MAX_PROJ", "SEM_NOALLOC_MAX_LOCAL"):
        m = re.search(r"#define\s+" + name + r"\s+(\d+)", txt)
        assert m and int(m.group(1)) == getattr(S, name), name
    for name in ("SEM_F64", "SEM_F32", "SEM_GS_ADD", "SEM_GS_MUL", "SEM_GS_MIN", "SEM_GS_MAX",
                 "SEM_PRECOND_JACOBI", "SEM_PRECOND_PMG", "SEM_SMOOTH_JACOBI", "SEM_SMOOTH_ASM",
                 "SEM_SMOOTH_RAS", "SEM_ADVECT_AUTO", "SEM_ADVECT_2D", "SEM_ADVECT_3D"):
        m = re.search(r"\b" + name + r"\s*=\s*(\d+)", txt)
        assert m and int(m.group(1)) == getattr(S, name), name
