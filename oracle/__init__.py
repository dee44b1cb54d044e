"""CPU oracle for the SEM Poisson/Helmholtz hot path (FP64).

TEST INFRASTRUCTURE: only tests, the smoke check and the CPU-baseline leg of
the benchmark may import this package.  It is written from the NekRS paper
(Sec. 2.3 for the operator and gather-scatter, Sec. 3.4 for the multigrid
preconditioner) as plain definitions and shares no code with the HIP library.

The arithmetic kernels live in ``sem_oracle.c`` (explicit loops, built into
``liboracle.so``); the iterations and the dense brute-force check are in
``solvers.py`` and ``dense.py`` (numpy).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "sem_oracle.c")

_lib = None


def build(force: bool = True) -> str:
    """Compile sem_oracle.c into liboracle.so with gcc (plain -O2, FP64,
    no -ffast-math, so the loops are evaluated as written)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        cmd = ["gcc", "-std=gnu11", "-O2", "-fPIC", "-shared", "-fno-fast-math",
               "-ffp-contract=off", _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _SO)
    return _SO


_timing = {}


def build_timing(dest_dir: str) -> str:
    """The same C file built for the all-core CPU timing, not for checking:
    -O3 -march=native (the host it runs on) and OpenMP over the elements of
    oracle_ax; -ffp-contract=off keeps every element's arithmetic that of the
    checked build.  Built into dest_dir on the host that times it."""
    so = os.path.join(dest_dir, "liboracle_omp.so")
    cmd = ["gcc", "-std=gnu11", "-O3", "-march=native", "-fopenmp", "-fPIC", "-shared",
           "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", so, "-lm"]
    subprocess.check_call(cmd)
    return so


def timing_lib(dest_dir: str):
    """ctypes handle of the all-core timing build (see build_timing)."""
    if dest_dir not in _timing:
        _timing[dest_dir] = _bind(ctypes.CDLL(build_timing(dest_dir)))
    return _timing[dest_dir]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        _lib = _bind(ctypes.CDLL(_SO))
    return _lib


def _bind(L):
    d = ctypes.POINTER(ctypes.c_double)
    i64 = ctypes.c_int64
    p64 = ctypes.POINTER(ctypes.c_int64)
    p32 = ctypes.POINTER(ctypes.c_int32)
    L.oracle_gll.argtypes = [ctypes.c_int, d, d]
    L.oracle_dhat.argtypes = [ctypes.c_int, d, d]
    L.oracle_interp.argtypes = [ctypes.c_int, d, ctypes.c_int, d, d]
    L.oracle_geometry.argtypes = [ctypes.c_int, i64, d, d, d, d, d, d, d, d]
    L.oracle_ax.argtypes = [ctypes.c_int, i64, d, d, d, d, ctypes.c_double, ctypes.c_double, d, d]
    L.oracle_diag.argtypes = [ctypes.c_int, i64, d, d, d, d, ctypes.c_double, ctypes.c_double, d]
    L.oracle_qqt.argtypes = [i64, p64, d]
    L.oracle_gs_op.argtypes = [i64, p64, ctypes.c_int, d]
    L.oracle_multiplicity.argtypes = [i64, p64, p32]
    L.oracle_gs_maps.argtypes = [i64, p64, p64, p64, p32, p32]
    L.oracle_grad_k.argtypes = [ctypes.c_int, i64, d, d, ctypes.c_double, d, d, d]
    L.oracle_interp_lvec.argtypes = [ctypes.c_int, ctypes.c_int, i64, d, d, d]
    L.oracle_threads.restype = ctypes.c_int
    return L


def _d(a):
    if a is None:
        return ctypes.cast(None, ctypes.POINTER(ctypes.c_double))
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i64(a):
    assert a.dtype == np.int64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _i32(a):
    if a is None:
        return ctypes.cast(None, ctypes.POINTER(ctypes.c_int32))
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def gll(N: int):
    """GLL nodes and weights (Sec. 2.3)."""
    xi = np.zeros(N + 1)
    rho = np.zeros(N + 1)
    _check(lib().oracle_gll(N, _d(xi), _d(rho)), "gll")
    return xi, rho


def dhat(N: int, xi=None):
    """1D differentiation matrix Dh[i][l] = h_l'(xi_i), eq. (dh)."""
    if xi is None:
        xi, _ = gll(N)
    D = np.zeros((N + 1, N + 1))
    _check(lib().oracle_dhat(N, _d(np.ascontiguousarray(xi)), _d(D)), "dhat")
    return D


def interp_matrix(xs, xt):
    """J[i][j] = h_j(xt_i) for the Lagrange basis on xs."""
    xs = np.ascontiguousarray(xs, dtype=np.float64)
    xt = np.ascontiguousarray(xt, dtype=np.float64)
    J = np.zeros((xt.size, xs.size))
    _check(lib().oracle_interp(xs.size, _d(xs), xt.size, _d(xt), _d(J)), "interp")
    return J


def geometry(N: int, x, y, z, D=None, rho=None, allow_bad: bool = False, _lib=None):
    """Geometric factors G [6, nL] (G11,G12,G13,G22,G23,G33), mass B [nL],
    Jacobian J [nL]; eqs. (grad), (vBu), (gij).  _lib: a timing build."""
    if D is None:
        xi, rho = gll(N)
        D = dhat(N, xi)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1)
    y = np.ascontiguousarray(y, dtype=np.float64).reshape(-1)
    z = np.ascontiguousarray(z, dtype=np.float64).reshape(-1)
    nL = x.size
    E = nL // (N + 1) ** 3
    G = np.zeros((6, nL))
    B = np.zeros(nL)
    J = np.zeros(nL)
    rc = (_lib or lib()).oracle_geometry(N, E, _d(np.ascontiguousarray(D)), _d(np.ascontiguousarray(rho)),
                               _d(x), _d(y), _d(z), _d(G), _d(B), _d(J))
    if rc == -6 and not allow_bad:
        raise ValueError("mesh has a nonpositive Jacobian")
    if rc not in (0, -6):
        _check(rc, "geometry")
    return G, B, J


def ax(N: int, D, G, u, h1: float = 1.0, h2: float = 0.0, B=None, k=None, _lib=None):
    """Unassembled w_L = h1 A_L(k) u_L + h2 B_L u_L, eq. (Ae).  _lib: a
    timing build (timing_lib) instead of the checked one."""
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
    E = u.size // (N + 1) ** 3
    w = np.zeros_like(u)
    kk = None if k is None else np.ascontiguousarray(k, dtype=np.float64).reshape(-1)
    BB = None if B is None else np.ascontiguousarray(B, dtype=np.float64).reshape(-1)
    _check((_lib or lib()).oracle_ax(N, E, _d(np.ascontiguousarray(D)), _d(np.ascontiguousarray(G)), _d(BB),
                           _d(kk), h1, h2, _d(u), _d(w)), "ax")
    return w


def diag(N: int, D, G, h1: float = 1.0, h2: float = 0.0, B=None, k=None):
    """Diagonal of the unassembled h1 A_L(k) + h2 B_L."""
    nL = G.shape[1]
    E = nL // (N + 1) ** 3
    d = np.zeros(nL)
    kk = None if k is None else np.ascontiguousarray(k, dtype=np.float64).reshape(-1)
    BB = None if B is None else np.ascontiguousarray(B, dtype=np.float64).reshape(-1)
    _check(lib().oracle_diag(N, E, _d(np.ascontiguousarray(D)), _d(np.ascontiguousarray(G)), _d(BB),
                             _d(kk), h1, h2, _d(d)), "diag")
    return d


def qqt(gid, v):
    """Return QQ^T v (direct-stiffness summation), eq. (dssum) / gs_op(+)."""
    g = np.ascontiguousarray(gid, dtype=np.int64).reshape(-1)
    out = np.array(v, dtype=np.float64).reshape(-1).copy()
    _check(lib().oracle_qqt(g.size, _i64(g), _d(out)), "qqt")
    return out


GS_OPS = {"add": 0, "mul": 1, "min": 2, "max": 3}


def gs_op(gid, v, op: str = "add"):
    """gs_op(gsh, v, op) of Sec. 3.2: every copy of a shared node receives the
    sum ("add", equal to qqt), product, minimum or maximum of the node's copies
    in ascending local index order (the last three from the first copy)."""
    g = np.ascontiguousarray(gid, dtype=np.int64).reshape(-1)
    out = np.array(v, dtype=np.float64).reshape(-1).copy()
    _check(lib().oracle_gs_op(g.size, _i64(g), GS_OPS[op], _d(out)), "gs_op")
    return out


def multiplicity(gid):
    g = np.ascontiguousarray(gid, dtype=np.int64).reshape(-1)
    m = np.zeros(g.size, dtype=np.int32)
    _check(lib().oracle_multiplicity(g.size, _i64(g), _i32(m)), "multiplicity")
    return m


def gs_maps(gid):
    """(perm, offs): local indices of shared copies sorted by (gid, index),
    segment starts; only pointers held by two or more copies."""
    g = np.ascontiguousarray(gid, dtype=np.int64).reshape(-1)
    nc = np.zeros(1, dtype=np.int64)
    ns = np.zeros(1, dtype=np.int64)
    _check(lib().oracle_gs_maps(g.size, _i64(g), _i64(nc), _i64(ns), _i32(None), _i32(None)), "gs_maps")
    perm = np.zeros(int(nc[0]), dtype=np.int32)
    offs = np.zeros(int(ns[0]) + 1, dtype=np.int32)
    _check(lib().oracle_gs_maps(g.size, _i64(g), _i64(nc), _i64(ns), _i32(perm), _i32(offs)), "gs_maps")
    return perm, offs


def grad_k(N: int, D, G, u, lam, h1: float = 1.0):
    """dL/dk per copy = -h1 sum (D_m lam) G_mm' (D_m' u)."""
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
    lam = np.ascontiguousarray(lam, dtype=np.float64).reshape(-1)
    E = u.size // (N + 1) ** 3
    gk = np.zeros_like(u)
    _check(lib().oracle_grad_k(N, E, _d(np.ascontiguousarray(D)), _d(np.ascontiguousarray(G)), h1,
                               _d(u), _d(lam), _d(gk)), "grad_k")
    return gk


def interp_lvec(J, v, ns: int, nt: int):
    """Elementwise tensor-product interpolation (J (x) J (x) J) of an L-vector."""
    v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1)
    E = v.size // ns ** 3
    out = np.zeros(E * nt ** 3)
    _check(lib().oracle_interp_lvec(ns, nt, E, _d(np.ascontiguousarray(J)), _d(v), _d(out)),
           "interp_lvec")
    return out
