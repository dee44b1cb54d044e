"""Thin Python binding of libsem (include/sem.h).

Argument marshalling only: every step runs in the HIP library.  Device arrays
are torch tensors on the current GPU; the HIP stream is torch's current
stream.  The library must be built (``__graft_entry__.build()`` or
``python -m paper_2104_05829_amd.build``); importing works without it, every
call fails loudly if it is missing.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import inputs

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsem.so")

SEM_OK, SEM_EINVAL, SEM_ENOMEM, SEM_EHIP, SEM_ENOCONV, SEM_EBREAKDOWN, SEM_EMESH = 0, -1, -2, -3, -4, -5, -6
SEM_F64, SEM_F32 = 0, 1
SEM_PRECOND_JACOBI, SEM_PRECOND_PMG = 0, 1
SEM_SMOOTH_JACOBI, SEM_SMOOTH_ASM, SEM_SMOOTH_RAS = 0, 1, 2
SEM_ADVECT_AUTO, SEM_ADVECT_2D, SEM_ADVECT_3D = 0, 1, 2
SEM_GS_ADD, SEM_GS_MUL, SEM_GS_MIN, SEM_GS_MAX = 0, 1, 2, 3
SEM_MAX_RHS = 4
SEM_MAX_PROJ = 16
# largest level-0 L-vector of sem_pcg_solve_noalloc (its static scratch)
SEM_NOALLOC_MAX_LOCAL = 3142880

c_double_p = ctypes.POINTER(ctypes.c_double)


class SemError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(msg)
        self.code = code


class SemMesh(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int), ("E", ctypes.c_int64), ("x", ctypes.c_void_p),
                ("y", ctypes.c_void_p), ("z", ctypes.c_void_p), ("gid", ctypes.c_void_p),
                ("dirichlet", ctypes.c_void_p)]


class SemSetupOpts(ctypes.Structure):
    _fields_ = [("pmg", ctypes.c_int), ("n_levels", ctypes.c_int), ("levels", ctypes.c_int * 4)]


class SemSolveOpts(ctypes.Structure):
    _fields_ = [("h1", ctypes.c_double), ("h2", ctypes.c_double), ("k", ctypes.c_void_p),
                ("tol", ctypes.c_double), ("maxit", ctypes.c_int), ("precond", ctypes.c_int),
                ("check_every", ctypes.c_int), ("cheb_degree", ctypes.c_int),
                ("lanczos_steps", ctypes.c_int), ("cheb_lo", ctypes.c_double),
                ("cheb_hi", ctypes.c_double), ("coarse_tol", ctypes.c_double),
                ("coarse_maxit", ctypes.c_int), ("zero_guess", ctypes.c_int),
                ("proj_dim", ctypes.c_int), ("smoother", ctypes.c_int), ("use_graphs", ctypes.c_int),
                ("timers", ctypes.c_int)]


class SemSolveStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("converged", ctypes.c_int), ("rel_res", ctypes.c_double),
                ("true_rel_res", ctypes.c_double), ("ms_solve", ctypes.c_double),
                ("ms_setup", ctypes.c_double), ("coarse_iters", ctypes.c_int),
                ("proj_vectors", ctypes.c_int), ("proj_rel_res", ctypes.c_double),
                ("ms_ax", ctypes.c_double), ("ms_gs", ctypes.c_double), ("ms_vec", ctypes.c_double),
                ("ms_prec", ctypes.c_double), ("ms_coarse", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class SemInfo(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int), ("E", ctypes.c_int64), ("n_local", ctypes.c_int64),
                ("n_unique", ctypes.c_int64), ("n_shared_copies", ctypes.c_int64),
                ("n_segments", ctypes.c_int64), ("n_levels", ctypes.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


# every symbol the header declares, with its ctypes signature
_VP = ctypes.c_void_p
_SIGS = {
    "sem_setup": (ctypes.c_int, [ctypes.POINTER(SemMesh), ctypes.POINTER(SemSetupOpts), _VP,
                                 ctypes.POINTER(_VP)]),
    "sem_free": (ctypes.c_int, [_VP]),
    "sem_ax": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_double, ctypes.c_double, _VP, _VP]),
    "sem_gs": (ctypes.c_int, [_VP, _VP, ctypes.c_int, _VP]),
    "sem_ax_level": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, _VP, _VP, ctypes.c_double,
                                    ctypes.c_double, _VP]),
    "sem_gs_level": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, _VP, _VP]),
    "sem_ax_multi": (ctypes.c_int, [_VP, ctypes.c_int, _VP, _VP, ctypes.c_int64, ctypes.c_double,
                                    ctypes.c_double, _VP]),
    "sem_gs_multi": (ctypes.c_int, [_VP, ctypes.c_int, _VP, ctypes.c_int64, _VP]),
    "sem_ax_level_multi": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, _VP, _VP,
                                          ctypes.c_int64, ctypes.c_double, ctypes.c_double, _VP]),
    "sem_gs_level_multi": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, _VP,
                                          ctypes.c_int64, _VP]),
    "sem_pcg_solve_multi": (ctypes.c_int, [_VP, ctypes.c_int, _VP, _VP, ctypes.c_int64,
                                           ctypes.POINTER(SemSolveOpts), _VP, _VP]),
    "sem_solve_opts_default": (None, [ctypes.POINTER(SemSolveOpts)]),
    "sem_proj_reset": (ctypes.c_int, [_VP]),
    "sem_schwarz_setup_host": (ctypes.c_int, [ctypes.c_int, ctypes.c_int64, _VP, _VP, _VP, _VP, _VP,
                                              _VP, _VP, _VP]),
    "sem_smoother_apply": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                          ctypes.c_double, _VP, _VP, _VP]),
    "sem_advect_setup": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int), _VP]),
    "sem_advect_velocity": (ctypes.c_int, [_VP, _VP, ctypes.c_int64, _VP, _VP]),
    "sem_advect": (ctypes.c_int, [_VP, _VP, ctypes.c_int, _VP, ctypes.c_int64, _VP, ctypes.c_int64, _VP]),
    "sem_pcg_solve": (ctypes.c_int, [_VP, _VP, _VP, ctypes.POINTER(SemSolveOpts),
                                     ctypes.POINTER(SemSolveStats), _VP]),
    "sem_pmg_apply": (ctypes.c_int, [_VP, _VP, _VP, ctypes.POINTER(SemSolveOpts), _VP]),
    "sem_pcg_solve_noalloc": (ctypes.c_int, [_VP, _VP, _VP, ctypes.POINTER(SemSolveOpts),
                                             ctypes.POINTER(SemSolveStats), _VP]),
    "sem_grad_k": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_double, _VP, _VP]),
    "sem_rhs": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "sem_adjoint": (ctypes.c_int, [_VP, _VP, _VP, ctypes.POINTER(SemSolveOpts), _VP, _VP, _VP,
                                   ctypes.POINTER(SemSolveStats), _VP]),
    "sem_info": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.POINTER(SemInfo)]),
    "sem_get_maps": (ctypes.c_int, [_VP, ctypes.c_int, _VP, _VP, _VP]),
    "sem_get_geometry": (ctypes.c_int, [_VP, ctypes.c_int, _VP, _VP, _VP]),
    "sem_get_weights": (ctypes.c_int, [_VP, ctypes.c_int, _VP, _VP, _VP]),
    "sem_gll": (ctypes.c_int, [ctypes.c_int, _VP, _VP, _VP]),
    "sem_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "sem_last_error": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """Load libsem.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "or python -m paper_2104_05829_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc, what):
    if rc != SEM_OK:
        L = lib()
        raise SemError(rc, f"{what}: {L.sem_strerror(rc).decode()} -- {L.sem_last_error().decode()}")


def gll(N: int):
    """The library's GLL nodes, weights and Dh (host)."""
    xi = np.zeros(N + 1)
    rho = np.zeros(N + 1)
    D = np.zeros((N + 1) * (N + 1))
    _check(lib().sem_gll(N, xi.ctypes.data, rho.ctypes.data, D.ctypes.data), "sem_gll")
    return xi, rho, D.reshape(N + 1, N + 1)


def schwarz_setup_host(N, gid, dirichlet, lengths):
    """Host part of the library's Schwarz setup (numpy in, numpy out):
    (ix [E, ne, ne, ne], S [E, 3, ne, ne], lam [E, 3, ne], cover, weight)."""
    gid = np.ascontiguousarray(gid, dtype=np.int64).reshape(-1)
    nq = N + 1
    E = gid.size // nq ** 3
    ne = N + 3
    dirichlet = None if dirichlet is None else np.ascontiguousarray(dirichlet, dtype=np.uint8).reshape(-1)
    lengths = np.ascontiguousarray(lengths, dtype=np.float64).reshape(E, 3)
    ix = np.zeros((E, ne, ne, ne), dtype=np.int32)
    S = np.zeros((E, 3, ne, ne), dtype=np.float32)
    lam = np.zeros((E, 3, ne), dtype=np.float32)
    cover = np.zeros(gid.size, dtype=np.int32)
    weight = np.zeros(gid.size, dtype=np.float32)
    ptr = lambda a: None if a is None else ctypes.c_void_p(a.ctypes.data)  # noqa: E731
    _check(lib().sem_schwarz_setup_host(N, E, ptr(gid), ptr(dirichlet), ptr(lengths), ptr(ix), ptr(S),
                                        ptr(lam), ptr(cover), ptr(weight)), "sem_schwarz_setup_host")
    return ix, S, lam, cover, weight


def box_mesh(ex, ey, ez, N, **kw) -> inputs.BoxMesh:
    """Box mesh on the library's own GLL nodes (see inputs.box_mesh)."""
    xi, _, _ = gll(N)
    return inputs.box_mesh(ex, ey, ez, xi, **kw)


_T = None
_RAW_STREAM = None


def _torch():
    global _T
    if _T is None:
        import torch
        _T = torch
    return _T


def _stream():
    """Raw pointer (an int) of torch's current HIP stream on the current device."""
    global _RAW_STREAM
    torch = _torch()
    if _RAW_STREAM is None:
        C = torch._C
        if hasattr(C, "_cuda_getCurrentRawStream") and hasattr(C, "_cuda_getDevice"):
            _RAW_STREAM = lambda: C._cuda_getCurrentRawStream(C._cuda_getDevice())  # noqa: E731
        else:
            _RAW_STREAM = lambda: torch.cuda.current_stream().cuda_stream  # noqa: E731
    return _RAW_STREAM()


def _dev_ptr(t, dtype, n, name):
    """Device address of tensor t after checking its placement, dtype,
    layout and size (a plain int, passed as a void pointer)."""
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on the GPU")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} entries, expected {n}")
    return t.data_ptr()


def _dev_batch(t, dtype, n, name):
    """(pointer, nrhs, ld) of a [nrhs, n] device tensor with unit inner stride."""
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on the GPU")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if t.dim() != 2 or t.shape[1] != n or t.stride(1) != 1 or (t.shape[0] > 1 and t.stride(0) < n):
        raise ValueError(f"{name} must be [nrhs, {n}] with rows of unit stride, got shape "
                         f"{tuple(t.shape)} strides {t.stride()}")
    return ctypes.c_void_p(t.data_ptr()), int(t.shape[0]), int(t.stride(0))


class Sem:
    """A libsem handle on the current GPU.

    mesh: an inputs.BoxMesh (or any object with N, E, x, y, z, gid, dirichlet
    host arrays in L-vector layout).  levels: p-multigrid orders, e.g.
    (7, 3, 1); None for no multigrid.
    """

    def __init__(self, mesh, levels=None):
        torch = _torch()
        L = lib()
        self._h = None
        self.N = int(mesh.N)
        nq = self.N + 1
        self._x = np.ascontiguousarray(mesh.x, dtype=np.float64).reshape(-1)
        self._y = np.ascontiguousarray(mesh.y, dtype=np.float64).reshape(-1)
        self._z = np.ascontiguousarray(mesh.z, dtype=np.float64).reshape(-1)
        self._g = np.ascontiguousarray(mesh.gid, dtype=np.int64).reshape(-1)
        dirichlet = getattr(mesh, "dirichlet", None)
        self._d = None if dirichlet is None else np.ascontiguousarray(dirichlet, dtype=np.uint8).reshape(-1)
        self.E = self._x.size // nq ** 3
        self.n_local = self._x.size
        m = SemMesh(self.N, self.E, self._x.ctypes.data, self._y.ctypes.data, self._z.ctypes.data,
                    self._g.ctypes.data, None if self._d is None else self._d.ctypes.data)
        opts = SemSetupOpts(0, 1, (ctypes.c_int * 4)(self.N, 0, 0, 0))
        if levels is not None and len(levels) > 1:
            lv = list(levels) + [0] * (4 - len(levels))
            opts = SemSetupOpts(1, len(levels), (ctypes.c_int * 4)(*lv))
        self.levels = tuple(levels) if levels is not None else (self.N,)
        h = ctypes.c_void_p()
        self.device = torch.cuda.current_device()
        try:
            _check(L.sem_setup(ctypes.byref(m), ctypes.byref(opts), _stream(), ctypes.byref(h)),
                   "sem_setup")
        finally:
            # the library copied the mesh; drop the host copies
            del self._x, self._y, self._z, self._g, self._d
        self._h = h
        self.info0 = self.info(0)

    # -- lifecycle --------------------------------------------------------
    def free(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().sem_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def _handle(self):
        if self._h is None or not self._h.value:
            raise RuntimeError("handle freed")
        return self._h

    # -- operator and gather-scatter ---------------------------------------
    def ax(self, u, w=None, h1=1.0, h2=0.0, k=None):
        torch = _torch()
        if w is None:
            w = torch.empty_like(u)
        pu = _dev_ptr(u, torch.float64, self.n_local, "u")
        pw = _dev_ptr(w, torch.float64, self.n_local, "w")
        pk = None if k is None else _dev_ptr(k, torch.float64, self.n_local, "k")
        _check(lib().sem_ax(self._handle(), pu, pw, float(h1), float(h2), pk, _stream()), "sem_ax")
        return w

    _GS_OPS = {"add": SEM_GS_ADD, "mul": SEM_GS_MUL, "min": SEM_GS_MIN, "max": SEM_GS_MAX}

    def gs(self, v, op="add"):
        """Gather-scatter in place: op "add" is QQ^T; "mul", "min", "max" give
        every copy the product / minimum / maximum over its node's copies."""
        torch = _torch()
        pv = _dev_ptr(v, torch.float64, self.n_local, "v")
        code = self._GS_OPS[op] if isinstance(op, str) else int(op)
        _check(lib().sem_gs(self._handle(), pv, code, _stream()), "sem_gs")
        return v

    def ax_level(self, level, u, w=None, h1=1.0, h2=0.0):
        torch = _torch()
        if w is None:
            w = torch.empty_like(u)
        dt = SEM_F64 if u.dtype == torch.float64 else SEM_F32
        n = self.info(level)["n_local"]
        pu = _dev_ptr(u, u.dtype, n, "u")
        pw = _dev_ptr(w, u.dtype, n, "w")
        _check(lib().sem_ax_level(self._handle(), level, dt, pu, pw, float(h1), float(h2), _stream()),
               "sem_ax_level")
        return w

    def gs_level(self, level, v):
        torch = _torch()
        dt = SEM_F64 if v.dtype == torch.float64 else SEM_F32
        n = self.info(level)["n_local"]
        pv = _dev_ptr(v, v.dtype, n, "v")
        _check(lib().sem_gs_level(self._handle(), level, dt, pv, _stream()), "sem_gs_level")
        return v

    def ax_multi(self, U, W=None, h1=1.0, h2=0.0):
        """Operator on the rows of U ([nrhs, n_local] FP64); G read once per batch."""
        torch = _torch()
        if W is None:
            W = torch.empty_like(U)
        pu, nr, ld = _dev_batch(U, torch.float64, self.n_local, "U")
        pw, nrw, ldw = _dev_batch(W, torch.float64, self.n_local, "W")
        if nrw != nr or ldw != ld:
            raise ValueError("U and W must have the same shape and strides")
        _check(lib().sem_ax_multi(self._handle(), nr, pu, pw, ld, float(h1), float(h2), _stream()),
               "sem_ax_multi")
        return W

    def gs_multi(self, V):
        torch = _torch()
        pv, nr, ld = _dev_batch(V, torch.float64, self.n_local, "V")
        _check(lib().sem_gs_multi(self._handle(), nr, pv, ld, _stream()), "sem_gs_multi")
        return V

    def ax_level_multi(self, level, U, W=None, h1=1.0, h2=0.0):
        torch = _torch()
        if W is None:
            W = torch.empty_like(U)
        dt = SEM_F64 if U.dtype == torch.float64 else SEM_F32
        n = self.info(level)["n_local"]
        pu, nr, ld = _dev_batch(U, U.dtype, n, "U")
        pw, nrw, ldw = _dev_batch(W, U.dtype, n, "W")
        if nrw != nr or ldw != ld:
            raise ValueError("U and W must have the same shape and strides")
        _check(lib().sem_ax_level_multi(self._handle(), level, dt, nr, pu, pw, ld, float(h1), float(h2),
                                        _stream()), "sem_ax_level_multi")
        return W

    def gs_level_multi(self, level, V):
        torch = _torch()
        dt = SEM_F64 if V.dtype == torch.float64 else SEM_F32
        n = self.info(level)["n_local"]
        pv, nr, ld = _dev_batch(V, V.dtype, n, "V")
        _check(lib().sem_gs_level_multi(self._handle(), level, dt, nr, pv, ld, _stream()),
               "sem_gs_level_multi")
        return V

    def grad_k(self, u, lam, h1=1.0, out=None):
        torch = _torch()
        if out is None:
            out = torch.empty_like(u)
        _check(lib().sem_grad_k(self._handle(), _dev_ptr(u, torch.float64, self.n_local, "u"),
                                _dev_ptr(lam, torch.float64, self.n_local, "lam"), float(h1),
                                _dev_ptr(out, torch.float64, self.n_local, "gk"), _stream()),
               "sem_grad_k")
        return out

    # -- solver ---------------------------------------------------------
    @staticmethod
    def default_opts() -> SemSolveOpts:
        o = SemSolveOpts()
        lib().sem_solve_opts_default(ctypes.byref(o))
        return o

    def _opts(self, kw):
        torch = _torch()
        o = self.default_opts()
        kw = dict(kw)
        kk = kw.pop("k", None)
        pre = kw.pop("precond", None)
        if pre is not None:
            o.precond = {"jacobi": SEM_PRECOND_JACOBI, "pmg": SEM_PRECOND_PMG}.get(pre, pre)
        smo = kw.pop("smoother", None)
        if smo is not None:
            o.smoother = {"jacobi": SEM_SMOOTH_JACOBI, "asm": SEM_SMOOTH_ASM,
                          "ras": SEM_SMOOTH_RAS}.get(smo, smo)
        for name, val in kw.items():
            if not hasattr(o, name):
                raise TypeError(f"unknown solver option {name}")
            setattr(o, name, val)
        if kk is not None:
            o.k = _dev_ptr(kk, torch.float64, self.n_local, "k")
        return o

    def rhs(self, f, out=None):
        """b = R QQ^T (B f): the assembled load of the weak form."""
        torch = _torch()
        if out is None:
            out = torch.empty_like(f)
        _check(lib().sem_rhs(self._handle(), _dev_ptr(f, torch.float64, self.n_local, "f"),
                             _dev_ptr(out, torch.float64, self.n_local, "b"), _stream()), "sem_rhs")
        return out

    def adjoint(self, u, g, need_grad_k=True, raise_on_error=True, **kw):
        """lam = A^{-1} R QQ^T g, grad_f = B lam, grad_k = -(D lam)^T G (D u).
        Returns (lam, grad_f, grad_k or None, stats, status)."""
        torch = _torch()
        o = self._opts(kw)
        lam = torch.empty_like(u)
        gf = torch.empty_like(u)
        gk = torch.empty_like(u) if need_grad_k else None
        st = SemSolveStats()
        rc = lib().sem_adjoint(self._handle(), _dev_ptr(u, torch.float64, self.n_local, "u"),
                               _dev_ptr(g, torch.float64, self.n_local, "g"), ctypes.byref(o),
                               _dev_ptr(lam, torch.float64, self.n_local, "lam"),
                               _dev_ptr(gf, torch.float64, self.n_local, "grad_f"),
                               None if gk is None else _dev_ptr(gk, torch.float64, self.n_local, "grad_k"),
                               ctypes.byref(st), _stream())
        if raise_on_error and rc not in (SEM_OK, SEM_ENOCONV):
            _check(rc, "sem_adjoint")
        return lam, gf, gk, st.as_dict(), rc

    def solve(self, b, x=None, raise_on_error=True, **kw):
        """Solve R(h1 A(k) + h2 B)R^T x = R b; returns (x, stats dict, status).
        Keyword options are the fields of sem_solve_opts (k as a tensor,
        precond as "jacobi"/"pmg")."""
        torch = _torch()
        o = self._opts(kw)
        if x is None:
            x = torch.zeros_like(b)
            o.zero_guess = 1
        st = SemSolveStats()
        rc = lib().sem_pcg_solve(self._handle(), _dev_ptr(b, torch.float64, self.n_local, "b"),
                                 _dev_ptr(x, torch.float64, self.n_local, "x"), ctypes.byref(o),
                                 ctypes.byref(st), _stream())
        if raise_on_error and rc not in (SEM_OK, SEM_ENOCONV):
            _check(rc, "sem_pcg_solve")
        return x, st.as_dict(), rc

    def pmg_apply(self, r, z=None, **kw):
        """z = M^{-1} r, one application of the p-multigrid preconditioner
        (sem_pmg_apply); keyword options as for solve()."""
        torch = _torch()
        o = self._opts(kw)
        if z is None:
            z = torch.empty_like(r)
        _check(lib().sem_pmg_apply(self._handle(), _dev_ptr(r, torch.float64, self.n_local, "r"),
                                   _dev_ptr(z, torch.float64, self.n_local, "z"), ctypes.byref(o),
                                   _stream()), "sem_pmg_apply")
        return z

    def solve_noalloc(self, b, x, raise_on_error=True, **kw):
        """sem_pcg_solve_noalloc: the Jacobi-PCG of solve() with every buffer
        beyond b and x in the library's static device scratch (x is caller
        storage: the initial guess unless zero_guess, then the solution).
        Returns (x, stats dict, status)."""
        torch = _torch()
        o = self._opts(kw)
        st = SemSolveStats()
        rc = lib().sem_pcg_solve_noalloc(self._handle(), _dev_ptr(b, torch.float64, self.n_local, "b"),
                                         _dev_ptr(x, torch.float64, self.n_local, "x"), ctypes.byref(o),
                                         ctypes.byref(st), _stream())
        if raise_on_error and rc not in (SEM_OK, SEM_ENOCONV):
            _check(rc, "sem_pcg_solve_noalloc")
        return x, st.as_dict(), rc

    def smoother_apply(self, level, r, z=None, smoother="asm", h1=1.0, h2=0.0):
        """z = M^{-1} r for the level's Schwarz smoother (FP32 L-vectors)."""
        torch = _torch()
        n = self.info(level)["n_local"]
        if z is None:
            z = torch.empty_like(r)
        code = {"asm": SEM_SMOOTH_ASM, "ras": SEM_SMOOTH_RAS}.get(smoother, smoother)
        _check(lib().sem_smoother_apply(self._handle(), level, code, float(h1), float(h2),
                                        _dev_ptr(r, torch.float32, n, "r"), _dev_ptr(z, torch.float32, n, "z"),
                                        _stream()), "sem_smoother_apply")
        return z

    # -- dealiased advection ----------------------------------------------
    def advect_setup(self, M=None, variant="auto"):
        """Metric factors for the M-point Gauss rule (None: the smallest rule
        exact for degree 3N) and the element kernel ("auto", "2d", "3d");
        returns M."""
        m = ctypes.c_int(0)
        code = {"auto": SEM_ADVECT_AUTO, "2d": SEM_ADVECT_2D, "3d": SEM_ADVECT_3D}.get(variant, variant)
        _check(lib().sem_advect_setup(self._handle(), int(M or 0), int(code), ctypes.byref(m), _stream()),
               "sem_advect_setup")
        self.adv_m = int(m.value)
        return self.adv_m

    def advect_velocity(self, C, ct=None):
        """Contravariant weighted velocity [E, 3, M^3] at the Gauss points for
        the velocity C ([3, n_local] FP64, rows x, y, z)."""
        torch = _torch()
        M = getattr(self, "adv_m", 0)
        if not M:
            raise SemError(SEM_EINVAL, "advect_velocity: call advect_setup first")
        pc, nr, ldc = _dev_batch(C, torch.float64, self.n_local, "C")
        if nr != 3:
            raise ValueError("C must have 3 rows (x, y, z components)")
        if ct is None:
            ct = torch.empty((self.E, 3, M ** 3), dtype=torch.float64, device=C.device)
        pt = _dev_ptr(ct, torch.float64, self.E * 3 * M ** 3, "ct")
        _check(lib().sem_advect_velocity(self._handle(), pc, ldc, pt, _stream()), "sem_advect_velocity")
        return ct

    def advect(self, ct, W, out=None):
        """Local dealiased advection of the rows of W ([nf, n_local] or
        [n_local], FP64) by ct (from advect_velocity)."""
        torch = _torch()
        M = getattr(self, "adv_m", 0)
        single = W.dim() == 1
        W2 = W.unsqueeze(0) if single else W
        if out is None:
            out = torch.empty_like(W2)
        O2 = out.unsqueeze(0) if out.dim() == 1 else out
        pw, nf, ldw = _dev_batch(W2, torch.float64, self.n_local, "W")
        po, nfo, ldo = _dev_batch(O2, torch.float64, self.n_local, "out")
        if nfo != nf:
            raise ValueError("W and out must have the same number of rows")
        pt = _dev_ptr(ct, torch.float64, self.E * 3 * M ** 3 if M else None, "ct")
        _check(lib().sem_advect(self._handle(), pt, nf, pw, max(ldw, self.n_local), po,
                                max(ldo, self.n_local), _stream()), "sem_advect")
        return O2[0] if single else O2

    def proj_reset(self):
        """Forget the stored solutions of the projected initial guesses."""
        _check(lib().sem_proj_reset(self._handle()), "sem_proj_reset")

    def solve_multi(self, B, X=None, raise_on_error=True, **kw):
        """nrhs solves with one operator in lockstep (rows of B, [nrhs, n_local],
        nrhs <= SEM_MAX_RHS); returns (X, [stats dict per row], status)."""
        torch = _torch()
        o = self._opts(kw)
        if X is None:
            X = torch.zeros_like(B)
            o.zero_guess = 1
        pb, nr, ld = _dev_batch(B, torch.float64, self.n_local, "B")
        px, nrx, ldx = _dev_batch(X, torch.float64, self.n_local, "X")
        if nrx != nr or ldx != ld:
            raise ValueError("B and X must have the same shape and strides")
        st = (SemSolveStats * max(nr, 1))()
        rc = lib().sem_pcg_solve_multi(self._handle(), nr, pb, px, ld, ctypes.byref(o),
                                       ctypes.cast(st, _VP), _stream())
        if raise_on_error and rc not in (SEM_OK, SEM_ENOCONV):
            _check(rc, "sem_pcg_solve_multi")
        return X, [st[i].as_dict() for i in range(nr)], rc

    # -- introspection ----------------------------------------------------
    def info(self, level=0):
        inf = SemInfo()
        _check(lib().sem_info(self._handle(), level, ctypes.byref(inf)), "sem_info")
        return inf.as_dict()

    def maps(self, level=0):
        torch = _torch()
        inf = self.info(level)
        perm = torch.empty(max(inf["n_shared_copies"], 1), dtype=torch.int32, device="cuda")
        offs = torch.empty(inf["n_segments"] + 1, dtype=torch.int32, device="cuda")
        _check(lib().sem_get_maps(self._handle(), level, ctypes.c_void_p(perm.data_ptr()),
                                  ctypes.c_void_p(offs.data_ptr()), _stream()), "sem_get_maps")
        return perm[: inf["n_shared_copies"]], offs

    def geometry(self, level=0):
        torch = _torch()
        n = self.info(level)["n_local"]
        G = torch.empty(6, n, dtype=torch.float64, device="cuda")
        B = torch.empty(n, dtype=torch.float64, device="cuda")
        _check(lib().sem_get_geometry(self._handle(), level, ctypes.c_void_p(G.data_ptr()),
                                      ctypes.c_void_p(B.data_ptr()), _stream()), "sem_get_geometry")
        return G, B

    def weights(self, level=0):
        torch = _torch()
        n = self.info(level)["n_local"]
        W = torch.empty(n, dtype=torch.float64, device="cuda")
        g = torch.empty(n, dtype=torch.int64, device="cuda")
        _check(lib().sem_get_weights(self._handle(), level, ctypes.c_void_p(W.data_ptr()),
                                     ctypes.c_void_p(g.data_ptr()), _stream()), "sem_get_weights")
        return W, g
