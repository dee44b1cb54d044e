"""Seeded synthetic inputs shared by the HIP path's tests, the benchmark and the
CPU oracle.

This module holds none of the method's arithmetic: no quadrature, no
differentiation, no geometric factors, no assembly.  It places given reference
points into a box of hexahedral elements, perturbs them, numbers them with
structured global pointers, and draws seeded random vectors.  Random numbers
are generated here once and handed to both sides as inputs.

Array layout everywhere: an element-local field is indexed [e][k][j][i] with i
fastest; element e = ex + Ex*(ey + Ey*ez).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class BoxMesh:
    """Node coordinates, global pointers and Dirichlet flags of a box mesh.

    x, y, z   : float64 [E, nq, nq, nq]  node coordinates (nq = N + 1)
    gid       : int64   [E, nq, nq, nq]  global pointer, >= 1; 0 = singleton
    dirichlet : uint8   [E, nq, nq, nq]  1 on copies of boundary nodes
    """

    N: int
    shape: tuple
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    gid: np.ndarray
    dirichlet: np.ndarray

    @property
    def E(self) -> int:
        return int(self.x.shape[0])

    @property
    def nq(self) -> int:
        return self.N + 1

    @property
    def n_local(self) -> int:
        return int(self.x.size)

    @property
    def n_unique(self) -> int:
        ex, ey, ez = self.shape
        N = self.N
        return (ex * N + 1) * (ey * N + 1) * (ez * N + 1)


def cyclic_perturbation(x, y, z, amp):
    """Node perturbation x += a sin(2 pi y) sin(2 pi z) and its two cyclic
    permutations, applied simultaneously to the undeformed coordinates."""
    s = lambda v: np.sin(2.0 * math.pi * v)
    return (x + amp * s(y) * s(z), y + amp * s(z) * s(x), z + amp * s(x) * s(y))


def box_mesh(ex: int, ey: int, ez: int, nodes_1d, L=(1.0, 1.0, 1.0), origin=(0.0, 0.0, 0.0),
             deform: str | None = None, amp: float = 0.05, bc: str = "dirichlet",
             interior_zero: bool = False) -> BoxMesh:
    """Box [o, o+L] split into ex*ey*ez equal hexahedra with nq = len(nodes_1d)
    points per direction.  ``nodes_1d`` are the caller's reference points on
    [-1, 1] (its own GLL nodes), so no quadrature rule lives here.

    deform: None (affine elements) or "cyclic" (cyclic_perturbation, amp).
    bc: "dirichlet" flags every copy of a node on the box boundary (decided on
        the structured index, not on the perturbed coordinates); "neumann"
        flags nothing.
    interior_zero: give element-interior copies global pointer 0 (singletons).
    """
    r = np.asarray(nodes_1d, dtype=np.float64)
    nq = r.size
    N = nq - 1
    if N < 1:
        raise ValueError("need at least two points per direction")
    E = ex * ey * ez
    hx, hy, hz = L[0] / ex, L[1] / ey, L[2] / ez
    e_idx = np.arange(E)
    exi = e_idx % ex
    eyi = (e_idx // ex) % ey
    ezi = e_idx // (ex * ey)
    t = 0.5 * (r + 1.0)  # in [0, 1]
    # broadcast shapes: [E, k, j, i]
    X = origin[0] + (exi[:, None, None, None] + t[None, None, None, :]) * hx
    Y = origin[1] + (eyi[:, None, None, None] + t[None, None, :, None]) * hy
    Z = origin[2] + (ezi[:, None, None, None] + t[None, :, None, None]) * hz
    X, Y, Z = np.broadcast_arrays(X, Y, Z)
    X, Y, Z = X.copy(), Y.copy(), Z.copy()
    # with nodes_1d[0] = -1 and nodes_1d[N] = 1, t is exactly 0 and 1 at the
    # element ends, so copies of a shared node get bit-identical coordinates.
    if deform == "cyclic":
        X, Y, Z = cyclic_perturbation(X, Y, Z, amp)
    elif deform not in (None, "none"):
        raise ValueError(f"unknown deformation {deform!r}")

    ii = np.arange(nq)
    gx = (exi[:, None, None, None] * N + ii[None, None, None, :])
    gy = (eyi[:, None, None, None] * N + ii[None, None, :, None])
    gz = (ezi[:, None, None, None] * N + ii[None, :, None, None])
    gx, gy, gz = np.broadcast_arrays(gx, gy, gz)
    nx, ny = ex * N + 1, ey * N + 1
    gid = (1 + gx + nx * (gy + ny * gz)).astype(np.int64)
    if bc == "dirichlet":
        dir_ = ((gx == 0) | (gx == ex * N) | (gy == 0) | (gy == ey * N)
                | (gz == 0) | (gz == ez * N)).astype(np.uint8)
    elif bc == "neumann":
        dir_ = np.zeros(gid.shape, dtype=np.uint8)
    else:
        raise ValueError(f"unknown bc {bc!r}")
    if interior_zero and N >= 2:
        inner = np.zeros((nq, nq, nq), dtype=bool)
        inner[1:N, 1:N, 1:N] = True
        gid = gid.copy()
        gid[:, inner] = 0
    return BoxMesh(N=N, shape=(ex, ey, ez), x=np.ascontiguousarray(X), y=np.ascontiguousarray(Y),
                   z=np.ascontiguousarray(Z), gid=np.ascontiguousarray(gid),
                   dirichlet=np.ascontiguousarray(dir_))


def uniform_lvector(n_local: int, seed: int, low: float = -1.0, high: float = 1.0) -> np.ndarray:
    """iid uniform[low, high] value per local copy (unassembled L-vector)."""
    return np.random.default_rng(seed).uniform(low, high, size=n_local)


def gaussian_per_node(gid: np.ndarray, seed: int) -> np.ndarray:
    """iid N(0, 1) value per global node, replicated to every copy of it.
    Values are drawn for the distinct nonzero pointers in ascending order, then
    for the pointer-0 copies in local order."""
    g = np.asarray(gid).reshape(-1)
    rng = np.random.default_rng(seed)
    nz = g != 0
    uniq, inv = np.unique(g[nz], return_inverse=True)
    vals = rng.standard_normal(uniq.size)
    out = np.empty(g.size)
    out[nz] = vals[inv]
    out[~nz] = rng.standard_normal(int((~nz).sum()))
    return out


def fourier_modes(kmax: int = 4, seed: int = 40):
    """Integer wave vectors kappa != 0 with |kappa| <= kmax, one per +-pair
    (first nonzero component positive), with N(0,1) cosine and sine
    amplitudes from default_rng(seed)."""
    ks = []
    r = range(-kmax, kmax + 1)
    for a in r:
        for b in r:
            for c in r:
                if a * a + b * b + c * c == 0 or a * a + b * b + c * c > kmax * kmax:
                    continue
                first = a if a != 0 else (b if b != 0 else c)
                if first > 0:
                    ks.append((a, b, c))
    ks = np.array(ks, dtype=np.float64)
    rng = np.random.default_rng(seed)
    amp_c = rng.standard_normal(len(ks))
    amp_s = rng.standard_normal(len(ks))
    return ks, amp_c, amp_s


def fourier_field(x, y, z, kmax: int = 4, seed: int = 40) -> np.ndarray:
    """Smooth random field g = sum_kappa (a cos 2pi kappa.x + b sin 2pi kappa.x)/sqrt(M)
    evaluated at the given coordinates (any shape)."""
    ks, ac, as_ = fourier_modes(kmax, seed)
    X = np.stack([np.asarray(x).reshape(-1), np.asarray(y).reshape(-1), np.asarray(z).reshape(-1)], 1)
    ph = 2.0 * math.pi * (X @ ks.T)
    g = (np.cos(ph) @ ac + np.sin(ph) @ as_) / math.sqrt(len(ks))
    return g.reshape(np.asarray(x).shape)


def sin3(x, y, z) -> np.ndarray:
    """u = sin(pi x) sin(pi y) sin(pi z); -lap u = 3 pi^2 u."""
    return np.sin(math.pi * x) * np.sin(math.pi * y) * np.sin(math.pi * z)


def vortex_velocity(x, y, z):
    """A divergence-free velocity tangential to the faces of the unit cube (a
    Taylor-Green-type vortex), returned as a [3, ...] array:
    (sin pi x cos pi y cos pi z, cos pi x sin pi y cos pi z,
     -2 cos pi x cos pi y sin pi z)."""
    px, py, pz = (math.pi * np.asarray(a, dtype=np.float64) for a in (x, y, z))
    return np.stack([np.sin(px) * np.cos(py) * np.cos(pz),
                     np.cos(px) * np.sin(py) * np.cos(pz),
                     -2.0 * np.cos(px) * np.cos(py) * np.sin(pz)])


def load_sequence(gid: np.ndarray, n_steps: int, seed: int = 60, period: float = 40.0,
                  eps: float = 1e-3):
    """Loads f_n for a sequence of solves with slowly varying right-hand sides
    (a stand-in for successive time steps): fields g0, g1, g2 and a fresh h_n
    per step from gaussian_per_node (seeds seed, seed+1, seed+2, seed+3+n),
        f_n = g0 + sin(2 pi n / period) g1 + (n / period)^2 g2 + eps h_n,
    n = 0 .. n_steps-1 (the eps term keeps the loads out of any fixed
    low-dimensional span)."""
    g0, g1, g2 = (gaussian_per_node(gid, seed + i) for i in range(3))
    out = []
    for n in range(n_steps):
        t = n / period
        f = g0 + np.sin(2.0 * np.pi * t) * g1 + t * t * g2
        if eps != 0.0:
            f = f + eps * gaussian_per_node(gid, seed + 3 + n)
        out.append(f)
    return out
