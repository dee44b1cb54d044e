"""Projection of initial guesses onto the solutions of earlier right-hand sides.

TEST INFRASTRUCTURE (see the package docstring).  Plain FP64 numpy over
replicated L-vectors with the W-weighted inner product of `solvers.Level`.

The method is the one the NekRS paper uses for its pressure solves in time
(Sec. 3.4 and Sec. 4, citing Fischer, "Projection techniques for iterative
solution of Ax = b with successive right-hand sides", Comput. Methods Appl.
Mech. Engrg. 163, 1998).  The paper gives no formulas; this follows the
published algorithm:

  space   l <= L vectors xt_1 .. xt_l, orthonormal in the A inner product
          ((xt_i, A xt_j)_W = delta_ij), and bt_i = A xt_i kept beside them;
  project for a new b:  alpha_i = (xt_i, b)_W,  xbar = sum_i alpha_i xt_i
          (the best approximation of A^{-1} b from the span in the A-norm),
          b' = b - sum_i alpha_i bt_i  (= b - A xbar);
  solve   A dx = b' until ||b' - A dx||_W <= tol ||b||_W (the tolerance stays
          relative to the original right-hand side);  x = xbar + dx;
  update  if l < L: A-orthogonalise dx against the space by classical
          Gram-Schmidt (gamma_i = (xt_i, A dx)_W), normalise in the A-norm and
          append it (skipped when nothing new is left);  if l = L: restart
          the space from the single vector x / ||x||_A.
"""
from __future__ import annotations

import math

import numpy as np

from .solvers import Level


class Projection:
    def __init__(self, lv: Level, max_vectors: int):
        if max_vectors < 1:
            raise ValueError("max_vectors >= 1")
        self.lv = lv
        self.L = max_vectors
        self.xt: list[np.ndarray] = []
        self.bt: list[np.ndarray] = []

    @property
    def size(self):
        return len(self.xt)

    def project(self, b):
        """(xbar, b') for right-hand side b."""
        b = np.asarray(b, dtype=np.float64).reshape(-1)
        xbar = np.zeros_like(b)
        bp = b.copy()
        for xt, bt in zip(self.xt, self.bt):
            a = self.lv.dot(xt, b)
            xbar += a * xt
            bp -= a * bt
        return xbar, bp

    def update(self, x, dx):
        """Grow the space by dx (or restart it from x when full)."""
        lv = self.lv
        if self.size >= self.L:
            ax = lv.apply(x)
            nu = math.sqrt(max(lv.dot(x, ax), 0.0))
            self.xt, self.bt = [], []
            if nu > 0.0:
                self.xt.append(x / nu)
                self.bt.append(ax / nu)
            return
        w = lv.apply(dx)
        gam = [lv.dot(xt, w) for xt in self.xt]
        v = np.array(dx, dtype=np.float64)
        bv = w.copy()
        for g, xt, bt in zip(gam, self.xt, self.bt):
            v -= g * xt
            bv -= g * bt
        nu2 = lv.dot(v, bv)
        if not nu2 > 1e-28 * max(lv.dot(dx, w), 1e-300):
            return  # dx already lies in the space
        nu = math.sqrt(nu2)
        self.xt.append(v / nu)
        self.bt.append(bv / nu)

    def solve(self, b, inner, tol):
        """x for A x = b: projection, inner solve of the remainder, update.

        inner(bp, tol_rel) -> (dx, iters) must solve A dx = bp to
        ||bp - A dx||_W <= tol_rel ||bp||_W.  Returns (x, iters, xbar)."""
        lv = self.lv
        b = np.asarray(b, dtype=np.float64).reshape(-1)
        xbar, bp = self.project(b)
        nb, nbp = lv.norm(b), lv.norm(bp)
        if nb == 0.0 or nbp <= tol * nb:
            dx, it = np.zeros_like(b), 0
        else:
            dx, it = inner(bp, tol * nb / nbp)
        x = xbar + dx
        self.update(x, dx)
        return x, it, xbar
