"""Regularization terms and the control problem on the closed interior (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 3.1.3 and App. C.  A material field f is the vector of its nodal values
on the closed interior box (x fastest).  Every integral uses the 3x3x3 LGL
rule of each interior brick, so the values of grad f at the rule's points
are linear maps of f, built here as sparse matrices Gx, Gy, Gz with one row
per (brick, point) pair.  With w the point weights w_q |J|:

* Tikhonov (8):  R_TN(f) = 1/2 sum_q w_q |grad f|_q^2,
                 dR_TN/df = sum_d G_d^T (w * G_d f)              (C.1b-c)
* TV (9):        R_TV(f) = sum_q w_q (|grad f|_q^2 + eps)^(1/2),
                 dR_TV/df = sum_d G_d^T (w * G_d f / (|grad f|^2 + eps)^(1/2))
  Reading: the denominator of (C.1d-e) is taken pointwise (as in (17)), and
  the functional carries R instead of the R/2 printed in (9), so that (17) is
  exactly its derivative.
* M~ (C.1a):     with the LGL rule the mass matrix of the basis chi is
                 diagonal, M~_jj = sum of w_q over the points at node j.
* (18):          g = M~^{-1} (g_mis + R g_reg).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .lgl import rule


def point_gradients(prob):
    """(Gx, Gy, Gz, w): sparse (n_pts, n_int) maps of nodal f to d f/dx_d at
    every LGL point of every interior brick, and the point weights."""
    ex, ey, ez = prob.ne_int
    nix, niy = 2 * ex + 1, 2 * ey + 1
    xi, w1, D = rule(2)
    h = prob.h
    rows, cols, vals = ([], [], []), ([], [], []), ([], [], [])
    weights = []
    r = 0
    for bz in range(ez):
        for by in range(ey):
            for bx in range(ex):
                for qz in range(3):
                    for qy in range(3):
                        for qx in range(3):
                            q = (qx, qy, qz)
                            weights.append(w1[qx] * w1[qy] * w1[qz] * (0.5 * h) ** 3)
                            for d in range(3):
                                for a in range(3):
                                    node = list(q)
                                    node[d] = a
                                    j = (2 * bx + node[0]) + nix * ((2 * by + node[1]) + niy * (2 * bz + node[2]))
                                    rows[d].append(r)
                                    cols[d].append(j)
                                    vals[d].append((2.0 / h) * D[q[d], a])
                            r += 1
    n_int = (2 * ex + 1) * (2 * ey + 1) * (2 * ez + 1)
    G = [sp.csr_matrix((vals[d], (rows[d], cols[d])), shape=(r, n_int)) for d in range(3)]
    return G[0], G[1], G[2], np.array(weights)


class Regularizer:
    """Tikhonov / TV values and gradients of nodal fields on one mesh."""

    def __init__(self, prob):
        self.Gx, self.Gy, self.Gz, self.w = point_gradients(prob)
        # M~ (C.1a): the weight of every point lumped on the node it sits on
        ex, ey, ez = prob.ne_int
        nix, niy = 2 * ex + 1, 2 * ey + 1
        n_int = nix * niy * (2 * ez + 1)
        self.mass = np.zeros(n_int)
        r = 0
        for bz in range(ez):
            for by in range(ey):
                for bx in range(ex):
                    for qz in range(3):
                        for qy in range(3):
                            for qx in range(3):
                                j = (2 * bx + qx) + nix * ((2 * by + qy) + niy * (2 * bz + qz))
                                self.mass[j] += self.w[r]
                                r += 1

    def tikhonov(self, f):
        """(value, gradient) of (8) for one field (R factor not included)."""
        gx, gy, gz = self.Gx @ f, self.Gy @ f, self.Gz @ f
        value = 0.5 * np.sum(self.w * (gx * gx + gy * gy + gz * gz))
        grad = self.Gx.T @ (self.w * gx) + self.Gy.T @ (self.w * gy) + self.Gz.T @ (self.w * gz)
        return value, grad

    def total_variation(self, f, eps):
        """(value, gradient) of (9) under the reading above (R factor not included)."""
        gx, gy, gz = self.Gx @ f, self.Gy @ f, self.Gz @ f
        root = np.sqrt(gx * gx + gy * gy + gz * gz + eps)
        value = np.sum(self.w * root)
        c = self.w / root
        grad = self.Gx.T @ (c * gx) + self.Gy.T @ (c * gy) + self.Gz.T @ (c * gz)
        return value, grad

    def finalize(self, g_mis, g_reg, R):
        """(18): g = M~^{-1} (g_mis + R g_reg)."""
        return (g_mis + R * g_reg) / self.mass
