"""Structured Q2 hexahedral mesh of the PML-truncated box (oracle).

Geometry (Fig. 3, Sec. 2): interior box Omega^RD = [-Lx/2, Lx/2] x
[-Ly/2, Ly/2] x [-Lz, 0] (z up, free surface z = 0), surrounded by a PML of
``npml_side`` elements on +-x, +-y and ``npml_bottom`` elements below.
Dirichlet condition u = 0 on the outer sides and bottom of the PML (2c).

Unknowns (Sec. 2 after (5a)): displacements on every node of the closed
domain except the Dirichlet nodes, and six symmetric stress components on
every node of the closed PML (the paper's counts in Sec. 4.2 and Sec. 4.5 are
reproduced by exactly this convention).  History unknowns (5b): the PML part
of d.

Everything here is computed by brute force: element membership is decided
from element-centre coordinates and node classes by marking the nodes of
each element.
"""
from __future__ import annotations

import numpy as np

from . import lgl

# Voigt order of the six stress components: (a, b) index pairs.
VOIGT = ((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))


class Mesh:
    def __init__(self, prob):
        self.prob = prob
        ex, ey, ez = prob.ne_int
        ps, pb, h = prob.npml_side, prob.npml_bottom, prob.h
        self.h = h
        self.Lx, self.Ly, self.Lz = ex * h, ey * h, ez * h
        self.Lpx, self.Lpy, self.Lpz = ps * h, ps * h, pb * h
        Ex, Ey, Ez = ex + 2 * ps, ey + 2 * ps, ez + pb
        self.E = (Ex, Ey, Ez)
        NX, NY, NZ = 2 * Ex + 1, 2 * Ey + 1, 2 * Ez + 1
        self.N = (NX, NY, NZ)
        self.n_nodes = NX * NY * NZ

        # node coordinates
        x = -(0.5 * self.Lx + self.Lpx) + 0.5 * h * np.arange(NX)
        y = -(0.5 * self.Ly + self.Lpy) + 0.5 * h * np.arange(NY)
        z = -(self.Lz + self.Lpz) + 0.5 * h * np.arange(NZ)
        gz, gy, gx = np.meshgrid(z, y, x, indexing="ij")
        self.xyz = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1)
        gk, gj, gi = np.meshgrid(np.arange(NZ), np.arange(NY), np.arange(NX),
                                 indexing="ij")
        self.ijk = np.stack([gi.ravel(), gj.ravel(), gk.ravel()], axis=1)

        # elements (x-fastest), connectivity with local node A = a + 3b + 9c
        ea, eb, ec = [v.ravel() for v in np.meshgrid(
            np.arange(Ex), np.arange(Ey), np.arange(Ez), indexing="ij")]
        order = np.lexsort((ea, eb, ec))
        ea, eb, ec = ea[order], eb[order], ec[order]
        la, lb, lc = np.meshgrid(np.arange(3), np.arange(3), np.arange(3),
                                 indexing="ij")
        la, lb, lc = la.transpose(2, 1, 0).ravel(), lb.transpose(2, 1, 0).ravel(), \
            lc.transpose(2, 1, 0).ravel()
        # local A = a + 3b + 9c  (check: la[A] == A % 3)
        A = np.arange(27)
        assert np.all(la == A % 3) and np.all(lb == (A // 3) % 3) and np.all(lc == A // 9)
        gi_ = 2 * ea[:, None] + la[None, :]
        gj_ = 2 * eb[:, None] + lb[None, :]
        gk_ = 2 * ec[:, None] + lc[None, :]
        self.conn = gi_ + NX * (gj_ + NY * gk_)
        self.n_elem = self.conn.shape[0]
        centre = self.xyz[self.conn[:, 13]]
        tol = 1e-9 * h
        self.is_rd = ((np.abs(centre[:, 0]) < 0.5 * self.Lx - tol) &
                      (np.abs(centre[:, 1]) < 0.5 * self.Ly - tol) &
                      (centre[:, 2] > -self.Lz + tol))
        self.is_pml = ~self.is_rd

        # node classes
        ii, jj, kk = self.ijk.T
        self.dirichlet = (ii == 0) | (ii == NX - 1) | (jj == 0) | (jj == NY - 1) | (kk == 0)
        self.in_pml = np.zeros(self.n_nodes, bool)
        self.in_pml[self.conn[self.is_pml].ravel()] = True
        self.in_rd = np.zeros(self.n_nodes, bool)
        self.in_rd[self.conn[self.is_rd].ravel()] = True

        # LGL rule and element quadrature weights w_q |J|
        xi, w1, D = lgl.rule(2)
        self.xi1, self.w1, self.D1 = xi, w1, D
        self.wq = (w1[la] * w1[lb] * w1[lc]) * (0.5 * h) ** 3
        self.local = np.stack([la, lb, lc], axis=1)

        # lumped masses: sum of w_q|J| over elements of each kind containing j
        self.m_rd = np.zeros(self.n_nodes)
        np.add.at(self.m_rd, self.conn[self.is_rd].ravel(),
                  np.tile(self.wq, int(self.is_rd.sum())))
        self.m_p = np.zeros(self.n_nodes)
        np.add.at(self.m_p, self.conn[self.is_pml].ravel(),
                  np.tile(self.wq, int(self.is_pml.sum())))

        # degree-of-freedom numbering
        free = ~self.dirichlet
        self.u_node = np.nonzero(free)[0]
        self.n_u = 3 * self.u_node.size
        self.u_dof = -np.ones((self.n_nodes, 3), np.int64)
        self.u_dof[self.u_node] = 3 * np.arange(self.u_node.size)[:, None] + np.arange(3)
        self.s_node = np.nonzero(self.in_pml)[0]
        self.n_s = 6 * self.s_node.size
        self.s_dof = -np.ones((self.n_nodes, 6), np.int64)
        self.s_dof[self.s_node] = self.n_u + 6 * np.arange(self.s_node.size)[:, None] + np.arange(6)
        self.n_state = self.n_u + self.n_s
        # history: the PML part of d (5b)
        hist_u = self.u_dof[self.in_pml & free].ravel()
        hist_s = self.s_dof[self.s_node].ravel()
        self.hist_dofs = np.sort(np.concatenate([hist_u, hist_s]))
        self.n_hist = self.hist_dofs.size

        # interior-closure (material) grid
        self.NI = tuple(2 * e + 1 for e in prob.ne_int)
        self.n_int_nodes = int(np.prod(self.NI))

    # ------------------------------------------------------------------
    def material_index(self):
        """Interior-closure id of every full-grid node.

        PML nodes take the value of their projection onto the closed
        interior box (the material at the interface is carried outward,
        Sec. 3.1.3 and Sec. 4.1).
        """
        h2 = 0.5 * self.h
        p = self.xyz.copy()
        p[:, 0] = np.clip(p[:, 0], -0.5 * self.Lx, 0.5 * self.Lx)
        p[:, 1] = np.clip(p[:, 1], -0.5 * self.Ly, 0.5 * self.Ly)
        p[:, 2] = np.clip(p[:, 2], -self.Lz, 0.0)
        jx = np.rint((p[:, 0] + 0.5 * self.Lx) / h2).astype(np.int64)
        jy = np.rint((p[:, 1] + 0.5 * self.Ly) / h2).astype(np.int64)
        jz = np.rint((p[:, 2] + self.Lz) / h2).astype(np.int64)
        NIX, NIY, _ = self.NI
        return jx + NIX * (jy + NIY * jz)

    def interior_full_ids(self):
        """Full-grid ids of the interior-closure nodes, in material order."""
        ex, ey, ez = self.prob.ne_int
        ps, pb = self.prob.npml_side, self.prob.npml_bottom
        NIX, NIY, NIZ = self.NI
        gk, gj, gi = np.meshgrid(np.arange(NIZ), np.arange(NIY), np.arange(NIX),
                                 indexing="ij")
        NX, NY, _ = self.N
        return ((gi + 2 * ps) + NX * ((gj + 2 * ps) + NY * (gk + 2 * pb))).ravel()

    def extend(self, field_int):
        """Nodal field on the interior closure -> every full-grid node."""
        return np.asarray(field_int)[self.material_index()]

    def u_nodal(self, vec):
        """u-part of a state vector -> (n_nodes, 3) array (zero at Dirichlet)."""
        out = np.zeros((self.n_nodes, 3) + vec.shape[1:])
        out[self.u_node] = vec[:self.n_u].reshape((-1, 3) + vec.shape[1:])
        return out

    def s_nodal(self, vec):
        out = np.zeros((self.n_nodes, 6) + vec.shape[1:])
        out[self.s_node] = vec[self.n_u:self.n_state].reshape((-1, 6) + vec.shape[1:])
        return out
