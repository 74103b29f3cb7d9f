"""System matrices M, C, K, G of (5a), read term by term from (3a)-(3b) (oracle).

Every element integral uses the 3x3x3 LGL rule at the element nodes (the
spectral-element choice that makes M diagonal, Sec. 2; used here for all
terms), so material values at quadrature points are the nodal values
(quadratic material approximation, Sec. 4.1).

u-rows (test function w~ = Phi_A e_i), from (3a):
  interior   int grad w~ : {mu[grad u + grad u^T] + lam div u I}         -> K
  PML        int grad w~ : (S'^T Le + S^T Lp + Sbar^T Lw)                 -> C, K, G
  PML        int w~ . rho (a u'' + b u' + c u + d ubar)                   -> M, C, K, G
  interior   int w~ . rho u''                                             -> M
S-rows (test function T~ = Psi_Q E_ab, one equation per symmetric
component ab), from (3b):
  int T~ : (a S'' + b S' + c S + d Sbar)                                  -> M, C, K, G
  - int T~ : mu[(grad u')Le + Le(grad u')^T + ...] + lam[div(Le u') + ...]I
                                                                          -> C, K, G
The six stress unknowns are (xx, yy, zz, yz, xz, xy).  Each S-row is the
component equation for its pair (a, b); scaling the off-diagonal rows by two
(a tensor test function with both E_ab and E_ba) scales M and the rest of
the row alike and leaves the solution, the misfit and its gradient unchanged.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import lgl, pml
from .mesh import VOIGT, Mesh


def reference_gradients(h):
    """g[Q, A, k] = d Phi_A / d x_k at element node Q (physical units)."""
    x, _, _ = lgl.rule(2)
    val, der = lgl.basis_values(2, x)       # val[i, a] = l_a(x_i)
    g = np.zeros((27, 27, 3))
    for Q in range(27):
        qa, qb, qc = Q % 3, (Q // 3) % 3, Q // 9
        for A in range(27):
            a, b, c = A % 3, (A // 3) % 3, A // 9
            g[Q, A, 0] = der[qa, a] * val[qb, b] * val[qc, c]
            g[Q, A, 1] = val[qa, a] * der[qb, b] * val[qc, c]
            g[Q, A, 2] = val[qa, a] * val[qb, b] * der[qc, c]
    return g * (2.0 / h)


def _interior_tables(g):
    """K_e = sum_Q wq [lam_Q Kl[Q] + mu_Q Km[Q]], dofs (A, i) -> 3A + i."""
    eye = np.eye(3)
    Kl = np.einsum("qai,qbj->qaibj", g, g)
    Km = (np.einsum("ij,qan,qbn->qaibj", eye, g, g)
          + np.einsum("qaj,qbi->qaibj", g, g))
    return Kl.reshape(27, 81, 81), Km.reshape(27, 81, 81)


def _pml_tables(g):
    """Coupling patterns of the PML blocks.

    Ruse[A, i, Q, v, k]: coefficient of Lambda_kk(Q) in the u-row (A, i),
    S-column (Q, v) of  grad w~ : (S Lambda).
    Rmu / Rla[Q, v, A, j, k]: coefficient of mu_Q Lambda_kk(Q) / lam_Q
    Lambda_kk(Q) in the S-row (Q, v), u-column (A, j) of
    mu[(grad u)Lambda + Lambda(grad u)^T] + lam tr((grad u)Lambda) I.
    """
    d = np.eye(3)
    Ruse = np.zeros((27, 3, 27, 6, 3))
    Rmu = np.zeros((27, 6, 27, 3, 3))
    Rla = np.zeros((27, 6, 27, 3, 3))
    for v, (a, b) in enumerate(VOIGT):
        for A in range(27):
            for Q in range(27):
                for i in range(3):
                    for k in range(3):
                        if a != b:
                            Ruse[A, i, Q, v, k] = (d[i, a] * d[k, b] * g[Q, A, b]
                                                   + d[i, b] * d[k, a] * g[Q, A, a])
                            Rmu[Q, v, A, i, k] = (d[a, i] * d[k, b] * g[Q, A, b]
                                                  + d[b, i] * d[k, a] * g[Q, A, a])
                        else:
                            Ruse[A, i, Q, v, k] = d[i, a] * d[k, a] * g[Q, A, a]
                            Rmu[Q, v, A, i, k] = 2.0 * d[a, i] * d[k, a] * g[Q, A, a]
                        Rla[Q, v, A, i, k] = (1.0 if a == b else 0.0) * d[k, i] * g[Q, A, i]
    return Ruse.reshape(81, 27, 6, 3), Rmu.reshape(27, 6, 81, 3), Rla.reshape(27, 6, 81, 3)


class System:
    """Assembled semi-discrete system (5a) for one material model.

    Attributes: ``M`` (diagonal, vector over the n_state dofs), sparse
    ``C``, ``K`` (n_state x n_state), ``G`` (n_state x n_hist), ``Krd`` (the
    interior stiffness alone), ``hist`` (dof ids of x0 = d|_PML).
    """

    def __init__(self, prob, rho_int, lam_int, mu_int, chunk=64):
        self.prob = prob
        self.mesh = m = Mesh(prob)
        self.coef = cf = pml.coefficients(m, prob.pml_alpha0, prob.pml_beta0,
                                          prob.pml_m)
        rho = m.extend(rho_int)
        lam = m.extend(lam_int)
        mu = m.extend(mu_int)
        self.rho, self.lam, self.mu = rho, lam, mu
        g = reference_gradients(prob.h)
        self.g = g
        wq = m.wq
        n = m.n_state
        rows, cols, vals = {k: [] for k in "CKGR"}, {k: [] for k in "CKGR"}, \
            {k: [] for k in "CKGR"}

        def add(key, r, c, v):
            keep = (r >= 0) & (c >= 0) & (v != 0.0)
            rows[key].append(r[keep])
            cols[key].append(c[keep])
            vals[key].append(v[keep])

        # ---- interior stiffness K_RD
        Kl, Km = _interior_tables(g)
        el_rd = np.nonzero(m.is_rd)[0]
        for s in range(0, el_rd.size, chunk):
            e = el_rd[s:s + chunk]
            nodes = m.conn[e]                                    # (E, 27)
            Ke = (np.einsum("eq,qxy->exy", wq[None] * lam[nodes], Kl)
                  + np.einsum("eq,qxy->exy", wq[None] * mu[nodes], Km))
            dof = m.u_dof[nodes].reshape(len(e), 81)
            r = np.broadcast_to(dof[:, :, None], Ke.shape)
            c = np.broadcast_to(dof[:, None, :], Ke.shape)
            add("R", r.ravel(), c.ravel(), Ke.ravel())

        # ---- PML coupling blocks
        Ruse, Rmu, Rla = _pml_tables(g)
        el_p = np.nonzero(m.is_pml)[0]
        lam_keys = (("Le", "C"), ("Lp", "K"), ("Lw", "G"))
        for s in range(0, el_p.size, chunk):
            e = el_p[s:s + chunk]
            nodes = m.conn[e]
            udof = m.u_dof[nodes].reshape(len(e), 81)
            sdof = m.s_dof[nodes].reshape(len(e), 162)
            for lk, key in lam_keys:
                Lam = cf[lk][nodes]                               # (E, 27, 3)
                Bus = np.einsum("xqvk,eqk,q->exqv", Ruse, Lam, wq).reshape(len(e), 81, 162)
                add(key, np.broadcast_to(udof[:, :, None], Bus.shape).ravel(),
                    np.broadcast_to(sdof[:, None, :], Bus.shape).ravel(), Bus.ravel())
                Bsu = -(np.einsum("qvyk,eqk,eq,q->eqvy", Rmu, Lam, mu[nodes], wq)
                        + np.einsum("qvyk,eqk,eq,q->eqvy", Rla, Lam, lam[nodes], wq))
                Bsu = Bsu.reshape(len(e), 162, 81)
                add(key, np.broadcast_to(sdof[:, :, None], Bsu.shape).ravel(),
                    np.broadcast_to(udof[:, None, :], Bsu.shape).ravel(), Bsu.ravel())

        # ---- nodal (diagonal) terms
        Mvec = np.zeros(n)
        diag = {k: np.zeros(n) for k in "CKG"}
        un = m.u_node
        for i in range(3):
            dof = m.u_dof[un, i]
            Mvec[dof] = rho[un] * (m.m_rd[un] + cf["a"][un] * m.m_p[un])
            diag["C"][dof] = rho[un] * m.m_p[un] * cf["b"][un]
            diag["K"][dof] = rho[un] * m.m_p[un] * cf["c"][un]
            diag["G"][dof] = rho[un] * m.m_p[un] * cf["d"][un]
        sn = m.s_node
        for v in range(6):
            dof = m.s_dof[sn, v]
            Mvec[dof] = cf["a"][sn] * m.m_p[sn]
            diag["C"][dof] = m.m_p[sn] * cf["b"][sn]
            diag["K"][dof] = m.m_p[sn] * cf["c"][sn]
            diag["G"][dof] = m.m_p[sn] * cf["d"][sn]

        def build(key, extra=None):
            r = np.concatenate(rows[key]) if rows[key] else np.zeros(0, np.int64)
            c = np.concatenate(cols[key]) if cols[key] else np.zeros(0, np.int64)
            v = np.concatenate(vals[key]) if vals[key] else np.zeros(0)
            A = sp.coo_matrix((v, (r, c)), shape=(n, n)).tocsr()
            if extra is not None:
                A = A + sp.diags(extra)
            A.sum_duplicates()
            return A

        self.Krd = build("R")
        self.M = Mvec
        self.Minv = 1.0 / Mvec
        self.C = build("C", diag["C"])
        self.K = (build("K", diag["K"]) + self.Krd).tocsr()
        Gfull = build("G", diag["G"])
        self.hist = m.hist_dofs
        outside = np.setdiff1d(np.arange(n), self.hist)
        assert abs(Gfull[:, outside]).sum() == 0.0, "G acts outside the PML"
        self.G = Gfull[:, self.hist].tocsr()
        self.n_state, self.n_hist = n, self.hist.size
        self.n_X = self.n_hist + 2 * n

    # ------------------------------------------------------------------
    def residual(self, x0, x1, x2):
        """G x0 + K x1 + C x2 (x0 on the history dofs)."""
        return self.G @ x0 + self.K @ x1 + self.C @ x2

    def residual_T3(self, z):
        """(G^T z, K^T z, C^T z); G^T z lives on the history dofs."""
        if not hasattr(self, "_T"):
            self._T = (self.G.T.tocsr(), self.K.T.tocsr(), self.C.T.tocsr())
        GT, KT, CT = self._T
        return GT @ z, KT @ z, CT @ z


def free_box_stiffness(ne, h, lam_fn, mu_fn, rho=1.0):
    """K_RD and the lumped mass on a box of ne = (ex, ey, ez) bricks with
    no boundary condition at all (every node free).

    lam_fn, mu_fn: callables of node coordinates (n, 3) -> (n,).
    Returns (K (sparse, 3 dofs per node, dof = 3*node + i), Mdiag, xyz).
    """
    ex, ey, ez = ne
    NX, NY, NZ = 2 * ex + 1, 2 * ey + 1, 2 * ez + 1
    gz, gy, gx = np.meshgrid(np.arange(NZ), np.arange(NY), np.arange(NX), indexing="ij")
    xyz = 0.5 * h * np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1)
    lam = lam_fn(xyz)
    mu = mu_fn(xyz)
    g = reference_gradients(h)
    Kl, Km = _interior_tables(g)
    _, w1, _ = lgl.rule(2)
    A = np.arange(27)
    la, lb, lc = A % 3, (A // 3) % 3, A // 9
    wq = w1[la] * w1[lb] * w1[lc] * (0.5 * h) ** 3
    rows, cols, vals = [], [], []
    Mdiag = np.zeros(3 * xyz.shape[0])
    for c in range(ez):
        for b in range(ey):
            for a in range(ex):
                nodes = (2 * a + la) + NX * ((2 * b + lb) + NY * (2 * c + lc))
                Ke = (np.einsum("q,qxy->xy", wq * lam[nodes], Kl)
                      + np.einsum("q,qxy->xy", wq * mu[nodes], Km))
                dof = (3 * nodes[:, None] + np.arange(3)).ravel()
                rows.append(np.repeat(dof, 81))
                cols.append(np.tile(dof, 81))
                vals.append(Ke.ravel())
                for i in range(3):
                    Mdiag[3 * nodes + i] += rho * wq
    n = 3 * xyz.shape[0]
    K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    return K, Mdiag, xyz
