"""Element-by-element (matrix-free) application of the operators (oracle).

Same discrete operators as ``assemble`` -- the weak forms (3a)-(3b) with the
3x3x3 LGL rule -- evaluated element batch by element batch with the dense
reference-gradient table g[Q, A, k] instead of assembled sparse matrices, so
meshes with millions of unknowns fit in memory.  Cross-checked against the
assembled matrices (and their transposes) on small meshes by the tests.

For a state split into (x0, x1, x2) = (history on the PML, d, d'):
  residual(x0, x1, x2) = G x0 + K x1 + C x2
  residual_T3(z)       = (G^T z restricted to the PML, K^T z, C^T z)
Element terms (w = LGL weight times |J|, S symmetric, Voigt (xx,yy,zz,yz,xz,xy)):
  interior u-rows   sum_Q w grad Phi_A : (lam tr(grad u) I + mu (grad u + grad u^T))
  PML u-rows        sum_Q w grad Phi_A : T,   T_ik = sum_L L_kk S^L_ik
  PML S-rows      - w [mu (H + H^T) + lam tr(H) I]_ab,  H_ik = sum_L L_kk d_k u^L_i
with (L, field) = (Le, x2), (Lp, x1), (Lw, x0), plus the diagonal (nodal)
PML terms rho m_p (b, c, d) and m_p (b, c, d), masses rho (m_rd + a m_p), a m_p.
"""
from __future__ import annotations

import numpy as np

from . import pml
from .assemble import reference_gradients
from .mesh import VOIGT, Mesh

_PAIRS = [(a, b) for a, b in VOIGT]


def _sym_from_voigt(S):
    """(..., 6) Voigt -> (..., 3, 3) symmetric tensor."""
    T = np.empty(S.shape[:-1] + (3, 3), dtype=S.dtype)
    for v, (a, b) in enumerate(_PAIRS):
        T[..., a, b] = S[..., v]
        T[..., b, a] = S[..., v]
    return T


class MatFree:
    def __init__(self, prob, rho_int, lam_int, mu_int, chunk=4096):
        self.prob = prob
        self.mesh = m = Mesh(prob)
        self.coef = cf = pml.coefficients_fast(m, prob.pml_alpha0, prob.pml_beta0, prob.pml_m)
        self.rho, self.lam, self.mu = m.extend(rho_int), m.extend(lam_int), m.extend(mu_int)
        self.g = reference_gradients(prob.h)
        self.wq = m.wq
        self.chunk = chunk
        n = m.n_state
        self.n_state = n
        self.hist = m.hist_dofs
        self.n_hist = self.hist.size
        self.n_X = self.n_hist + 2 * n
        # masses and diagonal PML terms (same formulas as the assembled path)
        M = np.zeros(n)
        self.dC, self.dK, self.dG = np.zeros(n), np.zeros(n), np.zeros(n)
        un, sn = m.u_node, m.s_node
        for i in range(3):
            d = m.u_dof[un, i]
            M[d] = self.rho[un] * (m.m_rd[un] + cf["a"][un] * m.m_p[un])
            self.dC[d] = self.rho[un] * m.m_p[un] * cf["b"][un]
            self.dK[d] = self.rho[un] * m.m_p[un] * cf["c"][un]
            self.dG[d] = self.rho[un] * m.m_p[un] * cf["d"][un]
        for v in range(6):
            d = m.s_dof[sn, v]
            M[d] = cf["a"][sn] * m.m_p[sn]
            self.dC[d] = m.m_p[sn] * cf["b"][sn]
            self.dK[d] = m.m_p[sn] * cf["c"][sn]
            self.dG[d] = m.m_p[sn] * cf["d"][sn]
        self.M = M
        self.Minv = 1.0 / M
        self.dG_hist = self.dG[self.hist]
        self.el_rd = np.nonzero(m.is_rd)[0]
        self.el_p = np.nonzero(m.is_pml)[0]
        # node-level dof tables with a trailing "zero" slot for absent dofs
        self.udof = np.where(m.u_dof >= 0, m.u_dof, n)            # (nn, 3)
        self.sdof = np.where(m.s_dof >= 0, m.s_dof, n)            # (nn, 6)

    # ------------------------------------------------------------------
    def _ext(self, v):
        """State vectors (n, s) -> (n+1, s) with a zero row for absent dofs."""
        return np.concatenate([v, np.zeros((1,) + v.shape[1:])], axis=0)

    def _scatter(self, out, dofs, vals):
        """out[dofs] += vals, skipping absent dofs (== n_state)."""
        d = dofs.ravel()
        keep = d < self.n_state
        ns = vals.shape[-1]
        v = vals.reshape(-1, ns)[keep]
        for s in range(ns):
            out[:, s] += np.bincount(d[keep], weights=v[:, s], minlength=self.n_state)

    def _grad(self, uel):
        """uel (E, 27, 3, s) -> grad (E, 27 points, 3 comps, 3 dirs, s)."""
        return np.einsum("qak,eais->eqiks", self.g, uel, optimize=True)

    def _div(self, Tq):
        """Tq (E, 27 points, 3, 3, s) weighted -> sum_Q g[Q,A,k] T[Q,i,k]: (E, 27, 3, s)."""
        return np.einsum("qak,eqiks->eais", self.g, Tq, optimize=True)

    # ------------------------------------------------------------------
    def residual(self, x0, x1, x2):
        m = self.mesh
        n = self.n_state
        ns = x1.shape[1]
        out = np.zeros((n, ns))
        x0f = np.zeros((n, ns))
        x0f[self.hist] = x0
        X0, X1, X2 = self._ext(x0f), self._ext(x1), self._ext(x2)
        wq = self.wq
        for s in range(0, self.el_rd.size, self.chunk):
            nodes = m.conn[self.el_rd[s:s + self.chunk]]
            ud = self.udof[nodes]                                  # (E, 27, 3)
            G = self._grad(X1[ud])
            la, mu = self.lam[nodes], self.mu[nodes]
            tr = np.einsum("eqiis->eqs", G)
            sig = mu[..., None, None, None] * (G + np.swapaxes(G, 2, 3))
            sig += (la[..., None] * tr)[:, :, None, None, :] * np.eye(3)[None, None, :, :, None]
            F = self._div(wq[None, :, None, None, None] * sig)
            self._scatter(out, ud, F)
        Ls = (("Le", X2), ("Lp", X1), ("Lw", X0))
        for s in range(0, self.el_p.size, self.chunk):
            nodes = m.conn[self.el_p[s:s + self.chunk]]
            ud, sd = self.udof[nodes], self.sdof[nodes]
            la, mu = self.lam[nodes], self.mu[nodes]
            T = 0.0
            H = 0.0
            for key, Xf in Ls:
                Lam = self.coef[key][nodes]                        # (E, 27, 3) at the points
                S = _sym_from_voigt(np.moveaxis(Xf[sd], -1, 2))   # (E, 27, s, 3, 3)
                S = np.moveaxis(S, 2, -1)                          # (E, 27, 3, 3, s)
                T = T + S * Lam[:, :, None, :, None]               # T_ik = S_ik L_kk
                H = H + self._grad(Xf[ud]) * Lam[:, :, None, :, None]
            F = self._div(wq[None, :, None, None, None] * T)
            self._scatter(out, ud, F)
            tr = np.einsum("eqiis->eqs", H)
            R = np.empty(H.shape[:2] + (6, ns))
            for v, (a, b) in enumerate(_PAIRS):
                R[:, :, v] = mu[..., None] * (H[:, :, a, b] + H[:, :, b, a])
                if a == b:
                    R[:, :, v] += la[..., None] * tr
            R *= -wq[None, :, None, None]
            self._scatter(out, sd, R)
        out += self.dC[:, None] * x2 + self.dK[:, None] * x1
        out += self.dG[:, None] * x0f
        return out

    def residual_T3(self, z):
        """(G^T z on the history dofs, K^T z, C^T z) for a state vector z."""
        m = self.mesh
        n = self.n_state
        ns = z.shape[1]
        outs = {k: np.zeros((n, ns)) for k in ("Le", "Lp", "Lw")}
        Z = self._ext(z)
        wq = self.wq
        # interior stiffness is symmetric: K_RD^T z = K_RD z
        for s in range(0, self.el_rd.size, self.chunk):
            nodes = m.conn[self.el_rd[s:s + self.chunk]]
            ud = self.udof[nodes]
            G = self._grad(Z[ud])
            la, mu = self.lam[nodes], self.mu[nodes]
            tr = np.einsum("eqiis->eqs", G)
            sig = mu[..., None, None, None] * (G + np.swapaxes(G, 2, 3))
            sig += (la[..., None] * tr)[:, :, None, None, :] * np.eye(3)[None, None, :, :, None]
            self._scatter(outs["Lp"], ud, self._div(wq[None, :, None, None, None] * sig))
        for s in range(0, self.el_p.size, self.chunk):
            nodes = m.conn[self.el_p[s:s + self.chunk]]
            ud, sd = self.udof[nodes], self.sdof[nodes]
            la, mu = self.lam[nodes], self.mu[nodes]
            Gz = self._grad(Z[ud])                                 # grad z_u at the points
            zS = np.moveaxis(Z[sd], -1, 2)                         # (E, 27, s, 6)
            ZS = np.moveaxis(_sym_from_voigt(zS), 2, -1)           # (E, 27, 3, 3, s)
            trZ = np.einsum("eqiis->eqs", ZS)
            # transpose of the S-rows: P_ik = -w (mu Z~_ik + lam tr(Z) d_ik), Z~ = Z with doubled diagonal
            Zt = ZS + ZS * np.eye(3)[None, None, :, :, None]
            P = mu[:, :, None, None, None] * Zt
            P += (la[..., None] * trZ)[:, :, None, None, :] * np.eye(3)[None, None, :, :, None]
            P *= -wq[None, :, None, None, None]
            for key in ("Le", "Lp", "Lw"):
                Lam = self.coef[key][nodes]
                # u-output: sum_Q g[Q,A,k] L_kk P_ik
                F = self._div(P * Lam[:, :, None, :, None])
                self._scatter(outs[key], ud, F)
                # S-output: w * (sum over the (i,k) pairs of v of L_kk grad z_u[i,k])
                GL = Gz * Lam[:, :, None, :, None]
                R = np.empty(GL.shape[:2] + (6, ns))
                for v, (a, b) in enumerate(_PAIRS):
                    R[:, :, v] = GL[:, :, a, b] + (GL[:, :, b, a] if a != b else 0.0)
                R *= wq[None, :, None, None]
                self._scatter(outs[key], sd, R)
        KT = outs["Lp"] + self.dK[:, None] * z
        CT = outs["Le"] + self.dC[:, None] * z
        GT = (outs["Lw"] + self.dG[:, None] * z)[self.hist]
        return GT, KT, CT


def bench_sample(wl, n_state, fwd_steps=1, adj_steps=1, nsrc=1):
    """Time the oracle on a bounded sample of a workload (host cores).

    Builds the matrix-free operators, runs ``fwd_steps`` forward RK4 steps
    and ``adj_steps`` reverse steps with the gradient terms for the first
    ``nsrc`` sources, and reports DOF-steps/s (n_state * nsrc per forward +
    reverse step pair / seconds).
    """
    import copy
    import os
    import time

    from .solve import Stepper
    wl = copy.copy(wl)
    wl.wavelet, wl.src_node, wl.src_dir = wl.wavelet[:nsrc], wl.src_node[:nsrc], wl.src_dir[:nsrc]
    t0 = time.perf_counter()
    op = MatFree(wl.prob, wl.rho, wl.lam, wl.mu)
    st = Stepper(op, wl.src_node, wl.src_dir, wl.rec_node)
    t_build = time.perf_counter() - t0
    t0 = time.perf_counter()
    X = np.zeros((op.n_X, wl.nsrc))
    states = [X]
    for n in range(fwd_steps):
        X = st.step(X, wl.wavelet, n)
        states.append(X)
    t_fwd = time.perf_counter() - t0
    t0 = time.perf_counter()
    L = np.random.default_rng(0).standard_normal((op.n_X, wl.nsrc))
    gl = np.zeros(op.mesh.n_int_nodes)
    gm = np.zeros_like(gl)
    for n in range(adj_steps - 1, -1, -1):
        Ys, _ = st.stages(states[n], wl.wavelet, n)
        L = st.adjoint_step(L, Ys, gl, gm)
    t_adj = time.perf_counter() - t0
    # forward + (recomputed stages + adjoint) per step, as one fwd+adj DOF-step rate
    per_step = t_fwd / fwd_steps + t_adj / adj_steps
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    return {"value": n_state * wl.nsrc / per_step, "unit": "DOF-steps/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{fwd_steps} forward + {adj_steps} reverse RK4 steps (stage recompute, "
                      f"gradient terms) of source 1 of the workload, matrix-free FP64 oracle; "
                      f"operator setup {t_build:.1f} s excluded",
            "seconds": t_fwd + t_adj}
