"""Time stepping, misfit, adjoint and gradient on the assembled system (oracle).

* ``forward``: classical RK4 on the first-order form (6),
      d/dt [x0; x1; M x2] = [[0, P, 0], [0, 0, I], [-G, -K, -C]] x + [0; 0; f],
  with x0 = d-bar restricted to the PML (5b), starting at rest (Sec. 2), the
  load sampled at t_n, t_n + dt/2 (twice) and t_{n+1}.
* ``misfit``: (7) with the time integral taken by the trapezoid rule over the
  step states n = 0..N (reading: the paper gives the continuous integral).
* ``adjoint_gradient``: the exact derivative of the discrete misfit with
  respect to the nodal Lame parameters of the closed interior (the
  "discretize-then-optimize" gradient of Sec. 4.1).  Reverse-mode sweep of
  the RK4 recurrence, stage by stage, with the transposed operator
  A^T k = (-G^T z, P^T k0 - K^T z, k1 - C^T z), z = M^{-1} k2.
  Following Sec. 3.1.3, only the interior stiffness depends on the
  parameters (the PML keeps the material carried out from the interface),
  so  k^T (dA/dm_j) Y = - z_u^T (dK_RD/dm_j) Y_u , i.e. the LGL-node values
  of div z div u (lambda) and 2 eps(z):eps(u) (mu) as in (C.1f)-(C.1g).
  The output is m-bar = M~ g with R = 0 ((18), (27)): the vector whose dot
  product with a direction is the directional derivative.
* ``adjoint_gradient_appb``: the paper's own reverse-time RK4 for (15), with
  the stages of Appendix B (transposes kept as in (B.2)), forcing f^adj at
  t_n, t_{n-1/2} (linear interpolation of the residual) and t_{n-1}, and the
  time integral of (C.1f)-(C.1g) by the trapezoid rule over the steps.
"""
from __future__ import annotations

import numpy as np


def source_vectors(mesh, n_state, src_node, src_dir):
    """Unit-amplitude nodal force vectors, one column per source."""
    F = np.zeros((n_state, len(src_node)))
    for s, (nd, dv) in enumerate(zip(src_node, src_dir)):
        d = mesh.u_dof[nd]
        assert np.all(d >= 0), "source on a Dirichlet node"
        F[d, s] += dv
    return F


def receiver_dofs(mesh, rec_node):
    d = mesh.u_dof[np.asarray(rec_node)]
    assert np.all(d >= 0), "receiver on a Dirichlet node"
    return d                                    # (nrec, 3)


class Stepper:
    """RK4, misfit and adjoints for an operator object with ``residual``,
    ``residual_T3``, ``Minv``, ``hist``, ``mesh``, ``g`` (the assembled
    ``System`` or the element-batched ``MatFree``)."""

    def __init__(self, system, src_node, src_dir, rec_node, loads=None, full_gradient=False):
        """loads: optional (load_src, load_node, load_vec) list of nodal loads
        (distributed surface tractions, ``oracle.loads``) replacing the point
        loads src_node / src_dir; the number of sources stays len(src_node).
        full_gradient: also differentiate the PML S-rows through the material
        carried from the interface into the PML (chain rule of the
        extension), instead of the interior bricks only (Sec. 3.1.3)."""
        self.full_gradient = full_gradient
        s = system
        self.s = s
        self.dt = s.prob.dt
        self.N = s.prob.nsteps
        self.nh, self.ns = s.n_hist, s.n_state
        if loads is None:
            self.Fsrc = source_vectors(s.mesh, s.n_state, src_node, src_dir)   # (n_state, nsrc)
        else:
            from .loads import load_matrix
            self.Fsrc = load_matrix(s.mesh, s.mesh.u_dof, s.n_state, len(src_node), *loads)
        self.rec = receiver_dofs(s.mesh, rec_node)                          # (nrec, 3)

    # -- X is (n_X, nsrc): [x0 (n_hist); x1 (n_state); x2 (n_state)]
    def split(self, X):
        nh, ns = self.nh, self.ns
        return X[:nh], X[nh:nh + ns], X[nh + ns:]

    def rhs(self, X, f):
        s = self.s
        x0, x1, x2 = self.split(X)
        acc = s.Minv[:, None] * (self.Fsrc * f[None, :] - s.residual(x0, x1, x2))
        return np.concatenate([x1[s.hist], x2, acc], axis=0)

    def rhs_T(self, k):
        """A^T k for the homogeneous part."""
        s = self.s
        k0, k1, k2 = self.split(k)
        z = s.Minv[:, None] * k2
        GT, KT, CT = s.residual_T3(z)
        y0 = -GT
        y1 = -KT
        y1[s.hist] += k0
        y2 = k1 - CT
        return np.concatenate([y0, y1, y2], axis=0)

    def stages(self, X, wav, n):
        dt = self.dt
        f0, fh, f1 = wav[:, 2 * n], wav[:, 2 * n + 1], wav[:, 2 * n + 2]
        Y1 = X
        K1 = self.rhs(Y1, f0)
        Y2 = X + 0.5 * dt * K1
        K2 = self.rhs(Y2, fh)
        Y3 = X + 0.5 * dt * K2
        K3 = self.rhs(Y3, fh)
        Y4 = X + dt * K3
        K4 = self.rhs(Y4, f1)
        return (Y1, Y2, Y3, Y4), (K1, K2, K3, K4)

    def step(self, X, wav, n):
        _, (K1, K2, K3, K4) = self.stages(X, wav, n)
        return X + (self.dt / 6.0) * (K1 + 2 * K2 + 2 * K3 + K4)

    def traces_of(self, X):
        x1 = X[self.nh:self.nh + self.ns]
        return np.moveaxis(x1[self.rec], -1, 0)                  # (nsrc, nrec, 3)

    def forward(self, wav, store=False, nsteps=None):
        N = self.N if nsteps is None else nsteps
        nsrc = wav.shape[0]
        X = np.zeros((self.nh + 2 * self.ns, nsrc))
        tr = np.zeros((nsrc, N + 1, self.rec.shape[0], 3))
        states = [X.copy()] if store else None
        for n in range(N):
            X = self.step(X, wav, n)
            tr[:, n + 1] = self.traces_of(X)
            if store:
                states.append(X.copy())
        return tr, (states if store else X)

    # ------------------------------------------------------------------
    def time_weights(self, N):
        w = np.ones(N + 1)
        w[0] = w[-1] = 0.5
        return w

    def misfit(self, traces, observed):
        N = traces.shape[1] - 1
        r = traces - observed
        w = self.time_weights(N)
        return 0.5 * self.dt * float(np.einsum("n,snrc,snrc->", w, r, r))

    def _grad_pair(self, kap, Y, g_lam, g_mu):
        """g -= z_u^T (dK_RD/dm) Y_u  with z = M^{-1} kap_2, summed over sources."""
        s = self.s
        m = s.mesh
        _, _, k2 = self.split(kap)
        _, y1, _ = self.split(Y)
        z = m.u_nodal(s.Minv[:, None] * k2)                       # (nn, 3, nsrc)
        u = m.u_nodal(y1)
        rd = np.nonzero(m.is_rd)[0]
        nodes = m.conn[rd]                                        # (E, 27)
        gz = np.einsum("qak,eais->eqiks", s.g, z[nodes])          # grad z at nodes
        gu = np.einsum("qak,eais->eqiks", s.g, u[nodes])
        divz = np.einsum("eqiis->eqs", gz)
        divu = np.einsum("eqiis->eqs", gu)
        ez = 0.5 * (gz + np.swapaxes(gz, 2, 3))
        eu = 0.5 * (gu + np.swapaxes(gu, 2, 3))
        pl = np.einsum("q,eqs,eqs->eq", m.wq, divz, divu)
        pm = 2.0 * np.einsum("q,eqiks,eqiks->eq", m.wq, ez, eu)
        mat = self._mat_index()[nodes]
        np.add.at(g_lam, mat.ravel(), -pl.ravel())
        np.add.at(g_mu, mat.ravel(), -pm.ravel())
        if self.full_gradient:
            self._grad_pair_pml(kap, Y, g_lam, g_mu)

    def _grad_pair_pml(self, kap, Y, g_lam, g_mu):
        """PML part of g -= z^T (dA/dm) Y under the material extension.

        The S-row of PML node j in brick e, (3b), is
        -w_q [mu_j (H + H^T) + lam_j tr(H) I] with H_ik = sum_L L_kk d_k u^L_i
        at the node's LGL point (u^L = x2, x1, x0 for L = Le, Lp, Lw), so
        d/d lam_j = -w_q tr(H) I and d/d mu_j = -w_q (H + H^T); lam_j, mu_j
        are the values of the interface node j projects onto (material_index),
        which collects the sum."""
        s = self.s
        m = s.mesh
        x0, x1, x2 = self.split(Y)
        nsrc = x1.shape[1]
        x0f = np.zeros((self.ns, nsrc))
        x0f[s.hist] = x0
        _, _, k2 = self.split(kap)
        zS = m.s_nodal(s.Minv[:, None] * k2)                          # (nn, 6, nsrc)
        fields = {"Le": m.u_nodal(x2), "Lp": m.u_nodal(x1), "Lw": m.u_nodal(x0f)}
        el_p = np.nonzero(m.is_pml)[0]
        mat_of = m.material_index()
        for c0 in range(0, el_p.size, 2048):
            nodes = m.conn[el_p[c0:c0 + 2048]]                          # (E, 27)
            H = 0.0
            for key, u in fields.items():
                Lam = s.coef[key][nodes]                                 # (E, 27, 3): L_kk at the points
                H = H + np.einsum("qak,eais->eqiks", s.g, u[nodes]) * Lam[:, :, None, :, None]
            trH = np.einsum("eqiis->eqs", H)
            z = zS[nodes]                                                # (E, 27, 6, nsrc)
            dl = m.wq[None, :, None] * trH * (z[:, :, 0] + z[:, :, 1] + z[:, :, 2])
            dm = 0.0
            for v, (a, b) in enumerate(((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))):
                dm = dm + z[:, :, v] * (H[:, :, a, b] + H[:, :, b, a])
            dm = m.wq[None, :, None] * dm
            mat = mat_of[nodes]
            np.add.at(g_lam, mat.ravel(), dl.sum(-1).ravel())
            np.add.at(g_mu, mat.ravel(), dm.sum(-1).ravel())

    def _mat_index(self):
        if not hasattr(self, "_mi"):
            m = self.s.mesh
            mi = -np.ones(m.n_nodes, np.int64)
            mi[m.interior_full_ids()] = np.arange(m.n_int_nodes)
            self._mi = mi
        return self._mi

    def adjoint_step(self, L, Ys=None, g_lam=None, g_mu=None):
        """Reverse of one RK4 step: Lambda^n - dJ_n/dX^n from Lambda^{n+1}.

        Stage order and weights follow the forward recurrence; with ``Ys``
        (the forward stage states of the step) the parameter-derivative
        terms k_i^T (dA/dm) Y_i are accumulated into g_lam, g_mu.
        """
        dt = self.dt
        k4 = (dt / 6.0) * L
        Yb4 = self.rhs_T(k4)
        k3 = (dt / 3.0) * L + dt * Yb4
        Yb3 = self.rhs_T(k3)
        k2 = (dt / 3.0) * L + 0.5 * dt * Yb3
        Yb2 = self.rhs_T(k2)
        k1 = (dt / 6.0) * L + 0.5 * dt * Yb2
        Yb1 = self.rhs_T(k1)
        if Ys is not None:
            for k, Y in zip((k1, k2, k3, k4), Ys):
                self._grad_pair(k, Y, g_lam, g_mu)
        return L + Yb1 + Yb2 + Yb3 + Yb4

    def adjoint_gradient(self, wav, observed, states=None):
        """Exact discrete (DTO) gradient m-bar = dJ/d(lam, mu) on Omega^RD nodes."""
        N = self.N
        dt = self.dt
        if states is None:
            _, states = self.forward(wav, store=True)
        tr = np.stack([self.traces_of(X) for X in states], axis=1)
        resid = tr - observed
        w = self.time_weights(N)
        nsrc = wav.shape[0]
        nX = self.nh + 2 * self.ns
        m = self.s.mesh
        g_lam = np.zeros(m.n_int_nodes)
        g_mu = np.zeros(m.n_int_nodes)

        def dj(n):
            out = np.zeros((nX, nsrc))
            x1 = out[self.nh:self.nh + self.ns]
            for c in range(3):
                np.add.at(x1, self.rec[:, c], dt * w[n] * resid[:, n, :, c].T)
            return out

        L = dj(N)
        for n in range(N - 1, -1, -1):
            Ys, _ = self.stages(states[n], wav, n)
            L = self.adjoint_step(L, Ys, g_lam, g_mu) + dj(n)
        return g_lam, g_mu, L

    # ------------------------------------------------------------------
    def adjoint_gradient_appb(self, wav, observed, states=None):
        """Optimize-then-discretize gradient: reverse RK4 of (15) per App. B."""
        s = self.s
        N, dt = self.N, self.dt
        if states is None:
            _, states = self.forward(wav, store=True)
        tr = np.stack([self.traces_of(X) for X in states], axis=1)
        resid = tr - observed                                     # (nsrc, N+1, nrec, 3)
        nsrc = wav.shape[0]
        nh, ns = self.nh, self.ns

        def fhat(r):                                              # r: (nsrc, nrec, 3)
            f = np.zeros((ns, nsrc))
            for c in range(3):
                np.add.at(f, self.rec[:, c], r[:, :, c].T)
            return s.Minv[:, None] * f

        def slope(y0, y1, y2, f):
            # d/dt (y0, y1, y2) = (P y1, y2, M^-1(G^T y0 - K^T y1 + C^T y2) + fhat)
            # G^T here maps PML-history vectors to state vectors: transpose of
            # the PML x PML block of G, extended by zero outside the PML.
            ghat = np.zeros((ns, nsrc))
            ext = np.zeros((ns, nsrc))
            ext[s.hist] = y0
            ghat[s.hist] = s.residual_T3(ext)[0]
            acc = s.Minv[:, None] * (ghat - s.residual_T3(y1)[1] + s.residual_T3(y2)[2]) + f
            return y1[s.hist], y2, acc

        y0 = np.zeros((nh, nsrc))
        y1 = np.zeros((ns, nsrc))
        y2 = np.zeros((ns, nsrc))
        m = s.mesh
        g_lam = np.zeros(m.n_int_nodes)
        g_mu = np.zeros(m.n_int_nodes)
        w = self.time_weights(N)

        def accumulate(y1v, n, weight):
            X = states[n]
            k = np.zeros((nh + 2 * ns, nsrc))
            # pair the adjoint displacement w = y1 with the forward state u^n:
            # _grad_pair forms z = M^{-1} k2, so pass k2 = M y1.
            k[nh + ns:] = s.M[:, None] * y1v
            gl = np.zeros_like(g_lam)
            gm = np.zeros_like(g_mu)
            self._grad_pair(k, X, gl, gm)
            g_lam[:] += weight * gl
            g_mu[:] += weight * gm

        accumulate(y1, N, dt * w[N])
        for n in range(N, 0, -1):
            fn = fhat(resid[:, n])
            fm = fhat(0.5 * (resid[:, n] + resid[:, n - 1]))
            f1 = fhat(resid[:, n - 1])
            k10, k11, k12 = slope(y0, y1, y2, fn)
            k20, k21, k22 = slope(y0 - 0.5 * dt * k10, y1 - 0.5 * dt * k11,
                                  y2 - 0.5 * dt * k12, fm)
            k30, k31, k32 = slope(y0 - 0.5 * dt * k20, y1 - 0.5 * dt * k21,
                                  y2 - 0.5 * dt * k22, fm)
            k40, k41, k42 = slope(y0 - dt * k30, y1 - dt * k31, y2 - dt * k32, f1)
            y0 = y0 - dt / 6.0 * (k10 + 2 * k20 + 2 * k30 + k40)
            y1 = y1 - dt / 6.0 * (k11 + 2 * k21 + 2 * k31 + k41)
            y2 = y2 - dt / 6.0 * (k12 + 2 * k22 + 2 * k32 + k42)
            accumulate(y1, n - 1, dt * w[n - 1])
        return g_lam, g_mu
