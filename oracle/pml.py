"""PML stretch tensors and scalar coefficients (oracle).

(1b)-(1c) and the symbol list after (2): Lambda_e, Lambda_p, Lambda_w are the
stretch tensors and a, b, c, d "products of certain elements" of them; the
paper defers their definition to its reference [13].  Reading used here
(derived, not quoted): complex coordinate stretching

    eps_s(x_s, omega) = alpha_s(x_s) + beta_s(x_s) / (i omega),   s = x, y, z,
    alpha_s = 1 + alpha_o (xi_s / L_s)^m,   beta_s = beta_o (xi_s / L_s)^m,

with xi_s the distance into the s-layer (zero outside it) and L_s the layer
thickness (alpha_o = 5, beta_o = 400 1/s, m = 2 in Sec. 4.1).  Multiplying the
stretched equilibrium and constitutive laws by eps_x eps_y eps_z and mapping
1/(i omega) to time integration gives (1b)-(1c) with

    Lambda(omega) = diag(eps_x eps_y eps_z / eps_k)
                  = Lambda_e + Lambda_p/(i omega) + Lambda_w/(i omega)^2,
    eps_x eps_y eps_z = a + b/(i omega) + c/(i omega)^2 + d/(i omega)^3.

The coefficients are obtained here literally as polynomial products in the
variable q = 1/(i omega).
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import polynomial as P


def stretch_params(mesh, alpha0, beta0, m):
    """alpha_s, beta_s at every node: arrays (n_nodes, 3)."""
    x, y, z = mesh.xyz.T
    xi = np.stack([
        np.maximum(0.0, np.abs(x) - 0.5 * mesh.Lx),
        np.maximum(0.0, np.abs(y) - 0.5 * mesh.Ly),
        np.maximum(0.0, -z - mesh.Lz),
    ], axis=1)
    L = np.array([mesh.Lpx, mesh.Lpy, mesh.Lpz])
    with np.errstate(invalid="ignore", divide="ignore"):
        r = np.where(L > 0, xi / np.where(L > 0, L, 1.0), 0.0)
    alpha = 1.0 + alpha0 * r ** m
    beta = beta0 * r ** m
    return alpha, beta


def coefficients(mesh, alpha0, beta0, m):
    """Return dict with Le, Lp, Lw (n_nodes, 3) and a, b, c, d (n_nodes,)."""
    alpha, beta = stretch_params(mesh, alpha0, beta0, m)
    n = alpha.shape[0]
    Lam = np.zeros((n, 3, 3))          # [node, k, power of q]
    abcd = np.zeros((n, 4))
    for j in range(n):
        eps = [np.array([alpha[j, s], beta[j, s]]) for s in range(3)]
        full = P.polymul(P.polymul(eps[0], eps[1]), eps[2])
        abcd[j, :len(full)] = full
        for k in range(3):
            o = [s for s in range(3) if s != k]
            prod = P.polymul(eps[o[0]], eps[o[1]])
            Lam[j, k, :len(prod)] = prod
    return dict(Le=Lam[:, :, 0], Lp=Lam[:, :, 1], Lw=Lam[:, :, 2],
                a=abcd[:, 0], b=abcd[:, 1], c=abcd[:, 2], d=abcd[:, 3],
                alpha=alpha, beta=beta)


def _pmul(p, q):
    """Row-wise product of polynomials given as coefficient arrays (n, dp), (n, dq)."""
    out = np.zeros((p.shape[0], p.shape[1] + q.shape[1] - 1))
    for i in range(p.shape[1]):
        for j in range(q.shape[1]):
            out[:, i + j] += p[:, i] * q[:, j]
    return out


def coefficients_fast(mesh, alpha0, beta0, m):
    """Same coefficients as ``coefficients``, the products taken for all nodes at once."""
    alpha, beta = stretch_params(mesh, alpha0, beta0, m)
    eps = [np.stack([alpha[:, s], beta[:, s]], axis=1) for s in range(3)]
    full = _pmul(_pmul(eps[0], eps[1]), eps[2])
    Lam = np.zeros((alpha.shape[0], 3, 3))
    for k in range(3):
        o = [s for s in range(3) if s != k]
        Lam[:, k, :] = _pmul(eps[o[0]], eps[o[1]])
    return dict(Le=Lam[:, :, 0], Lp=Lam[:, :, 1], Lw=Lam[:, :, 2],
                a=full[:, 0], b=full[:, 1], c=full[:, 2], d=full[:, 3],
                alpha=alpha, beta=beta)
