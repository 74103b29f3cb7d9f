"""1D Legendre-Gauss-Lobatto (LGL) rule and Lagrange basis (oracle).

Sec. 2 (after (5)): spectral elements with the LGL rule make M diagonal;
Sec. 4.1: quadratic 27-node bricks.  The element is the tensor product of the
1D quadratic element built here.

Everything is derived from definitions:
* nodes  = {-1, roots of P'_{p}, +1}   (Lobatto points for degree p),
* basis  = Lagrange polynomials through the nodes,
* weights = integrals of the basis polynomials over [-1, 1],
* D[i, a] = derivative of basis polynomial a at node i.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as L
from numpy.polynomial import polynomial as P


def lobatto_nodes(p: int) -> np.ndarray:
    """Nodes of the (p+1)-point LGL rule on [-1, 1]."""
    dleg = L.legder([0] * p + [1])          # derivative of P_p (Legendre basis)
    inner = np.sort(np.real(L.legroots(dleg))) if p > 1 else np.array([])
    return np.concatenate([[-1.0], inner, [1.0]])


def lagrange_polys(nodes: np.ndarray):
    """Power-series coefficients of each Lagrange polynomial."""
    polys = []
    for a, xa in enumerate(nodes):
        c = np.array([1.0])
        for b, xb in enumerate(nodes):
            if b != a:
                c = P.polymul(c, np.array([-xb, 1.0]) / (xa - xb))
        polys.append(c)
    return polys


def rule(p: int = 2):
    """Return (nodes, weights, D) for the degree-p LGL element."""
    x = lobatto_nodes(p)
    polys = lagrange_polys(x)
    w = np.array([P.polyval(1.0, P.polyint(c)) - P.polyval(-1.0, P.polyint(c))
                  for c in polys])
    D = np.array([[P.polyval(xi, P.polyder(c)) for c in polys] for xi in x])
    return x, w, D


def basis_values(p: int, pts: np.ndarray):
    """Values and derivatives of the Lagrange basis at arbitrary points."""
    x = lobatto_nodes(p)
    polys = lagrange_polys(x)
    val = np.array([[P.polyval(t, c) for c in polys] for t in pts])
    der = np.array([[P.polyval(t, P.polyder(c)) for c in polys] for t in pts])
    return val, der
