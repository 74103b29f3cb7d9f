"""Distributed surface loads (oracle; test infrastructure only).

Sec. 4 probes the medium with a vertical stress (traction) of 1 kPa applied
on the free surface over a square region, with a Gaussian-pulse time
signature (Table 1).  In the weak form of (2) the traction t enters each
displacement row as the surface integral of t times the node's basis
function; with the 3x3 LGL rule on every brick face in the region (the rule
the paper uses for the mass, and R3 for every other integral) that integral
is a sum over the faces of the 2D LGL weight of the node times the face's
Jacobian (h/2)^2.  Computed here face by face from the mesh's element
connectivity: the top face of every brick touching z = 0 whose extent lies
inside the region.
"""
from __future__ import annotations

import numpy as np

from . import lgl


def surface_traction_weights(mesh, xmin, xmax, ymin, ymax):
    """Full-grid node ids and integrals of their basis functions over the
    part of the free surface inside [xmin, xmax] x [ymin, ymax]."""
    _, w, _ = lgl.rule(2)
    h = mesh.h
    tol = 1e-9 * h
    acc = np.zeros(mesh.n_nodes)
    top = np.nonzero(np.abs(mesh.xyz[mesh.conn[:, 26], 2]) < tol)[0]     # bricks whose top face is z = 0
    for e in top:
        nodes = mesh.conn[e]
        xy = mesh.xyz[nodes, :2]
        if xy[:, 0].min() < xmin - tol or xy[:, 0].max() > xmax + tol:
            continue
        if xy[:, 1].min() < ymin - tol or xy[:, 1].max() > ymax + tol:
            continue
        for b in range(3):
            for a in range(3):
                acc[nodes[a + 3 * b + 18]] += w[a] * w[b] * (0.5 * h) ** 2
    ids = np.nonzero((acc != 0.0) & ~mesh.dirichlet)[0]
    return ids, acc[ids]


def load_matrix(mesh, u_dof, n_state, nsrc, load_src, load_node, load_vec):
    """Unit-amplitude nodal force vectors (n_state, nsrc) from a load list:
    entry e adds load_vec[e] at node load_node[e] for source load_src[e]."""
    F = np.zeros((n_state, nsrc))
    for s, nd, v in zip(load_src, load_node, np.asarray(load_vec).reshape(-1, 3)):
        d = u_dof[nd]
        assert np.all(d >= 0), "load on a Dirichlet node"
        F[d, s] += v
    return F
