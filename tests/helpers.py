"""Shared test helpers: oracle <-> nodal-field conversion, cached oracle runs."""
import functools

import numpy as np

import workloads as W
from oracle.assemble import System
from oracle.solve import Stepper


def nodal_from_state(sys_, vec):
    """Oracle state vector (n_state,) -> nodal fields (9, n_nodes)."""
    m = sys_.mesh
    u = m.u_nodal(vec[:, None])[..., 0]
    s = m.s_nodal(vec[:, None])[..., 0]
    return np.concatenate([u.T, s.T], axis=0)


def state_from_nodal(sys_, F):
    m = sys_.mesh
    v = np.zeros(sys_.n_state)
    v[:m.n_u] = F[:3, m.u_node].T.ravel()
    v[m.n_u:] = F[3:, m.s_node].T.ravel()
    return v


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


WORKLOADS = {
    "tiny": lambda: W.tiny(ne_int=(2, 2, 2), npml_side=1, npml_bottom=1, nsteps=30, seed=3),
    "tiny_ragged": lambda: W.tiny(ne_int=(5, 3, 3), npml_side=3, npml_bottom=2, nsteps=25, seed=4),
    "tiny_3src": lambda: W.tiny(ne_int=(3, 4, 2), npml_side=2, npml_bottom=1, nsteps=20, nsrc=3,
                                seed=5),
    "cfg1_100": lambda: W.config1(nsteps=100),
    "cfg1": lambda: W.config1(nsteps=400),
}


@functools.lru_cache(maxsize=None)
def workload(name):
    return WORKLOADS[name]()


@functools.lru_cache(maxsize=None)
def oracle_system(name):
    wl = workload(name)
    s = System(wl.prob, wl.rho, wl.lam, wl.mu)
    return s, Stepper(s, wl.src_node, wl.src_dir, wl.rec_node)


@functools.lru_cache(maxsize=None)
def observed(name):
    """Observed data from the target model (or a perturbed model), by the oracle."""
    wl = workload(name)
    if wl.lam_true is not None:
        lt, mt = wl.lam_true, wl.mu_true
    else:
        rng = np.random.default_rng(99)
        lt = wl.lam * (1 + 0.1 * rng.uniform(-1, 1, wl.lam.size))
        mt = wl.mu * (1 + 0.1 * rng.uniform(-1, 1, wl.mu.size))
    s = System(wl.prob, wl.rho, lt, mt)
    st = Stepper(s, wl.src_node, wl.src_dir, wl.rec_node)
    tr, _ = st.forward(wl.wavelet)
    return tr


@functools.lru_cache(maxsize=None)
def oracle_run(name):
    """(traces, J, g_lam, g_mu) of the oracle at the workload's model."""
    wl = workload(name)
    _, st = oracle_system(name)
    tr, states = st.forward(wl.wavelet, store=True)
    obs = observed(name)
    J = st.misfit(tr, obs)
    gl, gm, _ = st.adjoint_gradient(wl.wavelet, obs, states)
    return tr, J, gl, gm
