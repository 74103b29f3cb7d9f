"""Distributed surface tractions (Sec. 4 loads) and forward-only plans on the
GPU against the oracle: a heterogeneous PML problem loaded by a uniform
vertical traction over a surface rectangle (oracle: its own consistent nodal
weights), traces, misfit and gradient."""
import numpy as np
import pytest

import workloads as W
from helpers import rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_1504_08340_amd as pkg
    return pkg


@pytest.fixture(scope="module")
def oracle_run():
    from oracle.assemble import System
    from oracle.loads import surface_traction_weights
    from oracle.solve import Stepper
    wl = W.tiny_traction(ne_int=(5, 3, 2), npml_side=2, npml_bottom=1, nsteps=40, seed=6, half=1.5)
    s = System(wl.prob, wl.rho, wl.lam, wl.mu)
    xmin, xmax, ymin, ymax, d = wl.traction
    ids, w = surface_traction_weights(s.mesh, xmin, xmax, ymin, ymax)
    loads = (np.zeros(ids.size, int), ids, w[:, None] * np.asarray(d)[None, :])
    st = Stepper(s, wl.src_node, wl.src_dir, wl.rec_node, loads=loads)
    tr, states = st.forward(wl.wavelet, store=True)
    obs = 0.8 * tr + 1e-3 * np.abs(tr).max() * np.random.default_rng(1).standard_normal(tr.shape)
    J = st.misfit(tr, obs)
    gl, gm, _ = st.adjoint_gradient(wl.wavelet, obs, states)
    return wl, tr, obs, J, gl, gm


@pytest.mark.parametrize("prec,ttol,gtol", [(0, 1e-11, 1e-9), (1, 1e-5, 1e-4)])
def test_traction_forward_misfit_gradient_vs_oracle(P, oracle_run, prec, ttol, gtol):
    wl, tr_o, obs, J_o, gl_o, gm_o = oracle_run
    S = P.Solver(wl.prob, wl.src_node, wl.src_dir, wl.rec_node, precision=prec, traction=wl.traction)
    rho, lam, mu, wav = (S.tensor(a) for a in (wl.rho, wl.lam, wl.mu, wl.wavelet))
    tr = S.forward(rho, lam, mu, wav)
    J, res = S.misfit(tr, S.tensor(obs))
    gl, gm = S.adjoint_gradient(rho, lam, mu, wav, res)
    e = (rel_l2(tr.cpu().numpy(), tr_o), abs(J.item() - J_o) / J_o, rel_l2(gl.cpu().numpy(), gl_o),
         rel_l2(gm.cpu().numpy(), gm_o))
    print(f"precision {prec}: traces {e[0]:.2e} J {e[1]:.2e} g_lam {e[2]:.2e} g_mu {e[3]:.2e}")
    assert e[0] <= ttol and e[1] <= ttol and e[2] <= gtol and e[3] <= gtol
    S.close()


def test_forward_only_plan(P, oracle_run):
    """ckpt_every = -1: the same traces, a smaller workspace, and the adjoint
    refused with FWI_ERR_STATE."""
    wl, tr_o, obs, _, _, _ = oracle_run
    S = P.Solver(wl.prob, wl.src_node, wl.src_dir, wl.rec_node, traction=wl.traction)
    F = P.Solver(wl.prob, wl.src_node, wl.src_dir, wl.rec_node, traction=wl.traction, ckpt_every=-1)
    assert F.sizes.workspace_bytes < S.sizes.workspace_bytes
    args = [F.tensor(a) for a in (wl.rho, wl.lam, wl.mu, wl.wavelet)]
    a = S.forward(*args).cpu().numpy()
    tr = F.forward(*args)
    assert np.array_equal(tr.cpu().numpy(), a)
    J, res = F.misfit(tr, F.tensor(obs))
    with pytest.raises(P.FwiError, match="forward-only") as e:
        F.adjoint_gradient(*args, res)
    assert e.value.status == -4
    S.close()
    F.close()
