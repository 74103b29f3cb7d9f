"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances: FP64 -- operator applications 1e-13 (max relative), traces 1e-11
and gradients 1e-9 (relative L2): a few hundred steps of rounding at 1e-16.
FP32 -- the stated targets: traces 1e-5 relative L2, gradients 1e-4.
"""
import numpy as np
import pytest

from helpers import (nodal_from_state, observed, oracle_run, oracle_system, rel_l2,
                     state_from_nodal, workload)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_1504_08340_amd as pkg
    return pkg


def _solver(P, wl, precision=0, ckpt=0):
    return P.Solver(wl.prob, wl.src_node, wl.src_dir, wl.rec_node, precision=precision, ckpt_every=ckpt)


def _inputs(S, wl):
    return [S.tensor(a) for a in (wl.rho, wl.lam, wl.mu, wl.wavelet)]


@pytest.mark.parametrize("name", ["tiny", "tiny_ragged", "cfg1"])
def test_operator_parity(P, name):
    import torch
    wl = workload(name)
    s, _ = oracle_system(name)
    S = _solver(P, wl)
    rng = np.random.default_rng(1)
    x1 = rng.standard_normal(s.n_state)
    x2 = rng.standard_normal(s.n_state)
    h = rng.standard_normal(s.n_hist)
    x0 = np.zeros(s.n_state)
    x0[s.hist] = h
    X = [S.tensor(np.repeat(nodal_from_state(s, v)[None], wl.nsrc, 0)) for v in (x0, x1, x2)]
    rho, lam, mu, _ = _inputs(S, wl)
    ref = s.Minv * -(s.G @ h + s.K @ x1 + s.C @ x2)
    out = S.apply_operator(0, rho, lam, mu, *X)
    torch.cuda.synchronize()
    got = state_from_nodal(s, out[0].cpu().numpy())
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    ghat = np.zeros(s.n_state)
    ghat[s.hist] = s.G[s.hist, :].T @ h
    refT = s.Minv * -(ghat + s.K.T @ x1 + s.C.T @ x2)
    outT = S.apply_operator(1, rho, lam, mu, *X)
    gotT = state_from_nodal(s, outT[0].cpu().numpy())
    assert np.abs(gotT - refT).max() <= 1e-13 * np.abs(refT).max()


@pytest.mark.parametrize("name,ckpt", [("tiny", 0), ("tiny", 7), ("tiny_ragged", 0), ("tiny_3src", 4),
                                       ("cfg1_100", 0), ("cfg1_100", 30)])
def test_forward_adjoint_gradient_fp64(P, name, ckpt):
    import torch
    wl = workload(name)
    tr_o, J_o, gl_o, gm_o = oracle_run(name)
    S = _solver(P, wl, 0, ckpt)
    rho, lam, mu, wav = _inputs(S, wl)
    tr = S.forward(rho, lam, mu, wav)
    obs = S.tensor(observed(name))
    J, res = S.misfit(tr, obs)
    gl, gm = S.adjoint_gradient(rho, lam, mu, wav, res)
    torch.cuda.synchronize()
    assert rel_l2(tr.cpu().numpy(), tr_o) <= 1e-11
    assert abs(J.item() - J_o) <= 1e-11 * J_o
    assert rel_l2(gl.cpu().numpy(), gl_o) <= 1e-9
    assert rel_l2(gm.cpu().numpy(), gm_o) <= 1e-9


def test_config1_full_fp64_and_fp32(P):
    """8x8x4 m interior, 400 RK4 steps: FP64 and the FP32 tolerances (traces 1e-5, gradients 1e-4)."""
    import torch
    name = "cfg1"
    wl = workload(name)
    tr_o, J_o, gl_o, gm_o = oracle_run(name)
    obs_np = observed(name)
    for prec, ttol, gtol in ((0, 1e-11, 1e-9), (1, 1e-5, 1e-4)):
        S = _solver(P, wl, prec, 0)
        rho, lam, mu, wav = _inputs(S, wl)
        tr = S.forward(rho, lam, mu, wav)
        J, res = S.misfit(tr, S.tensor(obs_np))
        gl, gm = S.adjoint_gradient(rho, lam, mu, wav, res)
        torch.cuda.synchronize()
        e = (rel_l2(tr.cpu().numpy(), tr_o), abs(J.item() - J_o) / J_o,
             rel_l2(gl.cpu().numpy(), gl_o), rel_l2(gm.cpu().numpy(), gm_o))
        print(f"precision={prec} traces {e[0]:.2e} J {e[1]:.2e} g_lam {e[2]:.2e} g_mu {e[3]:.2e}")
        assert e[0] <= ttol and e[1] <= 10 * ttol and e[2] <= gtol and e[3] <= gtol


def test_adjoint_before_forward_is_rejected(P):
    wl = workload("tiny")
    S = _solver(P, wl)
    rho, lam, mu, wav = _inputs(S, wl)
    res = S.empty_traces().zero_()
    with pytest.raises(P.FwiError, match="call order"):
        S.adjoint_gradient(rho, lam, mu, wav, res)


def test_bad_receiver_node_is_rejected(P):
    wl = workload("tiny")
    with pytest.raises(P.FwiError):
        P.Solver(wl.prob, wl.src_node, wl.src_dir, np.array([0], np.int32))   # Dirichlet corner


@pytest.mark.parametrize("name,ckpt,prec", [("tiny", 0, 0), ("tiny", 7, 0), ("tiny_ragged", 0, 0),
                                            ("tiny_3src", 4, 0), ("cfg1_100", 0, 0), ("cfg1_100", 0, 1)])
def test_appendix_b_gradient_vs_oracle(P, name, ckpt, prec):
    """The paper's reverse-time RK4 (App. B) against the oracle's App. B."""
    import torch
    wl = workload(name)
    _, st = oracle_system(name)
    tr_o, states = st.forward(wl.wavelet, store=True)
    obs = observed(name)
    gl_o, gm_o = st.adjoint_gradient_appb(wl.wavelet, obs, states)
    S = _solver(P, wl, prec, ckpt)
    rho, lam, mu, wav = _inputs(S, wl)
    tr = S.forward(rho, lam, mu, wav)
    J, res = S.misfit(tr, S.tensor(obs))
    gl, gm = S.adjoint_gradient(rho, lam, mu, wav, res, scheme="appb")
    torch.cuda.synchronize()
    tol = 1e-9 if prec == 0 else 1e-4
    e = (rel_l2(gl.cpu().numpy(), gl_o), rel_l2(gm.cpu().numpy(), gm_o))
    print(f"{name} ckpt {ckpt} precision {prec}: App. B g_lam {e[0]:.2e} g_mu {e[1]:.2e}")
    assert e[0] <= tol and e[1] <= tol
