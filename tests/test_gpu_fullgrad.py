"""Full chain-rule gradient (grad_full = 1) on the GPU against the oracle's
full gradient: the interior-brick terms plus the PML S-row terms of the
material carried outward from the interface, on tiny, ragged-tile,
3-source (with checkpoints) and 864-brick problems."""
import numpy as np
import pytest

from helpers import observed, oracle_system, rel_l2, workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_1504_08340_amd as pkg
    return pkg


_cache = {}


def oracle_full(name):
    if name not in _cache:
        from oracle.solve import Stepper
        wl = workload(name)
        s, _ = oracle_system(name)
        st = Stepper(s, wl.src_node, wl.src_dir, wl.rec_node, full_gradient=True)
        tr, states = st.forward(wl.wavelet, store=True)
        obs = observed(name)
        gl, gm, _ = st.adjoint_gradient(wl.wavelet, obs, states)
        _cache[name] = (obs, gl, gm)
    return _cache[name]


@pytest.mark.parametrize("name,prec,ckpt,tol", [
    ("tiny", 0, 0, 1e-9), ("tiny_ragged", 0, 0, 1e-9), ("tiny_3src", 0, 7, 1e-9),
    ("cfg1_100", 0, 0, 1e-9), ("cfg1_100", 1, 0, 1e-4), ("tiny_ragged", 1, 4, 1e-4)])
def test_full_gradient_vs_oracle(P, name, prec, ckpt, tol):
    wl = workload(name)
    obs, gl_o, gm_o = oracle_full(name)
    S = P.Solver(wl.prob, wl.src_node, wl.src_dir, wl.rec_node, precision=prec, ckpt_every=ckpt, grad_full=True)
    rho, lam, mu, wav = (S.tensor(a) for a in (wl.rho, wl.lam, wl.mu, wl.wavelet))
    tr = S.forward(rho, lam, mu, wav)
    J, res = S.misfit(tr, S.tensor(obs))
    gl, gm = S.adjoint_gradient(rho, lam, mu, wav, res)
    e = (rel_l2(gl.cpu().numpy(), gl_o), rel_l2(gm.cpu().numpy(), gm_o))
    print(f"{name} precision {prec} ckpt {ckpt}: g_lam {e[0]:.2e} g_mu {e[1]:.2e}")
    assert e[0] <= tol and e[1] <= tol
    S.close()


def test_full_gradient_differs_from_restricted_only_on_the_interface(P):
    wl = workload("tiny_ragged")
    obs = observed("tiny_ragged")
    out = []
    for full in (False, True):
        S = P.Solver(wl.prob, wl.src_node, wl.src_dir, wl.rec_node, grad_full=full)
        rho, lam, mu, wav = (S.tensor(a) for a in (wl.rho, wl.lam, wl.mu, wl.wavelet))
        tr = S.forward(rho, lam, mu, wav)
        J, res = S.misfit(tr, S.tensor(obs))
        out.append([g.cpu().numpy() for g in S.adjoint_gradient(rho, lam, mu, wav, res)])
        S.close()
    nix, niy, niz = wl.prob.nn_int
    gk, gj, gi = np.meshgrid(np.arange(niz), np.arange(niy), np.arange(nix), indexing="ij")
    iface = ((gi == 0) | (gi == nix - 1) | (gj == 0) | (gj == niy - 1) | (gk == 0)).ravel()
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a[~iface], b[~iface])
        assert np.abs(a[iface] - b[iface]).max() > 1e-3 * np.abs(b).max()


def test_appendix_b_refuses_the_full_gradient(P):
    wl = workload("tiny")
    S = P.Solver(wl.prob, wl.src_node, wl.src_dir, wl.rec_node, grad_full=True)
    rho, lam, mu, wav = (S.tensor(a) for a in (wl.rho, wl.lam, wl.mu, wl.wavelet))
    tr = S.forward(rho, lam, mu, wav)
    J, res = S.misfit(tr, S.tensor(observed("tiny")))
    with pytest.raises(P.FwiError, match="exact adjoint only"):
        S.adjoint_gradient(rho, lam, mu, wav, res, scheme="appb")
    S.close()
