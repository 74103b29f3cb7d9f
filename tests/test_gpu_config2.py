"""Parity at the size bench.py times: 40x40x20 m interior, 62,500 bricks.

The FP64 HIP path is compared with the matrix-free FP64 oracle where the
oracle finishes in seconds (one source, operator applications, 3 RK4 steps
forward and back); the FP32 path at the bench's exact launch configuration
(4 sources, 2000 steps, stage displacements kept) is compared with the FP64
path, which the oracle pins.
"""
import numpy as np
import pytest

import workloads as W
from helpers import nodal_from_state, rel_l2, state_from_nodal

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_1504_08340_amd as pkg
    return pkg


@pytest.fixture(scope="module")
def cfg2_1src():
    wl = W.config2(nsteps=3)
    wl.wavelet, wl.src_node, wl.src_dir = wl.wavelet[:1], wl.src_node[:1], wl.src_dir[:1]
    from oracle.matfree import MatFree
    return wl, MatFree(wl.prob, wl.rho, wl.lam, wl.mu)


def test_cfg2_operator_parity_fp64(P, cfg2_1src):
    import torch
    wl, op = cfg2_1src
    S = P.Solver(wl.prob, wl.src_node, wl.src_dir, wl.rec_node)
    rng = np.random.default_rng(3)
    x1 = rng.standard_normal((op.n_state, 1))
    x2 = rng.standard_normal((op.n_state, 1))
    h = rng.standard_normal((op.n_hist, 1))
    x0 = np.zeros((op.n_state, 1))
    x0[op.hist] = h
    X = [S.tensor(nodal_from_state(op, v[:, 0])[None]) for v in (x0, x1, x2)]
    rho, lam, mu = (S.tensor(a) for a in (wl.rho, wl.lam, wl.mu))
    ref = (op.Minv[:, None] * -op.residual(h, x1, x2))[:, 0]
    got = state_from_nodal(op, S.apply_operator(0, rho, lam, mu, *X)[0].cpu().numpy())
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    ghat = np.zeros((op.n_state, 1))
    ghat[op.hist] = op.residual_T3(x0)[0]
    refT = (op.Minv[:, None] * -(ghat + op.residual_T3(x1)[1] + op.residual_T3(x2)[2]))[:, 0]
    gotT = state_from_nodal(op, S.apply_operator(1, rho, lam, mu, *X)[0].cpu().numpy())
    assert np.abs(gotT - refT).max() <= 1e-12 * np.abs(refT).max()
    torch.cuda.synchronize()


@pytest.mark.parametrize("prec,ttol,gtol", [(0, 1e-11, 1e-9), (1, 1e-5, 1e-4)])
def test_cfg2_short_run_vs_oracle(P, cfg2_1src, prec, ttol, gtol):
    from oracle.solve import Stepper
    wl, op = cfg2_1src
    st = Stepper(op, wl.src_node, wl.src_dir, wl.rec_node)
    tr_o, states = st.forward(wl.wavelet, store=True)
    obs = np.random.default_rng(5).standard_normal(tr_o.shape) * np.abs(tr_o).max()
    J_o = st.misfit(tr_o, obs)
    gl_o, gm_o, _ = st.adjoint_gradient(wl.wavelet, obs, states)
    S = P.Solver(wl.prob, wl.src_node, wl.src_dir, wl.rec_node, precision=prec)
    rho, lam, mu, wav = (S.tensor(a) for a in (wl.rho, wl.lam, wl.mu, wl.wavelet))
    tr = S.forward(rho, lam, mu, wav)
    J, res = S.misfit(tr, S.tensor(obs))
    gl, gm = S.adjoint_gradient(rho, lam, mu, wav, res)
    e = (rel_l2(tr.cpu().numpy(), tr_o), abs(J.item() - J_o) / J_o,
         rel_l2(gl.cpu().numpy(), gl_o), rel_l2(gm.cpu().numpy(), gm_o))
    print(f"precision={prec}: traces {e[0]:.2e} J {e[1]:.2e} g_lam {e[2]:.2e} g_mu {e[3]:.2e}")
    assert e[0] <= ttol and e[1] <= ttol and e[2] <= gtol and e[3] <= gtol


def _run(P, wl, prec, ckpt=0):
    S = P.Solver(wl.prob, wl.src_node, wl.src_dir, wl.rec_node, precision=prec, ckpt_every=ckpt)
    rho, lam, mu, wav = (S.tensor(a) for a in (wl.rho, wl.lam, wl.mu, wl.wavelet))
    obs = S.forward(rho, S.tensor(wl.lam_true), S.tensor(wl.mu_true), wav).clone()
    tr = S.forward(rho, lam, mu, wav)
    J, res = S.misfit(tr, obs)
    gl, gm = S.adjoint_gradient(rho, lam, mu, wav, res)
    out = tr.cpu().numpy(), J.item(), gl.cpu().numpy(), gm.cpu().numpy()
    S.close()
    del S, rho, lam, mu, wav, obs, tr, J, res, gl, gm
    import gc
    import torch
    gc.collect()
    torch.cuda.empty_cache()
    return out


def test_cfg2_batched_sources_equal_single_runs(P):
    wl = W.config2(nsteps=40)
    tr4, _, _, _ = _run(P, wl, 1)
    for s in (0, 3):
        w1 = W.config2(nsteps=40)
        w1.wavelet, w1.src_node, w1.src_dir = w1.wavelet[s:s + 1], w1.src_node[s:s + 1], w1.src_dir[s:s + 1]
        tr1, _, _, _ = _run(P, w1, 1)
        assert np.array_equal(tr1[0], tr4[s])


def test_cfg2_fp32_vs_fp64_at_bench_configuration(P):
    """4 sources x 2000 RK4 steps: FP32 state against the oracle-pinned FP64 path."""
    wl = W.config2(nsteps=2000)
    t64, J64, gl64, gm64 = _run(P, wl, 0, ckpt=100)     # FP64 with checkpoints + recompute
    t32, J32, gl32, gm32 = _run(P, wl, 1)               # the bench's launch configuration
    e = (rel_l2(t32, t64), abs(J32 - J64) / J64, rel_l2(gl32, gl64), rel_l2(gm32, gm64))
    print(f"FP32 vs FP64, 4 sources x 2000 steps: traces {e[0]:.2e} J {e[1]:.2e} "
          f"g_lam {e[2]:.2e} g_mu {e[3]:.2e}")
    assert e[0] <= 1e-5 and e[1] <= 1e-5 and e[2] <= 1e-4 and e[3] <= 1e-4
