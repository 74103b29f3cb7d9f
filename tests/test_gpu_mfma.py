"""Interior stiffness and PML operator on the matrix cores (FWI_FP32_MFMA,
FWI_FP32_BF16X3).

The dense reference-matrix forms must give the operator of the scalar
kernels (interior and PML rows, forward and transposed): one application against the FP64 oracle at FP32 rounding level
(ragged tiles, several sources), then forward, misfit and gradient against
the oracle at the FP32 tolerances (traces 1e-5, gradients 1e-4), on
the 864-brick workload and, for 3 steps, on the 62,500-brick mesh.
"""
import numpy as np
import pytest

import workloads as W
from helpers import nodal_from_state, observed, oracle_run, oracle_system, rel_l2, state_from_nodal, workload

pytestmark = pytest.mark.gpu

MODES = {"mfma_f32": 2, "mfma_bf16x3": 3}


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_1504_08340_amd as pkg
    return pkg


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("name", ["tiny_ragged", "tiny_3src", "cfg1"])
def test_operator_matches_oracle(P, mode, name):
    import torch
    wl = workload(name)
    s, _ = oracle_system(name)
    S = P.Solver(wl.prob, wl.src_node, wl.src_dir, wl.rec_node, precision=MODES[mode])
    rng = np.random.default_rng(21)
    rho, lam, mu = (S.tensor(a) for a in (wl.rho, wl.lam, wl.mu))
    errs = []
    for which in (0, 1):
        x1 = rng.standard_normal(s.n_state)
        zero_h = np.zeros(s.n_state)
        X1 = S.tensor(np.repeat(nodal_from_state(s, x1)[None], wl.nsrc, 0))
        Z = S.tensor(np.repeat(nodal_from_state(s, zero_h)[None], wl.nsrc, 0))
        out = S.apply_operator(which, rho, lam, mu, Z, X1, Z)
        torch.cuda.synchronize()
        K = s.K if which == 0 else s.K.T
        ref = s.Minv * -(K @ x1)
        for src in range(wl.nsrc):
            got = state_from_nodal(s, out[src].cpu().numpy())
            errs.append(np.abs(got - ref).max() / np.abs(ref).max())
    print(f"{mode} {name}: max rel err {max(errs):.2e}")
    assert max(errs) < 2e-6
    S.close()


@pytest.mark.parametrize("mode", list(MODES))
def test_config1_forward_gradient_vs_oracle(P, mode):
    import torch
    name = "cfg1"
    wl = workload(name)
    tr_o, J_o, gl_o, gm_o = oracle_run(name)
    S = P.Solver(wl.prob, wl.src_node, wl.src_dir, wl.rec_node, precision=MODES[mode])
    rho, lam, mu, wav = (S.tensor(a) for a in (wl.rho, wl.lam, wl.mu, wl.wavelet))
    tr = S.forward(rho, lam, mu, wav)
    J, res = S.misfit(tr, S.tensor(observed(name)))
    gl, gm = S.adjoint_gradient(rho, lam, mu, wav, res)
    torch.cuda.synchronize()
    e = (rel_l2(tr.cpu().numpy(), tr_o), abs(J.item() - J_o) / J_o,
         rel_l2(gl.cpu().numpy(), gl_o), rel_l2(gm.cpu().numpy(), gm_o))
    print(f"{mode}: traces {e[0]:.2e} J {e[1]:.2e} g_lam {e[2]:.2e} g_mu {e[3]:.2e}")
    assert e[0] <= 1e-5 and e[1] <= 1e-4 and e[2] <= 1e-4 and e[3] <= 1e-4
    S.close()


@pytest.mark.parametrize("mode", list(MODES))
def test_cfg2_mesh_operator(P, mode):
    """62,500 bricks: interior operator (which = 0) against the matrix-free oracle."""
    import torch
    from oracle.matfree import MatFree
    wl = W.config2(nsteps=3)
    wl.wavelet, wl.src_node, wl.src_dir = wl.wavelet[:1], wl.src_node[:1], wl.src_dir[:1]
    op = MatFree(wl.prob, wl.rho, wl.lam, wl.mu)
    S = P.Solver(wl.prob, wl.src_node, wl.src_dir, wl.rec_node, precision=MODES[mode])
    rng = np.random.default_rng(22)
    x1 = rng.standard_normal((op.n_state, 1))
    z = np.zeros((op.n_state, 1))
    X1 = S.tensor(nodal_from_state(op, x1[:, 0])[None])
    Z = S.tensor(nodal_from_state(op, z[:, 0])[None])
    rho, lam, mu = (S.tensor(a) for a in (wl.rho, wl.lam, wl.mu))
    ref = (op.Minv[:, None] * -op.residual(np.zeros((op.n_hist, 1)), x1, z))[:, 0]
    got = state_from_nodal(op, S.apply_operator(0, rho, lam, mu, Z, X1, Z)[0].cpu().numpy())
    torch.cuda.synchronize()
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"{mode} cfg2 operator: {err:.2e}")
    assert err < 2e-6
    S.close()
