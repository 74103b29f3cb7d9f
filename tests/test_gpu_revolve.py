"""Binomial checkpointing (ckpt_slots > 0) on the GPU: the recomputed
segments reproduce the forward states bit for bit, so the gradient equals
the store-all gradient exactly, for the exact adjoint (restricted and full)
and for App. B; the oracle pins the store-all value."""
import numpy as np
import pytest

from helpers import observed, oracle_run, rel_l2, workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_1504_08340_amd as pkg
    return pkg


def _grad(P, wl, obs, scheme="discrete", **kw):
    S = P.Solver(wl.prob, wl.src_node, wl.src_dir, wl.rec_node, **kw)
    rho, lam, mu, wav = (S.tensor(a) for a in (wl.rho, wl.lam, wl.mu, wl.wavelet))
    tr = S.forward(rho, lam, mu, wav)
    J, res = S.misfit(tr, S.tensor(obs))
    gl, gm = S.adjoint_gradient(rho, lam, mu, wav, res, scheme=scheme)
    out = gl.cpu().numpy(), gm.cpu().numpy(), int(S.sizes.ckpt_states), int(S.sizes.adjoint_forward_steps)
    S.close()
    return out


@pytest.mark.parametrize("name,k,slots", [("tiny_3src", 2, 1), ("tiny_3src", 2, 3), ("tiny_ragged", 3, 2),
                                          ("cfg1_100", 5, 2)])
def test_revolve_gradient_equals_store_all(P, name, k, slots):
    wl = workload(name)
    obs = observed(name)
    ref = _grad(P, wl, obs)
    got = _grad(P, wl, obs, ckpt_every=k, ckpt_slots=slots)
    print(f"{name} k={k} slots={slots}: states {got[2]}, adjoint forward steps {got[3]} "
          f"(N = {wl.prob.nsteps})")
    assert got[2] == slots and got[3] > wl.prob.nsteps
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
    _, _, gl_o, gm_o = oracle_run(name)
    assert rel_l2(got[0], gl_o) <= 1e-9 and rel_l2(got[1], gm_o) <= 1e-9


def test_revolve_with_full_gradient_and_appendix_b(P):
    wl = workload("tiny_ragged")
    obs = observed("tiny_ragged")
    a = _grad(P, wl, obs, grad_full=True)
    b = _grad(P, wl, obs, grad_full=True, ckpt_every=2, ckpt_slots=2)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    a = _grad(P, wl, obs, scheme="appb")
    b = _grad(P, wl, obs, scheme="appb", ckpt_every=2, ckpt_slots=3)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
