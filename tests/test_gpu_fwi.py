"""The inversion loop (Algorithms 1-2, (24), (25), frequency continuation) on
the GPU against the oracle's loop, iterate by iterate.

Both run in FP64 on the same small PML-truncated problem from the same
start model; every decision (number of halvings in each line search) must
agree, and the misfit history and final models match to 1e-9.
"""
import numpy as np
import pytest

import workloads as W
from helpers import observed, rel_l2, workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_1504_08340_amd as pkg
    return pkg


def _oracle(wl, stages_obs, reg, max_iter, tv_eps):
    import oracle.fwi as F
    from oracle.assemble import System
    from oracle.regularize import Regularizer
    from oracle.solve import Stepper

    def make(lam, mu):
        return Stepper(System(wl.prob, wl.rho, lam, mu), wl.src_node, wl.src_dir, wl.rec_node)

    r = Regularizer(wl.prob)
    opts = F.Options(reg=reg, tv_eps=tv_eps, max_iter=max_iter)
    stages = [F.OracleStage(make, r, wav, obs, opts) for wav, obs in stages_obs]
    return F.invert(stages, wl.lam, wl.mu, r.mass, opts)


def _gpu(P, wl, stages_obs, reg, max_iter, tv_eps):
    import torch
    from paper_1504_08340_amd import fwi
    S = P.Solver(wl.prob, wl.src_node, wl.src_dir, wl.rec_node)
    opts = fwi.FwiOptions(reg=reg, tv_eps=tv_eps, max_iter=max_iter)
    rho = S.tensor(wl.rho)
    stages = [fwi.FwiStage(S, rho, S.tensor(wav), S.tensor(obs), opts) for wav, obs in stages_obs]
    mass = torch.empty(S.sizes.n_int_nodes, dtype=torch.float64, device=S.device)
    P.fwi_material_mass(S.plan, None, mass)
    lam, mu, h = fwi.invert(stages, S.tensor(wl.lam), S.tensor(wl.mu), mass, opts)
    out = lam.cpu().numpy(), mu.cpu().numpy(), h
    S.close()
    return out


@pytest.mark.parametrize("reg", ["tikhonov", "tv"])
def test_one_stage_matches_oracle(P, reg):
    name = "tiny"
    wl = workload(name)
    st = [(wl.wavelet, observed(name))]
    lo, mo, ho = _oracle(wl, st, reg, 3, 1e10)
    lg, mg, hg = _gpu(P, wl, st, reg, 3, 1e10)
    print(reg, "oracle J", ho.J, "backtracks", ho.backtracks)
    print(reg, "gpu    J", hg.J, "backtracks", hg.backtracks)
    assert hg.backtracks == ho.backtracks
    assert np.allclose(hg.J, ho.J, rtol=1e-9, atol=0)
    assert rel_l2(lg, lo) < 1e-9 and rel_l2(mg, mo) < 1e-9


def test_frequency_continuation_matches_oracle(P):
    """Two stages: a low-frequency Ricker, then the workload's own wavelet."""
    from oracle.assemble import System
    from oracle.solve import Stepper
    name = "tiny"
    wl = workload(name)
    low = np.stack([W.sample_wavelet(lambda t: W.ricker(t, 8.0), wl.prob.dt, wl.prob.nsteps, 1000.0)]
                   * wl.nsrc)
    rng = np.random.default_rng(99)
    lt = wl.lam * (1 + 0.1 * rng.uniform(-1, 1, wl.lam.size))
    mt = wl.mu * (1 + 0.1 * rng.uniform(-1, 1, wl.mu.size))
    target = Stepper(System(wl.prob, wl.rho, lt, mt), wl.src_node, wl.src_dir, wl.rec_node)
    obs_low = target.forward(low)[0]
    st = [(low, obs_low), (wl.wavelet, observed(name))]
    lo, mo, ho = _oracle(wl, st, "tikhonov", 2, 1e10)
    lg, mg, hg = _gpu(P, wl, st, "tikhonov", 2, 1e10)
    assert hg.backtracks == ho.backtracks
    assert np.allclose(hg.J, ho.J, rtol=1e-9, atol=0)
    assert rel_l2(lg, lo) < 1e-9 and rel_l2(mg, mo) < 1e-9
