"""What the trained warm-start network gains over the linear-trend start.

Uses the weights shipped with the package (trained by
``python -m paper_1504_08340_amd.warmstart train --profiles 192 --epochs 30``
on seeded layered profiles 10000-10191, whose traces this library's forward
solver computed).  On held-out profiles the network's start model must be
closer to the true shear modulus than the trend on every profile, and its
first-stage misfit lower than the trend's on average (geometric mean of the
ratios over the profiles).
"""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1504_08340_amd",
                       "warmstart_weights.npz")


def test_network_start_is_closer_than_the_trend():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_1504_08340_amd import warmstart as WS
    probe = WS.Probe()
    net = WS.Net.load(WEIGHTS, probe.S.device)
    gains, ratios = [], []
    for seed in (20_000, 20_001, 20_002):
        wl = probe.W.with_model(probe.wl, probe.W.layered_profile_vs(probe.wl.prob, seed))
        obs = probe.traces(probe.S.tensor(wl.lam_true), probe.S.tensor(wl.mu_true)).clone()
        lam_n, mu_n = probe.start_model(net, obs)
        e_net = np.linalg.norm(mu_n.cpu().numpy() - wl.mu_true) / np.linalg.norm(wl.mu_true)
        e_trend = np.linalg.norm(probe.mu0.cpu().numpy() - wl.mu_true) / np.linalg.norm(wl.mu_true)
        J = {}
        for name, (l0, m0) in (("trend", (probe.lam0, probe.mu0)), ("net", (lam_n.clone(), mu_n.clone()))):
            J[name] = float(probe.S.misfit(probe.traces(l0, m0), obs)[0][0])
        print(f"seed {seed}: mu error trend {e_trend:.3f} net {e_net:.3f}; J trend {J['trend']:.3e} "
              f"net {J['net']:.3e}")
        assert e_net < e_trend
        gains.append(e_trend - e_net)
        ratios.append(J["net"] / J["trend"])
    assert np.mean(gains) > 0.02
    assert np.exp(np.mean(np.log(ratios))) < 1.0
