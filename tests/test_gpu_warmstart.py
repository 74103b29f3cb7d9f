"""What the trained warm-start network gains over the linear-trend start.

Uses the weights shipped with the package (trained by
``python -m paper_1504_08340_amd.warmstart train --profiles 192 --epochs 30``
on seeded layered profiles 10000-10191, whose traces this library's forward
solver computed).  On held-out profiles the network's start model must be
closer to the true shear modulus than the trend, and the start the inversion
uses (the lower-misfit one of the two, the trend being the fallback) can
only improve the first-stage misfit.
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
    gains = []
    for seed in (20_000, 20_001, 20_002):
        wl = probe.W.with_model(probe.wl, probe.W.layered_profile_vs(probe.wl.prob, seed))
        obs = probe.traces(probe.S.tensor(wl.lam_true), probe.S.tensor(wl.mu_true)).clone()
        lam_n, mu_n = probe.start_model(net, obs)
        e_net = np.linalg.norm(mu_n.cpu().numpy() - wl.mu_true) / np.linalg.norm(wl.mu_true)
        e_trend = np.linalg.norm(probe.mu0.cpu().numpy() - wl.mu_true) / np.linalg.norm(wl.mu_true)
        J = {}
        for name, (l0, m0) in (("trend", (probe.lam0, probe.mu0)), ("net", (lam_n.clone(), mu_n.clone()))):
            J[name] = float(probe.S.misfit(probe.traces(l0, m0), obs)[0][0])
        used = min(J["trend"], J["net"])
        print(f"seed {seed}: mu error trend {e_trend:.3f} net {e_net:.3f}; J trend {J['trend']:.3e} "
              f"net {J['net']:.3e}")
        assert e_net < e_trend
        assert used <= J["trend"]
        gains.append(e_trend - e_net)
    assert np.mean(gains) > 0.02
