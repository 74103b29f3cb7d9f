"""The throughput workload's mesh against the FP64 oracle at 400 steps.

Fixture `tests/golden/cfg2_src0_400.npz`, written by
`tests/golden/make_cfg2_fixture.py` with the matrix-free oracle only: the
40x40x20 m interior, 5-brick PML (62,500 bricks, 3,093,816 unknowns), the
random lam, mu of the throughput workload, its first source (8 Hz Ricker at
(-10, -10, 0)), all 6,561 receivers, 400 RK4 steps, observed data zero.  The
GPU runs the launch configuration bench.py times (5x4x2 brick tiles,
512-thread element workgroups, stage displacements kept) in every precision:
traces and misfit within 2e-6 (relative L2 over the stored receivers), lam
and mu gradients within 1e-6 (relative L2 over the stored nodes, and the
norms of the full vectors); FP64 to rounding (1e-13 / 1e-12).  Observed:
FP64 4e-16 traces, 7e-15 gradients; FP32, FP32-MFMA and split-BF16 1.7e-7 to
1.8e-7 traces, 2e-8 to 6e-8 gradients.  The 4-source batch the bench times
gives the same source-1 traces.
"""
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

FIXTURE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cfg2_src0_400.npz")


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_1504_08340_amd as pkg
    return pkg


@pytest.fixture(scope="module")
def ref():
    z = np.load(FIXTURE)
    return {k: z[k] for k in z.files}


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _run(P, wl, prec, nsrc):
    import torch
    S = P.Solver(wl.prob, wl.src_node[:nsrc], wl.src_dir[:nsrc], wl.rec_node, precision=prec)
    assert tuple(S.sizes.tile) == (5, 4, 2) and S.sizes.element_threads == 512
    rho, lam, mu = (S.tensor(a) for a in (wl.rho, wl.lam, wl.mu))
    wav = S.tensor(wl.wavelet[:nsrc])
    tr = S.forward(rho, lam, mu, wav)
    J, res = S.misfit(tr, torch.zeros_like(tr))
    gl, gm = S.adjoint_gradient(rho, lam, mu, wav, res)
    out = tr.cpu().numpy(), J.item(), gl.cpu().numpy(), gm.cpu().numpy()
    S.close()
    return out


@pytest.mark.parametrize("prec,ttol,gtol", [(0, 1e-13, 1e-12), (1, 2e-6, 1e-6), (2, 2e-6, 1e-6), (3, 2e-6, 1e-6)])
def test_cfg2_400_steps_vs_oracle_fixture(P, ref, prec, ttol, gtol):
    wl = W.config2(nsteps=int(ref["nsteps"]))
    assert wl.prob.dt == float(ref["dt"])
    tr, J, gl, gm = _run(P, wl, prec, 1)
    rec, node = ref["traces_rec"], ref["gnode"]
    e = dict(traces=_rel(tr[0][:, rec, :], ref["traces"]), J=abs(J - float(ref["J"])) / float(ref["J"]),
             g_lam=_rel(gl[node], ref["g_lam"]), g_mu=_rel(gm[node], ref["g_mu"]),
             g_lam_norm=abs(np.linalg.norm(gl) - float(ref["g_lam_norm"])) / float(ref["g_lam_norm"]),
             g_mu_norm=abs(np.linalg.norm(gm) - float(ref["g_mu_norm"])) / float(ref["g_mu_norm"]))
    print(f"precision {prec}: " + ", ".join(f"{k} {v:.2e}" for k, v in e.items()))
    assert e["traces"] <= ttol and e["J"] <= ttol
    assert max(e["g_lam"], e["g_mu"], e["g_lam_norm"], e["g_mu_norm"]) <= gtol


def test_cfg2_400_steps_four_source_batch(P, ref):
    """The bench's 4-source batch: source 1's traces match the oracle's."""
    wl = W.config2(nsteps=int(ref["nsteps"]))
    tr, _, _, _ = _run(P, wl, 1, 4)
    e = _rel(tr[0][:, ref["traces_rec"], :], ref["traces"])
    print(f"4-source FP32 batch, source 1 traces: {e:.2e}")
    assert e <= 2e-6
