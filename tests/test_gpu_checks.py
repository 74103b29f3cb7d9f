"""Model validation and the RK4 stability bound (fwi_check_model).

The bound on the largest frequency must lie above the true largest
frequency of the interior operator (the oracle's eigenvalue of M^{-1} K for a
homogeneous box) and not far above it; a time step past the bound and
non-physical materials must be rejected with their status codes; the
workloads this library runs pass the check.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_1504_08340_amd as pkg
    return pkg


def test_bound_is_above_and_close_to_the_true_frequency(P):
    import scipy.sparse.linalg as spla
    from oracle.assemble import free_box_stiffness
    wl = W.tiny(ne_int=(3, 3, 2), npml_side=1, npml_bottom=1, nsteps=5, seed=3)
    lam0, mu0, rho0 = 4.0e7, 2.0e7, 2000.0
    S = P.Solver(wl.prob, wl.src_node, wl.src_dir, wl.rec_node)
    n = wl.lam.size
    info = P.fwi_check_model(S.plan, None, S.tensor(np.full(n, rho0)), S.tensor(np.full(n, lam0)),
                             S.tensor(np.full(n, mu0)))
    assert info[0] == rho0 and info[1] == mu0 and info[2] == 3 * lam0 + 2 * mu0
    assert info[3] == pytest.approx(np.sqrt((lam0 + 2 * mu0) / rho0))
    K, Md, _ = free_box_stiffness((4, 4, 4), wl.prob.h, lambda p: np.full(p.shape[0], lam0),
                                  lambda p: np.full(p.shape[0], mu0), rho=rho0)
    Ms = 1.0 / np.sqrt(Md)
    A = (K.multiply(Ms[:, None])).multiply(Ms[None, :]).tocsr()
    w_true = np.sqrt(spla.eigsh(A, k=1, which="LA", return_eigenvectors=False)[0])
    print(f"omega bound {info[4]:.2f}, true {w_true:.2f}, ratio {info[4] / w_true:.3f}")
    assert w_true <= info[4] <= 1.5 * w_true
    assert info[5] == pytest.approx(2 * np.sqrt(2) / info[4])
    S.close()


def test_unstable_step_and_bad_materials_are_rejected(P):
    wl = W.tiny(ne_int=(2, 2, 2), npml_side=1, npml_bottom=1, nsteps=5, seed=3)
    S = P.Solver(wl.prob, wl.src_node, wl.src_dir, wl.rec_node)
    rho, lam, mu = (S.tensor(a) for a in (wl.rho, wl.lam, wl.mu))
    info = P.fwi_check_model(S.plan, None, rho, lam, mu)
    S.close()
    fast = wl.prob.replace(dt=2.0 * info[5])
    S2 = P.Solver(fast, wl.src_node, wl.src_dir, wl.rec_node)
    with pytest.raises(P.FwiError, match="stability"):
        P.fwi_check_model(S2.plan, None, S2.tensor(wl.rho), S2.tensor(wl.lam), S2.tensor(wl.mu))
    bad = wl.mu.copy()
    bad[7] = -1.0
    with pytest.raises(P.FwiError, match="positive"):
        P.fwi_check_model(S2.plan, None, S2.tensor(wl.rho), S2.tensor(wl.lam), S2.tensor(bad))
    S2.close()


@pytest.mark.parametrize("make", [W.config1, W.config2, W.config3])
def test_workloads_pass_the_check(P, make):
    wl = make(nsteps=5)
    S = P.Solver(wl.prob, wl.src_node[:1], wl.src_dir[:1], wl.rec_node)
    info = P.fwi_check_model(S.plan, None, S.tensor(wl.rho), S.tensor(wl.lam), S.tensor(wl.mu))
    print(f"{wl.name}: dt {wl.prob.dt:.3e} <= stable {info[5]:.3e}")
    assert wl.prob.dt <= info[5]
    S.close()


def test_forward_and_adjoint_validate_the_model_before_any_launch(P):
    """fwi_forward / fwi_adjoint_gradient run the model check first: a step past
    the bound returns FWI_ERR_UNSTABLE, a negative mu or bulk term
    FWI_ERR_ARG, and nothing else is enqueued (the trace buffer keeps its
    sentinel values)."""
    import torch
    wl = W.tiny(ne_int=(2, 2, 2), npml_side=1, npml_bottom=1, nsteps=5, seed=3)
    S = P.Solver(wl.prob, wl.src_node, wl.src_dir, wl.rec_node)
    rho, lam, mu, wav = (S.tensor(a) for a in (wl.rho, wl.lam, wl.mu, wl.wavelet))
    info = P.fwi_check_model(S.plan, None, rho, lam, mu)
    S.close()
    fast = wl.prob.replace(dt=1.5 * info[5])
    S2 = P.Solver(fast, wl.src_node, wl.src_dir, wl.rec_node)
    tr = torch.full(S2.trace_shape, 7.0, dtype=torch.float64, device=S2.device)
    with pytest.raises(P.FwiError, match="stability") as e:
        S2.forward(rho, lam, mu, wav, tr)
    assert e.value.status == -5
    torch.cuda.synchronize()
    assert bool((tr == 7.0).all())
    S2.close()
    S3 = P.Solver(wl.prob, wl.src_node, wl.src_dir, wl.rec_node)
    for field, bad in (("mu", -1.0), ("lam", -1e12)):
        m = {"lam": wl.lam.copy(), "mu": wl.mu.copy()}
        m[field][5] = bad
        tr = torch.full(S3.trace_shape, 7.0, dtype=torch.float64, device=S3.device)
        with pytest.raises(P.FwiError, match="positive") as e:
            S3.forward(rho, S3.tensor(m["lam"]), S3.tensor(m["mu"]), wav, tr)
        assert e.value.status == -1
        torch.cuda.synchronize()
        assert bool((tr == 7.0).all())
    # a good forward, then an adjoint with a non-physical model: rejected too
    tr = S3.forward(rho, lam, mu, wav)
    J, res = S3.misfit(tr, torch.zeros_like(tr))
    bad = wl.mu.copy()
    bad[3] = 0.0
    with pytest.raises(P.FwiError, match="positive"):
        S3.adjoint_gradient(rho, lam, S3.tensor(bad), wav, res)
    S3.close()


def test_solver_rejects_mistyped_and_short_buffers(P):
    """Argument checks in Solver run before any C call."""
    import torch
    wl = W.tiny(ne_int=(2, 2, 2), npml_side=1, npml_bottom=1, nsteps=5, seed=3)
    S = P.Solver(wl.prob, wl.src_node, wl.src_dir, wl.rec_node)
    rho, lam, mu, wav = (S.tensor(a) for a in (wl.rho, wl.lam, wl.mu, wl.wavelet))
    with pytest.raises(ValueError, match="dtype"):
        S.forward(rho, lam.float(), mu, wav)
    with pytest.raises(ValueError, match="expected cuda"):
        S.forward(rho, lam, mu.cpu(), wav)
    with pytest.raises(ValueError, match="elements"):
        S.forward(rho, lam, mu, wav[:, :-3].contiguous())
    with pytest.raises(ValueError, match="contiguous"):
        S.forward(rho, lam, mu, torch.cat([wav, wav], 1)[:, ::2])
    tr = S.forward(rho, lam, mu, wav)
    with pytest.raises(ValueError, match="elements"):
        S.misfit(tr, torch.zeros(tr.numel() - 1, dtype=torch.float64, device=S.device))
    J, res = S.misfit(tr, torch.zeros_like(tr))
    with pytest.raises(ValueError, match="g_lam"):
        S.adjoint_gradient(rho, lam, mu, wav, res, g_lam=torch.empty(3, dtype=torch.float64, device=S.device))
    S.close()


def test_misfit_is_bit_reproducible(P):
    import torch
    wl = W.config1(nsteps=60)
    S = P.Solver(wl.prob, wl.src_node, wl.src_dir, wl.rec_node)
    rho, lam, mu, wav = (S.tensor(a) for a in (wl.rho, wl.lam, wl.mu, wl.wavelet))
    tr = S.forward(rho, lam, mu, wav)
    obs = 0.5 * tr
    Js = []
    for _ in range(3):
        J, _ = S.misfit(tr, obs)
        Js.append(J.item())
    torch.cuda.synchronize()
    assert Js[0] == Js[1] == Js[2]
    S.close()


def _interior_omega_max(wl):
    """Largest frequency of the interior operator M_RD^{-1} K_RD by the oracle
    (assembled interior stiffness, lumped interior mass, scipy eigsh)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    from oracle.assemble import System
    s = System(wl.prob, wl.rho, wl.lam, wl.mu)
    m = s.mesh
    nodes = np.nonzero(m.in_rd & (m.u_dof[:, 0] >= 0))[0]
    dofs = m.u_dof[nodes].ravel()
    K = s.Krd.tocsr()[dofs][:, dofs]
    M = np.repeat(s.rho[nodes] * m.m_rd[nodes], 3)
    Ms = sp.diags(1.0 / np.sqrt(M))
    w2 = spla.eigsh((Ms @ K @ Ms).tocsr(), k=1, which="LA", return_eigenvectors=False)[0]
    return float(np.sqrt(w2))


def test_time_step_between_the_brick_bound_and_the_true_limit(P):
    """A step above the brick-by-brick bound but below the true RK4 limit is
    accepted by fwi_forward (power-iteration estimate of the largest
    frequency); 5 % above the true limit it is rejected, and the estimate in
    the message lies within 2 % below the oracle's exact largest frequency."""
    import re
    wl = W.tiny(ne_int=(3, 3, 2), npml_side=1, npml_bottom=1, nsteps=4, seed=3)
    w_true = _interior_omega_max(wl)
    lim = 2.0 * np.sqrt(2.0) / w_true
    S = P.Solver(wl.prob, wl.src_node, wl.src_dir, wl.rec_node)
    info = P.fwi_check_model(S.plan, None, S.tensor(wl.rho), S.tensor(wl.lam), S.tensor(wl.mu))
    S.close()
    print(f"true limit {lim:.4e} s, brick bound {info[5]:.4e} s")
    assert info[5] < 0.9 * lim
    for scale, ok in ((0.97, True), (1.05, False)):
        prob = wl.prob.replace(dt=scale * lim)
        S = P.Solver(prob, wl.src_node, wl.src_dir, wl.rec_node)
        args = [S.tensor(a) for a in (wl.rho, wl.lam, wl.mu, wl.wavelet)]
        if ok:
            tr = S.forward(*args)
            assert np.isfinite(tr.cpu().numpy()).all()
        else:
            with pytest.raises(P.FwiError, match="power-iteration") as e:
                S.forward(*args)
            w_est = float(re.search(r"omega_max ([0-9.e+]+)", str(e.value)).group(1))
            print(f"estimate {w_est:.2f}, exact {w_true:.2f}")
            assert 0.98 * w_true <= w_est <= w_true * (1 + 1e-9)
        S.close()
