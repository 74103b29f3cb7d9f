"""Regularization, M~ and the control problem (18) on the GPU vs the oracle.

Through the C ABI: fwi_regularization (Tikhonov (8), TV (9): values and the
gradients (C.1b)-(C.1e)), fwi_material_mass (C.1a), fwi_gradient_finalize
(18) and fwi_dot, on a ragged small mesh, the 864-brick mesh and the
62,500-brick mesh the bench times.  FP64 throughout; the kernels sum in a
fixed order, so two calls give identical bits.
"""
import numpy as np
import pytest

import workloads as W
from oracle.regularize import Regularizer

pytestmark = pytest.mark.gpu

CASES = {
    "ragged": lambda: W.tiny(ne_int=(5, 3, 3), npml_side=3, npml_bottom=2, nsteps=5, seed=4),
    "cfg1": lambda: W.config1(nsteps=5),
    "cfg2": lambda: W.config2(nsteps=5),
}


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_1504_08340_amd as pkg
    return pkg


def _eps(r, f):
    return 1e-3 * float(np.max((r.Gx @ f) ** 2 + (r.Gy @ f) ** 2 + (r.Gz @ f) ** 2))


@pytest.mark.parametrize("case", list(CASES))
def test_regularization_mass_finalize_vs_oracle(P, case):
    import torch
    wl = CASES[case]()
    r = Regularizer(wl.prob)
    S = P.Solver(wl.prob, wl.src_node, wl.src_dir, wl.rec_node)
    n = S.sizes.n_int_nodes
    for name, field in (("lam", wl.lam), ("mu", wl.mu)):
        f = S.tensor(field)
        for kind in (P.FWI_REG_TIKHONOV, P.FWI_REG_TV):
            eps = 0.0 if kind == P.FWI_REG_TIKHONOV else _eps(r, field)
            v = torch.empty(1, dtype=torch.float64, device=S.device)
            g = torch.empty(n, dtype=torch.float64, device=S.device)
            P.fwi_regularization(S.plan, None, kind, eps, f, v, g)
            v2 = torch.empty_like(v)
            g2 = torch.empty_like(g)
            P.fwi_regularization(S.plan, None, kind, eps, f, v2, g2)
            vo, go = r.tikhonov(field) if kind == P.FWI_REG_TIKHONOV else r.total_variation(field, eps)
            vg, gg = float(v[0]), g.cpu().numpy()
            print(f"{case} {name} kind {kind}: value rel {abs(vg - vo) / abs(vo):.2e}, "
                  f"grad max rel {np.abs(gg - go).max() / np.abs(go).max():.2e}")
            assert abs(vg - vo) <= 1e-12 * abs(vo)
            assert np.abs(gg - go).max() <= 1e-12 * np.abs(go).max()
            assert torch.equal(v, v2) and torch.equal(g, g2)
    m = torch.empty(n, dtype=torch.float64, device=S.device)
    P.fwi_material_mass(S.plan, None, m)
    assert np.allclose(m.cpu().numpy(), r.mass, rtol=1e-14, atol=0)
    rng = np.random.default_rng(5)
    gm, gr = rng.standard_normal((2, n))
    out = torch.empty(n, dtype=torch.float64, device=S.device)
    P.fwi_gradient_finalize(S.plan, None, S.tensor(gm), S.tensor(gr), 0.37, out)
    assert np.allclose(out.cpu().numpy(), r.finalize(gm, gr, 0.37), rtol=1e-14, atol=0)
    d = torch.empty(1, dtype=torch.float64, device=S.device)
    P.fwi_dot(None, n, S.tensor(gm), S.tensor(gr), m, d)
    ref = float(np.sum(gm * gr * r.mass))
    assert abs(float(d[0]) - ref) <= 1e-12 * np.sum(np.abs(gm * gr * r.mass))
    torch.cuda.synchronize()
    S.close()


def test_regularization_argument_errors(P):
    wl = CASES["ragged"]()
    S = P.Solver(wl.prob, wl.src_node, wl.src_dir, wl.rec_node)
    f = S.tensor(wl.mu)
    g = S.tensor(np.zeros(S.sizes.n_int_nodes))
    with pytest.raises(P.FwiError, match="eps"):
        P.fwi_regularization(S.plan, None, P.FWI_REG_TV, 0.0, f, None, g)
    with pytest.raises(P.FwiError, match="kind"):
        P.fwi_regularization(S.plan, None, 5, 1.0, f, None, g)
    S.close()


def test_optimizer_vector_kernels():
    """fwi_axpby (in place and out of place) and fwi_absmax against numpy."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_1504_08340_amd as P
    rng = np.random.default_rng(4)
    n = 100_003
    x, y = rng.standard_normal(n), rng.standard_normal(n)
    tx, ty = (torch.tensor(a, device="cuda") for a in (x, y))
    out = torch.empty_like(tx)
    P.binding.fwi_axpby(None, n, 0.7, tx, -1.3, ty, out)
    np.testing.assert_allclose(out.cpu().numpy(), 0.7 * x - 1.3 * y, rtol=1e-15, atol=1e-15)
    P.binding.fwi_axpby(None, n, 2.5, tx, 0.0, None, tx)
    np.testing.assert_allclose(tx.cpu().numpy(), 2.5 * x, rtol=1e-15)
    m = torch.empty(1, dtype=torch.float64, device="cuda")
    P.binding.fwi_absmax(None, n, ty, m)
    assert m.item() == np.abs(y).max()
