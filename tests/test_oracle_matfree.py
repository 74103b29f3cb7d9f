"""The element-batched (matrix-free) oracle equals the assembled oracle."""
import numpy as np
import pytest

import workloads as W
from oracle import pml
from oracle.assemble import System
from oracle.matfree import MatFree
from oracle.mesh import Mesh
from oracle.solve import Stepper


@pytest.fixture(scope="module")
def pair():
    wl = W.tiny(ne_int=(3, 2, 2), npml_side=2, npml_bottom=1, nsteps=12, nsrc=2, seed=21)
    return wl, System(wl.prob, wl.rho, wl.lam, wl.mu), MatFree(wl.prob, wl.rho, wl.lam, wl.mu, chunk=7)


def test_vectorized_coefficients_equal_polynomial_products():
    prob = W.Problem((3, 2, 2), 2, 2, 1.0, 1e-3, 1, 5.0, 400.0, 2)
    m = Mesh(prob)
    a, b = pml.coefficients(m, 5.0, 400.0, 2), pml.coefficients_fast(m, 5.0, 400.0, 2)
    for k in ("Le", "Lp", "Lw", "a", "b", "c", "d"):
        np.testing.assert_allclose(a[k], b[k], rtol=1e-15, atol=0)


def test_operator_and_transposes_match(pair):
    _, s, f = pair
    rng = np.random.default_rng(0)
    x0 = rng.standard_normal((s.n_hist, 2))
    x1 = rng.standard_normal((s.n_state, 2))
    x2 = rng.standard_normal((s.n_state, 2))
    ref = s.residual(x0, x1, x2)
    got = f.residual(x0, x1, x2)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    for a, b in zip(f.residual_T3(x1), s.residual_T3(x1)):
        assert np.abs(a - b).max() <= 1e-13 * np.abs(b).max()
    np.testing.assert_allclose(f.M, s.M, rtol=1e-15)


def test_traces_and_gradient_match(pair):
    wl, s, f = pair
    sa = Stepper(s, wl.src_node, wl.src_dir, wl.rec_node)
    sf = Stepper(f, wl.src_node, wl.src_dir, wl.rec_node)
    ta, _ = sa.forward(wl.wavelet)
    tf, _ = sf.forward(wl.wavelet)
    assert np.abs(tf - ta).max() <= 1e-12 * np.abs(ta).max()
    obs = 0.8 * ta
    gla, gma, _ = sa.adjoint_gradient(wl.wavelet, obs)
    glf, gmf, _ = sf.adjoint_gradient(wl.wavelet, obs)
    assert np.linalg.norm(glf - gla) <= 1e-12 * np.linalg.norm(gla)
    assert np.linalg.norm(gmf - gma) <= 1e-12 * np.linalg.norm(gma)
