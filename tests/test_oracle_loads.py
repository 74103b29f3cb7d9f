"""Distributed surface tractions (Sec. 4 loads): the oracle's consistent
nodal weights against closed forms, and the library's host-side weights
against the oracle's (host logic, no GPU)."""
import numpy as np
import pytest

import workloads as W
from oracle.loads import surface_traction_weights
from oracle.mesh import Mesh


@pytest.fixture(scope="module")
def mesh():
    return Mesh(W.Problem((8, 6, 3), 2, 2, 1.0, 1e-3, 1))


@pytest.mark.parametrize("rect", [(-3.0, 3.0, -2.0, 2.0), (-4.0, 1.0, -3.0, 3.0), (0.0, 2.0, -1.0, 3.0)])
def test_weights_integrate_polynomials_exactly(mesh, rect):
    """The weights are integrals of the Q2 basis functions: against nodal
    values of 1, x, y, x^2, y^2 and xy they give the exact integrals over the
    rectangle (the 3-point LGL rule is exact to degree 3 per face)."""
    a, b, c, d = rect
    ids, w = surface_traction_weights(mesh, *rect)
    x, y, z = mesh.xyz[ids].T
    assert np.all(np.abs(z) < 1e-12)
    area = (b - a) * (d - c)
    np.testing.assert_allclose(w.sum(), area, rtol=1e-14)
    np.testing.assert_allclose((w * x).sum(), 0.5 * (b * b - a * a) * (d - c), atol=1e-12)
    np.testing.assert_allclose((w * y).sum(), 0.5 * (d * d - c * c) * (b - a), atol=1e-12)
    np.testing.assert_allclose((w * x * x).sum(), (b ** 3 - a ** 3) / 3 * (d - c), rtol=1e-13)
    np.testing.assert_allclose((w * y * y).sum(), (d ** 3 - c ** 3) / 3 * (b - a), rtol=1e-13)
    np.testing.assert_allclose((w * x * y).sum(), 0.25 * (b * b - a * a) * (d * d - c * c), atol=1e-12)


def test_weight_values_of_the_lgl_rule(mesh):
    """A face-interior node carries (2h/3)^2, a face corner inside the region
    (h/3)^2 (four faces of (h/6)^2), a region corner (h/6)^2."""
    ids, w = surface_traction_weights(mesh, -3.0, 3.0, -2.0, 2.0)
    x, y, _ = mesh.xyz[ids].T
    def at(px, py):
        return w[np.nonzero((np.abs(x - px) < 1e-9) & (np.abs(y - py) < 1e-9))[0][0]]
    assert at(0.5, 0.5) == pytest.approx(4.0 / 9.0, rel=1e-14)
    assert at(1.0, 1.0) == pytest.approx(1.0 / 9.0, rel=1e-14)
    assert at(-3.0, -2.0) == pytest.approx(1.0 / 36.0, rel=1e-14)
    assert at(0.5, -2.0) == pytest.approx(2.0 / 3.0 / 6.0, rel=1e-14)


def test_library_weights_equal_the_oracle():
    from paper_1504_08340_amd import binding as B
    for wl in (W.section41("p20"), W.tiny_traction()):
        m = Mesh(wl.prob)
        xmin, xmax, ymin, ymax, _ = wl.traction
        ids_o, w_o = surface_traction_weights(m, xmin, xmax, ymin, ymax)
        ids_l, w_l = B.fwi_surface_traction(B.make_problem(wl.prob, 1, 1), xmin, xmax, ymin, ymax)
        o = np.argsort(ids_l)
        assert np.array_equal(ids_l[o], ids_o)
        np.testing.assert_allclose(w_l[o], w_o, rtol=1e-14, atol=0)


def test_point_load_list_equals_point_loads():
    """A one-entry load list reproduces the point load it describes."""
    from oracle.assemble import System
    from oracle.solve import Stepper
    wl = W.tiny(ne_int=(2, 2, 2), npml_side=1, npml_bottom=1, nsteps=12, seed=3)
    s = System(wl.prob, wl.rho, wl.lam, wl.mu)
    a, _ = Stepper(s, wl.src_node, wl.src_dir, wl.rec_node).forward(wl.wavelet)
    loads = ([0], [int(wl.src_node[0])], wl.src_dir[:1])
    b, _ = Stepper(s, wl.src_node, wl.src_dir, wl.rec_node, loads=loads).forward(wl.wavelet)
    assert np.array_equal(a, b)
