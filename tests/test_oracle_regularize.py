"""Pins of the regularization oracle (8), (9), (C.1a)-(C.1e), (18).

Closed forms: for a linear field the integrands are constant, and for
f = x^2 the Tikhonov integrand 4x^2 is a quadratic the 3-point LGL rule
integrates exactly; brute-force central differences for the gradients;
symmetry and null space of the Tikhonov matrix; M~ sums to the volume.
"""
import numpy as np
import pytest

import workloads as W
from oracle.regularize import Regularizer


def _coords(prob):
    x, y, z = W.interior_axes(prob)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return X.ravel(), Y.ravel(), Z.ravel()


@pytest.fixture(scope="module")
def small():
    prob = W.tiny(ne_int=(3, 2, 2), npml_side=1, npml_bottom=1).prob
    return prob, Regularizer(prob)


def test_linear_field_closed_forms(small):
    prob, r = small
    ex, ey, ez = prob.ne_int
    V = ex * ey * ez * prob.h ** 3
    X, Y, Z = _coords(prob)
    a = np.array([2.0, -3.0, 0.5])
    f = a[0] * X + a[1] * Y + a[2] * Z + 7.0
    v, _ = r.tikhonov(f)
    assert v == pytest.approx(0.5 * a @ a * V, rel=1e-13)
    eps = 0.3
    v, _ = r.total_variation(f, eps)
    assert v == pytest.approx(V * np.sqrt(a @ a + eps), rel=1e-13)


def test_quadratic_field_tikhonov_exact(small):
    prob, r = small
    ex, ey, ez = prob.ne_int
    Lx, Ly, Lz = ex * prob.h, ey * prob.h, ez * prob.h
    X, _, _ = _coords(prob)
    v, _ = r.tikhonov(X ** 2)
    # 1/2 int (2x)^2 = 2 Ly Lz int_{-Lx/2}^{Lx/2} x^2 dx = Ly Lz Lx^3 / 6
    assert v == pytest.approx(Ly * Lz * Lx ** 3 / 6.0, rel=1e-13)


@pytest.mark.parametrize("kind", ["tn", "tv"])
def test_gradients_match_central_differences(small, kind):
    prob, r = small
    rng = np.random.default_rng(11)
    f = rng.standard_normal(r.mass.size)
    eps = 0.05
    fn = (lambda x: r.tikhonov(x)) if kind == "tn" else (lambda x: r.total_variation(x, eps))
    _, g = fn(f)
    for j in rng.choice(f.size, 12, replace=False):
        e = np.zeros_like(f)
        e[j] = 1e-6
        fd = (fn(f + e)[0] - fn(f - e)[0]) / 2e-6
        assert fd == pytest.approx(g[j], rel=1e-6, abs=1e-9)


def test_tikhonov_matrix_symmetric_with_constant_null_space(small):
    _, r = small
    rng = np.random.default_rng(12)
    a, b = rng.standard_normal((2, r.mass.size))
    La, Lb = r.tikhonov(a)[1], r.tikhonov(b)[1]
    assert La @ b == pytest.approx(Lb @ a, rel=1e-12)
    const = np.full(r.mass.size, 3.0)
    assert np.abs(r.tikhonov(const)[1]).max() < 1e-12
    assert np.abs(r.total_variation(const, 0.1)[1]).max() < 1e-12


def test_linear_field_tikhonov_gradient_vanishes_inside(small):
    """A linear field is discretely harmonic: only boundary rows of L f survive."""
    prob, r = small
    X, Y, Z = _coords(prob)
    g = r.tikhonov(1.5 * X - 0.7 * Y + 2.0 * Z)[1]
    nx, ny, nz = prob.nn_int
    jx, jy, jz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    inner = ((jx > 0) & (jx < nx - 1) & (jy > 0) & (jy < ny - 1) & (jz > 0) & (jz < nz - 1))
    inner = inner.transpose(2, 1, 0).ravel()
    assert np.abs(g[inner]).max() < 1e-12
    assert np.abs(g[~inner]).max() > 1e-3


def test_material_mass_is_the_interior_volume(small):
    prob, r = small
    ex, ey, ez = prob.ne_int
    assert r.mass.sum() == pytest.approx(ex * ey * ez * prob.h ** 3, rel=1e-14)
    from oracle.mesh import Mesh
    m = Mesh(prob)
    assert np.allclose(r.mass, m.m_rd[m.interior_full_ids()], rtol=1e-14)


def test_finalize_divides_by_mass(small):
    _, r = small
    rng = np.random.default_rng(13)
    gm, gr = rng.standard_normal((2, r.mass.size))
    g = r.finalize(gm, gr, 0.25)
    assert np.allclose(g * r.mass, gm + 0.25 * gr, rtol=1e-14)
