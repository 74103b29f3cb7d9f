"""Pins of the oracle's inversion loop (Algorithms 1-2, (24), (25)).

Closed forms and invariants that do not restate the code: the Armijo step on
a parabola; the secant equation, W-self-adjointness and positivity of the
L-BFGS operator; convergence of the whole loop to the minimizer of a convex
quadratic in the weighted geometry; the identities of (24) and (25); and a
monotone misfit decrease on a small PML-truncated FWI problem.
"""
import numpy as np
import pytest

import oracle.fwi as F


def test_armijo_on_a_parabola():
    J = lambda a: (a - 0.3) ** 2
    alpha, Ja, nbt = F.armijo(J, J(0.0), -0.6, 1.0, 1e-4, 0.5, 20)
    assert (alpha, nbt) == (0.5, 1) and Ja == pytest.approx(0.04)
    assert F.armijo(lambda a: 1.0 + a, 1.0, -1.0, 1.0, 1e-4, 0.5, 5)[0] is None


def _pairs(n, k, seed, w):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n))
    A = A @ A.T + n * np.eye(n)          # SPD Hessian in the Euclidean sense
    pairs = []
    for _ in range(k):
        s = rng.standard_normal(n)
        y = np.linalg.solve(np.diag(w), A @ s)   # change of a W-representer gradient
        pairs.append((s, y))
    return pairs


@pytest.mark.parametrize("weighted", [False, True])
def test_lbfgs_operator_secant_symmetric_positive(weighted):
    n = 12
    w = np.linspace(0.5, 2.0, n) if weighted else np.ones(n)
    pairs = _pairs(n, 5, 1, w)
    H = lambda v: -F.lbfgs_direction(v, pairs, w)
    s_last, y_last = pairs[-1]
    assert np.allclose(H(y_last), s_last, rtol=1e-10, atol=1e-12)      # secant equation
    rng = np.random.default_rng(2)
    a, b = rng.standard_normal((2, n))
    assert F.wdot(H(a), b, w) == pytest.approx(F.wdot(a, H(b), w), rel=1e-10)
    assert F.wdot(H(a), a, w) > 0


def test_loop_converges_on_a_weighted_quadratic():
    n = 6
    rng = np.random.default_rng(3)
    A = rng.standard_normal((2 * n, 2 * n))
    A = A @ A.T + 2 * n * np.eye(2 * n)
    b = rng.standard_normal(2 * n)
    mass = np.linspace(0.7, 1.3, n)
    x_star = np.linalg.solve(A, b)

    class Quad(F.Problem):
        def forward(self, lam, mu):
            x = np.concatenate([lam, mu])
            self._x = x
            self.last_J = 0.5 * (x - x_star) @ A @ (x - x_star) + 1.0     # positive, like a misfit
            return self.last_J

        def gradient(self):
            g = A @ self._x - b
            return g[:n], g[n:]

    opts = F.Options(reg=None, bias_iters=0, max_iter=80, first_step=0.5)
    lam, mu, h = F.invert([Quad()], np.ones(n), np.ones(n), mass, opts)
    assert np.allclose(np.concatenate([lam, mu]), x_star, atol=1e-7)
    assert all(b2 <= a2 for a2, b2 in zip(h.J_total, h.J_total[1:]))


def test_regularization_factor_and_bias_identities():
    rng = np.random.default_rng(4)
    gm, gr = rng.standard_normal((2, 50))
    R = F.reg_factor(gm, gr, 0.4)
    assert R * np.linalg.norm(gr) == pytest.approx(0.4 * np.linalg.norm(gm))
    sl, sm = rng.standard_normal((2, 50))
    full = F.bias_lambda(sl, sm, 1.0)
    assert np.linalg.norm(full) == pytest.approx(np.linalg.norm(sl))
    assert np.allclose(full / np.linalg.norm(full), sm / np.linalg.norm(sm))
    assert np.array_equal(F.bias_lambda(sl, sm, 0.0), sl)


@pytest.mark.parametrize("reg", ["tikhonov", "tv"])
def test_fwi_on_a_small_pml_problem_decreases_the_misfit(reg):
    from helpers import observed, workload
    from oracle.assemble import System
    from oracle.regularize import Regularizer
    from oracle.solve import Stepper
    name = "tiny"
    wl = workload(name)
    obs = observed(name)

    def make(lam, mu):
        return Stepper(System(wl.prob, wl.rho, lam, mu), wl.src_node, wl.src_dir, wl.rec_node)

    r = Regularizer(wl.prob)
    opts = F.Options(reg=reg, tv_eps=1e10, max_iter=4)
    stage = F.OracleStage(make, r, wl.wavelet, obs, opts)
    lam, mu, h = F.invert([stage], wl.lam, wl.mu, r.mass, opts)
    assert len(h.J) == 5
    assert all(b <= a for a, b in zip(h.J_total, h.J_total[1:]))
    assert h.J[-1] < 0.5 * h.J[0]
