"""Reduced-space inversion of Sec. 3.2-3.3 (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The steps, in the paper's order (Algorithm 2):
  state problem -> misfit -> adjoint -> gradient (18) -> L-BFGS search
  direction -> Armijo backtracking (Algorithm 1) -> update (19).
Buttressing schemes: regularization factor R = wp |g_mis| / |g_reg| (24)
per iteration and field; source-frequency continuation (3.3.2: a list of
stages, each started from the previous result); biased lambda direction (25)
with a weight falling linearly from 1 to 0.

Readings where the paper is silent:
* L-BFGS (m = 15 pairs, footnote of Sec. 3.2) uses the M~-weighted inner
  product <a, b> = sum a_i b_i M~_i on the L2 representer g = M~^{-1} gbar of
  (18); the Armijo slope is then <g, s> = gbar . s, the directional
  derivative.  Initial scaling H0 = <s, y>/<y, y>; with no pairs the step is
  -g scaled so that max|s| = first_step * max|m|.
* R is fixed during an iteration's line search and recomputed from the
  gradient parts at the start of the next iteration.
* The norms of (22)-(25) are Euclidean, as the paper states.
* A pair (s, y) is kept only when <s, y> > 0; memory is cleared at every
  frequency stage.  A line search that fails after max_backtracks halvings
  ends the stage.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Options:
    reg: str | None = "tikhonov"      # "tikhonov", "tv" or None
    tv_eps: float = 1e-2
    wp_start: float = 0.5             # wp of (24) at the first iteration
    wp_end: float = 0.3               # ... reached after wp_iters iterations
    wp_iters: int = 50
    memory: int = 15
    c1: float = 1e-4
    rho: float = 0.5
    alpha0: float = 1.0
    max_backtracks: int = 20
    bias_iters: int = 50              # W of (25): 1 at iteration 0, 0 from here on
    first_step: float = 0.05
    invert_lam: bool = True
    invert_mu: bool = True
    max_iter: int = 10                # per stage
    tol: float = 0.0                  # stop when J_mis <= tol


@dataclass
class History:
    J: list = field(default_factory=list)          # J_mis after every accepted step (and the start)
    J_total: list = field(default_factory=list)
    alpha: list = field(default_factory=list)
    backtracks: list = field(default_factory=list)
    R: list = field(default_factory=list)


def wdot(a, b, w):
    return float(np.sum(a * b * w))


def lbfgs_direction(g, pairs, w):
    """-H g by the two-loop recursion in the w-weighted inner product."""
    if not pairs:
        return None
    q = g.copy()
    alphas = []
    for s, y in reversed(pairs):
        rho = 1.0 / wdot(y, s, w)
        a = rho * wdot(s, q, w)
        alphas.append((a, rho))
        q -= a * y
    s_last, y_last = pairs[-1]
    r = (wdot(s_last, y_last, w) / wdot(y_last, y_last, w)) * q
    for (s, y), (a, rho) in zip(pairs, reversed(alphas)):
        b = rho * wdot(y, r, w)
        r += (a - b) * s
    return -r


def armijo(J_of, J0, slope, alpha0, c1, rho, max_backtracks):
    """Algorithm 1: largest alpha = alpha0 rho^k with J(alpha) < J0 + c1 alpha slope."""
    alpha = alpha0
    for k in range(max_backtracks + 1):
        Ja = J_of(alpha)
        if Ja < J0 + c1 * alpha * slope:
            return alpha, Ja, k
        alpha *= rho
    return None, None, max_backtracks


def bias_lambda(s_lam, s_mu, W):
    """(25): s_lam <- |s_lam| (W s_mu/|s_mu| + (1-W) s_lam/|s_lam|)."""
    nl, nm = np.linalg.norm(s_lam), np.linalg.norm(s_mu)
    if W <= 0 or nl == 0 or nm == 0:
        return s_lam
    return nl * (W * s_mu / nm + (1 - W) * s_lam / nl)


def reg_factor(g_mis, g_reg, wp):
    """(24): R = wp |g_mis| / |g_reg| (0 when the field has no gradient)."""
    nr = np.linalg.norm(g_reg)
    return 0.0 if nr == 0 else wp * np.linalg.norm(g_mis) / nr


class Problem:
    """What the loop needs from the PDE side, for one frequency stage.

    forward(lam, mu) -> J_mis (and keeps what gradient() needs);
    gradient() -> (gbar_lam, gbar_mu) of J_mis at the last forward point;
    regularize(f) -> (value, gradient) of the chosen term;
    mass: M~ diagonal.
    """


def invert(stages, lam0, mu0, mass, opts: Options, history: History | None = None):
    """Algorithm 2 over the frequency stages; returns (lam, mu, history)."""
    h = history or History()
    lam, mu = lam0.copy(), mu0.copy()
    it = 0
    for prob in stages:
        pairs = []
        Jm = prob.forward(lam, mu)
        gl_mis, gm_mis = prob.gradient()
        for k in range(opts.max_iter):
            if Jm <= opts.tol:
                break
            wp = opts.wp_start + (opts.wp_end - opts.wp_start) * min(1.0, it / max(1, opts.wp_iters))
            # regularization at the current point, R from (24)
            Rl = Rm = 0.0
            vl = vm = 0.0
            gl_reg = np.zeros_like(lam)
            gm_reg = np.zeros_like(mu)
            if opts.reg is not None:
                vl, gl_reg = prob.regularize(lam)
                vm, gm_reg = prob.regularize(mu)
                Rl = reg_factor(gl_mis, gl_reg, wp) if opts.invert_lam else 0.0
                Rm = reg_factor(gm_mis, gm_reg, wp) if opts.invert_mu else 0.0
            J0 = Jm + Rl * vl + Rm * vm
            if k == 0:
                h.J.append(Jm)
                h.J_total.append(J0)
            # (18): representer of the total gradient
            gl = (gl_mis + Rl * gl_reg) / mass if opts.invert_lam else np.zeros_like(lam)
            gm = (gm_mis + Rm * gm_reg) / mass if opts.invert_mu else np.zeros_like(mu)
            g = np.concatenate([gl, gm])
            if np.abs(g).max() == 0.0:           # stationary point
                break
            w = np.concatenate([mass, mass])
            s = lbfgs_direction(g, pairs, w)
            if s is None:
                scale = opts.first_step * max(np.abs(lam).max(), np.abs(mu).max()) / np.abs(g).max()
                s = -scale * g
            n = lam.size
            s_lam, s_mu = s[:n], s[n:]
            if opts.invert_lam and opts.invert_mu:
                W = max(0.0, 1.0 - it / opts.bias_iters) if opts.bias_iters > 0 else 0.0
                s_lam = bias_lambda(s_lam, s_mu, W)
                s = np.concatenate([s_lam, s_mu])
            slope = wdot(g, s, w)
            if slope >= 0:                       # not a descent direction: restart
                pairs = []
                scale = opts.first_step * max(np.abs(lam).max(), np.abs(mu).max()) / np.abs(g).max()
                s = -scale * g
                s_lam, s_mu = s[:n], s[n:]
                slope = wdot(g, s, w)

            def J_of(alpha):
                lt, mt = lam + alpha * s_lam, mu + alpha * s_mu
                val = prob.forward(lt, mt)
                if opts.reg is not None:
                    val += Rl * prob.regularize(lt)[0] + Rm * prob.regularize(mt)[0]
                return val

            alpha, J1, nbt = armijo(J_of, J0, slope, opts.alpha0, opts.c1, opts.rho, opts.max_backtracks)
            h.backtracks.append(nbt)
            h.R.append((Rl, Rm))
            if alpha is None:
                break
            lam, mu = lam + alpha * s_lam, mu + alpha * s_mu
            # the last forward solve was at the accepted point
            Jm = prob.last_J
            gl_new, gm_new = prob.gradient()
            gl1 = (gl_new + Rl * (prob.regularize(lam)[1] if opts.reg else 0.0)) / mass if opts.invert_lam \
                else np.zeros_like(lam)
            gm1 = (gm_new + Rm * (prob.regularize(mu)[1] if opts.reg else 0.0)) / mass if opts.invert_mu \
                else np.zeros_like(mu)
            y = np.concatenate([gl1, gm1]) - g
            sk = alpha * s
            if wdot(sk, y, w) > 0:
                pairs.append((sk, y))
                if len(pairs) > opts.memory:
                    pairs.pop(0)
            gl_mis, gm_mis = gl_new, gm_new
            h.J.append(Jm)
            h.J_total.append(J1)
            h.alpha.append(alpha)
            it += 1
    return lam, mu, h


class OracleStage(Problem):
    """One frequency stage on the oracle solver: wavelet + observed traces.

    make_stepper(lam, mu) builds the oracle operators for a material model
    (the assembled ``System`` or ``MatFree`` in a ``Stepper``)."""

    def __init__(self, make_stepper, regularizer, wavelet, observed, opts: Options):
        self.make, self.reg, self.wav, self.obs, self.opts = make_stepper, regularizer, wavelet, observed, opts
        self.last_J = None
        self._st = None
        self._states = None

    def forward(self, lam, mu):
        self._st = self.make(lam, mu)
        tr, states = self._st.forward(self.wav, store=True)
        self._states = states
        self.last_J = self._st.misfit(tr, self.obs)
        return self.last_J

    def gradient(self):
        gl, gm, _ = self._st.adjoint_gradient(self.wav, self.obs, self._states)
        return gl, gm

    def regularize(self, f):
        if self.opts.reg == "tikhonov":
            return self.reg.tikhonov(f)
        return self.reg.total_variation(f, self.opts.tv_eps)
