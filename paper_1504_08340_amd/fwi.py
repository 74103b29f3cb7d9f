"""Reduced-space FWI (Sec. 3.2-3.3) on the GPU: Algorithm 2 with L-BFGS and
Algorithm 1 (Armijo backtracking), regularization factor rule (24),
source-frequency continuation (3.3.2) and the biased lambda direction (25).

Every PDE solve, the regularization terms (8)/(9), M~ (C.1a), the control
problem (18), every inner product, the vector updates (fwi_axpby: the L-BFGS
recursion, the model update (19), the biased direction (25), gradient
differences) and the max-norms (fwi_absmax) run in libpmlfwi.so; torch
holds the vectors and concatenates them.  FP64 for the model, the gradients, the misfit and
the optimizer's inner products; the wavefield precision is the solver's.

Choices the paper leaves open:
* L-BFGS keeps m pairs (m = 15 in the paper) in the M~-weighted inner
  product on the L2 representer g of (18), so the Armijo slope <g, s> is the
  directional derivative of J.  H0 = <s,y>/<y,y>; without pairs the step is
  -g scaled to max|s| = first_step * max|m|.  A pair is kept only when
  <s, y> > 0; memory is cleared at every frequency stage.
* R of (24) is recomputed at the start of every iteration with
  wp falling linearly from wp_start to wp_end over wp_iters iterations, and
  held fixed during that iteration's line search.  Norms in (22)-(25) are
  Euclidean.
* The bias weight W of (25) falls linearly from 1 at the first iteration to
  0 at bias_iters.
* A line search that fails after max_backtracks halvings ends the stage.
"""
from __future__ import annotations

import math

import time
from dataclasses import dataclass, field

import torch

from . import binding as B


@dataclass
class FwiOptions:
    reg: str | None = "tikhonov"      # "tikhonov", "tv" or None
    tv_eps: float = 1e-2
    wp_start: float = 0.5
    wp_end: float = 0.3
    wp_iters: int = 50
    memory: int = 15
    c1: float = 1e-4
    rho: float = 0.5
    alpha0: float = 1.0
    max_backtracks: int = 20
    bias_iters: int = 50
    first_step: float = 0.05
    invert_lam: bool = True
    invert_mu: bool = True
    max_iter: int = 10
    tol: float = 0.0


@dataclass
class FwiHistory:
    J: list = field(default_factory=list)
    J_total: list = field(default_factory=list)
    alpha: list = field(default_factory=list)
    backtracks: list = field(default_factory=list)
    R: list = field(default_factory=list)
    seconds: list = field(default_factory=list)     # wall time at each entry of J
    solves: int = 0                                  # forward solves
    adjoints: int = 0


class FwiStage:
    """One frequency stage: a wavelet and the observed traces it produced."""

    def __init__(self, solver, rho, wavelet, observed, opts: FwiOptions):
        self.S, self.rho, self.wav, self.obs, self.opts = solver, rho, wavelet, observed, opts
        self.last_J = None
        self._lam = self._mu = None
        self._res = None
        dev = solver.device
        self._J = torch.empty(1, dtype=torch.float64, device=dev)
        self._v = torch.empty(1, dtype=torch.float64, device=dev)
        self.counts = [0, 0]

    def forward(self, lam, mu):
        """J_mis of the model; +inf for a model the solver must not run (non-positive
        rho, mu or bulk term, or a time step above the model's stability bound),
        which the line search then rejects."""
        lam, mu = lam.contiguous(), mu.contiguous()
        try:
            tr = self.S.forward(self.rho, lam, mu, self.wav)   # checks the model first
        except B.FwiError as e:
            if e.status not in (B.FWI_ERR_ARG, B.FWI_ERR_UNSTABLE):
                raise
            self.last_J = float("inf")
            self._lam = None
            return self.last_J
        _, self._res = self.S.misfit(tr, self.obs, J=self._J)
        self._lam, self._mu = lam, mu
        self.counts[0] += 1
        self.last_J = float(self._J[0])
        if not math.isfinite(self.last_J):
            # a stable dt cannot blow up; treat it like a rejected model
            self.last_J = float("inf")
            self._lam = None
        return self.last_J

    def gradient(self):
        self.counts[1] += 1
        return self.S.adjoint_gradient(self.rho, self._lam, self._mu, self.wav, self._res)

    def regularize(self, f):
        kind = B.FWI_REG_TIKHONOV if self.opts.reg == "tikhonov" else B.FWI_REG_TV
        eps = 0.0 if kind == B.FWI_REG_TIKHONOV else self.opts.tv_eps
        g = torch.empty_like(f)
        B.fwi_regularization(self.S.plan, None, kind, eps, f, self._v, g)
        return float(self._v[0]), g


class _Dots:
    """Deterministic device inner products (fwi_dot), results on the host."""

    def __init__(self, dev):
        self.out = torch.empty(1, dtype=torch.float64, device=dev)

    def __call__(self, a, b, w=None):
        B.fwi_dot(None, a.numel(), a, b, w, self.out)
        return float(self.out[0])


def _axpby(alpha, x, beta=0.0, y=None, out=None):
    """alpha x + beta y on the device (fwi_axpby); a new tensor unless out."""
    out = torch.empty_like(x) if out is None else out
    B.fwi_axpby(None, x.numel(), alpha, x, beta, y, out)
    return out


class _AbsMax:
    def __init__(self, dev):
        self.out = torch.empty(1, dtype=torch.float64, device=dev)

    def __call__(self, x):
        B.fwi_absmax(None, x.numel(), x, self.out)
        return float(self.out[0])


def _lbfgs_direction(dot, g, pairs, w):
    if not pairs:
        return None
    q = _axpby(1.0, g)
    coef = []
    for s, y in reversed(pairs):
        r = 1.0 / dot(y, s, w)
        a = r * dot(s, q, w)
        coef.append((a, r))
        _axpby(1.0, q, -a, y, out=q)
    s_last, y_last = pairs[-1]
    _axpby(dot(s_last, y_last, w) / dot(y_last, y_last, w), q, out=q)
    for (s, y), (a, r) in zip(pairs, reversed(coef)):
        b = r * dot(y, q, w)
        _axpby(1.0, q, a - b, s, out=q)
    return _axpby(-1.0, q, out=q)


def invert(stages, lam0, mu0, mass, opts: FwiOptions, history: FwiHistory | None = None,
           on_iter=None):
    """Algorithm 2 over the stages; lam0, mu0, mass: FP64 device tensors (n_int).

    Returns (lam, mu, history).  on_iter(it, J_mis, lam, mu) is called after
    every accepted step (and may return True to stop)."""
    h = history or FwiHistory()
    t0 = time.perf_counter()
    dot = _Dots(lam0.device)
    absmax = _AbsMax(lam0.device)
    n = lam0.numel()
    lam, mu = lam0.clone(), mu0.clone()
    w = torch.cat([mass, mass])
    it = 0
    zeros = torch.zeros_like(lam)
    stop = False
    for st in stages:
        if stop:
            break
        pairs = []
        Jm = st.forward(lam, mu)
        if Jm == float("inf"):
            raise ValueError("the start model fails fwi_check_model (non-physical materials or "
                             "a time step above its stability bound)")
        gl_mis, gm_mis = st.gradient()
        for k in range(opts.max_iter):
            if Jm <= opts.tol:
                break
            wp = opts.wp_start + (opts.wp_end - opts.wp_start) * min(1.0, it / max(1, opts.wp_iters))
            Rl = Rm = 0.0
            vl = vm = 0.0
            gl_reg, gm_reg = zeros, zeros
            if opts.reg is not None:
                vl, gl_reg = st.regularize(lam)
                vm, gm_reg = st.regularize(mu)
                if opts.invert_lam:
                    nr = dot(gl_reg, gl_reg) ** 0.5
                    Rl = 0.0 if nr == 0 else wp * dot(gl_mis, gl_mis) ** 0.5 / nr
                if opts.invert_mu:
                    nr = dot(gm_reg, gm_reg) ** 0.5
                    Rm = 0.0 if nr == 0 else wp * dot(gm_mis, gm_mis) ** 0.5 / nr
            J0 = Jm + Rl * vl + Rm * vm
            if k == 0:
                h.J.append(Jm)
                h.J_total.append(J0)
                h.seconds.append(time.perf_counter() - t0)

            def representer(gm_l, gm_m, greg_l, greg_m):
                gl = torch.empty_like(lam)
                gmu = torch.empty_like(mu)
                if opts.invert_lam:
                    B.fwi_gradient_finalize(st.S.plan, None, gm_l, greg_l, Rl, gl)
                else:
                    gl.zero_()
                if opts.invert_mu:
                    B.fwi_gradient_finalize(st.S.plan, None, gm_m, greg_m, Rm, gmu)
                else:
                    gmu.zero_()
                return torch.cat([gl, gmu])

            g = representer(gl_mis, gm_mis, gl_reg, gm_reg)
            gmax = absmax(g)
            if gmax == 0.0:
                stop = True
                break
            mmax = max(absmax(lam), absmax(mu))
            s = _lbfgs_direction(dot, g, pairs, w)
            if s is None:
                s = _axpby(-opts.first_step * mmax / gmax, g)
            if opts.invert_lam and opts.invert_mu and opts.bias_iters > 0:
                W = max(0.0, 1.0 - it / opts.bias_iters)
                sl, sm = s[:n], s[n:]
                nl, nm = dot(sl, sl) ** 0.5, dot(sm, sm) ** 0.5
                if W > 0 and nl > 0 and nm > 0:
                    biased = torch.empty_like(s)
                    _axpby(W * nl / nm, sm, 1.0 - W, sl, out=biased[:n])     # (25)
                    biased[n:].copy_(sm)
                    s = biased
            slope = dot(g, s, w)
            if slope >= 0:
                pairs = []
                s = _axpby(-opts.first_step * mmax / gmax, g)
                slope = dot(g, s, w)
            s_lam, s_mu = s[:n], s[n:]

            alpha = opts.alpha0
            accepted = None
            nbt = 0
            for nbt in range(opts.max_backtracks + 1):
                lt, mt = _axpby(1.0, lam, alpha, s_lam), _axpby(1.0, mu, alpha, s_mu)      # (19)
                Ja = st.forward(lt, mt)
                if opts.reg is not None:
                    Ja += Rl * st.regularize(lt)[0] + Rm * st.regularize(mt)[0]
                if Ja < J0 + opts.c1 * alpha * slope:
                    accepted = (lt, mt, Ja)
                    break
                alpha *= opts.rho
            h.backtracks.append(nbt)
            h.R.append((Rl, Rm))
            if accepted is None:
                break
            lam, mu, J1 = accepted
            Jm = st.last_J
            gl_new, gm_new = st.gradient()
            if opts.reg is not None:
                greg_l = st.regularize(lam)[1] if opts.invert_lam else zeros
                greg_m = st.regularize(mu)[1] if opts.invert_mu else zeros
            else:
                greg_l = greg_m = zeros
            g1 = representer(gl_new, gm_new, greg_l, greg_m)
            y = _axpby(1.0, g1, -1.0, g)
            sk = _axpby(alpha, s)
            if dot(sk, y, w) > 0:
                pairs.append((sk, y))
                if len(pairs) > opts.memory:
                    pairs.pop(0)
            gl_mis, gm_mis = gl_new, gm_new
            h.J.append(Jm)
            h.J_total.append(J1)
            h.alpha.append(alpha)
            h.seconds.append(time.perf_counter() - t0)
            it += 1
            if on_iter is not None and on_iter(it, Jm, lam, mu):
                stop = True
                break
        h.solves += st.counts[0]
        h.adjoints += st.counts[1]
        st.counts = [0, 0]
    return lam, mu, h
