"""The misfit (7) as a differentiable function of the Lame parameters.

``misfit(lam, mu, solver, rho, wavelet, observed)`` returns J as a 0-d FP64
tensor.  Its backward is the adjoint-state gradient of Sec. 3 (adjoint
problem (15), gradient (18) with R = 0) restricted to the interior bricks as
Sec. 3.1.3 prescribes: the derivative of the discrete misfit with respect to
the nodal lam and mu on the closed interior, with the PML-brick terms left
out.  PML nodes take their material from the interface nodes, so on nodes of
the interface (the boundary of the closed interior box, free surface
excepted) this vector is not the full derivative of J; everywhere else it is
the exact derivative that finite differences of J converge to.  A caller who
composes this function with other torch operations gets the restricted
vector at the interface nodes.  Both directions run in the HIP library
behind ``solver``; this module only routes tensors.

The forward solve leaves in the solver's workspace what the adjoint sweep
reads: every stage displacement (``ckpt_every = 0``) or a full state every k
steps, from which each k-step segment is recomputed during the reverse sweep
(``ckpt_every = k``; workspace shrinks roughly by k, at the price of one more
forward solve).  A second forward solve on the same solver before
``backward`` overwrites that state; backward then raises instead of
returning a wrong gradient.
"""
from __future__ import annotations

import torch


class MisfitFunction(torch.autograd.Function):
    """J(lam, mu); d J / d(lam, mu) from one adjoint sweep."""

    @staticmethod
    def forward(ctx, lam, mu, solver, rho, wavelet, observed):
        lam_c, mu_c = lam.detach().contiguous(), mu.detach().contiguous()
        traces = solver.forward(rho, lam_c, mu_c, wavelet)
        J, residual = solver.misfit(traces, observed)
        if not torch.isfinite(J).all():
            raise FloatingPointError(f"misfit is not finite ({J.item()}): the forward solve diverged")
        ctx.solver = solver
        ctx.generation = solver.generation
        ctx.save_for_backward(rho, lam_c, mu_c, wavelet, residual)
        return J.reshape(())

    @staticmethod
    def backward(ctx, gJ):
        solver = ctx.solver
        if solver.generation != ctx.generation:
            raise RuntimeError("the solver ran another forward solve after this misfit was "
                               "evaluated; its stored states no longer belong to this graph")
        rho, lam, mu, wavelet, residual = ctx.saved_tensors
        g_lam, g_mu = solver.adjoint_gradient(rho, lam, mu, wavelet, residual)
        return gJ * g_lam, gJ * g_mu, None, None, None, None


def misfit(lam, mu, solver, rho, wavelet, observed):
    """J = 1/2 sum_n dt w_n |R u^n - d^n|^2 over sources, receivers and steps."""
    return MisfitFunction.apply(lam, mu, solver, rho, wavelet, observed)
