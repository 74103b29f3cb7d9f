"""Device buffers for one problem, held in torch tensors, and calls into the C ABI.

Nothing here computes: the tensors are allocated with torch (memory and
streams only) and every step of the method runs in libpmlfwi.so.
"""
from __future__ import annotations

import numpy as np
import torch

from . import binding as B


def check_tensor(name, t, numel, device, dtype=torch.float64):
    """Raise ValueError unless t is a contiguous tensor of dtype on device with
    numel elements: the C entry points take raw pointers and would read or
    write past a short or mistyped buffer."""
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name}: expected a torch.Tensor, got {type(t).__name__}")
    if t.dtype != dtype:
        raise ValueError(f"{name}: dtype {t.dtype}, expected {dtype}")
    if t.device != torch.device(device):
        raise ValueError(f"{name}: on {t.device}, expected {device}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: not contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name}: {t.numel()} elements, expected {numel}")
    return t


class Solver:
    """One plan + workspace on a CUDA/HIP device.

    Parameters mirror ``fwi_problem``; ``prob`` is any object with the fields
    of ``workloads.Problem`` (ne_int, npml_side, npml_bottom, h, dt, nsteps,
    pml_alpha0, pml_beta0, pml_m).
    """

    def __init__(self, prob, src_node, src_dir, rec_node, precision=B.FWI_FP64,
                 ckpt_every=0, device="cuda", traction=None, grad_full=False, ckpt_slots=0):
        """traction: None (point loads src_node / src_dir), or (xmin, xmax,
        ymin, ymax, direction) of a uniform surface traction applied by every
        source; the wavelet is then the traction in Pa.  ckpt_every = -1 makes
        a forward-only plan.  grad_full: the gradient includes the PML terms
        of the material carried outward from the interface.  ckpt_slots: with
        ckpt_every = k > 0, at most that many stored states and binomial
        checkpointing over the k-step segments (0: a state per segment)."""
        if not torch.cuda.is_available():
            raise RuntimeError("Solver needs a GPU (HIP device); no CPU fallback exists")
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device(self.device.type, torch.cuda.current_device())
        self.nsrc = int(len(src_node))
        self.nrec = int(len(rec_node))
        self.problem = B.make_problem(prob, self.nsrc, self.nrec, precision, ckpt_every, grad_full, ckpt_slots)
        self.sizes = B.fwi_query(self.problem)
        self.nsteps = prob.nsteps
        self.plan = B.fwi_plan_create(self.problem, np.asarray(src_node), np.asarray(src_dir),
                                      np.asarray(rec_node))
        if traction is not None:
            xmin, xmax, ymin, ymax, direction = traction
            node, weight = B.fwi_surface_traction(self.problem, xmin, xmax, ymin, ymax)
            vec = weight[:, None] * np.asarray(direction, np.float64)[None, :]
            B.fwi_plan_set_loads(self.plan, np.repeat(np.arange(self.nsrc), node.size),
                                 np.tile(node, self.nsrc), np.tile(vec, (self.nsrc, 1)))
        nbytes = int(self.sizes.workspace_bytes)
        try:
            self.workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        except torch.cuda.OutOfMemoryError as e:
            B.fwi_plan_destroy(self.plan)
            self.plan = None
            raise MemoryError(
                f"the workspace of this problem needs {nbytes / 2**30:.1f} GiB of device memory; keep fewer "
                "stages: ckpt_every = k > 0 stores a full state every k steps and recomputes the "
                "segment, ckpt_slots bounds the number of stored states") from e
        self.trace_shape = (self.nsrc, self.nsteps + 1, self.nrec, 3)
        self.generation = 0     # bumped by every forward solve (see autograd.py)

    def close(self):
        if self.plan is not None:
            B.fwi_plan_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers -----------------------------------------------------------
    def tensor(self, a, dtype=torch.float64):
        if isinstance(a, torch.Tensor):
            return a.to(device=self.device, dtype=dtype).contiguous()
        return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=self.device)

    def empty_traces(self):
        return torch.empty(self.trace_shape, dtype=torch.float64, device=self.device)

    # -- argument checks (before any C call) ---------------------------------
    def _model(self, rho, lam, mu):
        n = int(self.sizes.n_int_nodes)
        for name, t in (("rho", rho), ("lam", lam), ("mu", mu)):
            check_tensor(name, t, n, self.device)

    def _wavelet(self, wavelet):
        check_tensor("wavelet", wavelet, self.nsrc * (2 * self.nsteps + 1), self.device)

    def _trace(self, name, t):
        check_tensor(name, t, int(np.prod(self.trace_shape)), self.device)

    def _nodal(self, name, t):
        check_tensor(name, t, self.nsrc * 9 * int(self.sizes.n_nodes), self.device)

    # -- C ABI calls -------------------------------------------------------
    def forward(self, rho, lam, mu, wavelet, traces=None, stream=None):
        traces = self.empty_traces() if traces is None else traces
        self._model(rho, lam, mu)
        self._wavelet(wavelet)
        self._trace("traces", traces)
        self.generation += 1
        B.fwi_forward(self.plan, stream, rho, lam, mu, wavelet, self.workspace, traces)
        return traces

    def misfit(self, traces, observed, residual=None, J=None, stream=None):
        residual = torch.empty_like(traces) if residual is None else residual
        J = torch.empty(1, dtype=torch.float64, device=self.device) if J is None else J
        for name, t in (("traces", traces), ("observed", observed), ("residual", residual)):
            self._trace(name, t)
        check_tensor("J", J, 1, self.device)
        B.fwi_misfit(self.plan, stream, traces, observed, residual, J)
        return J, residual

    def adjoint_gradient(self, rho, lam, mu, wavelet, residual, g_lam=None, g_mu=None, stream=None,
                         scheme="discrete"):
        """scheme "discrete": exact derivative of the discrete misfit; "appb": the
        paper's reverse-time RK4 of App. B (optimize-then-discretize)."""
        n = int(self.sizes.n_int_nodes)
        g_lam = torch.empty(n, dtype=torch.float64, device=self.device) if g_lam is None else g_lam
        g_mu = torch.empty(n, dtype=torch.float64, device=self.device) if g_mu is None else g_mu
        self._model(rho, lam, mu)
        self._wavelet(wavelet)
        self._trace("residual", residual)
        check_tensor("g_lam", g_lam, n, self.device)
        check_tensor("g_mu", g_mu, n, self.device)
        fn = {"discrete": B.fwi_adjoint_gradient, "appb": B.fwi_adjoint_gradient_appb}[scheme]
        fn(self.plan, stream, rho, lam, mu, wavelet, residual, self.workspace, g_lam, g_mu)
        return g_lam, g_mu

    def apply_operator(self, which, rho, lam, mu, x0, x1, x2, out=None, stream=None):
        out = torch.empty_like(x1) if out is None else out
        self._model(rho, lam, mu)
        for name, t in (("x0", x0), ("x1", x1), ("x2", x2), ("out", out)):
            self._nodal(name, t)
        B.fwi_apply_operator(self.plan, stream, which, rho, lam, mu, x0, x1, x2, self.workspace, out)
        return out
