"""ctypes binding of libpmlfwi.so (argument marshalling only).

Every function here has the name of the C entry point it calls and forwards
plain device pointers taken from torch tensors; all computation happens in
the HIP kernels of the library.  Importing this module fails loudly when the
library has not been built.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("PMLFWI_LIB") or os.path.join(HERE, "libpmlfwi.so")

FWI_FP64, FWI_FP32, FWI_FP32_MFMA, FWI_FP32_BF16X3 = 0, 1, 2, 3

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
        "or `python paper_1504_08340_amd/_build.py` (hipcc, gfx950)")

# torch ships its own HIP runtime; it must be the one in the process before
# the library is loaded, so that the library's HIP calls and torch's device
# memory and streams share a single runtime (loading the library first pulls
# in a second runtime, which then sees no device).
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)


class fwi_problem(ctypes.Structure):
    _fields_ = [
        ("ne_int", ctypes.c_int32 * 3),
        ("npml_side", ctypes.c_int32),
        ("npml_bottom", ctypes.c_int32),
        ("h", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("nsteps", ctypes.c_int32),
        ("pml_alpha0", ctypes.c_double),
        ("pml_beta0", ctypes.c_double),
        ("pml_m", ctypes.c_int32),
        ("nsrc", ctypes.c_int32),
        ("nrec", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("ckpt_every", ctypes.c_int32),
        ("grad_full", ctypes.c_int32),
        ("ckpt_slots", ctypes.c_int32),
    ]


class fwi_sizes(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "n_nodes", "n_int_nodes", "n_pml_nodes", "n_state", "n_hist", "trace_len",
        "workspace_bytes", "register_bytes")] + [("tile", ctypes.c_int64 * 3)] + [
        (n, ctypes.c_int64) for n in ("tiles_interior", "tiles_pml", "element_threads", "ckpt_states",
                                      "schedule_advances", "adjoint_forward_steps")]


_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
_lib.fwi_query.argtypes = [ctypes.POINTER(fwi_problem), ctypes.POINTER(fwi_sizes)]
_lib.fwi_plan_create.argtypes = [ctypes.POINTER(fwi_problem), _P, _P, _P, ctypes.POINTER(_P)]
_lib.fwi_plan_destroy.argtypes = [_P]
_lib.fwi_forward.argtypes = [_P, _P, _P, _P, _P, _P, _P, _P]
_lib.fwi_forward_noalloc.argtypes = [_P, _P, _P, _P, _P, _P, _P]
_lib.fwi_plan_set_loads.argtypes = [_P, ctypes.c_int32, _P, _P, _P]
_lib.fwi_surface_traction.argtypes = [ctypes.POINTER(fwi_problem), ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_int32, _P, _P,
                                      ctypes.POINTER(ctypes.c_int32)]
_lib.fwi_misfit.argtypes = [_P, _P, _P, _P, _P, _P]
_lib.fwi_adjoint_gradient.argtypes = [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P]
_lib.fwi_adjoint_gradient_appb.argtypes = [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P]
_lib.fwi_apply_operator.argtypes = [_P, _P, ctypes.c_int, _P, _P, _P, _P, _P, _P, _P, _P]
_lib.fwi_timing_enable.argtypes = [_P, ctypes.c_int]
_lib.fwi_timing_read.argtypes = [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
_lib.fwi_status_string.argtypes = [ctypes.c_int]
_lib.fwi_status_string.restype = ctypes.c_char_p
_lib.fwi_last_error.argtypes = [_P]
_lib.fwi_last_error.restype = ctypes.c_char_p
_lib.fwi_regularization.argtypes = [_P, _P, ctypes.c_int, ctypes.c_double, _P, _P, _P]
_lib.fwi_material_mass.argtypes = [_P, _P, _P]
_lib.fwi_gradient_finalize.argtypes = [_P, _P, _P, _P, ctypes.c_double, _P]
_lib.fwi_dot.argtypes = [_P, ctypes.c_int64, _P, _P, _P, _P]
_lib.fwi_axpby.argtypes = [_P, ctypes.c_int64, ctypes.c_double, _P, ctypes.c_double, _P, _P]
_lib.fwi_absmax.argtypes = [_P, ctypes.c_int64, _P, _P]
_lib.fwi_check_model.argtypes = [_P, _P, _P, _P, _P, _P]


class fwi_conv_shape(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("N", "Ci", "D", "H", "W", "Co", "K", "sd", "sh", "sw")]


_CS = ctypes.POINTER(fwi_conv_shape)
_F = ctypes.c_float
_lib.fwi_conv3d_forward.argtypes = [_P, _CS, _P, _P, _P, ctypes.c_int, _P]
_lib.fwi_conv3d_backward.argtypes = [_P, _CS, _P, _P, _P, _P, ctypes.c_int, _P, _P, _P]
_lib.fwi_mse.argtypes = [_P, ctypes.c_int64, _P, _P, _P, _P]
_lib.fwi_to_bf16.argtypes = [_P, ctypes.c_int64, _P, _P]
_lib.fwi_conv3d_forward_bf16.argtypes = [_P, _CS, _P, _P, _P, ctypes.c_int, ctypes.c_int, _P]
_lib.fwi_adam.argtypes = [_P, ctypes.c_int64, _P, _P, _P, _P, _F, _F, _F, _F, ctypes.c_int]
_lib.fwi_trace_features.argtypes = [_P, _P, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P, ctypes.c_int,
                                    ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _F, _P]
_lib.fwi_grid_to_nodes.argtypes = [_P, _P, _P, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P, _P]
for _f in ("fwi_query", "fwi_plan_create", "fwi_plan_destroy", "fwi_plan_set_loads", "fwi_surface_traction", "fwi_forward", "fwi_forward_noalloc", "fwi_misfit",
           "fwi_adjoint_gradient", "fwi_adjoint_gradient_appb", "fwi_apply_operator", "fwi_timing_enable", "fwi_timing_read",
           "fwi_regularization", "fwi_material_mass", "fwi_gradient_finalize", "fwi_dot", "fwi_axpby", "fwi_absmax", "fwi_check_model",
           "fwi_conv3d_forward", "fwi_conv3d_backward", "fwi_to_bf16", "fwi_conv3d_forward_bf16", "fwi_mse", "fwi_adam", "fwi_trace_features",
           "fwi_grid_to_nodes"):
    getattr(_lib, _f).restype = ctypes.c_int

EXPORTS = ("fwi_query", "fwi_plan_create", "fwi_plan_destroy", "fwi_plan_set_loads", "fwi_surface_traction", "fwi_forward", "fwi_forward_noalloc", "fwi_misfit",
           "fwi_adjoint_gradient", "fwi_adjoint_gradient_appb", "fwi_apply_operator", "fwi_timing_enable", "fwi_timing_read",
           "fwi_regularization", "fwi_material_mass", "fwi_gradient_finalize", "fwi_dot", "fwi_axpby", "fwi_absmax", "fwi_check_model",
           "fwi_conv3d_forward", "fwi_conv3d_backward", "fwi_to_bf16", "fwi_conv3d_forward_bf16", "fwi_mse", "fwi_adam", "fwi_trace_features",
           "fwi_grid_to_nodes", "fwi_status_string", "fwi_last_error")
FWI_REG_TIKHONOV, FWI_REG_TV = 0, 1
KERNEL_CLASSES = ("interior", "pml", "nodal", "interior_adj", "pml_adj")


FWI_ERR_ARG, FWI_ERR_SHAPE, FWI_ERR_HIP, FWI_ERR_STATE, FWI_ERR_UNSTABLE, FWI_ERR_NOMEM = -1, -2, -3, -4, -5, -6


class FwiError(RuntimeError):
    """A non-zero fwi_status; ``status`` holds the code."""

    def __init__(self, msg, status=0):
        super().__init__(msg)
        self.status = status


def _check(status, plan=None, what=""):
    if status != 0:
        msg = _lib.fwi_status_string(status).decode()
        if plan or what == "fwi_plan_create":
            detail = _lib.fwi_last_error(plan or None).decode()
            if detail:
                msg += f": {detail}"
        raise FwiError(f"{what} failed ({status}): {msg}", status)


def make_problem(prob, nsrc, nrec, precision=FWI_FP64, ckpt_every=0, grad_full=0, ckpt_slots=0):
    """fwi_problem from a workloads.Problem-like object."""
    p = fwi_problem()
    p.ne_int[:] = list(prob.ne_int)
    p.npml_side = prob.npml_side
    p.npml_bottom = prob.npml_bottom
    p.h = prob.h
    p.dt = prob.dt
    p.nsteps = prob.nsteps
    p.pml_alpha0 = prob.pml_alpha0
    p.pml_beta0 = prob.pml_beta0
    p.pml_m = prob.pml_m
    p.nsrc = nsrc
    p.nrec = nrec
    p.precision = precision
    p.ckpt_every = ckpt_every
    p.grad_full = int(grad_full)
    p.ckpt_slots = int(ckpt_slots)
    return p


def fwi_query(problem: fwi_problem) -> fwi_sizes:
    out = fwi_sizes()
    _check(_lib.fwi_query(ctypes.byref(problem), ctypes.byref(out)), what="fwi_query")
    return out


def fwi_plan_create(problem: fwi_problem, src_node, src_dir, rec_node):
    """Host numpy arrays: src_node int32 (nsrc,), src_dir float64 (nsrc,3), rec_node int32 (nrec,)."""
    import numpy as np
    s = np.ascontiguousarray(src_node, dtype=np.int32)
    d = np.ascontiguousarray(src_dir, dtype=np.float64)
    r = np.ascontiguousarray(rec_node, dtype=np.int32)
    plan = _P()
    _check(_lib.fwi_plan_create(ctypes.byref(problem), s.ctypes.data, d.ctypes.data,
                                r.ctypes.data if r.size else None, ctypes.byref(plan)),
           what="fwi_plan_create")
    return plan


def fwi_plan_set_loads(plan, load_src, load_node, load_vec):
    """Host arrays: load_src int32 (n,), load_node int32 (n,), load_vec float64 (n, 3)."""
    import numpy as np
    s = np.ascontiguousarray(load_src, dtype=np.int32)
    n = np.ascontiguousarray(load_node, dtype=np.int32)
    v = np.ascontiguousarray(load_vec, dtype=np.float64).reshape(-1, 3)
    if not (s.size == n.size == v.shape[0]):
        raise ValueError("load_src, load_node and load_vec must have the same length")
    _check(_lib.fwi_plan_set_loads(plan, int(s.size), s.ctypes.data if s.size else None,
                                   n.ctypes.data if n.size else None, v.ctypes.data if v.size else None),
           plan, "fwi_plan_set_loads")


def fwi_surface_traction(problem: fwi_problem, xmin, xmax, ymin, ymax):
    """(node ids, weights) of a uniform surface traction over a rectangle."""
    import numpy as np
    count = ctypes.c_int32()
    st = _lib.fwi_surface_traction(ctypes.byref(problem), xmin, xmax, ymin, ymax, 0, None, None,
                                   ctypes.byref(count))
    if st not in (0, FWI_ERR_SHAPE):
        _check(st, what="fwi_surface_traction")
    node = np.zeros(count.value, np.int32)
    weight = np.zeros(count.value, np.float64)
    _check(_lib.fwi_surface_traction(ctypes.byref(problem), xmin, xmax, ymin, ymax, count.value,
                                     node.ctypes.data if node.size else None,
                                     weight.ctypes.data if weight.size else None, ctypes.byref(count)),
           what="fwi_surface_traction")
    return node, weight


def fwi_plan_destroy(plan):
    _check(_lib.fwi_plan_destroy(plan), what="fwi_plan_destroy")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(int(stream))


def fwi_forward(plan, stream, rho, lam, mu, wavelet, workspace, traces):
    _check(_lib.fwi_forward(plan, _stream(stream), _ptr(rho), _ptr(lam), _ptr(mu), _ptr(wavelet),
                            _ptr(workspace), _ptr(traces)), plan, "fwi_forward")


def fwi_forward_noalloc(plan, stream, rho, lam, mu, wavelet, traces):
    _check(_lib.fwi_forward_noalloc(plan, _stream(stream), _ptr(rho), _ptr(lam), _ptr(mu), _ptr(wavelet),
                                    _ptr(traces)), plan, "fwi_forward_noalloc")


def fwi_misfit(plan, stream, traces, observed, residual, J):
    _check(_lib.fwi_misfit(plan, _stream(stream), _ptr(traces), _ptr(observed), _ptr(residual),
                           _ptr(J)), plan, "fwi_misfit")


def fwi_adjoint_gradient(plan, stream, rho, lam, mu, wavelet, residual, workspace, g_lam, g_mu):
    _check(_lib.fwi_adjoint_gradient(plan, _stream(stream), _ptr(rho), _ptr(lam), _ptr(mu),
                                     _ptr(wavelet), _ptr(residual), _ptr(workspace), _ptr(g_lam),
                                     _ptr(g_mu)), plan, "fwi_adjoint_gradient")


def fwi_adjoint_gradient_appb(plan, stream, rho, lam, mu, wavelet, residual, workspace, g_lam, g_mu):
    _check(_lib.fwi_adjoint_gradient_appb(plan, _stream(stream), _ptr(rho), _ptr(lam), _ptr(mu),
                                          _ptr(wavelet), _ptr(residual), _ptr(workspace), _ptr(g_lam),
                                          _ptr(g_mu)), plan, "fwi_adjoint_gradient_appb")


def fwi_apply_operator(plan, stream, which, rho, lam, mu, x0, x1, x2, workspace, out):
    _check(_lib.fwi_apply_operator(plan, _stream(stream), int(which), _ptr(rho), _ptr(lam), _ptr(mu),
                                   _ptr(x0), _ptr(x1), _ptr(x2), _ptr(workspace), _ptr(out)),
           plan, "fwi_apply_operator")


def fwi_regularization(plan, stream, kind, eps, field, value, grad):
    _check(_lib.fwi_regularization(plan, _stream(stream), int(kind), float(eps), _ptr(field), _ptr(value),
                                   _ptr(grad)), plan, "fwi_regularization")


def fwi_material_mass(plan, stream, mdiag):
    _check(_lib.fwi_material_mass(plan, _stream(stream), _ptr(mdiag)), plan, "fwi_material_mass")


def fwi_gradient_finalize(plan, stream, g_mis, g_reg, R, g):
    _check(_lib.fwi_gradient_finalize(plan, _stream(stream), _ptr(g_mis), _ptr(g_reg), float(R), _ptr(g)),
           plan, "fwi_gradient_finalize")


def fwi_check_model(plan, stream, rho, lam, mu):
    """Returns the 6 host values of fwi_check_model; raises FwiError on a
    non-physical model (FWI_ERR_ARG) or an unstable dt (FWI_ERR_UNSTABLE)."""
    info = (ctypes.c_double * 6)()
    _check(_lib.fwi_check_model(plan, _stream(stream), _ptr(rho), _ptr(lam), _ptr(mu), info), plan,
           "fwi_check_model")
    return list(info)


def fwi_dot(stream, n, a, b, w, out):
    _check(_lib.fwi_dot(_stream(stream), int(n), _ptr(a), _ptr(b), _ptr(w), _ptr(out)), None, "fwi_dot")


def fwi_axpby(stream, n, alpha, x, beta, y, out):
    _check(_lib.fwi_axpby(_stream(stream), int(n), float(alpha), _ptr(x), float(beta), _ptr(y), _ptr(out)),
           None, "fwi_axpby")


def fwi_absmax(stream, n, x, out):
    _check(_lib.fwi_absmax(_stream(stream), int(n), _ptr(x), _ptr(out)), None, "fwi_absmax")


def conv_shape(N, Ci, D, H, W, Co, K, strides):
    s = fwi_conv_shape()
    s.N, s.Ci, s.D, s.H, s.W, s.Co, s.K = N, Ci, D, H, W, Co, K
    s.sd, s.sh, s.sw = strides
    return s


def fwi_conv3d_forward(stream, shape, x, w, b, relu, y):
    _check(_lib.fwi_conv3d_forward(_stream(stream), ctypes.byref(shape), _ptr(x), _ptr(w), _ptr(b), int(relu),
                                   _ptr(y)), None, "fwi_conv3d_forward")


def fwi_conv3d_backward(stream, shape, x, w, y, dy, relu, dx, dw, db):
    _check(_lib.fwi_conv3d_backward(_stream(stream), ctypes.byref(shape), _ptr(x), _ptr(w), _ptr(y), _ptr(dy),
                                    int(relu), _ptr(dx), _ptr(dw), _ptr(db)), None, "fwi_conv3d_backward")


def fwi_to_bf16(stream, n, x, out):
    _check(_lib.fwi_to_bf16(_stream(stream), int(n), _ptr(x), _ptr(out)), None, "fwi_to_bf16")


def fwi_conv3d_forward_bf16(stream, shape, x, w, b, relu, out_fp32, y):
    _check(_lib.fwi_conv3d_forward_bf16(_stream(stream), ctypes.byref(shape), _ptr(x), _ptr(w), _ptr(b), int(relu),
                                        int(out_fp32), _ptr(y)), None, "fwi_conv3d_forward_bf16")


def fwi_mse(stream, n, y, t, loss, grad):
    _check(_lib.fwi_mse(_stream(stream), int(n), _ptr(y), _ptr(t), _ptr(loss), _ptr(grad)), None, "fwi_mse")


def fwi_adam(stream, n, param, grad, m, v, lr, beta1, beta2, eps, step):
    _check(_lib.fwi_adam(_stream(stream), int(n), _ptr(param), _ptr(grad), _ptr(m), _ptr(v), float(lr),
                         float(beta1), float(beta2), float(eps), int(step)), None, "fwi_adam")


def fwi_trace_features(stream, traces, nsrc, nsteps, nrec, rec_idx, hw, T, t0, tstride, comp, scale, out):
    _check(_lib.fwi_trace_features(_stream(stream), _ptr(traces), int(nsrc), int(nsteps), int(nrec), _ptr(rec_idx),
                                   int(hw), int(T), int(t0), int(tstride), int(comp), float(scale), _ptr(out)),
           None, "fwi_trace_features")


def fwi_grid_to_nodes(plan, stream, coarse, gx, gy, gz, base, out):
    _check(_lib.fwi_grid_to_nodes(plan, _stream(stream), _ptr(coarse), int(gx), int(gy), int(gz), _ptr(base),
                                  _ptr(out)), plan, "fwi_grid_to_nodes")


def fwi_timing_enable(plan, stride):
    _check(_lib.fwi_timing_enable(plan, int(stride)), plan, "fwi_timing_enable")


def fwi_timing_read(plan, kernel_class):
    """(mean_ms, samples, launches) of the sampled launches of one kernel class."""
    m = ctypes.c_double()
    s = ctypes.c_int64()
    n = ctypes.c_int64()
    _check(_lib.fwi_timing_read(plan, int(kernel_class), ctypes.byref(m), ctypes.byref(s),
                                ctypes.byref(n)), plan, "fwi_timing_read")
    return m.value, s.value, n.value


def fwi_status_string(status: int) -> str:
    return _lib.fwi_status_string(status).decode()


def fwi_last_error(plan) -> str:
    return _lib.fwi_last_error(plan).decode()
