"""MI355X-native hot path of time-domain elastic FWI in PML-truncated 3D media.

Fathi, Kallivokas, Poursartip (arXiv:1504.08340): RK4 time stepping of the
hybrid displacement / displacement-stress PML system (6), misfit (7), adjoint
(15) and Lame-parameter gradient (18), as hand-written HIP kernels behind the
C ABI declared in ``include/pmlfwi.h``.

``binding`` is the thin ctypes layer (same names as the C entry points);
``solver`` holds device buffers in torch tensors and calls the binding;
``autograd`` exposes the misfit as a differentiable function of (lam, mu).
"""
from .binding import (FWI_FP32, FWI_FP32_BF16X3, FWI_FP32_MFMA, FWI_FP64,  # noqa: F401
                      FWI_REG_TIKHONOV, FWI_REG_TV,
                      FwiError, fwi_adjoint_gradient, fwi_adjoint_gradient_appb, fwi_apply_operator,
                      fwi_check_model, fwi_dot,
                      fwi_forward, fwi_gradient_finalize, fwi_last_error, fwi_material_mass,
                      fwi_misfit, fwi_plan_create, fwi_plan_destroy, fwi_query,
                      fwi_regularization, fwi_status_string, fwi_timing_enable,
                      fwi_timing_read, KERNEL_CLASSES, make_problem)
from .solver import Solver  # noqa: F401
from .autograd import MisfitFunction, misfit  # noqa: F401
