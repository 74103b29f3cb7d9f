"""Plain FP64 CPU oracle for the PML-truncated elastic FWI hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this
package.  The product path (the C-ABI library and its Python binding) never
calls it and shares no code with it; both sides read their inputs from the
``workloads`` module, which holds no arithmetic of the method.

Source: Fathi, Kallivokas, Poursartip, "Full-waveform inversion in
three-dimensional PML-truncated elastic media" (arXiv:1504.08340).

What it computes, and the passage each part follows:

* ``lgl``      -- 1D Legendre-Gauss-Lobatto nodes, weights and derivative
                  matrix of the quadratic spectral element (Sec. 2, the
                  lumped-mass remark after (5); Sec. 4.1 "27-noded bricks").
* ``mesh``     -- structured hexahedral mesh, node classes, lumped masses,
                  degree-of-freedom numbering (Fig. 3; (2c); (5); Sec. 4.2).
* ``pml``      -- stretch tensors Lambda_e, Lambda_p, Lambda_w and the scalars
                  a, b, c, d from the complex coordinate stretching (1b)-(1c).
* ``assemble`` -- the system matrices M, C, K, G of (5a), read term by term
                  from the weak forms (3a)-(3b).
* ``solve``    -- classical RK4 on the first-order form (6), the misfit (7),
                  the exact discrete adjoint of the RK4 recurrence and the
                  Lame-parameter gradient (16)/(C.1f)-(C.1g), and the paper's
                  reverse-time RK4 of Appendix B.
* ``matfree``  -- element-by-element application of the same operators for
                  meshes too large to assemble (cross-checked against
                  ``assemble`` on small meshes).
* ``regularize`` -- Tikhonov (8) and total-variation (9) terms with their
                  gradients (C.1b)-(C.1e), M~ (C.1a) and the control
                  problem (18).
* ``fwi``      -- the reduced-space inversion of Sec. 3.2: L-BFGS search
                  directions, Armijo backtracking (Algorithm 1), the loop of
                  Algorithm 2 with the regularization factor rule (24) and the
                  biased lambda direction (25).

Readings of the paper where it is silent or garbled are stated at the
functions that use them.
"""
