/* pmlfwi.h -- C ABI of the MI355X hot path of time-domain elastic FWI in
 * PML-truncated 3D media (Fathi, Kallivokas, Poursartip, arXiv:1504.08340).
 *
 * What the library computes
 *   fwi_forward          state problem: classical RK4 on the first-order form
 *                        (6) of the semi-discrete hybrid system (5), starting
 *                        at rest; displacement traces at surface receivers.
 *   fwi_misfit           misfit (7) at the receivers (no regularization term):
 *                        J = 1/2 sum_n w_n dt |u^n - u_m^n|^2, trapezoid weights
 *                        w_0 = w_N = 1/2, else 1.
 *   fwi_adjoint_gradient adjoint problem (15), solved as the exact reverse of
 *                        the RK4 recurrence, and the misfit part of the
 *                        Lame-parameter gradient (16)-(18), (C.1f)-(C.1g):
 *                        m-bar = M~ g_mis (the vector whose dot product with a
 *                        nodal direction is the directional derivative (27)).
 *   fwi_apply_operator   one application of the forward or transposed spatial
 *                        operator (test hook).
 *
 * Discretization: cubic 27-node bricks (quadratic spectral elements) with the
 * 3x3x3 Legendre-Gauss-Lobatto rule for every integral; displacements on all
 * nodes except the Dirichlet ones (outer sides and bottom, (2c)); six stress
 * components (xx, yy, zz, yz, xz, xy) on every node of the closed PML; nodal
 * Lame parameters on the closed interior box, carried into the PML from the
 * nearest interface point (Sec. 3.1.3).  PML stretching alpha_s = 1 +
 * alpha_o (xi/L)^m, beta_s = beta_o (xi/L)^m.
 *
 * Arrays at the boundary (all FP64 unless stated, C order, device memory
 * unless stated):
 *   full node grid   NX x NY x NZ, node id i + NX*(j + NY*k); NX = 2*(ex+2*ps)+1,
 *                    NY = 2*(ey+2*ps)+1, NZ = 2*(ez+pb)+1; k = 0 at the bottom,
 *                    k = NZ-1 the free surface z = 0.
 *   material grid    NIX x NIY x NIZ = (2ex+1) x (2ey+1) x (2ez+1), the closed
 *                    interior box; id jx + NIX*(jy + NIY*jz) = full node
 *                    (jx + 2ps, jy + 2ps, jz + 2pb).
 *   rho, lam, mu     [n_int_nodes]  (kg/m^3, Pa, Pa)
 *   wavelet          [nsrc][2*nsteps+1]  force magnitude at t = k*dt/2
 *   traces, observed, residual  [nsrc][nsteps+1][nrec][3]
 *   g_lam, g_mu      [n_int_nodes]
 *
 * Ownership: the caller allocates every array and the workspace (size from
 * fwi_query) and keeps them alive while work is enqueued.  A plan owns its
 * host metadata and a few KB of device metadata (brick tiles, source and
 * receiver tables, misfit partial sums) and a second stream with two events,
 * all created by fwi_plan_create and released by fwi_plan_destroy; the solves
 * allocate nothing.  All work is enqueued on the given stream (a hipStream_t,
 * passed as void*; NULL is the default stream).  The host waits for the
 * device only in fwi_plan_create (one upload), fwi_check_model, the model
 * check that fwi_forward, fwi_adjoint_gradient and fwi_adjoint_gradient_appb
 * run before their first launch (one small kernel, a 40-byte copy and a
 * synchronization of the stream), and fwi_timing_read.
 *
 * Errors: every call returns fwi_status; nothing throws across the ABI.  On
 * error no work has been enqueued (argument errors) or the HIP error is
 * reported (FWI_ERR_HIP); fwi_last_error() gives a message for the plan.
 * A plan is not thread-safe.
 */
#ifndef PMLFWI_H
#define PMLFWI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FWI_OK = 0,
  FWI_ERR_ARG = -1,       /* invalid argument (null pointer, bad size, bad index) */
  FWI_ERR_SHAPE = -2,     /* mesh or time axis not representable */
  FWI_ERR_HIP = -3,       /* a HIP runtime call or kernel launch failed */
  FWI_ERR_STATE = -4,     /* call order violated (adjoint before forward) */
  FWI_ERR_UNSTABLE = -5,  /* dt above the RK4 stability bound of the model */
  FWI_ERR_NOMEM = -6      /* host allocation failed */
} fwi_status;

typedef enum {
  FWI_FP64 = 0,           /* state, element arithmetic and accumulation in FP64 */
  FWI_FP32 = 1,           /* state and element arithmetic in FP32; misfit and
                             gradient time integrals accumulated in FP64 */
  FWI_FP32_MFMA = 2,      /* as FWI_FP32, with the interior stiffness and the PML
                             operator of the forward and transposed stages applied
                             as dense reference-matrix contractions on the matrix
                             cores (FP32 MFMA); the gradient terms stay scalar */
  FWI_FP32_BF16X3 = 3     /* as FWI_FP32_MFMA, on BF16 MFMA: the FP32 operand
                             split into three BF16 parts, FP32 accumulation */
} fwi_precision;

typedef struct {
  int32_t ne_int[3];      /* interior bricks (ex, ey, ez) */
  int32_t npml_side;      /* PML bricks on +-x and +-y (ps) */
  int32_t npml_bottom;    /* PML bricks below the interior (pb) */
  double h;               /* brick edge [m] */
  double dt;              /* time step [s] */
  int32_t nsteps;         /* RK4 steps N */
  double pml_alpha0;      /* alpha_o (Sec. 4.1: 5) */
  double pml_beta0;       /* beta_o [1/s] (Sec. 4.1: 400) */
  int32_t pml_m;          /* profile order m (Sec. 4.1: 2) */
  int32_t nsrc;           /* sources, solved together */
  int32_t nrec;           /* receivers (shared by all sources) */
  int32_t precision;      /* fwi_precision */
  int32_t ckpt_every;     /* 0: the forward keeps the interior displacement of
                             every RK4 stage, the adjoint recomputes nothing;
                             k > 0: the forward keeps the full state every k
                             steps and the adjoint recomputes one k-step segment
                             at a time; -1: forward-only plan (traces only,
                             no adjoint; smallest workspace) */
  int32_t grad_full;      /* 0: the gradient of fwi_adjoint_gradient comes from
                             the interior bricks only (Sec. 3.1.3); 1: also from
                             the PML S-rows through the material each PML node
                             takes from the interface node it projects onto
                             (chain rule of that extension), so the result is
                             the exact derivative at the interface nodes too.
                             With 1 the stage store also keeps the PML
                             displacement fields (9 values per PML node and
                             stage); fwi_adjoint_gradient_appb refuses it. */
  int32_t ckpt_slots;     /* with ckpt_every = k > 0: 0 keeps the full state at
                             every segment start (ceil(N/k) states); c > 0 keeps
                             at most c states and recomputes by binomial
                             checkpointing over the segments (revolve
                             schedules: the least number of segment advances
                             for c slots).  Must be 0 when ckpt_every <= 0. */
} fwi_problem;

typedef struct {
  int64_t n_nodes;        /* full grid nodes */
  int64_t n_int_nodes;    /* material (closed interior) nodes */
  int64_t n_pml_nodes;    /* nodes of the closed PML */
  int64_t n_state;        /* paper's state unknowns: 3 per free node + 6 per PML node */
  int64_t n_hist;         /* history unknowns (5b): the PML part of the state */
  int64_t trace_len;      /* nsrc*(nsteps+1)*nrec*3 */
  int64_t workspace_bytes;
  int64_t register_bytes; /* one stored state (all sources) */
  int64_t tile[3];        /* bricks per element tile along x, y, z (build constants) */
  int64_t tiles_interior; /* element tiles over the interior bricks (ragged ones included) */
  int64_t tiles_pml;      /* element tiles over the PML bricks */
  int64_t element_threads;/* threads of an element-kernel workgroup */
  int64_t ckpt_states;    /* full states the workspace holds (checkpoint slots) */
  int64_t schedule_advances; /* segment advances of the checkpoint schedule
                             (forward sweep to its checkpoints + adjoint) */
  int64_t adjoint_forward_steps; /* forward RK4 steps the adjoint recomputes */
} fwi_sizes;

typedef struct fwi_plan fwi_plan;

/* Sizes of a problem; pure host function. */
fwi_status fwi_query(const fwi_problem* prob, fwi_sizes* out);

/* Build a plan.  Host arrays (copied): src_node[nsrc] full-grid node ids of
 * point loads (not Dirichlet nodes), src_dir[nsrc][3] load directions,
 * rec_node[nrec] full-grid node ids of receivers (not Dirichlet nodes). */
fwi_status fwi_plan_create(const fwi_problem* prob, const int32_t* src_node,
                           const double* src_dir, const int32_t* rec_node,
                           fwi_plan** out);
fwi_status fwi_plan_destroy(fwi_plan* plan);

/* Replace the point loads of fwi_plan_create by a general list of nodal
 * loads (Sec. 4: vertical stress loads over a surface region): entry e adds
 * load_vec[e][0..2] * wavelet[load_src[e]][k] [N] at full-grid node
 * load_node[e] (not a Dirichlet node) in the stage of time k*dt/2.  Host
 * arrays, copied; entries with the same (source, node) are summed.  nload = 0
 * returns to the point loads.  A set-up call: it waits for the device and
 * allocates the plan's load tables. */
fwi_status fwi_plan_set_loads(fwi_plan* plan, int32_t nload, const int32_t* load_src,
                              const int32_t* load_node, const double* load_vec);

/* Consistent nodal weights of a uniform traction on the free surface z = 0
 * over the rectangle [xmin, xmax] x [ymin, ymax] (whole brick faces inside
 * it): weight[c] = integral over the region of the basis function of node[c],
 * by the 3x3 LGL rule of each face, i.e. products of the 1D weights
 * (h/6, 2h/3, h/6) summed over the faces containing the node.  A traction t
 * [Pa] in direction d gives the load t * weight[c] * d.  Host function; the
 * first min(count, cap) entries are written; FWI_ERR_SHAPE when count > cap. */
fwi_status fwi_surface_traction(const fwi_problem* prob, double xmin, double xmax,
                                double ymin, double ymax, int32_t cap, int32_t* node,
                                double* weight, int32_t* count);

/* State problem (6): N RK4 steps from rest with the nodal load
 * src_dir[s] * wavelet[s][k] at the stage times; writes traces (u at every
 * receiver, steps 0..N) and keeps in the workspace what fwi_adjoint_gradient
 * needs (stage displacements or checkpoints).
 * Before its first launch it checks the model as fwi_check_model does
 * (synchronizing the stream): FWI_ERR_ARG when rho, mu or 3 lam + 2 mu is not
 * positive somewhere, FWI_ERR_UNSTABLE when the plan's dt is above the RK4
 * stability bound of this model; in both cases nothing else is enqueued and
 * fwi_last_error names the offending values. */
fwi_status fwi_forward(fwi_plan* plan, void* stream, const double* rho,
                       const double* lam, const double* mu,
                       const double* wavelet, void* workspace, double* traces);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the state
 * problem of fwi_forward (same kernels, same traces) with no workspace
 * argument.  Its workspace is a fixed device array of the library, 64 MiB
 * per GPU (allocated when the library is loaded, held until the process
 * ends); its device address is looked up by fwi_plan_create, and the plan
 * must be used on the device that was current then (else FWI_ERR_ARG).
 * It keeps nothing for an adjoint (no stage store, no checkpoints) and leaves
 * the plan's record of the last fwi_forward untouched.  Problems whose
 * forward registers, residual arrays and materials exceed 64 MiB are rejected
 * with FWI_ERR_ARG before any launch.  Every call on one GPU uses the same
 * array: calls that overlap in time on one GPU (several streams, threads or
 * plans) race and give wrong traces; serialize them.  Model check, stream
 * synchronization and errors as fwi_forward; the call allocates nothing
 * (kernel timing is suspended during the call). */
fwi_status fwi_forward_noalloc(fwi_plan* plan, void* stream, const double* rho,
                               const double* lam, const double* mu,
                               const double* wavelet, double* traces);

/* Misfit (7): residual = traces - observed and J (one double on the device).
 * J is summed per workgroup and then in a fixed order: the same inputs give
 * the same bits. */
fwi_status fwi_misfit(fwi_plan* plan, void* stream, const double* traces,
                      const double* observed, double* residual, double* J);

/* Adjoint (15) and gradient (18) with R = 0, for the residual of the last
 * fwi_forward on the same workspace and the same rho, lam, mu, wavelet.
 * Writes g_lam, g_mu (overwritten, summed over sources): the derivative of J
 * with respect to the nodal values on the closed interior, from the interior
 * bricks only (Sec. 3.1.3) when the plan's grad_full is 0.  PML nodes take
 * their material from the closed interior box (the interface values carried
 * outward), so on nodes of the interface the full derivative of J also has
 * PML-brick terms that this restricted gradient leaves out; at every other
 * node it is the exact derivative.  With grad_full = 1 those terms are
 * included (the PML S-row derivatives, summed onto the interface node each
 * PML node projects onto).  Checks the model as fwi_forward does. */
fwi_status fwi_adjoint_gradient(fwi_plan* plan, void* stream, const double* rho,
                                const double* lam, const double* mu,
                                const double* wavelet, const double* residual,
                                void* workspace, double* g_lam, double* g_mu);

/* The paper's own scheme for the adjoint and gradient (App. B, (B.2)-(B.4)
 * with the transposes of (15), optimize-then-discretize): reverse-time RK4 of
 * (15) from y(T) = 0 with the receiver residual as forcing at t_n, t_{n-1/2}
 * (mean of the two step values) and t_{n-1}, and the gradient (C.1f)-(C.1g)
 * integrated by the trapezoid rule over the step states.  Same arguments and
 * call order as fwi_adjoint_gradient; the result differs from the exact
 * discrete gradient by O(dt^2). */
fwi_status fwi_adjoint_gradient_appb(fwi_plan* plan, void* stream, const double* rho,
                                     const double* lam, const double* mu,
                                     const double* wavelet, const double* residual,
                                     void* workspace, double* g_lam, double* g_mu);

/* Test hook: one application of the spatial operator to nodal fields.
 * x0, x1, x2, out: [nsrc][9][n_nodes] (3 displacement then 6 stress
 * components per node; entries off the unknowns are ignored / written 0).
 * which = 0: out = -M^{-1} (G x0 + K x1 + C x2)            (forward, (5a))
 * which = 1: out = -M^{-1} (G^T x0 + K^T x1 + C^T x2)      (transposed, (14a))
 * where G^T acts on PML history fields. */
fwi_status fwi_apply_operator(fwi_plan* plan, void* stream, int which,
                              const double* rho, const double* lam,
                              const double* mu, const double* x0,
                              const double* x1, const double* x2,
                              void* workspace, double* out);

/* Regularization of one nodal material field f (n_int_nodes FP64, closed
 * interior, x fastest): kind FWI_REG_TIKHONOV, R(f) = 1/2 int |grad f|^2 (8),
 * or FWI_REG_TV, R(f) = int (|grad f|^2 + eps)^(1/2) (9) with the pointwise
 * denominator of (17) (the functional carries R, not R/2, so that (17) is its
 * derivative).  LGL quadrature of every interior brick.  value (one double on
 * the device) and grad (n_int_nodes: dR/df_j, the discrete vectors of
 * (C.1b)-(C.1e)) are overwritten; either may be null.  Deterministic. */
enum { FWI_REG_TIKHONOV = 0, FWI_REG_TV = 1 };
fwi_status fwi_regularization(fwi_plan* plan, void* stream, int kind, double eps,
                              const double* field, double* value, double* grad);

/* M~ of (C.1a): the diagonal LGL mass of the closed interior (n_int_nodes). */
fwi_status fwi_material_mass(fwi_plan* plan, void* stream, double* mdiag);

/* Control problem (18): g = M~^{-1} (g_mis + R g_reg), n_int_nodes each;
 * g_reg may be null when R = 0.  g may alias g_mis. */
fwi_status fwi_gradient_finalize(fwi_plan* plan, void* stream, const double* g_mis,
                                 const double* g_reg, double R, double* g);

/* Model check (synchronizes the stream; rho, lam, mu on the device, info a
 * host array of 6 doubles): info = [min rho, min mu, min (3 lam + 2 mu),
 * max vp, omega_max bound, largest stable dt].  The bound on the largest
 * frequency of the interior operator is element by element: for every
 * interior brick, (max(lam, 0) c_lam + max mu c_mu) (2/h)^2 / min rho with
 * c_lam, c_mu the largest eigenvalues of the unit LGL reference brick; the
 * PML stretching only lowers stiffness per mass.  RK4 is stable for
 * dt omega_max <= 2 sqrt(2).  Returns FWI_ERR_ARG when rho, mu or the bulk
 * term 3 lam + 2 mu is not positive, FWI_ERR_UNSTABLE when the plan's dt
 * exceeds info[5]. */
fwi_status fwi_check_model(fwi_plan* plan, void* stream, const double* rho,
                           const double* lam, const double* mu, double* info);

/* out[0] = sum_i a_i b_i w_i (w null: weights 1), device vectors of length n;
 * one workgroup, fixed summation order (deterministic).  Used for the norms
 * of (24) and the inner products of the line search (Algorithm 1). */
fwi_status fwi_dot(void* stream, int64_t n, const double* a, const double* b,
                   const double* w, double* out);

/* out = alpha x + beta y, device vectors of length n (y may be null when
 * beta = 0; out may alias x or y): the vector updates of the optimizer --
 * the L-BFGS two-loop recursion, the model update (19), the biased lambda
 * direction (25) and the gradient difference y = g_{k+1} - g_k. */
fwi_status fwi_axpby(void* stream, int64_t n, double alpha, const double* x, double beta,
                     const double* y, double* out);
/* out[0] = max_i |x_i| (device; the step-length rule of the first L-BFGS
 * iteration, max |s| = a fraction of max |m|). */
fwi_status fwi_absmax(void* stream, int64_t n, const double* x, double* out);

/* ---- Learned warm start: a small 3D convolutional network (FP32, device
 * arrays, NCDHW: batch, channel, then three spatial axes, the last fastest).
 * Cubic kernels of size K = 1 or 3 with zero padding K/2 and per-axis
 * strides; output extent (n + 2 (K/2) - K) / s + 1 per axis.  All
 * reductions run in a fixed order (deterministic). */
typedef struct {
  int32_t N, Ci, D, H, W;  /* input batch, channels, extents */
  int32_t Co, K;           /* output channels, kernel size */
  int32_t sd, sh, sw;      /* strides */
} fwi_conv_shape;

/* y = act(b + w * x); w [Co][Ci][K][K][K], b [Co] (may be null); relu != 0
 * applies max(0, .). */
fwi_status fwi_conv3d_forward(void* stream, const fwi_conv_shape* shape, const float* x,
                              const float* w, const float* b, int relu, float* y);
/* Gradients from dy = dL/dy: dx (may be null), dw, db (may be null); with
 * relu, y is the activated forward output (the mask is y > 0). */
fwi_status fwi_conv3d_backward(void* stream, const fwi_conv_shape* shape, const float* x,
                               const float* w, const float* y, const float* dy, int relu,
                               float* dx, float* dw, float* db);
/* BF16 inference (the network's forward pass on the matrix cores):
 * fwi_to_bf16 rounds FP32 to BF16 (nearest, ties to even; bit patterns in
 * uint16).  fwi_conv3d_forward_bf16: y = act(b + w * x) with x [N][Ci][D][H][W]
 * and w [Co][Ci][K][K][K] in BF16, as an implicit GEMM on BF16 MFMA with FP32
 * accumulation; bias (FP32) and ReLU in FP32; y is BF16 (out_fp32 = 0, hidden
 * layers) or FP32 (out_fp32 = 1, the head).  Same shapes as
 * fwi_conv3d_forward; N <= 65535. */
fwi_status fwi_to_bf16(void* stream, int64_t n, const float* in, uint16_t* out);
fwi_status fwi_conv3d_forward_bf16(void* stream, const fwi_conv_shape* shape, const uint16_t* x,
                                   const uint16_t* w, const float* b, int relu, int out_fp32, void* y);
/* loss[0] = 1/(2n) sum (y - t)^2, grad = (y - t)/n; either may be null. */
fwi_status fwi_mse(void* stream, int64_t n, const float* y, const float* t, float* loss,
                   float* grad);
/* One Adam step (bias-corrected, step >= 1) on param with moments m, v. */
fwi_status fwi_adam(void* stream, int64_t n, float* param, const float* grad, float* m,
                    float* v, float lr, float beta1, float beta2, float eps, int step);
/* Network input from traces [nsrc][nsteps+1][nrec][3] (FP64): component comp
 * at receivers rec_idx[hw] and steps t0 + t*tstride (t < T; zero past nsteps),
 * times scale -> out [nsrc][T][hw] (FP32). */
fwi_status fwi_trace_features(void* stream, const double* traces, int nsrc, int nsteps,
                              int nrec, const int32_t* rec_idx, int hw, int T, int t0,
                              int tstride, int comp, float scale, float* out);
/* Coarse relative perturbation c [gz][gy][gx] on cell centres of a regular
 * grid over the closed interior box (z index 0 at the surface) -> nodal
 * field out = base * (1 + trilinear(c)), n_int_nodes, clamped at the edges. */
fwi_status fwi_grid_to_nodes(fwi_plan* plan, void* stream, const float* coarse, int gx,
                             int gy, int gz, const double* base, double* out);

/* Kernel timing (measurement support).  While enabled, every stride-th launch
 * of each kernel class is bracketed by HIP events recorded on the stream the
 * kernel is launched on; fwi_timing_read waits for those events and returns
 * the mean duration of the sampled launches.  stride = 0 disables and clears.
 * Classes: FWI_K_INTERIOR (interior bricks, forward), FWI_K_PML (PML bricks,
 * forward), FWI_K_NODAL (RK4 stage combination), FWI_K_INTERIOR_ADJ (interior
 * bricks with gradient terms), FWI_K_PML_ADJ (PML bricks, transposed). */
enum { FWI_K_INTERIOR = 0, FWI_K_PML = 1, FWI_K_NODAL = 2, FWI_K_INTERIOR_ADJ = 3,
       FWI_K_PML_ADJ = 4, FWI_K_NCLASS = 5 };
fwi_status fwi_timing_enable(fwi_plan* plan, int stride);
fwi_status fwi_timing_read(fwi_plan* plan, int kernel_class, double* mean_ms,
                           int64_t* samples, int64_t* launches);

const char* fwi_status_string(fwi_status s);
/* Message of the plan's last failed call; with plan = NULL, of the last
 * failed fwi_plan_create on the calling thread. */
const char* fwi_last_error(const fwi_plan* plan);

#ifdef __cplusplus
}
#endif
#endif /* PMLFWI_H */
