"""The paper's layered-medium inversion (Sec. 4.3) on the GPU, shortened.

Problem: 40 x 40 x 45 m interior, 6.25 m PML, 1.25 m bricks (3,578,136 state
unknowns, the count Sec. 4.2 prints), dt = 1e-3 s, T = 0.45 s; target
lam = mu from (30) (80 / 101.25 / 125 MPa layers), rho = 2000; start: 80 MPa
everywhere; one vertical 1 kPa traction with the p20 pulse of Table 1 over
|x|, |y| <= 17.5 m, receivers at every grid point there.  Observed data from
the target on the refined mesh (0.625 m bricks, dt/2, read at the coarse
receivers every second step), so the inversion does not see its own
discretization.  Simultaneous lam and mu inversion with TV regularization
(eps = 0.01 MPa^2), the rule (24) for R and the biased lam direction (25),
L-BFGS with Armijo backtracking (Algorithms 1-2): the paper's setting, run
for --iters iterations instead of the paper's 310 (p20 stage).

    python -m paper_1504_08340_amd.layered_inversion [--iters K] [--json OUT]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

import workloads as W

from . import binding as B
from .fwi import FwiHistory, FwiOptions, FwiStage, invert
from .solver import Solver


def refined_data(pulse, nsteps, device):
    fine, coarse = W.section43(pulse, nsteps, refined=True), W.section43(pulse, nsteps)
    rec_f = W.surface_receivers(fine.prob, -17.5, 17.5, -17.5, 17.5, step=2)
    fx, fy, fz = W.node_axes(fine.prob)
    cx, cy, cz = W.node_axes(coarse.prob)
    pf = np.stack([fx[rec_f % fx.size], fy[(rec_f // fx.size) % fy.size], fz[rec_f // (fx.size * fy.size)]], 1)
    rc = coarse.rec_node
    pc = np.stack([cx[rc % cx.size], cy[(rc // cx.size) % cy.size], cz[rc // (cx.size * cy.size)]], 1)
    assert np.allclose(pf, pc), "fine receivers must sit on the coarse receiver nodes"
    S = Solver(fine.prob, fine.src_node, fine.src_dir, rec_f, precision=B.FWI_FP64, ckpt_every=-1,
               device=device, traction=fine.traction)
    tr = S.forward(*(S.tensor(a) for a in (fine.rho, fine.lam_true, fine.mu_true, fine.wavelet)))
    obs = tr[:, ::2].contiguous()
    torch.cuda.synchronize()
    S.close()
    return obs


def depth_profile(prob, field, x=0.0, y=0.0):
    """(z, values) of a closed-interior nodal field on the vertical line (x, y)."""
    ax, ay, az = W.interior_axes(prob)
    jx, jy = int(np.argmin(np.abs(ax - x))), int(np.argmin(np.abs(ay - y)))
    ids = [W.interior_node_id(prob, jx, jy, jz) for jz in range(az.size)]
    return az, field[np.asarray(ids)]


def run(iters=40, pulse="p20", nsteps=450, precision="fp32", device="cuda", log=print, grad_full=False):
    t0 = time.perf_counter()
    wl = W.section43(pulse, nsteps)
    obs = refined_data(pulse, nsteps, device)
    log(f"refined-mesh data: {time.perf_counter() - t0:.1f} s")
    prec = B.FWI_FP32 if precision == "fp32" else B.FWI_FP64
    S = Solver(wl.prob, wl.src_node, wl.src_dir, wl.rec_node, precision=prec, device=device,
               traction=wl.traction, grad_full=grad_full)
    rho, wav = S.tensor(wl.rho), S.tensor(wl.wavelet)
    lam0, mu0 = S.tensor(wl.lam), S.tensor(wl.mu)
    opts = FwiOptions(reg="tv", tv_eps=0.01e12, max_iter=iters)
    stage = FwiStage(S, rho, wav, obs, opts)
    mass = torch.empty(S.sizes.n_int_nodes, dtype=torch.float64, device=S.device)
    B.fwi_material_mass(S.plan, None, mass)
    t1 = time.perf_counter()

    def on_iter(it, Jm, lam, mu):
        if it % 5 == 0 or it == 1:
            log(f"iter {it}: J_mis {Jm:.6e} at {time.perf_counter() - t1:.1f} s")
        return False

    lam, mu, hist = invert([stage], lam0, mu0, mass, opts, FwiHistory(), on_iter)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t1
    lt, mt = wl.lam_true, wl.mu_true
    la, ma = lam.cpu().numpy(), mu.cpu().numpy()
    err = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    z, pl = depth_profile(wl.prob, la)
    _, pm = depth_profile(wl.prob, ma)
    _, pt = depth_profile(wl.prob, lt)
    out = dict(workload="Sec. 4.3 layered medium, 40x40x45 m, 1.25 m bricks, 6.25 m PML, p20, "
                        f"T = {nsteps * wl.prob.dt:.3f} s, refined-mesh data",
               n_state=int(S.sizes.n_state), precision=precision, iterations=len(hist.alpha),
               seconds=secs, solves=hist.solves, adjoints=hist.adjoints,
               J_start=hist.J[0], J_final=hist.J[-1], J_reduction=hist.J[0] / hist.J[-1],
               grad_full=bool(grad_full), J_history=hist.J, alpha=hist.alpha, backtracks=hist.backtracks,
               R=hist.R, lam_err_start=err(wl.lam, lt), mu_err_start=err(wl.mu, mt),
               lam_err=err(la, lt), mu_err=err(ma, mt),
               profile_00={"z": z.tolist(), "lam_MPa": (pl / 1e6).tolist(), "mu_MPa": (pm / 1e6).tolist(),
                           "target_MPa": (pt / 1e6).tolist()})
    S.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--iters", type=int, default=40)
    ap.add_argument("--precision", choices=("fp32", "fp64"), default="fp32")
    ap.add_argument("--full-gradient", action="store_true",
                    help="chain rule through the material carried into the PML instead of the gradient "
                         "restricted to the interior bricks (Sec. 3.1.3)")
    ap.add_argument("--json", default=None)
    args = ap.parse_args(argv)
    if not torch.cuda.is_available():
        sys.exit("the inversion runs on the GPU")
    out = run(args.iters, precision=args.precision, log=lambda m: print(m, flush=True),
              grad_full=args.full_gradient)
    print(json.dumps({k: v for k, v in out.items()
                      if k not in ("J_history", "profile_00", "alpha", "backtracks", "R")}), flush=True)
    if args.json:
        with open(args.json, "w") as f:
            json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
