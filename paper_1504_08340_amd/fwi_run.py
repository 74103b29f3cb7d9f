"""FWI time to a target misfit on the layered 32x32x16 m workload.

python -m paper_1504_08340_amd.fwi_run [--nsteps N] [--freqs 4,8,12]
        [--iters K] [--precision fp32|fp64] [--reg tikhonov|tv]
        [--target-frac F] [--start trend|file.npz] [--full-gradient]
        [--gradient-depth]

Model: three layers (vs 120 / 200 / 300 m/s, boundaries at 5 and 11 m
depth) and a 4x4x3 m soft block (vs 90 m/s), vp = 2 vs, rho = 2000; nine
vertical point loads on a 3x3 surface grid; receivers at every surface node
of the interior.  Observed traces come from the target model through the
same solver, one set per frequency stage (Ricker fc of the stage).  Start:
the linear vs trend 120 -> 300 m/s (or lam, mu from an .npz file).  The
inversion runs the stages in turn (source-frequency continuation, 3.3.2)
and stops when the misfit of the last stage falls below target-frac times
its value at the start model.  One JSON line on stdout: wall seconds to the
target (null if not reached), iterations, solves, misfits and the relative
L2 model errors.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def build(args):
    import torch

    import workloads as W
    from . import FWI_FP32, FWI_FP64, Solver
    wl = W.config3(nsteps=args.nsteps)
    prec = FWI_FP32 if args.precision == "fp32" else FWI_FP64
    S = Solver(wl.prob, wl.src_node, wl.src_dir, wl.rec_node, precision=prec, ckpt_every=args.ckpt,
               grad_full=args.full_gradient)
    rho = S.tensor(wl.rho)
    lam_t, mu_t = S.tensor(wl.lam_true), S.tensor(wl.mu_true)
    stages = []
    for fc in args.freqs:
        wav = np.stack([W.sample_wavelet(lambda t, f=fc: W.ricker(t, f), wl.prob.dt, wl.prob.nsteps, 1000.0)]
                       * wl.nsrc)
        wav_t = S.tensor(wav)
        obs = S.forward(rho, lam_t, mu_t, wav_t).clone()
        stages.append((fc, wav_t, obs))
    torch.cuda.synchronize()
    return wl, S, rho, stages


def run(args, wl, S, rho, stages, lam0, mu0, log=sys.stderr):
    import torch

    from . import fwi_material_mass
    from .fwi import FwiOptions, FwiStage, invert
    opts = FwiOptions(reg=args.reg, tv_eps=args.tv_eps, max_iter=args.iters)
    st = [FwiStage(S, rho, wav, obs, opts) for _, wav, obs in stages]
    mass = torch.empty(S.sizes.n_int_nodes, dtype=torch.float64, device=S.device)
    fwi_material_mass(S.plan, None, mass)
    J_last0 = st[-1].forward(lam0, mu0)
    target = args.target_frac * J_last0
    reached = {}
    t0 = time.perf_counter()
    stage_of_iter = []

    def on_iter(it, Jm, lam, mu):
        stage_of_iter.append(Jm)
        print(f"# iter {it}: J_mis {Jm:.6e} at {time.perf_counter() - t0:.1f} s", file=log, flush=True)
        return False

    # run all but the last stage, then the last with the target as tolerance
    lam, mu = lam0, mu0
    hist = None
    from .fwi import FwiHistory
    hist = FwiHistory()
    if len(st) > 1:
        lam, mu, hist = invert(st[:-1], lam, mu, mass, opts, hist, on_iter)
    opts_last = FwiOptions(**{**opts.__dict__, "tol": target})
    st[-1].opts = opts_last
    lam, mu, hist = invert(st[-1:], lam, mu, mass, opts_last, hist, on_iter)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    J_final = st[-1].forward(lam, mu)
    reached = J_final <= target
    lt, mt = wl.lam_true, wl.mu_true
    err = lambda a, b: float(np.linalg.norm(a.cpu().numpy() - b) / np.linalg.norm(b))
    return dict(seconds_to_target=secs if reached else None, seconds=secs, reached=bool(reached),
                iterations=len(hist.alpha), solves=hist.solves, adjoints=hist.adjoints,
                J_last_stage_start=J_last0, J_last_stage_final=J_final, target=target,
                lam_err_start=err(lam0, lt), mu_err_start=err(mu0, mt),
                lam_err=err(lam, lt), mu_err=err(mu, mt)), lam, mu


def gradient_depth(args, wl, S, rho, stages, log=sys.stdout):
    """Root mean square, over each depth plane of the interior, of the first
    stage's misfit gradient of mu at the start model (its L2 representer, the
    gradient divided by the material mass M~, no regularization) next to that of
    the model error mu_true - mu_start."""
    import torch

    import workloads as W
    from . import binding as B
    lam0, mu0 = S.tensor(wl.lam), S.tensor(wl.mu)
    _, wav, obs = stages[0]
    tr = S.forward(rho, lam0, mu0, wav)
    _, res = S.misfit(tr, obs)
    _, gm = S.adjoint_gradient(rho, lam0, mu0, wav, res)
    mass = torch.empty(S.sizes.n_int_nodes, dtype=torch.float64, device=S.device)
    B.fwi_material_mass(S.plan, None, mass)
    rep = (gm / mass).cpu().numpy()
    err = wl.mu_true - wl.mu
    ax, ay, az = W.interior_axes(wl.prob)
    plane = ax.size * ay.size
    rows = []
    for jz in range(az.size):
        sl = slice(jz * plane, (jz + 1) * plane)
        rows.append(dict(z=float(az[jz]), rms_representer=float(np.sqrt(np.mean(rep[sl] ** 2))),
                         rms_mu_error=float(np.sqrt(np.mean(err[sl] ** 2)))))
        print(f"z {az[jz]:6.2f}  rms representer {rows[-1]['rms_representer']:.3e}  "
              f"rms mu error {rows[-1]['rms_mu_error']:.3e}", file=log, flush=True)
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--nsteps", type=int, default=1500)
    ap.add_argument("--freqs", type=lambda s: [float(x) for x in s.split(",")], default=[4.0, 8.0, 12.0])
    ap.add_argument("--iters", type=int, default=10, help="iterations per stage")
    ap.add_argument("--precision", choices=("fp32", "fp64"), default="fp32")
    ap.add_argument("--ckpt", type=int, default=0)
    ap.add_argument("--reg", choices=("tikhonov", "tv"), default="tikhonov")
    ap.add_argument("--tv-eps", type=float, default=1e10)
    ap.add_argument("--target-frac", type=float, default=1e-2)
    ap.add_argument("--start", default="trend")
    ap.add_argument("--gradient-depth", action="store_true",
                    help="print the depth profile of the first stage's gradient at the start model and stop")
    ap.add_argument("--full-gradient", action="store_true",
                    help="chain rule through the material carried into the PML instead of the gradient "
                         "restricted to the interior bricks (Sec. 3.1.3)")
    args = ap.parse_args(argv)
    import torch
    wl, S, rho, stages = build(args)
    if args.gradient_depth:
        gradient_depth(args, wl, S, rho, stages)
        return
    if args.start == "trend":
        lam0, mu0 = S.tensor(wl.lam), S.tensor(wl.mu)
    else:
        z = np.load(args.start)
        lam0, mu0 = S.tensor(z["lam"]), S.tensor(z["mu"])
    res, _, _ = run(args, wl, S, rho, stages, lam0, mu0)
    res.update(metric="FWI time to target misfit", workload="32x32x16 m layered + block, 9 sources, "
               f"{args.nsteps} steps, fc {','.join(str(f) for f in args.freqs)} Hz",
               precision=args.precision, start=args.start, iters_per_stage=args.iters,
               grad_full=bool(args.full_gradient), reg=args.reg,
               device=torch.cuda.get_device_name(0))
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
