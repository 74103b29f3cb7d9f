"""Throughput of the hot path on one MI355X: RK4 DOF-steps/s, forward + adjoint.

Workload (default): 40x40x20 m interior of 1 m 27-node bricks with a 5-brick
PML (50x50x25 = 62,500 bricks, 3,093,816 state unknowns), smooth random
lambda, mu (+-25 % about a 100 -> 250 m/s shear-velocity trend), 4 vertical
Ricker point loads (8 Hz) solved together, 2000 RK4 steps at CFL 0.5,
receivers at all 6,561 surface nodes of the interior.

One bench step = one pass of the whole hot path on that batch: forward solve
(6) with traces, misfit (7), adjoint solve (15) and Lame-parameter gradient
(18).  value = n_state * nsteps * nsrc / (seconds per bench step).

Usage: python bench.py [--steps K] [--warmup W]
                       [--precision fp32|fp64|fp32-mfma|fp32-bf16x3]
                       [--ckpt k] [--nsteps N] [--no-cpu-baseline]
                       [--copy-probe-mib MiB]

--copy-probe-mib runs one plain element-wise copy of that size after the timed
region; hardware-counter runs use it to scale FETCH_SIZE / WRITE_SIZE.  The
roofline ``traffic`` field is read from the counter summary committed under
profiles/ and reported only while the kernel sources hash to the value
recorded there.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published
MFMA_PEAK_TFLOPS = {"fp32-mfma": 157.3, "fp32-bf16x3": 2500.0}   # dense, published
PRECISIONS = {"fp64": 0, "fp32": 1, "fp32-mfma": 2, "fp32-bf16x3": 3}
# Matrix-core work of one interior workgroup (one brick tile of NE bricks, one
# source): G = B U with B 81x27 padded to 96 rows and U 27 x 3NE; R = B^T S with
# 27 rows padded to 32, K = 81; NT = ceil(3NE / 16) column tiles.  FP32 16x16x4
# MFMA: 6 NT tiles x 7 steps + 2 NT tiles x 21 steps; split BF16 16x16x16:
# 6 NT x 2 + 2 NT x 6 steps, 3 products each.


def mfma_flops_per_tile(precision, ne):
    nt = -(-3 * ne // 16)
    if precision == "fp32-mfma":
        return (6 * nt * 7 + 2 * nt * 21) * 2 * 16 * 16 * 4
    return (6 * nt * 2 + 2 * nt * 6) * 3 * 2 * 16 * 16 * 16


def useful_flops_per_tile(ne):
    return 2 * (2 * 81 * 27 * 3 * ne)


CSRC = os.path.join(ROOT, "paper_1504_08340_amd", "csrc")
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "hbm_traffic__kernels__cfg40x40x20_4src_fp32.md")


def kernel_source_hash():
    """sha256 over the HIP sources, in name order."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def recorded_traffic(cls, precision):
    """Scaled HBM bytes per launch of a kernel class from the counter summary.

    The summary holds lines ``traffic <class> <precision> <bytes>`` and one
    ``source_sha256 <hex>`` line; None when the file is absent, the class is not
    listed, or the sources changed since the counters were taken.
    """
    try:
        with open(TRAFFIC_SUMMARY) as f:
            lines = [ln.split() for ln in f if ln.strip()]
    except OSError:
        return None
    sha = [ln[1] for ln in lines if len(ln) == 2 and ln[0] == "source_sha256"]
    if not sha or sha[0] != kernel_source_hash():
        return None
    for ln in lines:
        if len(ln) == 4 and ln[0] == "traffic" and ln[1] == cls and ln[2] == precision:
            return float(ln[3])
    return None


def history_nodes(prob):
    """PML nodes that carry history (at least two axes with beta > 0)."""
    import workloads as W
    x, y, z = W.node_axes(prob)
    ex, ey, ez = prob.ne_int
    bx = np.abs(x) > 0.5 * ex * prob.h + 1e-9
    by = np.abs(y) > 0.5 * ey * prob.h + 1e-9
    bz = -z > ez * prob.h + 1e-9
    cnt = (bz[:, None, None].astype(int) + by[None, :, None] + bx[None, None, :])
    return int((cnt >= 2).sum())


def restricted_history(prob):
    """History unknowns on the PML nodes that use them (at least two axes with
    beta > 0): 6 stress components per such node, 3 displacement components
    where the node is not a Dirichlet node."""
    import workloads as W
    x, y, z = W.node_axes(prob)
    ex, ey, ez = prob.ne_int
    bx = np.abs(x) > 0.5 * ex * prob.h + 1e-9
    by = np.abs(y) > 0.5 * ey * prob.h + 1e-9
    bz = -z > ez * prob.h + 1e-9
    hist = (bz[:, None, None].astype(int) + by[None, :, None] + bx[None, None, :]) >= 2
    dirichlet = np.zeros_like(hist)
    dirichlet[0] = True
    dirichlet[:, 0] = dirichlet[:, -1] = True
    dirichlet[:, :, 0] = dirichlet[:, :, -1] = True
    nh = int(hist.sum())
    return 6 * nh + 3 * (nh - int((hist & dirichlet).sum()))


def pass_bytes_per_dof_step(sizes, prob, nsrc, es, n_hist):
    """Compulsory HBM bytes of one forward + adjoint + gradient pass that keeps
    the stage displacements (no recompute), per DOF-step.

    Per RK4 step and source, three-register classical RK4 streams the state 16
    times: stage 1 reads its input (which is Xn) and writes the accumulator and
    the next stage input (3), stages 2 and 3 read the stage input, Xn and the
    accumulator and write the accumulator and the next input (5 each), stage 4
    reads the stage input and the accumulator and writes Xn (3): 4 n_X per
    stage on average, n_X = n_hist + 2 n_state; the forward writes and the adjoint
    reads the stage displacement on the closed interior (3 N_int).  Per stage,
    once for all sources: materials and masses (2 N_int + 2 N_nodes), and in
    the adjoint the FP64 gradient accumulators (read and write, 2 N_int).
    """
    nx = n_hist + 2 * sizes.n_state
    nint, nn = sizes.n_int_nodes, sizes.n_nodes
    per_src = 2 * 4 * es * (4 * nx + 3 * nint)
    shared = 2 * 4 * es * (2 * nint + 2 * nn) + 4 * 2 * 2 * nint * 8
    return (nsrc * per_src + shared) / (sizes.n_state * nsrc)


def algorithmic_bytes(cls, sizes, prob, nsrc, es):
    """Compulsory HBM bytes of one launch of a kernel class (all sources).

    nodal: per free node, stage input (6) + residual (3) + register traffic of
    the stage mode; per PML node, stage input stresses (12, +9 on history
    nodes) + residual (6) + register traffic; averaged over the 4 RK4 modes.
    element kernels: stage input read once, residual rows written once,
    materials once per launch.
    """
    nn = sizes.n_nodes
    nfree = sizes.n_state - 6 * sizes.n_pml_nodes
    nfree //= 3
    npml = sizes.n_pml_nodes
    nh = history_nodes(prob)
    nint = sizes.n_int_nodes
    if cls == "nodal":
        # register traffic besides the stage input, per RK4 mode, averaged over
        # the 4 stages (0, 1, 1, 2): mode 0 writes acc and Yout (its input is
        # Xn itself); mode 1 reads Xn and acc, writes acc and Yout; mode 2 reads
        # acc, writes Xn.  Register comps touched: 6 per free node, 12 per PML
        # node, 9 more on history nodes.
        reg = 3.0 * (6.0 * nfree + 12.0 * npml + 9.0 * nh)
        stage_in = 6.0 * nfree + 12.0 * npml + 9.0 * nh      # Y read by the rate evaluation
        resid = 3.0 * nfree + 6.0 * npml                      # partial array 0
        store = 3.0 * nint                                    # stage displacement kept for the adjoint
        return es * nsrc * (reg + stage_in + resid + store) + es * nn
    if cls in ("interior", "interior_adj"):
        b = es * nsrc * (3 * nint + 3 * nint) + es * 2 * nint
        if cls == "interior_adj":
            b += es * nsrc * 3 * nint + 8 * 2 * 2 * nint
        return b
    if cls in ("pml", "pml_adj"):
        pml_free = npml - (nn - nfree)
        return es * nsrc * (6 * pml_free + 12 * npml + 9 * nh + 3 * pml_free + 6 * npml)
    raise ValueError(cls)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=tuple(PRECISIONS), default="fp32")
    ap.add_argument("--ckpt", type=int, default=0)
    ap.add_argument("--nsteps", type=int, default=2000)
    ap.add_argument("--timing-stride", type=int, default=7)   # odd: samples every RK4 stage mode
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe-mib", type=int, default=0)
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the multi-GPU path (source-parallel gradient "
              "all-reduce or slab decomposition) is a design, not a build; run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1504_08340_amd as P
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    prec = PRECISIONS[args.precision]
    es = 8 if prec == 0 else 4
    wl = W.config2(nsteps=args.nsteps)
    prob = wl.prob
    t0 = time.time()
    S = P.Solver(prob, wl.src_node, wl.src_dir, wl.rec_node, precision=prec, ckpt_every=args.ckpt)
    rho, lam, mu, wav = (S.tensor(a) for a in (wl.rho, wl.lam, wl.mu, wl.wavelet))
    # observed data: traces of the unperturbed trend model (setup, untimed)
    lam_t, mu_t = S.tensor(wl.lam_true), S.tensor(wl.mu_true)
    obs = S.forward(rho, lam_t, mu_t, wav).clone()
    traces = S.empty_traces()
    resid = torch.empty_like(traces)
    J = torch.empty(1, dtype=torch.float64, device=S.device)
    gl = torch.empty(S.sizes.n_int_nodes, dtype=torch.float64, device=S.device)
    gm = torch.empty_like(gl)
    torch.cuda.synchronize()
    print(f"# setup {time.time() - t0:.1f} s, workspace {S.sizes.workspace_bytes / 2**30:.1f} GiB",
          file=sys.stderr, flush=True)

    def one_step():
        S.forward(rho, lam, mu, wav, traces)
        S.misfit(traces, obs, resid, J)
        S.adjoint_gradient(rho, lam, mu, wav, resid, gl, gm)

    for i in range(args.warmup):
        one_step()
        torch.cuda.synchronize()
        print(f"# warmup step {i} done", file=sys.stderr, flush=True)
    P.fwi_timing_enable(S.plan, args.timing_stride)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        one_step()
        print(f"# timed step {i} enqueued", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms = 1000.0 * elapsed / args.steps
    n_state = S.sizes.n_state
    value = n_state * prob.nsteps * wl.nsrc / (ms / 1000.0)

    kstats = {}
    for c, name in enumerate(P.KERNEL_CLASSES):
        mean_ms, samples, launches = P.fwi_timing_read(S.plan, c)
        if launches:
            kstats[name] = dict(mean_ms=mean_ms, samples=samples, launches=launches,
                                total_ms=mean_ms * launches / args.steps)
    P.fwi_timing_enable(S.plan, 0)
    if args.copy_probe_mib:
        n = args.copy_probe_mib * 2**20 // 4
        src = torch.ones(n, dtype=torch.float32, device=S.device)
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)          # reads and writes copy_probe_mib MiB once
        torch.cuda.synchronize()
        del src, dst
        print(f"# copy probe: {args.copy_probe_mib} MiB read + written", file=sys.stderr, flush=True)
    # whole pass against the HBM roofline: the compulsory bytes per DOF-step of
    # a keep-the-stages pass (paper-faithful history count and the history
    # restricted to the PML edges and corners that use it) times the DOF-step
    # rate; and the sum of the per-kernel algorithmic bytes over every launch
    bpd = {"paper": pass_bytes_per_dof_step(S.sizes, prob, wl.nsrc, es, S.sizes.n_hist),
           "restricted": pass_bytes_per_dof_step(S.sizes, prob, wl.nsrc, es, restricted_history(prob))}
    kernel_bytes = sum(algorithmic_bytes(k, S.sizes, prob, wl.nsrc, es) * v["launches"] / args.steps
                       for k, v in kstats.items())
    pass_line = {
        "bytes_per_dof_step": bpd,
        "achieved_GBs": {k: b * value / 1e9 for k, b in bpd.items()},
        "frac": {k: b * value / 1e9 / HBM_PEAK_GBS for k, b in bpd.items()},
        "ceiling_dof_steps_per_s": {k: HBM_PEAK_GBS * 1e9 / b for k, b in bpd.items()},
        "kernel_model_bytes": kernel_bytes,
        "kernel_model_frac": kernel_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
    }
    dom = max(kstats, key=lambda k: kstats[k]["total_ms"])
    alg = algorithmic_bytes(dom, S.sizes, prob, wl.nsrc, es)
    achieved = alg / (kstats[dom]["mean_ms"] * 1e-3) / 1e9
    print("# kernel classes (per bench step): " + ", ".join(
        f"{k}: {v['total_ms']:.1f} ms over {v['launches'] // args.steps} launches, mean {v['mean_ms']*1e3:.1f} us, "
        f"{algorithmic_bytes(k, S.sizes, prob, wl.nsrc, es) / (v['mean_ms'] * 1e-3) / 1e9:.0f} GB/s"
        for k, v in kstats.items()), file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle sample) ...", file=sys.stderr, flush=True)
        cpu = cpu_baseline(wl, n_state)

    mfma = None
    if args.precision in MFMA_PEAK_TFLOPS and "interior" in kstats:
        tiles = S.sizes.tiles_interior
        ne = S.sizes.tile[0] * S.sizes.tile[1] * S.sizes.tile[2]
        t = kstats["interior"]["mean_ms"] * 1e-3
        executed = tiles * wl.nsrc * mfma_flops_per_tile(args.precision, ne) / t / 1e12
        mfma = {"kernel": "interior", "executed_tflops": executed, "peak": MFMA_PEAK_TFLOPS[args.precision],
                "unit": "TFLOP/s", "frac": executed / MFMA_PEAK_TFLOPS[args.precision],
                "useful_tflops": tiles * wl.nsrc * useful_flops_per_tile(ne) / t / 1e12,
                "mean_launch_us": kstats["interior"]["mean_ms"] * 1e3}
    line = {
        "metric": "RK4 DOF-steps/s fwd+adj",
        "value": value,
        "unit": "DOF-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == 0 else "f32",
        "data": "synthetic",
        "config": {
            "workload": "40x40x20 m interior, 1 m Q2 bricks, 5-brick PML (62,500 bricks), "
                        f"random lam/mu, 4 Ricker 8 Hz sources, {prob.nsteps} RK4 steps; "
                        "forward + misfit + adjoint + gradient",
            "n_state": n_state, "nsrc": wl.nsrc, "nsteps": prob.nsteps,
            "ckpt_every": args.ckpt, "precision": args.precision,
        },
        "roofline": {
            "bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": recorded_traffic(dom, args.precision),
            "mean_launch_us": kstats[dom]["mean_ms"] * 1e3,
            "algorithmic_bytes_per_launch": alg,
            "pass_frac": pass_line["frac"]["restricted"],
            "pass_frac_paper": pass_line["frac"]["paper"],
            "pass": pass_line,
        },
        "cpu_baseline": cpu,
    }
    if mfma is not None:
        line["mfma"] = mfma
    print(json.dumps(line), flush=True)


def cpu_baseline(wl, n_state):
    """The FP64 oracle on a bounded sample of the same workload (host cores)."""
    try:
        from oracle import matfree  # noqa: F401
    except ImportError:
        return None
    return matfree.bench_sample(wl, n_state, fwd_steps=2, adj_steps=2)


if __name__ == "__main__":
    main()
