"""Learned warm start for the inversion: surface traces -> coarse (lam, mu).

A small 3D convolutional network (four stride-reducing stages of 32
channels and a 1x1x1 head) maps the vertical displacement traces of the nine
surface loads of the layered 32x32x16 m workload (32 x 32 receivers at 1 m
spacing, 256 time samples) to relative perturbations of lam and mu about
the linear vs trend on a 16 x 16 x 8 grid of 2 m cells; the start model is
the trend times (1 + interpolated perturbation).  Training runs in FP32,
inference in BF16 on the matrix cores (FP32 accumulation).  Training data are seeded
random layered profiles whose traces the forward solver of this library
computes; training, inference and every layer's forward and backward pass
run in the library's HIP kernels (fwi_conv3d_*, fwi_mse, fwi_adam), with
torch holding the buffers.  The linear trend stays the fallback: the start
with the lower misfit of the first stage is used.

python -m paper_1504_08340_amd.warmstart train --profiles 256 --out weights.npz
python -m paper_1504_08340_amd.warmstart compare --weights weights.npz --profiles 4
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import binding as B

# (in channels, out channels, kernel, strides, relu): input [9][256][32][32]
LAYERS = [
    (9, 32, 3, (4, 2, 2), True),    # -> [32][64][16][16]
    (32, 32, 3, (2, 1, 1), True),   # -> [32][32][16][16]
    (32, 32, 3, (2, 1, 1), True),   # -> [32][16][16][16]
    (32, 32, 3, (2, 1, 1), True),   # -> [32][8][16][16]
    (32, 2, 1, (1, 1, 1), False),   # -> [2][8][16][16]: (dlam, dmu) per cell, depth first
]
IN_SHAPE = (9, 256, 32, 32)
GRID = (8, 16, 16)                 # depth, y, x cells
NSTEPS = 1024                      # forward steps of the training and inference solves
T0, TSTRIDE = 4, 4                 # time samples: steps 4, 8, ..., 1024
FC = 8.0                           # Ricker central frequency of the probing loads


def _out(n, K, s):
    return (n + 2 * (K // 2) - K) // s + 1


class Net:
    """Parameters, Adam moments and the layer passes (device, FP32)."""

    def __init__(self, device, seed=0):
        self.dev = device
        rng = np.random.default_rng(seed)
        self.w, self.b = [], []
        for ci, co, k, _, _ in LAYERS:
            std = np.sqrt(2.0 / (ci * k ** 3))
            self.w.append(torch.tensor(rng.standard_normal((co, ci, k, k, k)) * std, dtype=torch.float32,
                                       device=device))
            self.b.append(torch.zeros(co, dtype=torch.float32, device=device))
        self.m = [torch.zeros_like(t) for t in self.w + self.b]
        self.v = [torch.zeros_like(t) for t in self.w + self.b]
        self.step = 0
        self.scale = 1.0                   # input normalisation of the traces

    def shapes(self, n):
        shp = []
        c, d, h, w = IN_SHAPE
        for ci, co, k, s, _ in LAYERS:
            shp.append(B.conv_shape(n, ci, d, h, w, co, k, s))
            d, h, w = _out(d, k, s[0]), _out(h, k, s[1]), _out(w, k, s[2])
        return shp

    def forward(self, x):
        """Activations of every layer (the last is the output)."""
        acts = [x]
        n = x.shape[0]
        for (ci, co, k, s, relu), sh, w, b in zip(LAYERS, self.shapes(n), self.w, self.b):
            d, h, ww = _out(sh.D, k, s[0]), _out(sh.H, k, s[1]), _out(sh.W, k, s[2])
            y = torch.empty((n, co, d, h, ww), dtype=torch.float32, device=self.dev)
            B.fwi_conv3d_forward(None, sh, acts[-1], w, b, relu, y)
            acts.append(y)
        return acts

    def forward_bf16(self, x):
        """Network output for input x (FP32) by BF16 inference on the matrix
        cores: input, weights and hidden activations rounded to BF16, FP32
        accumulation, bias and ReLU; the head's output in FP32."""
        if getattr(self, "_wbf", None) is None or self._wbf_step != self.step:
            self._wbf = []
            for w in self.w:
                t = torch.empty(w.shape, dtype=torch.bfloat16, device=self.dev)
                B.fwi_to_bf16(None, w.numel(), w, t)
                self._wbf.append(t)
            self._wbf_step = self.step
        n = x.shape[0]
        a = torch.empty(x.shape, dtype=torch.bfloat16, device=self.dev)
        B.fwi_to_bf16(None, x.numel(), x.contiguous(), a)
        last = len(LAYERS) - 1
        for li, ((ci, co, k, s, relu), sh, w, b) in enumerate(zip(LAYERS, self.shapes(n), self._wbf, self.b)):
            d, h, ww = _out(sh.D, k, s[0]), _out(sh.H, k, s[1]), _out(sh.W, k, s[2])
            y = torch.empty((n, co, d, h, ww), dtype=torch.float32 if li == last else torch.bfloat16,
                            device=self.dev)
            B.fwi_conv3d_forward_bf16(None, sh, a, w, b, relu, li == last, y)
            a = y
        return a

    def backward(self, acts, dy):
        """Parameter gradients (w then b, layer order) for dL/d(output) = dy."""
        n = acts[0].shape[0]
        gw = [None] * len(LAYERS)
        gb = [None] * len(LAYERS)
        for li in range(len(LAYERS) - 1, -1, -1):
            sh = self.shapes(n)[li]
            relu = LAYERS[li][4]
            gw[li] = torch.empty_like(self.w[li])
            gb[li] = torch.empty_like(self.b[li])
            dx = torch.empty_like(acts[li]) if li > 0 else None
            B.fwi_conv3d_backward(None, sh, acts[li], self.w[li], acts[li + 1], dy, relu, dx, gw[li], gb[li])
            dy = dx
        return gw + gb

    def adam(self, grads, lr, b1=0.9, b2=0.999, eps=1e-8):
        self.step += 1
        for p, g, m, v in zip(self.w + self.b, grads, self.m, self.v):
            B.fwi_adam(None, p.numel(), p, g, m, v, lr, b1, b2, eps, self.step)

    def save(self, path):
        np.savez(path, scale=self.scale, step=self.step,
                 **{f"w{i}": t.cpu().numpy() for i, t in enumerate(self.w)},
                 **{f"b{i}": t.cpu().numpy() for i, t in enumerate(self.b)})

    @classmethod
    def load(cls, path, device):
        z = np.load(path)
        net = cls(device)
        net.w = [torch.tensor(z[f"w{i}"], device=device) for i in range(len(LAYERS))]
        net.b = [torch.tensor(z[f"b{i}"], device=device) for i in range(len(LAYERS))]
        net.scale = float(z["scale"])
        net.step = int(z["step"])
        return net


class Probe:
    """The solver, loads and receiver selection shared by training and use."""

    def __init__(self, device="cuda", precision=B.FWI_FP32):
        import workloads as W
        from .solver import Solver
        self.W = W
        wl = W.config3(nsteps=NSTEPS)
        self.wl = wl
        self.S = Solver(wl.prob, wl.src_node, wl.src_dir, wl.rec_node, precision=precision, device=device)
        self.rho = self.S.tensor(wl.rho)
        wav = np.stack([W.sample_wavelet(lambda t: W.ricker(t, FC), wl.prob.dt, NSTEPS, 1000.0)] * wl.nsrc)
        self.wav = self.S.tensor(wav)
        nix = wl.prob.nn_int[0]
        jj = 1 + 2 * np.arange(32)                    # every second surface node from x, y = -15.5 m
        rec = (jj[:, None] * nix + jj[None, :]).ravel()   # receiver order: y slow, x fast
        self.rec_idx = torch.tensor(rec.astype(np.int32), device=self.S.device)
        self.lam0, self.mu0 = self.S.tensor(wl.lam), self.S.tensor(wl.mu)   # linear trend

    def traces(self, lam, mu):
        return self.S.forward(self.rho, lam, mu, self.wav)

    def features(self, traces, scale, out):
        wl = self.wl
        B.fwi_trace_features(None, traces, wl.nsrc, NSTEPS, wl.nrec, self.rec_idx, 32 * 32, IN_SHAPE[1], T0,
                             TSTRIDE, 2, scale, out)

    def target(self, lam_t, mu_t):
        """Relative perturbations about the trend at the cell centres [2][8][16][16]."""
        p = self.wl.prob
        nix, niy, niz = p.nn_int
        ix = 2 + 4 * np.arange(16)                 # x, y = -15, -13, ..., 15 m
        iz = (niz - 1) - (2 + 4 * np.arange(8))    # depths 1, 3, ..., 15 m
        idx = (iz[:, None, None] * niy + ix[None, :, None]) * nix + ix[None, None, :]
        out = np.stack([lam_t[idx] / self.wl.lam[idx] - 1.0, mu_t[idx] / self.wl.mu[idx] - 1.0])
        return out.astype(np.float32)

    def start_model(self, net, traces, precision="bf16"):
        """(lam, mu) from the network for one set of traces; inference in BF16
        on the matrix cores (precision "bf16") or in FP32 ("fp32")."""
        x = torch.empty((1,) + IN_SHAPE, dtype=torch.float32, device=self.S.device)
        self.features(traces, net.scale, x[0])
        c = (net.forward_bf16(x) if precision == "bf16" else net.forward(x)[-1])[0]
        lam = torch.empty_like(self.lam0)
        mu = torch.empty_like(self.mu0)
        B.fwi_grid_to_nodes(self.S.plan, None, c[0].contiguous(), 16, 16, 8, self.lam0, lam)
        B.fwi_grid_to_nodes(self.S.plan, None, c[1].contiguous(), 16, 16, 8, self.mu0, mu)
        return lam, mu


def make_dataset(probe, seeds, log=sys.stderr):
    W = probe.W
    n = len(seeds)
    X = torch.empty((n,) + IN_SHAPE, dtype=torch.float32, device=probe.S.device)
    Y = torch.empty((n, 2) + GRID, dtype=torch.float32, device=probe.S.device)
    t0 = time.perf_counter()
    for i, sd in enumerate(seeds):
        vs = W.layered_profile_vs(probe.wl.prob, int(sd))
        w2 = W.with_model(probe.wl, vs)
        tr = probe.traces(probe.S.tensor(w2.lam_true), probe.S.tensor(w2.mu_true))
        probe.features(tr, 1.0, X[i])
        Y[i] = torch.from_numpy(probe.target(w2.lam_true, w2.mu_true))
        if (i + 1) % 32 == 0:
            torch.cuda.synchronize()
            print(f"# profiles {i + 1}/{n} in {time.perf_counter() - t0:.1f} s", file=log, flush=True)
    return X, Y


def train(probe, X, Y, epochs, batch, lr, seed=0, log=sys.stderr):
    net = Net(probe.S.device, seed)
    scale = 1.0 / float(X.abs().max())
    X.mul_(scale)
    net.scale = scale
    n = X.shape[0]
    rng = np.random.default_rng(seed)
    loss = torch.empty(1, dtype=torch.float32, device=X.device)
    hist = []
    for ep in range(epochs):
        order = rng.permutation(n)
        tot = 0.0
        for i in range(0, n - batch + 1, batch):
            idx = torch.tensor(order[i:i + batch], device=X.device)
            xb, yb = X[idx].contiguous(), Y[idx].contiguous()
            acts = net.forward(xb)
            dy = torch.empty_like(acts[-1])
            B.fwi_mse(None, dy.numel(), acts[-1], yb, loss, dy)
            net.adam(net.backward(acts, dy), lr)
            tot += float(loss[0])
        hist.append(tot / (n // batch))
        print(f"# epoch {ep}: loss {hist[-1]:.4e}", file=log, flush=True)
    return net, hist


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--profiles", type=int, default=256)
    t.add_argument("--holdout", type=int, default=8)
    t.add_argument("--epochs", type=int, default=30)
    t.add_argument("--batch", type=int, default=8)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--out", required=True)
    c = sub.add_parser("compare")
    c.add_argument("--weights", required=True)
    c.add_argument("--profiles", type=int, default=10)
    c.add_argument("--first", type=int, default=0, help="index of the first held-out profile (seed 20000 + i)")
    c.add_argument("--iters", type=int, default=8)
    c.add_argument("--nsteps", type=int, default=800)
    c.add_argument("--target-frac", type=float, default=0.2)
    args = ap.parse_args(argv)
    probe = Probe()
    if args.cmd == "train":
        seeds = 10_000 + np.arange(args.profiles)
        t0 = time.perf_counter()
        X, Y = make_dataset(probe, seeds)
        t_data = time.perf_counter() - t0
        t0 = time.perf_counter()
        net, hist = train(probe, X, Y, args.epochs, args.batch, args.lr)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        net.save(args.out)
        # held-out profiles: model error and misfit, trend vs network start
        res = []
        for i in range(args.holdout):
            w2 = probe.W.with_model(probe.wl, probe.W.layered_profile_vs(probe.wl.prob, 20_000 + i))
            obs = probe.traces(probe.S.tensor(w2.lam_true), probe.S.tensor(w2.mu_true)).clone()
            lam_n, mu_n = probe.start_model(net, obs)
            J = {}
            for name, (l0, m0) in (("trend", (probe.lam0, probe.mu0)), ("net", (lam_n, mu_n))):
                tr = probe.traces(l0, m0)
                J[name] = float(probe.S.misfit(tr, obs)[0][0])
                J[name + "_mu_err"] = float(np.linalg.norm(m0.cpu().numpy() - w2.mu_true) / np.linalg.norm(w2.mu_true))
            res.append(J)
        print(json.dumps(dict(profiles=args.profiles, epochs=args.epochs, data_seconds=t_data,
                              train_seconds=t_train, loss=hist, holdout=res)), flush=True)
    else:
        net = Net.load(args.weights, probe.S.device)
        out = []
        for i in range(args.first, args.first + args.profiles):
            out.append(compare_one(probe, net, 20_000 + i, args))
            print(json.dumps(out[-1]), file=sys.stderr, flush=True)
        print(json.dumps(dict(metric="FWI time to target misfit, plain vs warm start", runs=out)), flush=True)


def compare_one(probe, net, seed, args):
    """FWI from the trend and from the network start on one held-out profile."""
    import workloads as W
    from .fwi import FwiOptions, FwiStage, invert
    from .solver import Solver
    wl = W.with_model(W.config3(nsteps=args.nsteps), W.layered_profile_vs(probe.wl.prob, seed))
    # the measured data the network reads (probing traces of the true model;
    # data, not part of either inversion's cost)
    obs_probe = probe.traces(probe.S.tensor(wl.lam_true), probe.S.tensor(wl.mu_true)).clone()
    torch.cuda.synchronize()
    S = Solver(wl.prob, wl.src_node, wl.src_dir, wl.rec_node, precision=B.FWI_FP32)
    rho = S.tensor(wl.rho)
    stages = []
    for fc in (4.0, 8.0):
        wav = S.tensor(np.stack([W.sample_wavelet(lambda t, f=fc: W.ricker(t, f), wl.prob.dt, args.nsteps, 1000.0)]
                                * wl.nsrc))
        obs = S.forward(rho, S.tensor(wl.lam_true), S.tensor(wl.mu_true), wav).clone()
        stages.append((wav, obs))
    opts = FwiOptions(reg="tikhonov", max_iter=args.iters)
    mass = torch.empty(S.sizes.n_int_nodes, dtype=torch.float64, device=S.device)
    B.fwi_material_mass(S.plan, None, mass)
    result = {"seed": int(seed)}
    # the same target for both starts: a fraction of the trend start's last-stage misfit
    st_last = FwiStage(S, rho, stages[-1][0], stages[-1][1], opts)
    J_trend_last = st_last.forward(probe.lam0, probe.mu0)
    target = args.target_frac * J_trend_last
    J_first = {}
    for name in ("trend", "warm"):
        t0 = time.perf_counter()
        if name == "trend":
            l0, m0 = probe.lam0, probe.mu0
        else:
            # the warm start's clock includes the network inference and the
            # choice between its model and the trend (two first-stage solves)
            lam_n, mu_n = probe.start_model(net, obs_probe)
            lam_n, mu_n = lam_n.clone(), mu_n.clone()
            for cand, (lc, mc) in (("trend", (probe.lam0, probe.mu0)), ("net", (lam_n, mu_n))):
                J_first[cand] = FwiStage(S, rho, stages[0][0], stages[0][1], opts).forward(lc, mc)
            use_net = J_first["net"] < J_first["trend"]          # fallback: the trend
            l0, m0 = (lam_n, mu_n) if use_net else (probe.lam0, probe.mu0)
        sts = [FwiStage(S, rho, w, o, opts) for w, o in stages[:-1]]
        lam, mu, h = invert(sts, l0, m0, mass, opts)
        o2 = FwiOptions(**{**opts.__dict__, "tol": target})
        lam, mu, h = invert([FwiStage(S, rho, stages[-1][0], stages[-1][1], o2)], lam, mu, mass, o2, h)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        Jf = st_last.forward(lam, mu)
        result[name] = dict(seconds=secs, reached=Jf <= target, J_final=Jf, iterations=len(h.alpha),
                            mu_err=float(np.linalg.norm(mu.cpu().numpy() - wl.mu_true) / np.linalg.norm(wl.mu_true)))
    result.update(target=target, J_first_stage=J_first, used_net=bool(use_net))
    S.close()
    return result


if __name__ == "__main__":
    main()
