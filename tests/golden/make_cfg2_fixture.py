"""Write the 62,500-brick parity fixture with the FP64 oracle only.

Workload: the 40x40x20 m interior of 1 m bricks with a 5-brick PML (62,500
bricks, 3,093,816 state unknowns) and the smooth random lam, mu of the
throughput workload, its first source (vertical 8 Hz Ricker point load at
(-10, -10, 0)), all 6,561 surface receivers, N RK4 steps at the workload's
dt.  Observed data are zero, so the residual is the trace itself and
J = 1/2 sum_n w_n dt |u^n|^2 (misfit (7) with the trapezoid rule).

Stored (tests/golden/cfg2_src0_<N>.npz):
  traces_rec, traces   traces at a fixed receiver subset, all steps (FP64)
  J                    misfit
  gnode, g_lam, g_mu   exact discrete gradient (R = 0, interior bricks,
                       Sec. 3.1.3) at the brick-vertex nodes of the closed
                       interior (every second node per axis)
  g_lam_norm, g_mu_norm  Euclidean norms of the full gradient vectors

Every value comes from ``oracle.matfree`` (element-batched operators) and
``oracle.solve`` (RK4, misfit, reverse sweep); ``workloads`` provides the
inputs.  The forward states go to ``--state-dir`` (about 68 MB per step) and
are read back by the reverse sweep, so nothing is recomputed.

  python tests/golden/make_cfg2_fixture.py --nsteps 400 --state-dir DIR
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle.matfree import MatFree  # noqa: E402
from oracle.solve import Stepper  # noqa: E402

# receivers kept in the fixture: every 97th of the 6,561 plus the 9 around
# the source (the largest traces)
REC_STRIDE = 97


def fixture_receivers(wl):
    rec = list(range(0, wl.nrec, REC_STRIDE))
    nx = wl.prob.ne_int[0] * 2 + 1                       # receivers: interior surface grid, x fastest
    # source 0 sits at (-10, -10, 0): receiver grid index (20, 20) on the 81 x 81 surface grid
    c = 20 + nx * 20
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            rec.append(c + dx + nx * dy)
    return np.array(sorted(set(rec)), np.int64)


class DiskStates:
    """Sequence of forward states X^0..X^N stored as .npy files."""

    def __init__(self, d, n):
        self.d, self.n = d, n

    def path(self, i):
        return os.path.join(self.d, f"X{i:05d}.npy")

    def __len__(self):
        return self.n

    def __getitem__(self, i):
        if i < 0:
            i += self.n
        if not 0 <= i < self.n:
            raise IndexError(i)
        return np.load(self.path(i), mmap_mode="r")

    def __iter__(self):
        for i in range(self.n):
            yield self[i]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--nsteps", type=int, default=400)
    ap.add_argument("--state-dir", required=True)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    N = args.nsteps
    out = args.out or os.path.join(os.path.dirname(os.path.abspath(__file__)), f"cfg2_src0_{N}.npz")
    os.makedirs(args.state_dir, exist_ok=True)

    wl = W.config2(nsteps=N)
    wav, src, sdir = wl.wavelet[:1], wl.src_node[:1], wl.src_dir[:1]
    t0 = time.time()
    op = MatFree(wl.prob, wl.rho, wl.lam, wl.mu)
    st = Stepper(op, src, sdir, wl.rec_node)
    print(f"operators built in {time.time() - t0:.1f} s; n_state {op.n_state}, dt {wl.prob.dt:.6e}",
          flush=True)

    states = DiskStates(args.state_dir, N + 1)
    X = np.zeros((op.n_X, 1))
    np.save(states.path(0), X)
    t0 = time.time()
    for n in range(N):
        X = st.step(X, wav, n)
        np.save(states.path(n + 1), X)
        if (n + 1) % 10 == 0:
            print(f"forward step {n + 1}/{N}, {time.time() - t0:.0f} s", flush=True)

    tr = np.stack([st.traces_of(np.asarray(x)) for x in states], axis=1)      # (1, N+1, nrec, 3)
    obs = np.zeros_like(tr)
    J = st.misfit(tr, obs)
    print(f"J = {J:.17e}", flush=True)

    # the reverse sweep of Stepper.adjoint_gradient, with progress lines
    t0 = time.time()

    class Progress:
        def __init__(self, s):
            self.s = s

        def __len__(self):
            return len(self.s)

        def __iter__(self):
            return iter(self.s)

        def __getitem__(self, i):
            if i % 10 == 0:
                print(f"reverse step {i}, {time.time() - t0:.0f} s", flush=True)
            return self.s[i]

    gl, gm, _ = st.adjoint_gradient(wav, obs, Progress(states))
    print(f"|g_lam| {np.linalg.norm(gl):.6e} |g_mu| {np.linalg.norm(gm):.6e}", flush=True)

    p = wl.prob
    nix, niy, niz = 2 * p.ne_int[0] + 1, 2 * p.ne_int[1] + 1, 2 * p.ne_int[2] + 1
    jz, jy, jx = np.meshgrid(np.arange(0, niz, 2), np.arange(0, niy, 2), np.arange(0, nix, 2), indexing="ij")
    gnode = (jx + nix * (jy + niy * jz)).ravel().astype(np.int64)
    rec = fixture_receivers(wl)
    np.savez_compressed(
        out, nsteps=N, dt=p.dt, source=0, traces_rec=rec, traces=tr[0][:, rec, :], J=J,
        gnode=gnode, g_lam=gl[gnode], g_mu=gm[gnode],
        g_lam_norm=np.linalg.norm(gl), g_mu_norm=np.linalg.norm(gm))
    print(f"wrote {out}", flush=True)


if __name__ == "__main__":
    main()
