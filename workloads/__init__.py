"""Seeded synthetic inputs shared by the oracle and the device path.

This module only *describes* problems and produces input arrays: grid sizes,
material fields sampled at node coordinates, source wavelets, source and
receiver node indices.  None of the method's arithmetic (element operators,
PML stretching, time stepping, misfit, adjoint, gradient) lives here, so the
oracle and the HIP path can both use it without sharing any of the method.

Array conventions (the same ones the C ABI documents):

* Full node grid: ``NX x NY x NZ`` nodes at spacing ``h/2`` (27-node bricks of
  edge ``h``).  Node id ``ix + NX*(iy + NY*iz)``; ``iz = 0`` is the bottom of
  the PML, ``iz = NZ-1`` the free surface ``z = 0``.
* Interior-closure grid (the nodes of the closed interior box, where the
  material parameters live): ``NIX x NIY x NIZ``, id ``jx + NIX*(jy + NIY*jz)``,
  with full-grid indices ``(jx + 2*ps, jy + 2*ps, jz + 2*pb)``.
* Wavelet: ``(nsrc, 2*nsteps+1)`` force magnitude [N] at ``t = k*dt/2``.
* Traces / observed data: ``(nsrc, nsteps+1, nrec, 3)``.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Problem", "Workload", "node_axes", "interior_axes", "full_node_id",
    "interior_node_id", "surface_receivers", "ricker", "gaussian_pulse",
    "lame_from_velocities", "config1", "config2", "config3", "tiny",
    "cfl_dt", "TABLE1", "section41", "section43", "tiny_traction",
]


@dataclasses.dataclass(frozen=True)
class Problem:
    """Geometry, time axis and PML parameters of one simulation."""

    ne_int: tuple            # interior elements (ex, ey, ez)
    npml_side: int           # PML elements on +-x and +-y
    npml_bottom: int         # PML elements below the interior
    h: float                 # element edge [m]
    dt: float                # time step [s]
    nsteps: int
    pml_alpha0: float = 5.0  # alpha_o  (Sec. 4.1 values)
    pml_beta0: float = 400.0  # beta_o [1/s]
    pml_m: int = 2           # polynomial order of the attenuation profile

    @property
    def ne(self):
        ex, ey, ez = self.ne_int
        return (ex + 2 * self.npml_side, ey + 2 * self.npml_side,
                ez + self.npml_bottom)

    @property
    def nn(self):
        return tuple(2 * e + 1 for e in self.ne)

    @property
    def nn_int(self):
        return tuple(2 * e + 1 for e in self.ne_int)

    @property
    def n_nodes(self):
        a, b, c = self.nn
        return a * b * c

    @property
    def n_int_nodes(self):
        a, b, c = self.nn_int
        return a * b * c

    def replace(self, **kw):
        return dataclasses.replace(self, **kw)


@dataclasses.dataclass
class Workload:
    """A problem plus every input array one forward/adjoint run needs."""

    name: str
    prob: Problem
    rho: np.ndarray          # (n_int_nodes,) [kg/m^3]
    lam: np.ndarray          # (n_int_nodes,) [Pa]
    mu: np.ndarray           # (n_int_nodes,) [Pa]
    wavelet: np.ndarray      # (nsrc, 2*nsteps+1) [N]
    src_node: np.ndarray     # (nsrc,) int32 full-grid node ids
    src_dir: np.ndarray      # (nsrc, 3) unit force direction
    rec_node: np.ndarray     # (nrec,) int32 full-grid node ids
    lam_true: np.ndarray | None = None   # target model (observed data)
    mu_true: np.ndarray | None = None
    # uniform surface traction replacing the point loads, or None:
    # (xmin, xmax, ymin, ymax) of the loaded rectangle on z = 0 and the unit
    # direction; the wavelet then holds the traction [Pa] over time.  The
    # nodal loads (integrals of the basis functions) are formed by each side.
    traction: tuple | None = None

    @property
    def nsrc(self):
        return int(self.src_node.shape[0])

    @property
    def nrec(self):
        return int(self.rec_node.shape[0])


# ----------------------------------------------------------------------------
# grid description


def node_axes(prob: Problem):
    """Coordinates of the node planes: x (NX,), y (NY,), z (NZ,)."""
    ex, ey, ez = prob.ne_int
    ps, pb, h = prob.npml_side, prob.npml_bottom, prob.h
    nx, ny, nz = prob.nn
    x = -(0.5 * ex + ps) * h + 0.5 * h * np.arange(nx)
    y = -(0.5 * ey + ps) * h + 0.5 * h * np.arange(ny)
    z = -(ez + pb) * h + 0.5 * h * np.arange(nz)
    return x, y, z


def interior_axes(prob: Problem):
    ex, ey, ez = prob.ne_int
    h = prob.h
    nx, ny, nz = prob.nn_int
    x = -0.5 * ex * h + 0.5 * h * np.arange(nx)
    y = -0.5 * ey * h + 0.5 * h * np.arange(ny)
    z = -ez * h + 0.5 * h * np.arange(nz)
    return x, y, z


def full_node_id(prob: Problem, ix, iy, iz):
    nx, ny, _ = prob.nn
    return np.asarray(ix) + nx * (np.asarray(iy) + ny * np.asarray(iz))


def interior_node_id(prob: Problem, jx, jy, jz):
    nx, ny, _ = prob.nn_int
    return np.asarray(jx) + nx * (np.asarray(jy) + ny * np.asarray(jz))


def _nearest_full_node(prob: Problem, xyz):
    x, y, z = node_axes(prob)
    ix = int(np.argmin(np.abs(x - xyz[0])))
    iy = int(np.argmin(np.abs(y - xyz[1])))
    iz = int(np.argmin(np.abs(z - xyz[2])))
    return int(full_node_id(prob, ix, iy, iz))


def surface_receivers(prob: Problem, xmin=None, xmax=None, ymin=None,
                      ymax=None, step=1):
    """Full-grid ids of free-surface nodes of the closed interior box.

    Optional bounds restrict the region; ``step`` keeps every step-th node.
    """
    ps, pb = prob.npml_side, prob.npml_bottom
    nix, niy, niz = prob.nn_int
    x, y, _ = interior_axes(prob)
    jx = np.arange(nix)[::step]
    jy = np.arange(niy)[::step]
    if xmin is not None:
        jx = jx[(x[jx] >= xmin - 1e-9) & (x[jx] <= xmax + 1e-9)]
    if ymin is not None:
        jy = jy[(y[jy] >= ymin - 1e-9) & (y[jy] <= ymax + 1e-9)]
    iz = prob.nn[2] - 1
    gy, gx = np.meshgrid(jy, jx, indexing="ij")
    ids = full_node_id(prob, gx.ravel() + 2 * ps, gy.ravel() + 2 * ps, iz)
    return ids.astype(np.int32)


# ----------------------------------------------------------------------------
# source time functions


def ricker(t, fc, t0=None):
    """Ricker wavelet (1 - 2 pi^2 fc^2 tau^2) exp(-pi^2 fc^2 tau^2)."""
    if t0 is None:
        t0 = 1.2 / fc
    a = (math.pi * fc * (np.asarray(t) - t0)) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def gaussian_pulse(t, mean, var):
    """Gaussian pulse exp(-(t - mean)^2 / var) (Table 1, Sec. 4).

    ``var`` is the tabulated sigma-bar read as a variance in s^2.
    """
    return np.exp(-((np.asarray(t) - mean) ** 2) / var)


def sample_wavelet(fn, dt, nsteps, amplitude):
    """Sample at the RK4 stage times t = k*dt/2, k = 0..2*nsteps."""
    t = 0.5 * dt * np.arange(2 * nsteps + 1)
    return amplitude * fn(t)


# ----------------------------------------------------------------------------
# material models


def lame_from_velocities(rho, vs, vp):
    mu = rho * vs ** 2
    lam = rho * (vp ** 2 - 2.0 * vs ** 2)
    return lam, mu


def _interior_grid(prob):
    x, y, z = interior_axes(prob)
    gz, gy, gx = np.meshgrid(z, y, x, indexing="ij")
    return gx.ravel(), gy.ravel(), gz.ravel()


def linear_trend_vs(prob, vs_top, vs_bottom):
    _, _, gz = _interior_grid(prob)
    depth = prob.ne_int[2] * prob.h
    return vs_top + (vs_bottom - vs_top) * (-gz) / depth


def cfl_dt(prob, vp_max, cfl=0.5):
    """dt = cfl * (node spacing) / vp_max, node spacing = h/2."""
    return cfl * 0.5 * prob.h / vp_max


def _model_from_vs(rho, vs):
    vp = 2.0 * vs
    return lame_from_velocities(rho, vs, vp)


def tiny(ne_int=(2, 2, 2), npml_side=1, npml_bottom=1, h=1.0, nsteps=40,
         nsrc=1, seed=0, alpha0=5.0, beta0=400.0, fc=25.0, rho0=2000.0,
         hetero=0.2):
    """Small seeded problem for brute-force checks (heterogeneous model)."""
    rng = np.random.default_rng(seed)
    prob0 = Problem(tuple(ne_int), npml_side, npml_bottom, h, 1.0, nsteps,
                    alpha0, beta0, 2)
    n = prob0.n_int_nodes
    vs = 100.0 * (1.0 + hetero * rng.uniform(-1, 1, n))
    rho = np.full(n, rho0)
    lam, mu = _model_from_vs(rho, vs)
    dt = cfl_dt(prob0, float(np.max(2.0 * vs)))
    prob = prob0.replace(dt=dt)
    rec = surface_receivers(prob)
    src_choices = rng.choice(rec, size=nsrc, replace=False)
    dirs = rng.normal(size=(nsrc, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    wav = np.stack([sample_wavelet(lambda t: ricker(t, fc), dt, nsteps,
                                   1000.0 * (1 + 0.1 * s)) for s in range(nsrc)])
    return Workload("tiny", prob, rho, lam, mu, wav,
                    src_choices.astype(np.int32), dirs, rec)


def config1(nsteps=400):
    """8x8x4 m interior, 1 m Q2 bricks, 2-element PML; 10 Hz Ricker.

    Model: vs linear 80 -> 140 m/s with depth, vp = 2 vs, rho = 2000.
    Target: vs * (1 + 0.3 exp(-|x - xc|^2 / (2 sigma^2))), xc = (0,0,-2),
    sigma = 1.5 m.  dt at CFL 0.5 of the trend model.
    """
    prob0 = Problem((8, 8, 4), 2, 2, 1.0, 1.0, nsteps)
    rho0 = 2000.0
    vs = linear_trend_vs(prob0, 80.0, 140.0)
    gx, gy, gz = _interior_grid(prob0)
    bump = np.exp(-(gx ** 2 + gy ** 2 + (gz + 2.0) ** 2) / (2 * 1.5 ** 2))
    vs_true = vs * (1.0 + 0.3 * bump)
    rho = np.full(prob0.n_int_nodes, rho0)
    lam, mu = _model_from_vs(rho, vs)
    lam_t, mu_t = _model_from_vs(rho, vs_true)
    prob = prob0.replace(dt=cfl_dt(prob0, 2.0 * 140.0))
    src = np.array([_nearest_full_node(prob, (0.0, 0.0, 0.0))], np.int32)
    dirs = np.array([[0.0, 0.0, -1.0]])
    wav = sample_wavelet(lambda t: ricker(t, 10.0), prob.dt, nsteps, 1000.0)[None]
    rec = surface_receivers(prob)
    return Workload("cfg1", prob, rho, lam, mu, wav, src, dirs, rec,
                    lam_t, mu_t)


def random_field(prob, seed, corr_len=6.0, amp=0.25):
    """Gaussian-filtered N(0,1) noise on the interior-closure grid.

    Filter sigma = corr_len/2 in metres; scaled so max |delta| = amp.
    """
    from scipy.ndimage import gaussian_filter
    nix, niy, niz = prob.nn_int
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((niz, niy, nix))
    sig = 0.5 * corr_len / (0.5 * prob.h)
    f = gaussian_filter(f, sigma=sig, mode="nearest")
    f *= amp / np.max(np.abs(f))
    return f.ravel()


def config2(nsteps=2000, seed=7, ne_int=(40, 40, 20), npml=5):
    """40x40x20 m interior, 1 m bricks, 5-element PML; 4 Ricker 8 Hz sources.

    Model: vs trend 100 -> 250 m/s with depth, lam and mu perturbed by
    independent smooth random fields (corr. length 6 m, +-25 %).
    Observed-data model: the unperturbed trend.
    """
    prob0 = Problem(tuple(ne_int), npml, npml, 1.0, 1.0, nsteps)
    rho0 = 2000.0
    vs = linear_trend_vs(prob0, 100.0, 250.0)
    rho = np.full(prob0.n_int_nodes, rho0)
    lam_t, mu_t = _model_from_vs(rho, vs)
    lam = lam_t * (1.0 + random_field(prob0, seed))
    mu = mu_t * (1.0 + random_field(prob0, seed + 1))
    vp_max = float(np.max(np.sqrt((lam + 2 * mu) / rho)))
    prob = prob0.replace(dt=cfl_dt(prob0, vp_max))
    half = 0.25 * min(ne_int[0], ne_int[1]) * prob.h
    pos = [(-half, -half, 0.0), (half, -half, 0.0), (-half, half, 0.0),
           (half, half, 0.0)]
    src = np.array([_nearest_full_node(prob, p) for p in pos], np.int32)
    dirs = np.tile([0.0, 0.0, -1.0], (4, 1))
    wav = np.stack([sample_wavelet(lambda t: ricker(t, 8.0), prob.dt, nsteps,
                                   1000.0)] * 4)
    rec = surface_receivers(prob)
    return Workload("cfg2", prob, rho, lam, mu, wav, src, dirs, rec,
                    lam_t, mu_t)


def config3(nsteps=1500, fc=4.0):
    """32x32x16 m interior, 5-element PML, three layers + soft block, 9 sources."""
    prob0 = Problem((32, 32, 16), 5, 5, 1.0, 1.0, nsteps)
    rho0 = 2000.0
    gx, gy, gz = _interior_grid(prob0)
    d = -gz
    vs_t = np.where(d <= 5.0, 120.0, np.where(d <= 11.0, 200.0, 300.0))
    block = (gx >= 2) & (gx <= 6) & (gy >= -2) & (gy <= 2) & (d >= 2) & (d <= 5)
    vs_t = np.where(block, 90.0, vs_t)
    vs0 = linear_trend_vs(prob0, 120.0, 300.0)
    rho = np.full(prob0.n_int_nodes, rho0)
    lam, mu = _model_from_vs(rho, vs0)
    lam_t, mu_t = _model_from_vs(rho, vs_t)
    prob = prob0.replace(dt=cfl_dt(prob0, 600.0))
    pos = [(sx, sy, 0.0) for sy in (-8.0, 0.0, 8.0) for sx in (-8.0, 0.0, 8.0)]
    src = np.array([_nearest_full_node(prob, p) for p in pos], np.int32)
    dirs = np.tile([0.0, 0.0, -1.0], (9, 1))
    wav = np.stack([sample_wavelet(lambda t: ricker(t, fc), prob.dt, nsteps,
                                   1000.0)] * 9)
    rec = surface_receivers(prob)
    return Workload("cfg3", prob, rho, lam, mu, wav, src, dirs, rec,
                    lam_t, mu_t)


def layered_profile_vs(prob, seed):
    """Seeded random profile on the closed interior, shaped like the paper's
    layered hosts: three layers (interfaces at 3-7 m and 9-13 m depth, vs
    100-150 / 170-230 / 250-300 m/s), with probability 0.6 a box inclusion
    (3-5 m edges, 2-8 m deep, vs x0.7-1.3) and a smooth +-5 % random field;
    vs clipped to [80, 300] m/s."""
    rng = np.random.default_rng(seed)
    gx, gy, gz = _interior_grid(prob)
    d = -gz
    d1, d2 = rng.uniform(3.0, 7.0), rng.uniform(9.0, 13.0)
    v1, v2, v3 = rng.uniform(100, 150), rng.uniform(170, 230), rng.uniform(250, 300)
    vs = np.where(d <= d1, v1, np.where(d <= d2, v2, v3))
    if rng.uniform() < 0.6:
        cx, cy, cd = rng.uniform(-10, 10), rng.uniform(-10, 10), rng.uniform(2.0, 8.0)
        sx, sy, sz = rng.uniform(3.0, 5.0, 3)
        inside = (np.abs(gx - cx) <= sx / 2) & (np.abs(gy - cy) <= sy / 2) & (np.abs(d - cd) <= sz / 2)
        vs = np.where(inside, vs * rng.uniform(0.7, 1.3), vs)
    vs = vs * (1.0 + 0.2 * random_field(prob, seed + 1000, corr_len=6.0, amp=0.25))
    return np.clip(vs, 80.0, 300.0)


def with_model(wl, vs, rho=2000.0):
    """The workload wl with its target model replaced by the profile vs."""
    lam_t, mu_t = _model_from_vs(np.full(vs.shape, rho), vs)
    return Workload(wl.name, wl.prob, wl.rho, wl.lam, wl.mu, wl.wavelet, wl.src_node, wl.src_dir,
                    wl.rec_node, lam_t, mu_t)


# ----------------------------------------------------------------------------
# the paper's Sec. 4 problems (distributed surface tractions, Gaussian pulses)

# Table 1: name -> (f_max [Hz], mean [s], sigma-bar [s^2, a variance], t_end [s])
TABLE1 = {"p20": (20.0, 0.11, 0.0014, 0.20), "p30": (30.0, 0.08, 0.0007, 0.15),
          "p40": (40.0, 0.06, 0.0004, 0.12)}


def _traction_workload(name, prob, lam, mu, pulse, half_region, amplitude=1000.0):
    """One source: a vertical traction (downward, `amplitude` Pa times the
    Gaussian pulse of Table 1) on the surface over |x|, |y| <= half_region,
    receivers at every surface node of that region."""
    _, mean, var, _ = TABLE1[pulse]
    wav = sample_wavelet(lambda t: gaussian_pulse(t, mean, var), prob.dt, prob.nsteps, amplitude)[None]
    rho = np.full(prob.n_int_nodes, 2000.0)
    centre = np.array([_nearest_full_node(prob, (0.0, 0.0, 0.0))], np.int32)
    down = np.array([[0.0, 0.0, -1.0]])
    rec = surface_receivers(prob, -half_region, half_region, -half_region, half_region)
    return Workload(name, prob, rho, lam, mu, wav, centre, down, rec,
                    traction=(-half_region, half_region, -half_region, half_region, (0.0, 0.0, -1.0)))


def material_28(z):
    """(28): lam = mu = 80 + 0.45 |z| + 35 exp(-(|z| - 22.5)^2 / 150) MPa."""
    d = np.abs(z)
    return 1e6 * (80.0 + 0.45 * d + 35.0 * np.exp(-(d - 22.5) ** 2 / 150.0))


def section41(pulse="p20", refined=False):
    """Sec. 4.1 gradient check: 24 x 24 x 45 m interior, 5 m PML, 1 m bricks,
    dt = 9e-4 s, T = 0.5 s; lam = mu from (28), rho = 2000; vertical 1 kPa
    traction with a Table 1 pulse over |x|, |y| <= 11 m; receivers at every
    grid point of that region.  refined: the data mesh of the same problem,
    0.5 m bricks and dt = 4.5e-4 s (every coarse node is a node of it)."""
    if refined:
        prob = Problem((48, 48, 90), 10, 10, 0.5, 4.5e-4, 1112)
    else:
        prob = Problem((24, 24, 45), 5, 5, 1.0, 9e-4, 556)
    _, _, gz = _interior_grid(prob)
    lam = material_28(gz)
    return _traction_workload(f"sec41_{pulse}{'_fine' if refined else ''}", prob, lam, lam.copy(), pulse, 11.0)


def material_30(z):
    """(30): layers of 80 / 101.25 / 125 MPa (lam = mu) at 0..-12, -12..-27,
    below -27 m; a node on an interface takes the shallower layer's value."""
    return 1e6 * np.where(z >= -12.0 - 1e-9, 80.0, np.where(z >= -27.0 - 1e-9, 101.25, 125.0))


def section43(pulse="p20", nsteps=450, refined=False):
    """Sec. 4.3 layered medium: 40 x 40 x 45 m interior, 6.25 m PML, 1.25 m
    bricks, dt = 1e-3 s (T = 0.45 s for p20); target (30); start: homogeneous
    80 MPa; 1 kPa vertical traction over |x|, |y| <= 17.5 m, receivers at
    every grid point there.  refined: 0.625 m bricks, dt/2 (data mesh)."""
    if refined:
        prob = Problem((64, 64, 72), 10, 10, 0.625, 5e-4, 2 * nsteps)
    else:
        prob = Problem((32, 32, 36), 5, 5, 1.25, 1e-3, nsteps)
    _, _, gz = _interior_grid(prob)
    lam_t = material_30(gz)
    start = np.full(prob.n_int_nodes, 80e6)
    wl = _traction_workload(f"sec43_{pulse}{'_fine' if refined else ''}", prob, start, start.copy(), pulse, 17.5)
    wl.lam_true, wl.mu_true = lam_t, lam_t.copy()
    return wl


def tiny_traction(ne_int=(4, 4, 2), npml_side=1, npml_bottom=1, nsteps=40, seed=0, half=1.0, pulse="p40"):
    """Small heterogeneous problem with a surface traction (parity checks)."""
    base = tiny(ne_int=ne_int, npml_side=npml_side, npml_bottom=npml_bottom, nsteps=nsteps, seed=seed)
    _, mean, var, _ = TABLE1[pulse]
    wav = sample_wavelet(lambda t: gaussian_pulse(t, 0.3 * mean, 0.3 * var), base.prob.dt, nsteps, 1000.0)[None]
    return Workload("tiny_traction", base.prob, base.rho, base.lam, base.mu, wav, base.src_node[:1],
                    np.array([[0.0, 0.0, -1.0]]), base.rec_node,
                    traction=(-half, half, -half, half, (0.0, 0.0, -1.0)))
