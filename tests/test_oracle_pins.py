"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: values the
paper prints, textbook closed forms, invariants (rigid-body modes, energy,
reciprocity) and brute force (finite differences).
"""
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle import lgl, pml
from oracle.assemble import System, free_box_stiffness
from oracle.mesh import Mesh
from oracle.solve import Stepper

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    out = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                out.append(line.split())
    return out


# ---------------------------------------------------------------- LGL rule
def test_lgl_matches_textbook_rule():
    x, w, D = lgl.rule(2)
    ref = np.array([[float(v) for v in r] for r in _rows("lgl3.txt")])
    np.testing.assert_allclose(x, ref[:, 0], atol=1e-15)
    np.testing.assert_allclose(w, ref[:, 1], rtol=1e-14)
    # exact for polynomials up to degree 2p-1 = 3
    for k in range(4):
        exact = (1 - (-1) ** (k + 1)) / (k + 1)
        assert abs(np.dot(w, x ** k) - exact) < 1e-14
    # derivative matrix differentiates quadratics exactly
    for coeffs in ([1.0, 0, 0], [0, 1.0, 0], [0.3, -2.0, 1.7]):
        f = np.polyval(coeffs[::-1], x)
        df = np.polyval(np.polyder(np.array(coeffs[::-1])), x)
        np.testing.assert_allclose(D @ f, df, atol=1e-13)


# ---------------------------------------------------------------- problem sizes
@pytest.mark.parametrize("row", _rows("paper_sizes.txt"), ids=lambda r: r[0])
def test_paper_problem_sizes(row):
    _, Lx, Ly, Lz, Lp, h, n_state, n_mat = row
    Lx, Ly, Lz, Lp, h = map(float, (Lx, Ly, Lz, Lp, h))
    ne = (round(Lx / h), round(Ly / h), round(Lz / h))
    npml = round(Lp / h)
    prob = W.Problem(ne, npml, npml, h, 1e-3, 1)
    m = Mesh(prob)
    assert m.n_state == int(n_state)
    assert 2 * m.n_int_nodes == int(n_mat)
    assert int(m.in_rd.sum()) == m.n_int_nodes


# ---------------------------------------------------------------- stiffness
def _rigid_modes(xyz):
    n = xyz.shape[0]
    modes = []
    for i in range(3):
        v = np.zeros((n, 3))
        v[:, i] = 1.0
        modes.append(v.ravel())
    for axis in np.eye(3):
        modes.append(np.cross(axis, xyz).ravel())
    return np.array(modes).T


def test_element_and_free_mesh_have_six_rigid_modes():
    rng = np.random.default_rng(3)
    lam_fn = lambda p: 1e8 * (1 + 0.5 * rng.uniform(size=p.shape[0]))
    mu_fn = lambda p: 5e7 * (1 + 0.5 * rng.uniform(size=p.shape[0]))
    for ne in ((1, 1, 1), (3, 3, 3)):
        K, Mdiag, xyz = free_box_stiffness(ne, 1.3, lam_fn, mu_fn)
        Kd = K.toarray()
        assert np.allclose(Kd, Kd.T, rtol=0, atol=1e-6 * np.abs(Kd).max())
        R = _rigid_modes(xyz)
        assert np.abs(Kd @ R).max() < 1e-7 * np.abs(Kd).max()
        if ne == (1, 1, 1):
            ev = np.linalg.eigvalsh(Kd)
            scale = ev.max()
            assert np.sum(np.abs(ev) < 1e-10 * scale) == 6
            assert ev.min() > -1e-10 * scale
        else:
            # nullity 6: the 7 smallest generalized eigenvalues
            Minv_sqrt = 1.0 / np.sqrt(Mdiag)
            A = (Minv_sqrt[:, None] * Kd) * Minv_sqrt[None, :]
            ev = np.linalg.eigvalsh(A)
            assert np.all(np.abs(ev[:6]) < 1e-8 * ev[-1])
            assert ev[6] > 1e-6 * ev[-1]


def test_lumped_masses_are_volumes():
    prob = W.Problem((4, 3, 2), 2, 1, 0.7, 1e-3, 1)
    m = Mesh(prob)
    Vin = 4 * 3 * 2 * 0.7 ** 3
    Vtot = (4 + 4) * (3 + 4) * (2 + 1) * 0.7 ** 3
    assert abs(m.m_rd.sum() - Vin) < 1e-12 * Vin
    assert abs(m.m_p.sum() - (Vtot - Vin)) < 1e-12 * Vtot
    wl = W.tiny(ne_int=(4, 3, 2), npml_side=2, npml_bottom=1, h=0.7)
    s = System(wl.prob, wl.rho, wl.lam, wl.mu)
    # rows of the u mass are rho * (m_rd + a m_p): with the PML off, a = 1 and
    # the u-mass sums to rho times the free-node volume share
    assert np.all(s.M > 0)


# ---------------------------------------------------------------- PML stretching
def test_pml_coefficients_reproduce_frequency_domain_stretching():
    prob = W.Problem((2, 2, 2), 2, 2, 1.0, 1e-3, 1, 5.0, 400.0, 2)
    m = Mesh(prob)
    cf = pml.coefficients(m, 5.0, 400.0, 2)
    rng = np.random.default_rng(0)
    for omega in rng.uniform(5.0, 500.0, size=4):
        q = 1.0 / (1j * omega)
        eps = cf["alpha"] + cf["beta"] * q                  # (n, 3)
        prod = eps[:, 0] * eps[:, 1] * eps[:, 2]
        lam_w = np.stack([eps[:, 1] * eps[:, 2], eps[:, 0] * eps[:, 2],
                          eps[:, 0] * eps[:, 1]], axis=1)
        np.testing.assert_allclose(cf["Le"] + cf["Lp"] * q + cf["Lw"] * q * q, lam_w,
                                   rtol=1e-13)
        np.testing.assert_allclose(cf["a"] + cf["b"] * q + cf["c"] * q ** 2 + cf["d"] * q ** 3,
                                   prod, rtol=1e-13)
    inside = ~m.in_pml | (np.isclose(np.abs(m.xyz[:, 0]), 1.0) & (np.abs(m.xyz[:, 1]) <= 1.0)
                          & (m.xyz[:, 2] >= -2.0))
    assert np.all(cf["Le"][inside] == 1.0) and np.all(cf["Lp"][inside] == 0.0)
    assert np.all(cf["a"][inside] == 1.0) and np.all(cf["d"][inside] == 0.0)
    # profile: at the outer +x face alpha = 1 + alpha_o, beta = beta_o
    outer = np.isclose(m.xyz[:, 0], m.xyz[:, 0].max())
    assert np.allclose(cf["alpha"][outer, 0], 6.0) and np.allclose(cf["beta"][outer, 0], 400.0)
    mid = np.isclose(m.xyz[:, 0], 1.0 + 1.0)
    assert np.allclose(cf["beta"][mid, 0], 100.0)


# ---------------------------------------------------------------- invariants of the forward map
def _stepper(wl, lam=None, mu=None):
    s = System(wl.prob, wl.rho, wl.lam if lam is None else lam, wl.mu if mu is None else mu)
    return s, Stepper(s, wl.src_node, wl.src_dir, wl.rec_node)


def _energy(s, X):
    m = s.mesh
    nh, ns, nu = s.n_hist, s.n_state, m.n_u
    x1 = X[nh:nh + ns, 0]
    x2 = X[nh + ns:, 0]
    Ek = 0.5 * np.dot(x2[:nu] * s.M[:nu], x2[:nu])
    Ep = 0.5 * np.dot(x1[:nu], s.Krd[:nu, :nu] @ x1[:nu])
    sig = x2[nu:].reshape(-1, 6)
    sn = m.s_node
    Es = 0.0
    for j, node in enumerate(sn):
        C = s.lam[node] * np.outer([1, 1, 1, 0, 0, 0], [1, 1, 1, 0, 0, 0]) + \
            s.mu[node] * np.diag([2, 2, 2, 1, 1, 1.0])
        Es += 0.5 * m.m_p[node] * sig[j] @ np.linalg.solve(C, sig[j])
    return Ek + Ep + Es


def _energy_run(dt_scale):
    wl = W.tiny(ne_int=(2, 2, 2), npml_side=1, npml_bottom=1, nsteps=1,
                alpha0=0.0, beta0=0.0, fc=40.0, seed=5)
    dt = wl.prob.dt * dt_scale
    n0 = int(round(0.05 / dt))
    N = n0 + int(round(0.04 / dt))
    prob = wl.prob.replace(dt=dt, nsteps=N)
    wav = W.sample_wavelet(lambda t: W.ricker(t, 40.0), dt, N, 1000.0)[None]
    wav[:, 2 * n0:] = 0.0
    s = System(prob, wl.rho, wl.lam, wl.mu)
    st = Stepper(s, wl.src_node, wl.src_dir, wl.rec_node)
    X = np.zeros((s.n_X, 1))
    E = []
    for n in range(N):
        X = st.step(X, wav, n)
        if n + 1 >= n0:
            E.append(_energy(s, X))
    return np.array(E)


def test_energy_conserved_with_pml_off():
    E1 = _energy_run(0.5)
    assert E1[0] > 0
    assert np.all(np.diff(E1) <= 1e-13 * E1[0])         # RK4 never adds energy
    loss1 = (E1[0] - E1[-1]) / E1[0]
    E2 = _energy_run(0.25)
    loss2 = (E2[0] - E2[-1]) / E2[0]
    assert loss1 < 1e-3
    # RK4 dissipation of a mode per unit time ~ dt^5: halving dt cuts it ~32x
    assert 16.0 < loss1 / loss2 < 40.0


def test_pml_absorbs():
    def run(alpha0, beta0):
        wl = W.tiny(ne_int=(4, 4, 2), npml_side=2, npml_bottom=2, nsteps=1,
                    alpha0=alpha0, beta0=beta0, fc=40.0, seed=2, hetero=0.0)
        dt = wl.prob.dt
        n0 = int(round(0.05 / dt))
        N = n0 + int(round(0.45 / dt))
        prob = wl.prob.replace(nsteps=N)
        wav = W.sample_wavelet(lambda t: W.ricker(t, 40.0), dt, N, 1000.0)[None]
        wav[:, 2 * n0:] = 0.0
        s = System(prob, wl.rho, wl.lam, wl.mu)
        st = Stepper(s, wl.src_node, wl.src_dir, wl.rec_node)
        X = np.zeros((s.n_X, 1))
        nu = s.mesh.n_u
        interior = s.mesh.u_dof[~s.mesh.in_pml & ~s.mesh.dirichlet].ravel()
        e = []
        for n in range(N):
            X = st.step(X, wav, n)
            x1 = X[s.n_hist:s.n_hist + s.n_state, 0]
            x2 = X[s.n_hist + s.n_state:, 0]
            if n + 1 >= n0:
                e.append(0.5 * np.dot(x2[interior] * s.M[interior], x2[interior]))
        return np.array(e)
    on = run(5.0, 400.0)
    off = run(0.0, 0.0)
    # interior kinetic energy at the end relative to when the source stopped:
    # the PML drains it, without the PML it only moves around the box
    k = len(on) // 10
    assert on[-k:].mean() < 0.03 * on[0]
    assert off[-k:].mean() > 0.2 * off[0]


def test_source_receiver_reciprocity_with_pml():
    wl = W.tiny(ne_int=(4, 4, 2), npml_side=2, npml_bottom=1, nsteps=120, seed=9)
    rec = wl.rec_node
    A, B = rec[7], rec[-5]
    s = System(wl.prob, wl.rho, wl.lam, wl.mu)
    wav = wl.wavelet[:1]
    for da in range(3):
        for db in range(3):
            ea = np.eye(3)[da][None]
            eb = np.eye(3)[db][None]
            stA = Stepper(s, np.array([A]), ea, np.array([B]))
            stB = Stepper(s, np.array([B]), eb, np.array([A]))
            tAB, _ = stA.forward(wav)
            tBA, _ = stB.forward(wav)
            x = tAB[0, :, 0, db]
            y = tBA[0, :, 0, da]
            assert np.abs(x - y).max() <= 1e-11 * np.abs(x).max()


# ---------------------------------------------------------------- adjoint and gradient
def test_adjoint_step_is_transpose_of_step():
    wl = W.tiny(seed=4, nsteps=3)
    s, st = _stepper(wl)
    rng = np.random.default_rng(1)
    X = rng.standard_normal((s.n_X, 1))
    L = rng.standard_normal((s.n_X, 1))
    zero = np.zeros((1, 2 * wl.prob.nsteps + 1))
    lhs = float(np.sum(st.step(X, zero, 0) * L))
    rhs = float(np.sum(X * st.adjoint_step(L)))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0) * 10


def _fd_setup(seed=11, nsteps=60):
    wl = W.tiny(ne_int=(2, 2, 2), npml_side=1, npml_bottom=1, nsteps=nsteps, seed=seed)
    rng = np.random.default_rng(seed)
    lam_t = wl.lam * (1 + 0.15 * rng.uniform(-1, 1, wl.lam.size))
    mu_t = wl.mu * (1 + 0.15 * rng.uniform(-1, 1, wl.mu.size))
    _, st_t = _stepper(wl, lam_t, mu_t)
    obs, _ = st_t.forward(wl.wavelet)
    return wl, obs


def _J(wl, obs, lam, mu):
    _, st = _stepper(wl, lam, mu)
    tr, _ = st.forward(wl.wavelet)
    return st.misfit(tr, obs)


def _interface_mask(prob):
    nix, niy, niz = prob.nn_int
    gk, gj, gi = np.meshgrid(np.arange(niz), np.arange(niy), np.arange(nix), indexing="ij")
    return ((gi == 0) | (gi == nix - 1) | (gj == 0) | (gj == niy - 1) | (gk == 0)).ravel()


def test_gradient_matches_central_differences():
    wl, obs = _fd_setup()
    _, st = _stepper(wl)
    g_lam, g_mu, _ = st.adjoint_gradient(wl.wavelet, obs)
    rng = np.random.default_rng(5)
    mask = _interface_mask(wl.prob)
    for which in ("lam", "mu", "both"):
        d_l = rng.uniform(-1, 1, wl.lam.size) * (which != "mu")
        d_m = rng.uniform(-1, 1, wl.mu.size) * (which != "lam")
        d_l[mask] = 0.0
        d_m[mask] = 0.0
        eps = 1e-5
        hl = eps * np.abs(wl.lam).max()
        hm = eps * np.abs(wl.mu).max()
        Jp = _J(wl, obs, wl.lam + hl * d_l, wl.mu + hm * d_m)
        Jm = _J(wl, obs, wl.lam - hl * d_l, wl.mu - hm * d_m)
        fd = (Jp - Jm) / 2.0
        co = hl * np.dot(d_l, g_lam) + hm * np.dot(d_m, g_mu)
        assert abs(fd - co) <= 1e-6 * abs(co), (which, fd, co)


def test_full_gradient_matches_central_differences_on_the_interface():
    """With the chain rule through the material carried into the PML, the
    gradient is the exact derivative everywhere, interface nodes included:
    central differences along unrestricted directions (and along directions
    supported on the interface alone) agree; the restricted gradient does
    not, and the two differ only on the interface nodes."""
    wl, obs = _fd_setup()
    s, _ = _stepper(wl)
    st_full = Stepper(s, wl.src_node, wl.src_dir, wl.rec_node, full_gradient=True)
    st_int = Stepper(s, wl.src_node, wl.src_dir, wl.rec_node)
    gl_f, gm_f, _ = st_full.adjoint_gradient(wl.wavelet, obs)
    gl_r, gm_r, _ = st_int.adjoint_gradient(wl.wavelet, obs)
    mask = _interface_mask(wl.prob)
    assert np.array_equal(gl_f[~mask], gl_r[~mask]) and np.array_equal(gm_f[~mask], gm_r[~mask])
    assert np.abs(gl_f[mask] - gl_r[mask]).max() > 1e-3 * np.abs(gl_f).max()
    rng = np.random.default_rng(15)
    for which in ("lam", "mu", "both", "interface"):
        d_l = rng.uniform(-1, 1, wl.lam.size) * (which != "mu")
        d_m = rng.uniform(-1, 1, wl.mu.size) * (which != "lam")
        if which == "interface":
            d_l[~mask] = 0.0
            d_m[~mask] = 0.0
        eps = 1e-5
        hl = eps * np.abs(wl.lam).max()
        hm = eps * np.abs(wl.mu).max()
        fd = (_J(wl, obs, wl.lam + hl * d_l, wl.mu + hm * d_m)
              - _J(wl, obs, wl.lam - hl * d_l, wl.mu - hm * d_m)) / 2.0
        co = hl * np.dot(d_l, gl_f) + hm * np.dot(d_m, gm_f)
        co_r = hl * np.dot(d_l, gl_r) + hm * np.dot(d_m, gm_r)
        assert abs(fd - co) <= 1e-6 * abs(co), (which, fd, co)
        assert abs(fd - co_r) > 1e-3 * abs(fd), (which, fd, co_r)


def test_taylor_remainder_is_second_order():
    wl, obs = _fd_setup(seed=12, nsteps=40)
    _, st = _stepper(wl)
    g_lam, g_mu, _ = st.adjoint_gradient(wl.wavelet, obs)
    tr, _ = st.forward(wl.wavelet)
    J0 = st.misfit(tr, obs)
    rng = np.random.default_rng(8)
    mask = _interface_mask(wl.prob)
    d_l = rng.uniform(-1, 1, wl.lam.size) * np.abs(wl.lam).max()
    d_m = rng.uniform(-1, 1, wl.mu.size) * np.abs(wl.mu).max()
    d_l[mask] = d_m[mask] = 0.0
    rem = []
    for eps in (4e-2, 2e-2, 1e-2):
        J = _J(wl, obs, wl.lam + eps * d_l, wl.mu + eps * d_m)
        rem.append(abs(J - J0 - eps * (d_l @ g_lam + d_m @ g_mu)))
    r1, r2 = rem[0] / rem[1], rem[1] / rem[2]
    assert 3.0 < r1 < 5.0 and 3.0 < r2 < 5.0, rem


def test_misfit_and_gradient_vanish_at_target():
    wl, _ = _fd_setup(nsteps=30)
    _, st = _stepper(wl)
    obs, _ = st.forward(wl.wavelet)
    assert st.misfit(obs, obs) == 0.0
    g_lam, g_mu, _ = st.adjoint_gradient(wl.wavelet, obs)
    assert np.all(g_lam == 0.0) and np.all(g_mu == 0.0)


def test_appendix_b_gradient_converges_to_discrete_gradient():
    """The paper's reverse RK4 (App. B) approximates the exact discrete
    gradient; the gap shrinks at second order when dt is halved."""
    gaps = []
    for k in (1, 2):
        wl = W.tiny(ne_int=(2, 2, 2), npml_side=1, npml_bottom=1, nsteps=1, seed=13, fc=20.0)
        dt = wl.prob.dt / (2 * k)
        N = int(round(0.08 / dt))
        prob = wl.prob.replace(dt=dt, nsteps=N)
        wav = W.sample_wavelet(lambda t: W.ricker(t, 20.0), dt, N, 1000.0)[None]
        rng = np.random.default_rng(13)
        s_t = System(prob, wl.rho, wl.lam * (1 + 0.1 * rng.uniform(-1, 1, wl.lam.size)), wl.mu)
        st_t = Stepper(s_t, wl.src_node, wl.src_dir, wl.rec_node)
        obs, _ = st_t.forward(wav)
        s = System(prob, wl.rho, wl.lam, wl.mu)
        st = Stepper(s, wl.src_node, wl.src_dir, wl.rec_node)
        _, states = st.forward(wav, store=True)
        gl, gm, _ = st.adjoint_gradient(wav, obs, states)
        al, am = st.adjoint_gradient_appb(wav, obs, states)
        gaps.append(np.linalg.norm(np.r_[al - gl, am - gm]) / np.linalg.norm(np.r_[gl, gm]))
    assert gaps[0] < 0.05
    assert gaps[0] / gaps[1] > 3.0, gaps


# ---------------------------------------------------------------- time accuracy of (6) and the misfit (7)
def _traces_at_dt(wl, dt, T, fc, stage_times="rk4"):
    """Traces of a fixed model up to time T at step dt (load: Ricker of fc).

    stage_times="rk4" is the oracle as it stands; "t_n" plants a mistake in
    a copy of it (every stage sees the load at t_n) to show what the pin
    catches."""
    N = int(round(T / dt))
    prob = wl.prob.replace(dt=dt, nsteps=N)
    s = System(prob, wl.rho, wl.lam, wl.mu)
    st = Stepper(s, wl.src_node, wl.src_dir, wl.rec_node)
    if stage_times == "t_n":
        exact = st.stages

        def stages(X, wav, n):
            w = wav.copy()
            w[:, 2 * n + 1] = wav[:, 2 * n]
            w[:, 2 * n + 2] = wav[:, 2 * n]
            return exact(X, w, n)
        st.stages = stages
    wav = W.sample_wavelet(lambda t: W.ricker(t, fc), dt, N, 1000.0)[None]
    tr, _ = st.forward(wav)
    return tr


@pytest.mark.parametrize("stage_times,lo,hi", [("rk4", 13.0, 19.0), ("t_n", 1.5, 2.5)])
def test_forward_traces_converge_at_fourth_order_in_dt(stage_times, lo, hi):
    """Classical RK4 with the load at t_n, t_n + dt/2 (twice), t_n + dt is
    fourth-order accurate in time: on a PML mesh with a smooth load, the
    trace differences between dt, dt/2 and dt/4 (same horizon T) fall by
    2^4 = 16.  Sampling the load at t_n in every stage makes the scheme
    first order in the forcing (ratio 2), which this pin rejects."""
    wl = W.tiny(ne_int=(2, 2, 2), npml_side=1, npml_bottom=1, nsteps=1, seed=3)
    dt, T, fc = 0.5 * wl.prob.dt, 0.08, 25.0
    a, b, c = (_traces_at_dt(wl, dt / k, T, fc, stage_times) for k in (1, 2, 4))
    d1 = np.linalg.norm(a - b[:, ::2])
    d2 = np.linalg.norm(b[:, ::2] - c[:, ::4])
    assert d2 > 0
    assert lo < d1 / d2 < hi, (d1, d2)


def test_misfit_trapezoid_closed_forms():
    """(7) by the trapezoid rule over the step states: a constant residual r
    in every component gives 1/2 r^2 T per component exactly; a residual
    linear in time, a + b t, gives the trapezoid value of the quadratic
    (a + b t)^2, which is its integral plus dt^2 (f'(T) - f'(0)) / 12
    (Euler-Maclaurin ends at the first correction for a quadratic)."""
    wl = W.tiny(ne_int=(2, 2, 2), npml_side=1, npml_bottom=1, nsteps=37, seed=3)
    _, st = _stepper(wl)
    N, dt = wl.prob.nsteps, wl.prob.dt
    T = N * dt
    nrec = len(wl.rec_node)
    shape = (1, N + 1, nrec, 3)
    r = 0.37
    J = st.misfit(np.full(shape, r), np.zeros(shape))
    np.testing.assert_allclose(J, 0.5 * r * r * T * nrec * 3, rtol=1e-13)
    a, b = -0.8, 23.0
    t = dt * np.arange(N + 1)
    res = np.broadcast_to((a + b * t)[None, :, None, None], shape)
    integral = ((a + b * T) ** 3 - a ** 3) / (3.0 * b)
    trap = integral + dt * dt * (2.0 * b * b * T) / 12.0
    J = st.misfit(np.array(res) + 1.5, np.full(shape, 1.5))
    np.testing.assert_allclose(J, 0.5 * trap * nrec * 3, rtol=1e-12)


# ---------------------------------------------------------------- time step of the paper
def _material28_max():
    z = np.linspace(0.0, 45.0, 45001)
    return float(np.max(80.0 + 0.45 * z + 35.0 * np.exp(-(z - 22.5) ** 2 / 150.0))) * 1e6


def test_paper_time_steps_are_rk4_stable():
    """Sec. 4.1 (h = 1 m, dt = 9e-4 s) and Sec. 4.2 (h = 1.25 m, dt = 1e-3 s)
    ran stably; with the LGL rule for every integral the largest frequency of
    M^{-1}K stays inside RK4's imaginary-axis limit 2 sqrt(2)."""
    lm = _material28_max()
    for h, dt in ((1.0, 9e-4), (1.25, 1e-3)):
        K, Md, _ = free_box_stiffness((4, 4, 4), h, lambda p: np.full(p.shape[0], lm),
                                      lambda p: np.full(p.shape[0], lm), rho=2000.0)
        Ms = 1.0 / np.sqrt(Md)
        A = (K.multiply(Ms[:, None])).multiply(Ms[None, :]).tocsr()
        wmax2 = spla.eigsh(A, k=1, which="LA", return_eigenvectors=False)[0]
        theta = dt * np.sqrt(wmax2)
        assert 2.0 < theta < 2.0 * np.sqrt(2.0), theta


# ---------------------------------------------------------------- Table 1 pulses
def test_table1_pulses_read_sigma_as_variance():
    rows = [r for r in _rows("table1_pulses.txt")]
    for name, fmax, mean, sig, tend in rows:
        fmax, mean, sig, tend = map(float, (fmax, mean, sig, tend))
        t = np.linspace(0.0, 1.0, 200001)
        dtt = t[1] - t[0]
        for var, expect_small in ((sig, True), (sig ** 2, False)):
            f = W.gaussian_pulse(t, mean, var)
            spec0 = abs(np.sum(f)) * dtt
            specm = abs(np.sum(f * np.exp(-2j * np.pi * fmax * t))) * dtt
            if expect_small:
                assert specm < 0.01 * spec0, name
                assert W.gaussian_pulse(0.0, mean, var) < 1e-3
                assert W.gaussian_pulse(tend, mean, var) < 5e-2
            else:
                assert specm > 0.9 * spec0, name
