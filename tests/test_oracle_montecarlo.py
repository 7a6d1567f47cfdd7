"""Brute-force particle pins of the FP64 oracle.

1. Discrete Markov chain (exact for the upwind scheme): every particle sits
   in a phase-space cell; streaming moves it by s*(j-h) sites; the upwind
   drift moves it one velocity cell toward u with probability |nu_j|; the
   diffusion moves it one cell up / down with probability D each (blocked
   at the outer faces).  The expected histogram of this chain is exactly the
   upwind lattice update of Sec. 2 of arXiv:1508.02899, so the oracle must
   match the particle histogram within Monte-Carlo noise.
2. Continuous Langevin particles (Eq. 5) and the closed-form Ornstein-
   Uhlenbeck moments: the lattice must converge to them at first order in
   dv (Sec. 3.2 reports first-order convergence).
"""
import math

import numpy as np
import pytest

import oracle


def _chain_1d(rng, n, nx, nv, s, u, tau_p, kappa, dx, dt, nsteps, x0, j0):
    h = (nv - 1) // 2
    dv = s * dx / dt
    D = kappa * dt / dv ** 2
    x = x0.copy()
    j = j0.copy()
    for _ in range(nsteps):
        x = (x + s * (j - h)) % nx
        nu = dt * (u[x] - (j - h) * dv) / (tau_p * dv)
        r = rng.random(n)
        up = (nu > 0) & (j < nv - 1) & (r < nu)
        dn = (nu < 0) & (j > 0) & (r < -nu)
        j = j + up - dn
        r = rng.random(n)
        up = (r < D) & (j < nv - 1)
        dn = (r >= D) & (r < 2 * D) & (j > 0)
        j = j + up - dn
    return x, j


def test_upwind_equals_markov_chain_1d():
    rng = np.random.default_rng(11)
    nx, nv, s = 8, 7, 1
    dx, dt = 0.25, 0.125
    dv = dx / dt
    # |u| reaches past Vmax = 6 at some sites: the zero-flux outer faces
    # (Sec. 2) then block moves out of the velocity range
    u = rng.uniform(-8.0, 8.0, nx)
    tau_p, kappa = 1.0, 0.15 * dv * dv / dt
    n = 400_000
    nsteps = 6
    # start: all particles at site 2, velocity index 1
    x0 = np.full(n, 2)
    j0 = np.full(n, 1)
    x, j = _chain_1d(rng, n, nx, nv, s, u, tau_p, kappa, dx, dt, nsteps, x0, j0)
    hist = np.zeros((nv, nx))
    np.add.at(hist, (j, x), 1.0)
    hist /= n
    f0 = np.zeros((nv, nx))
    f0[1, 2] = 1.0
    cfl, Dn = oracle.stability(u[None], dim=1, nx=nx, ny=1, nv=nv, dx=dx,
                               tau_p=tau_p, kappa=kappa, dt=dt)
    assert cfl < 1 and Dn < 0.5
    out = oracle.step(f0, u[None], dim=1, dx=dx, dt=dt, tau_p=tau_p,
                      kappa=kappa, nsteps=nsteps, scheme="upwind")
    sigma = np.sqrt(np.maximum(out * (1 - out), 1e-12) / n)
    assert np.all(np.abs(hist - out) <= 5 * sigma + 1e-9), \
        np.max(np.abs(hist - out) / (sigma + 1e-12))


def test_upwind_equals_markov_chain_2d_with_stride_and_nsub():
    """2D order A_x, A_y, D_x, D_y per sub-step, nsub = 2, stride s = 2."""
    rng = np.random.default_rng(12)
    nx, ny, nv, s, nsub = 5, 4, 5, 2, 2
    h = (nv - 1) // 2
    dx, dt = 0.2, 0.1
    dv = s * dx / dt
    dts = dt / nsub
    ux = rng.uniform(-3, 3, (ny, nx))
    uy = rng.uniform(-3, 3, (ny, nx))
    tau_p = 0.5
    kappa = 0.2 * dv * dv / dts
    D = kappa * dts / dv ** 2
    n = 400_000
    nsteps = 3
    x = np.full(n, 1)
    y = np.full(n, 2)
    jx = np.full(n, 3)
    jy = np.full(n, 1)

    def drift(j, ucomp):
        nu = dts * (ucomp - (j - h) * dv) / (tau_p * dv)
        r = rng.random(n)
        up = (nu > 0) & (j < nv - 1) & (r < nu)
        dn = (nu < 0) & (j > 0) & (r < -nu)
        return j + up - dn

    def diffuse(j):
        r = rng.random(n)
        up = (r < D) & (j < nv - 1)
        dn = (r >= D) & (r < 2 * D) & (j > 0)
        return j + up - dn

    for _ in range(nsteps):
        x = (x + s * (jx - h)) % nx
        y = (y + s * (jy - h)) % ny
        for _ in range(nsub):
            jx = drift(jx, ux[y, x])
            jy = drift(jy, uy[y, x])
            jx = diffuse(jx)
            jy = diffuse(jy)
    hist = np.zeros((nv * nv, ny, nx))
    np.add.at(hist, (jy * nv + jx, y, x), 1.0)
    hist /= n
    f0 = np.zeros((nv * nv, ny, nx))
    f0[1 * nv + 3, 2, 1] = 1.0
    u = np.stack([ux, uy])[None]
    cfl, Dn = oracle.stability(u, dim=2, nx=nx, ny=ny, nv=nv, dx=dx,
                               tau_p=tau_p, kappa=kappa, dt=dt, s=s, nsub=nsub)
    assert cfl < 1 and Dn < 0.5
    out = oracle.step(f0, u, dim=2, dx=dx, dt=dt, tau_p=tau_p, kappa=kappa,
                      nsteps=nsteps, scheme="upwind", s=s, nsub=nsub)
    sigma = np.sqrt(np.maximum(out * (1 - out), 1e-12) / n)
    assert np.all(np.abs(hist - out) <= 5 * sigma + 1e-9)


def _ou_lattice(nv, dt, vmax, tau_p, kappa, T, scheme, nx=1):
    """Lattice with u = 0, all mass at v = 0, uniform in x."""
    h = (nv - 1) // 2
    dv = vmax / h
    dx = dv * dt
    nsteps = int(round(T / dt))
    f = np.zeros((nv, nx))
    f[h, :] = 1.0 / (nx * dx * dv)
    u = np.zeros((1, nx))
    cfl, D = oracle.stability(u, dim=1, nx=nx, ny=1, nv=nv, dx=dx,
                              tau_p=tau_p, kappa=kappa, dt=dt)
    assert cfl <= 0.5 and D < 0.5  # Eqs. 3 and 4
    out = oracle.step(f, u, dim=1, dx=dx, dt=dt, tau_p=tau_p, kappa=kappa,
                      nsteps=nsteps, scheme=scheme)
    return oracle.moments(out, dim=1, dx=dx, dt=dt)


def test_velocity_variance_converges_to_ou_closed_form_upwind():
    """u = 0: Eq. 5 is an Ornstein-Uhlenbeck process; from v(0) = 0,
    Var v(t) = kappa tau_p (1 - exp(-2t/tau_p)).  The upwind lattice error
    halves when dv and dt are halved (first order, Sec. 3.2)."""
    tau_p, kappa, vmax, T = 1.0, 0.25, 2.5, 1.5
    exact = kappa * tau_p * (1 - math.exp(-2 * T / tau_p))
    errs = []
    for nv, dt in [(21, 0.02), (41, 0.01), (81, 0.005)]:
        m = _ou_lattice(nv, dt, vmax, tau_p, kappa, T, "upwind")
        assert abs(m["momentum"][0]) < 1e-12
        errs.append(abs(m["variance"] - exact) / exact)
    assert errs[0] < 0.25
    for a, b in zip(errs, errs[1:]):
        assert 0.4 < b / a < 0.6


def test_velocity_variance_converges_to_ou_closed_form_koren():
    """Same closed form; the limited scheme converges faster in dv, leaving
    the O(dt) splitting error: refining dv and dt drives the error to 0."""
    tau_p, kappa, vmax, T = 1.0, 0.25, 2.5, 1.5
    exact = kappa * tau_p * (1 - math.exp(-2 * T / tau_p))
    errs = []
    for nv, dt in [(21, 0.02), (81, 0.0025), (161, 0.0005)]:
        m = _ou_lattice(nv, dt, vmax, tau_p, kappa, T, "koren")
        errs.append(abs(m["variance"] - exact) / exact)
    assert errs[0] < 0.02 and errs[1] < 5e-4 and errs[2] < 1e-4
    assert errs[2] < errs[1] < errs[0]


def test_stationary_variance_tends_to_kappa_taup():
    """Balance of drag and diffusion (Sec. 3.1): v_d^2 = kappa tau_p."""
    tau_p, kappa, vmax = 0.5, 0.5, 2.0
    errs = []
    for nv, dt in [(17, 0.03), (33, 0.008), (65, 0.002)]:
        m = _ou_lattice(nv, dt, vmax, tau_p, kappa, 6.0, "koren")
        errs.append(abs(m["variance"] - kappa * tau_p) / (kappa * tau_p))
    assert errs[2] < 0.02
    assert errs[1] < errs[0] and errs[2] < errs[1]


def test_position_variance_converges_to_langevin_closed_form():
    """Full step (stream, drift, diffusion) with u = 0, from x = 0, v = 0:
    Var x(t) = 2 kappa tau_p^3 [t/tau_p - 2(1 - e^{-t/tau_p})
    + (1 - e^{-2t/tau_p})/2] for the Langevin particle of Eq. 5."""
    tau_p, kappa, vmax, T = 1.0, 0.3, 2.0, 2.0
    a = T / tau_p
    exact = 2 * kappa * tau_p ** 3 * (a - 2 * (1 - math.exp(-a))
                                      + 0.5 * (1 - math.exp(-2 * a)))
    errs = []
    for nv, dt in [(9, 0.08), (17, 0.04), (33, 0.02)]:
        h = (nv - 1) // 2
        dv = vmax / h
        dx = dv * dt
        nx = 2 * int(math.ceil(6 * math.sqrt(exact) / dx)) + 1
        nsteps = int(round(T / dt))
        f = np.zeros((nv, nx))
        f[h, nx // 2] = 1.0
        cfl, D = oracle.stability(np.zeros((1, nx)), dim=1, nx=nx, ny=1, nv=nv,
                                  dx=dx, tau_p=tau_p, kappa=kappa, dt=dt)
        assert cfl <= 0.5 and D < 0.5  # Eqs. 3 and 4
        out = oracle.step(f, np.zeros((1, nx)), dim=1, dx=dx, dt=dt,
                          tau_p=tau_p, kappa=kappa, nsteps=nsteps)
        rho = out.sum(axis=0)
        xs = (np.arange(nx) - nx // 2) * dx
        var = (rho * xs ** 2).sum() / rho.sum() - ((rho * xs).sum() / rho.sum()) ** 2
        errs.append(abs(var - exact) / exact)
    assert errs[2] < 0.05
    assert errs[1] < errs[0] and errs[2] < errs[1]


def test_lattice_matches_langevin_particles_in_random_flow():
    """The paper's own validation (Sec. 3.2): Lagrangian particles of Eq. 5
    in a two-mode flow (Eq. 6 with frozen amplitudes) vs the lattice on a
    small grid, in the paper's geometry dt = dx/dv.  Compared: the velocity
    variance and the coarse-grained density at r = L/8 after four response
    times.  The lattice error is O(dv): it must be small and shrink when the
    velocity lattice is refined (nv 17 -> 33, nx 1024 -> 4096)."""
    rng = np.random.default_rng(13)
    L, vmax, tau_p, kappa, T = 2 * np.pi, 2.0, 1.0, 0.05, 4.0
    A1, A2 = 0.8, -0.6

    def flow(x):
        return A1 * np.cos(2 * np.pi * x / L) + A2 * np.sin(2 * np.pi * x / L)

    n = 100_000
    xp = rng.random(n) * L
    vp = np.zeros(n)
    hdt = 0.005
    for _ in range(int(round(T / hdt))):
        up = flow(xp)
        xp = (xp + vp * hdt) % L
        vp = vp + (up - vp) / tau_p * hdt + math.sqrt(2 * kappa * hdt) * rng.standard_normal(n)
    rho_par = np.histogram(xp, bins=8, range=(0, L))[0] / n

    var_err, rho_err = [], []
    for nx, nv in [(1024, 17), (4096, 33)]:
        dx = L / nx
        h = (nv - 1) // 2
        dv = vmax / h
        dt = dx / dv
        # lattice sites sit at cell centres (i + 1/2) dx so that 8 boxes of
        # nx/8 cells tile [0, L) like the particle histogram
        u = flow((np.arange(nx) + 0.5) * dx)
        cfl, D = oracle.stability(u[None], dim=1, nx=nx, ny=1, nv=nv, dx=dx,
                                  tau_p=tau_p, kappa=kappa, dt=dt)
        assert cfl <= 0.5 and D < 0.5  # Eqs. 3 and 4
        nsteps = int(round(T / dt))
        f = np.zeros((nv, nx))
        f[h, :] = 1.0 / (L * dv)
        out = oracle.step(f, u[None], dim=1, dx=dx, dt=dt, tau_p=tau_p,
                          kappa=kappa, nsteps=nsteps, scheme="koren")
        m = oracle.moments(out, dim=1, dx=dx, dt=dt)
        assert abs(m["momentum"][0] / m["mass"] - vp.mean()) < 0.01
        var_err.append(abs(m["variance"] - vp.var()) / vp.var())
        rho_lat = out.sum(axis=0).reshape(8, -1).sum(axis=1)
        rho_err.append(np.abs(rho_lat / rho_lat.sum() - rho_par).max())
    assert var_err[0] < 0.1 and var_err[1] < 0.05
    assert var_err[1] < var_err[0]
    assert rho_err[0] < 0.02 and rho_err[1] < 0.01
