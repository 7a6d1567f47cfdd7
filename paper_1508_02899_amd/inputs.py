"""Seeded synthetic inputs: carrier flows and initial conditions.

This module produces inputs only; it contains none of the lattice update.
Both the GPU library and the CPU oracle are fed from the arrays it returns
(the oracle sees the same FP32-rounded values cast to FP64).

Flows (shapes and statistics of the paper's carrier flows, Secs. 3-4):
  * 1D random Fourier flows: u(x,t) = sum_k a_k(t) cos(k x 2pi/L)
    + b_k(t) sin(k x 2pi/L) with Gaussian amplitudes (Eq. 6 generalised
    to K modes); the amplitudes are either renewed (fresh independent
    draws) every ``renew`` steps, or evolve as Ornstein-Uhlenbeck processes
    with correlation time tau_f (Eq. 7), advanced with the exact OU update
    a <- a e^{-dt/tau_f} + sigma sqrt(1 - e^{-2dt/tau_f}) N(0,1);
  * 2D incompressible flows from a random streamfunction with energy shell
    spectrum E(k) ~ k^-3 on 1 <= |k| <= kmax (the direct-cascade
    Batchelor-Kraichnan range of Sec. 4.2), u = (d_y psi, -d_x psi), OU in
    time per mode;
  * the tilted cellular flow of Sec. 4.1 (closed form).
All flows are normalised to a per-component r.m.s. of ``urms`` over the
sampled slices' statistics (the modal variances are scaled so that the
ensemble r.m.s. is urms).

Initial condition: uniform in space, Gaussian in each velocity component
(standard deviation sigma0), normalised so that sum f dx^d dv^d = 1.
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 150802899


def seed_for(config: int, realization: int = 0, extra: int = 0) -> int:
    return SEED_BASE + 1000 * config + 10 * realization + extra


# ---------------------------------------------------------------------------
# initial conditions
def gaussian_ic(dim: int, nx: int, nv: int, dx: float, dv: float,
                ny: int = 1, sigma0: float = 1.0, dtype=np.float32):
    """f0(x, v) proportional to exp(-|v|^2 / (2 sigma0^2)), uniform in x,
    normalised in FP64 to unit mass, then rounded to ``dtype``."""
    h = (nv - 1) // 2
    v = (np.arange(nv) - h) * dv
    g = np.exp(-v * v / (2.0 * sigma0 * sigma0))
    if dim == 1:
        f = np.repeat(g[:, None], nx, axis=1)
        w = dx * dv
    else:
        gg = (g[:, None] * g[None, :]).reshape(nv * nv)  # [jy*nv + jx]
        f = np.repeat(gg[:, None], ny * nx, axis=1).reshape(nv * nv, ny, nx)
        w = dx * dx * dv * dv
    f = f / (f.sum(dtype=np.float64) * w)
    return np.ascontiguousarray(f.astype(dtype))


def random_state(rng: np.random.Generator, shape, dtype=np.float32,
                 power: float = 2.0):
    """Non-negative random state (for parity tests): U(0,1)^power."""
    return np.ascontiguousarray((rng.random(shape) ** power).astype(dtype))


# ---------------------------------------------------------------------------
# 1D random Fourier flows
def _mode_sigmas(kmodes: np.ndarray, spectrum: str) -> np.ndarray:
    if spectrum == "k-1":          # amplitude std proportional to 1/k
        s = 1.0 / kmodes
    elif spectrum == "k-5/3":      # amplitude variance proportional to k^-5/3
        s = kmodes ** (-5.0 / 6.0)
    elif spectrum == "flat":
        s = np.ones_like(kmodes, dtype=float)
    else:
        raise ValueError(spectrum)
    # each mode has a cos and a sin amplitude; per-point variance of u is
    # sum_k sigma_k^2 (cos^2 + sin^2 average) = sum_k sigma_k^2
    return s / np.sqrt(np.sum(s * s))


def flow1d(nx: int, L: float, nslices: int, *, modes: int = 8,
           spectrum: str = "k-1", urms: float = 1.0, renew: int | None = None,
           tau_f: float | None = None, dt: float = 1.0, seed: int = 0,
           dtype=np.float32):
    """u[slice, 1, nx] for a 1D random Fourier flow.

    ``renew``: consecutive slices are independent draws (each slice is held
    for ``renew`` steps by the caller through u_hold).  ``tau_f``: slices
    are consecutive times dt apart of an OU evolution (Eq. 7)."""
    rng = np.random.default_rng(seed)
    k = np.arange(1, modes + 1, dtype=float)
    sig = urms * _mode_sigmas(k, spectrum)
    x = np.arange(nx) * (L / nx)
    ph = 2.0 * np.pi * np.outer(k, x) / L  # [modes, nx]
    C, S = np.cos(ph), np.sin(ph)
    a = sig * rng.standard_normal(modes)
    b = sig * rng.standard_normal(modes)
    out = np.empty((nslices, 1, nx), dtype=np.float64)
    if tau_f is not None:
        rho = np.exp(-dt / tau_f)
        q = np.sqrt(1.0 - rho * rho)
    for s in range(nslices):
        if s > 0:
            if tau_f is not None:
                a = rho * a + sig * q * rng.standard_normal(modes)
                b = rho * b + sig * q * rng.standard_normal(modes)
            else:
                a = sig * rng.standard_normal(modes)
                b = sig * rng.standard_normal(modes)
        out[s, 0] = a @ C + b @ S
    return np.ascontiguousarray(out.astype(dtype))


# ---------------------------------------------------------------------------
# 2D incompressible flows
def flow2d_streamfunction(n: int, L: float, nslices: int, *, kmin: int = 1,
                          kmax: int = 32, slope: float = -3.0,
                          urms: float = 1.0, tau_f: float = 1.0,
                          dt: float = 1.0, seed: int = 0, dtype=np.float32):
    """u[slice, 2, n, n] = (d_y psi, -d_x psi) for a random streamfunction
    with energy shell spectrum E(k) ~ k^slope on kmin <= |k| <= kmax and OU
    time evolution (correlation time tau_f) of every Fourier mode."""
    rng = np.random.default_rng(seed)
    kx = np.fft.rfftfreq(n, d=1.0 / n)          # 0..n/2
    ky = np.fft.fftfreq(n, d=1.0 / n)           # 0..n/2-1, -n/2..-1
    KX, KY = np.meshgrid(kx, ky)                # [n, n//2+1]
    K = np.sqrt(KX * KX + KY * KY)
    band = (K >= kmin) & (K <= kmax)
    # E(k) dk = sum over the shell of |k|^2 |psi_k|^2 / 2; the shell holds
    # ~2 pi k modes, so <|psi_k|^2> ~ E(k) / (k^3)
    var = np.zeros_like(K)
    var[band] = K[band] ** slope / (K[band] ** 3)
    amp = np.sqrt(var)
    shape = K.shape

    def draw():
        return amp * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))

    psi_hat = draw()
    rho = np.exp(-dt / tau_f)
    q = np.sqrt(1.0 - rho * rho)
    k2pi = 2.0 * np.pi / L
    out = np.empty((nslices, 2, n, n), dtype=np.float64)
    for s in range(nslices):
        if s > 0:
            psi_hat = rho * psi_hat + q * draw()
        ux = np.fft.irfft2(1j * KY * k2pi * psi_hat, s=(n, n))
        uy = np.fft.irfft2(-1j * KX * k2pi * psi_hat, s=(n, n))
        out[s, 0] = ux
        out[s, 1] = uy
    # ensemble normalisation: the stationary per-component variance is the
    # same for every slice; scale by the measured r.m.s. over all slices
    r = np.sqrt(0.5 * (np.mean(out[:, 0] ** 2) + np.mean(out[:, 1] ** 2)))
    out *= urms / r
    return np.ascontiguousarray(out.astype(dtype))


def cellular_flow(n: int, L: float, U: float = 1.0, dtype=np.float32):
    """Tilted cellular flow of Sec. 4.1: psi = U sin(pi(x+y)/L)
    sin(pi(x-y)/L), u = (d_y psi, -d_x psi); one slice [1, 2, n, n]."""
    x = np.arange(n) * (L / n)
    X, Y = np.meshgrid(x, x)  # [y, x]
    a, b = np.pi * (X + Y) / L, np.pi * (X - Y) / L
    k = np.pi / L
    dpsi_dx = U * k * (np.cos(a) * np.sin(b) + np.sin(a) * np.cos(b))
    dpsi_dy = U * k * (np.cos(a) * np.sin(b) - np.sin(a) * np.cos(b))
    u = np.stack([dpsi_dy, -dpsi_dx])[None]
    return np.ascontiguousarray(u.astype(dtype))


def choose_vmax(nx: int, L: float, nv: int, tau_p: float, umax: float,
                cfl_target: float = 0.45, quantum: float = 0.5) -> float:
    """Smallest multiple of ``quantum`` for Vmax such that the drift CFL of
    Eq. 3, (dt/dv)(umax + Vmax)/tau_p with dt = dx/dv and dv = Vmax/h,
    stays below cfl_target."""
    h = (nv - 1) // 2
    dx = L / nx
    v = quantum
    while True:
        dv = v / h
        dt = dx / dv
        if (dt / dv) * (umax + v) / tau_p <= cfl_target:
            return v
        v += quantum
