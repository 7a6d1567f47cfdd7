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


def flow1d_modes(nslices: int, *, modes: int = 8, spectrum: str = "k-1",
                 urms: float = 1.0, renew: int | None = None,
                 tau_f: float | None = None, dt: float = 1.0, seed: int = 0):
    """Mode table [slice, mode, 2] (FP64) of a 1D random Fourier flow:
    u(x) = sum_k a_k cos(2 pi k x / L) + b_k sin(2 pi k x / L), k = 1..modes.

    ``renew``: consecutive slices are independent draws (each slice is held
    for ``renew`` steps by the caller through u_hold).  ``tau_f``: slices
    are consecutive times dt apart of an OU evolution (Eq. 7)."""
    rng = np.random.default_rng(seed)
    k = np.arange(1, modes + 1, dtype=float)
    sig = urms * _mode_sigmas(k, spectrum)
    a = sig * rng.standard_normal(modes)
    b = sig * rng.standard_normal(modes)
    out = np.empty((nslices, modes, 2))
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
        out[s, :, 0] = a
        out[s, :, 1] = b
    return out


def flow1d(nx: int, L: float, nslices: int, *, modes: int = 8,
           spectrum: str = "k-1", urms: float = 1.0, renew: int | None = None,
           tau_f: float | None = None, dt: float = 1.0, seed: int = 0,
           dtype=np.float32):
    """u[slice, 1, nx] of the flow1d_modes table (prestaged form)."""
    tab = flow1d_modes(nslices, modes=modes, spectrum=spectrum, urms=urms,
                       renew=renew, tau_f=tau_f, dt=dt, seed=seed)
    k = np.arange(1, modes + 1, dtype=float)
    x = np.arange(nx) * (L / nx)
    ph = 2.0 * np.pi * np.outer(k, x) / L  # [modes, nx]
    C, S = np.cos(ph), np.sin(ph)
    out = (tab[:, :, 0] @ C + tab[:, :, 1] @ S)[:, None, :]
    return np.ascontiguousarray(out.astype(dtype))


# ---------------------------------------------------------------------------
# 2D incompressible flows
def _psi_hat_slices(n: int, nslices: int, kmin: int, kmax: int, slope: float,
                    tau_f: float, dt: float, seed: int):
    """Streamfunction Fourier amplitudes on the rfft grid [n, n//2+1], one
    array per slice: energy shell spectrum E(k) ~ k^slope on kmin <= |k| <=
    kmax, every mode an OU process in time (correlation time tau_f)."""
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
    for s in range(nslices):
        if s > 0:
            psi_hat = rho * psi_hat + q * draw()
        yield KX, KY, psi_hat


def _mean_square(A):
    """Grid mean of f = sum Re(A e^{i theta}) over a table with kx >= 0
    (rows ky = -K..K, columns kx = 0..K), by Parseval: kx >= 1 modes give
    |A|^2 / 2; the kx = 0 column pairs (ky, -ky) give |A_ky + conj A_-ky|^2
    / 2 for ky > 0."""
    K = A.shape[1] - 1
    ms = 0.5 * np.sum(np.abs(A[:, 1:]) ** 2)
    col = A[:, 0]
    for ky in range(1, K + 1):
        ms += 0.5 * abs(col[K + ky] + np.conj(col[K - ky])) ** 2
    return ms


def flow2d_modes(n: int, L: float, nslices: int, *, kmin: int = 1,
                 kmax: int = 32, slope: float = -3.0, urms: float = 1.0,
                 tau_f: float = 1.0, dt: float = 1.0, seed: int = 0):
    """Streamfunction mode table c[slice, ky + kmax, kx, 2] (FP32, re/im;
    ky = -kmax..kmax, kx = 0..kmax) with psi(ix, iy) = sum Re(c
    e^{2 pi i (kx ix + ky iy)/n}); u = (d_y psi, -d_x psi) has per-component
    r.m.s. urms over all slices.  Same random draws as
    flow2d_streamfunction (which evaluates this table on the grid)."""
    K = kmax
    assert 2 * K < n
    tab = np.empty((nslices, 2 * K + 1, K + 1), dtype=np.complex128)
    rows = np.r_[np.arange(n - K, n), np.arange(0, K + 1)]  # ky = -K..K
    w = np.full(K + 1, 2.0)
    w[0] = 1.0  # the kx = 0 column is counted once (real part)
    k2pi = 2.0 * np.pi / L
    kxv = np.arange(K + 1, dtype=float)
    kyv = np.arange(-K, K + 1, dtype=float)
    msum = 0.0
    for s, (_, _, ph) in enumerate(_psi_hat_slices(n, nslices, kmin, kmax,
                                                   slope, tau_f, dt, seed)):
        c = ph[rows][:, :K + 1] * (w / (n * n))
        tab[s] = c
        ax = 1j * k2pi * kyv[:, None] * c
        ay = -1j * k2pi * kxv[None, :] * c
        msum += 0.5 * (_mean_square(ax) + _mean_square(ay))
    r = np.sqrt(msum / nslices)
    tab *= urms / r
    out = np.empty(tab.shape + (2,), dtype=np.float32)
    out[..., 0] = tab.real
    out[..., 1] = tab.imag
    return out


def flow2d_streamfunction(n: int, L: float, nslices: int, *, kmin: int = 1,
                          kmax: int = 32, slope: float = -3.0,
                          urms: float = 1.0, tau_f: float = 1.0,
                          dt: float = 1.0, seed: int = 0, dtype=np.float32,
                          norm_slices: int | None = None):
    """u[slice, 2, n, n] = (d_y psi, -d_x psi) for a random streamfunction
    with energy shell spectrum E(k) ~ k^slope on kmin <= |k| <= kmax and OU
    time evolution (correlation time tau_f) of every Fourier mode
    (prestaged form of flow2d_modes, evaluated with inverse real FFTs).
    The r.m.s. that sets the scale is taken over the first norm_slices
    slices (all of them by default), so that a longer flow with a fixed
    norm_slices starts with the same slices as a shorter one."""
    k2pi = 2.0 * np.pi / L
    out = np.empty((nslices, 2, n, n), dtype=np.float64)
    for s, (KX, KY, psi_hat) in enumerate(_psi_hat_slices(
            n, nslices, kmin, kmax, slope, tau_f, dt, seed)):
        out[s, 0] = np.fft.irfft2(1j * KY * k2pi * psi_hat, s=(n, n))
        out[s, 1] = np.fft.irfft2(-1j * KX * k2pi * psi_hat, s=(n, n))
    # ensemble normalisation: the stationary per-component variance is the
    # same for every slice; scale by the r.m.s. over the leading slices
    m = nslices if norm_slices is None else norm_slices
    if not 1 <= m <= nslices:
        raise ValueError("norm_slices must be in 1..nslices")
    r = np.sqrt(0.5 * (np.mean(out[:m, 0] ** 2) + np.mean(out[:m, 1] ** 2)))
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
