"""FP64 oracle of the flow synthesis from mode tables -- TEST
INFRASTRUCTURE ONLY (tests/ may import it; the GPU library never does).

Direct evaluation of the Fourier sums at the lattice sites, in double
precision, with the angles 2 pi k j / n formed from integers:
* 1D random Fourier flow (Sec. 3): u(x_j) = sum_k a_k cos(2 pi k j/nx)
  + b_k sin(2 pi k j/nx), k = 1..K;
* 2D streamfunction flow (Sec. 4): psi = sum Re(c e^{2 pi i (kx ix/nx +
  ky iy/ny)}), u = (d psi/dy, -d psi/dx) on a domain nx dx by ny dx.
"""
from __future__ import annotations

import numpy as np


def _angle(k, j, n):
    return 2.0 * np.pi * (np.outer(k, j) % n) / n


def flow1d(tab: np.ndarray, nx: int) -> np.ndarray:
    """tab [slices, K, 2] -> u [slices, 1, nx]."""
    tab = np.asarray(tab, dtype=np.float64)
    K = tab.shape[1]
    th = _angle(np.arange(1, K + 1), np.arange(nx), nx)  # [K, nx]
    u = tab[:, :, 0] @ np.cos(th) + tab[:, :, 1] @ np.sin(th)
    return u[:, None, :]


def flow2d(tab: np.ndarray, nx: int, ny: int, dx: float) -> np.ndarray:
    """tab [slices, 2K+1, K+1, 2] -> u [slices, 2, ny, nx]."""
    tab = np.asarray(tab, dtype=np.float64)
    c = tab[..., 0] + 1j * tab[..., 1]
    ns, nky, nkx = c.shape
    K = nkx - 1
    gx = 2.0 * np.pi / (nx * dx)
    gy = 2.0 * np.pi / (ny * dx)
    ex = np.exp(1j * _angle(np.arange(nkx), np.arange(nx), nx))        # [kx, x]
    ey = np.exp(1j * _angle(np.arange(-K, K + 1), np.arange(ny), ny))  # [ky, y]
    kx = np.arange(nkx)
    ky = np.arange(-K, K + 1)
    u = np.empty((ns, 2, ny, nx))
    for s in range(ns):
        # sum over (ky, kx) of a(ky, kx) e^{i ky y} e^{i kx x}
        ax = 1j * gy * ky[:, None] * c[s]
        ay = -1j * gx * kx[None, :] * c[s]
        u[s, 0] = np.real(ey.T @ ax @ ex)
        u[s, 1] = np.real(ey.T @ ay @ ex)
    return u
