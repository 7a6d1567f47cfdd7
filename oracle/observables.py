"""FP64 oracle of the density observables -- TEST INFRASTRUCTURE ONLY.

Only tests/ (and the benchmark's CPU baseline) may import this module; the
GPU library never does.  Plain numpy in double precision.

* Coarse-grained density (Sec. 3.1: mass in a window of size r; Sec. 3.2:
  evaluated on a tiling with boxes of size r) and its second moment
  <rho_r^2> (Sec. 4.2.1), normalised so that <rho_r> = 1:
  rho_r = (m_b / M) N_b, <rho_r^2> = N_b sum_b m_b^2 / M^2.
* The distance-averaged relative error of Sec. 4.2.1 (Eq. for E(N_v,
  V_max)): the r-weighted mean of |<rho_r^2>_A - <rho_r^2>_B| over the
  r-weighted mean of <rho_r^2>_B, with the integral over r taken as a
  sum over the tiling scales r = 2^k dx with weight r dr, dr = r (a
  log-spaced grid), i.e. weight r^2.
"""
from __future__ import annotations

import numpy as np


def density(f: np.ndarray, dim: int, dv: float) -> np.ndarray:
    """rho(x) = dv^dim sum_j f(x, v_j); f [nv^dim, (ny,) nx]."""
    f = np.asarray(f, dtype=np.float64)
    return f.sum(axis=0) * dv ** dim


def rho_r2(rho: np.ndarray, levels: int) -> np.ndarray:
    """<rho_r^2> for boxes of 2^k sites per direction, k = 0..levels-1."""
    rho = np.asarray(rho, dtype=np.float64)
    if rho.ndim == 1:
        rho = rho[None, :]
        dim = 1
    else:
        dim = 2 if rho.shape[0] > 1 else 1
    ny, nx = rho.shape
    out = np.empty(levels)
    for k in range(levels):
        b = 2 ** k
        by = b if dim == 2 else 1
        assert nx % b == 0 and ny % by == 0
        m = rho.reshape(ny // by, by, nx // b, b).sum(axis=(1, 3))
        nb = m.size
        out[k] = nb * np.sum(m * m) / np.sum(m) ** 2
    return out


def distance_averaged_error(a: np.ndarray, b: np.ndarray, dx: float) -> float:
    """Relative error of <rho_r^2>_A against <rho_r^2>_B over the scales
    r_k = 2^k dx (weights r_k^2, see the module docstring)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    r = dx * 2.0 ** np.arange(len(a))
    w = r * r
    return float(np.sum(w * np.abs(a - b)) / np.sum(w * np.abs(b)))
