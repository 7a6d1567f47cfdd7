"""FP64 oracle of the Eulerian velocity structure function -- TEST
INFRASTRUCTURE ONLY (tests/ may import it; the GPU library never does).

S1(r) of Eq. 11 (Sec. 3.1), written out from its definition: the x-average
of sum_{v, v'} f(x, v) f(x + r, v') |v - v'| over the x-average of
sum_{v, v'} f(x, v) f(x + r, v'), with periodic x.  1D: r along x.  2D:
|v - v'| is the Euclidean norm; the separations r e_x and r e_y are
averaged (a reading: the lattice axes stand in for the isotropic average).
"""
from __future__ import annotations

import numpy as np


def velocities(nv: int, dv: float) -> np.ndarray:
    return (np.arange(nv) - (nv - 1) // 2) * dv


def s1(f: np.ndarray, dim: int, dv: float, rs) -> np.ndarray:
    f = np.asarray(f, dtype=np.float64)
    if dim == 1:
        nv = f.shape[0]
        v = velocities(nv, dv)
        A = np.abs(v[:, None] - v[None, :])
        out = []
        for r in rs:
            g = np.roll(f, -int(r), axis=1)       # g[:, x] = f[:, x + r]
            num = np.einsum("jx,jk,kx->", f, A, g)
            den = np.sum(f.sum(axis=0) * g.sum(axis=0))
            out.append(num / den)
        return np.array(out)
    nv = int(round(np.sqrt(f.shape[0])))
    v = velocities(nv, dv)
    VX = np.tile(v, nv)          # plane J = jy * nv + jx
    VY = np.repeat(v, nv)
    A = np.sqrt((VX[:, None] - VX[None, :]) ** 2 + (VY[:, None] - VY[None, :]) ** 2)
    F = f.reshape(nv * nv, -1)
    out = []
    for r in rs:
        est = []
        for axis in (2, 1):     # x, then y
            g = np.roll(f, -int(r), axis=axis).reshape(nv * nv, -1)
            num = np.einsum("js,jk,ks->", F, A, g)
            den = np.sum(F.sum(axis=0) * g.sum(axis=0))
            est.append(num / den)
        out.append(0.5 * (est[0] + est[1]))
    return np.array(out)
