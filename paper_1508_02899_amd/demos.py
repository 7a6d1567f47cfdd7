"""Paper-style demonstration runs on the GPU lattice.

* Tilted cellular flow (Sec. 4.1): psi = U sin(pi(x+y)/L) sin(pi(x-y)/L),
  St = tau_p U / L, dimensionless diffusivity K = kappa L / U^3 (the
  definition of Sec. 3 with the flow's own scales).  Particles relax onto a
  stationary distribution concentrated along the separatrices between the
  cells (small St) or on ballistic trajectories across them (larger St).

Only library calls are sequenced here (flow, steps, density, statistics).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

from .lattice import Lattice, LatticeSpec
from . import inputs


@dataclass
class CellularRun:
    spec: LatticeSpec
    u: object          # flow slice [1, 2, n, n] (device)
    tau_p: float
    kappa: float
    dt: float
    dv: float


def cellular_setup(n: int = 256, nv: int = 19, St: float = 1 / (2 * math.pi),
                   K: float = 8 * math.pi * 1e-3, L: float = 2 * math.pi,
                   U: float = 1.0, vmax: float = 1.5,
                   scheme: str = "koren") -> CellularRun:
    """Lattice, flow and parameters of the cellular-flow run; the number of
    collision sub-steps is chosen for the drift CFL bound of Eq. 3."""
    import torch
    u = torch.from_numpy(inputs.cellular_flow(n, L, U)).cuda()
    tau_p = St * L / U
    kappa = K * U ** 3 / L
    dx = L / n
    dv = vmax / ((nv - 1) // 2)
    dt = dx / dv
    base = LatticeSpec(dim=2, nx=n, ny=n, nv=nv, dx=dx, scheme=scheme)
    lat = Lattice(base)
    cfl, dnum = lat.stability(u, tau_p, kappa, dt)
    lat.close()
    bound = 0.45 if scheme == "koren" else 0.9
    nsub = max(1, math.ceil(cfl / bound), math.ceil(dnum / 0.45))
    spec = LatticeSpec(dim=2, nx=n, ny=n, nv=nv, dx=dx, scheme=scheme,
                       nsub=nsub)
    return CellularRun(spec, u, tau_p, kappa, dt, dv)


def cellular_run(run: CellularRun, time: float, sigma0: float = 0.3,
                 levels: int = 6):
    """Evolve a uniform-in-space, Gaussian-in-velocity (sigma0) state for
    the given physical time; returns (f, density rho [n, n], <rho_r^2>
    for r = 2^k dx, k < levels, S1 at r = 2^k dx)."""
    import torch
    s = run.spec
    f = torch.from_numpy(inputs.gaussian_ic(2, s.nx, s.nv, s.dx, run.dv,
                                            ny=s.ny, sigma0=sigma0)).cuda()
    lat = Lattice(s)
    steps = max(1, int(round(time / run.dt)))
    lat.step(f, run.u, run.tau_p, run.kappa, run.dt, steps)
    lat.sync()
    rho = lat.density(f, run.dt)
    r2 = lat.rho_r2(rho, levels)
    s1 = lat.s1(f, run.dt, [2 ** k for k in range(levels)])
    lat.close()
    return f, rho, r2, s1
