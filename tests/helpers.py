"""Shared helpers for the GPU parity tests (inputs, runners, norms)."""
from __future__ import annotations

import math
import sys

import numpy as np

from paper_1508_02899_amd import inputs

FP32_REL_L2 = 1e-5   # parity bound for FP32 state vs the FP64 oracle
FP64_REL_L2 = 1e-12  # parity bound for FP64 state vs the FP64 oracle


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def make_case(dim, nx, nv, *, ny=1, dtype="f32", seed=0, slices=1, s=1,
              cfl=0.4, scheme="koren", nsub=1, umax=1.0, kappa_frac=0.2,
              L=2 * math.pi):
    """A seeded random state and flow with drift CFL ~ cfl and diffusion
    number ~ kappa_frac * 1/2.  Returns (f0, u, params) with numpy arrays in
    the library layouts and the dtype of the state."""
    rng = np.random.default_rng(seed)
    npdt = np.float64 if dtype == "f64" else np.float32
    shape = (nv, nx) if dim == 1 else (nv * nv, ny, nx)
    f0 = inputs.random_state(rng, shape, npdt)
    ushape = (slices, 1, nx) if dim == 1 else (slices, 2, ny, nx)
    u = (umax * np.tanh(rng.standard_normal(ushape))).astype(npdt)
    dx = L / nx
    h = (nv - 1) // 2
    dt = 0.05
    dv = s * dx / dt
    vmax = h * dv
    dts = dt / nsub
    # CFL = (dts/dv)(umax + vmax)/tau_p  ->  tau_p
    tau_p = (dts / dv) * (umax + vmax) / cfl
    kappa = kappa_frac * 0.5 * dv * dv / dts
    return f0, u, dict(dim=dim, dx=dx, dt=dt, tau_p=tau_p, kappa=kappa,
                       s=s, nsub=nsub, scheme=scheme)


def run_oracle(f0, u, p, nsteps, u_hold=0):
    import oracle
    return oracle.step(f0.astype(np.float64), u.astype(np.float64),
                       dim=p["dim"], dx=p["dx"], tau_p=p["tau_p"],
                       kappa=p["kappa"], dt=p["dt"], nsteps=nsteps,
                       scheme=p["scheme"], s=p["s"], nsub=p["nsub"],
                       u_hold=u_hold)


def spec_for(f0, p, dtype, u_hold=0):
    from paper_1508_02899_amd import LatticeSpec
    if p["dim"] == 1:
        nv, nx = f0.shape
        ny = 1
    else:
        nvv, ny, nx = f0.shape
        nv = int(round(nvv ** 0.5))
    return LatticeSpec(dim=p["dim"], nx=nx, ny=ny, nv=nv, dx=p["dx"],
                       vstride=p["s"], scheme=p["scheme"], dtype=dtype,
                       nsub=p["nsub"], u_hold=u_hold)


def run_gpu(f0, u, p, nsteps, dtype="f32", u_hold=0, lat=None):
    import torch
    from paper_1508_02899_amd import Lattice
    spec = spec_for(f0, p, dtype, u_hold)
    own = lat is None
    if own:
        lat = Lattice(spec)
    f = torch.from_numpy(np.ascontiguousarray(f0)).cuda()
    ut = torch.from_numpy(np.ascontiguousarray(u)).cuda()
    lat.step(f, ut, p["tau_p"], p["kappa"], p["dt"], nsteps)
    lat.sync()
    out = f.cpu().numpy()
    if own:
        lat.close()
    return out
