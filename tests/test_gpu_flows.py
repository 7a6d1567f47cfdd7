"""Flow synthesis on the GPU from mode tables vs the FP64 oracle
(oracle/flows.py), and lattice steps driven by device-synthesised flows
vs the same steps with prestaged flows."""
import math

import numpy as np
import pytest

from helpers import rel_l2, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype,nx,K,ns", [("f32", 1000, 32, 7),
                                           ("f64", 256, 8, 3)])
def test_flow1d_modes_match_oracle(dtype, nx, K, ns):
    import torch
    from oracle import flows as F
    from paper_1508_02899_amd import Lattice, LatticeSpec, inputs
    tab = inputs.flow1d_modes(ns, modes=K, spectrum="k-5/3", tau_f=1.0,
                              dt=0.1, seed=21).astype(np.float32)
    lat = Lattice(LatticeSpec(dim=1, nx=nx, nv=9, dx=2 * math.pi / nx,
                              dtype=dtype))
    u = lat.flow_from_modes(torch.from_numpy(tab).cuda()).cpu().numpy()
    want = F.flow1d(tab, nx)
    err = rel_l2(u, want)
    say(f"  1D {dtype}: rel L2 {err:.2e}")
    assert err < (2e-6 if dtype == "f32" else 1e-12)
    lat.close()


@pytest.mark.parametrize("dtype,nx,ny,K,ns", [("f32", 96, 64, 16, 3),
                                              ("f32", 512, 512, 32, 1),
                                              ("f64", 40, 48, 8, 2)])
def test_flow2d_modes_match_oracle(dtype, nx, ny, K, ns):
    import torch
    from oracle import flows as F
    from paper_1508_02899_amd import Lattice, LatticeSpec
    rng = np.random.default_rng(22 + nx)
    tab = rng.standard_normal((ns, 2 * K + 1, K + 1, 2)).astype(np.float32)
    dx = 0.05
    lat = Lattice(LatticeSpec(dim=2, nx=nx, ny=ny, nv=3, dx=dx, dtype=dtype))
    u = lat.flow_from_modes(torch.from_numpy(tab).cuda()).cpu().numpy()
    want = F.flow2d(tab, nx, ny, dx)
    err = rel_l2(u, want)
    say(f"  2D {dtype} {nx}x{ny} K={K}: rel L2 {err:.2e}")
    assert err < (5e-6 if dtype == "f32" else 1e-12)
    lat.close()


def test_steps_with_device_flow_match_prestaged_flow():
    """2D Koren steps driven by flows synthesised on the device equal the
    steps driven by the prestaged inverse-FFT flows up to the FP32 rounding
    of u."""
    import torch
    from paper_1508_02899_amd import Lattice, LatticeSpec, inputs
    n, nv, L, steps = 64, 17, 2 * math.pi, 20
    dx = L / n
    dv = 3.0 / ((nv - 1) // 2)
    dt = dx / dv
    kw = dict(kmax=16, tau_f=1.0, dt=dt, seed=inputs.seed_for(3, 9))
    u_pre = torch.from_numpy(inputs.flow2d_streamfunction(n, L, steps, **kw)).cuda()
    tab = torch.from_numpy(inputs.flow2d_modes(n, L, steps, **kw)).cuda()
    spec = LatticeSpec(dim=2, nx=n, ny=n, nv=nv, dx=dx, u_hold=1)
    lat = Lattice(spec)
    u_dev = lat.flow_from_modes(tab)
    du = rel_l2(u_dev.cpu().numpy(), u_pre.cpu().numpy())
    f0 = torch.from_numpy(inputs.gaussian_ic(2, n, nv, dx, dv, ny=n)).cuda()
    a, b = f0.clone(), f0.clone()
    lat.step(a, u_pre, 4 * math.pi, 1e-4, dt, steps)
    lat.step(b, u_dev, 4 * math.pi, 1e-4, dt, steps)
    lat.sync()
    err = rel_l2(b.cpu().numpy(), a.cpu().numpy())
    say(f"  u rel L2 {du:.2e}; state after {steps} steps rel L2 {err:.2e}")
    assert du < 1e-6 and err < 1e-5
    lat.close()
