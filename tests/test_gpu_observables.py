"""GPU <rho_r^2> on tilings vs the FP64 oracle (oracle/observables.py)."""
import math

import numpy as np
import pytest

from helpers import say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dim,nx,ny,levels", [(2, 64, 32, 6), (2, 48, 16, 4),
                                              (1, 1024, 1, 11), (2, 8, 8, 1)])
def test_rho_r2_matches_oracle(dim, nx, ny, levels):
    import torch
    from oracle import observables as O
    from paper_1508_02899_amd import Lattice, LatticeSpec
    rng = np.random.default_rng(60 + nx)
    nv = 9
    shape = (nv ** dim, ny, nx) if dim == 2 else (nv, nx)
    f = (rng.random(shape) ** 4).astype(np.float32)
    dx = 2 * math.pi / nx
    dt = 0.1
    lat = Lattice(LatticeSpec(dim=dim, nx=nx, ny=ny, nv=nv, dx=dx))
    fd = torch.from_numpy(f).cuda()
    rho = lat.density(fd, dt)
    got = lat.rho_r2(rho, levels)
    dv = dx / dt
    want = O.rho_r2(O.density(f, dim, dv).reshape(ny, nx), levels)
    say(f"  <rho_r^2> {np.round(got, 4)}")
    assert np.allclose(got, want, rtol=1e-12, atol=0)
    # bit-reproducible
    assert np.array_equal(got, lat.rho_r2(rho, levels))
    lat.close()


def test_rho_r2_rejects_bad_tiling():
    import torch
    from paper_1508_02899_amd import Lattice, LatticeSpec, LatticeError
    lat = Lattice(LatticeSpec(dim=2, nx=24, ny=16, nv=3, dx=0.1))
    rho = torch.ones((16, 24), dtype=torch.float64, device="cuda")
    assert lat.rho_r2(rho, 4)[0] == pytest.approx(1.0)
    with pytest.raises(LatticeError):
        lat.rho_r2(rho, 5)  # 24 is not a multiple of 16
    lat.close()
