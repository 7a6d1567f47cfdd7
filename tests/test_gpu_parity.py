"""GPU parity: the HIP lattice update against the FP64 oracle.

Same seeded inputs on both sides (the oracle gets the FP32-rounded values
cast to FP64).  Bounds: relative L2 <= 1e-5 for FP32 state, <= 1e-12 for
FP64 state, bit-exact for pure streaming.  Sizes span several tiles and a
ragged tail (nx not a multiple of the 256-lane block or of the 2D
wavefront tile).
"""
import math

import numpy as np
import pytest

from helpers import (FP32_REL_L2, FP64_REL_L2, make_case, rel_l2, run_gpu,
                     run_oracle, say)

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nv", [3, 5, 9, 17, 33, 65, 129])
@pytest.mark.parametrize("scheme", ["koren", "upwind"])
def test_1d_f32_parity(nv, scheme):
    say(f"1d f32 nv={nv} {scheme}")
    f0, u, p = make_case(1, 300, nv, seed=nv, scheme=scheme)
    got = run_gpu(f0, u, p, 12)
    want = run_oracle(f0, u, p, 12)
    err = rel_l2(got, want)
    say("  rel L2", err)
    assert err <= FP32_REL_L2


@pytest.mark.parametrize("nx,nv", [(1, 17), (7, 33), (31, 65), (45, 129),
                                   (64, 33), (65, 17), (1000, 129)])
def test_1d_split_column_short_and_ragged(nx, nv):
    """The split-column 1D pass on lattices shorter than one workgroup's
    sites and with ragged tails; nsub = 3 and stride 4 on the way."""
    say(f"1d split-column nx={nx} nv={nv}")
    f0, u, p = make_case(1, nx, nv, seed=300 + nx + nv, slices=2, s=4,
                         nsub=3)
    got = run_gpu(f0, u, p, 6, u_hold=3)
    want = run_oracle(f0, u, p, 6, u_hold=3)
    err = rel_l2(got, want)
    say("  rel L2", err)
    assert err <= FP32_REL_L2


@pytest.mark.parametrize("scheme", ["koren", "upwind"])
def test_1d_long_lattice_one_lane_per_site(scheme):
    """Past 2^19 sites the 1D pass gives each site one lane (the whole
    column in registers); nx = 2^19 + 37 with 33 velocities."""
    nx = (1 << 19) + 37
    say(f"1d one-lane-per-site nx={nx} nv=33 {scheme}")
    f0, u, p = make_case(1, nx, 33, seed=401, scheme=scheme)
    got = run_gpu(f0, u, p, 3)
    want = run_oracle(f0, u, p, 3)
    err = rel_l2(got, want)
    say("  rel L2", err)
    assert err <= FP32_REL_L2


@pytest.mark.parametrize("nv", [3, 9, 17, 33, 65])
@pytest.mark.parametrize("scheme", ["koren", "upwind"])
def test_1d_f64_parity(nv, scheme):
    say(f"1d f64 nv={nv} {scheme}")
    f0, u, p = make_case(1, 257, nv, seed=100 + nv, dtype="f64", scheme=scheme)
    got = run_gpu(f0, u, p, 10, dtype="f64")
    want = run_oracle(f0, u, p, 10)
    assert rel_l2(got, want) <= FP64_REL_L2


def test_1d_f64_256x33_1000_steps_renewed_flow():
    """1D periodic 256 x 33 in FP64, random 8-mode flow renewed every 50
    steps (u_hold = 50), St = 1, kappa = 1e-3, 1000 steps, Koren."""
    from paper_1508_02899_amd import inputs
    say("1d f64 256x33, 1000 steps, u_hold 50")
    nx, nv, L = 256, 33, 2 * math.pi
    nsteps, hold = 1000, 50
    u = inputs.flow1d(nx, L, nsteps // hold, modes=8, spectrum="k-1",
                      renew=hold, seed=inputs.seed_for(1), dtype=np.float64)
    tau_p = 1.0 * L  # St = tau_p u_rms / L = 1
    vmax = 5.0
    h = (nv - 1) // 2
    dv = vmax / h
    dx = L / nx
    dt = dx / dv
    f0 = inputs.gaussian_ic(1, nx, nv, dx, dv, dtype=np.float64)
    p = dict(dim=1, dx=dx, dt=dt, tau_p=tau_p, kappa=1e-3, s=1, nsub=1,
             scheme="koren")
    got = run_gpu(f0, u, p, nsteps, dtype="f64", u_hold=hold)
    want = run_oracle(f0, u, p, nsteps, u_hold=hold)
    err = rel_l2(got, want)
    say("  rel L2", err)
    assert err <= FP64_REL_L2


@pytest.mark.parametrize("nv", [3, 5, 7, 9, 11, 13, 15, 17, 19, 21, 25, 33])
def test_2d_f32_parity_koren(nv):
    say(f"2d f32 nv={nv} koren")
    f0, u, p = make_case(2, 70, nv, ny=9, seed=200 + nv)
    got = run_gpu(f0, u, p, 4)
    want = run_oracle(f0, u, p, 4)
    err = rel_l2(got, want)
    say("  rel L2", err)
    assert err <= FP32_REL_L2


@pytest.mark.parametrize("nv", [5, 17, 33])
def test_2d_f32_parity_upwind(nv):
    say(f"2d f32 nv={nv} upwind")
    f0, u, p = make_case(2, 45, nv, ny=7, seed=300 + nv, scheme="upwind")
    got = run_gpu(f0, u, p, 4)
    want = run_oracle(f0, u, p, 4)
    assert rel_l2(got, want) <= FP32_REL_L2


def test_2d_f32_parity_nv65():
    say("2d f32 nv=65 koren")
    f0, u, p = make_case(2, 37, 65, ny=5, seed=465)
    got = run_gpu(f0, u, p, 3)
    want = run_oracle(f0, u, p, 3)
    err = rel_l2(got, want)
    say("  rel L2", err)
    assert err <= FP32_REL_L2


def _vy_drift_case(nv, flow, nx, ny, seed, dtype):
    """A state with a chosen vertical flow u_y, which sets where the vy drift
    nu(t) = (dt/tau_p)(u_y/dv - (t - h)) changes sign along the rows t: the
    2D pass skips the split half of that drift that is zero on a whole
    wavefront, in loops chosen by that sign change."""
    from paper_1508_02899_amd import inputs
    rng = np.random.default_rng(seed)
    npdt = np.float64 if dtype == "f64" else np.float32
    f0 = inputs.random_state(rng, (nv * nv, ny, nx), npdt)
    L, dt = 2 * math.pi, 0.05
    dx = L / nx
    h = (nv - 1) // 2
    dv = dx / dt
    vmax = h * dv
    ux = 0.5 * np.tanh(rng.standard_normal((ny, nx)))
    uy = {
        # sign change at a row a little past the middle / before it, the
        # same for every site
        "up": np.full((ny, nx), 0.3 * vmax),
        "down": np.full((ny, nx), -0.3 * vmax),
        # a different row for each wavefront of a workgroup
        "wave": 0.5 * vmax * np.sin(2 * math.pi * np.arange(nx) / nx)
        * np.ones((ny, 1)),
        # past either end of the velocity axis: one half is zero throughout
        "beyond": np.full((ny, nx), 1.2 * vmax),
        "below": np.full((ny, nx), -1.2 * vmax),
        # no drag at all (tau_p infinite): both halves are zero
        "nodrag": np.zeros((ny, nx)),
    }[flow]
    u = np.stack([ux, uy])[None].astype(npdt)
    umax = float(np.abs(u).max())
    tau_p = math.inf if flow == "nodrag" else (dt / dv) * (umax + vmax) / 0.4
    kappa = 0.2 * 0.5 * dv * dv / dt
    p = dict(dim=2, dx=dx, dt=dt, tau_p=tau_p, kappa=kappa, s=1, nsub=1,
             scheme="koren")
    return f0, u, p


@pytest.mark.parametrize("flow", ["up", "down", "wave", "beyond", "below",
                                  "nodrag"])
@pytest.mark.parametrize("nv", [17, 33, 65])
def test_2d_vy_drift_half_skipped_where_zero(nv, flow):
    """Each skip mode of the streamed vy drift, and the moves between them
    at the same or at different rows across the wavefronts of a workgroup,
    against the oracle (which always computes both split halves); 300
    sites per row: several workgroups, interior and edge tiles, a ragged
    tail."""
    ny = 3 if nv == 65 else 4
    say(f"2d vy-drift skip nv={nv} flow={flow}")
    f0, u, p = _vy_drift_case(nv, flow, 300, ny, 700 + nv, "f32")
    got = run_gpu(f0, u, p, 3)
    want = run_oracle(f0, u, p, 3)
    err = rel_l2(got, want)
    say("  rel L2", err)
    assert err <= FP32_REL_L2
    assert np.isfinite(got).all()


@pytest.mark.parametrize("flow", ["up", "wave", "below"])
def test_2d_vy_drift_half_skipped_f64(flow):
    say(f"2d f64 vy-drift skip nv=33 flow={flow}")
    f0, u, p = _vy_drift_case(33, flow, 200, 3, 800, "f64")
    got = run_gpu(f0, u, p, 3, dtype="f64")
    want = run_oracle(f0, u, p, 3)
    assert rel_l2(got, want) <= FP64_REL_L2


@pytest.mark.parametrize("nx,ny,nv", [(1, 1, 9), (1, 5, 33), (7, 1, 17),
                                      (3, 2, 33), (2, 3, 65), (1, 2, 5)])
def test_2d_degenerate_lattices(nx, ny, nv):
    """Lattices of one or a few sites per axis (every streaming shift wraps
    several times; all but a few lanes of a workgroup are duplicates),
    velocity stride 4 and two collision sub-steps."""
    say(f"2d degenerate {nx}x{ny} nv={nv}")
    f0, u, p = make_case(2, nx, nv, ny=ny, seed=600 + 7 * nx + ny + nv,
                         slices=2, s=4, nsub=2)
    got = run_gpu(f0, u, p, 4, u_hold=2)
    want = run_oracle(f0, u, p, 4, u_hold=2)
    err = rel_l2(got, want)
    say("  rel L2", err)
    assert err <= FP32_REL_L2


@pytest.mark.parametrize("nv", [3, 5, 9, 17, 33])
def test_2d_f64_parity(nv):
    say(f"2d f64 nv={nv}")
    f0, u, p = make_case(2, 40, nv, ny=6, seed=500 + nv, dtype="f64")
    got = run_gpu(f0, u, p, 3, dtype="f64")
    want = run_oracle(f0, u, p, 3)
    assert rel_l2(got, want) <= FP64_REL_L2


@pytest.mark.parametrize("dim", [1, 2])
def test_nsub_stride_and_u_hold(dim):
    """nsub = 3 collision sub-steps, velocity stride 4 (coarse lattice),
    three u slices held two steps each."""
    say(f"nsub/stride/u_hold dim={dim}")
    nv = 9
    if dim == 1:
        f0, u, p = make_case(1, 130, nv, seed=7, slices=3, s=4, nsub=3)
    else:
        f0, u, p = make_case(2, 50, nv, ny=11, seed=8, slices=3, s=4, nsub=3)
    got = run_gpu(f0, u, p, 6, u_hold=2)
    want = run_oracle(f0, u, p, 6, u_hold=2)
    err = rel_l2(got, want)
    say("  rel L2", err)
    assert err <= FP32_REL_L2


@pytest.mark.parametrize("dim", [1, 2])
def test_drift_without_diffusion(dim):
    """kappa = 0 is accepted and gives the oracle's drift-only update."""
    nx, ny = (300, 1) if dim == 1 else (70, 5)
    say(f"{dim}d drift only (kappa = 0)")
    f0, u, p = make_case(dim, nx, 17, ny=ny, seed=920 + dim)
    p = dict(p, kappa=0.0)
    got = run_gpu(f0, u, p, 4)
    want = run_oracle(f0, u, p, 4)
    err = rel_l2(got, want)
    say("  rel L2", err)
    assert err <= FP32_REL_L2


def test_work_runs_on_the_given_stream():
    """The library queues its work on the stream it is given: a side stream
    is held up by a bounded GPU sleep, then the state is refilled and
    stepped on it with no host synchronisation in between; work queued
    anywhere else would read the zeros left before the refill."""
    import torch
    from paper_1508_02899_amd import Lattice
    from helpers import spec_for
    say("2d step queued behind a sleeping side stream")
    f0, u, p = make_case(2, 70, 9, ny=6, seed=930)
    want = run_oracle(f0, u, p, 3)
    side = torch.cuda.Stream()  # default priority
    lat = Lattice(spec_for(f0, p, "f32"), stream=side)
    src = torch.from_numpy(np.ascontiguousarray(f0)).cuda()
    ut = torch.from_numpy(np.ascontiguousarray(u)).cuda()
    f = torch.zeros_like(src)
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        torch.cuda._sleep(50_000_000)  # about 20 ms of spinning
        f.copy_(src)
    lat.step(f, ut, p["tau_p"], p["kappa"], p["dt"], 3)
    lat.sync()
    torch.cuda.synchronize()
    err = rel_l2(f.cpu().numpy(), want)
    lat.close()
    say("  rel L2", err)
    assert err <= FP32_REL_L2


@pytest.mark.parametrize("dim,nv", [(1, 33), (1, 129), (2, 9), (2, 33)])
def test_pure_streaming_bit_exact(dim, nv):
    """tau_p = inf and kappa = 0: exact periodic permutation (np.roll)."""
    say(f"streaming dim={dim} nv={nv}")
    if dim == 1:
        f0, u, p = make_case(1, 200, nv, seed=9)
    else:
        f0, u, p = make_case(2, 33, nv, ny=10, seed=10)
    p = dict(p, tau_p=math.inf, kappa=0.0)
    nsteps = 5
    got = run_gpu(f0, u, p, nsteps)
    h = (nv - 1) // 2
    if dim == 1:
        want = np.stack([np.roll(f0[j], (j - h) * nsteps) for j in range(nv)])
    else:
        want = np.empty_like(f0)
        for jy in range(nv):
            for jx in range(nv):
                want[jy * nv + jx] = np.roll(
                    f0[jy * nv + jx], ((jy - h) * nsteps, (jx - h) * nsteps),
                    axis=(0, 1))
    assert np.array_equal(got, want)


@pytest.mark.parametrize("dim", [1, 2])
def test_translation_and_determinism_bit_exact(dim):
    """Rolling f and u by (3, 5) sites rolls the GPU result exactly, and two
    runs are bit-identical (tile placement does not change arithmetic)."""
    nv = 33 if dim == 1 else 17
    if dim == 1:
        f0, u, p = make_case(1, 600, nv, seed=11)
        sh, ax, axu = 5, (1,), (2,)
        shift = (sh,)
    else:
        f0, u, p = make_case(2, 96, nv, ny=8, seed=12)
        shift, ax, axu = (3, 5), (1, 2), (2, 3)
    a = run_gpu(f0, u, p, 5)
    b = run_gpu(f0, u, p, 5)
    assert np.array_equal(a, b)
    c = run_gpu(np.ascontiguousarray(np.roll(f0, shift, axis=ax)),
                np.ascontiguousarray(np.roll(u, shift, axis=axu)), p, 5)
    assert np.array_equal(np.roll(a, shift, axis=ax), c)


@pytest.mark.parametrize("dim,dtype", [(1, "f64"), (2, "f64"), (1, "f32"),
                                       (2, "f32")])
def test_moments_and_mass_conservation(dim, dtype):
    """FP64 moments on the GPU equal the oracle's moments of the same state;
    mass is conserved to 1e-12 (FP64 state) / 1e-6 (FP32 state)."""
    import torch
    import oracle
    from paper_1508_02899_amd import Lattice
    from helpers import spec_for
    if dim == 1:
        f0, u, p = make_case(1, 512, 33, seed=13, dtype=dtype)
    else:
        f0, u, p = make_case(2, 64, 17, ny=16, seed=14, dtype=dtype)
    lat = Lattice(spec_for(f0, p, dtype))
    f = torch.from_numpy(f0).cuda()
    ut = torch.from_numpy(u).cuda()
    m0 = lat.moments(f, p["dt"])
    o0 = oracle.moments(f0, dim=dim, dx=p["dx"], dt=p["dt"])
    assert m0["mass"] == pytest.approx(o0["mass"], rel=1e-13)
    for k in range(dim):
        assert m0["momentum"][k] == pytest.approx(o0["momentum"][k], rel=1e-11,
                                                  abs=1e-13)
        assert m0["second_moment"][k] == pytest.approx(o0["second_moment"][k],
                                                       rel=1e-12)
    assert m0["variance"] == pytest.approx(o0["variance"], rel=1e-11)
    lat.step(f, ut, p["tau_p"], p["kappa"], p["dt"], 40)
    m1 = lat.moments(f, p["dt"])
    drift = abs(m1["mass"] - m0["mass"]) / m0["mass"]
    say(f"  mass drift {dtype} dim={dim}: {drift:.3e}")
    assert drift <= (1e-12 if dtype == "f64" else 1e-6)
    assert float(f.min()) >= -1e-7 * float(f.max())
    lat.close()


def test_density_matches_velocity_sum():
    import torch
    from paper_1508_02899_amd import Lattice
    from helpers import spec_for
    f0, u, p = make_case(2, 50, 9, ny=12, seed=15, dtype="f64")
    lat = Lattice(spec_for(f0, p, "f64"))
    rho = lat.density(torch.from_numpy(f0).cuda(), p["dt"]).cpu().numpy()
    dv = p["dx"] / p["dt"]
    np.testing.assert_allclose(rho, f0.sum(axis=0) * dv * dv, rtol=1e-14)
    lat.close()


def test_cfl_violation_is_sticky_and_leaves_f():
    """|u| past the bound of Eq. 3: flag set on the device, the call's
    steps are no-ops, lattice_sync reports ECFL once and clears it."""
    import torch
    from paper_1508_02899_amd import Lattice, LatticeError
    from paper_1508_02899_amd.lattice import ECFL
    from helpers import spec_for
    f0, u, p = make_case(1, 256, 17, seed=16)
    lat = Lattice(spec_for(f0, p, "f32"))
    f = torch.from_numpy(f0).cuda()
    bad = torch.from_numpy(u * 50.0).cuda()
    lat.step(f, bad, p["tau_p"], p["kappa"], p["dt"], 3)
    assert lat.sync(check=False) == ECFL
    assert np.array_equal(f.cpu().numpy(), f0)
    assert lat.sync(check=False) == 0  # cleared
    nan = torch.from_numpy(u).cuda()
    nan[0, 0, 5] = float("nan")
    lat.step(f, nan, p["tau_p"], p["kappa"], p["dt"], 2)
    with pytest.raises(LatticeError):
        lat.sync()
    # a good call afterwards works
    lat.step(f, torch.from_numpy(u).cuda(), p["tau_p"], p["kappa"], p["dt"], 2)
    lat.sync()
    lat.close()


def test_host_side_errors():
    import torch
    from paper_1508_02899_amd import Lattice, LatticeError
    from paper_1508_02899_amd.lattice import EDIFF, EINVAL, ECFL
    from helpers import spec_for
    f0, u, p = make_case(1, 64, 9, seed=17)
    lat = Lattice(spec_for(f0, p, "f32"))
    f = torch.from_numpy(f0).cuda()
    ut = torch.from_numpy(u).cuda()
    dv = p["dx"] / p["dt"]
    with pytest.raises(LatticeError) as e:
        lat.step(f, ut, p["tau_p"], 0.6 * dv * dv / p["dt"], p["dt"], 1)
    assert e.value.code == EDIFF
    with pytest.raises(LatticeError) as e:
        lat.step(f, ut, -1.0, p["kappa"], p["dt"], 1)
    assert e.value.code == EINVAL
    with pytest.raises(LatticeError) as e:  # Vmax alone violates CFL
        lat.step(f, ut, 1e-6, p["kappa"], p["dt"], 1)
    assert e.value.code == ECFL
    with pytest.raises(LatticeError) as e:  # not enough u slices
        from paper_1508_02899_amd import LatticeSpec
        lat2 = Lattice(LatticeSpec(dim=1, nx=64, nv=9, dx=p["dx"], u_hold=1))
        lat2.step(f, ut, p["tau_p"], p["kappa"], p["dt"], 3)
    assert e.value.code == EINVAL
    lat.step(f, ut, p["tau_p"], p["kappa"], p["dt"], 0)  # no-op
    assert np.array_equal(f.cpu().numpy(), f0)
    lat.close()


@pytest.mark.parametrize("padded", [True, False])
def test_2d_512x512_v33_full_size_sampled_sites(padded):
    """2D 512^2 x 33^2 FP32 (1.14 GB state), the bench launch (padded
    planes at the recommended pitch, as the benchmark runs) and the
    contiguous layout: one step on the GPU; 64 sampled sites (corners,
    edges, interior) recomputed one by one by the oracle from their
    streamed velocity columns."""
    import torch
    import oracle
    from paper_1508_02899_amd import Lattice, LatticeSpec, inputs
    from paper_1508_02899_amd.lattice import recommended_pitch
    say(f"config-3 full size sampled parity, padded={padded}")
    n, nv, L = 512, 33, 2 * math.pi
    h = (nv - 1) // 2
    u = inputs.flow2d_streamfunction(n, L, 1, seed=inputs.seed_for(3))
    vmax = 3.0
    dv = vmax / h
    dx = L / n
    dt = dx / dv
    tau_p = 2 * math.pi  # St = 1
    p = dict(dim=2, dx=dx, dt=dt, tau_p=tau_p, kappa=1e-4, s=1, nsub=1,
             scheme="koren")
    rng = np.random.default_rng(16)
    f0 = torch.rand((nv * nv, n, n), generator=torch.Generator().manual_seed(3),
                    dtype=torch.float32)
    spec = LatticeSpec(dim=2, nx=n, ny=n, nv=nv, dx=dx)
    if padded:
        spec.plane_pitch = recommended_pitch(spec)
        assert spec.plane_pitch == n * n + 64
        fd = spec.state_from(f0)
    else:
        fd = f0.cuda()
    lat = Lattice(spec)
    lat.step(fd, torch.from_numpy(u).cuda(), tau_p, p["kappa"], dt, 1)
    lat.sync()
    out = fd.cpu().numpy()
    f0n = f0.numpy()
    sites = [(0, 0), (0, n - 1), (n - 1, 0), (n - 1, n - 1), (5, 17), (511, 200)]
    sites += [tuple(rng.integers(0, n, 2)) for _ in range(58)]
    jy, jx = np.divmod(np.arange(nv * nv), nv)
    worst = 0.0
    for (y, x) in sites:
        col = f0n[np.arange(nv * nv), (y - (jy - h)) % n, (x - (jx - h)) % n]
        uu = u[:, :, y:y + 1, x:x + 1].astype(np.float64)
        # a 1x1 periodic lattice: streaming is the identity, the oracle
        # applies exactly the collision of this site
        ref = oracle.step(col.reshape(nv * nv, 1, 1).astype(np.float64), uu,
                          dim=2, dx=dx, tau_p=tau_p, kappa=p["kappa"], dt=dt,
                          nsteps=1)
        worst = max(worst, rel_l2(out[:, y, x], ref[:, 0, 0]))
    say("  worst site rel L2", worst)
    assert worst <= FP32_REL_L2
    lat.close()


def test_1d_16384x129_full_size_full_state():
    """1D 16384 x 129 FP32 (configuration 2 shape: 32 OU modes with k^-5/3
    variance, St = 1, Vmax = 2, kappa = 1e-4, one flow slice per step,
    Koren), 6 steps on the GPU against the oracle over the whole state."""
    import torch
    from paper_1508_02899_amd import Lattice, LatticeSpec, inputs
    say("config-2 full size parity")
    n, nv, L, steps = 16384, 129, 2 * math.pi, 6
    h = (nv - 1) // 2
    dx = L / n
    dv = 2.0 / h
    dt = dx / dv
    tau_p = 2 * math.pi
    u = inputs.flow1d(n, L, steps, modes=32, spectrum="k-5/3", tau_f=1.0,
                      dt=dt, seed=inputs.seed_for(2))
    f0 = inputs.gaussian_ic(1, n, nv, dx, dv)
    p = dict(dim=1, dx=dx, dt=dt, tau_p=tau_p, kappa=1e-4, s=1, nsub=1,
             scheme="koren", u_hold=1)
    lat = Lattice(LatticeSpec(dim=1, nx=n, nv=nv, dx=dx, u_hold=1))
    fd = torch.from_numpy(f0).cuda()
    lat.step(fd, torch.from_numpy(u).cuda(), tau_p, p["kappa"], dt, steps)
    lat.sync()
    got = fd.cpu().numpy()
    want = run_oracle(f0, u, p, steps, u_hold=1)
    err = rel_l2(got, want)
    say("  rel L2", err)
    assert err <= FP32_REL_L2
    lat.close()


def test_2d_256x256_v65_full_size_sampled_sites():
    """2D 256^2 x 65^2 FP32 (the fine lattice of configuration 5, 1.1 GB
    state), St = 2 with 4 collision sub-steps: one step on the GPU; 40
    sampled sites recomputed one by one by the oracle."""
    import torch
    import oracle
    from paper_1508_02899_amd import Lattice, LatticeSpec, inputs
    say("config-5 fine lattice full size sampled parity")
    n, nv, L, nsub = 256, 65, 2 * math.pi, 4
    h = (nv - 1) // 2
    u = inputs.flow2d_streamfunction(n, L, 1, seed=inputs.seed_for(5))
    dv = 3.0 / h
    dx = L / n
    dt = dx / dv
    tau_p = 2 * 2 * math.pi  # St = 2
    kappa = 1e-4
    f0 = torch.rand((nv * nv, n, n), generator=torch.Generator().manual_seed(5),
                    dtype=torch.float32)
    lat = Lattice(LatticeSpec(dim=2, nx=n, ny=n, nv=nv, dx=dx, nsub=nsub))
    ud = torch.from_numpy(u).cuda()
    cfl, _ = lat.stability(ud, tau_p, kappa, dt)
    assert cfl <= 0.5
    fd = f0.cuda()
    lat.step(fd, ud, tau_p, kappa, dt, 1)
    lat.sync()
    out = fd.cpu().numpy()
    f0n = f0.numpy()
    rng = np.random.default_rng(17)
    sites = [(0, 0), (n - 1, n - 1), (0, n - 1), (128, 3)]
    sites += [tuple(rng.integers(0, n, 2)) for _ in range(36)]
    jy, jx = np.divmod(np.arange(nv * nv), nv)
    worst = 0.0
    for (y, x) in sites:
        col = f0n[np.arange(nv * nv), (y - (jy - h)) % n, (x - (jx - h)) % n]
        uu = u[:, :, y:y + 1, x:x + 1].astype(np.float64)
        ref = oracle.step(col.reshape(nv * nv, 1, 1).astype(np.float64), uu,
                          dim=2, dx=dx, tau_p=tau_p, kappa=kappa, dt=dt,
                          nsteps=1, nsub=nsub)
        worst = max(worst, rel_l2(out[:, y, x], ref[:, 0, 0]))
    say("  worst site rel L2", worst)
    assert worst <= FP32_REL_L2
    lat.close()
