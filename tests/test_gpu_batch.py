"""GPU parity of the batched 1D form: every member against the FP64 oracle
run on its own; graph replays, work decompositions and member freezing."""
import math

import numpy as np
import pytest

from helpers import FP32_REL_L2, rel_l2, say

pytestmark = pytest.mark.gpu


def _members(rng, specs, nsteps):
    """specs: (nx, nv, St, kappa_frac, u_hold, cfl)."""
    from paper_1508_02899_amd import Member
    mems, states, flows = [], [], []
    L = 2 * math.pi
    for nx, nv, St, kf, hold, cfl in specs:
        h = (nv - 1) // 2
        dx = L / nx
        tau_p = St * L
        umax = 1.0
        # choose dt so that the drift CFL (Eq. 3) is about cfl:
        # (dt/dv)(umax + h dv)/tau_p with dv = dx/dt
        # -> dt^2 umax/dx + dt h = cfl tau_p
        a, b, c = umax / dx, h, -cfl * tau_p
        dt = (-b + math.sqrt(b * b - 4 * a * c)) / (2 * a)
        dv = dx / dt
        kappa = kf * 0.5 * dv * dv / dt
        nsl = (nsteps + hold - 1) // hold if hold else 1
        mems.append(Member(nx=nx, nv=nv, dx=dx, dt=dt, tau_p=tau_p,
                           kappa=kappa, u_hold=hold, n_u_slices=nsl))
        states.append((rng.random((nv, nx)) ** 2).astype(np.float32))
        flows.append((umax * np.tanh(rng.standard_normal((nsl, nx))))
                     .astype(np.float32))
    return mems, states, flows


SPECS = [(130, 5, 0.5, 0.2, 0, 0.4), (257, 9, 2.0, 0.1, 3, 0.45),
         (300, 17, 1.0, 0.3, 1, 0.3), (513, 33, 3.0, 0.2, 2, 0.4),
         (700, 65, 5.0, 0.05, 0, 0.45), (640, 129, 10.0, 0.1, 4, 0.4),
         (64, 33, 0.2, 0.2, 1, 0.25)]


def _oracle_member(m, f0, u, nsteps, scheme="koren"):
    import oracle
    return oracle.step(f0.astype(np.float64), u.astype(np.float64)[:, None, :],
                       dim=1, dx=m.dx, tau_p=m.tau_p, kappa=m.kappa, dt=m.dt,
                       nsteps=nsteps, scheme=scheme, u_hold=m.u_hold)


def _run(batch, fpack, upack, nsteps, graph_steps=0):
    import torch
    f = torch.from_numpy(fpack.copy()).cuda()
    u = torch.from_numpy(upack).cuda()
    batch.step(f, u, nsteps, graph_steps=graph_steps)
    batch.sync()
    return f.cpu().numpy()


@pytest.mark.parametrize("scheme", ["koren", "upwind"])
def test_batch_members_match_oracle(scheme):
    from paper_1508_02899_amd import Batch
    nsteps = 9
    rng = np.random.default_rng(21)
    mems, states, flows = _members(rng, SPECS, nsteps)
    b = Batch(mems, scheme=scheme)
    out = b.unpack_state(_run(b, b.pack_state(states), b.pack_flow(flows),
                              nsteps))
    for m, f0, u, got in zip(mems, states, flows, out):
        want = _oracle_member(m, f0, u, nsteps, scheme)
        err = rel_l2(got, want)
        say(f"  member nx={m.nx} nv={m.nv}: rel L2 {err:.2e}")
        assert err <= FP32_REL_L2
    b.close()


def test_batch_graph_replays_and_tuning_are_bit_identical():
    """HIP-graph replays (several, with eager work in between) and every
    work decomposition give exactly the eager result."""
    import torch
    from paper_1508_02899_amd import Batch
    nsteps = 10
    rng = np.random.default_rng(22)
    mems, states, flows = _members(rng, SPECS, 3 * nsteps)
    b = Batch(mems)
    fp, up = b.pack_state(states), b.pack_flow(flows)
    ref = _run(b, fp, up, nsteps)
    u = torch.from_numpy(up).cuda()
    f = torch.from_numpy(fp.copy()).cuda()
    for rep in range(3):
        f.copy_(torch.from_numpy(fp))
        b.step(f, u, nsteps, graph_steps=4)  # 2 replays + 2 eager steps
        b.sync()
        m = b.moments(f)  # eager work between replays
        assert np.isfinite(m).all()
        assert np.array_equal(f.cpu().numpy(), ref), f"replay {rep}"
    for block, gpc in [(64, 1), (128, 2), (256, 4), (64, 0)]:
        for cap in Batch.CAPS:
            b.tune(cap, block, gpc)
        assert np.array_equal(_run(b, fp, up, nsteps, graph_steps=2), ref)
    b.close()


# members with nv equal to their class capacity (split-column tiles allowed)
SPLIT_SPECS = [(512, 33, 0.3, 0.2, 2, 0.4), (45, 17, 1.0, 0.3, 0, 0.3),
               (700, 65, 5.0, 0.05, 1, 0.45), (1000, 129, 10.0, 0.1, 3, 0.4),
               (31, 129, 2.0, 0.2, 0, 0.35), (8192, 33, 0.1, 0.1, 0, 0.45)]


@pytest.mark.parametrize("scheme", ["koren", "upwind"])
def test_batch_split_column_tiles_match_oracle(scheme):
    """Split-column tiles (block 0) for every class: members against the
    oracle, eager and graph replays bit-identical, persistent grids (tiles
    walked by fewer workgroups) bit-identical to one workgroup per tile."""
    from paper_1508_02899_amd import Batch
    nsteps = 8
    rng = np.random.default_rng(23)
    mems, states, flows = _members(rng, SPLIT_SPECS, nsteps)
    b = Batch(mems, scheme=scheme)
    for cap in (17, 33, 65, 129):
        b.tune(cap, 0, 0)
    fp, up = b.pack_state(states), b.pack_flow(flows)
    ref = _run(b, fp, up, nsteps)
    for m, f0, u, got in zip(mems, states, flows, b.unpack_state(ref)):
        want = _oracle_member(m, f0, u, nsteps, scheme)
        err = rel_l2(got, want)
        say(f"  member nx={m.nx} nv={m.nv}: rel L2 {err:.2e}")
        assert err <= FP32_REL_L2
    for gpc in (1, 4):
        for cap in (17, 33, 65, 129):
            b.tune(cap, 0, gpc)
        assert np.array_equal(_run(b, fp, up, nsteps, graph_steps=4), ref)
    b.close()


def test_batch_split_column_needs_nv_equal_to_capacity():
    """A class holding a member with nv below its capacity refuses
    split-column tiles and keeps working with its previous decomposition."""
    from paper_1508_02899_amd import Batch, LatticeError
    rng = np.random.default_rng(24)
    mems, states, flows = _members(rng, [(200, 31, 1.0, 0.2, 0, 0.4),
                                         (100, 33, 1.0, 0.2, 0, 0.4)], 4)
    b = Batch(mems)
    with pytest.raises(LatticeError):
        b.tune(33, 0, 0)
    with pytest.raises(LatticeError):
        b.tune(9, 0, 0)
    out = b.unpack_state(_run(b, b.pack_state(states), b.pack_flow(flows), 4))
    for m, f0, u, got in zip(mems, states, flows, out):
        assert rel_l2(got, _oracle_member(m, f0, u, 4)) <= FP32_REL_L2
    b.close()


def test_batch_moments_match_oracle():
    import torch
    import oracle
    from paper_1508_02899_amd import Batch
    rng = np.random.default_rng(23)
    mems, states, flows = _members(rng, SPECS, 1)
    b = Batch(mems)
    m = b.moments(torch.from_numpy(b.pack_state(states)).cuda())
    for k, (mem, f0) in enumerate(zip(mems, states)):
        o = oracle.moments(f0, dim=1, dx=mem.dx, dt=mem.dt)
        assert m[k, 0] == pytest.approx(o["mass"], rel=1e-13)
        assert m[k, 1] == pytest.approx(o["momentum"][0], rel=1e-11, abs=1e-12)
        assert m[k, 2] == pytest.approx(o["second_moment"][0], rel=1e-12)
        assert m[k, 3] == pytest.approx(o["variance"], rel=1e-11)
    b.close()


def test_batch_freezes_only_the_violating_member():
    import torch
    from paper_1508_02899_amd import Batch
    from paper_1508_02899_amd.lattice import ECFL
    rng = np.random.default_rng(24)
    mems, states, flows = _members(rng, SPECS[:4], 4)
    flows[2] = flows[2] * 1000.0
    b = Batch(mems)
    fp = b.pack_state(states)
    f = torch.from_numpy(fp.copy()).cuda()
    b.step(f, torch.from_numpy(b.pack_flow(flows)).cuda(), 4)
    rc, flags = b.sync(check=False)
    assert rc == ECFL
    assert list(flags) == [0, 0, 1, 0]
    out = b.unpack_state(f.cpu().numpy())
    assert np.array_equal(out[2], states[2])
    assert not np.array_equal(out[1], states[1])
    assert b.sync(check=False)[0] == 0
    b.close()


def test_batch_flow_check_reaches_the_last_slice():
    """A new flow slice every step and many steps: the check of a member's
    slices is spread over many workgroups; one value past the drift bound
    in the very last slice still freezes exactly that member."""
    import torch
    from paper_1508_02899_amd import Batch
    from paper_1508_02899_amd.lattice import ECFL
    rng = np.random.default_rng(25)
    nsteps = 400
    specs = [(700, 33, 1.0, 0.2, 1, 0.4), (513, 17, 2.0, 0.2, 1, 0.4),
             (900, 65, 5.0, 0.1, 1, 0.4)]
    mems, states, flows = _members(rng, specs, nsteps)
    flows[1][-1, 257] = 1000.0  # last slice, one site
    b = Batch(mems)
    fp = b.pack_state(states)
    f = torch.from_numpy(fp.copy()).cuda()
    b.step(f, torch.from_numpy(b.pack_flow(flows)).cuda(), nsteps,
           graph_steps=50)
    rc, flags = b.sync(check=False)
    assert rc == ECFL
    assert list(flags) == [0, 1, 0]
    out = b.unpack_state(f.cpu().numpy())
    assert np.array_equal(out[1], states[1])
    assert not np.array_equal(out[0], states[0])
    b.close()


def test_batch_256_members_full_size_sampled():
    """256 realizations, nx uniform in [512, 8192], nv in {33, 65, 129},
    St log-uniform in [0.1, 10], own flow each: a few steps on the GPU,
    five members (largest, smallest, three random) recomputed by the
    oracle."""
    import torch
    from paper_1508_02899_amd import Batch, Member, inputs
    rng = np.random.default_rng(inputs.seed_for(4))
    nsteps, L = 4, 2 * math.pi
    mems, states, flows = [], [], []
    for r in range(256):
        nx = int(rng.integers(512, 8193))
        nv = int(rng.choice([33, 65, 129]))
        St = float(10 ** rng.uniform(-1, 1))
        tau_p = St * L
        vmax = inputs.choose_vmax(nx, L, nv, tau_p, 4.0)
        h = (nv - 1) // 2
        dv = vmax / h
        dx = L / nx
        dt = dx / dv
        mems.append(Member(nx=nx, nv=nv, dx=dx, dt=dt, tau_p=tau_p,
                           kappa=1e-4, u_hold=50, n_u_slices=1))
        states.append(inputs.gaussian_ic(1, nx, nv, dx, dv))
        flows.append(inputs.flow1d(nx, L, 1, modes=8, spectrum="k-1",
                                   renew=50, seed=inputs.seed_for(4, r))[:, 0])
    b = Batch(mems)
    say(f"  batch of 256: {b.total_cells} cells")
    fp = b.pack_state(states)
    f = torch.from_numpy(fp.copy()).cuda()
    u = torch.from_numpy(b.pack_flow(flows)).cuda()
    b.step(f, u, nsteps, graph_steps=2)
    b.sync()
    out = b.unpack_state(f.cpu().numpy())
    # the resident schedule on the same batch: the same bits
    from paper_1508_02899_amd.lattice import RESIDENT
    for cap in (33, 65, 129):
        b.tune(cap, 0, 0)
    f.copy_(torch.from_numpy(fp))
    b.step(f, u, nsteps)
    b.sync()
    split = f.cpu().numpy()
    b.schedule(RESIDENT)
    f.copy_(torch.from_numpy(fp))
    b.step(f, u, nsteps)
    b.sync()
    assert np.array_equal(f.cpu().numpy(), split)
    sizes = [m.nx * m.nv for m in mems]
    pick = {int(np.argmax(sizes)), int(np.argmin(sizes))}
    pick |= set(int(i) for i in rng.choice(256, 3, replace=False))
    for k in sorted(pick):
        want = _oracle_member(mems[k], states[k], flows[k], nsteps)
        err = rel_l2(out[k], want)
        say(f"  member {k} nx={mems[k].nx} nv={mems[k].nv}: {err:.2e}")
        assert err <= FP32_REL_L2
    b.close()


def _split_batch(scheme, nsteps, seed):
    from paper_1508_02899_amd import Batch
    rng = np.random.default_rng(seed)
    mems, states, flows = _members(rng, SPLIT_SPECS, nsteps)
    b = Batch(mems, scheme=scheme)
    for cap in (17, 33, 65, 129):
        b.tune(cap, 0, 0)
    return b, mems, states, flows


@pytest.mark.parametrize("scheme", ["koren", "upwind"])
@pytest.mark.parametrize("nsteps", [7, 12])
def test_batch_resident_schedule_matches_per_step_and_oracle(scheme, nsteps):
    """The resident schedule (one launch per call, per-member step barriers
    on device counters, members split among the XCDs) gives exactly the
    per-step result, for odd and even step counts, several grid sizes and
    work chunks, and every member matches the oracle."""
    from paper_1508_02899_amd.lattice import PER_STEP, RESIDENT
    b, mems, states, flows = _split_batch(scheme, nsteps, 31)
    fp, up = b.pack_state(states), b.pack_flow(flows)
    ref = _run(b, fp, up, nsteps)
    for gpc, chunk in ((0, 0), (1, 1), (3, 8), (0, 64)):
        b.schedule(RESIDENT, grid_per_cu=gpc, chunk=chunk)
        got = _run(b, fp, up, nsteps)
        assert np.array_equal(got, ref), f"grid per CU {gpc}, chunk {chunk}"
    for m, f0, u, g in zip(mems, states, flows, b.unpack_state(got)):
        err = rel_l2(g, _oracle_member(m, f0, u, nsteps, scheme))
        say(f"  member nx={m.nx} nv={m.nv}: rel L2 {err:.2e}")
        assert err <= FP32_REL_L2
    b.schedule(PER_STEP)
    assert np.array_equal(_run(b, fp, up, nsteps), ref)
    b.close()


def test_batch_resident_freezes_only_the_violating_member():
    import torch
    from paper_1508_02899_amd.lattice import ECFL, RESIDENT
    b, mems, states, flows = _split_batch("koren", 6, 32)
    flows[3] = flows[3] * 1000.0
    b.schedule(RESIDENT)
    f = torch.from_numpy(b.pack_state(states)).cuda()
    b.step(f, torch.from_numpy(b.pack_flow(flows)).cuda(), 6)
    rc, flags = b.sync(check=False)
    assert rc == ECFL
    assert list(flags) == [0, 0, 0, 1, 0, 0]
    out = b.unpack_state(f.cpu().numpy())
    assert np.array_equal(out[3], states[3])
    for k in (0, 2, 5):
        assert rel_l2(out[k], _oracle_member(mems[k], states[k], flows[k],
                                             6)) <= FP32_REL_L2
    b.close()


def test_batch_resident_wait_limit_reports_a_timeout():
    """Forced from the host: with a negative wait limit every wait gives up
    at once, the launch ends early and sync reports ETIMEOUT (once); the
    next calls with the normal limit are exact again."""
    import torch
    from paper_1508_02899_amd.lattice import ETIMEOUT, RESIDENT
    b, mems, states, flows = _split_batch("koren", 6, 33)
    fp, up = b.pack_state(states), b.pack_flow(flows)
    ref = _run(b, fp, up, 6)
    b.schedule(RESIDENT, wait_limit=-1)
    f = torch.from_numpy(fp.copy()).cuda()
    b.step(f, torch.from_numpy(up).cuda(), 6)
    rc, _ = b.sync(check=False)
    assert rc == ETIMEOUT
    assert b.sync(check=False)[0] == 0
    b.schedule(RESIDENT)
    assert np.array_equal(_run(b, fp, up, 6), ref)
    b.close()


def test_batch_resident_needs_split_column_velocity_counts():
    from paper_1508_02899_amd import Batch, LatticeError
    from paper_1508_02899_amd.lattice import RESIDENT
    rng = np.random.default_rng(34)
    mems, states, flows = _members(rng, [(200, 31, 1.0, 0.2, 0, 0.4),
                                         (100, 33, 1.0, 0.2, 0, 0.4)], 4)
    b = Batch(mems)
    with pytest.raises(LatticeError):
        b.schedule(RESIDENT)
    out = b.unpack_state(_run(b, b.pack_state(states), b.pack_flow(flows), 4))
    for m, f0, u, got in zip(mems, states, flows, out):
        assert rel_l2(got, _oracle_member(m, f0, u, 4)) <= FP32_REL_L2
    b.close()


def test_batch_velocity_stride_two_both_schedules():
    """Velocity stride 2 (each velocity index shifts 2(j-h) cells): the
    per-step and the resident schedules give the same bits, and every
    member matches the oracle run with the same stride."""
    import oracle
    from paper_1508_02899_amd import Batch
    from paper_1508_02899_amd.lattice import RESIDENT
    nsteps = 5
    rng = np.random.default_rng(35)
    mems, states, flows = _members(rng, SPLIT_SPECS, nsteps)
    b = Batch(mems, vstride=2)
    for cap in (17, 33, 65, 129):
        b.tune(cap, 0, 0)
    fp, up = b.pack_state(states), b.pack_flow(flows)
    ref = _run(b, fp, up, nsteps)
    b.schedule(RESIDENT)
    assert np.array_equal(_run(b, fp, up, nsteps), ref)
    for m, f0, u, got in zip(mems, states, flows, b.unpack_state(ref)):
        want = oracle.step(f0.astype(np.float64),
                           u.astype(np.float64)[:, None, :], dim=1, dx=m.dx,
                           tau_p=m.tau_p, kappa=m.kappa, dt=m.dt,
                           nsteps=nsteps, u_hold=m.u_hold, s=2)
        err = rel_l2(got, want)
        say(f"  member nx={m.nx} nv={m.nv}, stride 2: rel L2 {err:.2e}")
        assert err <= FP32_REL_L2
    b.close()
