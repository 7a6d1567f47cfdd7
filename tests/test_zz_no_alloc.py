"""lattice_step_noalloc (the step entry point that allocates nothing)
against lattice_step on the same inputs: the same kernels run in the same
order, so the results must be bit-identical.  Two calls in a row, the second
on a smaller lattice (the static scratch keeps the first call's contents),
then a call whose flow breaks the CFL bound of Eq. 3 (status set, f left
unchanged), then a good call again (the flag is cleared per call)."""
import numpy as np
import pytest

from helpers import FP32_REL_L2, make_case, rel_l2, run_oracle, say, spec_for

pytestmark = pytest.mark.gpu


def _both(f0, u, p, nsteps, u_hold):
    import torch
    from paper_1508_02899_amd import Lattice
    from paper_1508_02899_amd.lattice import step_noalloc
    spec = spec_for(f0, p, "f32", u_hold)
    ud = torch.from_numpy(np.ascontiguousarray(u)).cuda()
    with Lattice(spec) as lat:
        fa = torch.from_numpy(np.ascontiguousarray(f0)).cuda()
        lat.step(fa, ud, p["tau_p"], p["kappa"], p["dt"], nsteps)
        lat.sync()
    fb = torch.from_numpy(np.ascontiguousarray(f0)).cuda()
    status = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    step_noalloc(spec, fb, ud, p["tau_p"], p["kappa"], p["dt"], nsteps,
                 status=status)
    torch.cuda.synchronize()
    return fa.cpu().numpy(), fb.cpu().numpy(), int(status.item())


def test_noalloc_matches_lattice_step_two_calls_in_a_row():
    # first call: 2D 150 x 20 x 33^2 (two 128-site tiles), 5 steps (odd:
    # the state is copied into the twin first), a new flow slice every step
    say("noalloc 2d 150x20x33^2, 5 steps")
    f0, u, p = make_case(2, 150, 33, ny=20, seed=901, slices=5)
    a, b, st = _both(f0, u, p, 5, 1)
    assert st == 0
    assert np.array_equal(a, b)
    err = rel_l2(b, run_oracle(f0, u, p, 5, u_hold=1))
    say("  rel L2 vs oracle", err)
    assert err <= FP32_REL_L2
    # second call, smaller: 2D 40 x 7 x 9^2 with nsub 2, 4 steps (even)
    say("noalloc 2d 40x7x9^2 nsub 2, 4 steps")
    f0, u, p = make_case(2, 40, 9, ny=7, seed=902, slices=2, nsub=2)
    a, b, st = _both(f0, u, p, 4, 2)
    assert st == 0
    assert np.array_equal(a, b)
    # third call, 1D 300 x 33, 3 steps
    say("noalloc 1d 300x33, 3 steps")
    f0, u, p = make_case(1, 300, 33, seed=903)
    a, b, st = _both(f0, u, p, 3, 0)
    assert st == 0
    assert np.array_equal(a, b)


def test_noalloc_reports_cfl_violation_and_recovers():
    import torch
    from paper_1508_02899_amd.lattice import step_noalloc
    say("noalloc cfl status")
    f0, u, p = make_case(2, 64, 17, ny=8, seed=904)
    spec = spec_for(f0, p, "f32")
    f = torch.from_numpy(f0).cuda()
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    bad = torch.from_numpy(u * 50.0).cuda()
    step_noalloc(spec, f, bad, p["tau_p"], p["kappa"], p["dt"], 3,
                 status=status)
    torch.cuda.synchronize()
    assert int(status.item()) != 0
    assert np.array_equal(f.cpu().numpy(), f0)
    step_noalloc(spec, f, torch.from_numpy(u).cuda(), p["tau_p"], p["kappa"],
                 p["dt"], 2, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    err = rel_l2(f.cpu().numpy(), run_oracle(f0, u, p, 2))
    assert err <= FP32_REL_L2


def test_noalloc_refuses_a_state_past_the_scratch():
    import torch
    from paper_1508_02899_amd import LatticeError, LatticeSpec
    from paper_1508_02899_amd.lattice import ETOOBIG, step_noalloc
    spec = LatticeSpec(dim=2, nx=512, ny=64, nv=33, dx=0.01)
    f = torch.zeros(spec.state_shape, device="cuda")
    u = torch.zeros(1, 2, 64, 512, device="cuda")
    with pytest.raises(LatticeError) as e:
        step_noalloc(spec, f, u, 1.0, 0.0, 0.05, 1)
    assert e.value.code == ETOOBIG
