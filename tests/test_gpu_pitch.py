"""Padded velocity planes (lattice_desc.plane_pitch): the layout the 2D
benchmark runs in.  The update does not depend on where the planes sit, so
a padded run must give the same bits as a contiguous one, and the padding
between the planes is never read as state nor written in f: it is filled
with NaN here, and every result must stay finite."""
import math

import numpy as np
import pytest

from helpers import FP32_REL_L2, make_case, rel_l2, run_gpu, run_oracle, say
from helpers import spec_for

pytestmark = pytest.mark.gpu


def _padded(spec, f0, pad):
    """State tensor of spec with plane pitch sites + pad, the pads NaN."""
    import torch
    from dataclasses import replace
    sp = replace(spec, plane_pitch=spec.sites + pad)
    buf = torch.full((sp.nplanes * sp.pitch,), float("nan"),
                     dtype=torch.float64 if spec.dtype == "f64"
                     else torch.float32, device="cuda")
    f = buf.as_strided(sp.state_shape, sp.state_strides)
    f.copy_(torch.from_numpy(np.ascontiguousarray(f0)))
    return sp, buf, f


def _gaps(sp, buf):
    b = buf.view(sp.nplanes, sp.pitch)[:, sp.sites:]
    return b.cpu().numpy()


@pytest.mark.parametrize("nv,nsub,steps,pad", [(3, 1, 3, 64), (9, 2, 4, 7),
                                               (17, 1, 5, 64), (33, 1, 3, 64),
                                               (33, 2, 2, 1000),
                                               (65, 1, 3, 64)])
def test_padded_planes_give_the_contiguous_bits(nv, nsub, steps, pad):
    import torch
    from paper_1508_02899_amd import Lattice
    say(f"padded planes nv={nv} nsub={nsub} steps={steps} pad={pad}")
    f0, u, p = make_case(2, 150, nv, ny=7, seed=700 + nv + pad, slices=steps,
                         nsub=nsub)
    want = run_gpu(f0, u, p, steps, u_hold=1)
    spec = spec_for(f0, p, "f32", u_hold=1)
    sp, buf, f = _padded(spec, f0, pad)
    with Lattice(sp) as lat:
        lat.step(f, torch.from_numpy(u).cuda(), p["tau_p"], p["kappa"],
                 p["dt"], steps)
        m = lat.moments(f, p["dt"])
        rho = lat.density(f, p["dt"]).cpu().numpy()
    got = f.cpu().numpy()
    assert np.array_equal(got, want)
    assert np.isnan(_gaps(sp, buf)).all()
    assert math.isfinite(m["mass"]) and math.isfinite(m["variance"])
    with Lattice(spec) as lat:
        fc = torch.from_numpy(want).cuda()
        mc = lat.moments(fc, p["dt"])
        rhoc = lat.density(fc, p["dt"]).cpu().numpy()
    for k in ("mass", "variance"):
        assert m[k] == mc[k]
    assert m["momentum"] == mc["momentum"]
    assert np.array_equal(rho, rhoc)
    err = rel_l2(got, run_oracle(f0, u, p, steps, u_hold=1))
    say("  rel L2 vs oracle", err)
    assert err <= FP32_REL_L2


def test_padded_s1_and_copy():
    import torch
    from paper_1508_02899_amd import Lattice
    say("padded planes: S1 and state copy")
    f0, u, p = make_case(2, 64, 9, ny=32, seed=731)
    spec = spec_for(f0, p, "f32")
    sp, buf, f = _padded(spec, f0, 64)
    r = [0, 1, 3, 8]
    with Lattice(sp) as lat:
        s_pad = lat.s1(f, p["dt"], r)
        g = sp.empty_state()
        lat.copy_state(g, f)
        lat.sync()
        assert np.array_equal(g.cpu().numpy(), f0)
    with Lattice(spec) as lat:
        s_flat = lat.s1(torch.from_numpy(f0).cuda(), p["dt"], r)
    np.testing.assert_allclose(s_pad, s_flat, rtol=1e-6)
    assert np.isnan(_gaps(sp, buf)).all()


def test_padded_no_alloc_step():
    import torch
    from paper_1508_02899_amd.lattice import step_noalloc
    say("padded planes: step without allocation")
    f0, u, p = make_case(2, 100, 17, ny=9, seed=741)
    want = run_gpu(f0, u, p, 3)
    spec = spec_for(f0, p, "f32")
    sp, buf, f = _padded(spec, f0, 64)
    status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    step_noalloc(sp, f, torch.from_numpy(u).cuda(), p["tau_p"], p["kappa"],
                 p["dt"], 3, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    assert np.array_equal(f.cpu().numpy(), want)
    assert np.isnan(_gaps(sp, buf)).all()
