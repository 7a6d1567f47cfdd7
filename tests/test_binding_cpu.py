"""Argument checks of the Python binding: every tensor handed to the library
is validated before any call reaches it (the kernels trust the sizes that the
descriptors imply).  The handles below are built without the library (no
GPU here); a check that let a bad tensor through would reach the missing
handle and fail differently."""
import pytest
import torch

from paper_1508_02899_amd import lattice as B


def _fake(cls, **attrs):
    obj = object.__new__(cls)
    obj.lib = None
    for k, v in attrs.items():
        setattr(obj, k, v)
    return obj


def test_require_tensor_checks_each_property():
    good = torch.zeros(12, dtype=torch.float32)
    with pytest.raises(TypeError, match="torch tensor"):
        B.require_tensor(good.numpy(), "a", torch.float32)
    with pytest.raises(TypeError, match="dtype"):
        B.require_tensor(good.double(), "a", torch.float32)
    with pytest.raises(ValueError, match="contiguous"):
        B.require_tensor(torch.zeros(4, 6)[:, ::2], "a", torch.float32)
    with pytest.raises(ValueError, match="shape"):
        B.require_tensor(good, "a", torch.float32, shape=(3, 4))
    with pytest.raises(ValueError, match="needs 13"):
        B.require_tensor(good, "a", torch.float32, numel=13)
    with pytest.raises(ValueError, match="at least 20"):
        B.require_tensor(good, "a", torch.float32, min_numel=20)
    with pytest.raises(ValueError, match="dimensions"):
        B.require_tensor(good, "a", torch.float32, ndim=2)
    # everything right but the device
    with pytest.raises(TypeError, match="CUDA"):
        B.require_tensor(good, "a", torch.float32, numel=12, shape=(12,))
    B.require_tensor(good, "a", torch.float32, numel=12, cuda=False)


@pytest.mark.parametrize("f,u,err", [
    (torch.zeros(100, dtype=torch.float64), torch.zeros(40), TypeError),
    (torch.zeros(99), torch.zeros(40), ValueError),              # short f
    (torch.zeros(200)[::2], torch.zeros(40), ValueError),        # strided f
    (torch.zeros(100), torch.zeros(39), ValueError),             # short u
    (torch.zeros(100), torch.zeros(40, dtype=torch.float16), TypeError),
    (torch.zeros(100), torch.zeros(40), TypeError),              # on the CPU
])
def test_batch_step_refuses_bad_buffers(f, u, err):
    b = _fake(B.Batch, total_elems=100, total_cells=90, total_u=40, _B=None,
              members=[])
    with pytest.raises(err):
        b.step(f, u, 1)


def test_batch_moments_refuses_bad_state():
    b = _fake(B.Batch, total_elems=100, total_cells=90, total_u=40, _B=None,
              members=[])
    with pytest.raises(ValueError):
        b.moments(torch.zeros(101))
    with pytest.raises(TypeError):
        b.moments(torch.zeros(100, dtype=torch.float64))
    with pytest.raises(TypeError, match="CUDA"):
        b.moments(torch.zeros(100))


def test_lattice_state_shape_is_checked_everywhere():
    spec = B.LatticeSpec(dim=2, nx=8, ny=4, nv=5, dx=0.1)
    lat = _fake(B.Lattice, spec=spec, torch_dtype=torch.float32, _L=None)
    bad = torch.zeros(25, 4, 7)
    u = torch.zeros(1, 2, 4, 8)
    for call in (lambda: lat.moments(bad, 0.1),
                 lambda: lat.density(bad, 0.1),
                 lambda: lat.step(bad, u, 1.0, 0.0, 0.1, 1),
                 lambda: lat.copy_state(bad, bad)):
        with pytest.raises(ValueError, match="shape"):
            call()
    good = torch.zeros(25, 4, 8)
    with pytest.raises(ValueError, match="slices"):
        lat.step(good, torch.zeros(63), 1.0, 0.0, 0.1, 1)
    with pytest.raises(TypeError, match="dtype"):
        lat.step(good, u.double(), 1.0, 0.0, 0.1, 1)


def test_mlp_sample_sets_are_checked():
    with pytest.raises(ValueError, match=r"\[n, 8\]"):
        B.Mlp._samples_ptrs(torch.zeros(10, 7))
    with pytest.raises(ValueError, match="dimensions"):
        B.Mlp._samples_ptrs(torch.zeros(80))
    with pytest.raises(ValueError, match="needs 10"):
        B.Mlp._samples_ptrs(torch.zeros(10, 8).cuda() if False else
                            torch.zeros(10, 8), torch.zeros(9), None)
    with pytest.raises(TypeError, match="dtype"):
        B.Mlp._samples_ptrs(torch.zeros(10, 8, dtype=torch.float64))


@pytest.mark.parametrize("sites,err", [
    (torch.tensor([0, 5, 16], dtype=torch.int32), ValueError),   # 16 >= 16
    (torch.tensor([-1, 5], dtype=torch.int32), ValueError),
    (torch.tensor([0, 5], dtype=torch.int64), TypeError),
    (torch.zeros(0, dtype=torch.int32), ValueError),
    (torch.tensor([[0, 5]], dtype=torch.int32), ValueError),
    (torch.tensor([0, 15], dtype=torch.int32), TypeError),        # CPU only
])
def test_mlp_site_indices_are_checked(sites, err):
    with pytest.raises(err):
        B.Mlp._sites_ptr(sites, 16)


def test_mlp_samples_check_the_lattice_and_states():
    coarse = _fake(B.Lattice, spec=B.LatticeSpec(dim=2, nx=4, ny=4, nv=17,
                                                 dx=0.1, vstride=4),
                   torch_dtype=torch.float32, _L=None)
    m = _fake(B.Mlp, _M=None)
    sites = torch.tensor([0, 3], dtype=torch.int32)
    u = torch.zeros(1, 2, 4, 4)
    with pytest.raises(ValueError, match="shape"):
        m.samples(coarse, 0.1, 1.0, 2.0, torch.zeros(289, 4, 5),
                  torch.zeros(289, 4, 4), u, sites)
    with pytest.raises(ValueError, match="at least 32"):
        m.samples(coarse, 0.1, 1.0, 2.0, torch.zeros(289, 4, 4),
                  torch.zeros(289, 4, 4), torch.zeros(31), sites)
    other = _fake(B.Lattice, spec=B.LatticeSpec(dim=2, nx=4, ny=4, nv=33,
                                                dx=0.1),
                  torch_dtype=torch.float32, _L=None)
    with pytest.raises(ValueError, match="17"):
        m.samples(other, 0.1, 1.0, 2.0, torch.zeros(1089, 4, 4),
                  torch.zeros(1089, 4, 4), u, sites)
    with pytest.raises(ValueError, match="fine"):
        m.samples_natural(other, coarse, 0.1, 1.0, 1e-4, 2.0,
                          torch.zeros(1089, 4, 4), torch.zeros(289, 4, 4), u,
                          sites)


def test_restrict_checks_its_input():
    with pytest.raises(ValueError, match="4k"):
        B.restrict(torch.zeros(33 * 33 - 1, 4), 2)
    with pytest.raises(TypeError, match="dtype"):
        B.restrict(torch.zeros(65, 4, dtype=torch.float64), 1)
    with pytest.raises(ValueError, match="dim"):
        B.restrict(torch.zeros(65, 4), 3)


def test_padded_state_views_are_checked():
    """A state with padded velocity planes is a strided view of one buffer;
    the binding accepts exactly that view and refuses plain contiguous
    tensors, other strides and other shapes."""
    spec = B.LatticeSpec(dim=2, nx=8, ny=4, nv=5, dx=0.1, plane_pitch=40)
    assert spec.state_strides == (40, 8, 1)
    assert spec.state_span == 24 * 40 + 32
    good = spec.empty_state(device="cpu")
    assert tuple(good.stride()) == (40, 8, 1)
    with pytest.raises(TypeError, match="CUDA"):
        B.require_state(good, spec, "f", torch.float32)
    B.require_state(good, spec, "f", torch.float32, cuda=False)
    with pytest.raises(ValueError, match="strides"):
        B.require_state(torch.zeros(25, 4, 8), spec, "f", torch.float32)
    # a view of the right strides but the wrong shape
    with pytest.raises(ValueError, match="shape"):
        B.require_state(good[:, :3], spec, "f", torch.float32)
    with pytest.raises(TypeError, match="dtype"):
        B.require_state(good.double(), spec, "f", torch.float32)
    # values survive the round trip through the padded layout
    import numpy as np
    a = np.arange(25 * 32, dtype=np.float32).reshape(25, 4, 8)
    t = spec.state_from(a, device="cpu")
    assert np.array_equal(t.numpy(), a)
    # an unpadded spec takes plain contiguous tensors
    flat = B.LatticeSpec(dim=2, nx=8, ny=4, nv=5, dx=0.1)
    assert flat.pitch == 32
    B.require_state(torch.zeros(25, 4, 8), flat, "f", torch.float32,
                    cuda=False)
