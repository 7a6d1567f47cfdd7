"""Python binding of the C-ABI lattice library (liblattice.so).

Argument marshalling only: every step of the lattice update runs in the
HIP kernels behind ``include/lattice.h``.  PyTorch supplies device memory
and the current HIP stream.  The library must have been built
(``python -m paper_1508_02899_amd.build`` or ``__graft_entry__.build()``);
importing this module without it raises ``LatticeLibraryMissing``.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblattice.so")

UPWIND, KOREN = 0, 1
F32, F64 = 0, 1
SCHEMES = {"upwind": UPWIND, "koren": KOREN}

OK, EINVAL, ECFL, EDIFF, EHIP, ENOMEM, ENONFINITE, ENOTSUP, ETOOBIG = (
    0, -1, -2, -3, -4, -5, -6, -7, -8)
ETIMEOUT = -9
PER_STEP, RESIDENT = 0, 1  # lattice_batch_schedule modes
NOALLOC_MAX_BYTES = 64 << 20  # LATTICE_NOALLOC_MAX_BYTES

# every symbol declared in include/lattice.h
EXPORTS = (
    "lattice_desc_default", "lattice_plane_pitch", "lattice_velocity",
    "lattice_init", "lattice_step",
    "lattice_collide", "lattice_step_noalloc",
    "lattice_moments", "lattice_density", "lattice_stability",
    "lattice_copy_state", "lattice_sync", "lattice_profile", "lattice_rho_r2",
    "lattice_rho_r2_error",
    "lattice_flow1d_modes", "lattice_flow2d_modes", "lattice_s1",
    "lattice_profile_read", "lattice_destroy", "lattice_strerror",
    "lattice_last_error", "lattice_batch_init", "lattice_batch_layout",
    "lattice_batch_plane_pitch", "lattice_batch_tune",
    "lattice_batch_schedule", "lattice_batch_step",
    "lattice_batch_moments",
    "lattice_batch_sync", "lattice_batch_destroy", "lattice_batch_last_error",
    "lattice_restrict",
    "lattice_mlp_create", "lattice_mlp_set_params", "lattice_mlp_get_params",
    "lattice_mlp_samples", "lattice_mlp_samples_natural", "lattice_mlp_grad",
    "lattice_mlp_train",
    "lattice_mlp_forward", "lattice_mlp_attach", "lattice_mlp_destroy",
)

MLP_NPARAMS = 4801  # W1[8][64], b1[64], W2[64][64], b2[64], w3[64], b3


class LatticeLibraryMissing(RuntimeError):
    pass


class LatticeError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lattice error {code}: {msg}")
        self.code = code


class Desc(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32),
        ("nx", ctypes.c_int64),
        ("ny", ctypes.c_int64),
        ("nv", ctypes.c_int32),
        ("vstride", ctypes.c_int32),
        ("dx", ctypes.c_double),
        ("scheme", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("nsub", ctypes.c_int32),
        ("u_hold", ctypes.c_int64),
        ("stream", ctypes.c_void_p),
        ("plane_pitch", ctypes.c_int64),
    ]


class MemberDesc(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int64),
        ("nv", ctypes.c_int32),
        ("dx", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("tau_p", ctypes.c_double),
        ("kappa", ctypes.c_double),
        ("u_hold", ctypes.c_int64),
        ("n_u_slices", ctypes.c_int64),
    ]


class Moments(ctypes.Structure):
    _fields_ = [
        ("mass", ctypes.c_double),
        ("momentum", ctypes.c_double * 2),
        ("second_moment", ctypes.c_double * 2),
        ("variance", ctypes.c_double),
        ("nonfinite", ctypes.c_int32),
    ]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load liblattice.so (fails loudly when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise LatticeLibraryMissing(
            f"{path} not found: build the HIP library first "
            "(python -m paper_1508_02899_amd.build)")
    L = ctypes.CDLL(path)
    vp, i64, dbl, i32 = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_double,
                         ctypes.c_int)
    pdesc = ctypes.POINTER(Desc)
    L.lattice_desc_default.argtypes = [pdesc]
    L.lattice_plane_pitch.argtypes = [pdesc, ctypes.POINTER(i64)]
    L.lattice_velocity.argtypes = [pdesc, dbl, ctypes.POINTER(dbl),
                                   ctypes.POINTER(dbl)]
    L.lattice_init.argtypes = [pdesc, ctypes.POINTER(vp)]
    L.lattice_step.argtypes = [vp, vp, vp, i64, dbl, dbl, dbl, i64]
    L.lattice_collide.argtypes = [vp, vp, vp, i64, dbl, dbl, dbl, i64]
    L.lattice_step_noalloc.argtypes = [pdesc, vp, vp, i64, dbl, dbl, dbl,
                                       i64, vp]
    L.lattice_moments.argtypes = [vp, vp, dbl, ctypes.POINTER(Moments)]
    L.lattice_density.argtypes = [vp, vp, dbl, vp]
    L.lattice_stability.argtypes = [vp, vp, i64, dbl, dbl, dbl,
                                    ctypes.POINTER(dbl)]
    L.lattice_copy_state.argtypes = [vp, vp, vp]
    L.lattice_rho_r2.argtypes = [vp, vp, i32, ctypes.POINTER(dbl)]
    L.lattice_rho_r2_error.argtypes = [ctypes.POINTER(dbl),
                                       ctypes.POINTER(dbl), i32, dbl,
                                       ctypes.POINTER(dbl)]
    L.lattice_flow1d_modes.argtypes = [vp, i32, vp, i64, vp]
    L.lattice_s1.argtypes = [vp, vp, dbl, i32, ctypes.POINTER(i32),
                             ctypes.POINTER(dbl)]
    L.lattice_flow2d_modes.argtypes = [vp, i32, vp, i64, vp]
    L.lattice_sync.argtypes = [vp]
    L.lattice_profile.argtypes = [vp, i32]
    L.lattice_profile_read.argtypes = [vp, ctypes.POINTER(dbl),
                                       ctypes.POINTER(i64)]
    L.lattice_destroy.argtypes = [vp]
    L.lattice_strerror.argtypes = [i32]
    L.lattice_strerror.restype = ctypes.c_char_p
    L.lattice_last_error.argtypes = [vp]
    L.lattice_last_error.restype = ctypes.c_char_p
    pmem = ctypes.POINTER(MemberDesc)
    pi64 = ctypes.POINTER(i64)
    L.lattice_batch_init.argtypes = [pmem, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_int32, vp, ctypes.POINTER(vp)]
    L.lattice_batch_layout.argtypes = [vp, pi64, pi64, pi64, pi64]
    L.lattice_batch_plane_pitch.argtypes = [vp, pi64, pi64]
    L.lattice_batch_tune.argtypes = [vp, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_int32]
    L.lattice_batch_schedule.argtypes = [vp, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_int32, i64]
    L.lattice_batch_step.argtypes = [vp, vp, vp, i64, ctypes.c_int32,
                                     ctypes.c_int32]
    L.lattice_batch_moments.argtypes = [vp, vp, ctypes.POINTER(dbl)]
    L.lattice_batch_sync.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    L.lattice_batch_destroy.argtypes = [vp]
    L.lattice_batch_last_error.argtypes = [vp]
    L.lattice_batch_last_error.restype = ctypes.c_char_p
    pf = ctypes.POINTER(ctypes.c_float)
    L.lattice_restrict.argtypes = [ctypes.c_int32, i64, ctypes.c_int32, vp, vp,
                                   vp]
    L.lattice_mlp_create.argtypes = [vp, ctypes.POINTER(vp)]
    L.lattice_mlp_set_params.argtypes = [vp, pf]
    L.lattice_mlp_get_params.argtypes = [vp, pf]
    L.lattice_mlp_samples.argtypes = [vp, dbl, dbl, dbl, dbl, vp, vp, vp, vp,
                                      i64, vp, vp, vp]
    L.lattice_mlp_samples_natural.argtypes = [vp, vp, dbl, dbl, dbl, dbl, dbl,
                                              vp, vp, vp, vp, i64, vp, vp, vp]
    L.lattice_mlp_grad.argtypes = [vp, vp, vp, vp, i64, vp,
                                   ctypes.POINTER(dbl)]
    L.lattice_mlp_train.argtypes = [vp, vp, vp, vp, i64, i64, i64, dbl,
                                    ctypes.POINTER(dbl)]
    L.lattice_mlp_forward.argtypes = [vp, vp, i64, vp]
    L.lattice_mlp_attach.argtypes = [vp, vp, dbl, dbl]
    L.lattice_mlp_destroy.argtypes = [vp]
    for name in EXPORTS:
        getattr(L, name)  # every declared entry point must be exported
    _lib = L
    return L


@dataclass
class LatticeSpec:
    """Host-side description of a lattice (mirrors ``lattice_desc``)."""
    dim: int
    nx: int
    nv: int
    dx: float
    ny: int = 1
    vstride: int = 1
    scheme: str = "koren"
    dtype: str = "f32"
    nsub: int = 1
    u_hold: int = 0
    plane_pitch: int = 0   # elements between velocity planes; 0 = nx*ny

    @property
    def sites(self) -> int:
        return self.nx * (self.ny if self.dim == 2 else 1)

    @property
    def pitch(self) -> int:
        """Elements from one velocity plane of the state to the next."""
        return self.plane_pitch or self.sites

    @property
    def state_strides(self):
        """Element strides of a state tensor of shape state_shape."""
        if self.dim == 1:
            return (self.pitch, 1)
        return (self.pitch, self.nx, 1)

    @property
    def state_span(self) -> int:
        """Elements from the first to the last element of a state, + 1."""
        return (self.nplanes - 1) * self.pitch + self.sites

    def empty_state(self, device="cuda", dtype=None):
        """An uninitialised state tensor in this spec's layout (a strided
        view of one buffer when the plane pitch pads the planes)."""
        torch = _torch()
        if dtype is None:
            dtype = torch.float64 if self.dtype == "f64" else torch.float32
        buf = torch.empty(self.nplanes * self.pitch, dtype=dtype,
                          device=device)
        return buf.as_strided(self.state_shape, self.state_strides)

    def state_from(self, values, device="cuda"):
        """A state tensor in this spec's layout holding values (array-like
        of shape state_shape)."""
        import numpy as np
        torch = _torch()
        t = self.empty_state(device)
        src = values if isinstance(values, torch.Tensor) else \
            torch.from_numpy(np.ascontiguousarray(values))
        t.copy_(src)
        return t

    def velocity(self, dt: float):
        """(dv, Vmax) for time step dt: dv = vstride dx / dt, Vmax = h dv."""
        dv = self.vstride * self.dx / dt
        return dv, (self.nv - 1) // 2 * dv

    @property
    def nplanes(self) -> int:
        return self.nv ** self.dim

    @property
    def state_shape(self):
        if self.dim == 1:
            return (self.nv, self.nx)
        return (self.nv * self.nv, self.ny, self.nx)

    def u_shape(self, slices: int):
        if self.dim == 1:
            return (slices, 1, self.nx)
        return (slices, 2, self.ny, self.nx)


def _torch():
    import torch
    return torch


def require_tensor(t, name, dtype, shape=None, numel=None, min_numel=None,
                   ndim=None, cuda=True):
    """Raise unless t is a contiguous CUDA tensor of the given dtype and
    size.  Every pointer handed to the library passes through here first:
    the kernels trust the sizes the descriptors imply, so a short, wrongly
    typed or strided buffer must be refused before any launch.  Checks run
    in the order type, dtype, contiguity, size, device."""
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} dtype {t.dtype} != {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if ndim is not None and t.dim() != ndim:
        raise ValueError(f"{name} must have {ndim} dimensions, has {t.dim()}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} shape {tuple(t.shape)} != {tuple(shape)}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} holds {t.numel()} elements, needs {numel}")
    if min_numel is not None and t.numel() < min_numel:
        raise ValueError(
            f"{name} holds {t.numel()} elements, needs at least {min_numel}")
    if cuda and not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def require_state(t, spec, name, dtype, cuda=True):
    """Raise unless t is a state tensor of spec: dtype, shape state_shape,
    element strides state_strides (plain contiguity when the planes are not
    padded) and a buffer that holds the whole span; then the device."""
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} dtype {t.dtype} != {dtype}")
    if tuple(t.shape) != tuple(spec.state_shape):
        raise ValueError(f"{name} shape {tuple(t.shape)} != "
                         f"{tuple(spec.state_shape)}")
    if spec.pitch == spec.sites:
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
    else:
        if tuple(t.stride()) != tuple(spec.state_strides):
            raise ValueError(f"{name} strides {tuple(t.stride())} != "
                             f"{tuple(spec.state_strides)} (plane pitch "
                             f"{spec.pitch})")
        have = t.untyped_storage().nbytes() // t.element_size() - \
            t.storage_offset()
        if have < spec.state_span:
            raise ValueError(f"{name} buffer holds {have} elements, the "
                             f"padded state spans {spec.state_span}")
    if cuda and not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def require_cuda(**tensors):
    """Raise unless every named tensor lives on the GPU (checked after the
    sizes of all of them, so that a size error is reported first)."""
    for name, t in tensors.items():
        if t is not None and not t.is_cuda:
            raise TypeError(f"{name} must be a CUDA tensor")


class Lattice:
    """Handle over ``lattice_t``: owns the library's scratch buffer.

    ``f`` and ``u`` are CUDA (HIP) torch tensors in the library's layouts
    (see ``include/lattice.h``); their dtype must match ``spec.dtype``.
    Work is queued on ``stream`` (default: torch's current stream at
    construction).
    """

    def __init__(self, spec: LatticeSpec, stream=None):
        torch = _torch()
        self._L = None
        self.lib = load_library()
        self.spec = spec
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        d = _desc(spec, stream)
        h = ctypes.c_void_p()
        self._check(self.lib.lattice_init(ctypes.byref(d), ctypes.byref(h)))
        self._L = h
        self.torch_dtype = torch.float64 if spec.dtype == "f64" else torch.float32

    # -- helpers ---------------------------------------------------------
    def _check(self, rc: int):
        if rc != OK:
            msg = self.lib.lattice_strerror(rc).decode()
            if self._L is not None:
                detail = self.lib.lattice_last_error(self._L).decode()
                if detail:
                    msg = f"{msg} ({detail})"
            raise LatticeError(rc, msg)
        return rc

    def _tensor_ptr(self, t, shape=None, name="tensor", cuda=True):
        return require_tensor(t, name, self.torch_dtype, shape=shape,
                              cuda=cuda)

    def _state_ptr(self, t, name="f", cuda=True):
        return require_state(t, self.spec, name, self.torch_dtype, cuda=cuda)

    # -- API -------------------------------------------------------------
    def step(self, f, u, tau_p: float, kappa: float, dt: float, nsteps: int,
             check: bool = True):
        """Advance f in place by nsteps steps (asynchronous).

        u holds one or more slices ([slices, dim, ny, nx] or
        [slices, 1, nx] in 1D)."""
        return self._advance("lattice_step", f, u, tau_p, kappa, dt, nsteps,
                             check)

    def collide(self, f, u, tau_p: float, kappa: float, dt: float,
                nsteps: int = 1, check: bool = True):
        """The collision part of step() alone (no streaming, no learned
        correction)."""
        return self._advance("lattice_collide", f, u, tau_p, kappa, dt,
                             nsteps, check)

    def _advance(self, fn, f, u, tau_p, kappa, dt, nsteps, check):
        s = self.spec
        fp = self._state_ptr(f, "f", cuda=False)
        per = s.dim * s.nx * (s.ny if s.dim == 2 else 1)
        up = self._tensor_ptr(u, None, "u", cuda=False)
        if u.numel() % per or u.numel() == 0:
            raise ValueError("u is not a whole number of slices")
        require_cuda(f=f, u=u)
        rc = getattr(self.lib, fn)(self._L, fp, up, u.numel() // per, float(tau_p), float(kappa),
                float(dt), int(nsteps))
        if check:
            self._check(rc)
        return rc

    def moments(self, f, dt: float) -> dict:
        """FP64 mass / momentum / second moment / variance (synchronous)."""
        fp = self._state_ptr(f, "f")
        m = Moments()
        rc = self.lib.lattice_moments(self._L, fp, float(dt), ctypes.byref(m))
        out = {
            "mass": m.mass,
            "momentum": list(m.momentum)[: self.spec.dim],
            "second_moment": list(m.second_moment)[: self.spec.dim],
            "variance": m.variance,
            "nonfinite": bool(m.nonfinite),
            "rc": rc,
        }
        if rc not in (OK,):
            self._check(rc)
        return out

    def density(self, f, dt: float):
        """rho(x) = dv^dim sum_j f as a new FP64 CUDA tensor [ny, nx]."""
        torch = _torch()
        s = self.spec
        fp = self._state_ptr(f, "f")
        rho = torch.empty((s.ny if s.dim == 2 else 1, s.nx),
                          dtype=torch.float64, device=f.device)
        self._check(self.lib.lattice_density(self._L, fp, float(dt),
                                             ctypes.c_void_p(rho.data_ptr())))
        return rho

    def flow_from_modes(self, coef, out=None):
        """u slices synthesised on the device from a mode table (FP32 CUDA
        tensor): 1D [slices, K, 2] (a_k, b_k); 2D [slices, 2K+1, K+1, 2]
        (streamfunction amplitudes).  Returns [slices, dim, ny, nx] (2D) or
        [slices, 1, nx] (1D) in the lattice dtype."""
        torch = _torch()
        s = self.spec
        require_tensor(coef, "coef", torch.float32, ndim=3 if s.dim == 1 else 4)
        if coef.shape[-1] != 2:
            raise ValueError("coef must end in (cos, sin) pairs")
        if s.dim == 2 and coef.shape[1] != 2 * (coef.shape[2] - 1) + 1:
            raise ValueError("2D coef must be [slices, 2K+1, K+1, 2]")
        ns = coef.shape[0]
        dt = torch.float64 if s.dtype == "f64" else torch.float32
        shape = (ns, 2, s.ny, s.nx) if s.dim == 2 else (ns, 1, s.nx)
        if out is None:
            out = torch.empty(shape, dtype=dt, device=coef.device)
        require_tensor(out, "out", dt, shape=shape)
        if s.dim == 1:
            rc = self.lib.lattice_flow1d_modes(self._L, coef.shape[1],
                                               _ptr(coef), ns, _ptr(out))
        else:
            K = coef.shape[2] - 1
            rc = self.lib.lattice_flow2d_modes(self._L, K, _ptr(coef), ns,
                                               _ptr(out))
        self._check(rc)
        return out

    def s1(self, f, dt: float, r):
        """S1(r) of Eq. 11 for separations r (sites) as a numpy array."""
        import numpy as np
        rr = np.ascontiguousarray(np.asarray(r, dtype=np.int32))
        out = np.empty(rr.size, dtype=np.float64)
        self._check(self.lib.lattice_s1(
            self._L, self._state_ptr(f, "f"),
            float(dt), int(rr.size),
            rr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def rho_r2(self, rho, levels: int):
        """<rho_r^2> on tilings r = 2^k sites, k < levels (numpy array),
        from an FP64 density tensor such as density() returns."""
        import numpy as np
        require_tensor(rho, "rho", _torch().float64,
                       numel=self.spec.nx * (self.spec.ny
                                             if self.spec.dim == 2 else 1))
        out = np.empty(levels, dtype=np.float64)
        self._check(self.lib.lattice_rho_r2(
            self._L, ctypes.c_void_p(rho.data_ptr()), int(levels),
            out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def stability(self, u, tau_p: float, kappa: float, dt: float):
        """(CFL of Eq. 3, kappa dt_s / dv^2 of Eq. 4) for the slices in u."""
        s = self.spec
        per = s.dim * s.nx * (s.ny if s.dim == 2 else 1)
        up = self._tensor_ptr(u, None, "u")
        if u.numel() % per or u.numel() == 0:
            raise ValueError("u is not a whole number of slices")
        out = (ctypes.c_double * 2)()
        self._check(self.lib.lattice_stability(
            self._L, up, u.numel() // per,
            float(tau_p), float(kappa), float(dt), out))
        return out[0], out[1]

    def copy_state(self, dst, src):
        dp = self._state_ptr(dst, "dst", cuda=False)
        sp = self._state_ptr(src, "src", cuda=False)
        require_cuda(dst=dst, src=src)
        self._check(self.lib.lattice_copy_state(self._L, dp, sp))

    def sync(self, check: bool = True) -> int:
        rc = self.lib.lattice_sync(self._L)
        if check:
            self._check(rc)
        return rc

    def profile(self, enable: bool):
        self._check(self.lib.lattice_profile(self._L, 1 if enable else 0))

    def profile_read(self):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        self._check(self.lib.lattice_profile_read(self._L, ctypes.byref(ms),
                                                  ctypes.byref(n)))
        return ms.value, n.value

    def close(self):
        if self._L is not None:
            self.lib.lattice_destroy(self._L)
            self._L = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


@dataclass
class Member:
    """One realization of a batch (mirrors ``lattice_member_desc``)."""
    nx: int
    nv: int
    dx: float
    dt: float
    tau_p: float
    kappa: float
    u_hold: int = 0
    n_u_slices: int = 1


class Batch:
    """Handle over ``lattice_batch_t``: many independent 1D lattices (FP32)
    packed in one state buffer and advanced together."""

    CAPS = (9, 17, 33, 65, 129)

    def __init__(self, members, scheme: str = "koren", vstride: int = 1,
                 stream=None):
        torch = _torch()
        self._B = None
        self.lib = load_library()
        self.members = list(members)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        arr = (MemberDesc * len(self.members))()
        for i, m in enumerate(self.members):
            arr[i] = MemberDesc(m.nx, m.nv, m.dx, m.dt, m.tau_p, m.kappa,
                                m.u_hold, m.n_u_slices)
        h = ctypes.c_void_p()
        rc = self.lib.lattice_batch_init(arr, len(self.members),
                                         SCHEMES[scheme], vstride,
                                         ctypes.c_void_p(stream.cuda_stream),
                                         ctypes.byref(h))
        if rc != OK:
            raise LatticeError(rc, strerror(rc))
        self._B = h
        n = len(self.members)
        fo = (ctypes.c_int64 * n)()
        uo = (ctypes.c_int64 * n)()
        tc, tu = ctypes.c_int64(), ctypes.c_int64()
        self._check(self.lib.lattice_batch_layout(h, fo, uo, ctypes.byref(tc),
                                                  ctypes.byref(tu)))
        pt = (ctypes.c_int64 * n)()
        cells = ctypes.c_int64()
        self._check(self.lib.lattice_batch_plane_pitch(h, pt,
                                                       ctypes.byref(cells)))
        self.f_off = list(fo)
        self.u_off = list(uo)
        self.pitch = list(pt)
        self.total_elems = tc.value  # packed state elements (padding too)
        self.total_cells = cells.value  # lattice cells
        self.total_u = tu.value

    def _check(self, rc):
        if rc != OK:
            msg = strerror(rc)
            if self._B is not None:
                d = self.lib.lattice_batch_last_error(self._B).decode()
                if d:
                    msg = f"{msg} ({d})"
            raise LatticeError(rc, msg)
        return rc

    def pack_state(self, states):
        """Place per-member [nv, nx] arrays into one packed vector (each
        velocity plane at its member's pitch; padding zero)."""
        import numpy as np
        out = np.zeros(self.total_elems, dtype=np.float32)
        for m, o, p, a in zip(self.members, self.f_off, self.pitch, states):
            out[o:o + m.nv * p].reshape(m.nv, p)[:, :m.nx] = \
                np.asarray(a, np.float32).reshape(m.nv, m.nx)
        return out

    def unpack_state(self, flat):
        """Per-member [nv, nx] views of a packed state."""
        return [flat[o:o + m.nv * p].reshape(m.nv, p)[:, :m.nx]
                for m, o, p in zip(self.members, self.f_off, self.pitch)]

    def pack_flow(self, flows):
        import numpy as np
        out = np.empty(self.total_u, dtype=np.float32)
        for m, o, a in zip(self.members, self.u_off, flows):
            out[o:o + m.n_u_slices * m.nx] = np.asarray(a, np.float32).ravel()
        return out

    def tune(self, cap: int, block: int, grid_per_cu: int):
        self._check(self.lib.lattice_batch_tune(self._B, cap, block,
                                                grid_per_cu))

    def schedule(self, mode: int, grid_per_cu: int = 0, chunk: int = 0,
                 wait_limit: int = 0):
        """PER_STEP (launches per step and class) or RESIDENT (one launch
        per call, per-member step barriers on device counters, members
        split among the XCDs)."""
        self._check(self.lib.lattice_batch_schedule(
            self._B, int(mode), int(grid_per_cu), int(chunk),
            int(wait_limit)))

    def step(self, f, u, nsteps: int, graph_steps: int = 0):
        """Advance every member by nsteps (asynchronous); graph_steps > 0
        replays a captured HIP graph of that many (even) steps (per-step
        schedule only).  f: packed
        FP32 state of total_elems elements; u: packed FP32 flows of at
        least total_u elements."""
        torch = _torch()
        fp = require_tensor(f, "f", torch.float32, numel=self.total_elems,
                            cuda=False)
        up = require_tensor(u, "u", torch.float32, min_numel=self.total_u,
                            cuda=False)
        require_cuda(f=f, u=u)
        self._check(self.lib.lattice_batch_step(
            self._B, fp, up, int(nsteps), 1 if graph_steps else 0,
            int(graph_steps)))

    def moments(self, f):
        import numpy as np
        fp = require_tensor(f, "f", _torch().float32, numel=self.total_elems)
        out = (ctypes.c_double * (6 * len(self.members)))()
        self._check(self.lib.lattice_batch_moments(self._B, fp, out))
        return np.array(out).reshape(len(self.members), 6)

    def sync(self, check: bool = True):
        import numpy as np
        fl = (ctypes.c_int32 * len(self.members))()
        rc = self.lib.lattice_batch_sync(self._B, fl)
        if check:
            self._check(rc)
        return rc, np.array(fl)

    def close(self):
        if self._B is not None:
            self.lib.lattice_batch_destroy(self._B)
            self._B = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def restrict(f_fine, dim: int, stream=None):
    """Mass-conservative fine -> coarse (stride 4) restriction on the GPU;
    f_fine [nv_f^dim, ...] FP32 CUDA tensor; returns a new coarse tensor."""
    torch = _torch()
    L = load_library()
    if dim not in (1, 2):
        raise ValueError("dim must be 1 or 2")
    require_tensor(f_fine, "f_fine", torch.float32, cuda=False)
    nvf = int(round(f_fine.shape[0] ** (1.0 / dim))) if f_fine.dim() else 0
    if nvf < 5 or nvf ** dim != f_fine.shape[0] or (nvf - 1) % 4:
        raise ValueError("f_fine must be [nv_f^dim, ...] with nv_f = 4k + 1")
    require_cuda(f_fine=f_fine)
    nvc = (nvf - 1) // 4 + 1
    sites = f_fine.numel() // f_fine.shape[0]
    out = torch.empty((nvc ** dim,) + tuple(f_fine.shape[1:]),
                      dtype=torch.float32, device=f_fine.device)
    s = stream or torch.cuda.current_stream()
    rc = L.lattice_restrict(dim, sites, nvf, _ptr(f_fine), _ptr(out),
                            ctypes.c_void_p(s.cuda_stream))
    if rc != OK:
        raise LatticeError(rc, strerror(rc))
    return out


class Mlp:
    """The face-flux correction network (``lattice_mlp_t``)."""

    def __init__(self, stream=None):
        torch = _torch()
        self._M = None
        self.lib = load_library()
        self.stream = stream or torch.cuda.current_stream()
        h = ctypes.c_void_p()
        rc = self.lib.lattice_mlp_create(ctypes.c_void_p(self.stream.cuda_stream),
                                         ctypes.byref(h))
        if rc != OK:
            raise LatticeError(rc, strerror(rc))
        self._M = h

    def _check(self, rc):
        if rc != OK:
            raise LatticeError(rc, strerror(rc))

    def set_params(self, p):
        import numpy as np
        a = np.ascontiguousarray(np.asarray(p, dtype=np.float32).ravel())
        assert a.size == MLP_NPARAMS
        self._check(self.lib.lattice_mlp_set_params(
            self._M, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    def get_params(self):
        import numpy as np
        a = np.empty(MLP_NPARAMS, dtype=np.float32)
        self._check(self.lib.lattice_mlp_get_params(
            self._M, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return a

    @staticmethod
    def _samples_ptrs(X, t=None, w=None):
        """Pointers of a sample set: X [n, 8], t [n], w [n], FP32 CUDA."""
        torch = _torch()
        require_tensor(X, "X", torch.float32, ndim=2, cuda=False)
        n = X.shape[0]
        if X.shape[1] != 8:
            raise ValueError(f"X must be [n, 8], is {tuple(X.shape)}")
        ptrs = [_ptr(X)]
        for name, v in (("t", t), ("w", w)):
            if v is not None:
                ptrs.append(require_tensor(v, name, torch.float32, numel=n,
                                           cuda=False))
        require_cuda(X=X, t=t, w=w)
        return n, ptrs

    def grad(self, X, t, w):
        torch = _torch()
        n, (xp, tp, wp) = self._samples_ptrs(X, t, w)
        g = torch.empty(MLP_NPARAMS, dtype=torch.float32, device=X.device)
        loss = ctypes.c_double()
        self._check(self.lib.lattice_mlp_grad(self._M, xp, tp, wp, n, _ptr(g),
                                              ctypes.byref(loss)))
        return loss.value, g

    def train(self, X, t, w, batch: int, steps: int, lr: float):
        n, (xp, tp, wp) = self._samples_ptrs(X, t, w)
        loss = ctypes.c_double()
        self._check(self.lib.lattice_mlp_train(self._M, xp, tp, wp, n,
                                               int(batch), int(steps),
                                               float(lr), ctypes.byref(loss)))
        return loss.value

    def forward(self, X):
        torch = _torch()
        n, (xp,) = self._samples_ptrs(X)
        y = torch.empty(n, dtype=torch.float32, device=X.device)
        self._check(self.lib.lattice_mlp_forward(self._M, xp, n, _ptr(y)))
        return y

    @staticmethod
    def _sites_ptr(sites, nsites):
        """Site indices: int32 CUDA tensor with every value in [0, nsites)
        (the sample kernels index the state with them)."""
        torch = _torch()
        require_tensor(sites, "sites", torch.int32, ndim=1, cuda=False)
        if sites.numel() == 0:
            raise ValueError("sites is empty")
        lo, hi = int(sites.min()), int(sites.max())
        if lo < 0 or hi >= nsites:
            raise ValueError(f"site indices must lie in [0, {nsites}), "
                             f"got [{lo}, {hi}]")
        return require_tensor(sites, "sites", torch.int32)

    def samples(self, lat, dt, tau_p, St, f_pred, f_true, u, sites,
                rel_eps: float = 0.0):
        """Training samples at the given sites (int32 CUDA tensor); faces
        with stencil mass below rel_eps x site mass get zero weight."""
        torch = _torch()
        s = lat.spec
        if s.dim != 2 or s.nv != 17 or s.dtype != "f32":
            raise ValueError("samples need a 2D FP32 lattice of 17^2 "
                             "velocities")
        nsites = s.nx * s.ny
        pp = require_tensor(f_pred, "f_pred", torch.float32,
                            shape=s.state_shape, cuda=False)
        tp = require_tensor(f_true, "f_true", torch.float32,
                            shape=s.state_shape, cuda=False)
        up = require_tensor(u, "u", torch.float32, min_numel=2 * nsites,
                            cuda=False)
        require_cuda(f_pred=f_pred, f_true=f_true, u=u)
        sp = self._sites_ptr(sites, nsites)
        nf = 544
        n = sites.numel() * nf
        X = torch.empty((n, 8), dtype=torch.float32, device=f_pred.device)
        t = torch.empty(n, dtype=torch.float32, device=f_pred.device)
        w = torch.empty(n, dtype=torch.float32, device=f_pred.device)
        self._check(self.lib.lattice_mlp_samples(
            lat._L, float(dt), float(tau_p), float(St), float(rel_eps),
            pp, tp, up, sp, sites.numel(), _ptr(X), _ptr(t), _ptr(w)))
        return X, t, w

    def samples_natural(self, fine, lat, dt, tau_p, kappa, St, f_fine,
                        f_pred, u, sites, rel_eps: float = 0.0):
        """Training samples with natural flux targets at the given sites:
        f_fine = the fine state after streaming (before its collision),
        f_pred = the coarse collision of its restriction (lattice lat)."""
        torch = _torch()
        s, sf = lat.spec, fine.spec
        if s.dim != 2 or s.nv != 17 or s.dtype != "f32":
            raise ValueError("samples need a 2D FP32 lattice of 17^2 "
                             "velocities")
        if (sf.dim, sf.nx, sf.ny, sf.nv, sf.dtype) != (2, s.nx, s.ny, 65,
                                                       "f32"):
            raise ValueError("the fine lattice must be 2D FP32 65^2 on the "
                             "same sites")
        nsites = s.nx * s.ny
        fp = require_tensor(f_fine, "f_fine", torch.float32,
                            shape=sf.state_shape, cuda=False)
        pp = require_tensor(f_pred, "f_pred", torch.float32,
                            shape=s.state_shape, cuda=False)
        up = require_tensor(u, "u", torch.float32, min_numel=2 * nsites,
                            cuda=False)
        require_cuda(f_fine=f_fine, f_pred=f_pred, u=u)
        sp = self._sites_ptr(sites, nsites)
        nf = 544
        n = sites.numel() * nf
        X = torch.empty((n, 8), dtype=torch.float32, device=f_pred.device)
        t = torch.empty(n, dtype=torch.float32, device=f_pred.device)
        w = torch.empty(n, dtype=torch.float32, device=f_pred.device)
        self._check(self.lib.lattice_mlp_samples_natural(
            fine._L, lat._L, float(dt), float(tau_p), float(kappa), float(St),
            float(rel_eps), fp, pp, up, sp, sites.numel(), _ptr(X), _ptr(t),
            _ptr(w)))
        return X, t, w

    def attach(self, lat, St: float, line_eps: float = 1e-4):
        self._check(self.lib.lattice_mlp_attach(lat._L, self._M, float(St),
                                                float(line_eps)))

    @staticmethod
    def detach(lat):
        rc = load_library().lattice_mlp_attach(lat._L, None, 1.0, 0.0)
        if rc != OK:
            raise LatticeError(rc, strerror(rc))

    def close(self):
        if self._M is not None:
            self.lib.lattice_mlp_destroy(self._M)
            self._M = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def strerror(code: int) -> str:
    return load_library().lattice_strerror(code).decode()


def _desc(spec: LatticeSpec, stream=None) -> Desc:
    """The C descriptor of a LatticeSpec."""
    L = load_library()
    d = Desc()
    L.lattice_desc_default(ctypes.byref(d))
    d.dim, d.nx, d.ny, d.nv = spec.dim, spec.nx, spec.ny, spec.nv
    d.vstride, d.dx = spec.vstride, spec.dx
    d.scheme = SCHEMES[spec.scheme]
    d.dtype = F64 if spec.dtype == "f64" else F32
    d.nsub, d.u_hold = spec.nsub, spec.u_hold
    d.plane_pitch = spec.plane_pitch
    if stream is not None:
        d.stream = ctypes.c_void_p(stream.cuda_stream)
    return d


def recommended_pitch(spec: LatticeSpec) -> int:
    """The plane pitch the library recommends for this lattice
    (lattice_plane_pitch): nx*ny, or padded when a plane spans a multiple
    of 64 KiB."""
    p = ctypes.c_int64()
    rc = load_library().lattice_plane_pitch(ctypes.byref(_desc(spec)),
                                            ctypes.byref(p))
    if rc != OK:
        raise LatticeError(rc, strerror(rc))
    return p.value


def step_noalloc(spec: LatticeSpec, f, u, tau_p: float, kappa: float,
                 dt: float, nsteps: int, status=None, stream=None) -> int:
    """lattice_step_noalloc: advance f in place without a handle and without
    any device allocation (the library's static scratch holds the state's
    twin; states up to NOALLOC_MAX_BYTES).  status: optional int32 CUDA
    tensor of one element that receives 0 (all steps ran) or nonzero (the
    CFL check failed; the call's steps were no-ops).  Asynchronous on
    ``stream`` (default: torch's current stream).  Returns the library's
    return code after raising for any code but OK."""
    torch = _torch()
    dtype = torch.float64 if spec.dtype == "f64" else torch.float32
    fp = require_state(f, spec, "f", dtype, cuda=False)
    per = spec.dim * spec.nx * (spec.ny if spec.dim == 2 else 1)
    up = require_tensor(u, "u", dtype, cuda=False)
    if u.numel() % per or u.numel() == 0:
        raise ValueError("u is not a whole number of slices")
    sp = None
    if status is not None:
        sp = require_tensor(status, "status", torch.int32, numel=1,
                            cuda=False)
    require_cuda(f=f, u=u, status=status)
    if stream is None:
        stream = torch.cuda.current_stream()
    d = _desc(spec, stream)
    rc = load_library().lattice_step_noalloc(
        ctypes.byref(d), fp, up, u.numel() // per, float(tau_p),
        float(kappa), float(dt), int(nsteps), sp)
    if rc != OK:
        raise LatticeError(rc, strerror(rc))
    return rc


def rho_r2_error(a, b, dx: float) -> float:
    """Distance-averaged relative error of <rho_r^2>_a against <rho_r^2>_b
    on the tiling scales r = 2^k dx (lattice_rho_r2_error)."""
    import numpy as np
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    b = np.ascontiguousarray(np.asarray(b, dtype=np.float64))
    if a.shape != b.shape or a.ndim != 1:
        raise ValueError("a and b must be 1-D arrays of one length")
    out = ctypes.c_double()
    pd = ctypes.POINTER(ctypes.c_double)
    rc = load_library().lattice_rho_r2_error(a.ctypes.data_as(pd),
                                             b.ctypes.data_as(pd), a.size,
                                             float(dx), ctypes.byref(out))
    if rc != OK:
        raise LatticeError(rc, strerror(rc))
    return out.value


def velocity(spec: LatticeSpec, dt: float):
    """(dv, Vmax) computed by the library (host-only call)."""
    L = load_library()
    d = Desc()
    L.lattice_desc_default(ctypes.byref(d))
    d.dim, d.nx, d.ny, d.nv, d.vstride, d.dx = (spec.dim, spec.nx, spec.ny,
                                                spec.nv, spec.vstride, spec.dx)
    dv, vmax = ctypes.c_double(), ctypes.c_double()
    rc = L.lattice_velocity(ctypes.byref(d), float(dt), ctypes.byref(dv),
                            ctypes.byref(vmax))
    if rc != OK:
        raise LatticeError(rc, strerror(rc))
    return dv.value, vmax.value


__all__ = ["Lattice", "LatticeSpec", "LatticeError", "LatticeLibraryMissing",
           "require_tensor", "require_cuda", "require_state",
           "recommended_pitch",
           "Batch", "Member", "Mlp", "restrict", "load_library", "strerror",
           "velocity", "step_noalloc", "rho_r2_error", "EXPORTS", "MLP_NPARAMS",
           "NOALLOC_MAX_BYTES"]
