"""FP64 CPU oracle of the phase-space lattice update -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never calls it and
shares no code with it.  The arithmetic lives in ``oracle.c`` (plain,
single-threaded C in double precision, one function per step of Sec. 2 of
Laenen, Krstulovic & Bec, arXiv:1508.02899); this module only builds that
file with gcc and marshals numpy arrays through ctypes.

Array layouts (C order): ``f[jv, y, x]`` with ``jv = jy*nv + jx`` in 2D
(``f[j, x]`` in 1D) and ``u[slice, component, y, x]`` (``u[slice, x]`` or
``u[slice, 1, x]`` in 1D).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
# ORACLE_LIB names another build of oracle.c to load instead (used by the
# mutation test, which checks that the pins catch planted mistakes)
_SO = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")

SCHEMES = {"upwind": 0, "koren": 1}

_lib = None


# the same source built with OpenMP: only the benchmark's CPU baseline loads
# it (through ORACLE_LIB, in a process of its own), to time the oracle on
# several host cores; the tests use the single-threaded build
OMP_SO = os.path.join(_HERE, "liboracle_omp.so")


def build() -> str:
    """Compile oracle.c into liboracle.so (plain -O2, no fast-math, one
    thread) and liboracle_omp.so (the same with OpenMP)."""
    for so, extra in ((os.path.join(_HERE, "liboracle.so"), []),
                      (OMP_SO, ["-fopenmp"])):
        tmp = so + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-fPIC", "-shared",
             "-Wno-unknown-pragmas", *extra, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, so)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc_drift_line.argtypes = [dp, ctypes.c_int, dp, ctypes.c_int]
        L.orc_drift_line.restype = None
        L.orc_diffuse_line.argtypes = [dp, ctypes.c_int, ctypes.c_double]
        L.orc_diffuse_line.restype = None
        L.orc_stream.argtypes = [ctypes.c_int, ctypes.c_long, ctypes.c_long,
                                 ctypes.c_int, ctypes.c_int, dp, dp]
        L.orc_stream.restype = None
        L.orc_step.argtypes = [ctypes.c_int, ctypes.c_long, ctypes.c_long,
                               ctypes.c_int, ctypes.c_int, ctypes.c_double,
                               ctypes.c_int, ctypes.c_int, ctypes.c_long, dp,
                               dp, ctypes.c_long, ctypes.c_double,
                               ctypes.c_double, ctypes.c_double, ctypes.c_long]
        L.orc_step.restype = ctypes.c_int
        L.orc_moments.argtypes = [ctypes.c_int, ctypes.c_long, ctypes.c_long,
                                  ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                  ctypes.c_double, dp, dp]
        L.orc_moments.restype = None
        L.orc_stability.argtypes = [ctypes.c_int, ctypes.c_long, ctypes.c_long,
                                    ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_int, dp, ctypes.c_long,
                                    ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, dp]
        L.orc_stability.restype = None
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def drift_line(c, nu, scheme: str = "koren") -> np.ndarray:
    """One forward-Euler drift update of a velocity line (Sec. 2).

    ``nu[j]`` is the drift of cell j in cell widths per step,
    dt (u - v_j) / (tau_p dv).
    """
    c = _f64(c).copy()
    nu = _f64(nu)
    assert c.ndim == 1 and nu.shape == c.shape
    lib().orc_drift_line(_ptr(c), c.size, _ptr(nu), SCHEMES[scheme])
    return c


def diffuse_line(c, D: float) -> np.ndarray:
    """One forward-Euler diffusion update of a velocity line (Sec. 2, Eq. 4)."""
    c = _f64(c).copy()
    lib().orc_diffuse_line(_ptr(c), c.size, float(D))
    return c


def _shape(f: np.ndarray, dim: int):
    if dim == 1:
        nv, nx = f.shape
        return nx, 1, nv
    nvv, ny, nx = f.shape
    nv = int(round(nvv ** 0.5))
    assert nv * nv == nvv
    return nx, ny, nv


def stream(f, dim: int, s: int = 1) -> np.ndarray:
    """Exact pull streaming of f by s*(j-h) cells per component (Sec. 2)."""
    f = _f64(f)
    nx, ny, nv = _shape(f, dim)
    g = np.empty_like(f)
    lib().orc_stream(dim, nx, ny, nv, s, _ptr(f), _ptr(g))
    return g


def step(f, u, *, dim: int, dx: float, tau_p: float, kappa: float, dt: float,
         nsteps: int, scheme: str = "koren", s: int = 1, nsub: int = 1,
         u_hold: int = 0) -> np.ndarray:
    """``nsteps`` full lattice time steps (S, then A, then D) from f.

    Returns the new state; the input is not modified.  ``u`` holds one or
    more slices, step k uses slice k // u_hold (slice 0 if u_hold == 0).
    """
    f = _f64(f).copy()
    nx, ny, nv = _shape(f, dim)
    u = _f64(u)
    slice_len = dim * nx * ny
    assert u.size % slice_len == 0
    nsl = u.size // slice_len
    rc = lib().orc_step(dim, nx, ny, nv, s, float(dx), SCHEMES[scheme],
                        int(nsub), int(u_hold), _ptr(f), _ptr(u), nsl,
                        float(tau_p), float(kappa), float(dt), int(nsteps))
    if rc != 0:
        raise ValueError("oracle: invalid arguments")
    return f


def moments(f, *, dim: int, dx: float, dt: float, s: int = 1) -> dict:
    """Mass, momentum, second moment and velocity variance of f."""
    f = _f64(f)
    nx, ny, nv = _shape(f, dim)
    out = np.zeros(1 + 2 * dim + 1)
    lib().orc_moments(dim, nx, ny, nv, s, float(dx), float(dt), _ptr(f),
                      _ptr(out))
    return {
        "mass": out[0],
        "momentum": out[1:1 + dim].copy(),
        "second_moment": out[1 + dim:1 + 2 * dim].copy(),
        "variance": out[1 + 2 * dim],
    }


def stability(u, *, dim: int, nx: int, ny: int, nv: int, dx: float,
              tau_p: float, kappa: float, dt: float, s: int = 1,
              nsub: int = 1):
    """(CFL of Eq. 3, kappa dt/dv^2 of Eq. 4) for the given u slices."""
    u = _f64(u)
    if dim == 1:
        ny = 1
    nsl = u.size // (dim * nx * ny)
    out = np.zeros(2)
    lib().orc_stability(dim, nx, ny, nv, s, float(dx), int(nsub), _ptr(u), nsl,
                        float(tau_p), float(kappa), float(dt), _ptr(out))
    return float(out[0]), float(out[1])
