"""Pins of the FP64 oracle against what the paper and mathematics fix.

None of these compares the oracle with itself: each expected value is a
hand-derived worked example (tests/golden), a closed form, a library routine
(np.roll, cosine modes), an invariance, or a brute-force particle simulation
whose expectation equals the scheme.  Paper: arXiv:1508.02899, Sec. 2.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _parse_blocks(path):
    blocks, cur = [], {}
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if line.startswith("#"):
                continue
            if not line:
                if cur:
                    blocks.append(cur)
                    cur = {}
                continue
            k, v = line.split(":", 1)
            cur[k.strip()] = v.strip()
    if cur:
        blocks.append(cur)
    return blocks


def _fr(s):
    return [Fraction(t) for t in s.split()]


WORKED = _parse_blocks(os.path.join(GOLDEN, "worked_examples.txt"))


@pytest.mark.parametrize("ex", WORKED, ids=[b["name"] for b in WORKED])
def test_worked_example(ex):
    """Sec. 2 force / diffusion steps on one velocity line, exact rationals."""
    c = np.array([float(x) for x in _fr(ex["c"])])
    want = np.array([float(x) for x in _fr(ex["expect"])])
    if ex["op"] == "drift":
        nu = np.array([float(x) for x in _fr(ex["nu"])])
        got = oracle.drift_line(c, nu, ex["scheme"])
    else:
        got = oracle.diffuse_line(c, float(Fraction(ex["D"])))
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-14)
    assert abs(got.sum() - c.sum()) < 1e-14  # conservative form


def test_stationary_vector_nv5():
    """Fixed point of force-then-diffusion (Sec. 2) with u = 0, exact."""
    blk = _parse_blocks(os.path.join(GOLDEN, "stationary_nv5.txt"))[0]
    want = np.array([float(x) for x in _fr(blk["expect"])])
    nv = int(blk["nv"])
    r = Fraction(blk["dt_over_taup"])
    D = Fraction(blk["D"])
    # dx = dt = 1 -> dv = 1; dt/tau_p = r; kappa dt/dv^2 = D; nx = 1 so the
    # streaming is the identity.
    f = np.full((nv, 1), 1.0 / nv)
    u = np.zeros((1, 1))
    out = oracle.step(f, u, dim=1, dx=1.0, dt=1.0, tau_p=float(1 / r),
                      kappa=float(D), nsteps=3000, scheme="upwind")
    np.testing.assert_allclose(out[:, 0], want, rtol=0, atol=1e-13)


def test_streaming_is_exact_roll_1d():
    """tau_p = inf, kappa = 0: pure lattice streaming (Sec. 2), bit-exact."""
    rng = np.random.default_rng(1)
    nx, nv, s, nsteps = 37, 9, 1, 5
    f = rng.random((nv, nx))
    u = rng.standard_normal((1, nx))
    out = oracle.step(f, u, dim=1, dx=0.1, dt=0.05, tau_p=math.inf, kappa=0.0,
                      nsteps=nsteps)
    h = (nv - 1) // 2
    want = np.stack([np.roll(f[j], s * (j - h) * nsteps) for j in range(nv)])
    assert np.array_equal(out, want)


def test_streaming_is_exact_roll_2d_with_stride():
    rng = np.random.default_rng(2)
    nx, ny, nv, s, nsteps = 11, 7, 5, 2, 3
    f = rng.random((nv * nv, ny, nx))
    u = rng.standard_normal((1, 2, ny, nx))
    out = oracle.step(f, u, dim=2, dx=0.1, dt=0.05, tau_p=math.inf, kappa=0.0,
                      nsteps=nsteps, s=s)
    h = (nv - 1) // 2
    want = np.empty_like(f)
    for jy in range(nv):
        for jx in range(nv):
            jv = jy * nv + jx
            want[jv] = np.roll(f[jv], (s * (jy - h) * nsteps,
                                       s * (jx - h) * nsteps), axis=(0, 1))
    assert np.array_equal(out, want)


def test_streaming_worked_example_nx4_nv3():
    """Row n=+1 of (a,b,c,d) becomes (d,a,b,c); n=-1 gives (b,c,d,a)."""
    f = np.array([[1.0, 2.0, 3.0, 4.0],   # n = -1
                  [5.0, 6.0, 7.0, 8.0],   # n = 0
                  [9.0, 10.0, 11.0, 12.0]])  # n = +1
    g = oracle.stream(f, dim=1)
    assert np.array_equal(g, [[2, 3, 4, 1], [5, 6, 7, 8], [12, 9, 10, 11]])


@pytest.mark.parametrize("nv,k,D", [(9, 1, 0.1), (9, 4, 0.2), (33, 7, 0.45),
                                    (17, 16, 0.3)])
def test_diffusion_neumann_modes_decay(nv, k, D):
    """Discrete Laplacian with zero-flux faces (Sec. 2, Eq. 4): the cosine
    modes cos(pi k (j + 1/2)/nv) are eigenvectors with factor
    1 - 4 D sin^2(pi k / (2 nv))."""
    j = np.arange(nv)
    c = np.cos(np.pi * k * (j + 0.5) / nv)
    lam = 1.0 - 4.0 * D * np.sin(np.pi * k / (2 * nv)) ** 2
    got = oracle.diffuse_line(c, D)
    np.testing.assert_allclose(got, lam * c, rtol=0, atol=1e-14)


def test_koren_face_value_exact_for_quadratic_cell_averages():
    """The unlimited branch of the Koren scheme is the kappa = 1/3 (third-
    order) interpolant: for cell averages of a quadratic it returns the exact
    face value.  Constant nu, increasing convex data (limiter inactive):
    interior face k carries nu * q(k - 1/2)."""
    nv = 9
    j = np.arange(nv, dtype=float)
    q = lambda v: 0.5 * (v + 3.0) ** 2  # noqa: E731
    # cell averages over [j - 1/2, j + 1/2] of q: q(j) + q''/24
    c = q(j) + 1.0 / 24.0
    nu = np.full(nv, 0.2)
    got = oracle.drift_line(c, nu, "koren")
    # faces k = 2..nv-1 have two upwind cells inside the line, and the
    # limiter is inactive there (theta close to 1, psi = 1/3 + theta/6)
    F = np.zeros(nv + 1)
    for k in range(2, nv):
        F[k] = 0.2 * q(k - 0.5)
    # cells 2..nv-2 see only such faces
    for jj in range(2, nv - 1):
        assert got[jj] == pytest.approx(c[jj] - (F[jj + 1] - F[jj]), abs=1e-13)


def test_koren_reduces_to_upwind_on_monotone_steep_data():
    """psi(theta) = 0 when theta <= 0 (extremum): the Koren face flux equals
    the upwind one at a local maximum."""
    c = np.array([0.0, 0.0, 5.0, 0.0, 0.0])
    nu = np.full(5, 0.25)
    up = oracle.drift_line(c, nu, "upwind")
    ko = oracle.drift_line(c, nu, "koren")
    # face 3 (cells 2|3): upwind cell 2 is a maximum -> same flux; face 2:
    # upwind cell 1 has dp = 5 > 0, dm = 0 -> psi(0) = 0 -> same flux
    assert np.array_equal(up, ko)


def _random_columns(rng, n, nv):
    return rng.random((n, nv)) ** 3


def test_koren_positive_at_cfl_half():
    """With |nu| <= 1/2 the Koren update never produces negative mass."""
    rng = np.random.default_rng(3)
    nv = 9
    h = (nv - 1) // 2
    worst = 0.0
    for _ in range(3000):
        c = rng.random(nv) ** 4 * rng.integers(0, 2, nv)
        beta = rng.uniform(0.0, 0.5 / (h + 2))
        alpha = rng.uniform(-2.0, 2.0) * beta
        nu = alpha - beta * (np.arange(nv) - h)
        nu *= 0.5 / max(0.5, np.abs(nu).max())
        got = oracle.drift_line(c, nu, "koren")
        worst = min(worst, got.min() / max(c.max(), 1e-300))
    assert worst >= -1e-15


def test_upwind_positive_below_cfl_one():
    rng = np.random.default_rng(4)
    nv = 7
    for _ in range(2000):
        c = rng.random(nv) * rng.integers(0, 2, nv)
        nu = np.sort(rng.uniform(-0.99, 0.99, nv))[::-1]
        got = oracle.drift_line(c, nu, "upwind")
        assert got.min() >= -1e-15


def _rand_state(rng, dim, nx, ny, nv):
    if dim == 1:
        return rng.random((nv, nx))
    return rng.random((nv * nv, ny, nx))


@pytest.mark.parametrize("dim,scheme", [(1, "koren"), (1, "upwind"),
                                        (2, "koren"), (2, "upwind")])
def test_mass_conserved_to_roundoff(dim, scheme):
    """Conservative form (Sec. 2): fluxes telescope, mass drifts only by
    FP64 rounding (bound 1e-12 relative)."""
    rng = np.random.default_rng(5)
    nx, ny, nv = (64, 1, 17) if dim == 1 else (12, 10, 9)
    f = _rand_state(rng, dim, nx, ny, nv)
    ushape = (1, nx) if dim == 1 else (1, 2, ny, nx)
    u = 0.5 * rng.standard_normal(ushape)
    dx, dt = 2 * np.pi / nx, 0.05
    dv = dx / dt
    vmax = (nv - 1) / 2 * dv
    tau_p = 2.2 * dt * (np.abs(u).max() + vmax) / dv  # CFL ~ 0.45
    kappa = 0.2 * dv * dv / dt
    m0 = oracle.moments(f, dim=dim, dx=dx, dt=dt)["mass"]
    out = oracle.step(f, u, dim=dim, dx=dx, dt=dt, tau_p=tau_p, kappa=kappa,
                      nsteps=60 if dim == 1 else 20, scheme=scheme)
    m1 = oracle.moments(out, dim=dim, dx=dx, dt=dt)["mass"]
    assert abs(m1 - m0) / m0 <= 1e-12
    assert out.min() >= -1e-14 * out.max()


def test_translation_invariance_bit_exact():
    """Rolling f and u by k sites rolls the result by k (periodic lattice)."""
    rng = np.random.default_rng(6)
    nx, ny, nv = 9, 8, 5
    f = _rand_state(rng, 2, nx, ny, nv)
    u = 0.3 * rng.standard_normal((1, 2, ny, nx))
    kw = dict(dim=2, dx=0.2, dt=0.1, tau_p=1.5, kappa=0.02, nsteps=3)
    a = oracle.step(f, u, **kw)
    b = oracle.step(np.roll(f, (3, -2), axis=(1, 2)),
                    np.roll(u, (3, -2), axis=(2, 3)), **kw)
    assert np.array_equal(np.roll(a, (3, -2), axis=(1, 2)), b)


@pytest.mark.parametrize("scheme", ["koren", "upwind"])
def test_mirror_symmetry_1d(scheme):
    """x -> -x, v -> -v, u -> -u maps solutions to solutions (Eq. 2/5 are
    odd under the reflection); the scheme keeps it exactly."""
    rng = np.random.default_rng(7)
    nx, nv = 16, 9
    f = rng.random((nv, nx))
    u = 0.4 * rng.standard_normal((1, nx))
    kw = dict(dim=1, dx=0.2, dt=0.1, tau_p=2.0, kappa=0.01, nsteps=7,
              scheme=scheme)
    a = oracle.step(f, u, **kw)

    def mirror_x(arr):  # x -> -x on the periodic lattice: i -> (-i) mod nx
        return np.roll(arr[..., ::-1], 1, axis=-1)

    fm = mirror_x(f[::-1])
    um = -mirror_x(u)
    b = oracle.step(fm, um, **kw)
    np.testing.assert_allclose(mirror_x(b[::-1]), a, rtol=0, atol=1e-15)


def test_homogeneity_bit_exact():
    """The scheme is positively homogeneous of degree one (the Koren
    correction scales with its arguments): f -> 2f gives out -> 2 out."""
    rng = np.random.default_rng(8)
    nx, nv = 10, 7
    f = rng.random((nv, nx))
    u = 0.3 * rng.standard_normal((1, nx))
    kw = dict(dim=1, dx=0.2, dt=0.1, tau_p=2.0, kappa=0.02, nsteps=4)
    assert np.array_equal(2 * oracle.step(f, u, **kw),
                          oracle.step(2 * f, u, **kw))


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7])
def test_paper_1d_setup_cfl_threshold(n):
    """Sec. 3.2: Vmax = u_rms = 1, L = 2 pi, nv = 2^n + 1, nx = 2^(n+6),
    dt = dx/dv = 2^-6 pi, and CFL (Eq. 3) restricts nv < 1 + 128 St.
    With dv = 2 Vmax/(nv - 1) the oracle's geometry reproduces dt and Vmax,
    and its CFL number is (nv - 1)/(128 St) when max|u| = 1."""
    nv, nx = 2 ** n + 1, 2 ** (n + 6)
    L = 2 * np.pi
    dx = L / nx
    dt = np.pi / 64
    dv = dx / dt
    assert (nv - 1) / 2 * dv == pytest.approx(1.0, abs=1e-14)
    u = np.zeros((1, nx))
    u[0, 3] = -1.0
    for St in [0.05, 0.1, 0.25, 0.5, 1.0, 2.0]:
        tau_p = St * L  # St = tau_p u_rms / L
        cfl, _ = oracle.stability(u, dim=1, nx=nx, ny=1, nv=nv, dx=dx,
                                  tau_p=tau_p, kappa=0.0, dt=dt)
        assert cfl == pytest.approx((nv - 1) / (128 * St), rel=1e-12)
        assert (cfl < 1) == (nv < 1 + 128 * St)


def test_moments_closed_form_uniform():
    """f = 1 on every cell: M = L (2h+1) dv, P = 0,
    Q = L dv^3 h(h+1)(2h+1)/3 (sum of squares)."""
    nx, nv = 20, 9
    h = (nv - 1) // 2
    dx, dt = 0.3, 0.1
    dv = dx / dt
    L = nx * dx
    m = oracle.moments(np.ones((nv, nx)), dim=1, dx=dx, dt=dt)
    assert m["mass"] == pytest.approx(L * nv * dv, rel=1e-14)
    assert abs(m["momentum"][0]) < 1e-12
    Q = L * dv ** 3 * h * (h + 1) * (2 * h + 1) / 3
    assert m["second_moment"][0] == pytest.approx(Q, rel=1e-14)
    assert m["variance"] == pytest.approx(Q / (L * nv * dv), rel=1e-13)


def test_moments_closed_form_single_cell_2d():
    """Mass m in one cell (jx, jy): P = m w (vx, vy), Q = m w (vx^2, vy^2),
    variance 0 (w = dx^2 dv^2)."""
    nx, ny, nv = 4, 3, 5
    h = (nv - 1) // 2
    dx, dt = 0.5, 0.25
    dv = dx / dt
    f = np.zeros((nv * nv, ny, nx))
    jx, jy = 4, 1
    f[jy * nv + jx, 2, 3] = 3.0
    m = oracle.moments(f, dim=2, dx=dx, dt=dt)
    w = dx * dx * dv * dv
    vx, vy = (jx - h) * dv, (jy - h) * dv
    assert m["mass"] == pytest.approx(3.0 * w, rel=1e-15)
    np.testing.assert_allclose(m["momentum"], [3 * w * vx, 3 * w * vy], rtol=1e-15)
    np.testing.assert_allclose(m["second_moment"], [3 * w * vx ** 2, 3 * w * vy ** 2],
                               rtol=1e-15)
    assert abs(m["variance"]) < 1e-12


def test_u_hold_slicing():
    """Step k uses slice k // u_hold: two calls with one slice each agree
    with one call holding both slices."""
    rng = np.random.default_rng(9)
    nx, nv = 12, 5
    f = rng.random((nv, nx))
    u = 0.3 * rng.standard_normal((2, nx))
    kw = dict(dim=1, dx=0.2, dt=0.1, tau_p=2.0, kappa=0.02)
    both = oracle.step(f, u, nsteps=4, u_hold=2, **kw)
    half = oracle.step(f, u[0:1], nsteps=2, **kw)
    half = oracle.step(half, u[1:2], nsteps=2, **kw)
    assert np.array_equal(both, half)
