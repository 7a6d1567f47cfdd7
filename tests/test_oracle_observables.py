"""Pins of the density-observable oracle (oracle/observables.py) against
closed forms and brute force: the coarse-grained density of Sec. 3.1-3.2
on tilings, its second moment (Sec. 4.2.1) and the distance-averaged
error of Sec. 4.2.1."""
import itertools

import numpy as np
import pytest

from oracle import observables as O


def test_uniform_density_gives_one():
    assert np.allclose(O.rho_r2(np.full((16, 32), 3.7), 5), 1.0)
    assert np.allclose(O.rho_r2(np.full(64, 0.2), 7), 1.0)


def test_point_mass_gives_box_count():
    """All mass in one site: <rho_r^2> = N_b, the number of boxes."""
    rho = np.zeros((16, 32))
    rho[5, 9] = 2.5
    got = O.rho_r2(rho, 4)
    want = [16 * 32 / 4 ** k for k in range(4)]
    assert np.allclose(got, want)
    r1 = np.zeros(64)
    r1[17] = 1.0
    assert np.allclose(O.rho_r2(r1, 6), [64 / 2 ** k for k in range(6)])


def test_checkerboard():
    """Alternating 0 / 2: <rho^2> = 2 on single sites, 1 on every coarser
    tiling (each 2x2 or 2-site box holds the mean mass)."""
    y, x = np.mgrid[0:8, 0:8]
    rho = 2.0 * ((x + y) % 2)
    assert np.allclose(O.rho_r2(rho, 3), [2.0, 1.0, 1.0])
    r1 = 2.0 * (np.arange(16) % 2)
    assert np.allclose(O.rho_r2(r1, 4), [2.0, 1.0, 1.0, 1.0])


def test_brute_force_small():
    rng = np.random.default_rng(4)
    rho = rng.random((4, 8))
    M = rho.sum()
    for k, got in enumerate(O.rho_r2(rho, 3)):
        b = 2 ** k
        boxes = []
        for by, bx in itertools.product(range(4 // b), range(8 // b)):
            m = sum(rho[by * b + i, bx * b + j]
                    for i in range(b) for j in range(b))
            boxes.append(m / M * (32 // (b * b)))
        assert got == pytest.approx(np.mean(np.square(boxes)), rel=1e-13)


def test_density_sums_velocities():
    f = np.arange(3 * 2 * 4, dtype=float).reshape(3, 2, 4)
    assert np.allclose(O.density(f, 1, 0.5), 0.5 * f.sum(axis=0))
    assert np.allclose(O.density(f, 2, 0.5), 0.25 * f.sum(axis=0))


def test_distance_averaged_error():
    b = np.array([5.0, 3.0, 2.0, 1.5])
    assert O.distance_averaged_error(b, b, 0.1) == 0.0
    assert O.distance_averaged_error(1.03 * b, b, 0.1) == pytest.approx(0.03)
    # weights r^2: only the largest scale differs
    a = b.copy()
    a[3] += 1.0
    w = 4.0 ** np.arange(4)
    assert O.distance_averaged_error(a, b, 1.0) == pytest.approx(
        w[3] * 1.0 / np.sum(w * b))
