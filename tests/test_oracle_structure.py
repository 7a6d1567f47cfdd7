"""Pins of the structure-function oracle (oracle/structure.py): closed
forms for simple velocity distributions and brute force on tiny arrays."""
import math

import numpy as np
import pytest

from oracle import structure as S


def test_single_velocity_gives_zero():
    f = np.zeros((5, 16))
    f[3] = 1.0 + np.arange(16) % 3
    assert np.allclose(S.s1(f, 1, 0.5, [0, 1, 5]), 0.0)


def test_1d_two_velocities_closed_form():
    """Equal mass at v = +-a everywhere: E|v - v'| = a for every r."""
    nv, dv = 9, 0.25
    f = np.zeros((nv, 12))
    f[1] = f[7] = 1.0           # v = -3 dv and +3 dv
    a = 3 * dv
    assert np.allclose(S.s1(f, 1, dv, [0, 2, 7]), a)


def test_2d_four_velocities_closed_form():
    """Equal mass at (+-a, 0), (0, +-a): pairs equal (1/4) -> 0, opposite
    (1/4) -> 2a, perpendicular (1/2) -> sqrt(2) a."""
    nv, dv, n = 5, 0.5, 6
    f = np.zeros((nv * nv, n, n))
    c = 2
    for jy, jx in [(c, c + 2), (c, c - 2), (c + 2, c), (c - 2, c)]:
        f[jy * nv + jx] = 1.0
    a = 2 * dv
    want = 0.25 * 2 * a + 0.5 * math.sqrt(2) * a
    assert np.allclose(S.s1(f, 2, dv, [0, 1, 3]), want)


def test_brute_force_1d_and_2d():
    rng = np.random.default_rng(70)
    f1 = rng.random((4, 6))
    dv = 0.3
    v = (np.arange(4) - 1) * dv  # h = (nv - 1) // 2 = 1
    for r in (0, 2, 5):
        num = den = 0.0
        for x in range(6):
            for j in range(4):
                for k in range(4):
                    w = f1[j, x] * f1[k, (x + r) % 6]
                    num += w * abs(v[j] - v[k])
                    den += w
        assert S.s1(f1, 1, dv, [r])[0] == pytest.approx(num / den, rel=1e-12)
    nv, n = 3, 4
    f2 = rng.random((nv * nv, n, n))
    vv = (np.arange(nv) - 1) * dv
    for r in (1, 2):
        est = []
        for axis in ("x", "y"):
            num = den = 0.0
            for y in range(n):
                for x in range(n):
                    xs, ys = ((x + r) % n, y) if axis == "x" else (x, (y + r) % n)
                    for J in range(nv * nv):
                        for K in range(nv * nv):
                            w = f2[J, y, x] * f2[K, ys, xs]
                            dvx = vv[J % nv] - vv[K % nv]
                            dvy = vv[J // nv] - vv[K // nv]
                            num += w * math.hypot(dvx, dvy)
                            den += w
            est.append(num / den)
        assert S.s1(f2, 2, dv, [r])[0] == pytest.approx(np.mean(est), rel=1e-12)
