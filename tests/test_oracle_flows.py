"""Pins of the flow-synthesis oracle (oracle/flows.py): closed forms of
single modes, the independent inverse-FFT evaluation of the same tables,
and incompressibility of the 2D flows."""
import math

import numpy as np

from oracle import flows as F
from paper_1508_02899_amd import inputs


def test_1d_single_modes():
    nx = 16
    tab = np.zeros((2, 3, 2))
    tab[0, 2, 0] = 1.5   # 1.5 cos(3 x)
    tab[1, 0, 1] = -2.0  # -2 sin(x)
    x = 2 * np.pi * np.arange(nx) / nx
    u = F.flow1d(tab, nx)
    assert np.allclose(u[0, 0], 1.5 * np.cos(3 * x))
    assert np.allclose(u[1, 0], -2.0 * np.sin(x))


def test_2d_single_mode_by_hand():
    """psi = Re(c e^{i(2x + 3y)}) with c = 1 - 2i, L = 2 pi:
    psi = cos(2x + 3y) + 2 sin(2x + 3y); u = d_y psi, v = -d_x psi."""
    n, K = 16, 4
    tab = np.zeros((1, 2 * K + 1, K + 1, 2))
    tab[0, K + 3, 2] = [1.0, -2.0]
    x = 2 * np.pi * np.arange(n) / n
    X, Y = np.meshgrid(x, x)
    th = 2 * X + 3 * Y
    u = F.flow2d(tab, n, n, 2 * np.pi / n)
    assert np.allclose(u[0, 0], 3 * (-np.sin(th) + 2 * np.cos(th)))
    assert np.allclose(u[0, 1], -2 * (-np.sin(th) + 2 * np.cos(th)))


def test_2d_tables_match_inverse_fft_flows():
    n, L = 32, 2 * math.pi
    kw = dict(kmax=8, seed=7, dt=0.3)
    tab = inputs.flow2d_modes(n, L, 4, **kw)
    u_fft = inputs.flow2d_streamfunction(n, L, 4, dtype=np.float64, **kw)
    u = F.flow2d(tab, n, n, L / n)
    assert np.abs(u - u_fft).max() < 1e-6 * np.abs(u_fft).max()
    # the tables carry the r.m.s. normalisation
    assert abs(np.sqrt(np.mean(u ** 2)) - 1.0) < 1e-6


def test_2d_flows_are_divergence_free():
    n, L = 32, 2 * math.pi
    u = F.flow2d(inputs.flow2d_modes(n, L, 2, kmax=10, seed=9), n, n, L / n)
    k = np.fft.fftfreq(n, d=1.0 / n)
    KX, KY = np.meshgrid(k, k)
    for s in range(2):
        div = KX * np.fft.fft2(u[s, 0]) + KY * np.fft.fft2(u[s, 1])
        assert np.abs(div).max() < 1e-9 * np.abs(np.fft.fft2(u[s, 0])).max()


def test_1d_tables_match_prestaged_flows():
    tab = inputs.flow1d_modes(3, modes=8, seed=5, tau_f=1.0, dt=0.2)
    u = inputs.flow1d(48, 2 * math.pi, 3, modes=8, seed=5, tau_f=1.0, dt=0.2,
                      dtype=np.float64)
    assert np.allclose(F.flow1d(tab, 48), u, atol=1e-12)
