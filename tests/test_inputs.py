"""Statistics of the seeded synthetic inputs (no lattice arithmetic)."""
import math

import numpy as np
import pytest

from paper_1508_02899_amd import inputs


def test_gaussian_ic_unit_mass_and_variance():
    nx, nv, L = 64, 33, 2 * math.pi
    dx = L / nx
    dv = 5.0 / 16
    f = inputs.gaussian_ic(1, nx, nv, dx, dv, dtype=np.float64)
    v = (np.arange(nv) - 16) * dv
    assert f.sum() * dx * dv == pytest.approx(1.0, rel=1e-13)
    var = (f.sum(axis=1) * v * v).sum() * dx * dv
    assert var == pytest.approx(1.0, rel=0.02)  # sigma0 = 1 sampled at centres


def test_flow1d_rms_and_renewal():
    u = inputs.flow1d(512, 2 * math.pi, 400, modes=8, spectrum="k-1",
                      renew=50, seed=1, dtype=np.float64)
    assert u.shape == (400, 1, 512)
    assert np.sqrt(np.mean(u ** 2)) == pytest.approx(1.0, rel=0.1)
    # independent draws: lag-1 correlation of slices is ~0
    c = np.mean(u[1:] * u[:-1]) / np.mean(u * u)
    assert abs(c) < 0.15


def test_flow1d_ou_correlation_time():
    dt, tau = 0.05, 1.0
    u = inputs.flow1d(128, 2 * math.pi, 2000, modes=32, spectrum="k-5/3",
                      tau_f=tau, dt=dt, seed=2, dtype=np.float64)
    lag = int(round(tau / dt))
    c = np.mean(u[lag:] * u[:-lag]) / np.mean(u * u)
    assert c == pytest.approx(math.exp(-1.0), abs=0.12)


def test_flow2d_divergence_free_and_spectrum():
    n, L = 128, 2 * math.pi
    u = inputs.flow2d_streamfunction(n, L, 3, kmax=32, seed=3,
                                     dtype=np.float64)
    k = np.fft.fftfreq(n, d=1.0 / n)
    KX, KY = np.meshgrid(k, k)
    ux, uy = np.fft.fft2(u[0, 0]), np.fft.fft2(u[0, 1])
    div = np.fft.ifft2(1j * KX * ux + 1j * KY * uy).real
    assert np.abs(div).max() < 1e-10 * np.abs(u).max()
    assert np.sqrt(np.mean(u ** 2)) == pytest.approx(1.0, rel=1e-12)
    # shell energy spectrum slope ~ -3 between k = 2 and 24
    E = 0.5 * (np.abs(ux) ** 2 + np.abs(uy) ** 2)
    K = np.sqrt(KX ** 2 + KY ** 2)
    ks = np.arange(2, 25)
    Ek = np.array([E[(K >= q - 0.5) & (K < q + 0.5)].sum() for q in ks])
    slope = np.polyfit(np.log(ks), np.log(Ek), 1)[0]
    assert slope == pytest.approx(-3.0, abs=0.4)


def test_flow2d_fixed_normalisation_keeps_the_leading_slices():
    """With the scale taken over a fixed number of leading slices, a longer
    flow starts with the slices of a shorter one (the OU draws are
    sequential); by default the scale covers every slice, so the two
    differ."""
    kw = dict(kmax=8, seed=11, dtype=np.float64)
    short = inputs.flow2d_streamfunction(32, 2 * math.pi, 10, **kw)
    longer = inputs.flow2d_streamfunction(32, 2 * math.pi, 25, norm_slices=10,
                                          **kw)
    assert np.array_equal(short, longer[:10])
    u = longer[:10]
    assert np.sqrt(np.mean(u ** 2)) == pytest.approx(1.0, rel=1e-12)
    whole = inputs.flow2d_streamfunction(32, 2 * math.pi, 25, **kw)
    assert not np.array_equal(short, whole[:10])
    for bad in (0, 26):
        with pytest.raises(ValueError):
            inputs.flow2d_streamfunction(32, 2 * math.pi, 25, norm_slices=bad,
                                         **kw)


def test_cellular_flow_divergence_free():
    n, L = 64, 2 * math.pi
    u = inputs.cellular_flow(n, L, dtype=np.float64)[0]
    k = np.fft.fftfreq(n, d=L / n) * 2 * math.pi
    KX, KY = np.meshgrid(k, k)
    div = np.fft.ifft2(1j * KX * np.fft.fft2(u[0]) + 1j * KY * np.fft.fft2(u[1])).real
    assert np.abs(div).max() < 1e-10


def test_choose_vmax_satisfies_cfl():
    v = inputs.choose_vmax(512, 2 * math.pi, 129, 0.1 * 2 * math.pi, 4.0)
    h = 64
    dv = v / h
    dt = (2 * math.pi / 512) / dv
    assert (dt / dv) * (4.0 + v) / (0.1 * 2 * math.pi) <= 0.45
    assert v % 0.5 == 0
