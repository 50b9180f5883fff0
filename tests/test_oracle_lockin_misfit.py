"""Pins of the lock-in projection and the window misfit (exact finite sums)."""
import numpy as np
import pytest


@pytest.mark.parametrize("N,periods", [(3, 5), (7, 2), (200, 20), (256, 3)])
def test_lockin_discrete_orthogonality(orc, N, periods):
    """Samples of A sin(2 pi p/N - phi) plus a DC offset and harmonics 2..N/2-1 give back exactly
    (A, phi): the other terms are orthogonal to cos/sin of the fundamental over whole periods."""
    rng = np.random.default_rng(N)
    A, phi = 1.7e-8, -2.1
    p0 = 1
    k = np.arange(N * periods)
    th = 2 * np.pi * ((p0 + k) % N) / N
    u = A * np.sin(th - phi) + 3e-9
    for hmn in range(2, (N + 1) // 2):
        u += rng.normal() * 1e-9 * np.sin(hmn * th + rng.random() * 6)
    A_o, phi_o = orc.lockin(u, N, p0)
    assert abs(A_o / A - 1) < 1e-12
    assert abs(np.angle(np.exp(1j * (phi_o - phi)))) < 1e-12


def test_lockin_phase_convention(orc):
    """u = A sin(wd t - phi): a cosine lags by -pi/2 ... i.e. -cos gives phi = +pi/2."""
    N = 64
    th = 2 * np.pi * ((1 + np.arange(N)) % N) / N
    assert abs(orc.lockin(-np.cos(th), N, 1)[1] - np.pi / 2) < 1e-14
    assert abs(orc.lockin(np.sin(th), N, 1)[1]) < 1e-14
    assert abs(orc.lockin(np.cos(th), N, 1)[1] + np.pi / 2) < 1e-14


def test_misfit_identities(orc):
    rng = np.random.default_rng(3)
    U = rng.normal(size=1000) * 1e-8
    assert orc.misfit(U, U) == 0.0
    assert orc.misfit(U, np.zeros_like(U)) == 1.0
    for c in (0.5, 0.9, 2.0, -1.0):
        assert abs(orc.misfit(U, c * U) - (1 - c) ** 2) < 1e-14
    bad = U.copy()
    bad[10] = np.nan
    assert orc.misfit(U, bad) == np.inf
