"""Pins of the oracle's spectra (a plain definition: full-plane FFT and shell
sums): Parseval, single Fourier modes whose shell and amplitude are known in
closed form, and the exact-derivative enstrophy of a sine wave."""
import numpy as np

from paper_1507_02509_amd import inputs


def test_parseval_energy_and_enstrophy_of_random_field(orc):
    n = 64
    ux, uy = inputs.spectral(n, 6, 0.05, seed=3)
    E, Z = orc.spectra(ux, uy, kmax=int(np.ceil(n / np.sqrt(2))))
    assert abs(E.sum() - 0.5 * np.mean(ux ** 2 + uy ** 2)) < 1e-15
    # spectral vorticity: omega_hat = i (kx uy_hat - ky ux_hat) with k in 2 pi / n units
    k = 2 * np.pi * np.fft.fftfreq(n, d=1.0 / n) / n
    om = np.real(np.fft.ifft2(1j * (k[None, :] * np.fft.fft2(uy) - k[:, None] * np.fft.fft2(ux))))
    assert abs(Z.sum() - 0.5 * np.mean(om ** 2)) < 1e-12 * np.mean(om ** 2)


def test_axis_mode(orc):
    n, m, a = 32, 5, 0.03
    y = np.arange(n)
    ux = np.repeat((a * np.sin(2 * np.pi * m * y / n))[:, None], n, axis=1)
    uy = np.zeros_like(ux)
    E, Z = orc.spectra(ux, uy, kmax=20)
    want = np.zeros(21)
    want[m] = a * a / 4
    assert np.abs(E - want).max() < 1e-18
    assert abs(Z[m] - (2 * np.pi * m / n) ** 2 * a * a / 4) < 1e-18
    assert np.abs(np.delete(Z, m)).max() < 1e-20


def test_diagonal_mode_lands_in_shell_five(orc):
    n, a = 64, 0.02
    x = np.arange(n)
    X, Y = np.meshgrid(x, x, indexing="xy")
    ph = 2 * np.pi * (3 * X + 4 * Y) / n
    ux, uy = a * np.sin(ph), -0.75 * a * np.sin(ph)     # divergence-free: 3 ux + 4 uy = 0
    E, Z = orc.spectra(ux, uy, kmax=10)
    assert np.argmax(E) == 5 and abs(E.sum() - E[5]) < 1e-18
    assert abs(E[5] - 0.25 * (a * a + (0.75 * a) ** 2)) < 1e-18
    assert abs(Z[5] - (2 * np.pi * 5 / n) ** 2 * E[5]) < 1e-18
