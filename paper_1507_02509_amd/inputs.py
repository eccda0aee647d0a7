"""Seeded synthetic velocity fields for the paper's workloads.

This module is shared by the GPU path, the tests and the oracle runs.  It holds
no lattice Boltzmann arithmetic: it only produces macroscopic velocity fields
(float64 numpy arrays ``[ny, nx]`` indexed ``[y, x]``) in lattice units, which
each side then turns into populations with its own initialisation.

Workloads:
  * ``tgv`` -- the Green-Taylor vortex of the section of that name: the curl of
    the stream function (u0/k2) cos(k1 X) cos(k2 Y) exp(-nu (K1^2 + K2^2) t) on
    the periodic square (0, 2 pi)^2, sampled at X = 2 pi x / N, with lattice
    wavenumbers K = 2 pi k / N.
  * ``spectral`` -- the decaying-turbulence initial field: a zero-mean Gaussian
    random stream function with random phases and amplitudes from a prescribed
    energy spectrum, differentiated spectrally into a divergence-free velocity
    and rescaled to a given u_rms = sqrt(<u_x^2 + u_y^2>).  Two spectra:
    ``"gauss4"`` E(k) ~ k^4 exp(-2 (k/k0)^2) and ``"paper"``
    E(k) ~ k^6 / (1 + (k/k0)^18) (A = 6, B = 17 in the turbulence section).
    Coefficients are drawn on a fixed box |k_x|, |k_y| <= K of integer
    wavenumbers, so one seed gives the same physical field on every grid with
    N > 2 K + 1.
  * ``shear_layer`` -- the doubly periodic shear layer with its tanh profile
    and sinusoidal perturbation.
  * ``uniform_noise`` -- independent uniform velocity at every node, drawn on
    the device: the field for lattices too large for a spectral synthesis.
"""
from __future__ import annotations

import numpy as np


def tgv(n: int, u0: float, k1: int = 1, k2: int = 4, nu: float = 0.0, t: float = 0.0,
        with_grad: bool = False):
    """Green-Taylor vortex velocity (and optionally its exact lattice gradients).

    Returns ``ux, uy`` or ``ux, uy, grad`` with ``grad[4, n, n]`` =
    (d_x u_x, d_y u_x, d_x u_y, d_y u_y) in lattice units.
    """
    x = np.arange(n, dtype=np.float64)
    X = 2.0 * np.pi * x / n
    XX, YY = np.meshgrid(X, X, indexing="xy")  # XX varies along axis 1 (x), YY along axis 0 (y)
    K1 = 2.0 * np.pi * k1 / n
    K2 = 2.0 * np.pi * k2 / n
    decay = np.exp(-nu * (K1 * K1 + K2 * K2) * t)
    # psi = (u0/k2) cos(k1 X) cos(k2 Y); u = (d psi/dY, -d psi/dX)
    ux = -u0 * np.cos(k1 * XX) * np.sin(k2 * YY) * decay
    uy = u0 * (k1 / k2) * np.sin(k1 * XX) * np.cos(k2 * YY) * decay
    if not with_grad:
        return ux, uy
    s = 2.0 * np.pi / n
    g = np.empty((4, n, n))
    g[0] = s * u0 * k1 * np.sin(k1 * XX) * np.sin(k2 * YY) * decay           # d_x u_x
    g[1] = -s * u0 * k2 * np.cos(k1 * XX) * np.cos(k2 * YY) * decay          # d_y u_x
    g[2] = s * u0 * (k1 * k1 / k2) * np.cos(k1 * XX) * np.cos(k2 * YY) * decay  # d_x u_y
    g[3] = -s * u0 * k1 * np.sin(k1 * XX) * np.sin(k2 * YY) * decay          # d_y u_y
    return ux, uy, g


def shear_wave(n: int, amp: float, mode: int = 1):
    """u_x = amp sin(2 pi mode y / n), u_y = 0: a decaying transverse shear wave."""
    y = np.arange(n, dtype=np.float64)
    ux = np.repeat((amp * np.sin(2.0 * np.pi * mode * y / n))[:, None], n, axis=1)
    return ux, np.zeros_like(ux)


def _spectrum(k: np.ndarray, k0: float, kind: str) -> np.ndarray:
    k = np.asarray(k, dtype=np.float64)
    if kind == "gauss4":
        return k ** 4 * np.exp(-2.0 * (k / k0) ** 2)
    if kind == "paper":
        return k ** 6 / (1.0 + (k / k0) ** 18)
    raise ValueError(f"unknown spectrum {kind!r}")


def spectral(n: int, k0: float, u_rms: float, seed: int, kind: str = "gauss4",
             kmax: int | None = None, ny: int | None = None, device=None):
    """Divergence-free random velocity on an ``ny x n`` periodic grid (``ny``
    defaults to n).  With ``device`` set, the transforms run in torch on that
    device and torch float64 tensors are returned (same coefficients)."""
    ny = n if ny is None else ny
    if kmax is None:
        kmax = int(np.ceil(4 * k0))
    kmax = int(min(kmax, n // 2 - 1, ny // 2 - 1))
    if kmax < 1:
        raise ValueError("grid too small for a spectral field")
    rng = np.random.Generator(np.random.PCG64(seed))
    m = 2 * kmax + 1
    xi = rng.standard_normal((2, m, m))
    kk = np.arange(-kmax, kmax + 1, dtype=np.float64)
    KX, KY = np.meshgrid(kk, kk, indexing="xy")
    kmag = np.hypot(KX, KY)
    amp = np.zeros_like(kmag)
    nz = kmag > 0
    amp[nz] = np.sqrt(_spectrum(kmag[nz], k0, kind) / (np.pi * kmag[nz] ** 3))
    coef = amp * (xi[0] + 1j * xi[1]) / np.sqrt(2.0)
    # Hermitian symmetrisation: psi_hat(-k) = conj(psi_hat(k)), so psi is real
    coef = 0.5 * (coef + np.conj(coef[::-1, ::-1]))
    iy = (kk.astype(np.int64)) % ny
    ix = (kk.astype(np.int64)) % n
    if device is None:
        psi_hat = np.zeros((ny, n), dtype=np.complex128)
        psi_hat[np.ix_(iy, ix)] = coef
        kx_l = 2.0 * np.pi * np.fft.fftfreq(n)
        ky_l = 2.0 * np.pi * np.fft.fftfreq(ny)
        ux = np.real(np.fft.ifft2(1j * ky_l[:, None] * psi_hat))
        uy = np.real(np.fft.ifft2(-1j * kx_l[None, :] * psi_hat))
        rms = np.sqrt(np.mean(ux * ux + uy * uy))
        if rms == 0.0:
            raise ValueError("degenerate spectral field")
        s = u_rms / rms
        return np.ascontiguousarray(ux * s), np.ascontiguousarray(uy * s)
    import torch
    psi_hat = torch.zeros((ny, n), dtype=torch.complex128, device=device)
    iyt = torch.as_tensor(iy, device=device)
    ixt = torch.as_tensor(ix, device=device)
    psi_hat[iyt[:, None], ixt[None, :]] = torch.as_tensor(coef, device=device)
    kx_l = 2.0 * np.pi * torch.fft.fftfreq(n, device=device, dtype=torch.float64)
    ky_l = 2.0 * np.pi * torch.fft.fftfreq(ny, device=device, dtype=torch.float64)
    ux = torch.fft.ifft2(1j * ky_l[:, None] * psi_hat).real.contiguous()
    uy = torch.fft.ifft2(-1j * kx_l[None, :] * psi_hat).real.contiguous()
    del psi_hat
    rms = torch.sqrt(torch.mean(ux * ux + uy * uy)).item()
    if rms == 0.0:
        raise ValueError("degenerate spectral field")
    s = u_rms / rms
    return ux.mul_(s), uy.mul_(s)


def uniform_noise(nx: int, ny: int, amp: float, seed: int, device):
    """u_x and u_y drawn independently and uniformly from [-amp, amp] at every
    node by torch's seeded generator on `device`, as float64 tensors [ny, nx]
    (the same numbers on every run with the same seed and device type).  The
    field has no smoothness: every node's velocity, and so its populations,
    differ from its neighbours', which makes any misplaced row or column of a
    lattice show."""
    import torch
    g = torch.Generator(device=device).manual_seed(int(seed))
    ux = torch.empty((ny, nx), dtype=torch.float64, device=device).uniform_(-amp, amp, generator=g)
    uy = torch.empty((ny, nx), dtype=torch.float64, device=device).uniform_(-amp, amp, generator=g)
    return ux, uy


def shear_layer(n: int, u0: float = 0.04, kappa: float = 80.0, delta: float = 0.05):
    """Doubly periodic shear layer: tanh profiles about y = N/4 and 3N/4 plus a
    sinusoidal y-velocity perturbation of relative size delta."""
    y = np.arange(n, dtype=np.float64)
    x = np.arange(n, dtype=np.float64)
    prof = np.where(y <= n / 2, u0 * np.tanh(kappa * (y / n - 0.25)),
                    u0 * np.tanh(kappa * (0.75 - y / n)))
    ux = np.repeat(prof[:, None], n, axis=1)
    uy = np.repeat((delta * u0 * np.sin(2.0 * np.pi * (x / n + 0.25)))[None, :], n, axis=0)
    return np.ascontiguousarray(ux), np.ascontiguousarray(uy)


def ensemble_members(count: int = 256, master_seed: int = 4,
                     sizes=(128, 256, 512, 1024), nu_range=(1e-5, 1e-3)):
    """Draw (n, nu, seed) for each member of the uneven-grid ensemble: n uniform
    over ``sizes``, nu log-uniform over ``nu_range``, seed 1000 * master + r."""
    rng = np.random.Generator(np.random.PCG64(master_seed))
    ns = rng.choice(np.asarray(sizes), size=count)
    lo, hi = np.log(nu_range[0]), np.log(nu_range[1])
    nus = np.exp(rng.uniform(lo, hi, size=count))
    return [(int(ns[r]), float(nus[r]), 1000 * master_seed + r) for r in range(count)]
