"""Test-side helpers: layout conversions between the oracle's full spectrum
and the library's compact band, and common tolerances."""

import numpy as np


def band_k(n):
    return (n - 1) // 3


def natural_band_modes(K):
    """Mode numbers of the compact band axis in storage order (0..K, -K..-1)."""
    return np.concatenate([np.arange(K + 1), np.arange(-K, 0)])


def full_to_compact(fh, n):
    """Full spectrum (..., nz, ny, nx) -> compact band (..., 2Kz+1, 2Ky+1, Kx+1)."""
    nx, ny, nz = n
    Kx, Ky, Kz = band_k(nx), band_k(ny), band_k(nz)
    iz = natural_band_modes(Kz) % nz
    iy = natural_band_modes(Ky) % ny
    ix = np.arange(Kx + 1)
    return fh[..., iz[:, None, None], iy[None, :, None], ix[None, None, :]]


def rel_max(a, b):
    """max |a - b| / max |b|."""
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
