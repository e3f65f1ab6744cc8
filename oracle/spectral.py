"""Spectral operators of the pseudo-spectral method (oracle; test infrastructure only).

Sec. 4.1 solves the penalized equations in rotational form with a Fourier
pseudo-spectral discretization on a periodic uniform grid.  The paper does
not spell out the dealiasing rule; the reading used here (and by the HIP
path) is the 2/3 rule: a mode is kept iff 3|m_j| < N_j on every axis, which
also removes the Nyquist mode.  The Leray projection enforces div u = 0 and
is the identity at k = 0 (the mean flow may change under penalization drag).

Pins (tests/test_oracle_spectral.py): curl of the 3-D Taylor-Green field
against its closed form, k.P(v) = 0, P(P(v)) = P(v), P(grad phi) = 0, every
mode outside the band exactly zero after dealiasing.
"""

import numpy as np


def signed_modes(n):
    """Integer mode numbers m in natural FFT order: 0..n/2, then -(n/2-1)..-1.

    For even n the Nyquist index n/2 is taken as +n/2 (it is removed by the
    2/3 band anyway)."""
    j = np.arange(n)
    return np.where(j <= n // 2, j, j - n)


def wavenumbers(n, L):
    """Return (kx, ky, kz) broadcastable to (nz, ny, nx), k_j = 2 pi m_j / L_j."""
    nx, ny, nz = n
    lx, ly, lz = L
    kx = 2.0 * np.pi * signed_modes(nx) / lx
    ky = 2.0 * np.pi * signed_modes(ny) / ly
    kz = 2.0 * np.pi * signed_modes(nz) / lz
    return kx[None, None, :], ky[None, :, None], kz[:, None, None]


def band_mask(n):
    """Boolean (nz, ny, nx): True for modes kept by the 2/3 rule (3|m_j| < N_j on every axis)."""
    nx, ny, nz = n
    mx = np.abs(signed_modes(nx))[None, None, :]
    my = np.abs(signed_modes(ny))[None, :, None]
    mz = np.abs(signed_modes(nz))[:, None, None]
    return (3 * mx < nx) & (3 * my < ny) & (3 * mz < nz)


def dealias(vh, n):
    """Zero every mode outside the 2/3 band (applies to any leading component axes)."""
    return vh * band_mask(n)


def curl(uh, n, L):
    """Spectral curl: omega_hat = i k x u_hat."""
    kx, ky, kz = wavenumbers(n, L)
    ux, uy, uz = uh
    wx = 1j * (ky * uz - kz * uy)
    wy = 1j * (kz * ux - kx * uz)
    wz = 1j * (kx * uy - ky * ux)
    return np.stack([wx, wy, wz])


def project(vh, n, L):
    """Leray projection v - k (k.v)/|k|^2 for k != 0; identity at k = 0."""
    kx, ky, kz = wavenumbers(n, L)
    k2 = kx * kx + ky * ky + kz * kz
    kdotv = kx * vh[0] + ky * vh[1] + kz * vh[2]
    inv = np.where(k2 > 0, 1.0 / np.where(k2 > 0, k2, 1.0), 0.0)
    s = kdotv * inv
    return np.stack([vh[0] - kx * s, vh[1] - ky * s, vh[2] - kz * s])


def k_squared(n, L):
    kx, ky, kz = wavenumbers(n, L)
    return kx * kx + ky * ky + kz * kz


def cross(a, b):
    """Pointwise cross product of two (3, ...) fields."""
    return np.stack([
        a[1] * b[2] - a[2] * b[1],
        a[2] * b[0] - a[0] * b[2],
        a[0] * b[1] - a[1] * b[0],
    ])
