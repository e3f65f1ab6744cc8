"""Naive discrete Fourier transform by matrix products (oracle; test infrastructure only).

The pseudo-spectral method of Sec. 4.1 needs the 3-D DFT of periodic fields on
a uniform grid.  This module writes that definition out directly: the DFT
along one axis is the product with the N x N matrix
``M[m, j] = exp(-2 pi i ((m j) mod N) / N)``; the 3-D transform applies it
along x, y and z.  Forward transforms are normalized by 1/(nx ny nz), inverse
transforms are not.  Full complex spectra are kept (no half-spectrum
storage), with the natural FFT ordering of modes along each axis.

Pins (tests/test_oracle_dft.py): brute-force triple sum on 8^3 random data,
single-mode inputs giving exact deltas, Parseval, inverse(forward) = identity.
"""

import numpy as np


def dft_matrix(n, sign=-1):
    """The n x n DFT matrix exp(sign * 2 pi i (m j mod n) / n).

    The exponent is reduced mod n in integers before the trigonometric call, so
    every entry is one of the n exact roots of unity cos(2 pi q/n) + i sin(...).
    """
    m = np.arange(n)
    q = np.outer(m, m) % n
    ang = 2.0 * np.pi * q / n
    return np.cos(ang) + sign * 1j * np.sin(ang)


def _along_x(f, mat):
    # f[..., x] -> sum_x mat[m, x] f[..., x]
    return f @ mat.T


def _along_y(f, mat):
    # f[..., y, x] -> sum_y mat[m, y] f[..., y, x]
    return np.matmul(mat, f)


def _along_z(f, mat):
    # f[z, y, x] (optionally with a leading component axis)
    shp = f.shape
    nz = shp[-3]
    lead = shp[:-3]
    g = f.reshape(lead + (nz, shp[-2] * shp[-1]))
    out = np.matmul(mat, g)
    return out.reshape(lead + (nz, shp[-2], shp[-1]))


def forward(f):
    """Normalized forward 3-D DFT: fhat_k = (1/N^3) sum_x f(x) exp(-i k.x).

    ``f`` has shape (..., nz, ny, nx); the result is complex with the same shape.
    """
    nz, ny, nx = f.shape[-3:]
    g = np.asarray(f, dtype=np.complex128)
    g = _along_x(g, dft_matrix(nx, -1))
    g = _along_y(g, dft_matrix(ny, -1))
    g = _along_z(g, dft_matrix(nz, -1))
    return g / float(nx * ny * nz)


def inverse(fh):
    """Unnormalized inverse 3-D DFT: f(x) = sum_k fhat_k exp(+i k.x) (complex result)."""
    nz, ny, nx = fh.shape[-3:]
    g = np.asarray(fh, dtype=np.complex128)
    g = _along_x(g, dft_matrix(nx, +1))
    g = _along_y(g, dft_matrix(ny, +1))
    g = _along_z(g, dft_matrix(nz, +1))
    return g


def inverse_real(fh):
    """Real part of the inverse transform (the field is real when fh is Hermitian)."""
    return inverse(fh).real
