"""Pins of the oracle's naive DFT (Sec. 4.1: Fourier pseudo-spectral discretization).

Checked against what the mathematics fixes, not against the oracle itself:
a brute-force triple sum over all (k, x) pairs, exact deltas for single
modes, Parseval, the inverse, and numpy's FFT library routine.
"""

import numpy as np
import pytest

from oracle import dft


def brute_forward(f):
    nz, ny, nx = f.shape
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    out = np.zeros((nz, ny, nx), dtype=np.complex128)
    for mz in range(nz):
        for my in range(ny):
            for mx in range(nx):
                ph = 2 * np.pi * (mx * ix / nx + my * iy / ny + mz * iz / nz)
                out[mz, my, mx] = np.sum(f * np.exp(-1j * ph))
    return out / (nx * ny * nz)


@pytest.mark.parametrize("shape", [(8, 8, 8), (4, 6, 8), (6, 4, 10)])
def test_forward_matches_brute_force_sum(shape, rng):
    f = rng.standard_normal(shape)
    ref = brute_forward(f)
    got = dft.forward(f)
    assert np.max(np.abs(got - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


def test_single_modes_give_exact_deltas():
    nz, ny, nx = 6, 8, 10
    ix = np.arange(nx)[None, None, :]
    iy = np.arange(ny)[None, :, None]
    iz = np.arange(nz)[:, None, None]
    for (a, b, c) in [(1, 0, 0), (3, 2, 1), (4, 3, 2)]:
        f = np.cos(2 * np.pi * (a * ix / nx + b * iy / ny + c * iz / nz))
        fh = dft.forward(f)
        expect = np.zeros_like(fh)
        expect[c % nz, b % ny, a % nx] += 0.5
        expect[(-c) % nz, (-b) % ny, (-a) % nx] += 0.5
        assert np.max(np.abs(fh - expect)) < 1e-14


def test_parseval_and_inverse(rng):
    f = rng.standard_normal((8, 12, 10))
    fh = dft.forward(f)
    n3 = f.size
    assert abs(np.sum(np.abs(fh) ** 2) - np.sum(f * f) / n3) < 1e-13 * np.sum(f * f) / n3
    back = dft.inverse(fh)
    assert np.max(np.abs(back.imag)) < 1e-13
    assert np.max(np.abs(back.real - f)) < 1e-13


def test_agrees_with_numpy_fft(rng):
    f = rng.standard_normal((10, 8, 12))
    assert np.max(np.abs(dft.forward(f) - np.fft.fftn(f) / f.size)) < 1e-14
