"""Pins of the oracle's spectral operators (Sec. 4.1 penalized NS in rotational form).

Closed forms of the 3-D Taylor-Green field and invariants of the Leray
projection and of the 2/3 band.
"""

import numpy as np

from oracle import dft, spectral
import synth


def test_curl_and_cross_of_taylor_green_closed_form():
    n = (16, 12, 10)
    L = (2 * np.pi,) * 3
    u = synth.taylor_green_3d(n, L)
    uh = spectral.dealias(dft.forward(u), n)
    w = dft.inverse_real(spectral.curl(uh, n, L))
    x = np.arange(n[0])[None, None, :] * 2 * np.pi / n[0]
    y = np.arange(n[1])[None, :, None] * 2 * np.pi / n[1]
    z = np.arange(n[2])[:, None, None] * 2 * np.pi / n[2]
    wx = -np.cos(x) * np.sin(y) * np.sin(z)
    wy = -np.sin(x) * np.cos(y) * np.sin(z)
    wz = 2 * np.sin(x) * np.sin(y) * np.cos(z)
    assert np.max(np.abs(w[0] - wx)) < 1e-13
    assert np.max(np.abs(w[1] - wy)) < 1e-13
    assert np.max(np.abs(w[2] - wz)) < 1e-13
    ux = np.sin(x) * np.cos(y) * np.cos(z)
    uy = -np.cos(x) * np.sin(y) * np.cos(z)
    c = spectral.cross(u, w)
    assert np.max(np.abs(c[0] - uy * wz)) < 1e-13
    assert np.max(np.abs(c[1] + ux * wz)) < 1e-13
    assert np.max(np.abs(c[2] - (ux * wy - uy * wx))) < 1e-13


def test_curl_of_non_cubic_box_single_mode():
    # u = (0, 0, sin(2 pi 2 x / lx)) -> omega_y = -du_z/dx = -(4 pi/lx) cos(...)
    n = (12, 8, 6)
    L = (3.0, 5.0, 7.0)
    x = np.arange(n[0]) * L[0] / n[0]
    u = np.zeros((3, n[2], n[1], n[0]))
    u[2] = np.sin(2 * np.pi * 2 * x / L[0])[None, None, :]
    w = dft.inverse_real(spectral.curl(dft.forward(u), n, L))
    expect = -(4 * np.pi / L[0]) * np.cos(2 * np.pi * 2 * x / L[0])[None, None, :]
    assert np.max(np.abs(w[1] - expect)) < 1e-12
    assert np.max(np.abs(w[0])) < 1e-12 and np.max(np.abs(w[2])) < 1e-12


def test_projection_invariants(rng):
    n = (8, 10, 6)
    L = (1.0, 2.0, 3.0)
    vh = rng.standard_normal((3, 6, 10, 8)) + 1j * rng.standard_normal((3, 6, 10, 8))
    p = spectral.project(vh, n, L)
    kx, ky, kz = spectral.wavenumbers(n, L)
    kdot = kx * p[0] + ky * p[1] + kz * p[2]
    kmag = np.sqrt(kx * kx + ky * ky + kz * kz)
    pmag = np.sqrt(np.sum(np.abs(p) ** 2, axis=0))
    ratio = np.abs(kdot) / np.maximum(kmag * pmag, 1e-300)
    assert np.max(ratio) < 1e-14
    assert np.max(np.abs(spectral.project(p, n, L) - p)) < 1e-14
    # identity at k = 0
    assert np.max(np.abs(p[:, 0, 0, 0] - vh[:, 0, 0, 0])) == 0.0
    # gradients are removed
    phi = rng.standard_normal((6, 10, 8)) + 1j * rng.standard_normal((6, 10, 8))
    grad = np.stack([1j * kx * phi, 1j * ky * phi, 1j * kz * phi])
    assert np.max(np.abs(spectral.project(grad, n, L))) < 1e-13 * np.max(np.abs(grad))


def test_dealias_band_is_two_thirds_rule(rng):
    n = (12, 9, 8)
    vh = rng.standard_normal((8, 9, 12)) + 0j
    d = spectral.dealias(vh, n)
    for iz in range(8):
        for iy in range(9):
            for ix in range(12):
                mx = ix if ix <= 6 else ix - 12
                my = iy if iy <= 4 else iy - 9
                mz = iz if iz <= 4 else iz - 8
                keep = 3 * abs(mx) < 12 and 3 * abs(my) < 9 and 3 * abs(mz) < 8
                assert (d[iz, iy, ix] == vh[iz, iy, ix]) if keep else (d[iz, iy, ix] == 0.0)
