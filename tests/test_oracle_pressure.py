"""Pins of the oracle's pressure and wing loads (Sec. 4.1 coupling).

* The 4-point kernel satisfies the conditions it is built from: for every
  offset, sum phi = 1, first moment 0, sum phi^2 = 3/8, even and odd points
  each carry 1/2; phi(0) = 1/2, phi(1) = 1/4, phi(2) = 0.  So interpolation
  reproduces linear fields exactly.
* 3-D Taylor-Green: p = Pi - |u|^2/2 equals the classical closed form
  (cos 2x + cos 2y)(cos 2z + 2)/16 up to a constant.
* Pi is the gradient part of the nonlinear term: N' - grad Pi is divergence free.
* Loads: a linear pressure across a flat plate gives dp = 2 d G exactly and a
  total load -dp A n.
"""

import numpy as np
import pytest

from oracle import dft, pressure, spectral
from oracle.ns import OracleNS
import synth


@pytest.mark.parametrize("s", [0.0, 0.1, 0.37, 0.5, 0.81, 0.999])
def test_delta_kernel_moment_conditions(s):
    j = np.arange(-3, 5)
    r = s - j
    phi = pressure.delta4(r)
    assert np.sum(phi) == pytest.approx(1.0, abs=1e-15)
    assert np.sum(r * phi) == pytest.approx(0.0, abs=1e-15)
    assert np.sum(phi * phi) == pytest.approx(3.0 / 8.0, abs=1e-15)
    assert np.sum(phi[j % 2 == 0]) == pytest.approx(0.5, abs=1e-15)


def test_delta_kernel_values():
    assert pressure.delta4(0.0) == 0.5
    assert pressure.delta4(1.0) == pytest.approx(0.25, abs=1e-16)
    assert pressure.delta4(-1.0) == pytest.approx(0.25, abs=1e-16)
    assert pressure.delta4(2.0) == 0.0
    assert pressure.delta4(2.5) == 0.0


def test_interpolation_reproduces_linear_fields():
    n, L = 16, 4.0
    xs = np.arange(n) * L / n
    Z, Y, X = np.meshgrid(xs, xs, xs, indexing="ij")
    f = 0.3 + 1.1 * X - 0.7 * Y + 0.4 * Z
    rng = np.random.default_rng(0)
    pts = 1.0 + 2.0 * rng.random((20, 3))  # stencils stay inside the grid (no wrap)
    got = pressure.sample(f, (L, L, L), pts)
    assert np.allclose(got, 0.3 + 1.1 * pts[:, 0] - 0.7 * pts[:, 1] + 0.4 * pts[:, 2], atol=1e-13)


def test_taylor_green_pressure_closed_form():
    n = (32, 32, 32)
    L = (2 * np.pi,) * 3
    o = OracleNS(n, L, nu=0.01, eta=1.0)
    o.set_velocity(synth.taylor_green_3d(n))
    o.step(dt=1e-3)
    xs = np.arange(32) * 2 * np.pi / 32
    Z, Y, X = np.meshgrid(xs, xs, xs, indexing="ij")
    ref = (np.cos(2 * X) + np.cos(2 * Y)) * (np.cos(2 * Z) + 2.0) / 16.0
    p = o.p_last
    assert np.max(np.abs((p - p.mean()) - (ref - ref.mean()))) < 1e-13


def test_total_pressure_is_the_gradient_part():
    n = (16, 12, 10)
    L = (2.0, 1.5, 1.25)
    g = synth.random_field((3, 10, 12, 16), seed=4)
    nh = spectral.dealias(dft.forward(g), n)
    pih = pressure.total_pressure_hat(nh, n, L)
    kx, ky, kz = spectral.wavenumbers(n, L)
    rest = np.stack([nh[0] - 1j * kx * pih, nh[1] - 1j * ky * pih, nh[2] - 1j * kz * pih])
    div = kx * rest[0] + ky * rest[1] + kz * rest[2]
    assert np.max(np.abs(div)) < 1e-13 * np.max(np.abs(nh))
    # and it is what the projection removes
    assert np.allclose(rest, spectral.project(nh, n, L), atol=1e-14)


def test_linear_pressure_across_a_flat_plate():
    n, L = 32, 4.0
    xs = np.arange(n) * L / n
    Z, Y, X = np.meshgrid(xs, xs, xs, indexing="ij")
    G = 0.7
    p = 0.2 + G * Z  # pressure rising along the plate normal
    x, tri = synth.flat_rectangle((2.0, 2.0, 2.03), (1, 0, 0), (0, 1, 0), 0.6, 0.4, 5, 4)
    d = 0.25
    loads, dp = pressure.wing_loads(p, (L, L, L), x, tri, d)
    nz = np.cross(x[tri[0, 1]] - x[tri[0, 0]], x[tri[0, 2]] - x[tri[0, 0]])
    nz /= np.linalg.norm(nz)
    assert np.allclose(dp, 2 * d * G * nz[2], atol=1e-13)
    area = 1.2 * 0.8
    assert np.allclose(loads.sum(axis=0), -2 * d * G * nz[2] * area * nz, atol=1e-12)
