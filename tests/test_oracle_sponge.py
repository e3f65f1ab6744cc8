"""Pins of the oracle's vorticity sponge term (Sec. 4.1, the sponge term of the
penalized equations; sign and mask readings in oracle/sponge.py).

* chi_sp = 1: curl (-lap)^-1 curl u = u for a band-limited solenoidal u, so the
  term is exactly -u/C_sp (a wrong sign, a missing 1/|k|^2 or a curl applied to
  u instead of omega all fail);
* with chi_sp = 1 the 2-D Taylor-Green field (whose nonlinear term is a pure
  gradient) follows the scalar IF-AB2 recurrence of a linear damping 1/C_sp
  for any dt sequence;
* k.T_hat = 0 for any mask (the term is a curl);
* the mask places g_x along x, g_y along y, g_z along z and takes their maximum.
"""

import numpy as np

from oracle import ns, spectral, sponge, dft
import synth


def test_uniform_sponge_is_linear_damping(rng):
    n, L = (12, 10, 8), (2.0, 1.7, 1.3)
    o = ns.OracleNS(n, L, 0.01, 1.0)
    o.set_velocity(synth.random_solenoidal(n, L, seed=4))
    c_sp = 0.37
    chi = np.ones(n[::-1])
    th = sponge.sponge_term_hat(o.uh, chi, c_sp, n, L)
    assert np.max(np.abs(th + o.uh / c_sp)) < 1e-12 * np.max(np.abs(o.uh)) / c_sp


def test_uniform_sponge_scalar_recurrence(rng):
    n = (16, 16, 8)
    L = (2 * np.pi,) * 3
    nu, c_sp = 0.02, 0.3
    o = ns.OracleNS(n, L, nu, eta=1.0)
    u0 = synth.taylor_green_2d(n, L)
    o.set_velocity(u0)
    o.set_sponge(c_sp, gx=np.ones(n[0]))
    a_prev, a, dt_prev = None, 1.0, None
    for dt in rng.uniform(0.005, 0.03, 10):
        o.step(dt=dt)
        en = np.exp(-2 * nu * dt)
        if a_prev is None:
            a_new = en * (1 - dt / c_sp) * a
        else:
            xi = dt / dt_prev
            ep = np.exp(-2 * nu * dt_prev)
            a_new = en * (1 - dt * (1 + xi / 2) / c_sp) * a + dt * (xi / 2) / c_sp * en * ep * a_prev
        a_prev, a, dt_prev = a, a_new, dt
        assert np.max(np.abs(o.velocity() - a * u0)) < 1e-13


def test_sponge_term_is_solenoidal(rng):
    n, L = (12, 10, 8), (2.0, 1.7, 1.3)
    o = ns.OracleNS(n, L, 0.01, 1.0)
    o.set_velocity(synth.random_solenoidal(n, L, seed=5))
    chi = rng.uniform(0, 1, n[::-1])
    th = sponge.sponge_term_hat(o.uh, chi, 0.5, n, L)
    kx, ky, kz = spectral.wavenumbers(n, L)
    div = kx * th[0] + ky * th[1] + kz * th[2]
    assert np.max(np.abs(div)) < 1e-12 * np.max(np.abs(th)) * np.max(np.abs(kx))


def test_sponge_curl_is_projected_masked_vorticity(rng):
    """curl T = -(1/C_sp) P(chi_sp omega), written out with the spectral curl and
    projection (operators pinned in test_oracle_spectral)."""
    n, L = (12, 10, 8), (2.0, 1.7, 1.3)
    o = ns.OracleNS(n, L, 0.01, 1.0)
    o.set_velocity(synth.random_solenoidal(n, L, seed=6))
    chi = rng.uniform(0, 1, n[::-1])
    c_sp = 0.8
    th = sponge.sponge_term_hat(o.uh, chi, c_sp, n, L)
    w = dft.inverse_real(spectral.curl(o.uh, n, L))
    rhs = -(1.0 / c_sp) * spectral.project(dft.forward(chi[None] * w), n, L)
    rhs[:, 0, 0, 0] = 0.0  # T has no mean, P is the identity at k = 0
    assert np.max(np.abs(spectral.curl(th, n, L) - rhs)) < 1e-12 * np.max(np.abs(rhs))


def test_sponge_mask_axes():
    n = (5, 4, 3)
    gx, gy, gz = np.linspace(0, 0.4, 5), np.array([0.9, 0, 0, 0.1]), np.array([0, 0.5, 0])
    m = sponge.sponge_mask(n, gx, gy, gz)
    assert m.shape == (3, 4, 5)
    for z in range(3):
        for y in range(4):
            for x in range(5):
                assert m[z, y, x] == max(gx[x], gy[y], gz[z])
    assert np.array_equal(sponge.sponge_mask(n, gx), np.broadcast_to(gx, (3, 4, 5)))
