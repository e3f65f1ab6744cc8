"""Pins of the static (z-independent) penalization of the oracle: walls,
fixed obstacles and inflow layers of the channel workload (Sec. 4.1
penalized equations; Sec. 4.2.1 channel with a cylinder).

* a uniform static mask chi_st = c with u_st = U(y) e_x acting on a shear flow
  u = f(y) e_x: u x omega = f f' e_y is a pure gradient, so every Fourier mode
  of f follows the scalar integrating-factor AB2 recurrence of a relaxation
  towards U at rate c/eta (closed form, any dt sequence);
* two wall slabs, one at rest and one moving with U: the steady flow between
  them tends to plane Couette flow, and the wall interiors move with their
  walls up to O(eta);
* the static force of a uniform flow through the static mask, weighted per
  point: F_st = (dV/eta) sum w chi (U - u_st);
* the max rule: a static mask chi_st = 0 leaves the step unchanged bit for bit,
  chi_st = 1 everywhere hides the wing (its force is zero, the step equals the
  static-only step).
"""

import numpy as np
import pytest

from oracle import ns, mask as omask, dft
import synth


def shear_field(n, L, coeffs):
    """u = f(y) e_x with f = c0 + c1 cos(2 pi y / Ly) + c2 sin(4 pi y / Ly)."""
    nx, ny, nz = n
    y = np.arange(ny) * (L[1] / ny)
    th = 2 * np.pi * y / L[1]
    f = coeffs[0] + coeffs[1] * np.cos(th) + coeffs[2] * np.sin(2 * th)
    u = np.zeros((3, nz, ny, nx))
    u[0] = f[None, :, None]
    return u


def test_uniform_static_mask_recurrence(rng):
    n, L = (8, 16, 8), (1.0, 2.0, 1.5)
    nu, eta, c = 0.04, 0.05, 0.7
    nx, ny, nz = n
    o = ns.OracleNS(n, L, nu, eta)
    a = np.array([0.3, 1.1, -0.6])   # f(0): mean, cos(y), sin(2y)
    s = np.array([1.5, -0.4, 0.25])  # U(y) in the same three modes
    o.set_velocity(shear_field(n, L, a))
    us = shear_field(n, L, s)[:, 0]  # (3, ny, nx)
    o.set_static_mask(np.full((ny, nx), c), us)
    k2 = np.array([0.0, (2 * np.pi / L[1]) ** 2, (4 * np.pi / L[1]) ** 2])
    prev, dtp = None, None
    t = 0.0
    for dt in rng.uniform(2e-3, 2e-2, 8):
        e = np.exp(-nu * k2 * dt)
        nn = -(c / eta) * (a - s)
        if prev is None:
            a_new = e * (a + dt * nn)
        else:
            xi = dt / dtp
            ep = np.exp(-nu * k2 * dtp)
            a_new = e * (a + dt * (1 + 0.5 * xi) * nn) - dt * 0.5 * xi * e * ep * prev
        prev, dtp, a = nn, dt, a_new
        d = o.step(dt=dt)
        t += dt
        ref = shear_field(n, L, a)
        assert np.max(np.abs(o.velocity() - ref)) < 1e-13 * np.max(np.abs(ref))
        assert np.all(d["F"] == 0.0)  # no wing


def _wall_run(eta, n=(8, 64, 8), T=2.5, U=1.0):
    nx, ny, nz = n
    L = (0.25, 1.0, 0.25)
    y = np.arange(ny) * (L[1] / ny)
    h = 2 * L[1] / ny

    def slab(yc):
        d = np.abs((y - yc + 0.5) % 1.0 - 0.5)
        return omask.chi_profile(d, 0.1, h, omask.PROFILE_COS)

    chi_a, chi_b = slab(0.0), slab(0.5)
    chi = np.tile(np.maximum(chi_a, chi_b)[:, None], (1, nx))
    us = np.zeros((3, ny, nx))
    us[0] = np.where(chi_b > chi_a, U, 0.0)[:, None]
    o = ns.OracleNS(n, L, 0.05, eta)
    o.set_static_mask(chi, us)
    o.set_velocity(np.zeros((3, nz, ny, nx)))
    t, dt = 0.0, 2.0 / 3.0 * eta
    while t < T:
        o.step(dt=dt)
        t += dt
    f = o.velocity()[0, 0, :, 0]
    couette = np.where((y > 0.1) & (y < 0.4), U * (y - 0.1) / 0.3,
                       np.where((y > 0.6) & (y < 0.9), U * (0.9 - y) / 0.3, np.nan))
    fluid = ~np.isnan(couette)
    return (float(np.max(np.abs(f[fluid] - couette[fluid]))), float(np.max(np.abs(f[chi_a > 0.99]))),
            float(np.max(np.abs(f[chi_b > 0.99] - U))))


def test_moving_walls_give_couette_flow():
    """Penalized walls at rest (y in [-0.1, 0.1]) and moving with U = 1
    (y in [0.4, 0.6]): steady plane Couette flow in the two fluid gaps; inside
    the walls the flow follows the wall up to O(eta)."""
    e1, a1, b1 = _wall_run(1e-2)
    e2, a2, b2 = _wall_run(3e-3)
    print("Couette: eta 1e-2 fluid %.4f walls %.2e %.2e; eta 3e-3 fluid %.4f walls %.2e %.2e"
          % (e1, a1, b1, e2, a2, b2))
    assert e2 < 0.025 and e2 < e1  # linear profile between the walls
    for w1, w2 in ((a1, a2), (b1, b2)):
        assert w1 < 0.02 and w2 < w1 / 3.0  # at least linear in eta


def test_static_force_of_a_uniform_flow(rng):
    n, L = (8, 12, 10), (1.0, 1.5, 1.25)
    nx, ny, nz = n
    eta = 0.3
    U = np.array([0.7, -0.2, 0.4])
    o = ns.OracleNS(n, L, 0.01, eta)
    u = np.zeros((3, nz, ny, nx)) + U[:, None, None, None]
    o.set_velocity(u)
    chi = rng.uniform(0, 1, (ny, nx))
    us = rng.standard_normal((3, ny, nx))
    w = (rng.uniform(0, 1, (ny, nx)) > 0.5).astype(float)
    o.set_static_mask(chi, us, w)
    d = o.step(dt=1e-3)
    dV = np.prod(L) / np.prod(n)
    ref = (dV / eta) * nz * np.array([np.sum(w * chi * (U[c] - us[c])) for c in range(3)])
    assert np.max(np.abs(d["F_static"] - ref)) < 1e-12 * np.max(np.abs(ref))


def test_max_rule_with_the_wing():
    cfg = synth.config0(True)
    n, L = cfg["n"], cfg["L"]
    nx, ny, nz = n
    x, v, tri = cfg["wing"]
    v = v + np.array([0.3, -0.1, 0.2])
    u0 = synth.taylor_green_3d(n, L)

    def run(static):
        o = ns.OracleNS(n, L, cfg["nu"], cfg["eta"], cfg["tw"], cfg["h"], cfg["profile"])
        o.set_velocity(u0)
        o.set_wing(x, v, tri)
        if static is not None:
            o.set_static_mask(*static)
        F, Fs = [], []
        for _ in range(3):
            d = o.step(dt=cfg["dt"])
            F.append(d["F"])
            Fs.append(d["F_static"])
        return o.uh, np.array(F), np.array(Fs)

    us_st = np.zeros((3, ny, nx))
    us_st[1] = 0.4
    base = run(None)
    zero = run((np.zeros((ny, nx)), us_st, np.ones((ny, nx))))
    assert np.array_equal(base[0], zero[0]) and np.array_equal(base[1], zero[1])
    assert not np.any(zero[2])
    full = run((np.ones((ny, nx)), us_st, np.ones((ny, nx))))
    o = ns.OracleNS(n, L, cfg["nu"], cfg["eta"], cfg["tw"], cfg["h"], cfg["profile"])
    o.set_velocity(u0)
    o.set_static_mask(np.ones((ny, nx)), us_st, np.ones((ny, nx)))
    Fs = [o.step(dt=cfg["dt"])["F_static"] for _ in range(3)]
    assert not np.any(full[1])  # chi_st = 1 everywhere: the wing never wins
    assert np.array_equal(full[0], o.uh) and np.array_equal(full[2], np.array(Fs))
    assert np.max(np.abs(base[1])) > 1e-3
